// Band plan of the population scratch (see lelbm_plan.h).
#include "lelbm_plan.h"

#include <algorithm>
#include <climits>

#include "../../include/lelbm.h"

namespace lelbm {

// Bands of `rows` source tile rows and the schedule of their reconstruction
// and gathers for a largest reach of M cells (see Plan).
void build_plan(const PlanGeom &g, Plan &P, int rows, int M) {
    const int nty = g.nty, dty = g.dty;
    rows = std::max(1, std::min(rows, nty));
    const int nb = (nty + rows - 1) / rows;
    P.rows = rows;
    P.whole = false;
    P.m_plan = nb == 1 ? INT_MAX / 2 : M;
    P.bands.resize((size_t)nb);
    P.slot_of.assign((size_t)nb, -1);
    P.ops.clear();
    P.gdeps.clear();
    for (int k = 0; k < nb; k++) {
        P.bands[k].row0 = k * rows;
        P.bands[k].row1 = std::min(nty, (k + 1) * rows);
        P.bands[k].base = 0;
    }
    // the bands that hold sources within reach of destination tile row j:
    // padded cell rows j ty + wb - M ... (j + 1) ty - 1 + wb + M, wrapped on a
    // periodic axis (mirror images across slip walls lie within that range)
    const bool pery = g.pery != 0;
    auto needs = [&](int j, int k) {
        if (nb == 1) return true;
        const int y0 = j * g.ty + g.wb - M, y1 = (j + 1) * g.ty - 1 + g.wb + M;
        const int c0 = P.bands[k].row0 * g.ty, c1 = P.bands[k].row1 * g.ty - 1;   // the band's cell rows
        if (!pery) return std::max(y0, c0) <= std::min(y1, std::min(c1, g.syn - 1));
        if (y1 - y0 + 1 >= g.syn) return true;
        const int a = ((y0 % g.syn) + g.syn) % g.syn, b = ((y1 % g.syn) + g.syn) % g.syn;
        if (a <= b) return std::max(a, c0) <= std::min(b, c1);
        return c1 >= a || c0 <= b;
    };
    std::vector<int> &order = P.w_order;
    order.clear();
    if (pery && nb > 1) order.push_back(nb - 1);
    for (int k = 0; k < nb; k++)
        if (!(pery && nb > 1 && k == nb - 1)) order.push_back(k);
    P.w_flags.assign((size_t)4 * nb + (size_t)dty, 0);
    char *done = P.w_flags.data(), *live = done + nb, *slot_busy = live + nb, *gathered = slot_busy + 2 * nb;
    P.w_int.assign((size_t)4 * nb, -1);
    int *last_gather = P.w_int.data(), *slot_free_op = last_gather + nb, *epr_of = slot_free_op + nb;   // op indices
    int *freed_at = epr_of + nb;   // iteration that freed a slot
    int nslots = 0;
    // destination tile rows -> gather block rows
    const int bpr = g.gby / std::max(dty, 1);
    for (int it = 0; it < nb; it++) {
        const int k = order[it];
        // a slot freed by the gathers that followed one of the two previous
        // bands' reconstructions is not reused yet: reusing it would make
        // this reconstruction wait for those gathers, which wait for that
        // reconstruction, and the bands would not overlap (the oldest free
        // slot first).  Two bands back rather than one: the next band's
        // reconstruction then also fills the tail of the current one
        // (measured on the 8192 x 4096 Mach-10 channel at a 16 GiB budget:
        // 50.1 -> 48.7 ms per step in FP64).
        int slot = -1;
        const int delay = P.overlap ? 3 : 1;
        for (int sl = 0; sl < nslots; sl++)
            if (!slot_busy[sl] && freed_at[sl] <= it - delay && (slot < 0 || freed_at[sl] < freed_at[slot])) slot = sl;
        if (slot < 0) slot = nslots++;
        slot_busy[slot] = 1;
        P.slot_of[k] = slot;
        done[k] = live[k] = 1;
        epr_of[k] = (int)P.ops.size();
        P.ops.push_back(Op{OP_EPR, k, 1, slot_free_op[slot], 0});
        // every destination row whose bands are all reconstructed, in runs
        int run0 = -1;
        for (int j = 0; j <= dty; j++) {
            bool ready = j < dty && !gathered[j];
            for (int kk = 0; ready && kk < nb; kk++) ready = done[kk] || !needs(j, kk);
            if (ready) {
                gathered[j] = 1;
                if (run0 < 0) run0 = j;
            } else if (run0 >= 0) {
                const int gop = (int)P.ops.size();
                Op op{OP_GATHER, run0 * bpr, (j - run0) * bpr, (int)P.gdeps.size(), 0};
                for (int kk = 0; kk < nb; kk++) {
                    bool any = false;
                    for (int jj = run0; jj < j && !any; jj++) any = needs(jj, kk);
                    if (!any) continue;
                    last_gather[kk] = gop;
                    P.gdeps.push_back(epr_of[kk]);
                    op.ndep++;
                }
                P.ops.push_back(op);
                run0 = -1;
            }
        }
        // slots of bands no pending destination row needs are free again
        for (int kk = 0; kk < nb; kk++) {
            if (!live[kk]) continue;
            bool used = false;
            for (int j = 0; j < dty && !used; j++) used = !gathered[j] && needs(j, kk);
            if (!used) {
                live[kk] = 0;
                slot_busy[P.slot_of[kk]] = 0;
                slot_free_op[P.slot_of[kk]] = last_gather[kk];
                freed_at[P.slot_of[kk]] = it;
            }
        }
    }
    P.nslots = std::max(1, nslots);
    P.uploaded = false;
}

void set_bases(Plan &P) {
    for (size_t k = 0; k < P.bands.size(); k++) P.bands[k].base = (long long)P.slot_of[k] * P.slot_cap;
    P.uploaded = false;
}

// After a step found a band's records larger than its slot (err =
// ERR_OVERFLOW, need = the largest band's elements, total = all bands') or a
// reach beyond the plan (ERR_REPLAN): the next plan within `limit` elements
// of scratch.  When even bands of one tile row do not fit, the smaller of
// one band of the whole domain and bands of one row (the scratch then
// exceeds the limit); with a fixed scratch that is ENOMEM unless one band
// fits it.
int plan_adapt(const PlanGeom &g, Plan &P, long long limit, bool fixed, int err, long long need, long long total,
               int reach) {
    const int margin = std::max(4, reach / 4);
    if (P.whole && err == ERR_OVERFLOW) {
        // stays one band (bands of one row cost more before): it grows
        if (fixed && need > limit) return LELBM_ENOMEM;
        P.slot_cap = fixed ? limit : need + need / 4 + 1024;
    } else if (err == ERR_REPLAN) {
        build_plan(g, P, P.rows, reach + margin);
        P.slot_cap = std::min(P.slot_cap, limit / P.nslots);
    } else if (need <= limit / P.nslots) {
        P.slot_cap = std::min(limit / P.nslots, need + need / 4 + 1024);
    } else if (P.rows > 1) {
        // thinner bands, scaled by the share of a slot the largest band may
        // take (a thinner plan may keep more bands live at once)
        const long long per = limit / P.nslots;
        const int old_rows = P.rows;
        int rows = (int)std::max(1.0, 0.8 * old_rows * (double)per / (double)need);
        rows = std::min(rows, old_rows - 1);
        build_plan(g, P, rows, std::max(P.m_plan == INT_MAX / 2 ? 0 : P.m_plan, reach + margin));
        const long long est = (long long)((double)need * rows / old_rows * 1.25) + 1024;
        P.slot_cap = std::min(limit / P.nslots, est);
    } else if (P.overlap) {
        // bands of one row without the spare slot (no overlap of consecutive
        // bands' reconstructions) before giving up the budget
        P.overlap = false;
        build_plan(g, P, 1, std::max(P.m_plan == INT_MAX / 2 ? 0 : P.m_plan, reach + margin));
        P.slot_cap = limit / P.nslots;
    } else {
        const long long whole = total + total / 4 + 1024, rowwise = P.nslots * (need + need / 4 + 1024);
        if (whole <= rowwise || (fixed && whole <= limit)) {
            if (fixed && whole > limit) return LELBM_ENOMEM;
            build_plan(g, P, g.nty, 0);
            P.whole = true;
            P.slot_cap = fixed ? limit : whole;
        } else {
            if (fixed) return LELBM_ENOMEM;
            P.slot_cap = need + need / 4 + 1024;
        }
    }
    set_bases(P);
    return LELBM_OK;
}

void plan_first(const PlanGeom &g, Plan &P, long long limit, long long need, int reach) {
    // five slots: the most a periodic plan keeps live with bands wider than
    // the reach
    const long long want = need + need / 4 + 1024;
    if (want <= limit) {
        build_plan(g, P, g.nty, 0);
        P.slot_cap = want;
    } else {
        const int rows = (int)std::max(1.0, (double)g.nty * (double)limit / (5.0 * (double)want));
        build_plan(g, P, rows, reach + std::max(4, reach / 4));
        P.slot_cap = limit / P.nslots;
    }
    set_bases(P);
}

}  // namespace lelbm
