// Host checks of the band plan of the population scratch (lelbm_plan.cpp):
// built with g++ by test_plan.py, no GPU needed.  Prints one line per
// failure and "ALL OK (n plans)" at the end; exit status 1 on any failure.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lelbm_plan.h"
#include "lelbm.h"

using namespace lelbm;

static int failures = 0;
#define FAIL(...)                   \
    do {                            \
        std::printf(__VA_ARGS__);   \
        std::printf("\n");          \
        failures++;                 \
    } while (0)

// A 2D domain of ny interior rows with pads of `pad` cells on both y faces
// (none when periodic), 16 x 16 tiles and two gather block rows per tile row.
static PlanGeom geom(int ny, bool periodic, int pad) {
    PlanGeom g;
    const int w = periodic ? 0 : pad;
    g.ty = 16;
    g.wb = w;
    g.syn = ny + 2 * w;
    g.nty = (g.syn + 15) / 16;
    g.dty = (ny + 15) / 16;
    g.pery = periodic ? 1 : 0;
    g.gby = 2 * g.dty;
    return g;
}

// The band holding padded cell row y (wrapped on a periodic axis), -1 if
// outside the padded domain.
static int band_of_row(const PlanGeom &g, const Plan &P, int y) {
    if (g.pery) {
        y %= g.syn;
        if (y < 0) y += g.syn;
    } else if (y < 0 || y >= g.syn) {
        return -1;
    }
    return (y / g.ty) / P.rows;
}

// Every destination row is gathered once, after the reconstruction of every
// band within reach M of it, and before that band's slot is filled again.
static void check_schedule(const PlanGeom &g, const Plan &P, int M, const char *what) {
    const int nb = (int)P.bands.size(), nops = (int)P.ops.size();
    std::vector<int> epr_of(nb, -1);
    for (int i = 0; i < nops; i++) {
        const Op &op = P.ops[i];
        if (op.kind != OP_EPR) continue;
        if (op.a < 0 || op.a >= nb || epr_of[op.a] >= 0) FAIL("%s: band %d reconstructed twice or out of range", what, op.a);
        else epr_of[op.a] = i;
    }
    for (int k = 0; k < nb; k++) {
        if (epr_of[k] < 0) FAIL("%s: band %d never reconstructed", what, k);
        if (P.slot_of[k] < 0 || P.slot_of[k] >= P.nslots) FAIL("%s: band %d has slot %d of %d", what, k, P.slot_of[k], P.nslots);
        const int r0 = k * P.rows, r1 = std::min(g.nty, (k + 1) * P.rows);
        if (P.bands[k].row0 != r0 || P.bands[k].row1 != r1) FAIL("%s: band %d rows [%d, %d)", what, k, P.bands[k].row0, P.bands[k].row1);
    }
    if (failures) return;
    const int bpr = g.gby / g.dty;
    std::vector<int> gathered(g.gby, 0);
    for (int i = 0; i < nops; i++) {
        const Op &op = P.ops[i];
        if (op.kind != OP_GATHER) continue;
        for (int br = op.a; br < op.a + op.n; br++) {
            if (br < 0 || br >= g.gby) {
                FAIL("%s: gather %d of block row %d out of range", what, i, br);
                continue;
            }
            gathered[br]++;
            const int j = br / bpr;
            for (int y = j * g.ty + g.wb - M; y <= (j + 1) * g.ty - 1 + g.wb + M; y++) {
                const int k = band_of_row(g, P, y);
                if (k < 0 || k >= nb) continue;
                bool dep = false;
                for (int d = 0; d < op.ndep; d++) dep = dep || P.gdeps[op.dep + d] == epr_of[k];
                if (!dep) FAIL("%s: gather %d (row %d) does not wait for band %d", what, i, j, k);
                if (epr_of[k] > i) FAIL("%s: gather %d before the reconstruction of band %d", what, i, k);
                // the next reconstruction into band k's slot waits for this gather
                for (int e = epr_of[k] + 1; e < nops; e++) {
                    const Op &oe = P.ops[e];
                    if (oe.kind != OP_EPR || P.slot_of[oe.a] != P.slot_of[k]) continue;
                    if (oe.dep < i) FAIL("%s: band %d refills the slot of band %d before gather %d", what, oe.a, k, i);
                    break;
                }
            }
        }
    }
    for (int br = 0; br < g.gby; br++)
        if (gathered[br] != 1) FAIL("%s: block row %d gathered %d times", what, br, gathered[br]);
}

int main() {
    int n = 0;
    char what[160];
    // schedules over heights, boundary conditions, reaches and band heights
    for (int per = 0; per < 2; per++)
        for (int ny : {40, 128, 200, 2048, 4096})
            for (int M : {3, 12, 21, 40, 150})
                for (int rows : {1, 2, 3, 5, 8, 64, 1000}) {
                    const PlanGeom g = geom(ny, per != 0, 24);
                    Plan P;
                    build_plan(g, P, rows, M);
                    std::snprintf(what, sizeof what, "ny %d periodic %d rows %d M %d", ny, per, rows, M);
                    check_schedule(g, P, M, what);
                    n++;
                }
    // bands of one tile row keep at most the bands within reach plus the
    // spares live: with the reach inside one tile row, five slots
    {
        const PlanGeom g = geom(4096, false, 48);
        Plan P;
        build_plan(g, P, 1, 12);
        if (P.nslots > 5) FAIL("one-row bands at reach 12 use %d slots", P.nslots);
        n++;
    }
    // plan_first: one band when the records fit, else bands within the limit
    {
        const PlanGeom g = geom(4096, false, 48);
        Plan P;
        plan_first(g, P, 1000000, 500000, 20);
        if (P.bands.size() != 1 || P.slot_cap < 500000 || P.slot_cap > 1000000) FAIL("plan_first: records that fit");
        Plan Q;
        plan_first(g, Q, 1000000, 50000000, 20);
        if (Q.bands.size() < 2 || (long long)Q.nslots * Q.slot_cap > 1000000) FAIL("plan_first: banded plan over the limit");
        check_schedule(g, Q, Q.m_plan, "plan_first banded");
        if (Q.m_plan < 20) FAIL("plan_first: plan reach %d below the step's 20", Q.m_plan);
        n += 2;
    }
    // plan_adapt: on overflow the bands get thinner and the scratch stays
    // within the limit until bands of one row do not fit; a fixed scratch too
    // small for one-row bands is ENOMEM; a reach beyond the plan re-plans for
    // it
    {
        const PlanGeom g = geom(4096, false, 48);
        const long long limit = 64ll << 20;
        Plan P;
        plan_first(g, P, limit, 10 * limit, 16);
        for (int round = 0; round < 8; round++) {
            const long long need = P.slot_cap + P.slot_cap / 3;   // the largest band outgrew its slot
            const int r = plan_adapt(g, P, limit, false, ERR_OVERFLOW, need, 10 * limit, 16);
            if (r != LELBM_OK) FAIL("plan_adapt overflow round %d: %d", round, r);
            // over the limit only as the last resort: one band of the whole
            // domain, or bands of one row without the spare slot
            const bool last = P.whole || (P.rows == 1 && !P.overlap);
            if (!last && (long long)P.nslots * P.slot_cap > limit) FAIL("plan_adapt overflow round %d: over the limit", round);
            check_schedule(g, P, P.m_plan == INT_MAX / 2 ? 0 : P.m_plan, "plan_adapt overflow");
            n++;
        }
        Plan R;
        plan_first(g, R, limit, 10 * limit, 16);
        const int r = plan_adapt(g, R, limit, false, ERR_REPLAN, 0, 0, 40);
        if (r != LELBM_OK || R.m_plan < 40) FAIL("plan_adapt re-plan: status %d, reach %d", r, R.m_plan);
        check_schedule(g, R, R.m_plan, "plan_adapt re-plan");
        n++;
        Plan F;
        plan_first(g, F, 1024, 10 * limit, 16);
        F.rows = 1;
        F.overlap = false;
        build_plan(g, F, 1, 20);
        F.slot_cap = 1024 / F.nslots;
        const int rf = plan_adapt(g, F, 1024, true, ERR_OVERFLOW, 1 << 20, 1 << 26, 16);
        if (rf != LELBM_ENOMEM) FAIL("plan_adapt with a fixed scratch too small: status %d", rf);
        n++;
    }
    if (failures) {
        std::printf("FAILED (%d)\n", failures);
        return 1;
    }
    std::printf("ALL OK (%d plans)\n", n);
    return 0;
}
