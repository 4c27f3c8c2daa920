// Band plan of the population scratch: host logic only (no device code),
// built into the library and checked on the host by the tests.
//
// The source tiles are reconstructed in bands of whole tile rows; a band
// writes its records into one of nslots slots of slot_cap elements, and the
// gather of a destination tile row runs as soon as every band holding a
// source within reach of it (m_plan cells, the plan's largest reach) has
// been reconstructed.  A slot is reused once no pending destination row
// needs its band.  With a periodic y axis the last band is reconstructed
// first, so that the first destination rows, which reach across the wrap,
// are gathered early; the first and the last band then stay live to the end.
// The scratch is nslots x slot_cap elements, kept within the context's
// budget: more bands of fewer rows when a band's records outgrow their slot.
#pragma once

#include <vector>

namespace lelbm {

// Internal error codes: a band's population records exceed their scratch
// slot (the host grows the slots or re-plans the bands and repeats the step);
// a stencil reaches farther than the band plan allows for (the host re-plans
// and repeats the step).
constexpr int ERR_OVERFLOW = -100;
constexpr int ERR_REPLAN = -101;

// One band as the device sees it.
struct BandInfo {
    int row0, row1;          // source tile rows [row0, row1)
    long long base;          // first scratch element of the band's slot
};

// What the plan needs of the domain.
struct PlanGeom {
    int nty;                 // source tile rows (padded domain)
    int dty;                 // destination tile rows (interior)
    int ty;                  // cell rows per tile
    int wb;                  // pad width below the interior
    int syn;                 // padded cell rows
    int pery;                // 1: periodic y axis
    int gby;                 // gather block rows (a multiple of dty)
};

enum { OP_EPR = 0, OP_GATHER = 1 };
struct Op {
    int kind;    // OP_EPR: reconstruct band a; OP_GATHER: gather destination block rows [a, a + n)
    int a, n;
    // what must finish first: a reconstruction into a reused slot waits for
    // the last gather of the slot's former band (op dep, -1: none); a gather
    // waits for the reconstructions of the bands it needs (ops
    // Plan::gdeps[dep, dep + ndep))
    int dep, ndep;
};

struct Plan {
    int rows = 0;              // source tile rows per band (0: not built)
    int m_plan = 0;            // largest reach (cells) the plan allows for
    int nslots = 1;
    long long slot_cap = 0;    // elements per slot
    std::vector<BandInfo> bands;
    std::vector<int> slot_of;
    std::vector<Op> ops;
    std::vector<int> gdeps;    // reconstruction ops the gathers wait for
    bool uploaded = false;     // the device band table holds this plan
    bool whole = false;        // one band of the whole domain because bands of one tile row cost more
    bool overlap = true;       // a spare slot lets consecutive bands' reconstructions overlap
    // working arrays of build_plan, reserved at creation so that re-planning
    // allocates nothing
    std::vector<int> w_order, w_int;
    std::vector<char> w_flags;
};

// Bands of `rows` source tile rows and the schedule of their reconstruction
// and gathers for a largest reach of M cells.
void build_plan(const PlanGeom &g, Plan &P, int rows, int M);
// Each band's base: the first element of its slot.
void set_bases(Plan &P);
// After a step found a band's records larger than its slot (err =
// ERR_OVERFLOW, need = the largest band's elements, total = all bands') or a
// reach beyond the plan (ERR_REPLAN): the next plan within `limit` elements
// of scratch (fixed: the scratch cannot grow).  LELBM_OK or LELBM_ENOMEM.
int plan_adapt(const PlanGeom &g, Plan &P, long long limit, bool fixed, int err, long long need, long long total,
               int reach);
// The first plan of a context whose whole domain's records are `need`
// elements at reach `reach`: one band if they fit `limit` with a quarter to
// spare, else bands sized for about five slots.
void plan_first(const PlanGeom &g, Plan &P, long long limit, long long need, int reach);

}  // namespace lelbm
