// Host runtime of the LELBM library: the C ABI declared in include/lelbm.h.
//
// A context owns the padded state (two ping-pong buffers), the per-cell
// stencil descriptors, the per-tile scratch layout, the population scratch,
// error flags and statistics, all in device memory.  lelbm_step enqueues the
// kernels of each step on the context's stream and synchronises once at the
// end to read the error flags; a failed step leaves the previous state in
// place because every kernel returns early once a flag is set.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <vector>

#include "lelbm_3d.h"

using namespace lelbm;

// What the band plan needs of the domain.
static PlanGeom plan_geom(const Geom &g) {
    return PlanGeom{g.nty, g.dty, g.ty, g.wb, g.syn, g.dim == 2 && g.bc[2] == LELBM_BC_PERIODIC, gather_blocks_y(g)};
}

// pinned host staging memory (see stage_h2d / stage_d2h)
struct Stage {
    void *p = nullptr;
    size_t cap = 0;
};

struct lelbm_ctx {
    lelbm_params p;
    Geom g;
    Phys ph;
    Phys ph_step;            // ph with the current step's source mass (read at each launch)
    long long steps_done;    // completed steps (the time of a point mass source)
    int mixed;
    int nmom;
    hipStream_t stream;
    int device;
    Buffers b;
    int cur;                 // state buffer holding the current moments
    long last_fail_node;
    int last_fail_step;
    int last_fail_detail, last_fail_species;
    double last_fail_residual;
    int timing;
    hipEvent_t ev[2];
    double kms[LELBM_NTIMERS];
    long klaunch[LELBM_NTIMERS];
    // timing mode: event pairs recorded around each kernel, read after the
    // stream synchronisation at the end of lelbm_step
    std::vector<hipEvent_t> evpool;
    std::vector<int> evkind;
    size_t evused;
    // learned guess: device copies of the network (owned by the context)
    unsigned short *mlp_w;
    float *mlp_p, *mlp_n;
    int mlp_set;
    long long persistent_bytes;
    Stage stage;             // pinned host staging memory
    int gcap;                // staged sources per gather chunk
    long long budget;        // population scratch budget (bytes)
    Plan plan;               // band plan of lelbm_step (the context's scratch)
    Plan fixed_plan;         // band plan of lelbm_step_noalloc (the static array)
    // A banded step reconstructs the narrow and refined stencils of the even
    // bands on the caller's stream and of the odd bands on side[0], the wide
    // stencils of every band on side[2] and gathers on side[1] (all streams
    // at the default priority), so that the long tiles at the end of one
    // band's reconstruction overlap the next band's and the gathers; two
    // events per operation of the plan (and one for the step's start) order
    // the streams.
    hipStream_t side[3];
    std::vector<hipEvent_t> opev;
    Ctx3 *c3;                // the 3D path (dim = 3), else NULL
};

// HIP errors are reported as LELBM_EDEVICE; with LELBM_DEBUG set in the
// environment the failing call is also printed to stderr.
static void report_hip(hipError_t e, const char *what, int line) {
    if (getenv("LELBM_DEBUG")) fprintf(stderr, "lelbm: %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
}

#define HIPCHECK(x)                                  \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) {                      \
            report_hip(e_, #x, __LINE__);            \
            return LELBM_EDEVICE;                    \
        }                                            \
    } while (0)

// Host <-> device transfers go through pinned staging memory (hipHostMalloc)
// owned by the context or network; user memory is only touched by host
// memcpy, so nothing depends on how the runtime treats pageable memory.
static const size_t STAGE_MAX = (size_t)32 << 20;

static int stage_reserve(Stage &st, size_t bytes) {
    if (bytes <= st.cap) return LELBM_OK;
    if (st.p) HIPCHECK(hipHostFree(st.p));
    st.p = nullptr;
    st.cap = 0;
    if (hipHostMalloc(&st.p, bytes, hipHostMallocDefault) != hipSuccess) { st.p = nullptr; return LELBM_ENOMEM; }
    st.cap = bytes;
    return LELBM_OK;
}

static void stage_free(Stage &st) {
    if (st.p) (void)hipHostFree(st.p);
    st.p = nullptr;
    st.cap = 0;
}

// Contiguous copies in chunks of at most STAGE_MAX bytes.
static int stage_h2d(Stage &st, hipStream_t s, void *dev, const void *host, size_t bytes) {
    int r = stage_reserve(st, bytes < STAGE_MAX ? bytes : STAGE_MAX);
    if (r != LELBM_OK) return r;
    for (size_t o = 0; o < bytes; o += st.cap) {
        size_t n = bytes - o < st.cap ? bytes - o : st.cap;
        memcpy(st.p, (const char *)host + o, n);
        HIPCHECK(hipMemcpyAsync((char *)dev + o, st.p, n, hipMemcpyHostToDevice, s));
        HIPCHECK(hipStreamSynchronize(s));
    }
    return LELBM_OK;
}

static int stage_d2h(Stage &st, hipStream_t s, void *host, const void *dev, size_t bytes) {
    int r = stage_reserve(st, bytes < STAGE_MAX ? bytes : STAGE_MAX);
    if (r != LELBM_OK) return r;
    for (size_t o = 0; o < bytes; o += st.cap) {
        size_t n = bytes - o < st.cap ? bytes - o : st.cap;
        HIPCHECK(hipMemcpyAsync(st.p, (const char *)dev + o, n, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        memcpy((char *)host + o, st.p, n);
    }
    return LELBM_OK;
}

extern "C" int lelbm_num_moments(int dim) { return dim == 1 ? 6 : (dim == 2 ? 11 : (dim == 3 ? 17 : -1)); }

extern "C" int lelbm_moments_from_primitives(int dim, double K, long n, const double *rho, const double *ux,
                                             const double *uy, const double *RT, double *out) {
    int nm = lelbm_num_moments(dim);
    if ((dim != 1 && dim != 2) || n < 0 || !rho || !ux || !RT || !out || (dim == 2 && !uy)) return LELBM_EINVAL;
    for (long i = 0; i < n; i++) {
        double r = rho[i], x = ux[i], y = dim == 2 ? uy[i] : 0.0, T = RT[i];
        double m[11];
        if (dim == 1) {
            m[0] = r; m[1] = r * x; m[2] = r * (x * x + T); m[3] = r * (x * x + 3.0 * T) * x;
            m[4] = r * K * T; m[5] = r * K * T * x;
        } else {
            double uu = x * x + y * y;
            m[0] = r; m[1] = r * x; m[2] = r * y;
            m[3] = r * (x * x + T); m[4] = r * (x * y); m[5] = r * (y * y + T);
            m[6] = r * (uu + 4.0 * T) * x; m[7] = r * (uu + 4.0 * T) * y;
            m[8] = r * K * T; m[9] = r * K * T * x; m[10] = r * K * T * y;
        }
        for (int k = 0; k < nm; k++) out[(long)k * n + i] = m[k];
    }
    return LELBM_OK;
}

extern "C" int lelbm_moments_from_primitives3(double K, long n, const double *rho, const double *ux, const double *uy,
                                              const double *uz, const double *RT, double *out) {
    if (n < 0 || !rho || !ux || !uy || !uz || !RT || !out) return LELBM_EINVAL;
    for (long i = 0; i < n; i++) {
        const double r = rho[i], u[3] = {ux[i], uy[i], uz[i]}, T = RT[i];
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double m[17];
        m[0] = r;
        for (int a = 0; a < 3; a++) m[1 + a] = r * u[a];
        int k = 4;
        for (int a = 0; a < 3; a++)
            for (int c = a; c < 3; c++) m[k++] = r * (u[a] * u[c] + (a == c ? T : 0.0));
        for (int a = 0; a < 3; a++) m[10 + a] = r * (uu + 5.0 * T) * u[a];    // D + 2 = 5
        m[13] = r * K * T;
        for (int a = 0; a < 3; a++) m[14 + a] = r * K * T * u[a];
        for (int j = 0; j < 17; j++) out[(long)j * n + i] = m[j];
    }
    return LELBM_OK;
}

extern "C" const char *lelbm_strerror(int code) {
    switch (code) {
    case LELBM_OK: return "ok";
    case LELBM_EINVAL: return "invalid argument";
    case LELBM_ENOMEM: return "out of memory";
    case LELBM_EDEVICE: return "HIP device error";
    case LELBM_EEPR: return "entropic reconstruction failed (non-realizable state or Newton failure)";
    case LELBM_ENONFINITE: return "non-finite moments";
    case LELBM_EREACH:
        return "pad narrower than a stencil's reach, stencil out of the supported range, or a no-slip wall reached "
               "beyond what its bounce-back supports";
    default: return "unknown error";
    }
}

static int validate(const lelbm_params *p) {
    if (!p) return LELBM_EINVAL;
    if (p->dim != 1 && p->dim != 2) return LELBM_EINVAL;
    if (p->nz != 0 && p->nz != 1) return LELBM_EINVAL;
    if (p->nx <= 0 || p->ny <= 0 || (p->dim == 1 && p->ny != 1)) return LELBM_EINVAL;
    if (!(p->K > 0.0) || !(p->n_conf > 0.0) || p->r_min < 1) return LELBM_EINVAL;
    if (!(p->newton_tol > 0.0) || p->newton_max_it < 1) return LELBM_EINVAL;
    if (p->precision != LELBM_FP64 && p->precision != LELBM_MIXED) return LELBM_EINVAL;
    if (p->guess != LELBM_GUESS_EQ && p->guess != LELBM_GUESS_MLP && p->guess != LELBM_GUESS_LIN &&
        p->guess != LELBM_GUESS_PREV && p->guess != LELBM_GUESS_MLP_PREV)
        return LELBM_EINVAL;
    if ((p->guess == LELBM_GUESS_MLP || p->guess == LELBM_GUESS_MLP_PREV) && p->dim != 2) return LELBM_EINVAL;
    if (p->solid && p->dim != 2) return LELBM_EINVAL;
    for (int f = 0; f < 4; f++)
        if (p->bc[f] < LELBM_BC_PERIODIC || p->bc[f] > LELBM_BC_WALL) return LELBM_EINVAL;
    // no-slip walls (Sec. III.B): y faces of a 2D domain, without slip walls
    // or solid cells; the wall velocity is tangential (x)
    bool noslip = false;
    for (int f = 0; f < 4; f++) {
        if (!std::isfinite(p->wall_u[f])) return LELBM_EINVAL;
        if (p->bc[f] != LELBM_BC_WALL) {
            if (p->wall_u[f] != 0.0) return LELBM_EINVAL;
            continue;
        }
        if (p->dim != 2 || f < 2) return LELBM_EINVAL;
        noslip = true;
    }
    if (noslip) {
        if (p->solid) return LELBM_EINVAL;
        for (int f = 0; f < 4; f++)
            if (p->bc[f] == LELBM_BC_SLIPWALL) return LELBM_EINVAL;
    }
    for (int ax = 0; ax < p->dim; ax++) {
        int a = p->bc[2 * ax], b = p->bc[2 * ax + 1];
        if ((a == LELBM_BC_PERIODIC) != (b == LELBM_BC_PERIODIC)) return LELBM_EINVAL;
    }
    bool needpad = false;
    for (int f = 0; f < 2 * p->dim; f++)
        if (p->bc[f] == LELBM_BC_OUTFLOW || p->bc[f] == LELBM_BC_INFLOW) needpad = true;
    if (needpad && p->pad < 1) return LELBM_EINVAL;
    if (p->kn_limiter && !(p->kn_hi > p->kn_lo)) return LELBM_EINVAL;
    if (p->src_rate != 0.0) {
        if (!std::isfinite(p->src_rate) || !std::isfinite(p->src_omega) || !std::isfinite(p->src_t0))
            return LELBM_EINVAL;
        if (p->src_x < 0 || p->src_x >= p->nx || p->src_y < 0 || p->src_y >= p->ny) return LELBM_EINVAL;
        if (p->solid && p->solid[(long long)p->src_y * p->nx + p->src_x]) return LELBM_EINVAL;
    }
    return LELBM_OK;
}

// Three dimensions: periodic boxes, the Newton start of Eq. (IID13), its
// linearisation or the previous-step guess; no solids, walls, point sources,
// learned guess or harvest.
static int validate3(const lelbm_params *p) {
    if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return LELBM_EINVAL;
    if (!(p->K > 0.0) || !(p->n_conf > 0.0) || p->r_min < 1) return LELBM_EINVAL;
    if (!(p->newton_tol > 0.0) || p->newton_max_it < 1) return LELBM_EINVAL;
    if (p->precision != LELBM_FP64 && p->precision != LELBM_MIXED) return LELBM_EINVAL;
    if (p->guess != LELBM_GUESS_EQ && p->guess != LELBM_GUESS_LIN && p->guess != LELBM_GUESS_PREV)
        return LELBM_EINVAL;
    for (int f = 0; f < 4; f++)
        if (p->bc[f] != LELBM_BC_PERIODIC || p->wall_u[f] != 0.0) return LELBM_EINVAL;
    if (p->solid || p->src_rate != 0.0) return LELBM_EINVAL;
    if (p->kn_limiter && !(p->kn_hi > p->kn_lo)) return LELBM_EINVAL;
    return LELBM_OK;
}

static void free_ctx(lelbm_ctx *c) {
    if (!c) return;
    if (c->c3) ctx3_destroy(c->c3);
    c->c3 = nullptr;
    Buffers &b = c->b;
    void *ptrs[] = {b.mom[0], b.mom[1], b.desc_u, b.desc_rho, b.desc_rt, b.desc_rn, b.spans, b.tiles,
                    b.dwin, b.scratch, b.flags, b.stats, b.partial, b.harvest_n,
                    c->mlp_w, c->mlp_p, c->mlp_n, (void *)b.solid, (void *)b.tdist, b.maxreach, (void *)b.cdist, (void *)b.tdist_s, b.wcache, (void *)b.wslot, b.wbuilt, b.lamprev,
                    b.bpart, b.gpart, b.order, b.rlist, b.rcount, b.bands, b.wflag, b.wimg, b.wreach};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    for (hipEvent_t e : c->opev) (void)hipEventDestroy(e);
    for (hipStream_t q : c->side)
        if (q) (void)hipStreamDestroy(q);
    if (c->ev[0]) (void)hipEventDestroy(c->ev[0]);
    if (c->ev[1]) (void)hipEventDestroy(c->ev[1]);
    for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
    stage_free(c->stage);
    delete c;
}

static int reset_flags(lelbm_ctx *c) {
    HIPCHECK(launch_reset_flags(c->b.flags, c->stream));
    return LELBM_OK;
}

// Makes the population scratch hold at least `need` elements (the band
// plan sizes its slots with room to spare).
static int grow_scratch(lelbm_ctx *c, long long need) {
    if (need <= c->b.scratch_cap) return LELBM_OK;
    long long cap = need;
    size_t esz = c->mixed ? sizeof(float) : sizeof(double);
    HIPCHECK(hipStreamSynchronize(c->stream));
    if (c->b.scratch) HIPCHECK(hipFree(c->b.scratch));
    c->b.scratch = nullptr;
    c->b.scratch_cap = 0;
    if (hipMalloc(&c->b.scratch, (size_t)cap * esz) != hipSuccess) { c->b.scratch = nullptr; return LELBM_ENOMEM; }
    c->b.scratch_cap = cap;
    return LELBM_OK;
}

// Solid cells and slip walls block population paths.  The device gets the
// mask and, per destination tile, the Chebyshev distance from the tile to the
// nearest blocker (a solid cell, or the cell just beyond a slip wall), so the
// gather can tell the tiles that need path tracing.  Solids may not touch a
// pad face: pad cells copy the nearest interior cell.
static int setup_blockers(lelbm_ctx *c, const unsigned char *mask) {
    const Geom &g = c->g;
    const int nx = g.nx, ny = g.ny;
    bool walls = false;
    for (int f = 0; f < 2 * g.dim; f++) walls = walls || g.bc[f] == LELBM_BC_SLIPWALL;
    if (!mask && !walls) return LELBM_OK;
    const long long n = (long long)nx * ny;
    const int INF = 1 << 28;
    std::vector<int> d((size_t)n, INF);
    if (mask) {
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                if (!mask[(long long)y * nx + x]) continue;
                if ((x == 0 && g.wl) || (x == nx - 1 && g.wr) || (y == 0 && g.wb) || (y == ny - 1 && g.wt))
                    return LELBM_EINVAL;
                d[(long long)y * nx + x] = 0;
            }
        // Chebyshev distance transform: forward and backward sweeps over the
        // 8-neighbourhood (periodic axes wrap), repeated until stable
        const bool px = g.bc[0] == LELBM_BC_PERIODIC, py = g.bc[2] == LELBM_BC_PERIODIC;
        auto relax = [&](int x, int y, int ddx, int ddy, bool &chg) {
            int xx = x + ddx, yy = y + ddy;
            if (px) xx = (xx + nx) % nx;
            if (py) yy = (yy + ny) % ny;
            if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) return;
            int v = d[(long long)yy * nx + xx] + 1;
            int &me = d[(long long)y * nx + x];
            if (v < me) { me = v; chg = true; }
        };
        bool stable = false;
        for (int round = 0; round < 64 && !stable; round++) {
            bool chg = false;
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    relax(x, y, -1, 0, chg); relax(x, y, -1, -1, chg); relax(x, y, 0, -1, chg); relax(x, y, 1, -1, chg);
                }
            for (int y = ny - 1; y >= 0; y--)
                for (int x = nx - 1; x >= 0; x--) {
                    relax(x, y, 1, 0, chg); relax(x, y, 1, 1, chg); relax(x, y, 0, 1, chg); relax(x, y, -1, 1, chg);
                }
            stable = !chg;
        }
        // not settled: no distance is trusted (every cell traces its paths)
        if (!stable) std::fill(d.begin(), d.end(), 0);
    }
    const int nd = g.dtx * g.dty;
    std::vector<int> td((size_t)nd, INF), tds((size_t)nd, INF);
    std::vector<unsigned short> cd((size_t)n);
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            int v = d[(long long)y * nx + x];
            int &ts = tds[(size_t)(y / g.ty) * g.dtx + x / g.tx];
            ts = std::min(ts, v);
            if (g.bc[0] == LELBM_BC_SLIPWALL) v = std::min(v, x + 1);
            if (g.bc[1] == LELBM_BC_SLIPWALL) v = std::min(v, nx - x);
            if (g.dim == 2 && g.bc[2] == LELBM_BC_SLIPWALL) v = std::min(v, y + 1);
            if (g.dim == 2 && g.bc[3] == LELBM_BC_SLIPWALL) v = std::min(v, ny - y);
            int &t = td[(size_t)(y / g.ty) * g.dtx + x / g.tx];
            t = std::min(t, v);
            cd[(size_t)y * nx + x] = (unsigned short)std::min(v, 65535);
        }
    Buffers &b = c->b;
    int *dt = nullptr, *dts = nullptr;
    unsigned short *cdv = nullptr;
    unsigned char *sm = nullptr;
    if (hipMalloc((void **)&dt, (size_t)nd * sizeof(int)) != hipSuccess) return LELBM_ENOMEM;
    b.tdist = dt;
    if (hipMalloc((void **)&cdv, (size_t)n * sizeof(unsigned short)) != hipSuccess) return LELBM_ENOMEM;
    b.cdist = cdv;
    if (hipMalloc((void **)&dts, (size_t)nd * sizeof(int)) != hipSuccess) return LELBM_ENOMEM;
    b.tdist_s = dts;
    int r = stage_h2d(c->stage, c->stream, dt, td.data(), (size_t)nd * sizeof(int));
    if (r != LELBM_OK) return r;
    r = stage_h2d(c->stage, c->stream, cdv, cd.data(), (size_t)n * sizeof(unsigned short));
    if (r != LELBM_OK) return r;
    r = stage_h2d(c->stage, c->stream, dts, tds.data(), (size_t)nd * sizeof(int));
    if (r != LELBM_OK) return r;
    // cache of backward-walk results for the tiles that can need walks at a
    // reach up to WCACHE_M (fluid tiles near a solid; near a slip wall only
    // where the domain is narrow enough for a double reflection); without
    // the memory for it the walks run every step
    {
        const bool wx = g.bc[0] == LELBM_BC_SLIPWALL || g.bc[1] == LELBM_BC_SLIPWALL;
        const bool wy = g.dim == 2 && (g.bc[2] == LELBM_BC_SLIPWALL || g.bc[3] == LELBM_BC_SLIPWALL);
        const bool narrow = (wx && nx <= 2 * WCACHE_M + 2) || (wy && ny <= 2 * WCACHE_M + 2);
        std::vector<char> fluid_tile((size_t)nd, 0);
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++)
                if (!mask || !mask[(long long)y * nx + x]) fluid_tile[(size_t)(y / g.ty) * g.dtx + x / g.tx] = 1;
        std::vector<int> slot((size_t)nd, -1);
        int nslots = 0;
        for (int t = 0; t < nd; t++)
            if (fluid_tile[t] && (narrow ? td[t] : tds[t]) <= WCACHE_M + 1) slot[t] = nslots++;
        const size_t cbytes = (size_t)nslots * WCACHE_W * WCACHE_W * TILE_N * sizeof(unsigned short);
        int *ws = nullptr, *wb = nullptr;
        unsigned short *wc = nullptr;
        // at most an eighth of the free device memory: the record scratch
        // grows with the temperature and takes precedence
        size_t mfree = 0, mtotal = 0;
        const bool room = hipMemGetInfo(&mfree, &mtotal) == hipSuccess && cbytes <= mfree / 8;
        if (nslots > 0 && room && hipMalloc((void **)&wc, cbytes) == hipSuccess) {
            if (hipMalloc((void **)&ws, (size_t)nd * sizeof(int)) != hipSuccess ||
                hipMalloc((void **)&wb, sizeof(int)) != hipSuccess)
                return LELBM_ENOMEM;
            b.wcache = wc;
            b.wslot = ws;
            b.wbuilt = wb;
            if ((r = stage_h2d(c->stage, c->stream, ws, slot.data(), (size_t)nd * sizeof(int))) != LELBM_OK) return r;
            if (hipMemsetAsync(wb, 0xff, sizeof(int), c->stream) != hipSuccess) return LELBM_EDEVICE;
            c->persistent_bytes += (long long)cbytes + (long long)nd * sizeof(int);
        } else {
            (void)hipGetLastError();
        }
    }
    c->persistent_bytes += n * (long long)sizeof(unsigned short);
    if (mask) {
        if (hipMalloc((void **)&sm, (size_t)n) != hipSuccess) return LELBM_ENOMEM;
        b.solid = sm;
        r = stage_h2d(c->stage, c->stream, sm, mask, (size_t)n);
        if (r != LELBM_OK) return r;
        c->persistent_bytes += n;
    }
    c->persistent_bytes += (long long)2 * nd * sizeof(int);
    return LELBM_OK;
}

static int create_common(const lelbm_params *p, void *stream, lelbm_ctx **out, lelbm_ctx **cc) {
    int v = validate(p);
    if (v != LELBM_OK) return v;
    if (!out) return LELBM_EINVAL;
    lelbm_ctx *c = new (std::nothrow) lelbm_ctx();
    if (!c) return LELBM_ENOMEM;
    memset(&c->b, 0, sizeof(c->b));
    c->c3 = nullptr;
    c->ev[0] = c->ev[1] = nullptr;
    c->side[0] = c->side[1] = c->side[2] = nullptr;
    c->mlp_w = nullptr;
    c->mlp_p = nullptr;
    c->mlp_n = nullptr;
    c->mlp_set = 0;
    c->p = *p;
    c->p.solid = nullptr;      // the mask is copied to the device below
    c->mixed = p->precision == LELBM_MIXED;
    c->nmom = lelbm_num_moments(p->dim);
    c->stream = (hipStream_t)stream;
    c->cur = 0;
    c->last_fail_node = -1;
    c->last_fail_step = -1;
    c->last_fail_detail = 0;
    c->last_fail_species = -1;
    c->last_fail_residual = 0.0;
    c->timing = 0;
    c->evused = 0;
    // gather staging capacity (LDS per workgroup = 28 B x gcap); the
    // LELBM_GATHER_CAP environment variable overrides it for tuning
    c->gcap = GATHER_CAP;
    if (const char *e = getenv("LELBM_GATHER_CAP")) {
        int v = atoi(e);
        if (v >= 256 && v <= GATHER_CAP_MAX) c->gcap = v;
    }
    for (int k = 0; k < LELBM_NTIMERS; k++) { c->kms[k] = 0; c->klaunch[k] = 0; }
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return LELBM_EDEVICE; }
    Geom &g = c->g;
    memset(&g, 0, sizeof(g));
    g.dim = p->dim; g.nx = p->nx; g.ny = p->ny;
    for (int f = 0; f < 4; f++) g.bc[f] = f < 2 * p->dim ? p->bc[f] : LELBM_BC_PERIODIC;
    auto padw = [&](int f) { return (g.bc[f] == LELBM_BC_OUTFLOW || g.bc[f] == LELBM_BC_INFLOW) ? p->pad : 0; };
    g.wl = padw(0); g.wr = padw(1);
    g.wb = p->dim == 2 ? padw(2) : 0; g.wt = p->dim == 2 ? padw(3) : 0;
    g.sxn = g.nx + g.wl + g.wr;
    g.syn = g.ny + g.wb + g.wt;
    g.ns = (long long)g.sxn * g.syn;
    if (p->dim == 2) { g.tx = tile_x<2>(); g.ty = tile_y<2>(); }
    else { g.tx = tile_x<1>(); g.ty = tile_y<1>(); }
    g.ntx = (g.sxn + g.tx - 1) / g.tx; g.nty = (g.syn + g.ty - 1) / g.ty;
    g.dtx = (g.nx + g.tx - 1) / g.tx; g.dty = (g.ny + g.ty - 1) / g.ty;
    const bool noslip = p->dim == 2 && (g.bc[2] == LELBM_BC_WALL || g.bc[3] == LELBM_BC_WALL);
    g.wrows = noslip ? std::min(g.ny, LELBM_WALL_ROWS) : 0;
    Phys &ph = c->ph;
    ph.K = p->K; ph.omega_f = p->omega_f; ph.omega_b = p->omega_b; ph.omega_h = p->omega_h;
    ph.n_conf = p->n_conf; ph.r_min = p->r_min; ph.tol = p->newton_tol; ph.maxit = p->newton_max_it;
    // the mixed path stores FP32 moment fractions (relative rounding 6e-8), so
    // converging the multipliers beyond 1e-8 buys nothing
    if (p->precision == LELBM_MIXED && ph.tol < MIXED_TOL_FLOOR) ph.tol = MIXED_TOL_FLOOR;
    ph.kn_limiter = p->kn_limiter; ph.kn_lo = p->kn_lo; ph.kn_hi = p->kn_hi; ph.omega_H = p->omega_H;
    ph.kn_lo_lin = pow(10.0, p->kn_lo); ph.kn_hi_lin = pow(10.0, p->kn_hi);
    ph.in_rho = p->in_rho; ph.in_u[0] = p->in_u[0]; ph.in_u[1] = p->dim == 2 ? p->in_u[1] : 0.0;
    ph.in_RT = p->in_RT;
    ph.lin_guess = p->guess == LELBM_GUESS_LIN;
    ph.prev_guess = p->guess == LELBM_GUESS_PREV || p->guess == LELBM_GUESS_MLP_PREV;
    ph.src_node = p->src_rate != 0.0 ? (long long)(p->src_y + g.wb) * g.sxn + (p->src_x + g.wl) : -1;
    ph.src_mass = 0.0;
    ph.wall_ux[0] = p->dim == 2 ? p->wall_u[2] : 0.0;
    ph.wall_ux[1] = p->dim == 2 ? p->wall_u[3] : 0.0;
    c->ph_step = ph;
    c->steps_done = 0;

    Buffers &b = c->b;
    long long ns = g.ns;
    int nt = g.ntx * g.nty, nd = g.dtx * g.dty;
    bool ok = true;
    ok = ok && hipMalloc((void **)&b.mom[0], (size_t)c->nmom * ns * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.mom[1], (size_t)c->nmom * ns * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.desc_u, (size_t)2 * ns * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.desc_rho, (size_t)ns * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.desc_rt, (size_t)ns * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.desc_rn, (size_t)ns * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.spans, (size_t)nt * TILE_N * SPAN_ROWS * sizeof(unsigned short)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.tiles, (size_t)nt * sizeof(TileInfo)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.dwin, (size_t)nd * sizeof(DWin)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.flags, sizeof(Flags)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.stats, sizeof(DevStats)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.partial, (size_t)(num_sum_blocks(g) + 1) * 4 * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.harvest_n, sizeof(unsigned long long)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.bpart, (size_t)2 * nt * sizeof(DevStats)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.order, (size_t)nt * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.rlist, (size_t)nt * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.rcount, (size_t)g.nty * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.maxreach, sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b.bands, (size_t)g.nty * sizeof(BandInfo)) == hipSuccess;
    // arrival partials of the straight gather and of the backward-walk gather
    ok = ok && hipMalloc((void **)&b.gpart, (size_t)5 * gather_blocks_x(g) * gather_blocks_y(g) *
                                                sizeof(unsigned long long)) == hipSuccess;
    if (p->guess == LELBM_GUESS_PREV || p->guess == LELBM_GUESS_MLP_PREV) {
        ok = ok && hipMalloc((void **)&b.lamprev, (size_t)16 * ns * sizeof(double)) == hipSuccess;
        // all-ones bytes are a NaN: no stored correction yet
        ok = ok && hipMemset(b.lamprev, 0xff, (size_t)16 * ns * sizeof(double)) == hipSuccess;
    }
    if (g.wrows > 0) {
        // image store of the no-slip walls: both faces, g.wrows rows each
        const long long we = 2ll * g.wrows * g.sxn;
        ok = ok && hipMalloc((void **)&b.wflag, (size_t)we * sizeof(int)) == hipSuccess;
        ok = ok && hipMalloc((void **)&b.wimg, (size_t)we * WALL_REC * sizeof(double)) == hipSuccess;
        ok = ok && hipMalloc((void **)&b.wreach, sizeof(int)) == hipSuccess;
        ok = ok && hipMemset(b.wflag, 0, (size_t)we * sizeof(int)) == hipSuccess;
    }
    if (p->guess == LELBM_GUESS_MLP || p->guess == LELBM_GUESS_MLP_PREV) {
        ok = ok && hipMalloc((void **)&c->mlp_w, MLP_NPARAM * sizeof(unsigned short)) == hipSuccess;
        ok = ok && hipMalloc((void **)&c->mlp_p, MLP_NPARAM * sizeof(float)) == hipSuccess;
        ok = ok && hipMalloc((void **)&c->mlp_n, MLP_NORM * sizeof(float)) == hipSuccess;
    }
    if (!ok) { free_ctx(c); return LELBM_ENOMEM; }
    c->persistent_bytes = (long long)2 * c->nmom * ns * sizeof(double) + ns * (4 * sizeof(double) + sizeof(int)) +
                          nt * sizeof(TileInfo) + nd * sizeof(DWin) +
                          (b.lamprev ? (long long)16 * ns * sizeof(double) : 0) +
                          (long long)2 * g.wrows * g.sxn * (WALL_REC * sizeof(double) + sizeof(int));
    int r = setup_blockers(c, p->solid);
    if (r != LELBM_OK) { free_ctx(c); return r; }
    if (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side[0], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side[1], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side[2], hipStreamNonBlocking) != hipSuccess) {
        free_ctx(c);
        return LELBM_EDEVICE;
    }
    if (reset_flags(c) != LELBM_OK) { free_ctx(c); return LELBM_EDEVICE; }
    // pinned staging for flags, statistics and band plans, and room for the
    // plans' host arrays, reserved here so that stepping never has to
    // allocate them
    if (stage_reserve(c->stage, 4096 + (size_t)g.nty * sizeof(BandInfo)) != LELBM_OK) {
        free_ctx(c);
        return LELBM_ENOMEM;
    }
    for (Plan *P : {&c->plan, &c->fixed_plan}) {
        P->bands.reserve((size_t)g.nty);
        P->slot_of.reserve((size_t)g.nty);
        P->ops.reserve((size_t)4 * g.nty + 8);
        P->gdeps.reserve((size_t)16 * g.nty + 16);
        P->w_order.reserve((size_t)g.nty);
        P->w_int.reserve((size_t)4 * g.nty);
        P->w_flags.reserve((size_t)4 * g.nty + (size_t)g.dty);
    }
    c->budget = LELBM_DEFAULT_SCRATCH_BUDGET;
    *cc = c;
    return LELBM_OK;
}

// Copies interior moments (SoA [nmom][ny][nx], FP64 or FP32, on the host or
// the device) into the padded FP64 state buffer.  Host data is widened row by
// row into the pinned stage; device data is copied (and widened) by a kernel.
static int upload_interior(lelbm_ctx *c, const void *src, int src_fp32, hipMemcpyKind kind) {
    const Geom &g = c->g;
    const size_t esz = sizeof(double);
    const long long n = (long long)g.nx * g.ny;
    if (kind == hipMemcpyDeviceToDevice) {
        HIPCHECK(launch_load_interior(g, c->nmom, src, src_fp32, c->b.mom[c->cur], c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
        return LELBM_OK;
    }
    const size_t rowb = (size_t)g.nx * esz;
    const long long rows_per = (long long)(STAGE_MAX / rowb) > 0 ? (long long)(STAGE_MAX / rowb) : 1;
    int r = stage_reserve(c->stage, (size_t)(rows_per < g.ny ? rows_per : g.ny) * rowb);
    if (r != LELBM_OK) return r;
    for (int k = 0; k < c->nmom; k++) {
        for (long long y0 = 0; y0 < g.ny; y0 += rows_per) {
            const long long ny = g.ny - y0 < rows_per ? g.ny - y0 : rows_per;
            const long long e0 = (long long)k * n + y0 * g.nx, ne = ny * g.nx;
            for (long long i = 0; i < ne; i++)
                ((double *)c->stage.p)[i] = src_fp32 ? (double)((const float *)src)[e0 + i] : ((const double *)src)[e0 + i];
            char *dst = (char *)c->b.mom[c->cur] + ((size_t)k * g.ns + (size_t)(y0 + g.wb) * g.sxn + g.wl) * esz;
            HIPCHECK(hipMemcpy2DAsync(dst, (size_t)g.sxn * esz, c->stage.p, rowb, rowb, (size_t)ny,
                                      hipMemcpyHostToDevice, c->stream));
            HIPCHECK(hipStreamSynchronize(c->stream));
        }
    }
    return LELBM_OK;
}

static int upload_plan(lelbm_ctx *c, Plan &P) {
    if (P.uploaded) return LELBM_OK;
    int r = stage_h2d(c->stage, c->stream, c->b.bands, P.bands.data(), P.bands.size() * sizeof(BandInfo));
    if (r != LELBM_OK) return r;
    c->plan.uploaded = c->fixed_plan.uploaded = false;   // the device table holds one plan at a time
    P.uploaded = true;
    return LELBM_OK;
}

static int finish_create(lelbm_ctx *c) {
    // initial scratch: run the pre-pass once to size it
    hipStream_t s = c->stream;
    HIPCHECK(launch_zero_solid(c->g, c->nmom, c->b.mom[c->cur], c->b.solid, s));
    HIPCHECK(launch_fill_pads(c->g, c->ph, c->b.mom[c->cur], c->b.flags, s));
    HIPCHECK(launch_reset_step(c->g, c->b, s));
    HIPCHECK(launch_prepare(c->g, c->ph, c->b.mom[c->cur], c->b, 0, s));
    // one band of all rows with an empty slot: the scan reports the records
    // of the whole domain
    build_plan(plan_geom(c->g), c->plan, c->g.nty, 0);
    c->plan.slot_cap = 0;
    set_bases(c->plan);
    int rr = upload_plan(c, c->plan);
    if (rr != LELBM_OK) return rr;
    HIPCHECK(launch_scan(c->g, c->b, (int)c->plan.bands.size(), c->plan.slot_cap, c->plan.m_plan, 0, s));
    Flags f;
    rr = stage_d2h(c->stage, s, &f, c->b.flags, sizeof(Flags));
    if (rr != LELBM_OK) return rr;
    if (f.err == ERR_OVERFLOW) {
        // the first plan: one band if the whole domain's records fit the
        // budget, else bands
        const size_t esz = c->mixed ? sizeof(float) : sizeof(double);
        const long long limit = std::max<long long>(c->budget / (long long)esz, 1);
        plan_first(plan_geom(c->g), c->plan, limit, f.need, f.reach);
        int r = grow_scratch(c, (long long)c->plan.nslots * c->plan.slot_cap);
        if (r != LELBM_OK) return r;
    } else if (f.err != 0) {
        c->last_fail_node = (long)f.node;
        c->last_fail_step = -1;
        if (getenv("LELBM_DEBUG")) {
            fprintf(stderr, "lelbm: create pre-pass failed: err %d node %lld step %d\n", f.err, f.node, f.step);
            if (f.node >= 0 && f.node < c->g.ns) {
                for (int k = 0; k < c->nmom; k++) {
                    double v = 0.0;
                    const double *src = c->b.mom[c->cur] + (size_t)k * c->g.ns + (size_t)f.node;
                    if (stage_d2h(c->stage, s, &v, src, sizeof(double)) == LELBM_OK)
                        fprintf(stderr, "  moment %d = %.17g\n", k, v);
                }
            }
        }
        return f.err;
    }
    return reset_flags(c);
}

// A 3D context: the shell of lelbm_ctx (stream, timing, failure record)
// around the 3D path's own buffers.
static int create3(const lelbm_params *p, const void *moments, int src_fp32, int on_device, void *hip_stream,
                   lelbm_ctx **out) {
    int v = validate3(p);
    if (v != LELBM_OK) return v;
    if (!out) return LELBM_EINVAL;
    lelbm_ctx *c = new (std::nothrow) lelbm_ctx();
    if (!c) return LELBM_ENOMEM;
    memset(&c->b, 0, sizeof(c->b));
    c->c3 = nullptr;
    c->ev[0] = c->ev[1] = nullptr;
    c->side[0] = c->side[1] = c->side[2] = nullptr;
    c->mlp_w = nullptr; c->mlp_p = nullptr; c->mlp_n = nullptr; c->mlp_set = 0;
    c->c3 = nullptr;
    c->p = *p;
    c->mixed = p->precision == LELBM_MIXED;
    c->nmom = 17;
    c->stream = (hipStream_t)hip_stream;
    c->last_fail_node = -1; c->last_fail_step = -1; c->last_fail_detail = 0; c->last_fail_species = -1;
    c->last_fail_residual = 0.0;
    c->timing = 0;
    c->evused = 0;
    for (int k = 0; k < LELBM_NTIMERS; k++) { c->kms[k] = 0; c->klaunch[k] = 0; }
    c->budget = LELBM_DEFAULT_SCRATCH_BUDGET;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return LELBM_EDEVICE; }
    Phys &ph = c->ph;
    memset(&ph, 0, sizeof(ph));
    ph.K = p->K; ph.omega_f = p->omega_f; ph.omega_b = p->omega_b; ph.omega_h = p->omega_h;
    ph.n_conf = p->n_conf; ph.r_min = p->r_min; ph.tol = p->newton_tol; ph.maxit = p->newton_max_it;
    if (c->mixed && ph.tol < MIXED_TOL_FLOOR) ph.tol = MIXED_TOL_FLOOR;
    ph.kn_limiter = p->kn_limiter; ph.kn_lo = p->kn_lo; ph.kn_hi = p->kn_hi; ph.omega_H = p->omega_H;
    ph.kn_lo_lin = pow(10.0, p->kn_lo); ph.kn_hi_lin = pow(10.0, p->kn_hi);
    ph.src_node = -1;
    ph.lin_guess = p->guess == LELBM_GUESS_LIN;
    ph.prev_guess = p->guess == LELBM_GUESS_PREV;
    c->ph_step = ph;
    int r = ctx3_create(p, ph, c->mixed, moments, src_fp32, on_device, c->stream, &c->c3);
    if (r != LELBM_OK) { free_ctx(c); return r; }
    long long pb = 0;
    ctx3_memory(c->c3, &pb, nullptr);
    c->persistent_bytes = pb;
    *out = c;
    return LELBM_OK;
}

extern "C" int lelbm_create(const lelbm_params *p, const double *moments, void *hip_stream, lelbm_ctx **out) {
    if (!moments) return LELBM_EINVAL;
    if (p && p->dim == 3) return create3(p, moments, 0, 0, hip_stream, out);
    lelbm_ctx *c = nullptr;
    int r = create_common(p, hip_stream, out, &c);
    if (r != LELBM_OK) return r;
    r = upload_interior(c, moments, 0, hipMemcpyHostToDevice);
    if (r == LELBM_OK) r = finish_create(c);
    if (r != LELBM_OK) { free_ctx(c); return r; }
    *out = c;
    return LELBM_OK;
}

extern "C" int lelbm_create_device(const lelbm_params *p, const void *dev_moments, int dev_is_fp32,
                                   void *hip_stream, lelbm_ctx **out) {
    if (!dev_moments) return LELBM_EINVAL;
    if (p && p->dim == 3) return create3(p, dev_moments, dev_is_fp32, 1, hip_stream, out);
    lelbm_ctx *c = nullptr;
    int r = create_common(p, hip_stream, out, &c);
    if (r != LELBM_OK) return r;
    r = upload_interior(c, dev_moments, dev_is_fp32, hipMemcpyDeviceToDevice);
    if (r == LELBM_OK) r = finish_create(c);
    if (r != LELBM_OK) { free_ctx(c); return r; }
    *out = c;
    return LELBM_OK;
}

static int timed(lelbm_ctx *c, int k, hipError_t (*fn)(lelbm_ctx *, void *), void *arg,
                 hipStream_t st = nullptr) {
    if (!st) st = c->stream;
    if (!c->timing) {
        HIPCHECK(fn(c, arg));
        return LELBM_OK;
    }
    size_t i = c->evused;
    while (c->evpool.size() < 2 * (i + 1)) {
        hipEvent_t e;
        HIPCHECK(hipEventCreate(&e));
        c->evpool.push_back(e);
    }
    if (c->evkind.size() < i + 1) c->evkind.resize(i + 1);
    HIPCHECK(hipEventRecord(c->evpool[2 * i], st));
    HIPCHECK(fn(c, arg));
    HIPCHECK(hipEventRecord(c->evpool[2 * i + 1], st));
    c->evkind[i] = k;
    c->evused = i + 1;
    return LELBM_OK;
}

// Accumulates the recorded kernel durations (after a stream synchronisation).
static int collect_times(lelbm_ctx *c) {
    for (size_t i = 0; i < c->evused; i++) {
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, c->evpool[2 * i], c->evpool[2 * i + 1]));
        c->kms[c->evkind[i]] += ms;
        c->klaunch[c->evkind[i]]++;
    }
    c->evused = 0;
    return LELBM_OK;
}

struct StepArg {
    int step;
    const Plan *plan;
    int a, n;        // band / block rows of the operation
    hipStream_t gs;  // stream of the gathers
    hipStream_t es;  // stream of the operation's reconstruction (narrow and refined stencils)
    hipStream_t ws;  // stream of the wide stencils' reconstruction
};

static hipError_t do_fill(lelbm_ctx *c, void *) {
    return launch_fill_pads(c->g, c->ph, c->b.mom[c->cur], c->b.flags, c->stream);
}
static hipError_t do_prepare(lelbm_ctx *c, void *a) {
    hipError_t e = launch_reset_step(c->g, c->b, c->stream);
    if (e != hipSuccess) return e;
    return launch_prepare(c->g, c->ph, c->b.mom[c->cur], c->b, ((StepArg *)a)->step, c->stream);
}
static hipError_t do_scan(lelbm_ctx *c, void *a) {
    const StepArg &s = *(StepArg *)a;
    return launch_scan(c->g, c->b, (int)s.plan->bands.size(), s.plan->slot_cap, s.plan->m_plan, s.step, c->stream);
}
static hipError_t do_epr(lelbm_ctx *c, void *a) {
    const StepArg &s = *(StepArg *)a;
    const BandInfo &bd = s.plan->bands[s.a];
    return launch_epr(c->g, c->ph_step, c->mixed, c->b.mom[c->cur], c->b, s.step, bd.row0 * c->g.ntx,
                      (bd.row1 - bd.row0) * c->g.ntx, 0, s.es);
}
static hipError_t do_epr_wide(lelbm_ctx *c, void *a) {
    const StepArg &s = *(StepArg *)a;
    const BandInfo &bd = s.plan->bands[s.a];
    return launch_epr(c->g, c->ph_step, c->mixed, c->b.mom[c->cur], c->b, s.step, bd.row0 * c->g.ntx,
                      (bd.row1 - bd.row0) * c->g.ntx, 1, s.ws);
}
static hipError_t do_epr_ref(lelbm_ctx *c, void *a) {
    const StepArg &s = *(StepArg *)a;
    const BandInfo &bd = s.plan->bands[s.a];
    return launch_epr_ref(c->g, c->ph_step, c->mixed, c->b.mom[c->cur], c->b, s.step, bd.row0 * c->g.ntx,
                          (bd.row1 - bd.row0) * c->g.ntx, s.a, s.es);
}
static hipError_t do_wall_image(lelbm_ctx *c, void *a) {
    const StepArg &s = *(StepArg *)a;
    const BandInfo &bd = s.plan->bands[s.a];
    return launch_wall_image(c->g, c->ph_step, c->mixed, c->b.mom[c->cur], c->b, s.step, bd.row0 * c->g.ntx,
                             (bd.row1 - bd.row0) * c->g.ntx, s.es);
}
static hipError_t do_wall_gather(lelbm_ctx *c, void *) {
    return launch_wall_gather(c->g, c->b.mom[c->cur ^ 1], c->b, c->stream);
}
static hipError_t do_gather(lelbm_ctx *c, void *a) {
    const StepArg &s = *(StepArg *)a;
    return launch_gather(c->g, c->mixed, c->b.mom[c->cur ^ 1], c->b, c->gcap, s.a, s.n, s.gs);
}
static hipError_t do_totals(lelbm_ctx *c, void *) { return launch_step_totals(c->g, c->b, c->stream); }

// The steps of lelbm_step and lelbm_step_noalloc.  With fixed_scratch the
// record scratch is that fixed buffer (fixed_cap elements, with its own band
// plan) and nothing is allocated: a step whose bands of one tile row do not
// fit fails with LELBM_ENOMEM, keeping the state of the last completed step,
// and no timing events are recorded.
static int step_impl(lelbm_ctx *c, int nsteps, lelbm_stats *st, void *fixed_scratch, long long fixed_cap) {
    if (!c || nsteps < 0) return LELBM_EINVAL;
    if ((c->p.guess == LELBM_GUESS_MLP || c->p.guess == LELBM_GUESS_MLP_PREV) && !c->mlp_set) return LELBM_EINVAL;
    const bool noalloc = fixed_scratch != nullptr;
    if (noalloc && c->stage.cap < sizeof(DevStats) + sizeof(Flags)) return LELBM_EINVAL;
    hipStream_t s = c->stream;
    int r = reset_flags(c);
    if (r != LELBM_OK) return r;
    HIPCHECK(launch_reset_stats(c->b, s));
    // With noalloc the steps run on the static scratch, without timing; the
    // context's own scratch and timing mode are restored on every return.
    // (Without noalloc nothing is swapped: the context's scratch may grow
    // during the call and must stay the one it owns.)
    struct Swap {
        lelbm_ctx *c;
        bool on;
        void *p;
        long long cap;
        int timing;
        ~Swap() {
            if (!on) return;
            c->b.scratch = p;
            c->b.scratch_cap = cap;
            c->timing = timing;
        }
    } keep{c, noalloc, c->b.scratch, c->b.scratch_cap, c->timing};
    Plan &P = noalloc ? c->fixed_plan : c->plan;
    const size_t esz = c->mixed ? sizeof(float) : sizeof(double);
    const long long limit = noalloc ? fixed_cap : std::max<long long>(c->budget / (long long)esz, 1);
    if (noalloc) {
        c->b.scratch = fixed_scratch;
        c->b.scratch_cap = fixed_cap;
        c->timing = 0;
        if (P.rows == 0) {
            // first call: the context's own plan, its slots shrunk to the array
            P = c->plan;
            P.slot_cap = std::min(P.slot_cap, limit / P.nslots);
            set_bases(P);
        }
    }
    if ((r = upload_plan(c, P)) != LELBM_OK) return r;
    int base = 0;   // first step not known to be complete
    while (base < nsteps) {
        int cur0 = c->cur;
        // banded plans run on four streams; a plan of one band, or a
        // no-alloc call without enough events, runs on the caller's stream.
        // Events: 2 i after the narrow and refined stencils (or the gather)
        // of op i, 2 i + 1 after its wide stencils, 2 nops at the step's
        // start.
        const size_t nops = P.ops.size();
        if (!noalloc && nops > 2) {
            while (c->opev.size() < 2 * nops + 1) {
                hipEvent_t e;
                HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                c->opev.push_back(e);
            }
        }
        const bool multi = nops > 2 && c->opev.size() >= 2 * nops + 1;
        for (int k = base; k < nsteps; k++) {
            StepArg a{k, &P, 0, 0, multi ? c->side[1] : s, s, multi ? c->side[2] : s};
            // mass of a point source in this step (Eq. VC1 at the step's
            // collision time, Delta t = 1)
            c->ph_step.src_mass =
                c->ph.src_node >= 0 ? c->p.src_rate * sin(c->p.src_omega * (c->p.src_t0 + (double)(c->steps_done + k)))
                                    : 0.0;
            if ((r = timed(c, 0, do_fill, &a)) != LELBM_OK) return r;
            if ((r = timed(c, 1, do_prepare, &a)) != LELBM_OK) return r;
            if ((r = timed(c, 2, do_scan, &a)) != LELBM_OK) return r;
            if (multi) {
                HIPCHECK(hipEventRecord(c->opev[2 * nops], s));   // the step's descriptors and plan are ready
                HIPCHECK(hipStreamWaitEvent(c->side[0], c->opev[2 * nops], 0));
                HIPCHECK(hipStreamWaitEvent(c->side[2], c->opev[2 * nops], 0));
            }
            int last_odd = -1, last_wide = -1;
            for (size_t i = 0; i < nops; i++) {
                const Op &op = P.ops[i];
                a.a = op.a;
                a.n = op.n;
                if (op.kind == OP_EPR) {
                    a.es = multi && (op.a & 1) ? c->side[0] : s;
                    if (multi && op.dep >= 0) {
                        HIPCHECK(hipStreamWaitEvent(a.es, c->opev[2 * op.dep], 0));
                        HIPCHECK(hipStreamWaitEvent(a.ws, c->opev[2 * op.dep], 0));
                    }
                    if ((r = timed(c, 3, do_epr, &a, a.es)) != LELBM_OK) return r;
                    if ((r = timed(c, 7, do_epr_ref, &a, a.es)) != LELBM_OK) return r;
                    if ((r = timed(c, 3, do_epr_wide, &a, a.ws)) != LELBM_OK) return r;
                    if (c->b.wflag) {
                        // the image populations of the band's sources read its
                        // records (of both reconstruction streams); the gathers
                        // that wait for this band see them
                        if (multi && a.ws != a.es) {
                            HIPCHECK(hipEventRecord(c->opev[2 * i + 1], a.ws));
                            HIPCHECK(hipStreamWaitEvent(a.es, c->opev[2 * i + 1], 0));
                        }
                        if ((r = timed(c, 6, do_wall_image, &a, a.es)) != LELBM_OK) return r;
                    }
                    if (multi) {
                        HIPCHECK(hipEventRecord(c->opev[2 * i], a.es));
                        HIPCHECK(hipEventRecord(c->opev[2 * i + 1], a.ws));
                        if (op.a & 1) last_odd = (int)i;
                        last_wide = (int)i;
                    }
                } else {
                    if (multi)
                        for (int d = 0; d < op.ndep; d++) {
                            const int e = P.gdeps[op.dep + d];
                            HIPCHECK(hipStreamWaitEvent(c->side[1], c->opev[2 * e], 0));
                            HIPCHECK(hipStreamWaitEvent(c->side[1], c->opev[2 * e + 1], 0));
                        }
                    if ((r = timed(c, 4, do_gather, &a, a.gs)) != LELBM_OK) return r;
                    if (multi) HIPCHECK(hipEventRecord(c->opev[2 * i], c->side[1]));
                }
            }
            if (multi) {
                // the step's totals (and the next step) after the last gather
                // and the last reconstructions of the side streams
                HIPCHECK(hipStreamWaitEvent(s, c->opev[2 * (nops - 1)], 0));
                if (last_odd >= 0) HIPCHECK(hipStreamWaitEvent(s, c->opev[2 * last_odd], 0));
                if (last_wide >= 0) HIPCHECK(hipStreamWaitEvent(s, c->opev[2 * last_wide + 1], 0));
            }
            if (c->b.wflag && (r = timed(c, 6, do_wall_gather, &a)) != LELBM_OK) return r;
            if ((r = timed(c, 5, do_totals, &a)) != LELBM_OK) return r;
            c->cur ^= 1;
        }
        Flags f;
        if ((r = stage_d2h(c->stage, s, &f, c->b.flags, sizeof(Flags))) != LELBM_OK) return r;
        if (c->timing && (r = collect_times(c)) != LELBM_OK) return r;
        if (f.err == 0) {
            c->steps_done += nsteps;
            break;
        }
        // every kernel after the failing one returned early, so the state at
        // the start of step f.step is intact
        c->cur = (cur0 + (f.step - base)) & 1;
        if (f.err == ERR_OVERFLOW || f.err == ERR_REPLAN) {
            // re-plan the bands (and grow the context's scratch within its
            // budget), then repeat the step
            r = plan_adapt(plan_geom(c->g), P, limit, noalloc, f.err, f.need, f.total, f.reach);
            if (getenv("LELBM_DEBUG"))
                fprintf(stderr,
                        "lelbm: step %d %s (need %lld, total %lld, reach %d): %zu bands of %d rows, %d slots of "
                        "%lld elements, reach %d\n",
                        f.step, f.err == ERR_REPLAN ? "re-plan" : "overflow", f.need, f.total, f.reach,
                        P.bands.size(), P.rows, P.nslots, P.slot_cap, P.m_plan);
            if (r == LELBM_OK && !noalloc) r = grow_scratch(c, (long long)P.nslots * P.slot_cap);
            if (r == LELBM_OK) r = upload_plan(c, P);
            if (r == LELBM_OK) r = reset_flags(c);
            if (r == LELBM_OK) {
                base = f.step;
                continue;
            }
            c->steps_done += f.step;
            c->last_fail_node = -1;
            c->last_fail_step = f.step;
            c->last_fail_detail = 0;
            c->last_fail_species = -1;
            c->last_fail_residual = 0.0;
            return r;
        }
        c->steps_done += f.step;
        c->last_fail_node = (long)f.node;
        c->last_fail_step = f.step;
        c->last_fail_detail = f.detail;
        c->last_fail_species = f.species;
        c->last_fail_residual = f.residual;
        return f.err;
    }
    if (st) {
        HIPCHECK(launch_sums(c->g, c->b.mom[c->cur], c->b, s));
        DevStats ds;
        double sums[4];
        if ((r = stage_d2h(c->stage, s, &ds, c->b.stats, sizeof(DevStats))) != LELBM_OK) return r;
        if ((r = stage_d2h(c->stage, s, sums, c->b.partial + (size_t)num_sum_blocks(c->g) * 4, sizeof(sums))) !=
            LELBM_OK)
            return r;
        memset(st, 0, sizeof(*st));
        double cells = ds.cells ? (double)ds.cells : 1.0;
        st->it_mean_f = ds.it_sum_f / cells;
        st->it_mean_g = ds.it_sum_g / cells;
        st->it_max_f = ds.it_max_f;
        st->it_max_g = ds.it_max_g;
        st->fallbacks = (long)ds.fallbacks;
        st->limited = (long)ds.limited;
        st->q_min = ds.cells ? ds.q_min : 0;
        st->q_max = ds.q_max;
        st->q_mean = ds.q_sum / cells;
        double v;
        memcpy(&v, &ds.rt_min_bits, 8); st->rt_min = v;
        memcpy(&v, &ds.kn_max_bits, 8); st->kn_max = v;
        memcpy(&v, &ds.colat_max_bits, 8); st->colat_max = v;
        for (int k = 0; k < 4; k++) st->sum[k] = sums[k];
        st->cells = (long)ds.cells;
        st->point_passes = (long)ds.qpass_sum;
        st->arrivals = (long)ds.arrivals;
        st->point_passes_refined = (long)ds.qpass_ref_sum;
        st->wave_point_passes = (long)ds.wave_qpass;
        st->row_passes = (long)ds.row_passes;
    }
    return LELBM_OK;
}

// Event hooks of a 3D step: the same pool and kinds as timed().
static void t3_begin(void *cc, int kind, hipStream_t s) {
    lelbm_ctx *c = (lelbm_ctx *)cc;
    if (!c->timing) return;
    const size_t i = c->evused;
    while (c->evpool.size() < 2 * (i + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->evpool.push_back(e);
    }
    if (c->evkind.size() < i + 1) c->evkind.resize(i + 1);
    (void)hipEventRecord(c->evpool[2 * i], s);
    c->evkind[i] = kind;
}
static void t3_end(void *cc, int, hipStream_t s) {
    lelbm_ctx *c = (lelbm_ctx *)cc;
    if (!c->timing || c->evpool.size() < 2 * (c->evused + 1)) return;
    (void)hipEventRecord(c->evpool[2 * c->evused + 1], s);
    c->evused++;
}

static int step3(lelbm_ctx *c, int nsteps, lelbm_stats *st) {
    if (nsteps < 0) return LELBM_EINVAL;
    Step3Timer tm{c, t3_begin, t3_end};
    Step3Failure f{0, -1, 0, -1, -1, 0.0};
    int r = ctx3_step(c->c3, nsteps, st, tm, &f);
    if (c->timing) {
        (void)hipStreamSynchronize(c->stream);
        int rt = collect_times(c);
        if (r == LELBM_OK) r = rt;
    }
    if (f.err) {
        c->last_fail_node = (long)f.node;
        c->last_fail_step = f.step;
        c->last_fail_detail = f.detail;
        c->last_fail_species = f.species;
        c->last_fail_residual = f.residual;
    }
    return r;
}

extern "C" int lelbm_step(lelbm_ctx *c, int nsteps, lelbm_stats *st) {
    if (!c) return LELBM_EINVAL;
    int dev;
    HIPCHECK(hipGetDevice(&dev));
    if (dev != c->device) HIPCHECK(hipSetDevice(c->device));
    if (c->c3) return step3(c, nsteps, st);
    return step_impl(c, nsteps, st, nullptr, 0);
}

// ---------------------------------------------------------------------------
// Allocation-free stepping.  The record scratch of lelbm_step_noalloc is this
// file-scope device array: every GPU the library runs on holds its own copy
// (allocated with the code object, kept until the process ends).  In host
// code its name stands for a host-side shadow, not a device address, so the
// device address is looked up once per device (hipGetSymbolAddress, with the
// device current) and only that address is ever handed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LELBM_NOALLOC_SCRATCH_BYTES];

static constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex noalloc_mutex;
static void *noalloc_ptr[NOALLOC_MAX_DEVICES];

// Device address of this device's scratch array (set up on first use).
static int noalloc_scratch(int dev, void **out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return LELBM_EDEVICE;
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return LELBM_EDEVICE;
        noalloc_ptr[dev] = p;
    }
    *out = noalloc_ptr[dev];
    return LELBM_OK;
}

extern "C" int lelbm_step_noalloc(lelbm_ctx *c, int nsteps, lelbm_stats *st) {
    if (!c || c->c3) return LELBM_EINVAL;
    int dev;
    HIPCHECK(hipGetDevice(&dev));
    if (dev != c->device) HIPCHECK(hipSetDevice(c->device));
    void *p = nullptr;
    int r = noalloc_scratch(c->device, &p);
    if (r != LELBM_OK) return r;
    const long long cap = (long long)(LELBM_NOALLOC_SCRATCH_BYTES / (c->mixed ? sizeof(float) : sizeof(double)));
    return step_impl(c, nsteps, st, p, cap);
}

// Interior moments as FP64 SoA [nmom][ny][nx]: to the host through the
// pinned stage (row chunks), or to the device by a
// kernel.
static int read_common(const lelbm_ctx *cc, void *out, hipMemcpyKind kind, bool sync) {
    lelbm_ctx *c = const_cast<lelbm_ctx *>(cc);     // the stage is scratch state
    if (c->c3) return ctx3_read(c->c3, out, kind == hipMemcpyDeviceToDevice);
    const Geom &g = c->g;
    const size_t esz = sizeof(double);
    const long long n = (long long)g.nx * g.ny;
    if (kind == hipMemcpyDeviceToDevice) {
        HIPCHECK(launch_store_interior(g, c->nmom, c->b.mom[c->cur], (double *)out, c->stream));
        if (sync) HIPCHECK(hipStreamSynchronize(c->stream));
        return LELBM_OK;
    }
    const size_t rowb = (size_t)g.nx * esz;
    const long long rows_per = (long long)(STAGE_MAX / rowb) > 0 ? (long long)(STAGE_MAX / rowb) : 1;
    int r = stage_reserve(c->stage, (size_t)(rows_per < g.ny ? rows_per : g.ny) * rowb);
    if (r != LELBM_OK) return r;
    for (int k = 0; k < c->nmom; k++) {
        for (long long y0 = 0; y0 < g.ny; y0 += rows_per) {
            const long long ny = g.ny - y0 < rows_per ? g.ny - y0 : rows_per;
            const char *src = (const char *)c->b.mom[c->cur] + ((size_t)k * g.ns + (size_t)(y0 + g.wb) * g.sxn + g.wl) * esz;
            HIPCHECK(hipMemcpy2DAsync(c->stage.p, rowb, src, (size_t)g.sxn * esz, rowb, (size_t)ny,
                                      hipMemcpyDeviceToHost, c->stream));
            HIPCHECK(hipStreamSynchronize(c->stream));
            double *o = (double *)out + (long long)k * n + y0 * g.nx;
            const long long ne = ny * g.nx;
            memcpy(o, c->stage.p, (size_t)ne * sizeof(double));
        }
    }
    return LELBM_OK;
}

extern "C" int lelbm_read_moments(const lelbm_ctx *c, double *host_out) {
    if (!c || !host_out) return LELBM_EINVAL;
    return read_common(c, host_out, hipMemcpyDeviceToHost, true);
}

extern "C" int lelbm_read_moments_device(const lelbm_ctx *c, void *dev_out) {
    if (!c || !dev_out) return LELBM_EINVAL;
    return read_common(c, dev_out, hipMemcpyDeviceToDevice, false);
}

extern "C" int lelbm_last_failure(const lelbm_ctx *c, long *node, int *step) {
    if (!c) return LELBM_EINVAL;
    if (node) *node = c->last_fail_node;
    if (step) *step = c->last_fail_step;
    return LELBM_OK;
}

extern "C" int lelbm_last_failure_detail(const lelbm_ctx *c, int *reason, int *species, double *residual) {
    if (!c) return LELBM_EINVAL;
    if (reason) *reason = c->last_fail_detail;
    if (species) *species = c->last_fail_species;
    if (residual) *residual = c->last_fail_residual;
    return LELBM_OK;
}

extern "C" int lelbm_set_timing(lelbm_ctx *c, int enable) {
    if (!c) return LELBM_EINVAL;
    c->timing = enable != 0;
    for (int k = 0; k < LELBM_NTIMERS; k++) { c->kms[k] = 0; c->klaunch[k] = 0; }
    return LELBM_OK;
}

extern "C" int lelbm_kernel_times(const lelbm_ctx *c, double *ms, long *launches, int n) {
    if (!c || n < 0) return LELBM_EINVAL;
    for (int k = 0; k < n && k < LELBM_NTIMERS; k++) {
        if (ms) ms[k] = c->kms[k];
        if (launches) launches[k] = c->klaunch[k];
    }
    return LELBM_OK;
}

extern "C" int lelbm_set_scratch_budget(lelbm_ctx *c, long long bytes) {
    if (!c || bytes < 1) return LELBM_EINVAL;
    c->budget = bytes;
    if (c->c3) {
        ctx3_set_budget(c->c3, bytes);
        return LELBM_OK;
    }
    const size_t esz = c->mixed ? sizeof(float) : sizeof(double);
    const long long limit = std::max<long long>(bytes / (long long)esz, 1);
    // the plan starts again from one band of the whole domain (the next step
    // re-plans within the budget); a scratch beyond the budget is freed
    HIPCHECK(hipStreamSynchronize(c->stream));
    if (c->b.scratch_cap > limit) {
        if (c->b.scratch) HIPCHECK(hipFree(c->b.scratch));
        c->b.scratch = nullptr;
        c->b.scratch_cap = 0;
    }
    c->plan.overlap = true;
    build_plan(plan_geom(c->g), c->plan, c->g.nty, 0);
    c->plan.slot_cap = std::min(c->b.scratch_cap, limit);
    set_bases(c->plan);
    return LELBM_OK;
}

extern "C" int lelbm_memory(const lelbm_ctx *c, long *persistent_bytes, long *scratch_bytes) {
    if (!c) return LELBM_EINVAL;
    if (c->c3) {
        long long pb = 0, sb = 0;
        ctx3_memory(c->c3, &pb, &sb);
        if (persistent_bytes) *persistent_bytes = (long)pb;
        if (scratch_bytes) *scratch_bytes = (long)sb;
        return LELBM_OK;
    }
    if (persistent_bytes) *persistent_bytes = (long)c->persistent_bytes;
    if (scratch_bytes) *scratch_bytes = (long)(c->b.scratch_cap * (c->mixed ? 4 : 8));
    return LELBM_OK;
}

extern "C" void lelbm_destroy(lelbm_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_ctx(c);
}

// ---------------------------------------------------------------------------
// Warm-start network: trainer object, inference, harvesting
// ---------------------------------------------------------------------------
struct lelbm_mlp {
    hipStream_t stream;
    float *params, *m1, *m2;     // FP32 master parameters and Adam moments
    float *norm;                 // standardisation constants
    unsigned short *wb;          // BF16 weights
    float *partial, *lossp, *grad;
    long long part_cap;          // waves the partial buffer holds
    long long t;                 // Adam step counter
    Stage stage;                 // pinned host staging memory
};

static unsigned long long splitmix(unsigned long long &st) {
    unsigned long long z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void mlp_free(lelbm_mlp *m) {
    if (!m) return;
    void *ptrs[] = {m->params, m->m1, m->m2, m->wb, m->partial, m->lossp, m->grad, m->norm};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    stage_free(m->stage);
    delete m;
}

static int mlp_partials(lelbm_mlp *m, long long waves) {
    if (waves <= m->part_cap) return LELBM_OK;
    HIPCHECK(hipStreamSynchronize(m->stream));
    if (m->partial) HIPCHECK(hipFree(m->partial));
    if (m->lossp) HIPCHECK(hipFree(m->lossp));
    m->partial = nullptr;
    m->lossp = nullptr;
    m->part_cap = 0;
    if (hipMalloc((void **)&m->partial, (size_t)waves * MLP_NPARAM * sizeof(float)) != hipSuccess) return LELBM_ENOMEM;
    if (hipMalloc((void **)&m->lossp, (size_t)waves * sizeof(float)) != hipSuccess) return LELBM_ENOMEM;
    m->part_cap = waves;
    return LELBM_OK;
}

extern "C" int lelbm_mlp_create(const float *params, unsigned long long seed, void *hip_stream, lelbm_mlp **out) {
    if (!out) return LELBM_EINVAL;
    lelbm_mlp *m = new (std::nothrow) lelbm_mlp();
    if (!m) return LELBM_ENOMEM;
    m->stream = (hipStream_t)hip_stream;
    m->params = m->m1 = m->m2 = m->partial = m->lossp = m->grad = m->norm = nullptr;
    m->wb = nullptr;
    m->part_cap = 0;
    m->t = 0;
    bool ok = hipMalloc((void **)&m->params, MLP_NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->m1, MLP_NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->m2, MLP_NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->grad, MLP_NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->wb, MLP_NPARAM * sizeof(unsigned short)) == hipSuccess &&
              hipMalloc((void **)&m->norm, MLP_NORM * sizeof(float)) == hipSuccess;
    if (!ok) { mlp_free(m); return LELBM_ENOMEM; }
    std::vector<float> h(MLP_NPARAM, 0.f);
    if (params) {
        memcpy(h.data(), params, MLP_NPARAM * sizeof(float));
    } else {
        // He-uniform initialisation of the ReLU layers from a SplitMix64
        // stream; output layer scaled by 0.1; zero biases
        unsigned long long st = seed;
        struct L { int off, nin, nout; float gain; } layers[3] = {
            {MLP_OFF_W1, MLP_IN, MLP_H, 1.f}, {MLP_OFF_W2, MLP_H, MLP_H, 1.f}, {MLP_OFF_W3, MLP_H, MLP_OUT, 0.1f}};
        for (const L &ly : layers) {
            float a = ly.gain * sqrtf(6.f / ly.nin);
            for (int i = 0; i < ly.nin * ly.nout; i++) {
                double u = (splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
                h[ly.off + i] = (float)((2.0 * u - 1.0) * a);
            }
        }
    }
    std::vector<float> z(MLP_NPARAM, 0.f), nm(MLP_NORM, 0.f);
    for (int k = 0; k < 16; k++) { nm[16 + k] = 1.f; nm[48 + k] = 1.f; }   // identity standardisation
    if (stage_h2d(m->stage, m->stream, m->params, h.data(), MLP_NPARAM * sizeof(float)) != LELBM_OK ||
        stage_h2d(m->stage, m->stream, m->norm, nm.data(), MLP_NORM * sizeof(float)) != LELBM_OK ||
        stage_h2d(m->stage, m->stream, m->m1, z.data(), MLP_NPARAM * sizeof(float)) != LELBM_OK ||
        stage_h2d(m->stage, m->stream, m->m2, z.data(), MLP_NPARAM * sizeof(float)) != LELBM_OK ||
        launch_mlp_to_bf16(m->params, m->wb, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess) {
        mlp_free(m);
        return LELBM_EDEVICE;
    }
    *out = m;
    return LELBM_OK;
}

extern "C" int lelbm_mlp_get_params(const lelbm_mlp *m, float *host_out) {
    if (!m || !host_out) return LELBM_EINVAL;
    return stage_d2h(const_cast<lelbm_mlp *>(m)->stage, m->stream, host_out, m->params, MLP_NPARAM * sizeof(float));
}

extern "C" int lelbm_mlp_forward(lelbm_mlp *m, const float *dev_x, long long x_stride, long long n, float *dev_y) {
    if (!m || n < 0 || (n > 0 && (!dev_x || !dev_y)) || x_stride < MLP_IN) return LELBM_EINVAL;
    HIPCHECK(launch_mlp_forward(m->wb, m->params, m->norm, dev_x, x_stride, n, dev_y, m->stream));
    HIPCHECK(hipStreamSynchronize(m->stream));
    return LELBM_OK;
}

extern "C" int lelbm_mlp_gradient(lelbm_mlp *m, const float *dev_pairs, long long n, float *host_grad,
                                  double *loss) {
    if (!m || !dev_pairs || n <= 0) return LELBM_EINVAL;
    long long waves = (n + 63) / 64;
    int r = mlp_partials(m, waves);
    if (r != LELBM_OK) return r;
    HIPCHECK(launch_mlp_fwdbwd(m->wb, m->params, m->norm, dev_pairs, n, n, 0, 0, 0, m->partial, m->lossp, m->stream));
    HIPCHECK(launch_mlp_adam(m->partial, (int)waves, m->params, m->m1, m->m2, m->wb, 0.f, 1, 0, m->grad, m->stream));
    std::vector<float> lp(waves);
    if ((r = stage_d2h(m->stage, m->stream, lp.data(), m->lossp, waves * sizeof(float))) != LELBM_OK) return r;
    if (host_grad && (r = stage_d2h(m->stage, m->stream, host_grad, m->grad, MLP_NPARAM * sizeof(float))) != LELBM_OK)
        return r;
    if (loss) {
        double a = 0;
        for (float v : lp) a += v;
        *loss = a / ((double)n * MLP_OUT);
    }
    return LELBM_OK;
}

extern "C" int lelbm_mlp_train(lelbm_mlp *m, const float *dev_pairs, long long n, int steps, int batch, float lr,
                               unsigned long long seed, double *final_loss) {
    if (!m || !dev_pairs || n <= 0 || steps < 0 || batch < 64 || batch % 64 != 0 || !(lr > 0.f)) return LELBM_EINVAL;
    long long waves = batch / 64;
    int r = mlp_partials(m, waves);
    if (r != LELBM_OK) return r;
    for (int k = 0; k < steps; k++) {
        m->t++;
        HIPCHECK(launch_mlp_fwdbwd(m->wb, m->params, m->norm, dev_pairs, n, batch, 1, seed, (unsigned long long)m->t,
                                   m->partial, m->lossp, m->stream));
        HIPCHECK(launch_mlp_adam(m->partial, (int)waves, m->params, m->m1, m->m2, m->wb, lr, (int)m->t, 1, nullptr,
                                 m->stream));
    }
    if (final_loss) {
        std::vector<float> lp(waves);
        if ((r = stage_d2h(m->stage, m->stream, lp.data(), m->lossp, waves * sizeof(float))) != LELBM_OK) return r;
        double a = 0;
        for (float v : lp) a += v;
        *final_loss = a / ((double)batch * MLP_OUT);
    } else {
        HIPCHECK(hipStreamSynchronize(m->stream));
    }
    return LELBM_OK;
}

extern "C" int lelbm_mlp_fit_normalization(lelbm_mlp *m, const float *dev_pairs, long long n) {
    if (!m || !dev_pairs || n <= 0) return LELBM_EINVAL;
    HIPCHECK(launch_mlp_norm_fit(dev_pairs, n, m->norm, m->stream));
    HIPCHECK(hipStreamSynchronize(m->stream));
    return LELBM_OK;
}

extern "C" int lelbm_mlp_get_norm(const lelbm_mlp *m, float *host_out) {
    if (!m || !host_out) return LELBM_EINVAL;
    return stage_d2h(const_cast<lelbm_mlp *>(m)->stage, m->stream, host_out, m->norm, MLP_NORM * sizeof(float));
}

extern "C" int lelbm_mlp_set_norm(lelbm_mlp *m, const float *host_norm) {
    if (!m || !host_norm) return LELBM_EINVAL;
    for (int k = 0; k < 16; k++)
        if (!(host_norm[48 + k] > 0.f) || !std::isfinite(host_norm[16 + k])) return LELBM_EINVAL;
    return stage_h2d(m->stage, m->stream, m->norm, host_norm, MLP_NORM * sizeof(float));
}

extern "C" void lelbm_mlp_destroy(lelbm_mlp *m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    mlp_free(m);
}

extern "C" int lelbm_set_mlp(lelbm_ctx *c, const lelbm_mlp *m) {
    if (!c || !m || (c->p.guess != LELBM_GUESS_MLP && c->p.guess != LELBM_GUESS_MLP_PREV)) return LELBM_EINVAL;
    HIPCHECK(hipStreamSynchronize(m->stream));
    HIPCHECK(hipMemcpyAsync(c->mlp_p, m->params, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    HIPCHECK(hipMemcpyAsync(c->mlp_n, m->norm, MLP_NORM * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    HIPCHECK(launch_mlp_to_bf16(c->mlp_p, c->mlp_w, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    c->b.mlp_w = c->mlp_w;
    c->b.mlp_p = c->mlp_p;
    c->b.mlp_n = c->mlp_n;
    c->mlp_set = 1;
    return LELBM_OK;
}

extern "C" int lelbm_harvest(lelbm_ctx *c, float *dev_buf, long long capacity, int stride) {
    if (!c || c->c3) return LELBM_EINVAL;
    if (!dev_buf) {
        c->b.harvest = nullptr;
        c->b.harvest_cap = 0;
        return LELBM_OK;
    }
    if (capacity <= 0 || stride < 1 || c->p.dim != 2) return LELBM_EINVAL;
    c->b.harvest = dev_buf;
    c->b.harvest_cap = capacity;
    c->b.harvest_stride = stride;
    unsigned long long zero = 0;
    return stage_h2d(c->stage, c->stream, c->b.harvest_n, &zero, sizeof(zero));
}

extern "C" int lelbm_harvest_count(const lelbm_ctx *c, long long *n) {
    if (!c || !n) return LELBM_EINVAL;
    if (c->c3) {
        *n = 0;
        return LELBM_OK;
    }
    unsigned long long v = 0;
    int r = stage_d2h(const_cast<lelbm_ctx *>(c)->stage, c->stream, &v, c->b.harvest_n, sizeof(v));
    if (r != LELBM_OK) return r;
    *n = (long long)(v < (unsigned long long)c->b.harvest_cap ? v : (unsigned long long)c->b.harvest_cap);
    return LELBM_OK;
}
