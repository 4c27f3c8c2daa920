// The LELBM time step in three dimensions (D = 3) on periodic boxes: 17
// stored values per cell (13 fluon moments and 4 phonon moments, Sec. II.E),
// 19 fluon and 10 phonon constraints in the reconstruction.
//
// One step = k3_prepare (macroscopic variables, Eq. IIB6; stencil radius,
// Eq. IIC6; per-tile boxes of the record scratch) -> k3_scan (record offsets)
// -> k3_epr (collision, Eqs. IIB9-IIB18 and App. D; Newton-Cholesky
// reconstruction, Eqs. IID7-IID13; moment fractions of Eq. IIE3a into the
// records) -> k3_gather (moment streaming, Eq. IIE3b, as a deterministic
// gather).
//
// Cells are taken in tiles of 4 x 4 x 4 (one wavefront, one lane per cell).
// A tile's records hold, per displacement slot of the union of its cells'
// stencil boxes, the pair (w_f, w_g) of each of its 64 cells, so the lanes of
// a wavefront that read one displacement read 64 consecutive pairs.
//
// Cells with refined stencils (N_r > 0 in Eq. IIC9, RT <= 4/9) go to
// k3_epr_ref, which visits their points one by one (8 children per level)
// and writes, per base point, the pre-summed moments of its descendants; their
// tiles hold all 17 moments per slot.
//
// Scope: fully periodic boxes; up to 3 refinement levels and radii up to 64
// (other cells fail the step with LELBM_EREACH).
#include <hip/hip_runtime.h>
#include <math.h>

#include <string.h>

#include <algorithm>
#include <climits>
#include <vector>

#include "lelbm_3d.h"

namespace lelbm {
namespace d3 {

constexpr int NF = 19, NG = 10, NMF = 84, NMG = 35, NM = 17, TN = 64, TE = 4;
constexpr int MAX_R3 = 64, MAX_REFINE3 = 3;

// Exponents (a, b, c) of x^a y^b z^c of the fluon basis: 1, x, y, z, xx, xy,
// xz, yy, yz, zz, then the per-axis third-order pieces M~_{aa|g} (Eq. IIB14)
// (xx|x), (xx|y), (xx|z), (yy|x), (yy|y), (yy|z), (zz|x), (zz|y), (zz|z);
// the phonon basis is the first ten.
__host__ __device__ constexpr int bexp(int j, int k) {
    constexpr int t[NF][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {1, 1, 0}, {1, 0, 1},
                              {0, 2, 0}, {0, 1, 1}, {0, 0, 2}, {3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0},
                              {0, 3, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}, {0, 0, 3}};
    return t[j][k];
}
__host__ __device__ constexpr int border(int j) { return bexp(j, 0) + bexp(j, 1) + bexp(j, 2); }
// Monomials x^a y^b z^c of total degree d are numbered degree-major; inside
// a degree by b + c, then by c.  Degrees <= 6 (fluon sums) take 84 numbers,
// degrees <= 4 (phonon sums) the first 35.
__host__ __device__ constexpr int mono(int a, int b, int c) {
    return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}
__host__ __device__ constexpr int hidx(int i, int j) {
    return mono(bexp(i, 0) + bexp(j, 0), bexp(i, 1) + bexp(j, 1), bexp(i, 2) + bexp(j, 2));
}

struct Desc3 {
    double *rho, *ux, *uy, *uz, *rt;   // [n]
    int *r;                            // [n] R | N_r << 16 (radius, refinement levels), -1: no population
};

struct Tile3 {
    int ox, oy, oz, wx, wy, wz;   // slot box (first displacement, extents)
    int fmt;                      // 0: (w_f, w_g) per slot and cell; 1: the 17 moments (refined cells in the tile)
    long long size;               // elements (wx wy wz x 64 cells x 2)
    long long base;               // first element in the scratch
};

struct Buf3 {
    double *mom[2];               // [17][n] FP64 state
    Desc3 d;
    Tile3 *tiles;                 // [ntiles]
    void *scratch;
    long long scratch_cap;        // elements
    Flags *flags;
    DevStats *stats;
    int *maxreach;                // max over cells of max |round(u_a)| + R + 1
    long long *total;             // record elements of the step (k3_scan)
    double *partial;              // block sums of the conserved totals
    const double *ainv;           // inverse scaled Maxwellian Hessians of the linearised start, or NULL
    double *prev;                 // [19 + 10][n] previous-step guess: each cell's converged correction
                                  // beyond the linearised start, scaled by RT^(k/2); NaN: none; or NULL
};

struct G3 {
    int nx, ny, nz;
    long long n;
    int tnx, tny, tnz, ntiles;
};

// First failure of a step: its code, step and reason; the smallest failing cell.
__device__ inline void flag3(Flags *fl, int code, int step, long long node, int detail = 0, int species = -1,
                             double residual = 0.0) {
    if (atomicCAS(&fl->err, 0, code) == 0) {
        fl->step = step;
        fl->detail = detail;
        fl->species = species;
        fl->residual = residual;
    }
    if (fl->err == code) atomicMin((unsigned long long *)&fl->node, (unsigned long long)node);
}

__global__ void k3_reset_flags(Flags *f) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        f->err = 0; f->step = -1; f->node = LLONG_MAX; f->need = 0;
        f->detail = 0; f->species = -1; f->residual = 0.0; f->reach = 0; f->total = 0;
    }
}

__device__ inline int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// The decisions that define a stencil are taken without FMA contraction and
// in the order the CPU oracle uses, so that both select the same points.
__device__ inline bool in_ball(double cx, double cy, double cz, double ux, double uy, double uz, double rr) {
#pragma clang fp contract(off)
    const double ex = cx - ux, ey = cy - uy, ez = cz - uz;
    return ex * ex + ey * ey + ez * ez <= rr * rr;
}
__device__ inline int radius3(double RT, double n_conf, int r_min) {
#pragma clang fp contract(off)
    int R = (int)floor(n_conf * sqrt(RT) + 0.5);
    return R > r_min ? R : r_min;
}
__device__ inline int levels3(double RT) {
#pragma clang fp contract(off)
    return (int)floor(1.0 / (3.0 * sqrt(RT)) + 0.5);
}

// Integer cx of row (cy, cz) inside the ball, from the analytic estimate
// corrected with the exact predicate; false if the row is empty.
__device__ inline bool span3(int cy, int cz, double ux, double uy, double uz, double rr, int lo, int hi, int &xa,
                             int &xb) {
    const double ey = (double)cy - uy, ez = (double)cz - uz;
    const double rem = rr * rr - ey * ey - ez * ez;
    const double w = rem > 0.0 ? sqrt(rem) : 0.0;
    int a = (int)ceil(ux - w), b = (int)floor(ux + w);
    a = a < lo ? lo : (a > hi ? hi : a);
    b = b > hi ? hi : (b < lo ? lo : b);
    auto in = [&](int cx) { return in_ball((double)cx, (double)cy, (double)cz, ux, uy, uz, rr); };
    while (a > lo && in(a - 1)) a--;
    while (a <= b && !in(a)) a++;
    while (b < hi && in(b + 1)) b++;
    while (b >= a && !in(b)) b--;
    xa = a;
    xb = b;
    return a <= b;
}

// Macroscopic variables as the oracle forms them (Eq. IIB6 with D = 3).
__device__ inline void macro3(const double *mom, long long n, long long s, double K, double &rho, double &ux,
                              double &uy, double &uz, double &RT) {
#pragma clang fp contract(off)
    rho = mom[s];
    ux = mom[n + s] / rho;
    uy = mom[2 * n + s] / rho;
    uz = mom[3 * n + s] / rho;
    double uu = ux * ux;
    uu = uu + uy * uy;
    uu = uu + uz * uz;
    RT = ((mom[4 * n + s] + mom[7 * n + s] + mom[9 * n + s] + mom[13 * n + s]) / rho - uu) / (3.0 + K);
}

// ---------------------------------------------------------------------------
// k3_prepare: descriptors, tile boxes, reach
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k3_prepare(G3 g, Phys ph, const double *mom, Buf3 b, int step) {
    if (b.flags->err) return;
    const int t = blockIdx.x, l = threadIdx.x;
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    const int x = tx * TE + (l & 3), y = ty * TE + ((l >> 2) & 3), z = tz * TE + (l >> 4);
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    int lo[3] = {1 << 29, 1 << 29, 1 << 29}, hi[3] = {-(1 << 29), -(1 << 29), -(1 << 29)};
    int reach = 0, refined = 0;
    if (valid) {
        const long long s = ((long long)z * g.ny + y) * g.nx + x;
        double rho, ux, uy, uz, RT;
        macro3(mom, g.n, s, ph.K, rho, ux, uy, uz, RT);
        const bool ok = rho > 0.0 && isfinite(rho) && RT > 0.0 && isfinite(RT) && isfinite(ux) && isfinite(uy) &&
                        isfinite(uz);
        int R = -1;
        if (!ok) {
            flag3(b.flags, LELBM_EEPR, step, s);
        } else {
            R = radius3(RT, ph.n_conf, ph.r_min);
            const int Nr = levels3(RT);
            const double um = fmax(fabs(ux), fmax(fabs(uy), fabs(uz)));
            if (Nr > MAX_REFINE3 || R > MAX_R3 || !(um <= MAX_SPEED)) {
                flag3(b.flags, LELBM_EREACH, step, s);
                R = -1;
            } else {
                refined = Nr > 0;
                const int ub[3] = {(int)floor(ux + 0.5), (int)floor(uy + 0.5), (int)floor(uz + 0.5)};
                for (int a = 0; a < 3; a++) {
                    lo[a] = ub[a] - R - 1;
                    hi[a] = ub[a] + R + 1;
                    reach = max(reach, abs(ub[a]) + R + 1);
                }
                R |= Nr << 16;
            }
        }
        b.d.rho[s] = rho; b.d.ux[s] = ux; b.d.uy[s] = uy; b.d.uz[s] = uz; b.d.rt[s] = RT; b.d.r[s] = R;
    }
    for (int off = 32; off > 0; off >>= 1) {
        for (int a = 0; a < 3; a++) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], off));
            hi[a] = max(hi[a], __shfl_xor(hi[a], off));
        }
        reach = max(reach, __shfl_xor(reach, off));
        refined |= __shfl_xor(refined, off);
    }
    if (l == 0) {
        Tile3 ti;
        ti.fmt = refined;
        if (lo[0] > hi[0]) {
            ti.ox = ti.oy = ti.oz = 0; ti.wx = ti.wy = ti.wz = 0; ti.size = 0;
        } else {
            ti.ox = lo[0]; ti.oy = lo[1]; ti.oz = lo[2];
            ti.wx = hi[0] - lo[0] + 1; ti.wy = hi[1] - lo[1] + 1; ti.wz = hi[2] - lo[2] + 1;
            ti.size = (long long)ti.wx * ti.wy * ti.wz * TN * (refined ? NM : 2);
        }
        ti.base = 0;
        b.tiles[t] = ti;
        if (reach > __hip_atomic_load(b.maxreach, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(b.maxreach, reach);
    }
}

// Record elements of each layer of tiles (one workgroup per layer).
__global__ void __launch_bounds__(256) k3_layer_sizes(G3 g, Buf3 b, long long *layer) {
    __shared__ long long part[256];
    const int per = g.tnx * g.tny, t0 = blockIdx.x * per;
    long long s = 0;
    if (!b.flags->err)
        for (int i = threadIdx.x; i < per; i += 256) s += b.tiles[t0 + i].size;
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) layer[blockIdx.x] = part[0];
}

// Exclusive scan of the sizes of tiles [t0, t0 + nt) (one workgroup) from
// `base` on -> their record offsets (the tiles of one band, in its slot).
__global__ void __launch_bounds__(1024) k3_scan(int t0, int nt, long long base, Buf3 b) {
    __shared__ long long part[1024];
    if (b.flags->err) return;
    const int per = (nt + 1023) / 1024;
    const int a0 = t0 + threadIdx.x * per, a1 = min(t0 + nt, a0 + per);
    long long s = 0;
    for (int t = a0; t < a1; t++) s += b.tiles[t].size;
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = base;
        for (int i = 0; i < 1024; i++) {
            const long long v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    long long acc = part[threadIdx.x];
    for (int t = a0; t < a1; t++) {
        b.tiles[t].base = acc;
        acc += b.tiles[t].size;
    }
}

// ---------------------------------------------------------------------------
// collision (Eqs. IIB9-IIB18, App. D) with D = 3
// ---------------------------------------------------------------------------
__device__ inline void collide3(const Phys &ph, const double *mom, long long n, long long s, double rho, double ux,
                                double uy, double uz, double RT, double *mf, double *mg, double &kn, int &lim) {
    const double K = ph.K;
    const double u[3] = {ux, uy, uz};
    const double uu = ux * ux + uy * uy + uz * uz;
    auto M = [&](int k) { return mom[(long long)k * n + s]; };
    // Eq. (IIB9a); second-moment slot of (a, b)
    auto sec = [](int a, int c) { return a == 0 ? 4 + c : (a == 1 ? (c == 0 ? 5 : 6 + c) : (c == 0 ? 6 : 7 + c)); };
    double P[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) P[a][c] = M(sec(a, c)) - rho * (u[a] * u[c] + (a == c ? RT : 0.0));
    const double trP = P[0][0] + P[1][1] + P[2][2];
    double Q[3];
#pragma unroll
    for (int g = 0; g < 3; g++) {
        const double sp = u[0] * P[0][g] + u[1] * P[1][g] + u[2] * P[2][g];
        Q[g] = M(10 + g) - 2.0 * sp - u[g] * trP - rho * (uu + 5.0 * RT) * u[g];
    }
    const double G0 = M(13);
    const double g0 = G0 - rho * K * RT;
    double h[3];
#pragma unroll
    for (int g = 0; g < 3; g++) h[g] = M(14 + g) - u[g] * G0;
    // Eq. (D2)
    double sP = 0.0, sQ = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
        for (int c = 0; c < 3; c++) sP += fabs(P[a][c]);
        sQ += fabs(Q[a]) + fabs(h[a]);
    }
    const double knA = (sP + fabs(g0)) / (rho * (3.0 + K) * RT);
    const double knB = sQ / (rho * (5.0 + K) * RT * sqrt(RT));
    kn = fmax(knA, knB);
    double of = ph.omega_f, ob = ph.omega_b, oh = ph.omega_h;
    lim = 0;
    if (ph.kn_limiter && kn >= ph.kn_lo_lin) {
        // Eq. (D3) as worded after it: linear in log10 Kn between the thresholds
        auto lw = [&](double om) {
            if (kn > ph.kn_hi_lin) return ph.omega_H;
            return (ph.omega_H - om) / (ph.kn_hi - ph.kn_lo) * (log10(kn) - ph.kn_lo) + om;
        };
        of = lw(of); ob = lw(ob); oh = lw(oh);
        lim = (of != ph.omega_f) || (ob != ph.omega_b) || (oh != ph.omega_h);
    }
    // Eqs. (IIB10-11, IIB14, IIB16-18)
    const double bulk = -g0 / 3.0, irho = 1.0 / rho;
    mf[0] = 1.0; mf[1] = 0.0; mf[2] = 0.0; mf[3] = 0.0;
    int k = 4;
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int c = a; c < 3; c++) {
            const double bl = a == c ? bulk : 0.0;
            mf[k++] = (a == c ? RT : 0.0) + ((1.0 - of) * (P[a][c] - bl) + (1.0 - ob) * bl) * irho;
        }
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int g = 0; g < 3; g++) mf[10 + 3 * a + g] = (1.0 - oh) * ((a == g ? 3.0 : 1.0) / 5.0) * Q[g] * irho;
    const double rKT = rho * K * RT;
    mg[0] = 1.0 + (1.0 - ob) * g0 / rKT;
#pragma unroll
    for (int g = 0; g < 3; g++) mg[1 + g] = (1.0 - oh) * h[g] / rKT;
    mg[4] = RT; mg[5] = 0.0; mg[6] = 0.0; mg[7] = RT; mg[8] = 0.0; mg[9] = RT;
}

// ---------------------------------------------------------------------------
// Newton state of one species (registers), Sec. II.D: damped Newton on the
// convex dual (Armijo backtracking while the decrement exceeds 1e-8), the
// scaled residual as stop test, the stalled-residual rule, one polishing
// update after the stop.
// ---------------------------------------------------------------------------
// Multipliers lam and search direction del of one species: in registers, or
// in the lane's LDS column (entry j at j * TN), which keeps them out of the
// registers the stencil passes need.
template <int NB> struct RegStore3 {
    double l[NB], d[NB];
    __device__ double &lam(int j) { return l[j]; }
    __device__ double &del(int j) { return d[j]; }
    __device__ double lam(int j) const { return l[j]; }
    __device__ double del(int j) const { return d[j]; }
};
template <int NB> struct LdsStore3 {
    double *l, *d;
    __device__ double &lam(int j) const { return l[j * TN]; }
    __device__ double &del(int j) const { return d[j * TN]; }
};
template <int NB, class St = RegStore3<NB>> struct Sp3 {
    static constexpr int N = NB;
    St v;
    double t, dec, phi, res, res_prev;
    int phase, nit, ls;
    int lin;          // 1 while iterating from the linearised start
    __device__ double &lam(int j) { return v.lam(j); }
    __device__ double &del(int j) { return v.del(j); }
    __device__ double lam(int j) const { return v.lam(j); }
    __device__ double at(int j) const { return v.lam(j) + t * v.del(j); }
};

template <class SP> __device__ inline void sp3_init(SP &sp, double RT) {
    constexpr int NB = SP::N;
#pragma unroll
    for (int j = 0; j < NB; j++) { sp.lam(j) = 0.0; sp.del(j) = 0.0; }
    sp.lam(0) = -1.0 + 1.5 * log(2.0 * M_PI * RT);     // Eq. (IID13), D = 3
    sp.lam(4) = sp.lam(7) = sp.lam(9) = 1.0 / (2.0 * RT);
    sp.t = 0.0; sp.dec = 0.0; sp.phi = 0.0; sp.res = 0.0; sp.res_prev = 0.0;
    sp.phase = 0; sp.nit = 0; sp.ls = 0;
    sp.lin = 0;
}

// Linearised start: Eq. (IID13) plus one Newton step taken with the Hessian
// of the continuous Maxwellian.  In units scaled by RT^(k/2) (k the order of
// a basis function) that Hessian is the constant matrix of the moments
// <T_i T_j> of the unit normal distribution; ainv holds its inverse (fluon
// 19 x 19, then phonon 10 x 10), computed once on the host.  The step is
// A~ dl~ = (equilibrium moments - targets) / RT^(k/2).
// The step's scaled corrections: d[0..18] fluon, d[19..28] phonon.
__device__ inline void lin3_scaled(const double *mf, const double *mg, double RT, const double *ainv, double *d) {
    const double sq = sqrt(RT);
    const double sc[4] = {1.0, sq, RT, RT * sq};
    double rf[NF], rg[NG];
#pragma unroll
    for (int j = 0; j < NF; j++) {
        const bool diag = j == 4 || j == 7 || j == 9;
        const double eq = j == 0 ? 1.0 : (diag ? RT : 0.0);
        rf[j] = (eq - mf[j]) / sc[border(j)];
        if (j < NG) rg[j] = (eq - mg[j]) / sc[border(j)];
    }
#pragma unroll
    for (int i = 0; i < NF; i++) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < NF; j++) v += ainv[i * NF + j] * rf[j];
        d[i] = v;
    }
#pragma unroll
    for (int i = 0; i < NG; i++) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < NG; j++) v += ainv[NF * NF + i * NG + j] * rg[j];
        d[NF + i] = v;
    }
}

template <class SF, class SG>
__device__ inline void sp3_linear(SF &sf, SG &sg, const double *mf, const double *mg, double RT,
                                  const double *ainv) {
    const double sq = sqrt(RT);
    const double sc[4] = {1.0, sq, RT, RT * sq};
    double d[NF + NG];
    lin3_scaled(mf, mg, RT, ainv, d);
#pragma unroll
    for (int i = 0; i < NF; i++) sf.lam(i) += d[i] / sc[border(i)];
#pragma unroll
    for (int i = 0; i < NG; i++) sg.lam(i) += d[NF + i] / sc[border(i)];
    sf.lin = 1;
    sg.lin = 1;
}

// Previous-step guess (Sec. II.D suggests reusing stored multipliers): the
// linearised start plus the cell's stored correction beyond it, where one is
// stored.  The correction is kept in scaled units, so it carries over when
// the temperature changes, and beyond the linearised start, which follows
// the sign flip of the non-equilibrium targets at omega = 2.
template <class SF, class SG>
__device__ inline void sp3_prev(SF &sf, SG &sg, double RT, const double *prev, long long n,
                                long long s) {
    if (!(prev[s] == prev[s])) return;
    const double sq = sqrt(RT);
    const double sc[4] = {1.0, sq, RT, RT * sq};
#pragma unroll
    for (int i = 0; i < NF; i++) sf.lam(i) += prev[(long long)i * n + s] / sc[border(i)];
#pragma unroll
    for (int i = 0; i < NG; i++) sg.lam(i) += prev[(long long)(NF + i) * n + s] / sc[border(i)];
}

// Stores the converged multipliers' correction beyond Eq. (IID13) plus the
// linearised step, in scaled units, for the next step's guess.
template <class SF, class SG>
__device__ inline void sp3_store_prev(const SF &sf, const SG &sg, const double *mf, const double *mg,
                                      double RT, const double *ainv, double *prev, long long n, long long s) {
    const double sq = sqrt(RT);
    const double sc[4] = {1.0, sq, RT, RT * sq};
    const double l0 = -1.0 + 1.5 * log(2.0 * M_PI * RT);   // Eq. (IID13): lam_0; 1/(2 RT) on xx, yy, zz
    double d[NF + NG];
    lin3_scaled(mf, mg, RT, ainv, d);
#pragma unroll
    for (int i = 0; i < NF + NG; i++) {
        const int j = i < NF ? i : i - NF;
        const double lam = i < NF ? sf.lam(j) : sg.lam(j);
        const double eq = j == 0 ? l0 : ((j == 4 || j == 7 || j == 9) ? 0.5 : 0.0);   // scaled Eq. (IID13)
        prev[(long long)i * n + s] = lam * sc[border(j)] - eq - d[i];
    }
}

// Cholesky solve of A x = r with A_ij = S[hidx(i, j)] (Eq. IID11a).
template <int NB> __device__ inline bool chol3(const double *S, const double *r, double *x) {
    double L[NB * (NB + 1) / 2], inv[NB];
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) L[i * (i + 1) / 2 + j] = S[hidx(i, j)];
#pragma unroll
    for (int i = 0; i < NB; i++) {
#pragma unroll
        for (int j = 0; j <= i; j++) {
            double v = L[i * (i + 1) / 2 + j];
#pragma unroll
            for (int k = 0; k < j; k++) v -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
            if (i == j) {
                if (!(v > 0.0) || !isfinite(v)) return false;
                const double d = sqrt(v);
                L[i * (i + 1) / 2 + i] = d;
                inv[i] = 1.0 / d;
            } else {
                L[i * (i + 1) / 2 + j] = v * inv[j];
            }
        }
    }
    double y[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        double v = r[i];
#pragma unroll
        for (int k = 0; k < i; k++) v -= L[i * (i + 1) / 2 + k] * y[k];
        y[i] = v * inv[i];
    }
#pragma unroll
    for (int i = NB - 1; i >= 0; i--) {
        double v = y[i];
#pragma unroll
        for (int k = i + 1; k < NB; k++) v -= L[k * (k + 1) / 2 + i] * x[k];
        x[i] = v * inv[i];
    }
    return true;
}

// After a pass evaluated at lam + t del: accept / backtrack / step / polish.
// 0: continue, 1: polished, negative: failure reason.
template <class SP> __device__ inline int sp3_update(SP &sp, const double *S, const double *tg, const double *isc,
                                                     double tol, int maxit) {
    constexpr int NB = SP::N;
    double r[NB];
    double phit = S[0];
    bool fin = isfinite(S[0]);
#pragma unroll
    for (int j = 0; j < NB; j++) {
        r[j] = S[mono(bexp(j, 0), bexp(j, 1), bexp(j, 2))] - tg[j];
        phit += sp.at(j) * tg[j];
        fin = fin && isfinite(r[j]);
    }
    fin = fin && isfinite(phit);
    if (sp.phase == 0) {
        if (!fin) return sp.lin ? 2 : -1;
        sp.phase = 1;
    } else {
        if (!(fin && (sp.dec <= 1e-8 || phit <= sp.phi - 1e-4 * sp.t * sp.dec))) {
            sp.t *= 0.5;
            if (++sp.ls > 30) return -2;
            return 0;
        }
        sp.nit++;
    }
#pragma unroll
    for (int j = 0; j < NB; j++) sp.lam(j) = sp.at(j);
    sp.t = 0.0;
    sp.phi = phit;
    double res = 0.0;
#pragma unroll
    for (int j = 0; j < NB; j++) res = fmax(res, fabs(r[j]) * isc[border(j)]);
    sp.res = res;
    const bool stalled = sp.nit > 0 && res <= STALL_RES && !(res < sp.res_prev);
    // from the linearised start, an accepted update that does not lower the
    // residual sends the solve back to Eq. (IID13)
    if (sp.lin && sp.nit > 0 && res > tol && !stalled && !(res < sp.res_prev)) return 2;
    sp.res_prev = res;
    double dl[NB];
    if (res <= tol || stalled) {
        if (!chol3<NB>(S, r, dl)) return -3;
#pragma unroll
        for (int j = 0; j < NB; j++) { sp.lam(j) += dl[j]; sp.del(j) = 0.0; }
        sp.nit++;
        sp.phase = 2;
        return 1;
    }
    if (sp.nit >= maxit) return -4;
    if (!chol3<NB>(S, r, dl)) return -5;
    double dec = 0.0;
#pragma unroll
    for (int j = 0; j < NB; j++) { sp.del(j) = dl[j]; dec += r[j] * dl[j]; }
    sp.dec = dec;
    sp.t = 1.0;
    sp.ls = 0;
    return 0;
}

// Moments (Eq. IIE3b) of one arrival with velocity c and moment fractions
// (w_f, w_g), in the stored order.
__device__ inline void moments17(double cx, double cy, double cz, double wf, double wg, double *mo) {
    const double c[3] = {cx, cy, cz}, cc = cx * cx + cy * cy + cz * cz;
    mo[0] = wf;
    int k = 4;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        mo[1 + a] = c[a] * wf;
        mo[10 + a] = cc * c[a] * wf;
        mo[14 + a] = c[a] * wg;
#pragma unroll
        for (int bb = a; bb < 3; bb++) mo[k++] = c[a] * c[bb] * wf;
    }
    mo[13] = wg;
}

// Statistics of a wavefront's cells: one set of atomics per wavefront.
__device__ inline void stats3(DevStats *st, int itf, int itg, int q, int lim, int fb, int passes, int rows, double RT,
                              double kn, double colat, int l) {
    unsigned long long a[6] = {(unsigned long long)itf, (unsigned long long)itg, (unsigned long long)q,
                               (unsigned long long)lim, (unsigned long long)(q > 0 ? 1 : 0), (unsigned long long)fb};
    unsigned long long qp = (unsigned long long)q * (unsigned long long)passes;
    unsigned long long rp = (unsigned long long)rows * (unsigned long long)passes;
    int mxf = itf, mxg = itg, qmax = q, qmin = q > 0 ? q : INT_MAX;
    double rtmin = q > 0 ? RT : 1e300, knmax = kn, cmax = colat;
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 6; k++) a[k] += __shfl_xor(a[k], off);
        qp += __shfl_xor(qp, off);
        rp += __shfl_xor(rp, off);
        mxf = max(mxf, __shfl_xor(mxf, off));
        mxg = max(mxg, __shfl_xor(mxg, off));
        qmax = max(qmax, __shfl_xor(qmax, off));
        qmin = min(qmin, __shfl_xor(qmin, off));
        rtmin = fmin(rtmin, __shfl_xor(rtmin, off));
        knmax = fmax(knmax, __shfl_xor(knmax, off));
        cmax = fmax(cmax, __shfl_xor(cmax, off));
    }
    if (l == 0 && a[4] > 0) {
        atomicAdd(&st->it_sum_f, a[0]);
        atomicAdd(&st->it_sum_g, a[1]);
        atomicAdd(&st->q_sum, a[2]);
        atomicAdd(&st->limited, a[3]);
        atomicAdd(&st->cells, a[4]);
        if (a[5]) atomicAdd(&st->fallbacks, a[5]);
        atomicAdd(&st->qpass_sum, qp);
        atomicAdd(&st->row_passes, rp);
        atomicMax(&st->it_max_f, mxf);
        atomicMax(&st->it_max_g, mxg);
        atomicMax(&st->q_max, qmax);
        atomicMin(&st->q_min, qmin);
        atomicMin(&st->rt_min_bits, (unsigned long long)__double_as_longlong(rtmin));
        atomicMax(&st->kn_max_bits, (unsigned long long)__double_as_longlong(knmax));
        atomicMax(&st->colat_max_bits, (unsigned long long)__double_as_longlong(cmax));
    }
}

__device__ inline double dist3(double cx, double cy, double cz, double ux, double uy, double uz) {
#pragma clang fp contract(off)
    const double ex = cx - ux, ey = cy - uy, ez = cz - uz;
    return sqrt(ex * ex + ey * ey + ez * ez);
}

// Stencil enumeration with refinement (Eqs. IIC10-11 with D = 3): the base
// points of the ball row by row; a point within 3 2^-Lvl of u is replaced by
// its 8 children at +-h/4 (x, then y, then z sign bits), each with an eighth
// of its volume, for Lvl up to N_r.  leaf(c_x, c_y, c_z, dC) gets the exact
// velocity and volume; parent_end(d_x, d_y, d_z) follows the last leaf of a
// base point (all of whose descendants land at its displacement).
template <typename Leaf, typename End>
__device__ inline void for_each_point3(double ux, double uy, double uz, int R, int Nr, Leaf &&leaf, End &&parent_end) {
    const double rr = R + 0.5;
    const int ubx = (int)floor(ux + 0.5), uby = (int)floor(uy + 0.5), ubz = (int)floor(uz + 0.5);
    const int xlo = ubx - R - 1, xhi = ubx + R + 1;
    for (int cz = ubz - R - 1; cz <= ubz + R + 1; cz++) {
        for (int cy = uby - R - 1; cy <= uby + R + 1; cy++) {
            int xa, xb;
            if (!span3(cy, cz, ux, uy, uz, rr, xlo, xhi, xa, xb)) continue;
            for (int cx = xa; cx <= xb; cx++) {
                const double fx = cx, fy = cy, fz = cz;
                if (Nr == 0 || dist3(fx, fy, fz, ux, uy, uz) > 1.5) {
                    leaf(fx, fy, fz, 1.0);
                } else {
                    for (int k1 = 0; k1 < 8; k1++) {
                        const double ax = fx + ((k1 & 1) ? 0.25 : -0.25), ay = fy + ((k1 & 2) ? 0.25 : -0.25),
                                     az = fz + ((k1 & 4) ? 0.25 : -0.25);
                        if (Nr < 2 || dist3(ax, ay, az, ux, uy, uz) > 0.75) {
                            leaf(ax, ay, az, 0.125);
                            continue;
                        }
                        for (int k2 = 0; k2 < 8; k2++) {
                            const double bx = ax + ((k2 & 1) ? 0.125 : -0.125), by = ay + ((k2 & 2) ? 0.125 : -0.125),
                                         bz = az + ((k2 & 4) ? 0.125 : -0.125);
                            if (Nr < 3 || dist3(bx, by, bz, ux, uy, uz) > 0.375) {
                                leaf(bx, by, bz, 0.015625);
                                continue;
                            }
                            for (int k3 = 0; k3 < 8; k3++)
                                leaf(bx + ((k3 & 1) ? 0.0625 : -0.0625), by + ((k3 & 2) ? 0.0625 : -0.0625),
                                     bz + ((k3 & 4) ? 0.0625 : -0.0625), 0.001953125);
                        }
                    }
                }
                parent_end(cx, cy, cz);
            }
        }
    }
}

// Polynomial coefficients of the exponent along a stencil row (y, z fixed):
// sum_j l_j T_j = C0 + C1 x + C2 x^2 + C3 x^3 (fluon), D0 + D1 x + D2 x^2
// (phonon).
__device__ inline void row_coef(const double *lf, const double *lg, double y, double z, double *C, double *Dg) {
    const double py[4] = {1.0, y, y * y, y * y * y}, pz[4] = {1.0, z, z * z, z * z * z};
#pragma unroll
    for (int a = 0; a < 4; a++) C[a] = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) Dg[a] = 0.0;
#pragma unroll
    for (int j = 0; j < NF; j++) C[bexp(j, 0)] += lf[j] * (py[bexp(j, 1)] * pz[bexp(j, 2)]);
#pragma unroll
    for (int j = 0; j < NG; j++) Dg[bexp(j, 0)] += lg[j] * (py[bexp(j, 1)] * pz[bexp(j, 2)]);
}

// Product recurrences along a row.  With E(x) = -(1 + C0 + C1 x + C2 x^2 +
// C3 x^3) and H(x) = -(1 + D0 + D1 x + D2 x^2), unit steps in x multiply
// f = exp(E) by r = exp(E(x + 1) - E(x)), r by s2 = exp of the second
// difference and s2 by exp(-6 C3); g = exp(H) by rg, and rg by exp(-2 D2).
// row_start3 sets the five values at x0 by direct exponentials.
constexpr int REC3 = 16;   // points between direct restarts of a row's recurrences
constexpr int SPAN3_W = 13;   // k3_epr keeps the row spans of stencils with 2R + 3 <= SPAN3_W in LDS (4-bit offsets)

__device__ inline void row_start3(const double *C, const double *Dg, double x0, double &f, double &r, double &s2,
                                  double &gv, double &rg) {
    f = exp(-(1.0 + (C[0] + x0 * (C[1] + x0 * (C[2] + x0 * C[3])))));
    r = exp(-(C[1] + C[2] * (2.0 * x0 + 1.0) + C[3] * (3.0 * x0 * (x0 + 1.0) + 1.0)));
    s2 = exp(-(2.0 * C[2] + C[3] * (6.0 * x0 + 6.0)));
    gv = exp(-(1.0 + (Dg[0] + x0 * (Dg[1] + x0 * Dg[2]))));
    rg = exp(-(Dg[1] + Dg[2] * (2.0 * x0 + 1.0)));
}

// Start values in the normal range: products of them stay finite over a
// segment; otherwise the row's points are evaluated directly.
__device__ inline bool rec3_ok(double f, double r, double s2, double gv, double rg) {
    const double lo = 1e-280, hi = 1e280;
    return f > lo && f < hi && r > lo && r < hi && s2 > lo && s2 < hi && gv > lo && gv < hi && rg > lo && rg < hi;
}

// ---------------------------------------------------------------------------
// k3_epr: one lane per cell.  A pass walks the stencil row by row (z, then
// y); along a row the exponents are polynomials in x, the populations follow
// the product recurrences above (restarted every REC3 points) and the row
// accumulates sum f x^a (a <= 6) and sum g x^a (a <= 4); these are folded
// with the powers of y once per row into plane sums (sum f x^a y^b, a + b <=
// 6 and <= 4), and those with the powers of z once per plane into the
// monomial sums (degree <= 6 and <= 4) that give the residuals and Hessians.
// The final pass writes the moment fractions rho f' and rho K RT g' (Eq.
// IIE3a).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) k3_epr(G3 g, Phys ph, const double *mom, Buf3 b, int step, int tile0) {
    // LDS per workgroup (one wavefront): the row-span table (one byte per row
    // and lane) and the Newton state (multipliers and directions of both
    // species), 40,512 bytes, so that four workgroups share a CU
    __shared__ unsigned char s_span[SPAN3_W * SPAN3_W * TN];
    __shared__ double s_nw[2 * (NF + NG) * TN];
    if (b.flags->err) return;
    const int t = tile0 + blockIdx.x, l = threadIdx.x;
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    const int x = tx * TE + (l & 3), y = ty * TE + ((l >> 2) & 3), z = tz * TE + (l >> 4);
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    const long long s = valid ? ((long long)z * g.ny + y) * g.nx + x : 0;
    const int rn = valid ? b.d.r[s] : -1;
    const int R = rn & 0xffff;
    int itf = 0, itg = 0, q = 0, lim = 0, passes = 0, rows = 0, fb = 0;
    double kn = 0.0, RTc = 0.0, colat = 0.0;   // colat: |u| + R (Eq. IIC7)
    if (rn >= 0 && (rn >> 16) == 0) {
        const double rho = b.d.rho[s], ux = b.d.ux[s], uy = b.d.uy[s], uz = b.d.uz[s], RT = b.d.rt[s];
        RTc = RT;
        colat = sqrt(ux * ux + uy * uy + uz * uz) + R;
        double mf[NF], mg[NG];
        collide3(ph, mom, g.n, s, rho, ux, uy, uz, RT, mf, mg, kn, lim);
        const double rr = R + 0.5;
        const int ubx = (int)floor(ux + 0.5), uby = (int)floor(uy + 0.5), ubz = (int)floor(uz + 0.5);
        const int xlo = ubx - R - 1, xhi = ubx + R + 1, ylo = uby - R - 1, zlo = ubz - R - 1;
        // The row spans of the stencil are computed once and kept in LDS (each
        // lane its own column) for all passes, when they fit; wider stencils
        // compute them in every pass.
        const int W3 = 2 * R + 3;
        const bool tab = W3 <= SPAN3_W;
        if (tab) {
            for (int kz = 0; kz < W3; kz++)
                for (int ky = 0; ky < W3; ky++) {
                    int xa, xb;
                    unsigned char v = 0x0f;   // empty row: first offset 15, last 0
                    if (span3(ylo + ky, zlo + kz, ux, uy, uz, rr, xlo, xhi, xa, xb))
                        v = (unsigned char)((xa - xlo) | ((xb - xlo) << 4));
                    s_span[(kz * W3 + ky) * TN + l] = v;
                }
        }
        auto span = [&](int cy, int cz, int &xa, int &xb) -> bool {
            if (tab) {
                const unsigned v = s_span[((cz - zlo) * W3 + (cy - ylo)) * TN + l];
                xa = xlo + (int)(v & 0xfu);
                xb = xlo + (int)(v >> 4);
                return xa <= xb;
            }
            return span3(cy, cz, ux, uy, uz, rr, xlo, xhi, xa, xb);
        };
        Sp3<NF, LdsStore3<NF>> sf;
        Sp3<NG, LdsStore3<NG>> sg;
        sf.v.l = s_nw + l; sf.v.d = s_nw + NF * TN + l;
        sg.v.l = s_nw + 2 * NF * TN + l; sg.v.d = s_nw + (2 * NF + NG) * TN + l;
        sp3_init(sf, RT);
        sp3_init(sg, RT);
        if (b.ainv) sp3_linear(sf, sg, mf, mg, RT, b.ainv);
        if (b.prev) sp3_prev(sf, sg, RT, b.prev, g.n, s);
        const double isc[4] = {1.0, 1.0 / sqrt(RT), 1.0 / RT, 1.0 / (RT * sqrt(RT))};
        int fail = 0, fsp = -1;
        while (!fail && (sf.phase < 2 || sg.phase < 2)) {
            passes++;
            double Sf[NMF], Sg[NMG], lf[NF], lg[NG];
#pragma unroll
            for (int k = 0; k < NMF; k++) Sf[k] = 0.0;
#pragma unroll
            for (int k = 0; k < NMG; k++) Sg[k] = 0.0;
#pragma unroll
            for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
            for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
            // third and second differences of the exponents along x (basis
            // terms xxx and xx): the same on every row
            const double t3 = exp(-6.0 * lf[10]), sg2 = exp(-2.0 * lg[4]);
            for (int cz = ubz - R - 1; cz <= ubz + R + 1; cz++) {
                const double zz = (double)cz - uz;
                double Pf[28], Pg[15];   // plane sums, index (a + b)(a + b + 1)/2 + b
#pragma unroll
                for (int k = 0; k < 28; k++) Pf[k] = 0.0;
#pragma unroll
                for (int k = 0; k < 15; k++) Pg[k] = 0.0;
                bool any = false;
                for (int cy = uby - R - 1; cy <= uby + R + 1; cy++) {
                    int xa, xb;
                    if (!span(cy, cz, xa, xb)) continue;
                    any = true;
                    const double yy = (double)cy - uy;
                    double C[4], Dg[3];
                    row_coef(lf, lg, yy, zz, C, Dg);
                    double Rf[7] = {0, 0, 0, 0, 0, 0, 0}, Rg[5] = {0, 0, 0, 0, 0};
                    double f, r, s2, gv, rg;
                    bool direct = false;
                    for (int cx = xa; cx <= xb; cx++) {
                        const double xx = (double)cx - ux;
                        if (((cx - xa) & (REC3 - 1)) == 0) {
                            row_start3(C, Dg, xx, f, r, s2, gv, rg);
                            direct = !rec3_ok(f, r, s2, gv, rg);
                        }
                        if (direct) {
                            f = exp(-(1.0 + (C[0] + xx * (C[1] + xx * (C[2] + xx * C[3])))));
                            gv = exp(-(1.0 + (Dg[0] + xx * (Dg[1] + xx * Dg[2]))));
                        }
                        double p = f;
                        Rf[0] += p;
#pragma unroll
                        for (int a = 1; a < 7; a++) { p *= xx; Rf[a] += p; }
                        p = gv;
                        Rg[0] += p;
#pragma unroll
                        for (int a = 1; a < 5; a++) { p *= xx; Rg[a] += p; }
                        f *= r; r *= s2; s2 *= t3;
                        gv *= rg; rg *= sg2;
                    }
                    double py[7];
                    py[0] = 1.0;
#pragma unroll
                    for (int k = 1; k < 7; k++) py[k] = py[k - 1] * yy;
#pragma unroll
                    for (int a = 0; a < 7; a++)
#pragma unroll
                        for (int bb = 0; bb + a < 7; bb++) Pf[(a + bb) * (a + bb + 1) / 2 + bb] += Rf[a] * py[bb];
#pragma unroll
                    for (int a = 0; a < 5; a++)
#pragma unroll
                        for (int bb = 0; bb + a < 5; bb++) Pg[(a + bb) * (a + bb + 1) / 2 + bb] += Rg[a] * py[bb];
                }
                if (!any) continue;
                double pz[7];
                pz[0] = 1.0;
#pragma unroll
                for (int k = 1; k < 7; k++) pz[k] = pz[k - 1] * zz;
#pragma unroll
                for (int a = 0; a < 7; a++)
#pragma unroll
                    for (int bb = 0; bb + a < 7; bb++)
#pragma unroll
                        for (int c = 0; c + bb + a < 7; c++) Sf[mono(a, bb, c)] += Pf[(a + bb) * (a + bb + 1) / 2 + bb] * pz[c];
#pragma unroll
                for (int a = 0; a < 5; a++)
#pragma unroll
                    for (int bb = 0; bb + a < 5; bb++)
#pragma unroll
                        for (int c = 0; c + bb + a < 5; c++) Sg[mono(a, bb, c)] += Pg[(a + bb) * (a + bb + 1) / 2 + bb] * pz[c];
            }
            if (sg.phase < 2) {
                int r = sp3_update(sg, Sg, mg, isc, ph.tol, ph.maxit);
                if (r < 0 && r != -3 && sg.lin) r = 2;
                if (r < 0) { fail = -r; fsp = 1; }
                else if (r == 2) { sp3_init(sg, RT); fb = 1; }
            }
            if (sf.phase < 2 && !fail) {
                int r = sp3_update(sf, Sf, mf, isc, ph.tol, ph.maxit);
                if (r < 0 && r != -3 && sf.lin) r = 2;
                if (r < 0) { fail = -r; fsp = 0; }
                else if (r == 2) { sp3_init(sf, RT); fb = 1; }
            }
        }
        if (fail) {
            flag3(b.flags, LELBM_EEPR, step, s, fail, fsp, fsp ? sg.res : sf.res);
        } else {
            itf = sf.nit;
            itg = sg.nit;
            if (b.prev) sp3_store_prev(sf, sg, mf, mg, RT, b.ainv, b.prev, g.n, s);
            const double wsf = rho, wsg = rho * ph.K * RT;
            const Tile3 ti = b.tiles[t];
            T *P = (T *)b.scratch + ti.base;
            double lf[NF], lg[NG];
#pragma unroll
            for (int j = 0; j < NF; j++) lf[j] = sf.lam(j);
#pragma unroll
            for (int j = 0; j < NG; j++) lg[j] = sg.lam(j);
            const double t3 = exp(-6.0 * lf[10]), sg2 = exp(-2.0 * lg[4]);
            for (int cz = ubz - R - 1; cz <= ubz + R + 1; cz++) {
                const double zz = (double)cz - uz;
                for (int cy = uby - R - 1; cy <= uby + R + 1; cy++) {
                    int xa, xb;
                    if (!span(cy, cz, xa, xb)) continue;
                    rows++;
                    const double yy = (double)cy - uy;
                    double C[4], Dg[3];
                    row_coef(lf, lg, yy, zz, C, Dg);
                    const long long row = ((long long)(cz - ti.oz) * ti.wy + (cy - ti.oy)) * ti.wx - ti.ox;
                    double f, r, s2, gv, rg;
                    bool direct = false;
                    for (int cx = xa; cx <= xb; cx++) {
                        const double xx = (double)cx - ux;
                        if (((cx - xa) & (REC3 - 1)) == 0) {
                            row_start3(C, Dg, xx, f, r, s2, gv, rg);
                            direct = !rec3_ok(f, r, s2, gv, rg);
                        }
                        if (direct) {
                            f = exp(-(1.0 + (C[0] + xx * (C[1] + xx * (C[2] + xx * C[3])))));
                            gv = exp(-(1.0 + (Dg[0] + xx * (Dg[1] + xx * Dg[2]))));
                        }
                        const double wf = wsf * f, wg = wsg * gv;
                        if (ti.fmt == 0) {
                            const long long e = ((row + cx) * TN + l) * 2;
                            __builtin_nontemporal_store((T)wf, &P[e]);
                            __builtin_nontemporal_store((T)wg, &P[e + 1]);
                        } else {
                            double mo[NM];
                            moments17((double)cx, (double)cy, (double)cz, wf, wg, mo);
                            const long long e = ((row + cx) * TN + l) * NM;
#pragma unroll
                            for (int k = 0; k < NM; k++) P[e + k] = (T)mo[k];
                        }
                        f *= r; r *= s2; s2 *= t3;
                        gv *= rg; rg *= sg2;
                        q++;
                    }
                }
            }
            passes++;
        }
    }
    stats3(b.stats, itf, itg, q, lim, fb, passes, rows, RTc, kn, colat, l);
}

// ---------------------------------------------------------------------------
// k3_epr_ref: cells with refined stencils (their tiles only), one lane per
// cell, every point visited with direct exponentials of the full basis
// polynomials; the final pass writes, per base point, the 17 moments of its
// descendants' moment fractions with their exact velocities.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) k3_epr_ref(G3 g, Phys ph, const double *mom, Buf3 b, int step, int tile0) {
    __shared__ int s_skip;
    const int t = tile0 + blockIdx.x, l = threadIdx.x;
    if (l == 0) s_skip = b.flags->err || !b.tiles[t].fmt;
    __syncthreads();
    if (s_skip) return;
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    const int x = tx * TE + (l & 3), y = ty * TE + ((l >> 2) & 3), z = tz * TE + (l >> 4);
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    const long long s = valid ? ((long long)z * g.ny + y) * g.nx + x : 0;
    const int rn = valid ? b.d.r[s] : -1;
    const int R = rn & 0xffff, Nr = rn >> 16;
    int itf = 0, itg = 0, q = 0, lim = 0, passes = 0, fb = 0;
    double kn = 0.0, RTc = 0.0, colat = 0.0;   // colat: |u| + R (Eq. IIC7)
    if (rn >= 0 && Nr > 0) {
        const double rho = b.d.rho[s], ux = b.d.ux[s], uy = b.d.uy[s], uz = b.d.uz[s], RT = b.d.rt[s];
        RTc = RT;
        colat = sqrt(ux * ux + uy * uy + uz * uz) + R;
        double mf[NF], mg[NG];
        collide3(ph, mom, g.n, s, rho, ux, uy, uz, RT, mf, mg, kn, lim);
        Sp3<NF> sf;
        Sp3<NG> sg;
        sp3_init(sf, RT);
        sp3_init(sg, RT);
        if (b.ainv) sp3_linear(sf, sg, mf, mg, RT, b.ainv);
        const double isc[4] = {1.0, 1.0 / sqrt(RT), 1.0 / RT, 1.0 / (RT * sqrt(RT))};
        int fail = 0, fsp = -1;
        while (!fail && (sf.phase < 2 || sg.phase < 2)) {
            passes++;
            double Sf[NMF], Sg[NMG], lf[NF], lg[NG];
#pragma unroll
            for (int k = 0; k < NMF; k++) Sf[k] = 0.0;
#pragma unroll
            for (int k = 0; k < NMG; k++) Sg[k] = 0.0;
#pragma unroll
            for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
            for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
            for_each_point3(
                ux, uy, uz, R, Nr,
                [&](double cx, double cy, double cz, double dC) {
                    double px[7], py[7], pz[7];
                    px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
                    for (int k = 1; k < 7; k++) {
                        px[k] = px[k - 1] * (cx - ux);
                        py[k] = py[k - 1] * (cy - uy);
                        pz[k] = pz[k - 1] * (cz - uz);
                    }
                    double ef = 0.0, eg = 0.0;
#pragma unroll
                    for (int j = 0; j < NF; j++) ef += lf[j] * (px[bexp(j, 0)] * py[bexp(j, 1)] * pz[bexp(j, 2)]);
#pragma unroll
                    for (int j = 0; j < NG; j++) eg += lg[j] * (px[bexp(j, 0)] * py[bexp(j, 1)] * pz[bexp(j, 2)]);
                    const double f = dC * exp(-(1.0 + ef)), gv = dC * exp(-(1.0 + eg));
#pragma unroll
                    for (int a = 0; a < 7; a++)
#pragma unroll
                        for (int bb = 0; bb + a < 7; bb++)
#pragma unroll
                            for (int c = 0; c + bb + a < 7; c++) {
                                const double m = px[a] * (py[bb] * pz[c]);
                                Sf[mono(a, bb, c)] += f * m;
                                if (a + bb + c <= 4) Sg[mono(a, bb, c)] += gv * m;
                            }
                },
                [](int, int, int) {});
            if (sg.phase < 2) {
                int r = sp3_update(sg, Sg, mg, isc, ph.tol, ph.maxit);
                if (r < 0 && r != -3 && sg.lin) r = 2;
                if (r < 0) { fail = -r; fsp = 1; }
                else if (r == 2) { sp3_init(sg, RT); fb = 1; }
            }
            if (sf.phase < 2 && !fail) {
                int r = sp3_update(sf, Sf, mf, isc, ph.tol, ph.maxit);
                if (r < 0 && r != -3 && sf.lin) r = 2;
                if (r < 0) { fail = -r; fsp = 0; }
                else if (r == 2) { sp3_init(sf, RT); fb = 1; }
            }
        }
        if (fail) {
            flag3(b.flags, LELBM_EEPR, step, s, fail, fsp, fsp ? sg.res : sf.res);
        } else {
            itf = sf.nit;
            itg = sg.nit;
            // refined cells keep no correction: their next step starts from the
            // linearised guess
            if (b.prev)
                for (int i = 0; i < NF + NG; i++) b.prev[(long long)i * g.n + s] = __longlong_as_double(-1ll);
            const double wsf = rho, wsg = rho * ph.K * RT;
            const Tile3 ti = b.tiles[t];
            T *P = (T *)b.scratch + ti.base;
            double acc[NM];
#pragma unroll
            for (int k = 0; k < NM; k++) acc[k] = 0.0;
            for_each_point3(
                ux, uy, uz, R, Nr,
                [&](double cx, double cy, double cz, double dC) {
                    const double x1 = cx - ux, y1 = cy - uy, z1 = cz - uz;
                    const double px[4] = {1.0, x1, x1 * x1, x1 * x1 * x1}, py[4] = {1.0, y1, y1 * y1, y1 * y1 * y1},
                                 pz[4] = {1.0, z1, z1 * z1, z1 * z1 * z1};
                    double ef = 0.0, eg = 0.0;
#pragma unroll
                    for (int j = 0; j < NF; j++)
                        ef += sf.lam(j) * (px[bexp(j, 0)] * py[bexp(j, 1)] * pz[bexp(j, 2)]);
#pragma unroll
                    for (int j = 0; j < NG; j++)
                        eg += sg.lam(j) * (px[bexp(j, 0)] * py[bexp(j, 1)] * pz[bexp(j, 2)]);
                    double mo[NM];
                    moments17(cx, cy, cz, wsf * (dC * exp(-(1.0 + ef))), wsg * (dC * exp(-(1.0 + eg))), mo);
#pragma unroll
                    for (int k = 0; k < NM; k++) acc[k] += mo[k];
                    q++;
                },
                [&](int dx, int dy, int dz) {
                    const long long slot = ((long long)(dz - ti.oz) * ti.wy + (dy - ti.oy)) * ti.wx + (dx - ti.ox);
#pragma unroll
                    for (int k = 0; k < NM; k++) {
                        P[(slot * TN + l) * NM + k] = (T)acc[k];
                        acc[k] = 0.0;
                    }
                });
            passes++;
        }
    }
    stats3(b.stats, itf, itg, q, lim, fb, passes, 0, RTc, kn, colat, l);
}

// ---------------------------------------------------------------------------
// k3_gather: one lane per destination cell; every displacement d with
// |d_a| <= the step's reach M is tested against the stencil of its source x
// - d (wrapped) with the reconstruction's own predicate; a hit adds the
// source's record with velocity d (Eq. IIE3b).  A workgroup takes a
// GX x GY x 1 block of destinations (GY = 16, or 8 where the staged plane
// of 16 rows does not fit the LDS); for each d_z the descriptors of the
// source plane it needs ((GX + 2M) x (GY + 2M) cells: velocity, the test's
// terms that do not depend on d_x and d_y, and the address of the source's
// record of displacement (0, 0, d_z)) are staged in LDS, with the bounds of
// the plane's velocities and radii, which narrow each row of d_x to the
// displacements some source can reach.  Along a row of d_x the row sums of
// w_f c_x^k (k <= 3) and w_g c_x^k (k <= 1) are formed, and the 17 moments
// once per row.
// ---------------------------------------------------------------------------
constexpr int GX = 16;
constexpr int G3_ENTRY_BYTES = 44;
constexpr int G3U = 4;   // candidates per batch in the gather

// The (w_f, w_g) pair of a record, read as one load.
template <typename T> struct Pair3;
template <> struct Pair3<double> { using type = double2; };
template <> struct Pair3<float> { using type = float2; };

struct RowSums {
    double fr = 0, fx = 0, fxx = 0, fxxx = 0, gr = 0, gx = 0;
    __device__ void add(double wf, double wg, double cx) {
        const double w1 = cx * wf, w2 = cx * w1;
        fr += wf; fx += w1; fxx += w2; fxxx += cx * w2;
        gr += wg; gx += cx * wg;
    }
    __device__ void fold(double *acc, int dy, int dz) const {
        const double cy = (double)dy, cz = (double)dz, c2 = cy * cy + cz * cz;
        acc[0] += fr;
        acc[1] += fx; acc[2] += cy * fr; acc[3] += cz * fr;
        acc[4] += fxx; acc[5] += cy * fx; acc[6] += cz * fx;
        acc[7] += cy * cy * fr; acc[8] += cy * cz * fr; acc[9] += cz * cz * fr;
        // |c|^2 c_g = (c_x^2 + c_y^2 + c_z^2) c_g
        acc[10] += fxxx + c2 * fx;
        acc[11] += cy * fxx + c2 * cy * fr;
        acc[12] += cz * fxx + c2 * cz * fr;
        acc[13] += gr; acc[14] += gx; acc[15] += cy * gr; acc[16] += cz * gr;
    }
};

template <typename T, int GY>
__global__ void __launch_bounds__(GX * GY, 4) k3_gather(G3 g, double *out, Buf3 b, int M, int zb) {
    extern __shared__ double g3_lds[];
    if (b.flags->err) return;
    const int W = GX + 2 * M, H = GY + 2 * M, NE = W * H;
    // per staged source of the plane d_z: u_x, u_y, (d_z - u_z)^2, (R + 1/2)^2
    // (-1: no source, or one with all-moment records), the address of its
    // record of displacement (0, 0, d_z), the slot box row length w_x, and
    // R | fmt << 20 (-1: no source) for the sources with all-moment records
    // three 16-byte vectors per entry, so that a candidate takes three LDS reads
    double2 *s_u = (double2 *)g3_lds, *s_t = s_u + NE;   // (u_x, u_y), ((d_z - u_z)^2, (R + 1/2)^2)
    long long *s_aw = (long long *)(s_t + NE);          // record address << 16 | w_x
    int *s_r = (int *)(s_aw + NE);
    const int bx = (g.nx + GX - 1) / GX, by = (g.ny + GY - 1) / GY;
    // workgroups go to the eight XCDs in turn; each XCD is dealt one contiguous
    // run of the (x, y, z)-ordered blocks (a bijection onto [0, gridDim.x)), so
    // that neighbouring blocks, which read the same record lines, share an L2
    const int xq = gridDim.x / 8, xr = gridDim.x % 8, xcd = blockIdx.x % 8;
    const int blk = xcd * xq + min(xcd, xr) + blockIdx.x / 8;
    const int x0 = (blk % bx) * GX, y0 = ((blk / bx) % by) * GY, z = zb + blk / (bx * by);
    const int lx = threadIdx.x % GX, ly = threadIdx.x / GX;
    const int x = x0 + lx, y = y0 + ly;
    const bool mine = x < g.nx && y < g.ny;
    const T *SCR = (const T *)b.scratch;
    double acc[NM];
#pragma unroll
    for (int k = 0; k < NM; k++) acc[k] = 0.0;
    unsigned long long hits = 0;
    // bounds of the staged sources' velocities (in 1/1024 cells, rounded
    // outwards) and their largest radius: a row (d_y, d_z) can only hold hits
    // with |d_x - u_x| <= sqrt(rr^2 - dist(d_y, [u_y])^2 - dist(d_z, [u_z])^2)
    __shared__ int s_bnd[8];   // [7]: some staged source has all-moment records
    for (int dz = -M; dz <= M; dz++) {
        const int sz = wrapi(z - dz, g.nz);
        __syncthreads();
        if (threadIdx.x == 0) {
            s_bnd[0] = s_bnd[2] = s_bnd[4] = INT_MAX;
            s_bnd[1] = s_bnd[3] = s_bnd[5] = INT_MIN;
            s_bnd[6] = -1;
            s_bnd[7] = 0;
        }
        __syncthreads();
        int bl[3] = {INT_MAX, INT_MAX, INT_MAX}, bh[3] = {INT_MIN, INT_MIN, INT_MIN}, brm = -1, anyref = 0;
        for (int e = threadIdx.x; e < NE; e += GX * GY) {
            const int sx = wrapi(x0 - M + e % W, g.nx), sy = wrapi(y0 - M + e / W, g.ny);
            const long long s = ((long long)sz * g.ny + sy) * g.nx + sx;
            const int rn = b.d.r[s];
            if (rn < 0) {
                s_r[e] = -1;
                s_u[e] = make_double2(0.0, 0.0);
                s_t[e] = make_double2(0.0, -1.0);
                s_aw[e] = 0;
                continue;
            }
            const double uu[3] = {b.d.ux[s], b.d.uy[s], b.d.uz[s]};
#pragma unroll
            for (int k = 0; k < 3; k++) {
                bl[k] = min(bl[k], (int)floor(uu[k] * 1024.0));
                bh[k] = max(bh[k], (int)ceil(uu[k] * 1024.0));
            }
            brm = max(brm, rn & 0xffff);
            const Tile3 ti = b.tiles[(sz / TE * g.tny + sy / TE) * g.tnx + sx / TE];
            const int loc = (sz % TE) * 16 + (sy % TE) * 4 + (sx % TE);
            const long long rs = ti.fmt ? NM : 2;
            const double rr = (double)(rn & 0xffff) + 0.5, ez = (double)dz - uu[2];
            s_r[e] = (rn & 0xffff) | (ti.fmt << 20);
            anyref |= ti.fmt;
            s_u[e] = make_double2(uu[0], uu[1]);
            // the terms of the exact test (in_ball) that do not depend on d_x, d_y
            s_t[e] = make_double2(ez * ez, ti.fmt ? -1.0 : rr * rr);
            const long long a0 = ti.base + (long long)loc * rs +
                                 (((long long)(dz - ti.oz) * ti.wy - ti.oy) * ti.wx - ti.ox) * (TN * rs);
            s_aw[e] = (long long)((unsigned long long)a0 << 16) | (long long)ti.wx;
        }
        if (brm >= 0) {
#pragma unroll
            for (int k = 0; k < 3; k++) { atomicMin(&s_bnd[2 * k], bl[k]); atomicMax(&s_bnd[2 * k + 1], bh[k]); }
            atomicMax(&s_bnd[6], brm);
        }
        if (anyref) s_bnd[7] = 1;
        __syncthreads();
        if (!mine || s_bnd[6] < 0) continue;
        const bool ref = s_bnd[7] != 0;
        const double q = 1.0 / 1024.0, rrm = s_bnd[6] + 0.5;
        const double ddz = fmax(0.0, fmax(s_bnd[4] * q - (double)dz, (double)dz - s_bnd[5] * q));
        for (int dy = -M; dy <= M; dy++) {
            const double ddy = fmax(0.0, fmax(s_bnd[2] * q - (double)dy, (double)dy - s_bnd[3] * q));
            const double rem = rrm * rrm - ddz * ddz - ddy * ddy;
            if (rem < 0.0) continue;
            // the slack of 1e-6 covers the rounding of the exact test
            const double hw = sqrt(rem);
            const int dxlo = max(-M, (int)ceil(s_bnd[0] * q - hw - 1e-6));
            const int dxhi = min(M, (int)floor(s_bnd[1] * q + hw + 1e-6));
            RowSums rs;
            const int rowe = (ly - dy + M) * W + lx + M;
            const double cy = (double)dy;
            // Straight-line candidates: each reads its entry and one record
            // pair (a miss reads the scratch's first pair and adds zeros), so
            // no per-lane branches; G3U candidates per batch, their record
            // loads in flight together (entries past dxhi are masked and read
            // the row's first entry).
            for (int dxb = dxlo; dxb <= dxhi; dxb += G3U) {
                bool in[G3U];
                typename Pair3<T>::type v[G3U];
#pragma unroll
                for (int u = 0; u < G3U; u++) {
                    const int dx = dxb + u;
                    const int e = rowe - (dx <= dxhi ? dx : dxlo);
                    const double2 su = s_u[e], st = s_t[e];
                    const long long aw = s_aw[e], a0 = aw >> 16;
                    const int wx = (int)(aw & 0xffff);
                    const double ex = (double)dx - su.x, ey = cy - su.y;
                    bool hit;
                    {
                        // in_ball's expression, term for term
#pragma clang fp contract(off)
                        hit = ex * ex + ey * ey + st.x <= st.y;
                    }
                    in[u] = (dx <= dxhi) & hit;
                    const long long off = a0 + (long long)(dy * wx + dx) * (TN * 2);
                    v[u] = *(const typename Pair3<T>::type *)(SCR + (in[u] ? off : 0ll));
                }
#pragma unroll
                for (int u = 0; u < G3U; u++) {
                    hits += in[u] ? 1 : 0;
                    rs.add(in[u] ? (double)v[u].x : 0.0, in[u] ? (double)v[u].y : 0.0, (double)(dxb + u));
                }
            }
            if (ref) {
                // sources with all-moment records: the pre-summed moments of a
                // base point's descendants
                for (int dx = dxlo; dx <= dxhi; dx++) {
                    const int e = rowe - dx;
                    const int m = s_r[e];
                    if (m < 0 || !(m >> 20)) continue;
                    const double2 su = s_u[e];
                    const double ex = (double)dx - su.x, ey = cy - su.y, rr = (double)(m & 0xffff) + 0.5;
                    bool hit;
                    {
#pragma clang fp contract(off)
                        hit = ex * ex + ey * ey + s_t[e].x <= rr * rr;
                    }
                    if (!hit) continue;
                    hits++;
                    const long long aw = s_aw[e];
                    const T *P = SCR + (aw >> 16) + (long long)(dy * (int)(aw & 0xffff) + dx) * (TN * NM);
#pragma unroll
                    for (int k = 0; k < NM; k++) acc[k] += (double)P[k];
                }
            }
            rs.fold(acc, dy, dz);
        }
    }
    if (mine) {
        const long long o = ((long long)z * g.ny + y) * g.nx + x;
#pragma unroll
        for (int k = 0; k < NM; k++) out[k * g.n + o] = acc[k];
    }
    for (int off = 32; off > 0; off >>= 1) hits += __shfl_xor(hits, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(&b.stats->arrivals, hits);
}

// The same without staging, for reaches whose source planes do not fit the
// LDS: descriptors straight from global memory.
template <typename T>
__global__ void __launch_bounds__(64) k3_gather_wide(G3 g, double *out, Buf3 b, int tile0) {
    if (b.flags->err) return;
    const int t = tile0 + blockIdx.x, l = threadIdx.x;
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    const int x = tx * TE + (l & 3), y = ty * TE + ((l >> 2) & 3), z = tz * TE + (l >> 4);
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    const int M = *b.maxreach;
    const T *SCR = (const T *)b.scratch;
    double acc[NM];
#pragma unroll
    for (int k = 0; k < NM; k++) acc[k] = 0.0;
    unsigned long long hits = 0;
    for (int dz = -M; dz <= M; dz++) {
        const int sz = wrapi(z - dz, g.nz);
        for (int dy = -M; dy <= M; dy++) {
            const int sy = wrapi(y - dy, g.ny);
            RowSums rs;
            for (int dx = -M; dx <= M; dx++) {
                const int sx = wrapi(x - dx, g.nx);
                const long long s = ((long long)sz * g.ny + sy) * g.nx + sx;
                const int rn = b.d.r[s];
                if (rn < 0) continue;
                if (!in_ball((double)dx, (double)dy, (double)dz, b.d.ux[s], b.d.uy[s], b.d.uz[s], (rn & 0xffff) + 0.5))
                    continue;
                const Tile3 ti = b.tiles[(sz / TE * g.tny + sy / TE) * g.tnx + sx / TE];
                const int loc = (sz % TE) * 16 + (sy % TE) * 4 + (sx % TE);
                const long long slot = ((long long)(dz - ti.oz) * ti.wy + (dy - ti.oy)) * ti.wx + (dx - ti.ox);
                hits++;
                if (ti.fmt) {
                    const T *P = SCR + ti.base + (slot * TN + loc) * NM;
#pragma unroll
                    for (int k = 0; k < NM; k++) acc[k] += (double)P[k];
                    continue;
                }
                const T *P = SCR + ti.base + (slot * TN + loc) * 2;
                rs.add((double)P[0], (double)P[1], (double)dx);
            }
            rs.fold(acc, dy, dz);
        }
    }
    const long long o = ((long long)z * g.ny + y) * g.nx + x;
#pragma unroll
    for (int k = 0; k < NM; k++) out[k * g.n + o] = acc[k];
    for (int off = 32; off > 0; off >>= 1) hits += __shfl_xor(hits, off);
    if (l == 0) atomicAdd(&b.stats->arrivals, hits);
}

// Conserved totals (mass, x and y momentum, energy trace): block partials,
// then one ordered sum.
__global__ void __launch_bounds__(256) k3_sums(G3 g, const double *mom, double *partial) {
    __shared__ double sh[4][256];
    double a[4] = {0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (long long)gridDim.x * 256) {
        a[0] += mom[i];
        a[1] += mom[g.n + i];
        a[2] += mom[2 * g.n + i];
        a[3] += mom[4 * g.n + i] + mom[7 * g.n + i] + mom[9 * g.n + i] + mom[13 * g.n + i];
    }
    for (int k = 0; k < 4; k++) sh[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 4; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; k++) partial[blockIdx.x * 4 + k] = sh[k][0];
}

__global__ void k3_sums_final(int nb, double *partial) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a[4] = {0, 0, 0, 0};
        for (int i = 0; i < nb; i++)
            for (int k = 0; k < 4; k++) a[k] += partial[i * 4 + k];
        for (int k = 0; k < 4; k++) partial[nb * 4 + k] = a[k];
    }
}

__global__ void k3_reset(Buf3 b, int stats) {
    if (threadIdx.x == 0) {
        *b.maxreach = 0;
        if (stats) {
            DevStats z = {};
            z.q_min = INT_MAX;
            z.rt_min_bits = 0x7fefffffffffffffull;
            *b.stats = z;
        }
    }
}

__global__ void __launch_bounds__(256) k3_load(long long n, const void *src, int fp32, double *dst) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = fp32 ? (double)((const float *)src)[i] : ((const double *)src)[i];
}

}  // namespace d3

// ---------------------------------------------------------------------------
// host side of the 3D path
// ---------------------------------------------------------------------------
using namespace d3;

struct Ctx3 {
    G3 g;
    Phys ph;
    int mixed;
    hipStream_t stream;
    Buf3 b;
    int cur;
    int nsum;                 // blocks of k3_sums
    long long persistent;     // bytes
    void *host_small;         // pinned: flags, reach, statistics, layer sizes
    long long *layer;         // [tnz] record elements per layer of tiles (device)
    long long budget;         // record scratch budget (bytes)
    Plan plan;                // bands of tile layers and their schedule (host)
    std::vector<long long> hlayers;
    double *ainv_dev;         // the linearised start's matrices (device), or NULL
};

// Inverses of the scaled Maxwellian Hessians <T_i T_j> (unit normal
// distribution in 3D: E[x^n] = 0 for odd n, 1, 1, 3, 15 for n = 0, 2, 4, 6)
// of the fluon (19 x 19) and phonon (10 x 10) bases, by Gauss-Jordan
// elimination with partial pivoting.
static void lin_inverse(std::vector<double> &out) {
    auto gm = [](int n) { return n % 2 ? 0.0 : (n == 0 ? 1.0 : (n == 2 ? 1.0 : (n == 4 ? 3.0 : 15.0))); };
    out.clear();
    for (int nb : {NF, NG}) {
        std::vector<double> A((size_t)nb * 2 * nb, 0.0);
        for (int i = 0; i < nb; i++) {
            for (int j = 0; j < nb; j++)
                A[(size_t)i * 2 * nb + j] =
                    gm(bexp(i, 0) + bexp(j, 0)) * gm(bexp(i, 1) + bexp(j, 1)) * gm(bexp(i, 2) + bexp(j, 2));
            A[(size_t)i * 2 * nb + nb + i] = 1.0;
        }
        for (int c = 0; c < nb; c++) {
            int p = c;
            for (int r = c + 1; r < nb; r++)
                if (fabs(A[(size_t)r * 2 * nb + c]) > fabs(A[(size_t)p * 2 * nb + c])) p = r;
            for (int k = 0; k < 2 * nb; k++) std::swap(A[(size_t)c * 2 * nb + k], A[(size_t)p * 2 * nb + k]);
            const double piv = A[(size_t)c * 2 * nb + c];
            for (int k = 0; k < 2 * nb; k++) A[(size_t)c * 2 * nb + k] /= piv;
            for (int r = 0; r < nb; r++) {
                if (r == c) continue;
                const double f = A[(size_t)r * 2 * nb + c];
                for (int k = 0; k < 2 * nb; k++) A[(size_t)r * 2 * nb + k] -= f * A[(size_t)c * 2 * nb + k];
            }
        }
        for (int i = 0; i < nb; i++)
            for (int j = 0; j < nb; j++) out.push_back(A[(size_t)i * 2 * nb + nb + j]);
    }
}

#define H3(x)                                 \
    do {                                      \
        if ((x) != hipSuccess) return LELBM_EDEVICE; \
    } while (0)

static void free3(Ctx3 *c) {
    if (!c) return;
    Buf3 &b = c->b;
    void *ptrs[] = {b.mom[0], b.mom[1], b.d.rho, b.d.ux, b.d.uy, b.d.uz, b.d.rt, b.d.r, b.tiles, b.scratch,
                    b.flags, b.stats, b.maxreach, b.total, b.partial, c->layer, c->ainv_dev, b.prev};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->host_small) (void)hipHostFree(c->host_small);
    delete c;
}

int ctx3_create(const lelbm_params *p, const Phys &ph, int mixed, const void *moments, int src_fp32, int on_device,
                hipStream_t stream, Ctx3 **out) {
    Ctx3 *c = new Ctx3();
    memset(&c->b, 0, sizeof(c->b));
    c->host_small = nullptr;
    c->layer = nullptr;
    c->ainv_dev = nullptr;
    c->budget = LELBM_DEFAULT_SCRATCH_BUDGET;
    G3 &g = c->g;
    g.nx = p->nx; g.ny = p->ny; g.nz = p->nz;
    g.n = (long long)g.nx * g.ny * g.nz;
    g.tnx = (g.nx + TE - 1) / TE; g.tny = (g.ny + TE - 1) / TE; g.tnz = (g.nz + TE - 1) / TE;
    g.ntiles = g.tnx * g.tny * g.tnz;
    c->ph = ph;
    c->mixed = mixed;
    c->stream = stream;
    c->cur = 0;
    c->nsum = (int)std::min<long long>((g.n + 255) / 256, 1024);
    Buf3 &b = c->b;
    bool ok = true;
    auto alloc = [&](void **q, size_t bytes) { ok = ok && hipMalloc(q, bytes) == hipSuccess; };
    alloc((void **)&b.mom[0], (size_t)NM * g.n * sizeof(double));
    alloc((void **)&b.mom[1], (size_t)NM * g.n * sizeof(double));
    for (double **q : {&b.d.rho, &b.d.ux, &b.d.uy, &b.d.uz, &b.d.rt}) alloc((void **)q, (size_t)g.n * sizeof(double));
    alloc((void **)&b.d.r, (size_t)g.n * sizeof(int));
    alloc((void **)&b.tiles, (size_t)g.ntiles * sizeof(Tile3));
    alloc((void **)&b.flags, sizeof(Flags));
    alloc((void **)&b.stats, sizeof(DevStats));
    alloc((void **)&b.maxreach, sizeof(int));
    alloc((void **)&b.total, sizeof(long long));
    alloc((void **)&b.partial, (size_t)(c->nsum + 1) * 4 * sizeof(double));
    alloc((void **)&c->layer, (size_t)g.tnz * sizeof(long long));
    if (ph.prev_guess) {
        alloc((void **)&b.prev, (size_t)(NF + NG) * g.n * sizeof(double));
        // all-ones bytes are a NaN: no stored correction yet (on the context's
        // stream, ahead of its first step)
        if (ok) ok = hipMemsetAsync(b.prev, 0xff, (size_t)(NF + NG) * g.n * sizeof(double), stream) == hipSuccess;
    }
    if (ph.lin_guess || ph.prev_guess) {
        std::vector<double> ai;
        lin_inverse(ai);
        alloc((void **)&c->ainv_dev, ai.size() * sizeof(double));
        if (ok) ok = hipMemcpy(c->ainv_dev, ai.data(), ai.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
        b.ainv = c->ainv_dev;
    }
    ok = ok && hipHostMalloc(&c->host_small, 4096 + (size_t)g.tnz * sizeof(long long), hipHostMallocDefault) ==
                   hipSuccess;
    if (!ok) { free3(c); return LELBM_ENOMEM; }
    c->persistent = (long long)2 * NM * g.n * 8 + g.n * (5 * 8 + 4) + (long long)g.ntiles * sizeof(Tile3) +
                    (b.prev ? (long long)(NF + NG) * g.n * 8 : 0);
    // state
    const long long tot = (long long)NM * g.n;
    if (on_device) {
        hipLaunchKernelGGL(k3_load, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream, tot, moments, src_fp32,
                           b.mom[0]);
        if (hipGetLastError() != hipSuccess) { free3(c); return LELBM_EDEVICE; }
    } else {
        if (hipMemcpyAsync(b.mom[0], moments, (size_t)tot * sizeof(double), hipMemcpyHostToDevice, stream) !=
            hipSuccess) {
            free3(c);
            return LELBM_EDEVICE;
        }
    }
    hipLaunchKernelGGL(k3_reset_flags, dim3(1), dim3(64), 0, stream, b.flags);
    if (hipStreamSynchronize(stream) != hipSuccess) { free3(c); return LELBM_EDEVICE; }
    *out = c;
    return LELBM_OK;
}

void ctx3_destroy(Ctx3 *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free3(c);
}

int ctx3_memory(const Ctx3 *c, long long *persistent, long long *scratch) {
    if (persistent) *persistent = c->persistent;
    if (scratch) *scratch = c->b.scratch_cap * (c->mixed ? 4 : 8);
    return LELBM_OK;
}

int ctx3_read(const Ctx3 *c, void *out, int to_device) {
    const size_t bytes = (size_t)NM * c->g.n * sizeof(double);
    H3(hipMemcpyAsync(out, c->b.mom[c->cur], bytes, to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                      c->stream));
    if (!to_device) H3(hipStreamSynchronize(c->stream));
    return LELBM_OK;
}

// Reads the flags, the step's reach and, with `layers`, the record elements
// of each layer of tiles (one synchronisation).
static int read_small(Ctx3 *c, Flags *f, int *reach, std::vector<long long> *layers) {
    char *h = (char *)c->host_small;
    H3(hipMemcpyAsync(h, c->b.flags, sizeof(Flags), hipMemcpyDeviceToHost, c->stream));
    H3(hipMemcpyAsync(h + 512, c->b.maxreach, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    if (layers)
        H3(hipMemcpyAsync(h + 4096, c->layer, (size_t)c->g.tnz * sizeof(long long), hipMemcpyDeviceToHost,
                          c->stream));
    H3(hipStreamSynchronize(c->stream));
    memcpy(f, h, sizeof(Flags));
    memcpy(reach, h + 512, sizeof(int));
    if (layers) {
        layers->resize((size_t)c->g.tnz);
        memcpy(layers->data(), h + 4096, (size_t)c->g.tnz * sizeof(long long));
    }
    return LELBM_OK;
}

void ctx3_set_budget(Ctx3 *c, long long bytes) { c->budget = bytes; }

// Bands of tile layers (the z axis, periodic) whose records fit the budget:
// the fewest bands, each band's slot as large as its largest band; one band
// when everything fits, bands of one layer as the last resort (then over the
// budget).  The schedule is build_plan's: a destination layer is gathered
// once every band within the step's reach M of it has been reconstructed,
// and a slot is reused once no pending layer needs its band.
static void plan3(Ctx3 *c, const std::vector<long long> &layers, int M, long long limit) {
    const G3 &g = c->g;
    const PlanGeom pg{g.tnz, g.tnz, TE, 0, g.nz, 1, g.tnz};
    Plan &P = c->plan;
    P.overlap = false;     // one stream: a freed slot is reused at once
    for (int rows = g.tnz; rows >= 1; rows--) {
        build_plan(pg, P, rows, M);
        long long mx = 0;
        for (const BandInfo &bd : P.bands) {
            long long sz = 0;
            for (int r = bd.row0; r < bd.row1; r++) sz += layers[(size_t)r];
            mx = std::max(mx, sz);
        }
        P.slot_cap = std::max<long long>(mx, 1);
        if ((long long)P.nslots * P.slot_cap <= limit || rows == 1) break;
    }
    set_bases(P);
}

// LDS of the staged gather at reach M with GY destination rows per
// workgroup; 0 if it does not fit.
static size_t gather3_lds(int M, int GY) {
    const size_t bytes = (size_t)(GX + 2 * M) * (GY + 2 * M) * G3_ENTRY_BYTES;
    return bytes <= 64 * 1024 ? bytes : 0;
}

int ctx3_step(Ctx3 *c, int nsteps, lelbm_stats *st, const Step3Timer &tm, Step3Failure *fail) {
    const G3 &g = c->g;
    Buf3 &b = c->b;
    hipStream_t s = c->stream;
    hipLaunchKernelGGL(k3_reset_flags, dim3(1), dim3(64), 0, s, b.flags);
    hipLaunchKernelGGL(k3_reset, dim3(1), dim3(64), 0, s, b, 1);
    H3(hipGetLastError());
    const size_t esz = c->mixed ? sizeof(float) : sizeof(double);
    for (int k = 0; k < nsteps; k++) {
        double *in = b.mom[c->cur], *outm = b.mom[c->cur ^ 1];
        tm.begin(tm.ctx, 1, s);
        hipLaunchKernelGGL(k3_reset, dim3(1), dim3(64), 0, s, b, 0);
        hipLaunchKernelGGL(k3_prepare, dim3((unsigned)g.ntiles), dim3(64), 0, s, g, c->ph, (const double *)in, b, k);
        tm.end(tm.ctx, 1, s);
        tm.begin(tm.ctx, 2, s);
        hipLaunchKernelGGL(k3_layer_sizes, dim3((unsigned)g.tnz), dim3(256), 0, s, g, b, c->layer);
        tm.end(tm.ctx, 2, s);
        H3(hipGetLastError());
        Flags f;
        int M = 0;
        std::vector<long long> &layers = c->hlayers;
        int r = read_small(c, &f, &M, &layers);
        if (r != LELBM_OK) return r;
        if (f.err) {
            fail->err = f.err; fail->step = k; fail->node = f.node; fail->detail = f.detail;
            fail->species = f.species; fail->residual = f.residual;
            return f.err;
        }
        plan3(c, layers, M, std::max<long long>(c->budget / (long long)esz, 1));
        const Plan &P = c->plan;
        // at least one record pair: the gather's misses read the first one
        const long long need = std::max<long long>((long long)P.nslots * P.slot_cap, 2);
        if (need > b.scratch_cap) {
            if (b.scratch) H3(hipFree(b.scratch));
            b.scratch = nullptr;
            b.scratch_cap = 0;
            if (hipMalloc(&b.scratch, (size_t)need * esz) != hipSuccess) {
                b.scratch = nullptr;
                fail->err = LELBM_ENOMEM; fail->step = k; fail->node = -1; fail->detail = 0; fail->species = -1;
                fail->residual = 0.0;
                return LELBM_ENOMEM;
            }
            b.scratch_cap = need;
        }
        const int per = g.tnx * g.tny;
        tm.begin(tm.ctx, 2, s);
        for (const BandInfo &bd : P.bands)
            hipLaunchKernelGGL(k3_scan, dim3(1), dim3(1024), 0, s, bd.row0 * per, (bd.row1 - bd.row0) * per, bd.base,
                               b);
        tm.end(tm.ctx, 2, s);
        // 16-row blocks where their staged plane fits the LDS, else 8 rows
        const int GY = gather3_lds(M, 16) ? 16 : 8;
        const size_t lds = gather3_lds(M, GY);
        const int bxy = ((g.nx + GX - 1) / GX) * ((g.ny + GY - 1) / GY);
        for (const Op &op : P.ops) {
            if (op.kind == OP_EPR) {
                const BandInfo &bd = P.bands[(size_t)op.a];
                const unsigned nt = (unsigned)((bd.row1 - bd.row0) * per);
                tm.begin(tm.ctx, 3, s);
                if (c->mixed)
                    hipLaunchKernelGGL(k3_epr<float>, dim3(nt), dim3(64), 0, s, g, c->ph, (const double *)in, b, k,
                                       bd.row0 * per);
                else
                    hipLaunchKernelGGL(k3_epr<double>, dim3(nt), dim3(64), 0, s, g, c->ph, (const double *)in, b, k,
                                       bd.row0 * per);
                tm.end(tm.ctx, 3, s);
                tm.begin(tm.ctx, 7, s);
                if (c->mixed)
                    hipLaunchKernelGGL(k3_epr_ref<float>, dim3(nt), dim3(64), 0, s, g, c->ph, (const double *)in, b,
                                       k, bd.row0 * per);
                else
                    hipLaunchKernelGGL(k3_epr_ref<double>, dim3(nt), dim3(64), 0, s, g, c->ph, (const double *)in, b,
                                       k, bd.row0 * per);
                tm.end(tm.ctx, 7, s);
            } else {
                // destination layers [a, a + n): cell planes [4a, min(nz, 4(a + n)))
                const int z0 = op.a * TE, z1 = std::min(g.nz, (op.a + op.n) * TE);
                tm.begin(tm.ctx, 4, s);
                const dim3 grid((unsigned)(bxy * (z1 - z0))), blk((unsigned)(GX * GY));
                if (lds && GY == 16 && c->mixed)
                    hipLaunchKernelGGL((k3_gather<float, 16>), grid, blk, lds, s, g, outm, b, M, z0);
                else if (lds && GY == 16)
                    hipLaunchKernelGGL((k3_gather<double, 16>), grid, blk, lds, s, g, outm, b, M, z0);
                else if (lds && c->mixed)
                    hipLaunchKernelGGL((k3_gather<float, 8>), grid, blk, lds, s, g, outm, b, M, z0);
                else if (lds)
                    hipLaunchKernelGGL((k3_gather<double, 8>), grid, blk, lds, s, g, outm, b, M, z0);
                else if (c->mixed)
                    hipLaunchKernelGGL(k3_gather_wide<float>, dim3((unsigned)(op.n * per)), dim3(64), 0, s, g, outm,
                                       b, op.a * per);
                else
                    hipLaunchKernelGGL(k3_gather_wide<double>, dim3((unsigned)(op.n * per)), dim3(64), 0, s, g, outm,
                                       b, op.a * per);
                tm.end(tm.ctx, 4, s);
            }
        }
        H3(hipGetLastError());
        // a failed reconstruction leaves the step's output unwritten
        r = read_small(c, &f, &M, nullptr);
        if (r != LELBM_OK) return r;
        if (f.err) {
            fail->err = f.err; fail->step = k; fail->node = f.node; fail->detail = f.detail;
            fail->species = f.species; fail->residual = f.residual;
            return f.err;
        }
        c->cur ^= 1;
    }
    if (st) {
        hipLaunchKernelGGL(k3_sums, dim3((unsigned)c->nsum), dim3(256), 0, s, g, (const double *)b.mom[c->cur],
                           b.partial);
        hipLaunchKernelGGL(k3_sums_final, dim3(1), dim3(64), 0, s, c->nsum, b.partial);
        H3(hipGetLastError());
        char *h = (char *)c->host_small;
        H3(hipMemcpyAsync(h, b.stats, sizeof(DevStats), hipMemcpyDeviceToHost, s));
        H3(hipMemcpyAsync(h + 1024, b.partial + (size_t)c->nsum * 4, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        H3(hipStreamSynchronize(s));
        DevStats ds;
        double sums[4];
        memcpy(&ds, h, sizeof(ds));
        memcpy(sums, h + 1024, sizeof(sums));
        memset(st, 0, sizeof(*st));
        const double cells = ds.cells ? (double)ds.cells : 1.0;
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
        st->row_passes = (long)ds.row_passes;
    }
    return LELBM_OK;
}

}  // namespace lelbm
