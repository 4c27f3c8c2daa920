// HIP kernels of the LELBM time step for gfx950 (MI355X).
//
// One step = pad fill -> stencil pre-pass -> tile scan -> per-cell collision
// and entropic reconstruction -> moment-streaming gather.
//
//  * k_fill_pads   fluid boundary cells, Sec. III.A (inflow: equilibrium of the
//                  prescribed state; outflow: zero-gradient copy, non-equilibrium kept)
//  * k_prepare     macroscopic variables (Eq. IIB6), acoustic radius and
//                  refinement level (Eqs. IIC6, IIC9), per-tile slot boxes of
//                  the population scratch and per-destination-tile gather windows
//  * k_scan        exclusive scan of tile sizes -> scratch offsets
//  * k_epr         collision (Eqs. IIB9-IIB18, App. D), stencil enumeration
//                  (Sec. II.C), Newton-Cholesky reconstruction (Eqs. IID7-IID13),
//                  writes the moment fractions of Eq. (IIE3a) into the scratch
//  * k_gather      moment streaming, Eq. (IIE3b), as a deterministic gather:
//                  every destination cell sums the fractions that land on it
//                  (the paper scatters with atomics); slip walls by mirror
//                  sources (specular path reflection, Sec. III.B)
//
// Layout: the state is SoA [moment][cell] over the padded source domain.  The
// population scratch is tile-major; inside a tile it is plane-major, then
// slot-major, then cell-in-tile, so the 64 lanes of a wavefront that read the
// same displacement from neighbouring sources read consecutive addresses.
#include <hip/hip_runtime.h>
#include <math.h>

#include <climits>

#include "lelbm_internal.h"
#include "lelbm_mlp_dev.h"

namespace lelbm {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <int D> struct Basis;
template <> struct Basis<2> { static constexpr int NF = 10, NG = 6, NMF = 28, NMG = 15, NMOM = 11; };
template <> struct Basis<1> { static constexpr int NF = 4, NG = 3, NMF = 7, NMG = 5, NMOM = 6; };

// 2D monomials x^a y^b (a + b <= 6) are numbered degree-major, then by b.
// The first 10 are the fluon basis 1,x,y,xx,xy,yy,xxx,xxy,xyy,yyy and the
// first 6 the phonon basis.  1D monomials are x^k.
__host__ __device__ constexpr int deg_of(int k) {
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= k) d++;
    return d;
}
__host__ __device__ constexpr int mono_b(int k) { return k - deg_of(k) * (deg_of(k) + 1) / 2; }
__host__ __device__ constexpr int mono_a(int k) { return deg_of(k) - mono_b(k); }
__host__ __device__ constexpr int mono_idx(int a, int b) { return (a + b) * (a + b + 1) / 2 + b; }

template <int D> __host__ __device__ constexpr int hess_idx(int i, int j) {
    return D == 1 ? i + j : mono_idx(mono_a(i) + mono_a(j), mono_b(i) + mono_b(j));
}
template <int D> __host__ __device__ constexpr int order_of(int j) { return D == 1 ? j : deg_of(j); }

// Decisions that define the stencil are evaluated without FMA contraction so
// that every kernel (and the CPU) takes them identically.
__device__ inline int las_radius(double RT, double n_conf, int r_min) {
#pragma clang fp contract(off)
    int R = (int)floor(n_conf * sqrt(RT) + 0.5);
    return R > r_min ? R : r_min;
}
// Stencils with rows longer than REC_SEG points (R >= 15): their
// reconstruction restarts the product recurrences (k_epr<..., true>).
__host__ __device__ constexpr bool wide_stencil(int R) { return 2 * R + 3 > REC_SEG; }
__device__ inline int las_levels(double RT) {
#pragma clang fp contract(off)
    return (int)floor(1.0 / (3.0 * sqrt(RT)) + 0.5);
}
__device__ inline bool in_disk2(double cx, double cy, double ux, double uy, double rr) {
#pragma clang fp contract(off)
    double a = cx - ux, b = cy - uy;
    return a * a + b * b <= rr * rr;
}
__device__ inline bool in_disk1(double cx, double ux, double rr) {
#pragma clang fp contract(off)
    double a = cx - ux;
    return a * a <= rr * rr;
}
__device__ inline double dist2(double cx, double cy, double ux, double uy) {
#pragma clang fp contract(off)
    double a = cx - ux, b = cy - uy;
    return sqrt(a * a + b * b);
}

__device__ inline void flag_fail(Flags *fl, int code, int step, long long node, int detail = 0, int species = -1,
                                 double residual = 0.0) {
    if (atomicCAS(&fl->err, 0, code) == 0) {
        fl->step = step;
        fl->detail = detail;
        fl->species = species;
        fl->residual = residual;
    }
    if (fl->err == code) atomicMin((unsigned long long *)&fl->node, (unsigned long long)node);
}

// Faces whose sources the gather may see mirrored: slip walls, and no-slip
// walls (sources that reflect their absorbed populations specularly).
__host__ __device__ inline bool mirror_face(const Geom &g, int f) {
    return g.bc[f] == LELBM_BC_SLIPWALL || g.bc[f] == LELBM_BC_WALL;
}

// Reasons of a failed reconstruction (lelbm_last_failure_detail).
enum { FAIL_NONFINITE = 1, FAIL_LINESEARCH = 2, FAIL_CHOL_POLISH = 3, FAIL_MAXIT = 4, FAIL_CHOL_STEP = 5 };
// species_update asks for a restart from Eq. (IID13) when a solve started
// from a non-equilibrium guess (linearised, previous step, learned) does not
// lower its residual at the first update, or fails
constexpr int RESTART_EQ = 2;

__device__ inline void atomic_max_pos(unsigned long long *a, double v) {
    atomicMax(a, (unsigned long long)__double_as_longlong(v));
}
__device__ inline void atomic_min_pos(unsigned long long *a, double v) {
    atomicMin(a, (unsigned long long)__double_as_longlong(v));
}

// equilibrium raw moments (Eqs. IIB7a-d; App. A)
template <int D>
__device__ inline void eq_moments(double K, double rho, double ux, double uy, double RT, double *m) {
    if (D == 1) {
        m[0] = rho;
        m[1] = rho * ux;
        m[2] = rho * (ux * ux + RT);
        m[3] = rho * (ux * ux + 3.0 * RT) * ux;
        m[4] = rho * K * RT;
        m[5] = rho * K * RT * ux;
    } else {
        double uu = ux * ux + uy * uy;
        m[0] = rho;
        m[1] = rho * ux;
        m[2] = rho * uy;
        m[3] = rho * (ux * ux + RT);
        m[4] = rho * (ux * uy);
        m[5] = rho * (uy * uy + RT);
        m[6] = rho * (uu + 4.0 * RT) * ux;
        m[7] = rho * (uu + 4.0 * RT) * uy;
        m[8] = rho * K * RT;
        m[9] = rho * K * RT * ux;
        m[10] = rho * K * RT * uy;
    }
}

// ---------------------------------------------------------------------------
// pad fill (Sec. III.A)
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_fill_pads(Geom g, Phys ph, T *mom, Flags *fl) {
    if (fl->err) return;
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.ns) return;
    int px = (int)(s % g.sxn), py = (int)(s / g.sxn);
    int x = px - g.wl, y = py - g.wb;
    bool pad = x < 0 || x >= g.nx || y < 0 || y >= g.ny;
    if (!pad) return;
    bool inflow = (x < 0 && g.bc[0] == LELBM_BC_INFLOW) || (x >= g.nx && g.bc[1] == LELBM_BC_INFLOW) ||
                  (y < 0 && g.bc[2] == LELBM_BC_INFLOW) || (y >= g.ny && g.bc[3] == LELBM_BC_INFLOW);
    constexpr int NM = Basis<D>::NMOM;
    if (inflow) {
        double m[11];
        eq_moments<D>(ph.K, ph.in_rho, ph.in_u[0], ph.in_u[1], ph.in_RT, m);
#pragma unroll
        for (int k = 0; k < NM; k++) mom[k * g.ns + s] = (T)m[k];
    } else {
        int ix = x < 0 ? 0 : (x >= g.nx ? g.nx - 1 : x);
        int iy = y < 0 ? 0 : (y >= g.ny ? g.ny - 1 : y);
        long long src = (long long)(iy + g.wb) * g.sxn + (ix + g.wl);
#pragma unroll
        for (int k = 0; k < NM; k++) mom[k * g.ns + s] = mom[k * g.ns + src];
    }
}

// ---------------------------------------------------------------------------
// pre-pass: macroscopic variables, stencil radius/levels, tile slot boxes,
// destination gather windows
// ---------------------------------------------------------------------------
__device__ inline void periodic_or_clip(int r0, int r1, int n, bool periodic, int *a, int *b, int *cnt) {
    // splits [r0, r1] into at most two intervals inside [0, n)
    if (periodic) {
        if (r1 - r0 + 1 >= n) { a[0] = 0; b[0] = n - 1; *cnt = 1; return; }
        int p = ((r0 % n) + n) % n, q = ((r1 % n) + n) % n;
        if (p <= q) { a[0] = p; b[0] = q; *cnt = 1; }
        else { a[0] = p; b[0] = n - 1; a[1] = 0; b[1] = q; *cnt = 2; }
    } else {
        int p = r0 < 0 ? 0 : r0, q = r1 > n - 1 ? n - 1 : r1;
        if (p > q) { *cnt = 0; return; }
        a[0] = p; b[0] = q; *cnt = 1;
    }
}

__device__ inline void update_windows(const Geom &g, DWin *dwin, int rx0, int rx1, int ry0, int ry1, int lox,
                                      int loy, int hix, int hiy, const int *ub) {
    int ax[2], bx[2], ay[2], by[2], cx, cy;
    periodic_or_clip(rx0, rx1, g.nx, g.bc[0] == LELBM_BC_PERIODIC, ax, bx, &cx);
    periodic_or_clip(ry0, ry1, g.ny, g.dim == 2 && g.bc[2] == LELBM_BC_PERIODIC, ay, by, &cy);
    for (int i = 0; i < cx; i++)
        for (int j = 0; j < cy; j++)
            for (int ty = ay[j] / g.ty; ty <= by[j] / g.ty; ty++)
                for (int tx = ax[i] / g.tx; tx <= bx[i] / g.tx; tx++) {
                    DWin *w = &dwin[ty * g.dtx + tx];
                    atomicMin(&w->lox, lox);
                    atomicMin(&w->loy, loy);
                    atomicMax(&w->hix, hix);
                    atomicMax(&w->hiy, hiy);
                    atomicMin(&w->uxl, ub[0]);
                    atomicMax(&w->uxh, ub[1]);
                    atomicMin(&w->uyl, ub[2]);
                    atomicMax(&w->uyh, ub[3]);
                    atomicMax(&w->rmax, ub[4]);
                }
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_prepare(Geom g, Phys ph, const T *mom, Buffers b, int step) {
    __shared__ int red[9][256];
    __shared__ int redf[256], redw[256];
    __shared__ int s_err;
    if (threadIdx.x == 0) s_err = b.flags->err;
    __syncthreads();
    if (s_err) return;
    int t = blockIdx.x;
    int tx0 = (t % g.ntx) * g.tx, ty0 = (t / g.ntx) * g.ty;
    int l = threadIdx.x;
    int px = tx0 + l % g.tx, py = ty0 + l / g.tx;
    bool valid = px < g.sxn && py < g.syn;
    int lox = 1 << 29, loy = 1 << 29, hix = -(1 << 29), hiy = -(1 << 29), refined = 0, wide = 0;
    int uxl = 1 << 29, uxh = -(1 << 29), uyl = 1 << 29, uyh = -(1 << 29), rmx = -1;
    int reach = 0;
    if (valid && b.solid) {
        const int ix = px - g.wl, iy = py - g.wb;
        if (ix >= 0 && ix < g.nx && iy >= 0 && iy < g.ny && b.solid[(long long)iy * g.nx + ix]) {
            b.desc_rn[(long long)py * g.sxn + px] = -1;     // solid cell: no population
            valid = false;
        }
    }
    if (valid) {
        long long s = (long long)py * g.sxn + px;
        double M0 = (double)mom[s], Mx = (double)mom[g.ns + s];
        double My = 0.0, Mxx, Myy = 0.0, G0;
        if (D == 1) {
            Mxx = (double)mom[2 * g.ns + s];
            G0 = (double)mom[4 * g.ns + s];
        } else {
            My = (double)mom[2 * g.ns + s];
            Mxx = (double)mom[3 * g.ns + s];
            Myy = (double)mom[5 * g.ns + s];
            G0 = (double)mom[8 * g.ns + s];
        }
        double rho = M0, ux, uy = 0.0, RT;
        {
#pragma clang fp contract(off)
            ux = Mx / rho;
            if (D == 2) uy = My / rho;
            double uu = ux * ux + uy * uy;
            RT = ((Mxx + Myy + G0) / rho - uu) / (D + ph.K);
        }
        bool ok = rho > 0.0 && isfinite(rho) && RT > 0.0 && isfinite(RT) && isfinite(ux) && isfinite(uy);
        int rn = -1;
        if (!ok) {
            flag_fail(b.flags, LELBM_EEPR, step, s);
        } else {
            int R = las_radius(RT, ph.n_conf, ph.r_min);
            int Nr = las_levels(RT);
            double umax = fmax(fabs(ux), fabs(uy));
            int ubx = 0, uby = 0;
            bool over = Nr > MAX_REFINE || R > MAX_RADIUS || !(umax <= MAX_SPEED);
            if (!over) {
                ubx = (int)floor(ux + 0.5);
                uby = D == 2 ? (int)floor(uy + 0.5) : 0;
                // Pads (Sec. III) must hold every source within reach of the
                // interior: the cells beyond a pad are in the pad's state, so a
                // pad cell whose stencil box [u] +- R reaches farther toward the
                // interior than the pad is wide means missing arrivals.
                const int ix = px - g.wl, iy = py - g.wb;
                over = (ix < 0 && ubx + R > g.wl) || (ix >= g.nx && R - ubx > g.wr) ||
                       (iy < 0 && uby + R > g.wb) || (iy >= g.ny && R - uby > g.wt);
            }
            if (over) {
                flag_fail(b.flags, LELBM_EREACH, step, s);
            } else {
                rn = R | (Nr << 16);
                lox = ubx - R - 1; hix = ubx + R + 1;
                loy = D == 2 ? uby - R - 1 : 0; hiy = D == 2 ? uby + R + 1 : 0;
                refined = Nr > 0;
                wide = Nr == 0 && wide_stencil(R);
                reach = max(abs(ubx), abs(uby)) + R + 1;
                uxl = (int)floor(ux * 1024.0); uxh = (int)ceil(ux * 1024.0);
                uyl = D == 2 ? (int)floor(uy * 1024.0) : 0; uyh = D == 2 ? (int)ceil(uy * 1024.0) : 0;
                rmx = R;
            }
        }
        b.desc_u[s] = ux;
        b.desc_u[g.ns + s] = uy;
        b.desc_rho[s] = rho;
        b.desc_rt[s] = RT;
        b.desc_rn[s] = rn;
    }
    red[0][l] = lox; red[1][l] = loy; red[2][l] = hix; red[3][l] = hiy; redf[l] = refined; redw[l] = wide;
    red[4][l] = uxl; red[5][l] = uxh; red[6][l] = uyl; red[7][l] = uyh; red[8][l] = rmx;
    __shared__ int s_reach[4];
    if (b.maxreach) {
        for (int off = 32; off > 0; off >>= 1) reach = max(reach, __shfl_xor(reach, off));
        if ((l & 63) == 0) s_reach[l >> 6] = reach;
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (l < off) {
            red[0][l] = min(red[0][l], red[0][l + off]);
            red[1][l] = min(red[1][l], red[1][l + off]);
            red[2][l] = max(red[2][l], red[2][l + off]);
            red[3][l] = max(red[3][l], red[3][l + off]);
            red[4][l] = min(red[4][l], red[4][l + off]);
            red[5][l] = max(red[5][l], red[5][l + off]);
            red[6][l] = min(red[6][l], red[6][l + off]);
            red[7][l] = max(red[7][l], red[7][l + off]);
            red[8][l] = max(red[8][l], red[8][l + off]);
            redf[l] |= redf[l + off];
            redw[l] |= redw[l + off];
        }
        __syncthreads();
    }
    if (l == 0 && b.maxreach) {
        // one atomic per workgroup, and only while it raises the maximum
        // (same-address atomics from every wavefront serialise)
        const int r = max(max(s_reach[0], s_reach[1]), max(s_reach[2], s_reach[3]));
        if (r > __hip_atomic_load(b.maxreach, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(b.maxreach, r);
    }
    if (l == 0) {
        TileInfo ti;
        ti.wide = redw[0];
        if (red[0][0] > red[2][0]) {   // no emitting cell in the tile
            ti.ox = ti.oy = 0; ti.wx = ti.wy = 0; ti.fmt = 0; ti.size = 0; ti.base = 0;
        } else {
            ti.ox = red[0][0]; ti.oy = red[1][0];
            ti.wx = red[2][0] - red[0][0] + 1; ti.wy = red[3][0] - red[1][0] + 1;
            ti.fmt = redf[0];
            ti.size = (long long)ti.wx * ti.wy * TILE_N * (ti.fmt ? Basis<D>::NMOM : 2);
            ti.base = 0;
            // gather windows of the destination tiles this tile can reach
            int x0 = tx0 - g.wl, x1 = min(tx0 + g.tx, g.sxn) - 1 - g.wl;
            int y0 = ty0 - g.wb, y1 = min(ty0 + g.ty, g.syn) - 1 - g.wb;
            int lx = ti.ox, ly = ti.oy, hx = red[2][0], hy = red[3][0];
            // mirror images across slip walls (and no-slip walls, whose
            // absorbed populations may be reflected specularly): m = 0 none,
            // 1 low face, 2 high face
            bool slipx = mirror_face(g, 0) || mirror_face(g, 1);
            bool slipy = D == 2 && (mirror_face(g, 2) || mirror_face(g, 3));
            for (int mx = 0; mx < (slipx ? 3 : 1); mx++) {
                if (mx == 1 && !mirror_face(g, 0)) continue;
                if (mx == 2 && !mirror_face(g, 1)) continue;
                for (int my = 0; my < (slipy ? 3 : 1); my++) {
                    if (my == 1 && !mirror_face(g, 2)) continue;
                    if (my == 2 && !mirror_face(g, 3)) continue;
                    int gx0 = x0, gx1 = x1, glx = lx, ghx = hx;
                    if (mx == 1) { gx0 = -1 - x1; gx1 = -1 - x0; glx = -hx; ghx = -lx; }
                    if (mx == 2) { gx0 = 2 * g.nx - 1 - x1; gx1 = 2 * g.nx - 1 - x0; glx = -hx; ghx = -lx; }
                    int gy0 = y0, gy1 = y1, gly = ly, ghy = hy;
                    if (my == 1) { gy0 = -1 - y1; gy1 = -1 - y0; gly = -hy; ghy = -ly; }
                    if (my == 2) { gy0 = 2 * g.ny - 1 - y1; gy1 = 2 * g.ny - 1 - y0; gly = -hy; ghy = -ly; }
                    // velocity bounds serve the straight gather only (mirror images
                    // reverse velocities; tiles of domains with slip walls ignore them)
                    const int ub[5] = {red[4][0], red[5][0], red[6][0], red[7][0], red[8][0]};
                    update_windows(g, b.dwin, gx0 + glx, gx1 + ghx, gy0 + gly, gy1 + ghy, glx, gly, ghx, ghy, ub);
                }
            }
        }
        b.tiles[t] = ti;
    }
}

// ---------------------------------------------------------------------------
// record offsets and k_epr's tile order, band by band (one workgroup)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_scan(int ntx, int nbands, const BandInfo *bands, TileInfo *tiles,
                                               Flags *fl, long long slot_cap, int step, int *order, int *rlist,
                                               int *rcount, const int *maxreach, int m_plan) {
    // 16 wavefronts: scans within a wavefront by shuffles and ballots, across
    // the wavefronts of a 1024-tile chunk through LDS
    __shared__ long long s_wave[16];
    __shared__ int s_cnt[16][3];
    __shared__ long long s_carry, s_need, s_total;
    __shared__ int s_class[3], s_run[3], s_nref;
    if (fl->err) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_need = s_total = 0;
    for (int bd = 0; bd < nbands; bd++) {
        // the band's tiles: whole source tile rows [row0, row1), records from
        // its scratch slot's first element
        const BandInfo band = bands[bd];
        const int t0 = band.row0 * ntx, nt = (band.row1 - band.row0) * ntx;
        if (threadIdx.x == 0) s_carry = 0;
        if (threadIdx.x < 3) s_class[threadIdx.x] = s_run[threadIdx.x] = 0;
        __syncthreads();
        // record offsets: exclusive scan of the tile sizes
        for (int c0 = 0; c0 < nt; c0 += 1024) {
            const int i = c0 + threadIdx.x;
            const long long v = i < nt ? tiles[t0 + i].size : 0;
            long long incl = v;
            for (int off = 1; off < 64; off <<= 1) {
                const long long o = __shfl_up(incl, off);
                if (lane >= off) incl += o;
            }
            if (lane == 63) s_wave[w] = incl;
            __syncthreads();
            long long wbase = 0, ctot = 0;
            for (int k = 0; k < 16; k++) {
                const long long sk = s_wave[k];
                wbase += k < w ? sk : 0;
                ctot += sk;
            }
            if (i < nt) tiles[t0 + i].base = band.base + s_carry + wbase + incl - v;
            __syncthreads();
            if (threadIdx.x == 0) s_carry += ctot;
            __syncthreads();
        }
        const long long total = s_carry;
        if (threadIdx.x == 0) {
            s_need = total > s_need ? total : s_need;
            s_total += total;
            s_nref = 0;
        }
        // the band's tiles with refined cells, in index order, for k_epr_ref
        for (int c0 = 0; c0 < nt; c0 += 1024) {
            const int i = c0 + threadIdx.x;
            const bool f = i < nt && tiles[t0 + i].fmt != 0;
            const unsigned long long m = __ballot(f);
            const int rank = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) s_cnt[w][0] = __popcll(m);
            __syncthreads();
            int woff = 0, ctot = 0;
            for (int k = 0; k < 16; k++) {
                woff += k < w ? s_cnt[k][0] : 0;
                ctot += s_cnt[k][0];
            }
            if (f) rlist[t0 + s_nref + woff + rank] = t0 + i;
            __syncthreads();
            if (threadIdx.x == 0) s_nref += ctot;
            __syncthreads();
        }
        if (threadIdx.x == 0) rcount[bd] = s_nref;
        // Order in which k_epr takes the band's tiles: the heaviest first (a
        // tile's records measure its stencil work), so that the long ones do
        // not start last and leave the CUs idle at the end.  Stable partition
        // into tiles with at least twice the mean size, at least the mean, and
        // the rest: the class sizes first, then each tile's place.  Worth it
        // only while a launch spans few rounds of resident workgroups: with
        // many tiles the tail is short and the index order writes the records
        // more locally (measured: 16K tiles -9 % k_epr time, 33K about even,
        // 131K +4 %).
        if (nt > EPR_ORDER_MAX_TILES) {
            for (int i = threadIdx.x; i < nt; i += 1024) order[t0 + i] = t0 + i;
            __syncthreads();
            continue;
        }
        const auto class_of = [&](int i) {
            const long long v = tiles[t0 + i].size * (long long)nt;
            return v >= 2 * total ? 0 : (v >= total ? 1 : 2);
        };
        for (int c0 = 0; c0 < nt; c0 += 1024) {
            const int i = c0 + threadIdx.x;
            const int c = i < nt ? class_of(i) : -1;
            for (int k = 0; k < 3; k++) {
                const unsigned long long m = __ballot(c == k);
                if (lane == 0 && m) atomicAdd(&s_class[k], __popcll(m));
            }
        }
        __syncthreads();
        const int cbase[3] = {0, s_class[0], s_class[0] + s_class[1]};
        for (int c0 = 0; c0 < nt; c0 += 1024) {
            const int i = c0 + threadIdx.x;
            const int c = i < nt ? class_of(i) : -1;
            int rank = 0;
            for (int k = 0; k < 3; k++) {
                const unsigned long long m = __ballot(c == k);
                if (c == k) rank = __popcll(m & ((1ull << lane) - 1ull));
                if (lane == 0) s_cnt[w][k] = __popcll(m);
            }
            __syncthreads();
            if (c >= 0) {
                int woff = 0;
                for (int k = 0; k < w; k++) woff += s_cnt[k][c];
                order[t0 + cbase[c] + s_run[c] + woff + rank] = t0 + i;
            }
            __syncthreads();
            if (threadIdx.x < 3) {
                int t = 0;
                for (int k = 0; k < 16; k++) t += s_cnt[k][threadIdx.x];
                s_run[threadIdx.x] += t;
            }
            __syncthreads();
        }
    }
    // a band's records exceed its slot, or a stencil reaches farther than the
    // band plan allows for: the host re-plans and repeats the step
    if (threadIdx.x == 0) {
        const int M = *maxreach;
        if (s_need > slot_cap) {
            if (atomicCAS(&fl->err, 0, ERR_OVERFLOW) == 0) {
                fl->need = s_need;
                fl->total = s_total;
                fl->reach = M;
                fl->step = step;
            }
        } else if (M > m_plan) {
            if (atomicCAS(&fl->err, 0, ERR_REPLAN) == 0) {
                fl->need = M;
                fl->reach = M;
                fl->step = step;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// stencil enumeration (Sec. II.C): base points row by row; refined children
// replace their parent, level by level (Eqs. IIC10-11).  leaf(cx, cy, dC, dx,
// dy) gets the exact velocity, velocity volume and landing displacement;
// parent_end(dx, dy) is called after the last leaf of each base point.
// ---------------------------------------------------------------------------
template <int D, typename Leaf, typename End>
__device__ inline void for_each_point(double ux, double uy, int R, int Nr, Leaf &&leaf, End &&parent_end) {
    const double rr = R + 0.5;
    int ubx = (int)floor(ux + 0.5), uby = D == 2 ? (int)floor(uy + 0.5) : 0;
    int ylo = D == 2 ? uby - R - 1 : 0, yhi = D == 2 ? uby + R + 1 : 0;
    for (int cy = ylo; cy <= yhi; cy++) {
        for (int cx = ubx - R - 1; cx <= ubx + R + 1; cx++) {
            double fx = (double)cx, fy = (double)cy;
            bool in = D == 2 ? in_disk2(fx, fy, ux, uy, rr) : in_disk1(fx, ux, rr);
            if (!in) continue;
            double d0 = D == 2 ? dist2(fx, fy, ux, uy) : fabs(fx - ux);
            if (Nr == 0 || d0 > 1.5) {
                leaf(fx, fy, 1.0, cx, cy);
            } else {
                constexpr int NC = D == 2 ? 4 : 2;
                const double v1 = D == 2 ? 0.25 : 0.5;
                for (int k1 = 0; k1 < NC; k1++) {
                    double c1x = fx + ((k1 & 1) ? 0.25 : -0.25);
                    double c1y = D == 2 ? fy + ((k1 & 2) ? 0.25 : -0.25) : 0.0;
                    double d1 = D == 2 ? dist2(c1x, c1y, ux, uy) : fabs(c1x - ux);
                    if (Nr < 2 || d1 > 0.75) {
                        leaf(c1x, c1y, v1, cx, cy);
                        continue;
                    }
                    for (int k2 = 0; k2 < NC; k2++) {
                        double c2x = c1x + ((k2 & 1) ? 0.125 : -0.125);
                        double c2y = D == 2 ? c1y + ((k2 & 2) ? 0.125 : -0.125) : 0.0;
                        double d2 = D == 2 ? dist2(c2x, c2y, ux, uy) : fabs(c2x - ux);
                        if (Nr < 3 || d2 > 0.375) {
                            leaf(c2x, c2y, v1 * v1, cx, cy);
                            continue;
                        }
                        for (int k3 = 0; k3 < NC; k3++) {
                            double c3x = c2x + ((k3 & 1) ? 0.0625 : -0.0625);
                            double c3y = D == 2 ? c2y + ((k3 & 2) ? 0.0625 : -0.0625) : 0.0;
                            leaf(c3x, c3y, v1 * v1 * v1, cx, cy);
                        }
                    }
                }
            }
            parent_end(cx, cy);
        }
    }
}

// ---------------------------------------------------------------------------
// dense Cholesky solve of an SPD system assembled from monomial sums
// ---------------------------------------------------------------------------
template <int D, int N>
__device__ inline bool hess_solve(const double *S, const double *r, double *x) {
    // A_ij = S[T_i T_j] (Eq. IID11a), lower triangle, factored in place
    double L[N * (N + 1) / 2], inv[N];
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) L[i * (i + 1) / 2 + j] = S[hess_idx<D>(i, j)];
#pragma unroll
    for (int i = 0; i < N; i++) {
#pragma unroll
        for (int j = 0; j <= i; j++) {
            double s = L[i * (i + 1) / 2 + j];
#pragma unroll
            for (int k = 0; k < j; k++) s -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return false;
                double d = sqrt(s);
                L[i * (i + 1) / 2 + i] = d;
                inv[i] = 1.0 / d;
            } else {
                L[i * (i + 1) / 2 + j] = s * inv[j];
            }
        }
    }
    double y[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        double s = r[i];
#pragma unroll
        for (int k = 0; k < i; k++) s -= L[i * (i + 1) / 2 + k] * y[k];
        y[i] = s * inv[i];
    }
#pragma unroll
    for (int i = N - 1; i >= 0; i--) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < N; k++) s -= L[k * (k + 1) / 2 + i] * x[k];
        x[i] = s * inv[i];
    }
    return true;
}

// Newton state of one species (fluon or phonon), Sec. II.D.  The step is
// a damped Newton method on the convex dual Phi(l) = sum f + l.m' (Armijo
// backtracking while the Newton decrement exceeds 1e-8).  The multipliers and
// the current direction live either in registers or in LDS (one column per
// cell of the tile), which keeps the register file of the hot kernel small
// enough for two waves per SIMD.
template <int NB> struct RegStore {
    double lam_[NB], del_[NB];
    __device__ double &lam(int j) { return lam_[j]; }
    __device__ double &del(int j) { return del_[j]; }
};
template <int NB> struct LdsStore {
    double *lam_, *del_;   // column of the cell in [NB][TILE_N] arrays
    __device__ double &lam(int j) { return lam_[j * TILE_N]; }
    __device__ double &del(int j) { return del_[j * TILE_N]; }
};

template <int NB, class Store> struct Species {
    Store v;
    double t, dec, phi;
    int phase;        // 0: first evaluation, 1: iterating, 2: polished
    int nit, ls;
    double res;       // last scaled residual
    int mlp;          // 1 while iterating from the learned guess
    double res_prev;  // residual after the previous accepted step
    __device__ double at(int j) { return v.lam(j) + t * v.del(j); }   // multipliers of the current pass
};

// After a pass evaluated at lam + t*del: accept / backtrack / step / polish.
// Returns 0 to continue, 1 when polished, negative LELBM code on failure.
template <int D, int NB, int NM, class Store>
__device__ inline int species_update(Species<NB, Store> &sp, const double *S, const double *tg, const double *isc,
                                     double tol, int maxit) {
    double r[NB];
    double phit = S[0];
    bool fin = isfinite(S[0]);
#pragma unroll
    for (int j = 0; j < NB; j++) {
        r[j] = S[j] - tg[j];
        phit += sp.at(j) * tg[j];
        fin = fin && isfinite(r[j]);
    }
    fin = fin && isfinite(phit);
    if (sp.phase == 0) {
        if (!fin) return sp.mlp ? RESTART_EQ : -FAIL_NONFINITE;
        sp.phase = 1;
    } else {
        if (!(fin && (sp.dec <= 1e-8 || phit <= sp.phi - 1e-4 * sp.t * sp.dec))) {
            sp.t *= 0.5;
            if (++sp.ls > 30) return -FAIL_LINESEARCH;
            return 0;
        }
        sp.nit++;
    }
#pragma unroll
    for (int j = 0; j < NB; j++) sp.v.lam(j) = sp.at(j);
    sp.t = 0.0;
    sp.phi = phit;
    double res = 0.0;
#pragma unroll
    for (int j = 0; j < NB; j++) {
        double v = fabs(r[j]) * isc[order_of<D>(j)];
        res = v > res ? v : res;
    }
    sp.res = res;
    // a residual below STALL_RES that did not decrease at the last update has
    // reached the rounding floor of the sums: converged
    const bool stalled = sp.nit > 0 && res <= STALL_RES && !(res < sp.res_prev);
    if (sp.mlp && sp.nit > 0 && res > tol && !stalled && !(res < sp.res_prev)) return RESTART_EQ;
    sp.res_prev = res;
    double dl[NB];
    if (res <= tol || stalled) {
        if (!hess_solve<D, NB>(S, r, dl)) return -FAIL_CHOL_POLISH;
#pragma unroll
        for (int j = 0; j < NB; j++) { sp.v.lam(j) += dl[j]; sp.v.del(j) = 0.0; }
        sp.nit++;
        sp.phase = 2;
        return 1;
    }
    if (sp.nit >= maxit) return -FAIL_MAXIT;
    if (!hess_solve<D, NB>(S, r, dl)) return -FAIL_CHOL_STEP;
    double dec = 0.0;
#pragma unroll
    for (int j = 0; j < NB; j++) { sp.v.del(j) = dl[j]; dec += r[j] * dl[j]; }
    sp.dec = dec;
    sp.t = 1.0;
    sp.ls = 0;
    return 0;
}

// monomials of (x, y) up to total degree NMT (numbering of mono_idx)
template <int D, int NMT>
__device__ inline void monomials(double x, double y, double *m) {
    if (D == 1) {
        m[0] = 1.0;
#pragma unroll
        for (int k = 1; k < NMT; k++) m[k] = m[k - 1] * x;
    } else {
        double px[7], py[7];
        px[0] = 1.0; py[0] = 1.0;
#pragma unroll
        for (int k = 1; k < 7; k++) { px[k] = px[k - 1] * x; py[k] = py[k - 1] * y; }
#pragma unroll
        for (int k = 0; k < NMT; k++) m[k] = px[mono_a(k)] * py[mono_b(k)];
    }
}

// ---------------------------------------------------------------------------
// per-cell collision: normalised post-collision central-moment targets of the
// fluon (mf) and phonon (mg) reconstructions, Eqs. (IIB9-IIB18), with the
// Knudsen limiter of App. D, Eqs. (D2-D3)
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ inline void collide_targets(const Geom &g, const Phys &ph, const T *mom, long long s, double rho,
                                       double ux, double uy, double RT, double *mf, double *mg, double &kn_out,
                                       int &lim_out) {
    const double K = ph.K;
    double P[2][2] = {{0, 0}, {0, 0}}, Q[2] = {0, 0}, h[2] = {0, 0}, g0;
    double u[2] = {ux, uy};
    if (D == 1) {
        double Mxx = (double)mom[2 * g.ns + s], MD = (double)mom[3 * g.ns + s];
        double G0 = (double)mom[4 * g.ns + s], Gx = (double)mom[5 * g.ns + s];
        P[0][0] = Mxx - rho * (ux * ux + RT);
        Q[0] = MD - 2.0 * (ux * P[0][0]) - ux * P[0][0] - rho * (ux * ux + 3.0 * RT) * ux;
        g0 = G0 - rho * K * RT;
        h[0] = Gx - ux * G0;
    } else {
        double Mxx = (double)mom[3 * g.ns + s], Mxy = (double)mom[4 * g.ns + s];
        double Myy = (double)mom[5 * g.ns + s];
        double MD[2] = {(double)mom[6 * g.ns + s], (double)mom[7 * g.ns + s]};
        double G0 = (double)mom[8 * g.ns + s];
        double Gv[2] = {(double)mom[9 * g.ns + s], (double)mom[10 * g.ns + s]};
        double uu = ux * ux + uy * uy;
        P[0][0] = Mxx - rho * (ux * ux + RT);
        P[0][1] = P[1][0] = Mxy - rho * (ux * uy);
        P[1][1] = Myy - rho * (uy * uy + RT);
        double trP = P[0][0] + P[1][1];
#pragma unroll
        for (int gg = 0; gg < 2; gg++) {
            double sm = u[0] * P[0][gg] + u[1] * P[1][gg];
            Q[gg] = MD[gg] - 2.0 * sm - u[gg] * trP - rho * (uu + 4.0 * RT) * u[gg];
        }
        g0 = G0 - rho * K * RT;
#pragma unroll
        for (int gg = 0; gg < 2; gg++) h[gg] = Gv[gg] - u[gg] * G0;
    }
    double sP = 0.0, sQ = 0.0;
#pragma unroll
    for (int a = 0; a < D; a++) {
#pragma unroll
        for (int bb = 0; bb < D; bb++) sP += fabs(P[a][bb]);
        sQ += fabs(Q[a]) + fabs(h[a]);
    }
    double knA = (sP + fabs(g0)) / (rho * (D + K) * RT);
    double knB = sQ / (rho * (D + K + 2.0) * pow(RT, 1.5));
    double kn = knA > knB ? knA : knB;
    double of = ph.omega_f, ob = ph.omega_b, oh = ph.omega_h;
    int lim = 0;
    if (ph.kn_limiter && kn >= ph.kn_lo_lin) {
        if (kn > ph.kn_hi_lin) {
            of = ob = oh = ph.omega_H;
        } else {
            double k = log10(kn), span = ph.kn_hi - ph.kn_lo;
            of = (ph.omega_H - ph.omega_f) / span * (k - ph.kn_lo) + ph.omega_f;
            ob = (ph.omega_H - ph.omega_b) / span * (k - ph.kn_lo) + ph.omega_b;
            oh = (ph.omega_H - ph.omega_h) / span * (k - ph.kn_lo) + ph.omega_h;
        }
        lim = (of != ph.omega_f) || (ob != ph.omega_b) || (oh != ph.omega_h);
    }
    kn_out = kn;
    lim_out = lim;
    double bulk = -g0 / D;
    // normalised by the zeroth post-collision moment (Eq. IIB18): rho, plus
    // the mass a point source adds in its cell, whose Maxwellian (Eqs.
    // VC6-VC7) leaves the equilibrium parts RT delta unchanged
    const double rp = post_mass(ph, s, rho);
    double rKT = rp * K * RT;
    if (D == 1) {
        double shear = P[0][0] - bulk;
        mf[0] = 1.0; mf[1] = 0.0;
        mf[2] = RT + ((1.0 - of) * shear + (1.0 - ob) * bulk) / rp;
        mf[3] = (1.0 - oh) * Q[0] / rp;
        mg[0] = 1.0 + (1.0 - ob) * g0 / rKT;
        mg[1] = (1.0 - oh) * h[0] / rKT;
        mg[2] = RT;
    } else {
        double shxx = P[0][0] - bulk, shxy = P[0][1], shyy = P[1][1] - bulk;
        mf[0] = 1.0; mf[1] = 0.0; mf[2] = 0.0;
        mf[3] = RT + ((1.0 - of) * shxx + (1.0 - ob) * bulk) / rp;
        mf[4] = ((1.0 - of) * shxy) / rp;
        mf[5] = RT + ((1.0 - of) * shyy + (1.0 - ob) * bulk) / rp;
        mf[6] = (1.0 - oh) * (0.75 * Q[0]) / rp;
        mf[7] = (1.0 - oh) * (0.25 * Q[1]) / rp;
        mf[8] = (1.0 - oh) * (0.25 * Q[0]) / rp;
        mf[9] = (1.0 - oh) * (0.75 * Q[1]) / rp;
        mg[0] = 1.0 + (1.0 - ob) * g0 / rKT;
        mg[1] = (1.0 - oh) * h[0] / rKT;
        mg[2] = (1.0 - oh) * h[1] / rKT;
        mg[3] = RT; mg[4] = 0.0; mg[5] = RT;
    }
}

// Restarts one species from Eq. (IID13).
template <int D, int NB, class S>
__device__ inline void species_restart_eq(Species<NB, S> &sp, double RT) {
#pragma unroll
    for (int j = 0; j < NB; j++) { sp.v.lam(j) = 0.0; sp.v.del(j) = 0.0; }
    sp.v.lam(0) = -1.0 + 0.5 * D * log(2.0 * M_PI * RT);
    if (D == 1) sp.v.lam(2) = 1.0 / (2.0 * RT);
    else { sp.v.lam(3) = 1.0 / (2.0 * RT); sp.v.lam(5) = 1.0 / (2.0 * RT); }
    sp.t = 0.0; sp.dec = 0.0; sp.phi = 0.0;
    sp.phase = 0; sp.nit = 0; sp.ls = 0;
    sp.res = 0.0; sp.mlp = 0; sp.res_prev = 0.0;
}

// Initial multipliers of Eq. (IID13) for both species.
template <int D, int NF, int NG, class SF, class SG>
__device__ inline void species_init(Species<NF, SF> &sf, Species<NG, SG> &sg, double RT) {
#pragma unroll
    for (int j = 0; j < NF; j++) { sf.v.lam(j) = 0.0; sf.v.del(j) = 0.0; }
#pragma unroll
    for (int j = 0; j < NG; j++) { sg.v.lam(j) = 0.0; sg.v.del(j) = 0.0; }
    double l0 = -1.0 + 0.5 * D * log(2.0 * M_PI * RT), l2 = 1.0 / (2.0 * RT);
    sf.v.lam(0) = l0; sg.v.lam(0) = l0;
    if (D == 1) { sf.v.lam(2) = l2; sg.v.lam(2) = l2; }
    else { sf.v.lam(3) = l2; sf.v.lam(5) = l2; sg.v.lam(3) = l2; sg.v.lam(5) = l2; }
    sf.t = sg.t = 0.0; sf.dec = sg.dec = 0.0; sf.phi = sg.phi = 0.0;
    sf.phase = sg.phase = 0; sf.nit = sg.nit = 0; sf.ls = sg.ls = 0;
    sf.res = sg.res = 0.0;
    sf.mlp = sg.mlp = 0; sf.res_prev = sg.res_prev = 0.0;
}

// Linearised initial multipliers.  At the equilibrium multipliers of
// Eq. (IID13) the populations are the Maxwellian of variance RT, so one
// Newton step A dlambda = (equilibrium moments - targets) can be taken with
// the Hessian A_ij = <T_i T_j> of the continuous Maxwellian instead of the
// stencil sums.  In units scaled by RT^(k/2) (k = polynomial order) A is a
// constant matrix that splits by parity into blocks {1, x^2, y^2}, {xy},
// {x, x^3, x y^2}, {y, x^2 y, y^3} (fluon), {1, x^2, y^2}, {xy}, {x}, {y}
// (phonon); their inverses are written out below.  d receives the scaled
// corrections (fluon 0..NF-1, phonon NF..), to be added to Eq. (IID13)'s
// scaled values.  Targets: mf, mg as from collide_targets.
template <int D>
__device__ inline void lin_guess_scaled(const double *mf, const double *mg, double RT, double *d) {
    const double is = 1.0 / sqrt(RT), i2 = 1.0 / RT, i3 = i2 * is;
    if (D == 2) {
        // scaled target deviations from equilibrium (targets minus Maxwellian moments)
        const double a = mf[3] * i2 - 1.0, bxy = mf[4] * i2, c = mf[5] * i2 - 1.0;
        const double x3 = mf[6] * i3, x2y = mf[7] * i3, xy2 = mf[8] * i3, y3 = mf[9] * i3;
        const double n0 = mg[0] - 1.0, nx = mg[1] * is, ny = mg[2] * is;
        // inverse of [[1,1,1],[1,3,1],[1,1,3]] = [[2,-1/2,-1/2],[-1/2,1/2,0],[-1/2,0,1/2]]
        d[0] = 0.5 * (a + c);
        d[3] = -0.5 * a;
        d[5] = -0.5 * c;
        d[4] = -bxy;
        // inverse of [[1,3,1],[3,15,3],[1,3,3]] (x, x^3, x y^2) = [[3,-1/2,-1/2],[-1/2,1/6,0],[-1/2,0,1/2]]
        d[1] = 0.5 * (x3 + xy2);
        d[6] = -x3 / 6.0;
        d[8] = -0.5 * xy2;
        // the same block for (y, y^3, x^2 y)
        d[2] = 0.5 * (y3 + x2y);
        d[9] = -y3 / 6.0;
        d[7] = -0.5 * x2y;
        // phonons: only n0 and n_gamma deviate
        d[10 + 0] = -2.0 * n0;
        d[10 + 3] = 0.5 * n0;
        d[10 + 5] = 0.5 * n0;
        d[10 + 4] = 0.0;
        d[10 + 1] = -nx;
        d[10 + 2] = -ny;
    } else {
        const double a = mf[2] * i2 - 1.0, x3 = mf[3] * i3;
        const double n0 = mg[0] - 1.0, nx = mg[1] * is;
        // inverse of [[1,1],[1,3]] = [[3/2,-1/2],[-1/2,1/2]], of [[1,3],[3,15]] = [[5/2,-1/2],[-1/2,1/6]]
        d[0] = 0.5 * a;
        d[2] = -0.5 * a;
        d[1] = 0.5 * x3;
        d[3] = -x3 / 6.0;
        d[4 + 0] = -1.5 * n0;
        d[4 + 2] = 0.5 * n0;
        d[4 + 1] = -nx;
    }
}

// Adds the linearised correction to multipliers holding Eq. (IID13).
template <int D, int NF, int NG, class SF, class SG>
__device__ inline void species_linear(Species<NF, SF> &sf, Species<NG, SG> &sg, const double *mf, const double *mg,
                                      double RT) {
    double d[NF + NG];
    lin_guess_scaled<D>(mf, mg, RT, d);
    const double sq = sqrt(RT);
#pragma unroll
    for (int j = 0; j < NF + NG; j++) {
        const int jj = j < NF ? j : j - NF;
        const int k = order_of<D>(jj);
        const double scl = k == 0 ? 1.0 : (k == 1 ? sq : (k == 2 ? RT : RT * sq));
        if (j < NF) sf.v.lam(jj) += d[j] / scl;
        else sg.v.lam(jj) += d[j] / scl;
    }
    sf.mlp = sg.mlp = 1;
}

// Multiplier j of Eq. (IID13), unscaled: the Maxwellian of variance RT.
template <int D>
__device__ inline double iid13_value(int j, double RT) {
    if (j == 0) return -1.0 + 0.5 * D * log(2.0 * M_PI * RT);
    if (D == 2 ? (j == 3 || j == 5) : j == 2) return 0.5 / RT;
    return 0.0;
}

// Warm start from the previous step (Sec. II.D suggests reusing stored
// multipliers).  The stored quantity is the cell's correction beyond the
// linearised guess in scaled units, e_j = lambda_j RT^(k/2) - (IID13 + LIN)_j
// (k = basis order), which carries over smoothly across steps; the
// linearised part follows this step's targets, including the sign flip of
// their non-equilibrium part at omega = 2.  prev = NaN in row 0: none.
template <int D, int NF, int NG, class SF, class SG>
__device__ inline void species_prev(Species<NF, SF> &sf, Species<NG, SG> &sg, const double *mf, const double *mg,
                                    double RT, const double *prev, long long ns, long long s) {
    species_linear<D>(sf, sg, mf, mg, RT);
    if (!(prev[s] == prev[s])) return;
    const double sq = sqrt(RT);
#pragma unroll
    for (int j = 0; j < NF + NG; j++) {
        const int jj = j < NF ? j : j - NF;
        const int k = order_of<D>(jj);
        const double scl = k == 0 ? 1.0 : (k == 1 ? sq : (k == 2 ? RT : RT * sq));
        const double e = prev[(long long)j * ns + s];
        if (j < NF) sf.v.lam(jj) += e / scl;
        else sg.v.lam(jj) += e / scl;
    }
}

// Stores the converged multipliers' correction beyond IID13 + LIN (see
// species_prev) for the next step's guess.
template <int D, int NF, int NG, class SF, class SG>
__device__ inline void store_prev(Species<NF, SF> &sf, Species<NG, SG> &sg, const double *mf, const double *mg,
                                  double RT, double *prev, long long ns, long long s) {
    double d[NF + NG];
    lin_guess_scaled<D>(mf, mg, RT, d);
    const double sq = sqrt(RT);
#pragma unroll
    for (int j = 0; j < NF + NG; j++) {
        const int jj = j < NF ? j : j - NF;
        const int k = order_of<D>(jj);
        const double scl = k == 0 ? 1.0 : (k == 1 ? sq : (k == 2 ? RT : RT * sq));
        const double lam = j < NF ? sf.v.lam(jj) : sg.v.lam(jj);
        prev[(long long)j * ns + s] = (lam - iid13_value<D>(jj, RT)) * scl - d[j];
    }
}

// Per-cell statistics.
struct CellStats {
    int it_f = 0, it_g = 0, q = 0, lim = 0, pass = 0, fb = 0;
    int rows = 0;             // stencil rows holding points (unrefined stencils)
    double kn = 0.0, colat = 0.0, rt = 1e300;
    bool active = false;
    bool refined = false;    // handled by the refined-stencil kernel
};

// Sums, maxima and minima of CellStats over a set of cells (the fields of
// DevStats; an empty set is the neutral element).
struct StatSum {
    unsigned long long itf = 0, itg = 0, q = 0, lim = 0, cells = 0, qp = 0, qpr = 0, fb = 0;
    unsigned long long wq = 0;   // sum over wavefronts of 64 x the wavefront's largest q x passes
    unsigned long long rp = 0;   // rows x passes
    int mitf = 0, mitg = 0, mq = 0, nq = 1 << 30;
    double mkn = 0.0, mcolat = 0.0, nrt = 1e300;
    __device__ void add_cell(const CellStats &c) {
        if (!c.active) return;
        itf = c.it_f; itg = c.it_g; q = c.q; lim = c.lim; cells = 1;
        qp = (unsigned long long)c.q * c.pass; qpr = c.refined ? qp : 0ull; fb = c.fb;
        rp = (unsigned long long)c.rows * c.pass;
        mitf = c.it_f; mitg = c.it_g; mq = c.q; nq = c.q;
        mkn = c.kn; mcolat = c.colat; nrt = c.rt;
    }
    __device__ void add(const StatSum &o) {
        itf += o.itf; itg += o.itg; q += o.q; lim += o.lim; cells += o.cells; qp += o.qp; qpr += o.qpr;
        fb += o.fb; wq += o.wq; rp += o.rp;
        mitf = max(mitf, o.mitf); mitg = max(mitg, o.mitg); mq = max(mq, o.mq); nq = min(nq, o.nq);
        mkn = fmax(mkn, o.mkn); mcolat = fmax(mcolat, o.mcolat); nrt = fmin(nrt, o.nrt);
    }
    __device__ void wave_reduce() {
        for (int off = 32; off > 0; off >>= 1) {
            StatSum o;
            o.itf = __shfl_xor(itf, off); o.itg = __shfl_xor(itg, off); o.q = __shfl_xor(q, off);
            o.lim = __shfl_xor(lim, off); o.cells = __shfl_xor(cells, off); o.qp = __shfl_xor(qp, off);
            o.qpr = __shfl_xor(qpr, off); o.fb = __shfl_xor(fb, off); o.wq = __shfl_xor(wq, off);
            o.rp = __shfl_xor(rp, off);
            o.mitf = __shfl_xor(mitf, off); o.mitg = __shfl_xor(mitg, off); o.mq = __shfl_xor(mq, off);
            o.nq = __shfl_xor(nq, off);
            o.mkn = __shfl_xor(mkn, off); o.mcolat = __shfl_xor(mcolat, off); o.nrt = __shfl_xor(nrt, off);
            add(o);
        }
    }
    __device__ void load(const DevStats &d) {
        itf = d.it_sum_f; itg = d.it_sum_g; q = d.q_sum; lim = d.limited; cells = d.cells; qp = d.qpass_sum;
        qpr = d.qpass_ref_sum; fb = d.fallbacks; wq = d.wave_qpass; rp = d.row_passes;
        mitf = d.it_max_f; mitg = d.it_max_g; mq = d.q_max; nq = d.q_min;
        mkn = __longlong_as_double((long long)d.kn_max_bits);
        mcolat = __longlong_as_double((long long)d.colat_max_bits);
        nrt = __longlong_as_double((long long)d.rt_min_bits);
    }
    __device__ void store(DevStats &d) const {
        d.it_sum_f = itf; d.it_sum_g = itg; d.q_sum = q; d.limited = lim; d.cells = cells; d.qpass_sum = qp;
        d.qpass_ref_sum = qpr; d.fallbacks = fb; d.arrivals = 0; d.wave_qpass = wq; d.row_passes = rp;
        d.it_max_f = mitf; d.it_max_g = mitg; d.q_max = mq; d.q_min = nq;
        d.kn_max_bits = (unsigned long long)__double_as_longlong(mkn);
        d.colat_max_bits = (unsigned long long)__double_as_longlong(mcolat);
        d.rt_min_bits = (unsigned long long)__double_as_longlong(nrt);
    }
    // One atomic per field: for the few partials of a reduction (never per
    // wavefront of a large grid: same-address atomics serialise device-wide).
    __device__ void atomics_into(DevStats *st) const {
        if (cells == 0) return;
        atomicAdd(&st->it_sum_f, itf);
        atomicAdd(&st->it_sum_g, itg);
        atomicAdd(&st->q_sum, q);
        atomicAdd(&st->limited, lim);
        atomicAdd(&st->cells, cells);
        atomicAdd(&st->qpass_sum, qp);
        if (qpr) atomicAdd(&st->qpass_ref_sum, qpr);
        if (fb) atomicAdd(&st->fallbacks, fb);
        if (wq) atomicAdd(&st->wave_qpass, wq);
        if (rp) atomicAdd(&st->row_passes, rp);
        atomicMax(&st->it_max_f, mitf);
        atomicMax(&st->it_max_g, mitg);
        atomicMax(&st->q_max, mq);
        atomicMin(&st->q_min, nq);
        atomic_max_pos(&st->kn_max_bits, mkn);
        atomic_max_pos(&st->colat_max_bits, mcolat);
        atomic_min_pos(&st->rt_min_bits, nrt);
    }
};

// Lane occupancy of the stencil work: the lanes of a wavefront run in lock
// step, so a wavefront costs 64 x the largest q x passes of its cells.
__device__ inline unsigned long long wave_lanes_max(const CellStats &c) {
    unsigned long long m = c.active ? (unsigned long long)c.q * c.pass : 0ull;
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    return 64ull * m;
}

// Statistics of a workgroup's cells, one wave-reduced atomic set per wave
// (used by kernels that run on few workgroups).
__device__ inline void push_stats(DevStats *st, const CellStats &c) {
    StatSum a;
    a.add_cell(c);
    a.wave_reduce();
    a.wq = wave_lanes_max(c);
    if ((threadIdx.x & 63) == 0) a.atomics_into(st);
}

// Statistics of a 256-lane workgroup written as one partial (no atomics);
// k_stats_reduce sums the partials.  Every thread of the workgroup calls it.
__device__ inline void block_stats(DevStats *part, const CellStats &c) {
    __shared__ DevStats s_w[4];
    StatSum a;
    a.add_cell(c);
    a.wave_reduce();
    a.wq = wave_lanes_max(c);
    if ((threadIdx.x & 63) == 0) a.store(s_w[threadIdx.x >> 6]);
    __syncthreads();
    if (threadIdx.x == 0) {
        StatSum t;
        for (int w = 0; w < 4; w++) {
            StatSum o;
            o.load(s_w[w]);
            t.add(o);
        }
        t.store(part[blockIdx.x]);
    }
}

// Exact interval [xa, xb] of integer cx in row cy with |c - u| <= rr (the
// same predicate as the gather's), searched from the analytic estimate.
template <int D>
__device__ inline bool row_span(int cy, double ux, double uy, double rr, int lo, int hi, int &xa, int &xb) {
    double yy = D == 2 ? (double)cy - uy : 0.0;
    double rem = rr * rr - yy * yy;
    double w = rem > 0.0 ? sqrt(rem) : 0.0;
    int a = (int)ceil(ux - w), b = (int)floor(ux + w);
    a = a < lo ? lo : (a > hi ? hi : a);
    b = b > hi ? hi : (b < lo ? lo : b);
    auto in = [&](int cx) {
        return D == 2 ? in_disk2((double)cx, (double)cy, ux, uy, rr) : in_disk1((double)cx, ux, rr);
    };
    while (a > lo && in(a - 1)) a--;
    while (a <= b && !in(a)) a++;
    while (b < hi && in(b + 1)) b++;
    while (b >= a && !in(b)) b--;
    xa = a;
    xb = b;
    return a <= b;
}

// Learned guess inside the reconstruction kernel: every cell of a wavefront
// computes its 16 features, the 16 -> 64 -> 64 -> 16 network runs once per
// wavefront on MFMA (BF16 operands, FP32 accumulation), and each cell gets its
// destandardised output: the scaled correction beyond the linearised guess
// (the harvest target), from the cell's collision targets mf, mg.  The inputs
// (2 KB) and outputs (4 KB) of a wavefront are staged in the wavefront's own
// columns of the LDS direction arrays (dg: 6 x 64 doubles, df: 10 x 64, for
// NG = 6, NF = 10), which its cells' Newton state uses only afterwards, so a
// wavefront never waits for the others.
__device__ inline void mlp_guess_cells(const Buffers &b, const double *mf, const double *mg, double ux, double uy,
                                       double RT, int R, bool active, double *dg, double *df, float *out) {
    const int l = threadIdx.x, w64 = l & ~63, lane = l & 63;
    // sample r's inputs: chunk r / 16 of the wavefront's phonon-direction
    // columns (16 samples of 16 BF16 per 64-double chunk); outputs: chunk r / 8
    // of its fluon-direction columns (8 samples of 16 floats per chunk)
    auto xrow = [&](int r) { return (unsigned short *)(dg + (r >> 4) * TILE_N + w64) + (r & 15) * MLP_IN; };
    auto yrow = [&](int r) { return (float *)(df + (r >> 3) * TILE_N + w64) + (r & 7) * MLP_OUT; };
    float x[16];
#pragma unroll
    for (int k = 0; k < 16; k++) x[k] = 0.f;
    if (active) mlp_features(mf, mg, ux, uy, RT, R, x);
    unsigned short *xr = xrow(lane);
#pragma unroll
    for (int k = 0; k < 16; k++) xr[k] = f2bf(norm_in(b.mlp_n, k, x[k]));
    // LDS operations of one wavefront complete in order: the reads of other
    // lanes' rows below see these writes; the barrier keeps the compiler from
    // reordering them
    __builtin_amdgcn_wave_barrier();
    bf16x4 h1[4][4], h2[4][4];
    f32x4 y[4];
    mlp_forward_wave_rows(b.mlp_w, b.mlp_p, [&](int r) { return (const unsigned short *)xrow(r); }, h1, h2, y,
                          lane);
    const int r4 = 4 * (lane >> 4), c = lane & 15;
#pragma unroll
    for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int i = 0; i < 4; i++) yrow(16 * nt + c)[r4 + i] = y[nt][i];
    __builtin_amdgcn_wave_barrier();
    const float *yr = yrow(lane);
#pragma unroll
    for (int k = 0; k < 16; k++) out[k] = denorm_out(b.mlp_n, k, yr[k]);
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Reconstruction of cells without stencil refinement (N_r = 0).
//
// Along a stencil row (fixed c_y) the exponent of Eq. (IID7) is a cubic (fluon)
// or quadratic (phonon) polynomial of c_x, so consecutive populations follow
// from a product recurrence of exponentials of its finite differences: four
// (three) exponentials per row instead of two per point.  Row sums of f x^a
// are folded into the monomial sums S[a,b] = sum f x^a y^b (a + b <= 6 for the
// fluon, <= 4 for the phonon), from which the Newton residual and the Hessian
// A_ij = S[T_i T_j] (Eq. IID11a) are assembled.
// ---------------------------------------------------------------------------
template <int D>
__device__ inline void row_poly(const double *lf, const double *lg, double y, double *e, double *h) {
    if (D == 2) {
        double y2 = y * y, y3 = y2 * y;
        e[0] = -1.0 - (lf[0] + lf[2] * y + lf[5] * y2 + lf[9] * y3);
        e[1] = -(lf[1] + lf[4] * y + lf[8] * y2);
        e[2] = -(lf[3] + lf[7] * y);
        e[3] = -lf[6];
        h[0] = -1.0 - (lg[0] + lg[2] * y + lg[5] * y2);
        h[1] = -(lg[1] + lg[4] * y);
        h[2] = -lg[3];
    } else {
        e[0] = -1.0 - lf[0]; e[1] = -lf[1]; e[2] = -lf[2]; e[3] = -lf[3];
        h[0] = -1.0 - lg[0]; h[1] = -lg[1]; h[2] = -lg[2];
    }
}

// Starting value and ratios of the product recurrence at x0 = xa - ux.  The
// third difference of the fluon exponent (6 e3) and the second difference of
// the phonon exponent (2 h2) do not depend on the row; their exponentials
// t3 and sg2 are computed once per pass.
template <typename W>
__device__ inline void row_start(const double *e, const double *h, double x0, W &f, W &r, W &s2, W &gv, W &rg) {
    double E0 = e[0] + x0 * (e[1] + x0 * (e[2] + x0 * e[3]));
    double a2 = e[2] + 3.0 * e[3] * x0;
    double a1 = e[1] + x0 * (2.0 * e[2] + 3.0 * e[3] * x0);
    double H0 = h[0] + x0 * (h[1] + x0 * h[2]);
    double b1 = h[1] + 2.0 * h[2] * x0;
    if (sizeof(W) == 8) {
        f = exp(E0);
        r = exp(a1 + a2 + e[3]);
        s2 = exp(2.0 * a2 + 6.0 * e[3]);
        gv = exp(H0);
        rg = exp(b1 + h[2]);
    } else {
        f = expf((float)E0);
        r = expf((float)(a1 + a2 + e[3]));
        s2 = expf((float)(2.0 * a2 + 6.0 * e[3]));
        gv = expf((float)H0);
        rg = expf((float)(b1 + h[2]));
    }
}

template <typename W> __device__ inline W wexp(double v) {
    if (sizeof(W) == 8) return exp(v);
    return expf((float)v);
}

// Row starts along a column (2D).  The five exponents a stencil row needs at
// its first point -- E, its first and second x differences, H and its first x
// difference (see row_start) -- are polynomials in the row coordinate y at a
// fixed column x = X (cubic, quadratic, linear, quadratic, linear), so down
// the column they follow product recurrences of the exponentials of their
// forward differences in y: 14 exponentials per pass instead of 5 per row.
// Multipliers are in the basis order 1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2,
// y^3 (fluon) and 1, x, y, x^2, xy, y^2 (phonon).
struct ColumnStarts {
    double F, F1, F2, F3;   // exp(E(X, y)) and the exponentials of its y differences
    double R, R1, R2;       // exp(D_x E(X, y)) ...
    double S, S1;           // exp(D_x^2 E(X, y)) ...
    double G, G1, G2;       // exp(H(X, y)) ...
    double Q, Q1;           // exp(D_x H(X, y)) ...
    __device__ void init(const double *l, const double *g, double X, double y) {
        const double X2 = X * X;
        // E(X, y) = c0 + c1 y + c2 y^2 + c3 y^3
        const double c0 = -1.0 - (l[0] + l[1] * X + l[3] * X2 + l[6] * X2 * X);
        const double c1 = -(l[2] + l[4] * X + l[7] * X2), c2 = -(l[5] + l[8] * X), c3 = -l[9];
        F = exp(c0 + y * (c1 + y * (c2 + y * c3)));
        F1 = exp(c1 + c2 * (2.0 * y + 1.0) + c3 * (3.0 * y * y + 3.0 * y + 1.0));
        F2 = exp(2.0 * c2 + c3 * (6.0 * y + 6.0));
        F3 = exp(6.0 * c3);
        // D_x E(X, y) = d0 + d1 y + d2 y^2
        const double d0 = -l[1] - l[3] * (2.0 * X + 1.0) - l[6] * (3.0 * X2 + 3.0 * X + 1.0);
        const double d1 = -l[4] - l[7] * (2.0 * X + 1.0), d2 = -l[8];
        R = exp(d0 + y * (d1 + y * d2));
        R1 = exp(d1 + d2 * (2.0 * y + 1.0));
        R2 = exp(2.0 * d2);
        // D_x^2 E(X, y) = s0 + s1 y
        const double s0 = -2.0 * l[3] - l[6] * (6.0 * X + 6.0), s1 = -2.0 * l[7];
        S = exp(s0 + s1 * y);
        S1 = exp(s1);
        // H(X, y) = h0 + h1 y + h2 y^2
        const double h0 = -1.0 - (g[0] + g[1] * X + g[3] * X2), h1 = -(g[2] + g[4] * X), h2 = -g[5];
        G = exp(h0 + y * (h1 + y * h2));
        G1 = exp(h1 + h2 * (2.0 * y + 1.0));
        G2 = exp(2.0 * h2);
        // D_x H(X, y) = q0 + q1 y
        const double q0 = -g[1] - g[3] * (2.0 * X + 1.0), q1 = -g[4];
        Q = exp(q0 + q1 * y);
        Q1 = exp(q1);
    }
    __device__ void next() {
        F *= F1; F1 *= F2; F2 *= F3;
        R *= R1; R1 *= R2;
        S *= S1;
        G *= G1; G1 *= G2;
        Q *= Q1;
    }
};

// True when recurrence values can start a row (normal range, finite).
__device__ inline bool row_start_ok(double f, double r, double s2, double gv, double rg) {
    return f > 1e-280 && f < 1e280 && gv > 1e-280 && gv < 1e280 && r > 1e-280 && r < 1e280 && s2 > 1e-280 &&
           s2 < 1e280 && rg > 1e-280 && rg < 1e280;
}

// WIDE: the cells with wide stencils (wide_stencil(R)), on the tiles that
// hold any, with the recurrences restarted every REC_SEG points and rows;
// otherwise the other unrefined cells, whose rows are short enough to run
// each recurrence from one start.
template <typename T, int D, bool WIDE>
__global__ void __launch_bounds__(256, 2) k_epr(Geom g, Phys ph, const double *mom, Buffers b, int step, int tile0) {
    using BS = Basis<D>;
    constexpr int NF = BS::NF, NG = BS::NG, NMF = BS::NMF, NMG = BS::NMG, NM = BS::NMOM;
    // Per-point arithmetic stays FP64 in both paths: without packed FP32 math
    // an FP32 multiply-add costs the same issue slot as an FP64 one, and the
    // product recurrence in FP32 loses up to 1e-4 relative accuracy along long
    // rows (its rounding compounds cubically), which stalls the Newton line
    // search.  The mixed path gains from FP32 state, records and streaming.
    using W = double;
    __shared__ double s_lamf[NF * TILE_N], s_delf[NF * TILE_N], s_lamg[NG * TILE_N], s_delg[NG * TILE_N];
    __shared__ int s_err;
    // a band's tiles from tile0 on, heaviest first (k_scan)
    const int t = b.order[tile0 + blockIdx.x];
    DevStats *part = b.bpart + (WIDE ? (long long)g.ntx * g.nty : 0) + tile0;
    if (threadIdx.x == 0) s_err = b.flags->err || (WIDE && !b.tiles[t].wide);
    __syncthreads();
    if (s_err) {
        if (threadIdx.x == 0) StatSum().store(part[blockIdx.x]);
        return;
    }
    int tx0 = (t % g.ntx) * g.tx, ty0 = (t / g.ntx) * g.ty;
    int l = threadIdx.x;
    int px = tx0 + l % g.tx, py = ty0 + l / g.tx;
    bool valid = px < g.sxn && py < g.syn;
    long long s = (long long)py * g.sxn + px;
    int rn = valid ? b.desc_rn[s] : -1;
    CellStats cs;
    cs.active = rn >= 0 && (rn >> 16) == 0 && wide_stencil(rn & 0xffff) == WIDE;
    double rho = 0.0, ux = 0.0, uy = 0.0, RT = 1.0;
    double mf[NF], mg[NG];
    if (cs.active) {
        rho = b.desc_rho[s]; ux = b.desc_u[s]; uy = b.desc_u[g.ns + s]; RT = b.desc_rt[s];
        collide_targets<double, D>(g, ph, mom, s, rho, ux, uy, RT, mf, mg, cs.kn, cs.lim);
    }
    // learned guess: the network's correction, computed before the Newton
    // state takes over the LDS arrays it borrows
    float ynet[16];
    if constexpr (D == 2) {
        if (b.mlp_w)
            mlp_guess_cells(b, mf, mg, ux, uy, RT, rn & 0xffff, cs.active, s_delg, s_delf, ynet);
    }
    if (cs.active) {
        const TileInfo ti = b.tiles[t];
        const int R = rn & 0xffff;
        const double rr = R + 0.5;
        const int ubx = (int)floor(ux + 0.5), uby = D == 2 ? (int)floor(uy + 0.5) : 0;
        const int ylo = D == 2 ? uby - R - 1 : 0, yhi = D == 2 ? uby + R + 1 : 0;
        const int xlo = ubx - R - 1, xhi = ubx + R + 1;
        // stencil row spans, computed once and reused by every pass
        const bool tab = D == 1 ? 2 * R + 2 <= 255 : 2 * R + 3 <= SPAN_ROWS;
        // row k of the cell at spt[k * SW]: a row of a tile's 256 cells is
        // contiguous, so a wavefront reads one 128-byte line per row
        const long long SW = (long long)g.ntx * g.nty * TILE_N;
        unsigned short *spt = b.spans + (long long)t * TILE_N + l;
        if (tab) {
            for (int cy = ylo; cy <= yhi; cy++) {
                int xa, xb;
                unsigned short v = 0x00ff;
                if (row_span<D>(cy, ux, uy, rr, xlo, xhi, xa, xb)) v = (unsigned short)((xa - xlo) | ((xb - xlo) << 8));
                spt[(long long)(cy - ylo) * SW] = v;
            }
        }
        // Row cy's span from the table entry v (loaded one row ahead, so the
        // load latency hides behind the previous row's points) or, without a
        // table, computed directly.
        auto span = [&](unsigned v, int cy, int &xa, int &xb) -> bool {
            if (tab) {
                xa = xlo + (int)(v & 0xffu);
                xb = xlo + (int)(v >> 8);
                return xa <= xb;
            }
            return row_span<D>(cy, ux, uy, rr, xlo, xhi, xa, xb);
        };
        Species<NF, LdsStore<NF>> sf;
        Species<NG, LdsStore<NG>> sg;
        sf.v.lam_ = s_lamf + l; sf.v.del_ = s_delf + l;
        sg.v.lam_ = s_lamg + l; sg.v.del_ = s_delg + l;
        species_init<D, NF, NG>(sf, sg, RT);
        if (ph.lin_guess) species_linear<D>(sf, sg, mf, mg, RT);
        if (ph.prev_guess) species_prev<D>(sf, sg, mf, mg, RT, b.lamprev, g.ns, s);
        // learned guess: the linearised guess plus the network's scaled correction
        // (mlp_guess_cells); on top of the previous step's correction, where one
        // is stored, when the previous-step guess is on too (species_prev has then
        // applied the linearised guess and that correction)
        const bool prev_ok = ph.prev_guess && b.lamprev[s] == b.lamprev[s];
        if (D == 2 && b.mlp_w && (!ph.prev_guess || prev_ok)) {
            if (!ph.prev_guess) species_linear<D>(sf, sg, mf, mg, RT);
            const double sq = sqrt(RT);
#pragma unroll
            for (int j = 0; j < NF + NG; j++) {
                const int jj = j < NF ? j : j - NF;
                const int k = order_of<D>(jj);
                const double scl = k == 0 ? 1.0 : (k == 1 ? sq : (k == 2 ? RT : RT * sq));
                if (j < NF) sf.v.lam(jj) += (double)ynet[j] / scl;
                else sg.v.lam(jj) += (double)ynet[j] / scl;
            }
        }
        // residual scales RT^(-k/2) of basis order k (scale-free stopping test)
        const double isc[4] = {1.0, 1.0 / sqrt(RT), 1.0 / RT, 1.0 / (RT * sqrt(RT))};
        int fail = 0, fsp = -1;
        while (!fail && (sf.phase < 2 || sg.phase < 2)) {
            cs.pass++;
            double Sf[NMF], Sg[NMG];
#pragma unroll
            for (int k = 0; k < NMF; k++) Sf[k] = 0.0;
#pragma unroll
            for (int k = 0; k < NMG; k++) Sg[k] = 0.0;
            // multipliers of this pass live in LDS; registers hold them only
            // while the column and the rare direct row starts are set up
            unsigned nxt = tab ? spt[0] : 0u;
            const W t3 = wexp<W>(-6.0 * sf.at(D == 2 ? 6 : 3));
            const W sg2 = wexp<W>(-2.0 * sg.at(D == 2 ? 3 : 2));
            ColumnStarts col;
            if (D == 2) {
                double lf[NF], lg[NG];
#pragma unroll
                for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
                for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
                col.init(lf, lg, (double)xlo - ux, (double)ylo - uy);
            }
            for (int cy = ylo; cy <= yhi; cy++) {
                if constexpr (WIDE) {
                    if (D == 2 && cy != ylo && (cy - ylo) % REC_SEG == 0) {
                        double lf[NF], lg[NG];
#pragma unroll
                        for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
                        for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
                        col.init(lf, lg, (double)xlo - ux, (double)cy - uy);
                    }
                }
                W f = 0, r = 0, s2 = 0, gv = 0, rg = 0;
                if (D == 2) { f = col.F; r = col.R; s2 = col.S; gv = col.G; rg = col.Q; col.next(); }
                const unsigned cur = nxt;
                if (tab && cy < yhi) nxt = spt[(long long)(cy + 1 - ylo) * SW];
                int xa, xb;
                if (!span(cur, cy, xa, xb)) continue;
                double y = D == 2 ? (double)cy - uy : 0.0;
                const bool walk = D == 2 && (!WIDE || xa - xlo < REC_SEG);
                if (walk) {
                    // walk from the column to the row's first point
                    for (int k = xlo; k < xa; k++) { f *= r; r *= s2; s2 *= t3; gv *= rg; rg *= sg2; }
                }
                if (!walk || !row_start_ok(f, r, s2, gv, rg)) {
                    double lf[NF], lg[NG], e[4], h[3];
#pragma unroll
                    for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
                    for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
                    row_poly<D>(lf, lg, y, e, h);
                    row_start<W>(e, h, (double)xa - ux, f, r, s2, gv, rg);
                }
                W Rf[7], Rg[5];
#pragma unroll
                for (int k = 0; k < 7; k++) Rf[k] = 0;
#pragma unroll
                for (int k = 0; k < 5; k++) Rg[k] = 0;
                for (int cx = xa; cx <= xb; cx++) {
                    if constexpr (WIDE) {
                        if (cx != xa && (cx - xlo) % REC_SEG == 0) {
                            double lf[NF], lg[NG], e[4], h[3];
#pragma unroll
                            for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
                            for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
                            row_poly<D>(lf, lg, y, e, h);
                            row_start<W>(e, h, (double)cx - ux, f, r, s2, gv, rg);
                        }
                    }
                    W x = (W)((double)cx - ux);
                    W x2 = x * x, x3 = x2 * x, x4 = x2 * x2, x5 = x4 * x, x6 = x3 * x3;
                    Rf[0] += f; Rf[1] += f * x; Rf[2] += f * x2; Rf[3] += f * x3;
                    Rf[4] += f * x4; Rf[5] += f * x5; Rf[6] += f * x6;
                    Rg[0] += gv; Rg[1] += gv * x; Rg[2] += gv * x2; Rg[3] += gv * x3; Rg[4] += gv * x4;
                    f *= r; r *= s2; s2 *= t3;
                    gv *= rg; rg *= sg2;
                }
                if (D == 2) {
                    double py_[7];
                    py_[0] = 1.0;
#pragma unroll
                    for (int k = 1; k < 7; k++) py_[k] = py_[k - 1] * y;
#pragma unroll
                    for (int k = 0; k < NMF; k++) Sf[k] += py_[mono_b(k)] * (double)Rf[mono_a(k)];
#pragma unroll
                    for (int k = 0; k < NMG; k++) Sg[k] += py_[mono_b(k)] * (double)Rg[mono_a(k)];
                } else {
#pragma unroll
                    for (int k = 0; k < NMF; k++) Sf[k] += (double)Rf[k];
#pragma unroll
                    for (int k = 0; k < NMG; k++) Sg[k] += (double)Rg[k];
                }
            }
            if (sg.phase < 2) {
                int r = species_update<D, NG, NMG>(sg, Sg, mg, isc, ph.tol, ph.maxit);
                if (r < 0 && r != -FAIL_CHOL_POLISH && sg.mlp) r = RESTART_EQ;
                if (r < 0) { fail = -r; fsp = 1; }
                else if (r == RESTART_EQ) { species_restart_eq<D>(sg, RT); cs.fb = 1; }
            }
            if (sf.phase < 2 && !fail) {
                int r = species_update<D, NF, NMF>(sf, Sf, mf, isc, ph.tol, ph.maxit);
                if (r < 0 && r != -FAIL_CHOL_POLISH && sf.mlp) r = RESTART_EQ;
                if (r < 0) { fail = -r; fsp = 0; }
                else if (r == RESTART_EQ) { species_restart_eq<D>(sf, RT); cs.fb = 1; }
            }
        }
        if (fail) {
            flag_fail(b.flags, LELBM_EEPR, step, s, fail, fsp, fsp ? sg.res : sf.res);
        } else {
            // harvest: what the network should add to the context's own start --
            // the linearised guess, plus the stored correction with the
            // previous-step guess (cells without one are not harvested then)
            if (D == 2 && b.harvest && (!ph.prev_guess || prev_ok) &&
                ((s + (long long)step * 7919) % b.harvest_stride) == 0) {
                unsigned long long slot = atomicAdd(b.harvest_n, 1ull);
                if (slot < (unsigned long long)b.harvest_cap) {
                    float x[16];
                    mlp_features(mf, mg, ux, uy, RT, R, x);
                    float *hp = b.harvest + slot * 32;
#pragma unroll
                    for (int k = 0; k < 16; k++) hp[k] = x[k];
                    const double sq = sqrt(RT);
                    double dl[16];
                    lin_guess_scaled<2>(mf, mg, RT, dl);
#pragma unroll
                    for (int j = 0; j < NF + NG; j++) {
                        const int jj = j < NF ? j : j - NF;
                        const double lam = j < NF ? sf.v.lam(jj) : sg.v.lam(jj);
                        const int k = basis_order2(jj);
                        const double scl = k == 0 ? 1.0 : (k == 1 ? sq : (k == 2 ? RT : RT * sq));
                        const double e = prev_ok ? b.lamprev[(long long)j * g.ns + s] : 0.0;
                        hp[16 + j] = (float)(lam * scl - iid13_scaled(jj, RT) - dl[j] - e);
                    }
                }
            }
            if (ph.prev_guess) store_prev<D>(sf, sg, mf, mg, RT, b.lamprev, g.ns, s);
            // final pass: moment fractions rho f', rho K RT g' (Eq. IIE3a), rho plus
            // the mass a point source adds in its cell
            const double wsf = post_mass(ph, s, rho), wsg = wsf * ph.K * RT;
            T *P = (T *)b.scratch + ti.base;
            int q = 0;
            unsigned nxt = tab ? spt[0] : 0u;
            const W t3 = wexp<W>(-6.0 * sf.v.lam(D == 2 ? 6 : 3));
            const W sg2 = wexp<W>(-2.0 * sg.v.lam(D == 2 ? 3 : 2));
            const W wsfw = (W)wsf, wsgw = (W)wsg;
            ColumnStarts col;
            if (D == 2) {
                double lf[NF], lg[NG];
#pragma unroll
                for (int j = 0; j < NF; j++) lf[j] = sf.v.lam(j);
#pragma unroll
                for (int j = 0; j < NG; j++) lg[j] = sg.v.lam(j);
                col.init(lf, lg, (double)xlo - ux, (double)ylo - uy);
            }
            for (int cy = ylo; cy <= yhi; cy++) {
                if constexpr (WIDE) {
                    if (D == 2 && cy != ylo && (cy - ylo) % REC_SEG == 0) {
                        double lf[NF], lg[NG];
#pragma unroll
                        for (int j = 0; j < NF; j++) lf[j] = sf.v.lam(j);
#pragma unroll
                        for (int j = 0; j < NG; j++) lg[j] = sg.v.lam(j);
                        col.init(lf, lg, (double)xlo - ux, (double)cy - uy);
                    }
                }
                W f = 0, r = 0, s2 = 0, gv = 0, rg = 0;
                if (D == 2) { f = col.F; r = col.R; s2 = col.S; gv = col.G; rg = col.Q; col.next(); }
                const unsigned cur = nxt;
                if (tab && cy < yhi) nxt = spt[(long long)(cy + 1 - ylo) * SW];
                int xa, xb;
                if (!span(cur, cy, xa, xb)) continue;
                cs.rows++;
                double y = D == 2 ? (double)cy - uy : 0.0;
                const bool walk = D == 2 && (!WIDE || xa - xlo < REC_SEG);
                if (walk) {
                    for (int k = xlo; k < xa; k++) { f *= r; r *= s2; s2 *= t3; gv *= rg; rg *= sg2; }
                }
                if (!walk || !row_start_ok(f, r, s2, gv, rg)) {
                    double lf[NF], lg[NG], e[4], h[3];
#pragma unroll
                    for (int j = 0; j < NF; j++) lf[j] = sf.v.lam(j);
#pragma unroll
                    for (int j = 0; j < NG; j++) lg[j] = sg.v.lam(j);
                    row_poly<D>(lf, lg, y, e, h);
                    row_start<W>(e, h, (double)xa - ux, f, r, s2, gv, rg);
                }
                long long rowslot = (long long)(cy - ti.oy) * ti.wx - ti.ox;
                for (int cx = xa; cx <= xb; cx++) {
                    if constexpr (WIDE) {
                        if (cx != xa && (cx - xlo) % REC_SEG == 0) {
                            double lf[NF], lg[NG], e[4], h[3];
#pragma unroll
                            for (int j = 0; j < NF; j++) lf[j] = sf.v.lam(j);
#pragma unroll
                            for (int j = 0; j < NG; j++) lg[j] = sg.v.lam(j);
                            row_poly<D>(lf, lg, y, e, h);
                            row_start<W>(e, h, (double)cx - ux, f, r, s2, gv, rg);
                        }
                    }
                    W wf = wsfw * f, wg = wsgw * gv;
                    long long slot = rowslot + cx;
                    if (ti.fmt == 0) {
                        // streaming stores: the records are read once, by the gather
                        __builtin_nontemporal_store((T)wf, &P[(slot * TILE_N + l) * 2]);
                        __builtin_nontemporal_store((T)wg, &P[(slot * TILE_N + l) * 2 + 1]);
                    } else {
                        W c1 = (W)cx, c2 = (W)cy;
                        W mo[NM];
                        if constexpr (D == 1) {
                            mo[0] = wf; mo[1] = c1 * wf; mo[2] = c1 * c1 * wf; mo[3] = c1 * c1 * c1 * wf;
                            mo[4] = wg; mo[5] = c1 * wg;
                        } else {
                            W cc = c1 * c1 + c2 * c2;
                            mo[0] = wf; mo[1] = c1 * wf; mo[2] = c2 * wf;
                            mo[3] = c1 * c1 * wf; mo[4] = c1 * c2 * wf; mo[5] = c2 * c2 * wf;
                            mo[6] = cc * c1 * wf; mo[7] = cc * c2 * wf;
                            mo[8] = wg; mo[9] = c1 * wg; mo[10] = c2 * wg;
                        }
#pragma unroll
                        for (int k = 0; k < NM; k++) P[(slot * TILE_N + l) * NM + k] = mo[k];
                    }
                    f *= r; r *= s2; s2 *= t3;
                    gv *= rg; rg *= sg2;
                    q++;
                }
            }
            cs.pass++;
            cs.it_f = sf.nit;
            cs.it_g = sg.nit;
            cs.q = q;
            cs.rt = RT;
            cs.colat = (D == 2 ? sqrt(ux * ux + uy * uy) : fabs(ux)) + R;
        }
    }
    block_stats(part, cs);
}

// ---------------------------------------------------------------------------
// Reconstruction of cells with refined stencils (N_r > 0, RT < 4/9): points
// are visited one by one (Eqs. IIC10-11) with direct exponentials, and the
// moment fractions of each base point's descendants are pre-summed, since
// they all land in the base point's cell.  Runs only on tiles that hold
// refined cells.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ void epr_ref_tile(const Geom &g, const Phys &ph, const double *mom, Buffers &b, int step, int t) {
    using BS = Basis<D>;
    constexpr int NF = BS::NF, NG = BS::NG, NMF = BS::NMF, NMG = BS::NMG, NM = BS::NMOM;
    int tx0 = (t % g.ntx) * g.tx, ty0 = (t / g.ntx) * g.ty;
    int l = threadIdx.x;
    int px = tx0 + l % g.tx, py = ty0 + l / g.tx;
    bool valid = px < g.sxn && py < g.syn;
    long long s = (long long)py * g.sxn + px;
    int rn = valid ? b.desc_rn[s] : -1;
    CellStats cs;
    cs.active = rn >= 0 && (rn >> 16) > 0;
    cs.refined = true;
    if (cs.active) {
        // refined cells leave no correction for the next step's warm start
        if (ph.prev_guess) b.lamprev[s] = __builtin_nan("");
        const TileInfo ti = b.tiles[t];
        double rho = b.desc_rho[s], ux = b.desc_u[s], uy = b.desc_u[g.ns + s], RT = b.desc_rt[s];
        int R = rn & 0xffff, Nr = rn >> 16;
        double mf[NF], mg[NG];
        collide_targets<double, D>(g, ph, mom, s, rho, ux, uy, RT, mf, mg, cs.kn, cs.lim);
        Species<NF, RegStore<NF>> sf;
        Species<NG, RegStore<NG>> sg;
        species_init<D, NF, NG>(sf, sg, RT);
        // residual scales RT^(-k/2) of basis order k (scale-free stopping test)
        const double isc[4] = {1.0, 1.0 / sqrt(RT), 1.0 / RT, 1.0 / (RT * sqrt(RT))};
        int fail = 0, fsp = -1;
        while (!fail && (sf.phase < 2 || sg.phase < 2)) {
            cs.pass++;
            double Sf[NMF], Sg[NMG], lf[NF], lg[NG];
#pragma unroll
            for (int k = 0; k < NMF; k++) Sf[k] = 0.0;
#pragma unroll
            for (int k = 0; k < NMG; k++) Sg[k] = 0.0;
#pragma unroll
            for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
            for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
            for_each_point<D>(
                ux, uy, R, Nr,
                [&](double cx, double cy, double dC, int, int) {
                    double m[NMF];
                    monomials<D, NMF>(cx - ux, D == 2 ? cy - uy : 0.0, m);
                    double e = 0.0;
#pragma unroll
                    for (int j = 0; j < NF; j++) e += lf[j] * m[j];
                    double f = dC * exp(-(1.0 + e));
#pragma unroll
                    for (int k = 0; k < NMF; k++) Sf[k] += f * m[k];
                    double e2 = 0.0;
#pragma unroll
                    for (int j = 0; j < NG; j++) e2 += lg[j] * m[j];
                    double gv = dC * exp(-(1.0 + e2));
#pragma unroll
                    for (int k = 0; k < NMG; k++) Sg[k] += gv * m[k];
                },
                [&](int, int) {});
            if (sg.phase < 2) {
                int r = species_update<D, NG, NMG>(sg, Sg, mg, isc, ph.tol, ph.maxit);
                if (r < 0) { fail = -r; fsp = 1; }
            }
            if (sf.phase < 2 && !fail) {
                int r = species_update<D, NF, NMF>(sf, Sf, mf, isc, ph.tol, ph.maxit);
                if (r < 0) { fail = -r; fsp = 0; }
            }
        }
        if (fail) {
            flag_fail(b.flags, LELBM_EEPR, step, s, fail, fsp, fsp ? sg.res : sf.res);
        } else {
            const double wsf = post_mass(ph, s, rho), wsg = wsf * ph.K * RT;
            T *P = (T *)b.scratch + ti.base;
            double acc[NM];
#pragma unroll
            for (int k = 0; k < NM; k++) acc[k] = 0.0;
            int q = 0;
            for_each_point<D>(
                ux, uy, R, Nr,
                [&](double cx, double cy, double dC, int, int) {
                    double m[NF];
                    monomials<D, NF>(cx - ux, D == 2 ? cy - uy : 0.0, m);
                    double ef = 0.0, eg = 0.0;
#pragma unroll
                    for (int j = 0; j < NF; j++) ef += sf.v.lam(j) * m[j];
#pragma unroll
                    for (int j = 0; j < NG; j++) eg += sg.v.lam(j) * m[j];
                    double wf = wsf * (dC * exp(-(1.0 + ef)));
                    double wg = wsg * (dC * exp(-(1.0 + eg)));
                    q++;
                    if (D == 1) {
                        acc[0] += wf; acc[1] += cx * wf; acc[2] += cx * cx * wf; acc[3] += cx * cx * cx * wf;
                        acc[4] += wg; acc[5] += cx * wg;
                    } else {
                        double cc = cx * cx + cy * cy;
                        acc[0] += wf; acc[1] += cx * wf; acc[2] += cy * wf;
                        acc[3] += cx * cx * wf; acc[4] += cx * cy * wf; acc[5] += cy * cy * wf;
                        acc[6] += cc * cx * wf; acc[7] += cc * cy * wf;
                        acc[8] += wg; acc[9] += cx * wg; acc[10] += cy * wg;
                    }
                },
                [&](int dx, int dy) {
                    long long slot = (long long)(dy - ti.oy) * ti.wx + (dx - ti.ox);
#pragma unroll
                    for (int k = 0; k < NM; k++) {
                        P[(slot * TILE_N + l) * NM + k] = (T)acc[k];
                        acc[k] = 0.0;
                    }
                });
            cs.pass++;
            cs.it_f = sf.nit;
            cs.it_g = sg.nit;
            cs.q = q;
            cs.rt = RT;
            cs.colat = (D == 2 ? sqrt(ux * ux + uy * uy) : fabs(ux)) + R;
        }
    }
    push_stats(b.stats, cs);
}

// The band's tiles with refined cells (listed by k_scan), a fixed grid of
// workgroups taking them in turn: with none, the launch ends at once.  Two
// waves per SIMD (the kernel spills), so that its workgroups fit beside the
// other reconstruction kernels of the concurrent bands instead of waiting for
// a CU to drain.
template <typename T, int D>
__global__ void __launch_bounds__(256, 2) k_epr_ref(Geom g, Phys ph, const double *mom, Buffers b, int step, int tile0,
                                                    int band) {
    __shared__ int s_skip;
    if (threadIdx.x == 0) s_skip = b.flags->err;
    __syncthreads();
    if (s_skip) return;
    const int n = b.rcount[band];
    for (int j = blockIdx.x; j < n; j += gridDim.x) epr_ref_tile<T, D>(g, ph, mom, b, step, b.rlist[tile0 + j]);
}

// ---------------------------------------------------------------------------
// Learned initial multipliers for the unrefined cells of a tile (2D): the
// collision targets and stencil geometry of each cell are fed through the
// warm-start network (one wavefront = 64 cells, BF16 MFMA); the outputs are
// turned back into multipliers and stored for k_epr.  Refined cells keep
// Eq. (IID13) in k_epr_ref.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// moment-streaming gather, Eq. (IIE3b)
//
// One workgroup per 16x16 (2D) or 256x1 (1D) destination tile; one thread per
// destination cell.  Every destination scans the tile's window of landing
// displacements d; the source of displacement d is x - d (wrapped on periodic
// axes, mirrored across slip walls, which reflects the path specularly).  The
// descriptors of the sources a chunk of window rows needs (velocity, radius,
// scratch record address, mirror flags) are staged in LDS once per
// workgroup, so the per-candidate work is the exact disk test of the source's
// stencil (the same FP64 predicate its reconstruction used) and, on a hit, one
// coalesced read of the moment fractions.  Along a window row c_y is fixed,
// so the row accumulates sum w_f c_x^k (k <= 3) and sum w_g c_x^k (k <= 1)
// and the eleven moments are formed once per row.
// ---------------------------------------------------------------------------
constexpr int GU = 4;         // candidates per batch in the gather

struct Resolved {
    long long s;    // padded source index, -1 if none
    int px, py;     // padded source coordinates
    int fx, fy;     // 1 if the path is mirrored in x / y
    int wf;         // the no-slip wall face (0 ylo, 1 yhi) the path is mirrored across, -1 none
};

// Source tile and the cell's place in it from padded coordinates (tile
// shapes are powers of two, so these are shifts and masks).
template <int D>
__device__ inline void tile_of(const Geom &g, int px, int py, int &st, int &loc) {
    constexpr unsigned TX = tile_x<D>(), TY = tile_y<D>();
    const unsigned ux = (unsigned)px, uy = (unsigned)py;
    st = (int)(ux / TX + uy / TY * (unsigned)g.ntx);
    loc = (int)(ux % TX + uy % TY * TX);
}

template <int D>
__device__ inline Resolved resolve_source(const Geom &g, int xr, int yr) {
    Resolved r{-1, 0, 0, 0, 0, -1};
    int sx = xr, sy = yr;
    if (g.bc[0] == LELBM_BC_PERIODIC) { sx %= g.nx; if (sx < 0) sx += g.nx; }
    else if (sx < 0 && g.bc[0] == LELBM_BC_SLIPWALL) { sx = -1 - sx; r.fx = 1; }
    else if (sx >= g.nx && g.bc[1] == LELBM_BC_SLIPWALL) { sx = 2 * g.nx - 1 - sx; r.fx = 1; }
    if (sx < -g.wl || sx >= g.nx + g.wr) return r;
    if (D == 2) {
        if (g.bc[2] == LELBM_BC_PERIODIC) { sy %= g.ny; if (sy < 0) sy += g.ny; }
        else if (sy < 0 && g.bc[2] == LELBM_BC_SLIPWALL) { sy = -1 - sy; r.fy = 1; }
        else if (sy >= g.ny && g.bc[3] == LELBM_BC_SLIPWALL) { sy = 2 * g.ny - 1 - sy; r.fy = 1; }
        else if (sy < 0 && g.bc[2] == LELBM_BC_WALL) { sy = -1 - sy; r.fy = 1; r.wf = 0; }
        else if (sy >= g.ny && g.bc[3] == LELBM_BC_WALL) { sy = 2 * g.ny - 1 - sy; r.fy = 1; r.wf = 1; }
        if (sy < -g.wb || sy >= g.ny + g.wt) return r;
    } else {
        sy = 0;
    }
    r.px = sx + g.wl;
    r.py = sy + g.wb;
    r.s = (long long)r.py * g.sxn + r.px;
    return r;
}

// A path mirrored across a no-slip wall is absorbed there (Eq. IIIB8); it
// arrives only when its source reflects its absorbed populations
// specularly (no image population of the source crosses that wall).
__device__ inline bool wall_keeps(const Geom &g, const Buffers &b, const Resolved &r) {
    if (r.wf < 0) return true;
    const int sy = r.py - g.wb;
    const int row = r.wf == 0 ? sy : g.ny - 1 - sy;
    if (row < 0 || row >= g.wrows) return false;
    return (b.wflag[((long long)r.wf * g.wrows + row) * g.sxn + r.px] & WALL_FLAG_SPECULAR) != 0;
}

// Adds the moment fractions of one arriving record; (cx, cy) is the
// velocity after reflection; for pre-summed refined records the odd
// components are mirrored.
template <typename T, int D>
__device__ inline void deposit_record(double *acc, const T *P, int fmt, int dx, int dy, int fx, int fy) {
    if (fmt == 0) {
        const double wx_ = (double)P[0], wy_ = (double)P[1];
        double cx = (double)dx, cy = (double)dy;
        if (D == 1) {
            acc[0] += wx_; acc[1] += cx * wx_; acc[2] += cx * cx * wx_; acc[3] += cx * cx * cx * wx_;
            acc[4] += wy_; acc[5] += cx * wy_;
        } else {
            double cc = cx * cx + cy * cy;
            acc[0] += wx_; acc[1] += cx * wx_; acc[2] += cy * wx_;
            acc[3] += cx * cx * wx_; acc[4] += cx * cy * wx_; acc[5] += cy * cy * wx_;
            acc[6] += cc * cx * wx_; acc[7] += cc * cy * wx_;
            acc[8] += wy_; acc[9] += cx * wy_; acc[10] += cy * wy_;
        }
    } else {
        double sx1 = fx ? -1.0 : 1.0, sy1 = fy ? -1.0 : 1.0;
        if (D == 1) {
            acc[0] += (double)P[0]; acc[1] += sx1 * (double)P[1]; acc[2] += (double)P[2];
            acc[3] += sx1 * (double)P[3]; acc[4] += (double)P[4]; acc[5] += sx1 * (double)P[5];
        } else {
            acc[0] += (double)P[0]; acc[1] += sx1 * (double)P[1]; acc[2] += sy1 * (double)P[2];
            acc[3] += (double)P[3]; acc[4] += sx1 * sy1 * (double)P[4]; acc[5] += (double)P[5];
            acc[6] += sx1 * (double)P[6]; acc[7] += sy1 * (double)P[7];
            acc[8] += (double)P[8]; acc[9] += sx1 * (double)P[9]; acc[10] += sy1 * (double)P[10];
        }
    }
}

// Blockers of a population path (Sec. III.B): solid cells and the cells
// beyond a slip wall.
__device__ inline bool is_blocked(const Geom &g, const unsigned char *solid, int x, int y) {
    if (x < 0 && g.bc[0] == LELBM_BC_SLIPWALL) return true;
    if (x >= g.nx && g.bc[1] == LELBM_BC_SLIPWALL) return true;
    if (g.dim == 2 && y < 0 && g.bc[2] == LELBM_BC_SLIPWALL) return true;
    if (g.dim == 2 && y >= g.ny && g.bc[3] == LELBM_BC_SLIPWALL) return true;
    return solid && x >= 0 && x < g.nx && y >= 0 && y < g.ny && solid[(long long)y * g.nx + x];
}

// A population's path crosses the grid lines x = const and y = const in the
// order of its path parameter ((2k+1)/(2|v|) for the k-th crossing of each
// kind), an x crossing first where both coincide; a crossing into a blocker
// reverses that velocity component, otherwise the path enters the next cell.
// walk_back undoes such a path: from the landing cell with the landing
// velocity reversed it takes the same crossings in reverse order (so y
// first where they coincide), each of which exactly undoes its forward
// counterpart.  It returns the cell of origin and the signs the forward path
// applied to each component, or false if it leaves the padded domain (no
// source there).  The walk runs in unwrapped coordinates (each stays within
// |v| of the landing cell, each probe within |v| + 1); blocked(x, y) wraps
// periodic axes itself, and the origin is returned wrapped (ox, oy) and
// unwrapped (ux, uy).
__device__ inline int wrap_coord(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <int D>
__device__ inline bool blocked_wrapped(const Geom &g, const unsigned char *solid, int x, int y) {
    if (g.bc[0] == LELBM_BC_PERIODIC) x = wrap_coord(x, g.nx);
    if (D == 2 && g.bc[2] == LELBM_BC_PERIODIC) y = wrap_coord(y, g.ny);
    return is_blocked(g, solid, x, y);
}

template <int D, typename Blocked>
__device__ inline bool walk_back(const Geom &g, const Blocked &blocked, int x, int y, int vx, int vy, int &ox,
                                 int &oy, int &ux, int &uy, int &sgx, int &sgy) {
    // Every step is written with selects rather than branches (the crossing
    // order depends only on |v|, the same for all lanes of a call); a walk
    // that leaves the padded domain is finished and then rejected.
    const int ax = abs(vx), ay = abs(vy);
    // the crossing counters live in vector registers: the walk's selects then
    // run on the SIMDs instead of the CU's one scalar unit
    int kx, ky;
    asm volatile("v_mov_b32 %0, 0" : "=v"(kx));
    asm volatile("v_mov_b32 %0, 0" : "=v"(ky));
    int sx = vx < 0 ? -1 : 1, sy = vy < 0 ? -1 : 1;
    const bool perx = g.bc[0] == LELBM_BC_PERIODIC, pery = D == 2 && g.bc[2] == LELBM_BC_PERIODIC;
    bool out = false;
#pragma unroll 4
    for (int k = 0; k < ax + ay; k++) {
        const bool takey =
            kx >= ax || (ky < ay && __mul24(2 * ky + 1, ax) <= __mul24(2 * kx + 1, ay));  // < 2^31 for |v| < 2^15
        const int px = takey ? x : x + sx, py = takey ? y + sy : y;
        const bool bl = blocked(px, py);
        x = bl ? x : px;
        y = bl ? y : py;
        sx = (bl && !takey) ? -sx : sx;
        sy = (bl && takey) ? -sy : sy;
        kx += takey ? 0 : 1;
        ky += takey ? 1 : 0;
        out = out || (!perx && (x < -g.wl || x >= g.nx + g.wr)) || (!pery && (y < -g.wb || y >= g.ny + g.wt));
    }
    if (out) return false;
    ux = x;
    uy = y;
    ox = perx ? wrap_coord(x, g.nx) : x;
    oy = pery ? wrap_coord(y, g.ny) : y;
    // the forward path ends with velocity -(sx, sy) and started with -(vx, vy) times its flips
    sgx = (vx == 0 || (sx < 0) == (vx < 0)) ? 1 : -1;
    sgy = (vy == 0 || (sy < 0) == (vy < 0)) ? 1 : -1;
    return true;
}

// Distance from destination tile t to the blockers its arrivals must be
// traced around: solid cells always; slip walls only where one path could
// reflect off both walls of an axis (the domain at most 2M + 2 cells across).
// Elsewhere a path meets at most one wall per axis, and the straight gather's
// mirror images across the walls are exact (each reflection folds one
// coordinate, independently of the other axis).
__device__ inline int walk_distance(const Geom &g, const Buffers &b, int t, int M) {
    const bool wx = g.bc[0] == LELBM_BC_SLIPWALL || g.bc[1] == LELBM_BC_SLIPWALL;
    const bool wy = g.dim == 2 && (g.bc[2] == LELBM_BC_SLIPWALL || g.bc[3] == LELBM_BC_SLIPWALL);
    const bool narrow = (wx && g.nx <= 2 * M + 2) || (wy && g.ny <= 2 * M + 2);
    return narrow ? b.tdist[t] : b.tdist_s[t];
}

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Gather LDS per staged source: velocity (16 B), record base (8 B), meta (4 B).
constexpr int G_ENTRY_BYTES = 28;
// meta bits: [0,8) radius R, 8 / 9 mirrored in x / y, 10 refined (all-moment
// records), [11,32) slot box width of the source tile; -1 = no source
constexpr int META_FX = 1 << 8, META_FY = 1 << 9, META_REF = 1 << 10;

// WALLS: some face is a slip wall (sources may be mirror images).  Sources
// with refined stencils are skipped by the main scan and handled by a second
// scan that runs only in workgroups whose staged region holds one.  The sums
// are FP64 in both precision modes (the FP32 records are widened as they
// arrive); four wavefronts per SIMD (capped at five, the FP64 accumulators
// spill at the row level and the kernel is 19 % slower).
template <typename T, int D, bool WALLS>
__global__ void __launch_bounds__(256, 4) k_gather(Geom g, double *mom_out, Buffers b, int gcap, int br0, int nbr) {
    constexpr int NM = Basis<D>::NMOM;
    extern __shared__ double2 g_lds[];
    double2 *s_u = g_lds;
    long long *s_a0 = (long long *)(s_u + gcap);
    int *s_meta = (int *)(s_a0 + gcap);
    __shared__ int s_err, s_ref;
    if (threadIdx.x == 0) s_err = b.flags->err;
    __syncthreads();
    const int nbx = gather_blocks_x(g);
    if (s_err) {
        if (threadIdx.x == 0) b.gpart[(long long)br0 * nbx + blockIdx.x] = 0ull;
        return;
    }
    // Destination block of a workgroup: in 2D a GATHER_NTB x 16 wide and
    // 16 / GATHER_NTB high strip of GATHER_NTB x-neighbour tiles, each
    // wavefront 16 x 4 cells of one of them; in 1D one tile.  A record line
    // holds 16 cells of a source-tile row; the destination row segment it
    // lands on straddles two tiles, and with both in one workgroup the second
    // half is read from the L1 of the same CU.
    constexpr int TX = tile_x<D>(), TY = tile_y<D>();
    constexpr int NTB = D == 2 ? GATHER_NTB : 1;
    constexpr int BX = NTB * TX, BY = TY / NTB;
    // The launch covers block rows [br0, br0 + nbr).  Workgroups go to the 8
    // XCDs in turn.  Deal whole block rows to the XCDs instead (row r to XCD
    // r mod 8, in order), so that x-neighbour blocks, which read the two
    // halves of the record lines on their common edge, run on the same XCD at
    // about the same time and the second read hits its L2; rows that do not
    // fill a round of 8 keep the plain order.
    int t = blockIdx.x;
    {
        const int full = nbr / 8 * 8 * nbx;
        if (t < full) {
            const int k = t & 7, i = t >> 3;
            t = (i / nbx * 8 + k) * nbx + i % nbx;
        }
    }
    const int x0 = (t % nbx) * BX, y0 = (br0 + t / nbx) * BY;
    int lx, ly;                                  // the lane's cell in the block
    if (D == 2) {
        const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
        lx = (wv % NTB) * TX + (l & 15);
        ly = (wv / NTB) * 4 + (l >> 4);
    } else {
        lx = threadIdx.x;
        ly = 0;
    }
    const int x = x0 + lx, y = y0 + ly;
    const bool mine = x < g.nx && y < g.ny;
    // Tiles within reach of a blocker: every landing displacement d with
    // |d_x|, |d_y| <= the step's maximum reach M is traced back to the source
    // it comes from (walk_back), which finds the straight and the reflected
    // arrivals alike.  Elsewhere no path that ends in the tile can touch a
    // blocker (it would have to pass within M cells of the tile), so every
    // arrival comes straight from x - d.  The lane's own tile decides (uniform
    // per wavefront); the straight gather stages the union of the windows of
    // the block's other tiles (absent tiles past the domain's edge have none).
    const int tl = (y0 / TY) * g.dtx + x0 / TX;
    const int ntb = min(NTB, g.dtx - x0 / TX);  // tiles of the block in the domain
    const int M = b.maxreach ? *b.maxreach : 0;
    const int own = lx / TX;
    DWin w = b.dwin[tl + min(own, ntb - 1)];
    if (own >= ntb) { w.lox = w.loy = 1 << 29; w.hix = w.hiy = -(1 << 29); }
    const bool near = own < ntb && b.tdist && walk_distance(g, b, tl + own, M) <= M + 1;
    int ulox = 1 << 29, uhix = -(1 << 29), uloy = 1 << 29, uhiy = -(1 << 29);
    for (int k = 0; k < ntb; k++) {
        if (b.tdist && walk_distance(g, b, tl + k, M) <= M + 1) continue;
        const DWin wk = b.dwin[tl + k];
        ulox = min(ulox, wk.lox); uhix = max(uhix, wk.hix);
        uloy = min(uloy, wk.loy); uhiy = max(uhiy, wk.hiy);
    }
    using V2 = typename Vec2<T>::type;
    const T *SCR = (const T *)b.scratch;
    double acc[NM];
#pragma unroll
    for (int k = 0; k < NM; k++) acc[k] = 0;
    int hits = 0;
    // staged region: window columns plus GU - 1 more, so that a batch that
    // runs past the window's low edge reads real entries (whose disk test
    // fails: those displacements lie outside every reaching source's box)
    const int RW = BX + (uhix - ulox) + GU - 1;
    int rows = gcap / RW - (BY - 1);                // window rows per chunk
    if (ulox <= uhix && rows >= 1) {
        for (int dy0 = uhiy; dy0 >= uloy; dy0 -= rows) {
            const int dy1 = max(uloy, dy0 - rows + 1);
            const int RH = BY + (dy0 - dy1);
            const int rx0 = x0 - uhix, ry0 = y0 - dy0;
            __syncthreads();
            if (threadIdx.x == 0) s_ref = 0;
            __syncthreads();
            int anyref = 0;
            for (int i = threadIdx.x; i < RW * RH; i += 256) {
                Resolved rs = resolve_source<D>(g, rx0 + i % RW, ry0 + i / RW);
                int meta = -1;
                if (WALLS && rs.s >= 0 && !wall_keeps(g, b, rs)) rs.s = -1;
                if (rs.s >= 0) {
                    int rn = b.desc_rn[rs.s];
                    if (rn >= 0) {
                        const long long s = rs.s;
                        int st, loc;
                        tile_of<D>(g, rs.px, rs.py, st, loc);
                        const TileInfo ti = b.tiles[st];
                        long long recsz = ti.fmt ? NM : 2;
                        s_a0[i] = ti.base + (long long)loc * recsz -
                                  ((long long)ti.oy * ti.wx + ti.ox) * TILE_N * recsz;
                        s_u[i] = make_double2(b.desc_u[s], b.desc_u[g.ns + s]);
                        meta = (rn & 0xff) | (rs.fx ? META_FX : 0) | (rs.fy ? META_FY : 0) |
                               (ti.fmt ? META_REF : 0) | (ti.wx << 11);
                        anyref |= ti.fmt;
                    }
                }
                if (meta < 0) s_u[i] = make_double2(0.0, 0.0);
                s_meta[i] = meta;
            }
            if (anyref) s_ref = 1;
            __syncthreads();
            const bool ref = s_ref != 0;
            if (!mine || near) continue;
            // the rows of the chunk that the lane's own tile window holds
            for (int dy = min(dy0, w.hiy); dy >= max(dy1, w.loy); dy--) {
                const int rowbase = (ly + (dy0 - dy)) * RW + lx + uhix;
                // sums over the row of w_f c_x^k (k <= 3) and w_g c_x^k
                // (k <= 1); c_y enters once per row
                double a0 = 0, a1 = 0, a2 = 0, a3 = 0, h0 = 0, h1 = 0;
                const double cyd = (double)dy;
                // the row's displacements that a reaching source can hit: with
                // every source velocity in [ux0, ux1] x [uy0, uy1] and radius at
                // most rmax, |dx - u_x| <= sqrt(rr^2 - dist(dy, [uy0, uy1])^2)
                // (the slack of 1e-6 covers the rounding of the disk test)
                int rlo = w.lox, rhi = w.hix;
                if (!WALLS && w.rmax >= 0) {
                    const double rrm = w.rmax + 0.5, q = 1.0 / 1024.0;
                    const double dd = fmax(0.0, fmax(w.uyl * q - cyd, cyd - w.uyh * q));
                    const double rem = rrm * rrm - dd * dd;
                    if (rem < 0.0) {
                        rlo = 1; rhi = 0;
                    } else {
                        const double wv = sqrt(rem);
                        rlo = max(rlo, (int)ceil(w.uxl * q - wv - 1e-6));
                        rhi = min(rhi, (int)floor(w.uxh * q + wv + 1e-6));
                    }
                }
                // candidates in batches of GU so that the LDS and global
                // reads of a batch are in flight together
                for (int dxb = rhi; dxb >= rlo; dxb -= GU) {
                    const int ib = rowbase - dxb;
                    const double cxb = (double)dxb;
                    const T *pp[GU];
#pragma unroll
                    for (int u = 0; u < GU; u++) {
                        const int m = s_meta[ib + u];
                        const double2 cu = s_u[ib + u];
                        // exact FP64 disk test of the source's stencil
                        double a, bb;
                        int rdx = dxb - u, rdy = dy;
                        if (WALLS) {
                            if (m & META_FX) rdx = -rdx;
                            if (m & META_FY) rdy = -rdy;
                            a = (double)rdx - cu.x;
                            bb = (double)rdy - cu.y;
                        } else {
                            a = (cxb - (double)u) - cu.x;
                            bb = cyd - cu.y;
                        }
                        const double rr = (double)(m & 0xff) + 0.5;
                        bool in;
                        {
#pragma clang fp contract(off)
                            in = a * a + bb * bb <= rr * rr;
                        }
                        in = in && m >= 0 && !(m & META_REF);
                        const T *P = SCR + s_a0[ib + u] + (long long)(rdy * (m >> 11) + rdx) * (TILE_N * 2);
                        pp[u] = in ? P : nullptr;
                        hits += in ? 1 : 0;
                    }
                    V2 wv[GU];
#pragma unroll
                    for (int u = 0; u < GU; u++) {
                        wv[u].x = 0; wv[u].y = 0;
                        if (pp[u]) wv[u] = *(const V2 *)pp[u];
                    }
                    // the batch's values are taken here, after all of its
                    // loads: otherwise the compiler moves the FP32 -> FP64
                    // conversions into each load's branch and waits for every
                    // load before issuing the next
                    if constexpr (sizeof(V2) == 8) {
#pragma unroll
                        for (int u = 0; u < GU; u++) {
                            double d = __builtin_bit_cast(double, wv[u]);
                            asm volatile("" : "+v"(d));
                            wv[u] = __builtin_bit_cast(V2, d);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < GU; u++) {
                        const double cx = cxb - (double)u, wf = (double)wv[u].x, wg = (double)wv[u].y;
                        const double cw = cx * wf, c2w = cx * cw;
                        a0 += wf; a1 += cw; a2 += c2w; a3 += cx * c2w;
                        h0 += wg; h1 += cx * wg;
                    }
                }
                if (D == 1) {
                    acc[0] += a0; acc[1] += a1; acc[2] += a2; acc[3] += a3; acc[4] += h0; acc[5] += h1;
                } else {
                    const double cy = (double)dy, cy2 = cy * cy;
                    acc[0] += a0; acc[1] += a1; acc[2] += cy * a0;
                    acc[3] += a2; acc[4] += cy * a1; acc[5] += cy2 * a0;
                    acc[6] += a3 + cy2 * a1; acc[7] += cy * a2 + cy2 * cy * a0;
                    acc[8] += h0; acc[9] += h1; acc[10] += cy * h0;
                }
                if (ref) {
                    // sources with refined stencils: pre-summed moment records
                    for (int dx = w.hix; dx >= w.lox; dx--) {
                        const int m = s_meta[rowbase - dx];
                        if (m < 0 || !(m & META_REF)) continue;
                        const double2 cu = s_u[rowbase - dx];
                        const int fx = (m & META_FX) ? 1 : 0, fy = (m & META_FY) ? 1 : 0;
                        const int rdx = fx ? -dx : dx, rdy = fy ? -dy : dy;
                        const double rr = (m & 0xff) + 0.5;
                        bool in = D == 2 ? in_disk2((double)rdx, (double)rdy, cu.x, cu.y, rr)
                                         : in_disk1((double)rdx, cu.x, rr);
                        if (!in) continue;
                        hits++;
                        const T *P = SCR + s_a0[rowbase - dx] + (long long)(rdy * (m >> 11) + rdx) * (TILE_N * NM);
                        deposit_record<T, D>(acc, P, 1, dx, dy, fx, fy);
                    }
                }
            }
        }
    } else if (!near && w.lox <= w.hix && mine) {
        // window too wide to stage: descriptors straight from global memory
        for (int dy = w.hiy; dy >= w.loy; dy--) {
            for (int dx = w.hix; dx >= w.lox; dx--) {
                Resolved rs = resolve_source<D>(g, x - dx, y - dy);
                if (rs.s < 0 || !wall_keeps(g, b, rs)) continue;
                const long long s = rs.s;
                const int rn = b.desc_rn[s];
                if (rn < 0) continue;
                const int rdx = rs.fx ? -dx : dx, rdy = rs.fy ? -dy : dy;
                const double rr = (rn & 0xffff) + 0.5;
                bool in = D == 2 ? in_disk2((double)rdx, (double)rdy, b.desc_u[s], b.desc_u[g.ns + s], rr)
                                 : in_disk1((double)rdx, b.desc_u[s], rr);
                if (!in) continue;
                int st, loc;
                tile_of<D>(g, rs.px, rs.py, st, loc);
                const TileInfo ti = b.tiles[st];
                const long long recsz = ti.fmt ? NM : 2;
                long long slot = (long long)(rdy - ti.oy) * ti.wx + (rdx - ti.ox);
                const T *P = SCR + ti.base + (slot * TILE_N + loc) * recsz;
                hits++;
                deposit_record<T, D>(acc, P, ti.fmt, dx, dy, rs.fx, rs.fy);
            }
        }
    }
    if (mine && !near) {
        long long o = (long long)(y + g.wb) * g.sxn + (x + g.wl);
#pragma unroll
        for (int k = 0; k < NM; k++) mom_out[k * g.ns + o] = acc[k];
    }
    // arrivals of the workgroup as one partial (summed by k_sum_partials)
    __shared__ unsigned long long s_hits[4];
    unsigned long long hl = (unsigned long long)hits;
    for (int off = 32; off > 0; off >>= 1) hl += __shfl_xor(hl, off);
    if ((threadIdx.x & 63) == 0) s_hits[threadIdx.x >> 6] = hl;
    __syncthreads();
    if (threadIdx.x == 0) b.gpart[(long long)br0 * nbx + blockIdx.x] = s_hits[0] + s_hits[1] + s_hits[2] + s_hits[3];
}

// Destination tiles within reach of a blocker (the ones k_gather leaves
// out): every landing displacement d with |d_x|, |d_y| <= the step's maximum
// reach M is traced back to the source it comes from (walk_back), which finds
// the straight and the reflected arrivals alike.  Same workgroup blocks as
// k_gather; wavefronts of other tiles return at once.  The walks probe the
// blockers of the cells within M + 1 of the wavefront's 16 x 4 cells (64 x 1
// in 1D): staged once as one bit per cell in the wavefront's share of the LDS
// (mapb bytes) with their summed-area table, else read from global memory.
// Walk results go to the walk cache; a step at a reach the cache already holds
// reads them instead.  Candidates go in batches of GU so that the descriptor
// loads of a batch are in flight together.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_gather_near(Geom g, double *mom_out, Buffers b, int mapb, int br0) {
    constexpr int NM = Basis<D>::NMOM;
    constexpr int TX = tile_x<D>(), TY = tile_y<D>();
    constexpr int NTB = D == 2 ? GATHER_NTB : 1;
    constexpr int BX = NTB * TX, BY = TY / NTB;
    extern __shared__ double2 g_lds[];
    // Four workgroups per gather block (the launch covers block rows from br0
    // on), one per 16 x 4 cell group (64 x 1 in 1D).  A cell's candidates are
    // a chain of dependent loads (walk entry, descriptor, tile, record), so
    // the four wavefronts of the workgroup share its 64 cells and take every
    // fourth row of displacements (every fourth batch in 1D); their sums are
    // added in wavefront order at the end.
    const int nbx = gather_blocks_x(g), nd = nbx * gather_blocks_y(g);
    const int blk = blockIdx.x >> 2, grp = blockIdx.x & 3, part = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int x0 = (blk % nbx) * BX, y0 = (br0 + blk / nbx) * BY;
    int lx, ly;
    if (D == 2) {
        lx = (grp % NTB) * TX + (l & 15);
        ly = (grp / NTB) * 4 + (l >> 4);
    } else {
        lx = grp * 64 + l;
        ly = 0;
    }
    const int x = x0 + lx, y = y0 + ly;
    const bool mine = x < g.nx && y < g.ny;
    const int tl = (y0 / TY) * g.dtx + x0 / TX;
    const int ntb = min(NTB, g.dtx - x0 / TX);
    const int own = lx / TX;
    const int M = *b.maxreach;
    // uniform per workgroup (one cell group of one tile)
    const bool near = !b.flags->err && own < ntb && walk_distance(g, b, tl + own, M) <= M + 1;
    unsigned long long *gp = b.gpart + nd + 4LL * br0 * nbx + blockIdx.x;
    if (!near) {
        if (threadIdx.x == 0) *gp = 0;
        return;
    }
    const T *SCR = (const T *)b.scratch;
    int hits = 0;
    // walk results of the tile, cached once the reach has been seen (entry of
    // displacement d at ((d_y + WCACHE_M) * WCACHE_W + d_x + WCACHE_M) * TILE_N:
    // 0xffff no source, else bits [0,6) and [6,12) the origin's offset + 32,
    // 12 / 13 the flips of x / y)
    const int slot = near && b.wcache ? b.wslot[tl + own] : -1;
    const bool use_cache = slot >= 0 && M <= WCACHE_M;
    const bool cached = use_cache && M <= *b.wbuilt;
    unsigned short *wrow =
        use_cache ? b.wcache + (size_t)slot * WCACHE_W * WCACHE_W * TILE_N + (x % TX) + (y % TY) * TX : nullptr;
    const auto wentry = [&](int dx, int dy) -> unsigned short & {
        return wrow[((dy + WCACHE_M) * WCACHE_W + dx + WCACHE_M) * TILE_N];
    };
    if (near) {
        constexpr int WX = D == 2 ? 16 : 64, WY = D == 2 ? 4 : 1;
        const int xw = x0 + (lx & ~(WX - 1)), yw = y0 + (ly & ~(WY - 1));
        const int bx0 = xw - M - 1, by0 = D == 2 ? yw - M - 1 : 0;
        const int bw = WX + 2 * M + 2, bh = D == 2 ? WY + 2 * M + 2 : 1;
        // blocker bits of the region (one 32-bit word per 32 cells of a row),
        // then their summed-area table (u16, (bh + 1) x (bw + 1)): a
        // displacement whose box between x - d and x holds no blocker has a
        // straight path, with no walk
        const int wpr = (bw + 31) >> 5, satw = bw + 1;
        const bool staged_map = !cached && 4LL * wpr * bh + 2LL * satw * (bh + 1) <= mapb;
        unsigned *bits = (unsigned *)((unsigned char *)g_lds + (size_t)(threadIdx.x >> 6) * mapb);
        unsigned short *sat = (unsigned short *)(bits + wpr * bh);
        const int lane = threadIdx.x & 63;
        const auto wave_sync = [] {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        if (staged_map) {
            for (int i = lane; i < wpr * bh; i += 64) bits[i] = 0u;
            wave_sync();
            for (int i = lane; i < bw * bh; i += 64) {
                const int cx = i % bw, cy = i / bw;
                if (blocked_wrapped<D>(g, b.solid, bx0 + cx, by0 + cy)) atomicOr(&bits[cy * wpr + (cx >> 5)], 1u << (cx & 31));
            }
            wave_sync();
            for (int j = lane; j <= bh; j += 64) {
                int run = 0;
                sat[j * satw] = 0;
                for (int i = 0; i < bw; i++) {
                    run += j > 0 ? (int)((bits[(j - 1) * wpr + (i >> 5)] >> (i & 31)) & 1u) : 0;
                    sat[j * satw + i + 1] = (unsigned short)run;
                }
            }
            wave_sync();
            for (int i = lane; i <= bw; i += 64)
                for (int j = 1; j <= bh; j++) sat[j * satw + i] = (unsigned short)(sat[j * satw + i] + sat[(j - 1) * satw + i]);
            wave_sync();
        }
        const int rx = x - bx0, ry = y - by0;    // the lane's cell in the region
        const auto box_clear = [&](int dx, int dy) {
            const int xa = rx - dx, ya = ry - dy;
            const int xl = min(rx, xa), xh = max(rx, xa) + 1, yl = min(ry, ya), yh = max(ry, ya) + 1;
            return (int)sat[yh * satw + xh] - (int)sat[yl * satw + xh] - (int)sat[yh * satw + xl] +
                       (int)sat[yl * satw + xl] == 0;
        };
        const auto blocked_lds = [&](int px, int py) {
            const int cx = px - bx0;
            return ((bits[(py - by0) * wpr + (cx >> 5)] >> (cx & 31)) & 1u) != 0;
        };
        const auto blocked_glb = [&](int px, int py) { return blocked_wrapped<D>(g, b.solid, px, py); };
        double acc[NM];
#pragma unroll
        for (int k = 0; k < NM; k++) acc[k] = 0;
        const bool fluid = mine && !(b.solid && b.solid[(long long)y * g.nx + x]);
        // a path of displacement d with max(|d_x|, |d_y|) below the cell's
        // distance to the nearest blocker stays in the box between x - d and
        // x, which holds no blocker: it comes straight from x - d
        const int clear = mine ? (int)b.cdist[(long long)y * g.nx + x] : 0;
        const bool perx = g.bc[0] == LELBM_BC_PERIODIC, pery = D == 2 && g.bc[2] == LELBM_BC_PERIODIC;
        // With the walks cached, only displacements some source of the region
        // can have are tried: a source's own displacement lies in its tile's
        // slot box, and the landing displacement has the same magnitudes.
        // (A step that fills the cache tries every |d| <= M.)
        int mx = M, my = D == 2 ? M : 0;
        if (cached) {
            int ax[2], bx[2], ay[2], by[2], cnx, cny;
            if (perx) periodic_or_clip(bx0, bx0 + bw - 1, g.nx, true, ax, bx, &cnx);
            else { ax[0] = max(bx0, -g.wl); bx[0] = min(bx0 + bw - 1, g.nx + g.wr - 1); cnx = ax[0] <= bx[0]; }
            if (D == 2 && pery) periodic_or_clip(by0, by0 + bh - 1, g.ny, true, ay, by, &cny);
            else if (D == 2) { ay[0] = max(by0, -g.wb); by[0] = min(by0 + bh - 1, g.ny + g.wt - 1); cny = ay[0] <= by[0]; }
            else { ay[0] = by[0] = 0; cny = 1; }
            int bxm = 0, bym = 0;
            for (int i = 0; i < cnx; i++)
                for (int j = 0; j < cny; j++) {
                    const int t0x = (ax[i] + g.wl) / TX, t1x = (bx[i] + g.wl) / TX;
                    const int t0y = (ay[j] + g.wb) / TY, t1y = (by[j] + g.wb) / TY;
                    const int ntl = (t1x - t0x + 1) * (t1y - t0y + 1);
                    for (int k = lane; k < ntl; k += 64) {
                        const TileInfo ti = b.tiles[(t0y + k / (t1x - t0x + 1)) * g.ntx + t0x + k % (t1x - t0x + 1)];
                        if (ti.wx <= 0) continue;          // no emitting cell
                        bxm = max(bxm, max(abs(ti.ox), abs(ti.ox + ti.wx - 1)));
                        bym = max(bym, max(abs(ti.oy), abs(ti.oy + ti.wy - 1)));
                    }
                }
            for (int off = 32; off > 0; off >>= 1) {
                bxm = max(bxm, __shfl_xor(bxm, off));
                bym = max(bym, __shfl_xor(bym, off));
            }
            mx = min(mx, bxm);
            my = min(my, bym);
        }
        const auto candidates = [&](const auto &blocked) {
            if (fluid) {
                for (int dy = my - (D == 2 ? part : 0); dy >= -my; dy -= (D == 2 ? 4 : 1)) {
                    int batch = 0;
                    for (int dxb = mx; dxb >= -mx; dxb -= GU, batch++) {
                        if (D == 1 && (batch & 3) != part) continue;
                        long long sv[GU];
                        int sg[GU], spx[GU], spy[GU];
#pragma unroll
                        for (int u = 0; u < GU; u++) {
                            const int dx = dxb - u;
                            sv[u] = -1;
                            if (dx < -mx) continue;
                            int ux, uy, fl;           // unwrapped origin, flips
                            bool ok;
                            if (cached) {
                                const unsigned e = wentry(dx, dy);
                                ok = e != 0xffffu;
                                ux = x + (int)(e & 63u) - 32;
                                uy = y + (int)((e >> 6) & 63u) - 32;
                                fl = (int)(e >> 12) & 3;
                            } else if (max(abs(dx), abs(dy)) < clear || (staged_map && box_clear(dx, dy))) {
                                ux = x - dx;
                                uy = y - dy;
                                fl = 0;
                                ok = (perx || (ux >= -g.wl && ux < g.nx + g.wr)) &&
                                     (pery || (uy >= -g.wb && uy < g.ny + g.wt));
                            } else {
                                int ox, oy, sgx, sgy;
                                ok = walk_back<D>(g, blocked, x, y, -dx, -dy, ox, oy, ux, uy, sgx, sgy);
                                fl = (sgx < 0 ? 1 : 0) | (sgy < 0 ? 2 : 0);
                            }
                            if (use_cache && !cached)
                                wentry(dx, dy) = ok ? (unsigned short)((ux - x + 32) | ((uy - y + 32) << 6) | (fl << 12))
                                                    : (unsigned short)0xffff;
                            if (ok) {
                                const int ox = perx ? wrap_coord(ux, g.nx) : ux;
                                const int oy = pery ? wrap_coord(uy, g.ny) : uy;
                                spx[u] = ox + g.wl;
                                spy[u] = oy + g.wb;
                                sv[u] = (long long)spy[u] * g.sxn + spx[u];
                                sg[u] = fl;
                            }
                        }
                        int rn[GU];
                        double ux[GU], uy[GU];
#pragma unroll
                        for (int u = 0; u < GU; u++) {
                            rn[u] = -1;
                            if (sv[u] >= 0) {
                                rn[u] = b.desc_rn[sv[u]];
                                ux[u] = b.desc_u[sv[u]];
                                uy[u] = D == 2 ? b.desc_u[g.ns + sv[u]] : 0.0;
                            }
                        }
#pragma unroll
                        for (int u = 0; u < GU; u++) {
                            if (rn[u] < 0) continue;
                            const int dx = dxb - u;
                            const int fx = sg[u] & 1, fy = sg[u] >> 1;
                            const int cx = fx ? -dx : dx, cy = fy ? -dy : dy;   // the source's own displacement
                            const double rr = (rn[u] & 0xffff) + 0.5;
                            const bool in = D == 2 ? in_disk2((double)cx, (double)cy, ux[u], uy[u], rr)
                                                   : in_disk1((double)cx, ux[u], rr);
                            if (!in) continue;
                            int st, loc;
                            tile_of<D>(g, spx[u], spy[u], st, loc);
                            const TileInfo ti = b.tiles[st];
                            const long long recsz = ti.fmt ? NM : 2;
                            const long long sl = (long long)(cy - ti.oy) * ti.wx + (cx - ti.ox);
                            const T *P = SCR + ti.base + (sl * TILE_N + loc) * recsz;
                            hits++;
                            deposit_record<T, D>(acc, P, ti.fmt, dx, dy, fx, fy);
                        }
                    }
                }
            }
        };
        if (staged_map) candidates(blocked_lds);
        else candidates(blocked_glb);
        // the four wavefronts' sums of each cell, added in wavefront order
        // (the LDS of the blocker maps is free again once all are done)
        __syncthreads();
        double *red = (double *)g_lds;
#pragma unroll
        for (int k = 0; k < NM; k++) red[(part * NM + k) * 64 + l] = acc[k];
        __syncthreads();
        if (part == 0 && mine) {
            long long o = (long long)(y + g.wb) * g.sxn + (x + g.wl);
#pragma unroll
            for (int k = 0; k < NM; k++) {
                double v = red[k * 64 + l];
                v += red[(NM + k) * 64 + l];
                v += red[(2 * NM + k) * 64 + l];
                v += red[(3 * NM + k) * 64 + l];
                mom_out[k * g.ns + o] = v;
            }
        }
    }
    __shared__ unsigned long long s_hits[4];
    unsigned long long hl = (unsigned long long)hits;
    for (int off = 32; off > 0; off >>= 1) hl += __shfl_xor(hl, off);
    if (l == 0) s_hits[part] = hl;
    __syncthreads();
    if (threadIdx.x == 0) *gp = s_hits[0] + s_hits[1] + s_hits[2] + s_hits[3];
}

// ---------------------------------------------------------------------------
// resets and conserved totals
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// No-slip walls on the y faces: the extended bounce-back of Sec. III.B.
//
// The gather drops every population whose straight path crosses such a wall
// (its mirror-image source, see wall_keeps): it is absorbed, and its moment
// fractions add to the mass and phonon imbalances Delta m, Delta g of its
// source and wall (Eq. IIIB8).  k_wall_image takes them from the source's
// records, right after the reconstruction of its band, and for each wall with
// Delta m > 0 reconstructs image populations: the same normalised
// post-collision targets (the non-equilibrium part of the cell at unchanged
// RT, Eqs. IIIB9-10) on the stencil around u_n = u - 2 u_w (Eq. IIIB11;
// u_w along x), solved like any cell (Eq. IIIB13).  They stream with -c_i;
// those whose path crosses the wall land at the mirror image of x - c_i with
// velocity (-c_x, c_y), their sum Delta m' (Eq. IIIB14), and enter scaled by
// Delta m / Delta m' (Eq. IIIB15); phonons by Delta g / Delta g'.  The store
// keeps the multipliers and factors, and k_wall_gather evaluates the image
// populations at their destinations after the step's gathers.  When no image
// population crosses the wall the source's absorbed populations are
// reflected specularly instead (the gather keeps their mirror-image source).
// A stencil that crosses both walls, a refined one that crosses a wall, a
// source farther than the store's rows from a wall it reaches, and a
// population that would land only after a second reflection fail the step
// with LELBM_EREACH.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_wall_image(Geom g, Phys ph, const double *mom, Buffers b, int step,
                                                    int tile0) {
    using BS = Basis<2>;
    constexpr int NF = BS::NF, NG = BS::NG, NMF = BS::NMF, NMG = BS::NMG, NM = BS::NMOM;
    __shared__ int s_err;
    if (threadIdx.x == 0) s_err = b.flags->err;
    __syncthreads();
    if (s_err) return;
    const int t = tile0 + blockIdx.x;
    const int l = threadIdx.x;
    const int px = (t % g.ntx) * g.tx + l % g.tx, py = (t / g.ntx) * g.ty + l / g.tx;
    if (px >= g.sxn || py >= g.syn) return;
    const int sy = py - g.wb;
    const long long s = (long long)py * g.sxn + px;
    const int WR = g.wrows;
    // the cell's entries in the stores of the two walls
    long long e[2] = {-1, -1};
    if (g.bc[2] == LELBM_BC_WALL && sy < WR) e[0] = (long long)sy * g.sxn + px;
    if (g.bc[3] == LELBM_BC_WALL && g.ny - 1 - sy < WR) e[1] = ((long long)WR + (g.ny - 1 - sy)) * g.sxn + px;
    if (e[0] >= 0) b.wflag[e[0]] = 0;
    if (e[1] >= 0) b.wflag[e[1]] = 0;
    const int rn = b.desc_rn[s];
    if (rn < 0) return;
    const int R = rn & 0xffff, Nr = rn >> 16;
    const double ux = b.desc_u[s], uy = b.desc_u[g.ns + s];
    const double rr = R + 0.5;
    const int ubx = (int)floor(ux + 0.5), uby = (int)floor(uy + 0.5);
    const int xlo = ubx - R - 1, xhi = ubx + R + 1, ylo = uby - R - 1, yhi = uby + R + 1;
    const bool lo = g.bc[2] == LELBM_BC_WALL && sy + ylo < 0;
    const bool hi = g.bc[3] == LELBM_BC_WALL && sy + yhi > g.ny - 1;
    if (!lo && !hi) return;
    // Delta m and Delta g per wall: the records of the points whose path crosses it
    const TileInfo ti = b.tiles[t];
    const T *P = (const T *)b.scratch + ti.base;
    const long long recsz = ti.fmt ? NM : 2, og = ti.fmt ? 8 : 1;
    double dm[2] = {0.0, 0.0}, dg[2] = {0.0, 0.0};
    for (int cy = ylo; cy <= yhi; cy++) {
        const int f = sy + cy < 0 ? 0 : (sy + cy > g.ny - 1 ? 1 : -1);
        if (f < 0 || g.bc[2 + f] != LELBM_BC_WALL) continue;
        int xa, xb;
        if (!row_span<2>(cy, ux, uy, rr, xlo, xhi, xa, xb)) continue;
        if (Nr > 0 || e[f] < 0) {
            flag_fail(b.flags, LELBM_EREACH, step, s);
            return;
        }
        for (int cx = xa; cx <= xb; cx++) {
            const long long slot = (long long)(cy - ti.oy) * ti.wx + (cx - ti.ox);
            dm[f] += (double)P[(slot * TILE_N + l) * recsz];
            dg[f] += (double)P[(slot * TILE_N + l) * recsz + og];
        }
    }
    if (dm[0] > 0.0 && dm[1] > 0.0) {
        flag_fail(b.flags, LELBM_EREACH, step, s);
        return;
    }
    const double rho = b.desc_rho[s], RT = b.desc_rt[s];
    double mf[NF], mg[NG], kn;
    int lim;
    collide_targets<double, 2>(g, ph, mom, s, rho, ux, uy, RT, mf, mg, kn, lim);
    const double wsf = post_mass(ph, s, rho), wsg = wsf * ph.K * RT;
    const double isc[4] = {1.0, 1.0 / sqrt(RT), 1.0 / RT, 1.0 / (RT * sqrt(RT))};
    for (int f = 0; f < 2; f++) {
        if (!(dm[f] > 0.0)) continue;
        const double unx = ux - 2.0 * ph.wall_ux[f];
        Species<NF, RegStore<NF>> sf;
        Species<NG, RegStore<NG>> sg;
        species_init<2, NF, NG>(sf, sg, RT);
        int fail = 0, fsp = -1;
        while (!fail && (sf.phase < 2 || sg.phase < 2)) {
            double Sf[NMF], Sg[NMG], lf[NF], lg[NG];
#pragma unroll
            for (int k = 0; k < NMF; k++) Sf[k] = 0.0;
#pragma unroll
            for (int k = 0; k < NMG; k++) Sg[k] = 0.0;
#pragma unroll
            for (int j = 0; j < NF; j++) lf[j] = sf.at(j);
#pragma unroll
            for (int j = 0; j < NG; j++) lg[j] = sg.at(j);
            for_each_point<2>(
                unx, uy, R, 0,
                [&](double cx, double cy, double, int, int) {
                    double m[NMF];
                    monomials<2, NMF>(cx - unx, cy - uy, m);
                    double ef = 0.0, eg = 0.0;
#pragma unroll
                    for (int j = 0; j < NF; j++) ef += lf[j] * m[j];
#pragma unroll
                    for (int j = 0; j < NG; j++) eg += lg[j] * m[j];
                    const double fv = exp(-(1.0 + ef)), gv = exp(-(1.0 + eg));
#pragma unroll
                    for (int k = 0; k < NMF; k++) Sf[k] += fv * m[k];
#pragma unroll
                    for (int k = 0; k < NMG; k++) Sg[k] += gv * m[k];
                },
                [&](int, int) {});
            if (sg.phase < 2) {
                int r = species_update<2, NG, NMG>(sg, Sg, mg, isc, ph.tol, ph.maxit);
                if (r < 0) { fail = -r; fsp = 1; }
            }
            if (sf.phase < 2 && !fail) {
                int r = species_update<2, NF, NMF>(sf, Sf, mf, isc, ph.tol, ph.maxit);
                if (r < 0) { fail = -r; fsp = 0; }
            }
        }
        if (fail) {
            flag_fail(b.flags, LELBM_EEPR, step, s, fail, fsp, fsp ? sg.res : sf.res);
            return;
        }
        // the image points that cross the wall (streamed with -c_i) and their sums
        double dmi = 0.0, dgi = 0.0;
        int reach = 0;
        bool out = false;
        for_each_point<2>(
            unx, uy, R, 0,
            [&](double cx, double cy, double, int dx, int dy) {
                const int yu = sy - dy;
                if (f == 0 ? yu >= 0 : yu <= g.ny - 1) return;
                const int ly = f == 0 ? -1 - yu : 2 * g.ny - 1 - yu;
                out = out || ly < 0 || ly > g.ny - 1;
                double m[NF];
                monomials<2, NF>(cx - unx, cy - uy, m);
                double ef = 0.0, eg = 0.0;
#pragma unroll
                for (int j = 0; j < NF; j++) ef += sf.v.lam(j) * m[j];
#pragma unroll
                for (int j = 0; j < NG; j++) eg += sg.v.lam(j) * m[j];
                dmi += wsf * exp(-(1.0 + ef));
                dgi += wsg * exp(-(1.0 + eg));
                reach = max(reach, max(abs(dx), abs(dy)));
            },
            [&](int, int) {});
        if (out) {
            flag_fail(b.flags, LELBM_EREACH, step, s);
            return;
        }
        if (dmi > 0.0 && dgi > 0.0) {
            double *rec = b.wimg + e[f] * WALL_REC;
#pragma unroll
            for (int j = 0; j < NF; j++) rec[j] = sf.v.lam(j);
#pragma unroll
            for (int j = 0; j < NG; j++) rec[NF + j] = sg.v.lam(j);
            rec[16] = unx;
            rec[17] = uy;
            rec[18] = wsf * (dm[f] / dmi);
            rec[19] = wsg * (dg[f] / dgi);
            b.wflag[e[f]] = WALL_FLAG_IMAGE | (R << 8);
            if (reach > __hip_atomic_load(b.wreach, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(b.wreach, reach);
        } else {
            // specular reflection of the absorbed points: each must land after one reflection
            for (int cy = ylo; cy <= yhi; cy++) {
                const int yu = sy + cy;
                if (f == 0 ? yu >= 0 : yu <= g.ny - 1) continue;
                int xa, xb;
                if (!row_span<2>(cy, ux, uy, rr, xlo, xhi, xa, xb)) continue;
                const int ly = f == 0 ? -1 - yu : 2 * g.ny - 1 - yu;
                if (ly < 0 || ly > g.ny - 1) {
                    flag_fail(b.flags, LELBM_EREACH, step, s);
                    return;
                }
            }
            b.wflag[e[f]] = WALL_FLAG_SPECULAR;
        }
    }
}

// Arrivals of the image populations (after the step's gathers): one thread
// per destination cell of the rows within the store's reach of a no-slip
// wall; the image source of displacement d is the cell whose image point d,
// streamed with -d and reflected by the wall, lands here: (x + d_x, d_y - y
// - 1) for the ylo wall, mirrored for yhi.
__global__ void __launch_bounds__(256) k_wall_gather(Geom g, double *mom_out, Buffers b) {
    constexpr int NF = Basis<2>::NF, NG = Basis<2>::NG, NM = Basis<2>::NMOM;
    __shared__ int s_err;
    if (threadIdx.x == 0) s_err = b.flags->err;
    __syncthreads();
    if (s_err) return;
    const int WR = g.wrows;
    const int nr = min(g.ny, 2 * WR);
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)nr * g.nx) return;
    const int x = (int)(i % g.nx), k = (int)(i / g.nx);
    const int y = (g.ny <= 2 * WR || k < WR) ? k : g.ny - 2 * WR + k;
    const int M = *b.wreach;
    const bool perx = g.bc[0] == LELBM_BC_PERIODIC;
    double acc[NM];
#pragma unroll
    for (int j = 0; j < NM; j++) acc[j] = 0.0;
    for (int f = 0; f < 2; f++) {
        if (g.bc[2 + f] != LELBM_BC_WALL) continue;
        const int yd = f == 0 ? y : g.ny - 1 - y;   // rows between the destination and the wall
        for (int r = 0; r < WR && yd + 1 + r <= M; r++) {
            const int dy = f == 0 ? yd + 1 + r : -(yd + 1 + r);
            const long long row = ((long long)f * WR + r) * g.sxn;
            for (int dx = -M; dx <= M; dx++) {
                int sx = x + dx;
                if (perx) sx = wrap_coord(sx, g.nx);
                const int pxs = sx + g.wl;
                if (pxs < 0 || pxs >= g.sxn) continue;
                const int fl = b.wflag[row + pxs];
                if ((fl & 3) != WALL_FLAG_IMAGE) continue;
                const double *rec = b.wimg + (row + pxs) * WALL_REC;
                const double unx = rec[16], uny = rec[17];
                if (!in_disk2((double)dx, (double)dy, unx, uny, (double)(fl >> 8) + 0.5)) continue;
                double m[NF];
                monomials<2, NF>((double)dx - unx, (double)dy - uny, m);
                double ef = 0.0, eg = 0.0;
#pragma unroll
                for (int j = 0; j < NF; j++) ef += rec[j] * m[j];
#pragma unroll
                for (int j = 0; j < NG; j++) eg += rec[NF + j] * m[j];
                const double wf = rec[18] * exp(-(1.0 + ef)), wg = rec[19] * exp(-(1.0 + eg));
                const double cx = -(double)dx, cy = (double)dy, cc = cx * cx + cy * cy;
                acc[0] += wf; acc[1] += cx * wf; acc[2] += cy * wf;
                acc[3] += cx * cx * wf; acc[4] += cx * cy * wf; acc[5] += cy * cy * wf;
                acc[6] += cc * cx * wf; acc[7] += cc * cy * wf;
                acc[8] += wg; acc[9] += cx * wg; acc[10] += cy * wg;
            }
        }
    }
    const long long o = (long long)(y + g.wb) * g.sxn + (x + g.wl);
#pragma unroll
    for (int j = 0; j < NM; j++) mom_out[j * g.ns + o] += acc[j];
}

__global__ void k_reset_windows(int n, DWin *w, int *maxreach, int *wreach) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        w[i].lox = 1 << 29; w[i].loy = 1 << 29; w[i].hix = -(1 << 29); w[i].hiy = -(1 << 29);
        w[i].uxl = 1 << 29; w[i].uyl = 1 << 29; w[i].uxh = -(1 << 29); w[i].uyh = -(1 << 29); w[i].rmax = -1;
    }
    if (i == 0 && maxreach) *maxreach = 0;
    if (i == 0 && wreach) *wreach = 0;
}

// Zeroes the state of solid cells (they hold no gas).
template <typename T>
__global__ void __launch_bounds__(256) k_zero_solid(Geom g, int nmom, T *mom, const unsigned char *solid) {
    const long long n = (long long)g.nx * g.ny;
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n || !solid[i]) return;
    const int y = (int)(i / g.nx), x = (int)(i - (long long)y * g.nx);
    for (int k = 0; k < nmom; k++) mom[k * g.ns + (long long)(y + g.wb) * g.sxn + x + g.wl] = (T)0;
}

// Interior copies between a contiguous SoA array [nmom][ny][nx] and the
// padded state, with precision conversion (device to device).
template <typename S, typename T>
__global__ void __launch_bounds__(256) k_load_interior(Geom g, int nmom, const S *src, T *dst) {
    const long long n = (long long)g.nx * g.ny;
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n * nmom) return;
    const long long k = i / n, r = i - k * n;
    const int y = (int)(r / g.nx), x = (int)(r - (long long)y * g.nx);
    dst[k * g.ns + (long long)(y + g.wb) * g.sxn + x + g.wl] = (T)src[i];
}

template <typename T>
__global__ void __launch_bounds__(256) k_store_interior(Geom g, int nmom, const T *src, double *dst) {
    const long long n = (long long)g.nx * g.ny;
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n * nmom) return;
    const long long k = i / n, r = i - k * n;
    const int y = (int)(r / g.nx), x = (int)(r - (long long)y * g.nx);
    dst[i] = (double)src[k * g.ns + (long long)(y + g.wb) * g.sxn + x + g.wl];
}

// Flags are cleared on the device, in stream order: no host staging memory
// has to outlive the call that enqueues the reset.
__global__ void k_reset_flags(Flags *f) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        f->err = 0; f->step = -1; f->node = LLONG_MAX; f->need = 0;
        f->detail = 0; f->species = -1; f->residual = 0.0; f->reach = 0; f->total = 0;
    }
}

__global__ void k_reset_stats(DevStats *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->it_sum_f = st->it_sum_g = st->q_sum = st->limited = st->cells = st->fallbacks = 0;
        st->qpass_sum = st->qpass_ref_sum = st->arrivals = st->wave_qpass = st->row_passes = 0;
        st->it_max_f = st->it_max_g = st->q_max = 0;
        st->q_min = 1 << 30;
        st->rt_min_bits = (unsigned long long)__double_as_longlong(1e300);
        st->kn_max_bits = 0;
        st->colat_max_bits = 0;
    }
}

// Sums the per-workgroup partials of k_epr into the step statistics: each
// workgroup folds a strided share, then adds it with one atomic per field.
__global__ void __launch_bounds__(256) k_stats_reduce(const DevStats *part, int n, DevStats *st) {
    __shared__ DevStats s_w[4];
    StatSum a;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        StatSum p;
        p.load(part[i]);
        a.add(p);
    }
    a.wave_reduce();
    if ((threadIdx.x & 63) == 0) a.store(s_w[threadIdx.x >> 6]);
    __syncthreads();
    if (threadIdx.x == 0) {
        StatSum t;
        for (int w = 0; w < 4; w++) {
            StatSum o;
            o.load(s_w[w]);
            t.add(o);
        }
        t.atomics_into(st);
    }
}

// Adds n per-workgroup counts to *out: a strided share per workgroup, one
// atomic per workgroup.
__global__ void __launch_bounds__(256) k_sum_partials(const unsigned long long *part, int n,
                                                      unsigned long long *out) {
    __shared__ unsigned long long s_w[4];
    unsigned long long a = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) a += part[i];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (t) atomicAdd(out, t);
    }
}

// Totals of mass, momentum and energy over the interior, in a fixed order:
// block partial sums, then a one-block final sum.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_sums(Geom g, const T *mom, double *partial) {
    __shared__ double sh[4][256];
    long long n = (long long)g.nx * g.ny;
    double a[4] = {0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        int x = (int)(i % g.nx), y = (int)(i / g.nx);
        long long s = (long long)(y + g.wb) * g.sxn + (x + g.wl);
        a[0] += (double)mom[s];
        a[1] += (double)mom[g.ns + s];
        if (D == 2) {
            a[2] += (double)mom[2 * g.ns + s];
            a[3] += (double)mom[3 * g.ns + s] + (double)mom[5 * g.ns + s] + (double)mom[8 * g.ns + s];
        } else {
            a[3] += (double)mom[2 * g.ns + s] + (double)mom[4 * g.ns + s];
        }
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

__global__ void k_sums_final(int nb, double *partial) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a[4] = {0, 0, 0, 0};
        for (int i = 0; i < nb; i++)
            for (int k = 0; k < 4; k++) a[k] += partial[i * 4 + k];
        for (int k = 0; k < 4; k++) partial[nb * 4 + k] = a[k];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int num_sum_blocks(const Geom &g) {
    long long n = (long long)g.nx * g.ny;
    long long nb = (n + 255) / 256;
    return (int)(nb < 1024 ? nb : 1024);
}

// The state (moments, SoA over the padded domain) is FP64 in both
// precision modes; only the population records of the mixed mode are FP32.
hipError_t launch_fill_pads(const Geom &g, const Phys &ph, double *mom, Flags *fl, hipStream_t s) {
    if (g.wl + g.wr + g.wb + g.wt == 0) return hipSuccess;
    unsigned nb = (unsigned)((g.ns + 255) / 256);
    if (g.dim == 1) hipLaunchKernelGGL((k_fill_pads<double, 1>), dim3(nb), dim3(256), 0, s, g, ph, mom, fl);
    else hipLaunchKernelGGL((k_fill_pads<double, 2>), dim3(nb), dim3(256), 0, s, g, ph, mom, fl);
    return hipGetLastError();
}

hipError_t launch_reset_step(const Geom &g, Buffers &b, hipStream_t s) {
    int n = g.dtx * g.dty;
    hipLaunchKernelGGL(k_reset_windows, dim3((n + 255) / 256), dim3(256), 0, s, n, b.dwin, b.maxreach, b.wreach);
    return hipGetLastError();
}

hipError_t launch_load_interior(const Geom &g, int nmom, const void *src, int src_fp32, double *dst, hipStream_t s) {
    const long long tot = (long long)g.nx * g.ny * nmom;
    if (tot == 0) return hipSuccess;
    dim3 grid((unsigned)((tot + 255) / 256));
    if (src_fp32)
        hipLaunchKernelGGL((k_load_interior<float, double>), grid, dim3(256), 0, s, g, nmom, (const float *)src, dst);
    else
        hipLaunchKernelGGL((k_load_interior<double, double>), grid, dim3(256), 0, s, g, nmom, (const double *)src, dst);
    return hipGetLastError();
}

hipError_t launch_store_interior(const Geom &g, int nmom, const double *src, double *dst, hipStream_t s) {
    const long long tot = (long long)g.nx * g.ny * nmom;
    if (tot == 0) return hipSuccess;
    dim3 grid((unsigned)((tot + 255) / 256));
    hipLaunchKernelGGL((k_store_interior<double>), grid, dim3(256), 0, s, g, nmom, src, dst);
    return hipGetLastError();
}

hipError_t launch_zero_solid(const Geom &g, int nmom, double *mom, const unsigned char *solid, hipStream_t s) {
    const long long n = (long long)g.nx * g.ny;
    if (!solid || n == 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL((k_zero_solid<double>), grid, dim3(256), 0, s, g, nmom, mom, solid);
    return hipGetLastError();
}

hipError_t launch_reset_flags(Flags *f, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_flags, dim3(1), dim3(64), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_reset_stats(Buffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, s, b.stats);
    return hipGetLastError();
}

hipError_t launch_prepare(const Geom &g, const Phys &ph, const double *mom, Buffers &b, int step, hipStream_t s) {
    unsigned nt = (unsigned)(g.ntx * g.nty);
    if (g.dim == 1) hipLaunchKernelGGL((k_prepare<double, 1>), dim3(nt), dim3(256), 0, s, g, ph, mom, b, step);
    else hipLaunchKernelGGL((k_prepare<double, 2>), dim3(nt), dim3(256), 0, s, g, ph, mom, b, step);
    return hipGetLastError();
}

hipError_t launch_scan(const Geom &g, Buffers &b, int nbands, long long slot_cap, int m_plan, int step,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, g.ntx, nbands, (const BandInfo *)b.bands, b.tiles, b.flags,
                       slot_cap, step, b.order, b.rlist, b.rcount, (const int *)b.maxreach, m_plan);
    return hipGetLastError();
}

// variant 0: cells with narrow stencils, 1: refined stencils (of band
// `band`: a grid of at most EPR_REF_GRID workgroups over its list), 2: wide
template <typename T, int D>
static void epr_launch(const Geom &g, const Phys &ph, const double *mom, Buffers &b, int step, int variant,
                       int tile0, int ntiles, int band, hipStream_t s) {
    const dim3 grid((unsigned)ntiles), blk(256);
    if (variant == 1)
        hipLaunchKernelGGL((k_epr_ref<T, D>), dim3((unsigned)std::min(ntiles, EPR_REF_GRID)), blk, 0, s, g, ph, mom, b,
                           step, tile0, band);
    else if (variant == 2)
        hipLaunchKernelGGL((k_epr<T, D, true>), grid, blk, 0, s, g, ph, mom, b, step, tile0);
    else
        hipLaunchKernelGGL((k_epr<T, D, false>), grid, blk, 0, s, g, ph, mom, b, step, tile0);
}

static void epr_dispatch(const Geom &g, const Phys &ph, int mixed, const double *mom, Buffers &b, int step,
                         int variant, int tile0, int ntiles, int band, hipStream_t s) {
    if (ntiles <= 0) return;
    if (mixed) {
        if (g.dim == 1) epr_launch<float, 1>(g, ph, mom, b, step, variant, tile0, ntiles, band, s);
        else epr_launch<float, 2>(g, ph, mom, b, step, variant, tile0, ntiles, band, s);
    } else {
        if (g.dim == 1) epr_launch<double, 1>(g, ph, mom, b, step, variant, tile0, ntiles, band, s);
        else epr_launch<double, 2>(g, ph, mom, b, step, variant, tile0, ntiles, band, s);
    }
}

hipError_t launch_epr(const Geom &g, const Phys &ph, int mixed, const double *mom, Buffers &b, int step, int tile0,
                      int ntiles, int wide, hipStream_t s) {
    epr_dispatch(g, ph, mixed, mom, b, step, wide ? 2 : 0, tile0, ntiles, 0, s);
    return hipGetLastError();
}

hipError_t launch_epr_ref(const Geom &g, const Phys &ph, int mixed, const double *mom, Buffers &b, int step,
                          int tile0, int ntiles, int band, hipStream_t s) {
    epr_dispatch(g, ph, mixed, mom, b, step, 1, tile0, ntiles, band, s);
    return hipGetLastError();
}

hipError_t launch_wall_image(const Geom &g, const Phys &ph, int mixed, const double *mom, Buffers &b, int step,
                             int tile0, int ntiles, hipStream_t s) {
    if (!b.wflag || ntiles <= 0) return hipSuccess;
    if (mixed)
        hipLaunchKernelGGL((k_wall_image<float>), dim3((unsigned)ntiles), dim3(256), 0, s, g, ph, mom, b, step, tile0);
    else
        hipLaunchKernelGGL((k_wall_image<double>), dim3((unsigned)ntiles), dim3(256), 0, s, g, ph, mom, b, step, tile0);
    return hipGetLastError();
}

hipError_t launch_wall_gather(const Geom &g, double *mom_out, Buffers &b, hipStream_t s) {
    if (!b.wflag) return hipSuccess;
    const long long n = (long long)std::min(g.ny, 2 * g.wrows) * g.nx;
    hipLaunchKernelGGL(k_wall_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, mom_out, b);
    return hipGetLastError();
}

// After the backward-walk gather: a step that filled the walk cache (at a
// reach above the one it held) makes that reach available to later steps.
__global__ void k_mark_built(const Flags *fl, const int *maxreach, int *wbuilt) {
    const int M = *maxreach;
    if (!fl->err && M <= WCACHE_M && M > *wbuilt) *wbuilt = M;
}

template <typename T, int D>
static void gather_launch(const Geom &g, double *mom_out, Buffers &b, int gcap, int br0, int nbr, hipStream_t s) {
    const unsigned nt = (unsigned)(gather_blocks_x(g) * nbr);
    const size_t lds = (size_t)gcap * G_ENTRY_BYTES;
    bool walls = false;
    for (int f = 0; f < 2 * D; f++) walls = walls || mirror_face(g, f);
    if (walls)
        hipLaunchKernelGGL((k_gather<T, D, true>), dim3(nt), dim3(256), lds, s, g, mom_out, b, gcap, br0, nbr);
    else
        hipLaunchKernelGGL((k_gather<T, D, false>), dim3(nt), dim3(256), lds, s, g, mom_out, b, gcap, br0, nbr);
    if (b.tdist) {
        // 8 KB of LDS per wavefront for its blocker bits and summed-area table
        // (five workgroups per CU)
        const size_t lds_near = 32768;
        hipLaunchKernelGGL((k_gather_near<T, D>), dim3(4 * nt), dim3(256), lds_near, s, g, mom_out, b,
                           (int)(lds_near / 4), br0);
    }
}

hipError_t launch_gather(const Geom &g, int mixed, double *mom_out, Buffers &b, int gcap, int br0, int nbr,
                         hipStream_t s) {
    if (nbr <= 0) return hipSuccess;
    if (mixed) {
        if (g.dim == 1) gather_launch<float, 1>(g, mom_out, b, gcap, br0, nbr, s);
        else gather_launch<float, 2>(g, mom_out, b, gcap, br0, nbr, s);
    } else {
        if (g.dim == 1) gather_launch<double, 1>(g, mom_out, b, gcap, br0, nbr, s);
        else gather_launch<double, 2>(g, mom_out, b, gcap, br0, nbr, s);
    }
    return hipGetLastError();
}

hipError_t launch_step_totals(const Geom &g, Buffers &b, hipStream_t s) {
    // partials of both k_epr variants
    const int nt = 2 * g.ntx * g.nty;
    const int nb = (nt + 255) / 256 < 256 ? (nt + 255) / 256 : 256;
    hipLaunchKernelGGL(k_stats_reduce, dim3(nb), dim3(256), 0, s, (const DevStats *)b.bpart, nt, b.stats);
    // arrival partials of k_gather, then of k_gather_near (four per block,
    // when it runs)
    const int nd = gather_blocks_x(g) * gather_blocks_y(g) * (b.tdist ? 5 : 1);
    const int nb2 = (nd + 255) / 256 < 256 ? (nd + 255) / 256 : 256;
    hipLaunchKernelGGL(k_sum_partials, dim3(nb2), dim3(256), 0, s, (const unsigned long long *)b.gpart, nd,
                       &b.stats->arrivals);
    if (b.wcache) hipLaunchKernelGGL(k_mark_built, dim3(1), dim3(1), 0, s, b.flags, b.maxreach, b.wbuilt);
    return hipGetLastError();
}

hipError_t launch_sums(const Geom &g, const double *mom, Buffers &b, hipStream_t s) {
    int nb = num_sum_blocks(g);
    if (g.dim == 1) hipLaunchKernelGGL((k_sums<double, 1>), dim3(nb), dim3(256), 0, s, g, mom, b.partial);
    else hipLaunchKernelGGL((k_sums<double, 2>), dim3(nb), dim3(256), 0, s, g, mom, b.partial);
    hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(64), 0, s, nb, b.partial);
    return hipGetLastError();
}

}  // namespace lelbm
