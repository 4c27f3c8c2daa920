// Internal declarations shared by the host runtime and the kernels of the
// LELBM library.  Not part of the public ABI (see include/lelbm.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lelbm.h"
#include "lelbm_plan.h"

namespace lelbm {

// Source cells are processed in tiles of TILE_N cells: 16 x 16 in 2D and
// 256 x 1 in 1D.  One workgroup handles one tile in every per-cell kernel.
constexpr int TILE_N = 256;
constexpr int WCACHE_M = 31;              // largest reach whose walks are cached
constexpr int EPR_ORDER_MAX_TILES = 32768; // above: k_epr takes the tiles in index order
constexpr int EPR_REF_GRID = 512;          // workgroups of a k_epr_ref launch (two per CU)
constexpr int WCACHE_W = 2 * WCACHE_M + 1;
template <int D> constexpr int tile_x() { return D == 2 ? 16 : 256; }
template <int D> constexpr int tile_y() { return D == 2 ? 16 : 1; }
constexpr int MAX_REFINE = 3;       // supported stencil refinement levels
constexpr int MAX_RADIUS = 128;     // largest acoustic radius (RT up to ~1000)
constexpr double MAX_SPEED = 2048.0;  // largest |u| component in cells per step
// Stencil row spans cached per cell for the reconstruction passes: row k
// (c_y = round(u_y) - R - 1 + k) holds (xa - x0) | (xb - x0) << 8 with
// x0 = round(u_x) - R - 1; 0x00ff = empty.  Cells with more rows (R > 30)
// recompute their spans in every pass.
constexpr int SPAN_ROWS = 64;
// The reconstruction's product recurrences (along a stencil row, and down
// the column of row starts) accumulate rounding as the cube of their length;
// stencils with longer rows (R >= 15) are reconstructed by a variant of the
// kernel that restarts them from exact exponentials every REC_SEG points and
// rows, which keeps the populations of the widest stencils within ~1e-13
// (without restarts, a radius of 33 stalls Newton at a residual of ~2e-12).
constexpr int REC_SEG = 32;
// staged sources per gather chunk (28 B of LDS each)
constexpr int GATHER_CAP = 1024;
constexpr int GATHER_CAP_MAX = 2340;      // 64 KiB of LDS
// Newton stopping tolerance of the mixed path: the polishing update after the
// stop squares the residual (quadratic convergence), landing near 1e-8, the
// rounding level of the path's FP32 records and state
constexpr double MIXED_TOL_FLOOR = 1e-4;
// A Newton solve whose scaled residual is below this and did not decrease at
// the last update has reached the rounding floor of its sums (large, badly
// conditioned stencils stall just above 1e-12) and is taken as converged.
constexpr double STALL_RES = 1e-10;

// Warm-start network: 16 inputs, two hidden layers of 64, 16 outputs.
// Canonical FP32 parameter vector: W1[16][64], b1[64], W2[64][64], b2[64],
// W3[64][16], b3[16] (row-major [in][out]).
constexpr int MLP_IN = 16, MLP_H = 64, MLP_OUT = 16;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 1024, MLP_OFF_W2 = 1088, MLP_OFF_B2 = 5184, MLP_OFF_W3 = 5248,
              MLP_OFF_B3 = 6272, MLP_NPARAM = 6288;
constexpr int MLP_NORM = 64;   // standardisation constants (input/output mean and scale)

struct Geom {
    int dim, nx, ny;
    int wl, wr, wb, wt;       // pad widths on xlo, xhi, ylo, yhi
    int sxn, syn;             // padded (source) domain extent
    long long ns;             // sxn * syn
    int bc[4];
    int tx, ty;               // tile extent (16,16) or (256,1)
    int ntx, nty;             // source tiles over the padded domain
    int dtx, dty;             // destination tiles over the interior
    int wrows;                // no-slip walls: rows of each face's image store (0: no such wall)
};

// Gather workgroups: in 2D one per strip of GATHER_NTB x-neighbour
// destination tiles, 16 / GATHER_NTB cells high; in 1D one per tile.
constexpr int GATHER_NTB = 2;
__host__ __device__ inline int gather_blocks_x(const Geom &g) {
    return g.dim == 2 ? (g.dtx + GATHER_NTB - 1) / GATHER_NTB : g.dtx;
}
__host__ __device__ inline int gather_blocks_y(const Geom &g) { return g.dim == 2 ? GATHER_NTB * g.dty : g.dty; }

struct Phys {
    double K, omega_f, omega_b, omega_h;
    double n_conf;
    int r_min;
    double tol;
    int maxit;
    int kn_limiter;
    double kn_lo, kn_hi, omega_H;
    double kn_lo_lin, kn_hi_lin;  // 10^kn_lo, 10^kn_hi
    double in_rho, in_u[2], in_RT;
    int lin_guess;                  // 1: start Newton from the linearised guess (lin_guess_scaled)
    int prev_guess;                 // 1: linearised guess plus the cell's previous-step correction
    long long src_node;             // padded index of the mass-source cell, -1: none
    double src_mass;                // mass the source adds in the current step
    double wall_ux[2];              // x velocity of the no-slip walls of the ylo / yhi faces
};

// Image store of the no-slip walls (Sec. III.B), per wall face f, per row r
// < Geom::wrows counted from the face, per padded column: entry
// (f * wrows + r) * sxn + px.  wflag: 0 nothing, 1 image populations
// (bits 8 and up: their radius R), 2 the absorbed populations are reflected
// specularly; wimg: WALL_REC doubles per entry, the image species'
// multipliers (fluon 10, phonon 6), u_n (2) and the factors turning the
// normalised image populations into moment fractions (fluon, phonon).
constexpr int WALL_REC = 20;
constexpr int WALL_FLAG_IMAGE = 1, WALL_FLAG_SPECULAR = 2;

// Zeroth post-collision moment of cell s: rho, plus the mass of a point
// source (Sec. IV.C, Eq. VC8) in its cell.
__host__ __device__ inline double post_mass(const Phys &ph, long long s, double rho) {
    return s == ph.src_node ? rho + ph.src_mass : rho;
}

struct Flags {
    int err;                 // 0 or first error code
    int step;                // step index of the failure
    long long node;          // smallest failing cell index of that kernel
    long long need;          // scratch elements needed (ERR_OVERFLOW)
    int detail;              // reason of an LELBM_EEPR failure (see lelbm_last_failure_detail)
    int species;             // 0 fluon, 1 phonon
    double residual;         // last scaled moment residual of the failing solve
    int reach;               // the step's largest reach (with ERR_OVERFLOW, ERR_REPLAN)
    long long total;         // elements of all bands' records (with ERR_OVERFLOW)
};

struct DevStats {
    unsigned long long it_sum_f, it_sum_g, q_sum, limited, cells, fallbacks, qpass_sum, arrivals, qpass_ref_sum;
    unsigned long long wave_qpass;   // sum over wavefronts of 64 x the wavefront's largest q x passes
    unsigned long long row_passes;   // sum over cells of stencil rows x passes (unrefined stencils)
    int it_max_f, it_max_g, q_max, q_min;
    unsigned long long rt_min_bits, kn_max_bits, colat_max_bits;
};

// Per-source-tile layout of the population scratch.
struct TileInfo {
    int ox, oy;              // displacement of slot (0, 0)
    int wx, wy;              // slot box extent
    int fmt;                 // 0: (w_f, w_g) per slot; 1: all moments per slot
    int wide;                // 1: holds cells with wide stencils (unrefined, 2R + 3 > REC_SEG)
    long long size;          // elements used by the tile
    long long base;          // first element of the tile
};

// Per-destination-tile window of displacements to scan in the gather.
struct DWin {
    int lox, loy, hix, hiy;
    // bounds of the velocities (in 1/1024 cells, rounded outwards) and the
    // largest radius of the sources that can reach the tile: the gather
    // narrows each window row to the displacements such sources can hit
    // (periodic and open faces only)
    int uxl, uxh, uyl, uyh, rmax;
};

struct Buffers {
    double *mom[2];          // state (padded domain), FP64 in both modes, SoA [nmom][ns]
    double *desc_u;          // [2][ns]  cell velocity
    double *desc_rho;        // [ns]
    double *desc_rt;         // [ns]
    int *desc_rn;            // [ns]  R | (N_r << 16), -1 = no emission
    unsigned short *spans;   // [SPAN_ROWS][tiles * 256] stencil row spans by source tile and cell of the
                             // tile, so a wavefront reads one row of its 64 cells in one line (k_epr)
    TileInfo *tiles;         // [ntx*nty]
    DWin *dwin;              // [dtx*dty]
    void *scratch;           // population scratch (the bands' slots)
    long long scratch_cap;   // elements
    Flags *flags;
    DevStats *stats;
    double *partial;         // block partial sums for conserved totals
    // learned Newton guess
    const unsigned short *mlp_w;   // BF16 weights (canonical order), NULL = none
    const float *mlp_p;            // FP32 parameters (biases read from here)
    const float *mlp_n;            // standardisation constants (64)
    DevStats *bpart;               // [2][ntx*nty] per-workgroup statistics of k_epr (narrow, wide stencils)
    int *order;                    // [ntx*nty] source tiles in the order k_epr takes them (k_scan)
    int *rlist;                    // [ntx*nty] per band from its first tile on: its tiles with refined cells
    int *rcount;                   // [nty] per band: how many (k_scan)
    unsigned long long *gpart;     // arrival counts per workgroup: [dtx*dty] of k_gather, then 4 per block of k_gather_near
    double *lamprev;               // [16][ns] scaled correction beyond the linearised guess, last step
                                   // (NaN in row 0: none); allocated for LELBM_GUESS_PREV only
    // harvesting of (features, converged multipliers) pairs
    float *harvest;                // [cap][32], NULL = off
    long long harvest_cap;
    int harvest_stride;
    unsigned long long *harvest_n; // pairs written (device counter)
    // blockers: solid cells and slip walls
    const unsigned char *solid;    // [ny][nx] 1 = solid cell, NULL = none
    const int *tdist;              // [dtx*dty] Chebyshev distance from the tile to the nearest
                                   // blocker (solid cell or the cell beyond a slip wall); NULL = none
    int *maxreach;                 // max over sources of max(|round(u)|) + R + 1 (this step)
    BandInfo *bands;               // [nty] the band plan of the population scratch
    const unsigned short *cdist;   // [ny][nx] the same distance per cell (capped at 65535)
    const int *tdist_s;            // [dtx*dty] Chebyshev distance from the tile to the nearest solid cell
    // backward-walk results (the geometry is fixed, so a walk's result never
    // changes): per cached destination tile, per displacement |d| <= WCACHE_M,
    // per cell, the origin's offset and the path's flips
    unsigned short *wcache;        // [slots][WCACHE_W^2][TILE_N], NULL = not cached
    const int *wslot;              // [dtx*dty] cache slot of a destination tile, -1 = none
    int *wbuilt;                   // largest reach the cache holds every near tile's walks for, -1 = none
    // no-slip walls (NULL without them): the image store and the largest
    // displacement of an image population that enters the domain (this step)
    int *wflag;
    double *wimg;
    int *wreach;
};

// Kernel launchers (defined in lelbm_kernels.hip).  All enqueue on `s`.
hipError_t launch_fill_pads(const Geom &g, const Phys &ph, double *mom, Flags *fl, hipStream_t s);
hipError_t launch_prepare(const Geom &g, const Phys &ph, const double *mom, Buffers &b, int step, hipStream_t s);
hipError_t launch_scan(const Geom &g, Buffers &b, int nbands, long long slot_cap, int m_plan, int step,
                       hipStream_t s);
// reconstruction of the tiles [tile0, tile0 + ntiles) of the scan's order:
// the cells with narrow stencils, or (wide != 0) those with wide ones
hipError_t launch_epr(const Geom &g, const Phys &ph, int mixed, const double *mom, Buffers &b, int step, int tile0,
                      int ntiles, int wide, hipStream_t s);
// reconstruction of the refined-stencil tiles of band `band` (tiles
// [tile0, tile0 + ntiles))
hipError_t launch_epr_ref(const Geom &g, const Phys &ph, int mixed, const double *mom, Buffers &b, int step,
                          int tile0, int ntiles, int band, hipStream_t s);
// gather of the destination block rows [br0, br0 + nbr)
hipError_t launch_gather(const Geom &g, int mixed, double *mom_out, Buffers &b, int gcap, int br0, int nbr,
                         hipStream_t s);
// no-slip walls: image populations of the sources of band tiles [tile0,
// tile0 + ntiles) (after their reconstruction, before the gathers that read
// them), and their arrivals (after the step's last gather)
hipError_t launch_wall_image(const Geom &g, const Phys &ph, int mixed, const double *mom, Buffers &b, int step,
                             int tile0, int ntiles, hipStream_t s);
hipError_t launch_wall_gather(const Geom &g, double *mom_out, Buffers &b, hipStream_t s);
// statistics and arrival counts of a step (after its last gather)
hipError_t launch_step_totals(const Geom &g, Buffers &b, hipStream_t s);
hipError_t launch_sums(const Geom &g, const double *mom, Buffers &b, hipStream_t s);
hipError_t launch_reset_step(const Geom &g, Buffers &b, hipStream_t s);
hipError_t launch_reset_stats(Buffers &b, hipStream_t s);
hipError_t launch_reset_flags(Flags *f, hipStream_t s);
hipError_t launch_zero_solid(const Geom &g, int nmom, double *mom, const unsigned char *solid, hipStream_t s);
hipError_t launch_load_interior(const Geom &g, int nmom, const void *src, int src_fp32, double *dst, hipStream_t s);
hipError_t launch_store_interior(const Geom &g, int nmom, const double *src, double *dst, hipStream_t s);
int num_sum_blocks(const Geom &g);
hipError_t launch_mlp_fwdbwd(const unsigned short *Wb, const float *bias, const float *nm, const float *pairs,
                             long long n, long long nsamp, int draw, unsigned long long seed, unsigned long long step,
                             float *partial, float *lossp, hipStream_t s);
hipError_t launch_mlp_norm_fit(const float *pairs, long long n, float *nm, hipStream_t s);
hipError_t launch_mlp_adam(const float *partial, int nparts, float *params, float *m1, float *m2, unsigned short *Wb,
                           float lr, int t, int apply, float *grad_out, hipStream_t s);
hipError_t launch_mlp_to_bf16(const float *params, unsigned short *Wb, hipStream_t s);
hipError_t launch_mlp_forward(const unsigned short *Wb, const float *bias, const float *nm, const float *x,
                              long long xstride, long long n, float *y, hipStream_t s);

}  // namespace lelbm
