/*
 * lelbm.h -- C ABI of the MI355X (gfx950) LELBM time step.
 *
 * The library advances the per-cell raw moments {M, G} of the Lagrangian
 * entropic lattice Boltzmann method (arXiv 2508.06911) by whole time steps on
 * one GPU.  One step is the paper's single-cell operation (Sec. II.F, Fig. of
 * the modular flowchart) applied to every cell, followed by moment streaming:
 *
 *   collision      Sec. II.B, Eqs. (IIB6-IIB18), Knudsen limiter of App. D
 *   stencil (LAS)  Sec. II.C, Eqs. (IIC6, IIC9-IIC11)
 *   EPR            Sec. II.D, Eqs. (IID7-IID13)
 *   streaming (MS) Sec. II.E, Eqs. (IIE3a-b); only moments are stored
 *   fluid BCs      Sec. III.A; slip walls by specular path reflection, Sec. III.B
 *
 * Units are lattice units (dV = dx = dt = 1).  Moment order per cell:
 *   2D (11): M0 Mx My Mxx Mxy Myy MDx MDy G0 Gx Gy
 *   1D  (6): M0 Mx Mxx Mxxx G0 Gx
 * Host and device moment arrays are SoA [moment][y][x] over the nx*ny interior
 * cells, FP64 unless stated otherwise.
 *
 * Conventions
 *   - Every call returns an int status (LELBM_OK = 0 or a negative code);
 *     lelbm_strerror() names it.
 *   - The library copies every input; a context owns all device memory it
 *     allocates; the caller owns every output buffer.
 *   - All GPU work of a context is issued on the HIP stream given at creation
 *     (NULL = the default stream).  Calls that return host data synchronise
 *     that stream.
 *   - Contexts share no global state; one context must not be used from two
 *     threads at once.
 *   - lelbm_step is transactional: if a step fails, the context keeps the state
 *     of the last completed step and lelbm_last_failure() names the cell and
 *     the step.
 */
#ifndef LELBM_H
#define LELBM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lelbm_ctx lelbm_ctx;

enum {
    LELBM_OK = 0,
    LELBM_EINVAL = -1,      /* invalid argument or parameter combination */
    LELBM_ENOMEM = -2,      /* device or host allocation failed */
    LELBM_EDEVICE = -3,     /* HIP runtime error */
    LELBM_EEPR = -4,        /* non-realizable cell state (rho <= 0, RT <= 0),
                               Newton iteration cap, Cholesky breakdown or line
                               search exhausted in the entropic reconstruction */
    LELBM_ENONFINITE = -5,  /* non-finite moments */
    LELBM_EREACH = -6       /* a pad is narrower than the reach of its
                               cells' stencils toward the interior
                               ([u_n] + R > pad width, u_n the velocity
                               component toward the interior; Sec. III), or
                               a cell is outside the supported stencil
                               range: more than 3 refinement levels
                               (RT < 0.0123), acoustic radius above 128
                               (RT > ~1030) or |u| above 2048 cells per
                               step, or a stencil reaches a no-slip wall
                               beyond what LELBM_BC_WALL supports */
};

/* LELBM_BC_WALL: a no-slip (optionally moving) adiabatic wall on a y face of
 * a 2D domain, by the extended bounce-back of Sec. III.B (Eqs. IIIB8-15):
 * populations whose straight path crosses the wall are absorbed; each source
 * cell that lost mass Delta m to the wall reconstructs image populations with
 * its own normalised post-collision targets around u_n = u - 2 u_w
 * (Eq. IIIB11), streams them with -c_i, and those whose path crosses the
 * wall enter the domain after a specular reflection, scaled by
 * Delta m / Delta m' (their own sum; phonons by their own ratio).  When no
 * image population crosses the wall (flow toward it faster than the image
 * stencil reaches back) the absorbed populations are reflected specularly
 * instead.  Requires: both walls' faces on y, x faces periodic, outflow or
 * inflow, no slip walls and no solid cells; a stencil may cross one wall
 * only, unrefined (RT >= 4/9), from at most LELBM_WALL_ROWS rows away, and
 * every image or reflected population must land after one reflection;
 * otherwise lelbm_step fails with LELBM_EREACH. */
enum { LELBM_BC_PERIODIC = 0, LELBM_BC_OUTFLOW = 1, LELBM_BC_INFLOW = 2, LELBM_BC_SLIPWALL = 3, LELBM_BC_WALL = 4 };
#define LELBM_WALL_ROWS 64

/* LELBM_FP64: every stage in FP64.
 * LELBM_MIXED: the reconstruction records (population multipliers and moment
 * fractions, the bulk of the HBM traffic) in FP32; the stored moments, the
 * gather's sums, collision, per-point reconstruction arithmetic, Hessian
 * solves and the final conserved-moment correction in FP64.  Newton stops at
 * a scaled residual of max(newton_tol, 1e-4); the polishing update that
 * follows squares it (quadratic convergence) to about 1e-8, the rounding level
 * of the FP32 records.  Keeping the state in FP64 keeps the per-step rounding
 * of large raw moments (the energy moment grows with |u|^2) from adding up
 * over long runs. */
enum { LELBM_FP64 = 0, LELBM_MIXED = 1 };

/* Newton initial guess.  EQ: Eq. (IID13), the equilibrium multipliers.
 * LIN: Eq. (IID13) plus one Newton step taken in closed form with the
 * moments of the continuous Maxwellian (the linear response of the
 * multipliers to the non-equilibrium targets); it coincides with the first
 * discrete Newton step up to the stencil's quadrature error.  MLP: LIN plus
 * the correction predicted by the learned network (lelbm_set_mlp).  With
 * PREV: LIN plus the cell's own correction beyond LIN from the previous
 * step (the warm start from stored multipliers the paper suggests in
 * Sec. II.D).  The correction is kept in scaled units, so it carries over
 * when the temperature changes; at omega = 2 the non-equilibrium part of the
 * targets flips sign every step, and LIN, not the stored correction, follows
 * that flip.  The context keeps 16 doubles per cell for it; the first step,
 * and cells whose previous step used refined stencils, start from LIN.
 * With MLP_PREV (2D): PREV plus the learned network's correction of it, in
 * the cells that have a stored correction (the others start from LIN); the
 * network is then one trained on pairs harvested in PREV mode (lelbm_harvest).
 * With LIN, MLP, PREV and MLP_PREV a cell whose first Newton update does not lower
 * the residual, or whose first evaluation is not finite, restarts from
 * Eq. (IID13); in 2D so does one whose solve fails (Cholesky breakdown, line
 * search exhausted, iteration cap), while in 3D such a failure fails the
 * step with LELBM_EEPR (state unchanged; run it again with LELBM_GUESS_EQ).
 * The converged result is the same in all modes (the multipliers are
 * unique). */
enum { LELBM_GUESS_EQ = 0, LELBM_GUESS_MLP = 1, LELBM_GUESS_LIN = 2, LELBM_GUESS_PREV = 3, LELBM_GUESS_MLP_PREV = 4 };

typedef struct {
    int dim, nx, ny;                  /* dim = 1 requires ny = 1 */
    double K;                         /* internal DoF: gamma = (D+K+2)/(D+K), App. B Eqs. (B22a-b); K > 0 */
    double omega_f, omega_b, omega_h; /* shear, bulk, heat-flux collision frequencies, Eq. (IIB16);
                                         omega = 1/(tau/dt + 1/2), App. C Eq. (C7) */
    double n_conf;                    /* conformation number n of Eq. (IIC6) (paper: 4) */
    int r_min;                        /* minimum acoustic radius of Eq. (IIC6) (paper: 2) */
    double newton_tol;                /* scaled moment residual ending Newton (paper: 1e-12) */
    int newton_max_it;                /* iteration cap, e.g. 50 */
    int kn_limiter;                   /* 1: Knudsen limiter of App. D, Eqs. (D2-D3) */
    double kn_lo, kn_hi, omega_H;     /* log10 Kn thresholds and target frequency (paper: -2, -1, 1) */
    int precision;                    /* LELBM_FP64 | LELBM_MIXED */
    int guess;                        /* LELBM_GUESS_EQ | _MLP | _LIN | _PREV | _MLP_PREV */
    int bc[4];                        /* faces xlo, xhi, ylo, yhi: LELBM_BC_*; periodic faces pair up */
    int pad;                          /* pad width W of outflow/inflow faces (Sec. III, Fig. 5) */
    double in_rho, in_u[2], in_RT;    /* inflow (Dirichlet) state of LELBM_BC_INFLOW faces */
    const unsigned char *solid;       /* 2D only: nx*ny legoland mask [ny][nx], nonzero = solid cell, or
                                         NULL; copied at create.  Solid cells hold no gas (their moments
                                         read as 0) and reflect population paths like slip walls
                                         (Sec. III.B); they may not touch an outflow or inflow face. */
    /* Oscillating point mass source (Sec. IV.C, Eqs. VC1, VC6-VC8): each step
     * adds mass src_rate * sin(src_omega * t) (Delta t = 1) to interior cell
     * (src_x, src_y) as a Maxwellian at rest in the cell's frame at its RT,
     * with t = src_t0 + the number of steps the context has completed.
     * src_rate = 0: no source.  The cell must be an interior fluid cell
     * (src_y = 0 in 1D); rho + the added mass must stay positive (otherwise
     * the reconstruction fails with LELBM_EEPR). */
    int src_x, src_y;
    double src_rate, src_omega, src_t0;
    /* Tangential (x) velocity u_w of the LELBM_BC_WALL wall on each face
     * (xlo, xhi, ylo, yhi); entries of other faces must be 0. */
    double wall_u[4];
    /* Cells along z (dim = 3; 0 or 1 otherwise).  Three dimensions: 17 stored
     * values per cell, SoA [17][nz][ny][nx] in the order M0 Mx My Mz Mxx Mxy
     * Mxz Myy Myz Mzz MDx MDy MDz G0 Gx Gy Gz (Sec. II.E: 13 + 4 values); 19
     * fluon constraints (1, the first and second moments and the per-axis
     * third-order pieces M~_{aa|g} of Eq. IIB14) and 10 phonon constraints.
     * Supported: periodic boxes (bc all LELBM_BC_PERIODIC, z periodic too),
     * LELBM_GUESS_EQ, _LIN or _PREV (the stored correction is 19 + 10
     * doubles per cell; cells with refined stencils keep none), both
     * precisions, up to 3 refinement levels (8 children per level) and radii
     * up to 64 (beyond: LELBM_EREACH).  Not in 3D: solids, walls, point
     * sources, the learned guesses, harvest, and
     * lelbm_step_noalloc (LELBM_EINVAL).  The records are banded over layers
     * of 4 cells in z within lelbm_set_scratch_budget as in 2D.  lelbm_stats
     * sum[] holds mass, x and y momentum and the energy trace. */
    int nz;
} lelbm_params;

/* Statistics accumulated over the steps of one lelbm_step call.  Newton
 * iterations count every multiplier update, including the final polishing
 * update.  q is the number of stencil points of a cell (refined points
 * counted individually).  sum[] = interior totals of mass, x/y momentum and
 * energy (M0, Mx, My, Mxx+Myy+G0) after the last step. */
typedef struct {
    double it_mean_f, it_mean_g;
    int it_max_f, it_max_g;
    long fallbacks;                   /* cells restarted from Eq. (IID13) because their LIN, MLP or PREV
                                         guess did not lower the residual at the first update, or
                                         its Newton solve failed */
    long limited;                     /* cells whose frequencies the limiter changed */
    long q_min, q_max;
    double q_mean;
    double rt_min, kn_max, colat_max; /* colat: Eq. (IIC7), |u| + R */
    double sum[4];
    long cells;                       /* cells processed (interior + pads) */
    long point_passes;                /* sum over cells of q x reconstruction passes
                                         (Newton evaluations + the final population pass) */
    long arrivals;                    /* stencil points deposited into interior cells */
    long point_passes_refined;        /* the part of point_passes spent on cells with
                                         refined stencils (Eqs. IIC10-11) */
    long wave_point_passes;           /* sum over the reconstruction's wavefronts (64 cells each)
                                         of 64 x the largest q x passes of their cells: the lanes
                                         of a wavefront run in lock step, so
                                         point_passes / wave_point_passes is the share of lane
                                         time spent on stencil points */
    long row_passes;                  /* sum over cells with unrefined stencils of the stencil rows
                                         holding points x reconstruction passes */
} lelbm_stats;

/* Number of stored moments per cell: 6 (1D), 11 (2D) or 17 (3D); -1 for
 * other dim. */
int lelbm_num_moments(int dim);

/* Equilibrium raw moments of primitive fields (Eqs. IIB7a-d, App. A Eqs. A3,
 * A7): out[k*n + i] for k < lelbm_num_moments(dim).  uy is ignored in 1D and
 * may be NULL there.  Host pointers; EINVAL on dim other than 1 or 2 (see
 * lelbm_moments_from_primitives3) or n < 0. */
int lelbm_moments_from_primitives(int dim, double K, long n, const double *rho, const double *ux,
                                  const double *uy, const double *RT, double *out);

/* The same in 3D: out[k*n + i] for the 17 moments of lelbm_params.nz's
 * layout (App. A with D = 3: M_Dg = rho (|u|^2 + 5 RT) u_g).  Host pointers;
 * EINVAL on a NULL pointer or n < 0. */
int lelbm_moments_from_primitives3(double K, long n, const double *rho, const double *ux, const double *uy,
                                   const double *uz, const double *RT, double *out);

/* Create a context from host moments (SoA, nmom*nx*ny doubles).  hip_stream
 * is a hipStream_t (NULL = default stream).  On success *out owns all device
 * memory of the run.  EINVAL on inconsistent parameters, ENOMEM on allocation
 * failure, EDEVICE on a HIP error. */
int lelbm_create(const lelbm_params *p, const double *moments, void *hip_stream, lelbm_ctx **out);

/* As lelbm_create, from device moments (FP64, or FP32 if dev_is_fp32 != 0);
 * the data is copied on hip_stream. */
int lelbm_create_device(const lelbm_params *p, const void *dev_moments, int dev_is_fp32, void *hip_stream,
                        lelbm_ctx **out);

/* Advance nsteps >= 0 time steps.  st may be NULL.  Synchronises the stream
 * once at the end.  On failure the state of the last completed step is kept. */
int lelbm_step(lelbm_ctx *c, int nsteps, lelbm_stats *st);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lelbm_step with no
 * allocation of any kind.  The population scratch of the steps is a static
 * device array of LELBM_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on (until the process ends), instead of the context's
 * own buffer, banded like the context's scratch (see
 * lelbm_set_scratch_budget) but within the array; no timing events are
 * recorded (lelbm_set_timing has no effect on this call).  A step whose
 * bands of a single tile row do not fit the array fails with LELBM_ENOMEM
 * and the context keeps the state of the last completed step
 * (lelbm_last_failure names the step; node = -1).  All calls on one GPU
 * share the array: calls that overlap in time on the same GPU (two contexts
 * on different streams, or two threads) race and must be serialised by the
 * caller.  Results equal those of lelbm_step bit for bit.  Error behaviour
 * is otherwise that of lelbm_step. */
#define LELBM_NOALLOC_SCRATCH_BYTES (64u << 20)
int lelbm_step_noalloc(lelbm_ctx *c, int nsteps, lelbm_stats *st);

/* Copy the current moments to caller-owned host memory (nmom*nx*ny FP64). */
int lelbm_read_moments(const lelbm_ctx *c, double *host_out);

/* Copy the current moments to caller-owned device memory (nmom*nx*ny FP64),
 * ordered on the context's stream (no host synchronisation). */
int lelbm_read_moments_device(const lelbm_ctx *c, void *dev_out);

/* Cell index (row-major over the padded source domain, pads included) and
 * step (0-based within the failing lelbm_step call) of the first failure. */
int lelbm_last_failure(const lelbm_ctx *c, long *node, int *step);

/* Why the reconstruction of the failing cell failed (after LELBM_EEPR):
 * reason 1 non-finite populations at the first evaluation, 2 line search
 * exhausted (30 halvings), 3 Cholesky breakdown in the polishing update,
 * 4 Newton iteration cap, 5 Cholesky breakdown in a Newton step; 0 when the
 * failure was not in the Newton solve (e.g. rho <= 0 or RT <= 0).  species:
 * 0 fluon, 1 phonon, -1 none.  residual: last scaled moment residual. */
int lelbm_last_failure_detail(const lelbm_ctx *c, int *reason, int *species, double *residual);

/* Per-kernel timing: when enabled, lelbm_step records HIP events around each
 * kernel and lelbm_kernel_times returns accumulated milliseconds and launch
 * counts for: [0] pad fill, [1] stencil pre-pass, [2] tile scan,
 * [3] collision + reconstruction of cells with unrefined stencils (narrow and
 * wide stencils; one launch pair per band of the scratch plan), [4]
 * moment-streaming gather (one launch per run of destination rows), [5] step
 * totals (statistics and arrival counts), [6] no-slip walls: image
 * reconstruction (one launch per band) and image arrivals (one per step)
 * (the learned guess runs inside the reconstruction kernel [3]), [7]
 * collision + reconstruction of cells with refined stencils.
 * n is the capacity of ms and launches (at most LELBM_NTIMERS are filled). */
#define LELBM_NTIMERS 8
int lelbm_set_timing(lelbm_ctx *c, int enable);
int lelbm_kernel_times(const lelbm_ctx *c, double *ms, long *launches, int n);

/* Device bytes held by the context: persistent state (moments, descriptors;
 * with solid cells or slip walls also the blocker distances and, when it fits
 * in an eighth of the free device memory, the cache of backward-walk results
 * around the solids) and the transient population scratch. */
int lelbm_memory(const lelbm_ctx *c, long *persistent_bytes, long *scratch_bytes);

/* Population scratch budget.  The moment fractions of Eq. (IIE3a) exist only
 * within a step, between the reconstruction of a source and the gather of
 * its destinations (Sec. II.E).  The library reconstructs the source tiles
 * in bands of whole tile rows and gathers each destination row as soon as
 * the bands within its reach are done, reusing the scratch slots of bands
 * no longer needed; the bands are as wide as the budget allows (one band
 * when the whole domain's records fit) and are re-planned, before the step
 * is repeated, when a band outgrows its slot or a stencil reaches farther
 * than the plan allows for.  The scratch therefore stays within the budget
 * whatever the temperature, unless a band of a single tile row (16 rows of
 * cells) needs more, which then sets the scratch size.  Results do not
 * depend on the banding (bit for bit).  Default LELBM_DEFAULT_SCRATCH_BUDGET
 * bytes; a budget below the current scratch frees it.  EINVAL for bytes < 1. */
#define LELBM_DEFAULT_SCRATCH_BUDGET (16ll << 30)
int lelbm_set_scratch_budget(lelbm_ctx *c, long long bytes);

const char *lelbm_strerror(int code);
void lelbm_destroy(lelbm_ctx *c);

/* ------------------------------------------------------------------------
 * Learned warm start of the Newton solve (2D).  Not part of the paper: the
 * paper starts every solve from Eq. (IID13) and suggests storing multipliers
 * between steps (Sec. II.D).  Here a 16-64-64-16 ReLU network maps a cell's
 * normalised post-collision moments and stencil geometry to its multipliers;
 * Eq. (IID13) remains the fallback whenever the residual of a solve started
 * from the network does not drop, so converged results equal those of the
 * plain path (the dual problem has a unique minimiser).
 *
 * Parameters: 6288 FP32 values in the order W1[16][64], b1[64], W2[64][64],
 * b2[64], W3[64][16], b3[16] (row-major [in][out]).  Inputs x[16] and
 * targets y[16] of a training pair are described in the README of the
 * package; pairs are harvested by the step itself (lelbm_harvest).  Training
 * and inference run in the library's BF16-MFMA kernels with FP32
 * accumulation and FP32 master weights (Adam).
 * ------------------------------------------------------------------------ */
#define LELBM_MLP_NPARAM 6288
typedef struct lelbm_mlp lelbm_mlp;

/* New network: params (host, LELBM_MLP_NPARAM floats) or NULL for a seeded
 * He-uniform initialisation.  All work is issued on hip_stream. */
int lelbm_mlp_create(const float *params, unsigned long long seed, void *hip_stream, lelbm_mlp **out);
/* Current FP32 parameters to caller-owned host memory. */
int lelbm_mlp_get_params(const lelbm_mlp *m, float *host_out);
/* Inference: dev_x rows of 16 floats with a stride of x_stride floats,
 * dev_y: n x 16 floats (device memory, caller-owned). */
int lelbm_mlp_forward(lelbm_mlp *m, const float *dev_x, long long x_stride, long long n, float *dev_y);
/* Gradient of the mean squared error over n pairs (dev_pairs: n x 32 floats,
 * inputs then targets) with respect to the parameters; host_grad may be
 * NULL; loss receives the mean squared error. */
int lelbm_mlp_gradient(lelbm_mlp *m, const float *dev_pairs, long long n, float *host_grad, double *loss);
/* steps Adam updates (learning rate lr, beta 0.9/0.999) on batches of
 * `batch` pairs (multiple of 64) drawn with replacement by a counter-based
 * generator seeded with seed; final_loss (nullable) receives the mean squared
 * error of the last batch. */
int lelbm_mlp_train(lelbm_mlp *m, const float *dev_pairs, long long n, int steps, int batch, float lr,
                    unsigned long long seed, double *final_loss);
/* Standardisation: the network sees (x - mean_x) / sd_x and predicts
 * (y - mean_y) / sd_y.  The 64 constants are mean_x[16], 1/sd_x[16],
 * mean_y[16], sd_y[16] (identity at creation).  fit computes them from n
 * pairs on the device (columns with sd < 1e-12 get unit scale). */
#define LELBM_MLP_NNORM 64
int lelbm_mlp_fit_normalization(lelbm_mlp *m, const float *dev_pairs, long long n);
int lelbm_mlp_get_norm(const lelbm_mlp *m, float *host_out);
int lelbm_mlp_set_norm(lelbm_mlp *m, const float *host_norm);
void lelbm_mlp_destroy(lelbm_mlp *m);

/* Copies the network into a context created with guess = LELBM_GUESS_MLP
 * or LELBM_GUESS_MLP_PREV (required before its first step). */
int lelbm_set_mlp(lelbm_ctx *c, const lelbm_mlp *m);
/* Harvest (features, converged multipliers) pairs during lelbm_step into a
 * caller-owned device buffer of capacity x 32 floats: cell s at step k is
 * recorded when (s + 7919 k) is divisible by stride (unrefined 2D cells).
 * The target is the scaled correction of the converged multipliers beyond
 * the context's own non-learned start: LIN, or in PREV and MLP_PREV modes
 * LIN plus the stored correction (there only cells that have one are
 * recorded).  dev_buf = NULL stops harvesting.  The order of the pairs is
 * not fixed. */
int lelbm_harvest(lelbm_ctx *c, float *dev_buf, long long capacity, int stride);
int lelbm_harvest_count(const lelbm_ctx *c, long long *n);

#ifdef __cplusplus
}
#endif
#endif
