/*
 * Plain FP64 CPU oracle of one LELBM time step (Lagrangian entropic lattice
 * Boltzmann method, arXiv 2508.06911).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * links, loads or calls it.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.
 *
 * Every stage follows the paper's statement of the method directly, in FP64,
 * with a fixed loop order and no blocking or fusion:
 *   - macroscopic variables ............ Sec. II.B, Eq. (IIB6a-c)
 *   - non-equilibrium central moments .. Sec. II.B, Eqs. (IIB9a-d)
 *   - bulk/shear split ................. Eqs. (IIB10-11)
 *   - third-order per-axis split ....... Eq. (IIB14)
 *   - Knudsen limiter .................. App. D, Eqs. (D2-D3), as worded in
 *                                        the text that follows Eq. (D3b)
 *   - post-collision central moments ... Eqs. (IIB16a-f, IIB17), normalised
 *                                        by Eq. (IIB18)
 *   - Lagrangian acoustic stencil ...... Sec. II.C, Eqs. (IIC6, IIC9-11)
 *   - entropic reconstruction .......... Sec. II.D, Eqs. (IID7-11, IID13)
 *   - moment streaming ................. Sec. II.E, Eqs. (IIE3a-b)
 *   - fluid boundaries ................. Sec. III.A (pads of width W; a pad
 *                                        narrower than a stencil's reach toward
 *                                        the interior is an error, Sec. III)
 *   - slip walls and solid cells ....... Sec. III.B (specular reflection of
 *                                        the population path at every face
 *                                        it would cross into a blocker)
 *   - oscillating point mass source .... Sec. IV.C, Eqs. (VC1, VC6-VC8)
 *   - no-slip / moving walls ........... Sec. III.B, Eqs. (IIIB8-IIIB15),
 *                                        extended bounce-back on the y faces
 *
 * Readings taken where the paper is ambiguous are listed in the header
 * comment of each function.
 *
 * Moment layout (raw moments, lattice units dV = dx = dt = 1):
 *   2D: M0 Mx My Mxx Mxy Myy MDx MDy G0 Gx Gy   (11 values)
 *   1D: M0 Mx Mxx Mxxx G0 Gx                    ( 6 values)
 * Arrays are SoA: [moment][y][x].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* residual below which a Newton solve that stops decreasing is converged */
#define ORC_STALL_RES 1e-10

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EEPR = -4, ORC_ENONFINITE = -5, ORC_EREACH = -6 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_INFLOW = 2, ORC_BC_SLIPWALL = 3, ORC_BC_WALL = 4 };

/* Parameters of one run.  Mirrored field by field by the Python wrapper. */
typedef struct {
    int dim, nx, ny;
    double K;                        /* internal degrees of freedom */
    double omega_f, omega_b, omega_h;/* shear, bulk, heat-flux collision frequencies */
    double n_conf;                   /* conformation number n of Eq. (IIC6) */
    int r_min;                       /* minimum acoustic radius of Eq. (IIC6) */
    double newton_tol;               /* scaled moment residual that stops Newton */
    int newton_max_it;
    int kn_limiter;                  /* 1: apply the Knudsen limiter of App. D */
    double kn_lo, kn_hi, omega_H;    /* log10 thresholds and target frequency */
    int bc[4];                       /* xlo, xhi, ylo, yhi */
    int pad;                         /* pad width for outflow/inflow faces */
    double in_rho, in_u[2], in_RT;   /* inflow state */
    const unsigned char *solid;      /* nx*ny legoland mask (1 = solid cell) or NULL */
    /* oscillating point mass source, Sec. IV.C: rate*sin(omega*t) in cell
     * (src_x, src_y) of the interior; rate = 0: none.  src_t is the time of
     * the first step's collision (steps of orc_run follow at src_t + k). */
    int src_x, src_y;
    double src_rate, src_omega, src_t;
    /* no-slip walls (ORC_BC_WALL, y faces of a 2D domain): velocity of the
     * wall along x, per face (entries 2 and 3 used) */
    double wall_u[4];
} orc_params;

typedef struct {
    long cells;                      /* source cells processed (interior + pads) */
    long it_sum_f, it_sum_g;
    int it_max_f, it_max_g;
    long q_sum; int q_min, q_max;
    long limited;                    /* cells where the limiter changed omega */
    double rt_min, kn_max, colat_max;
    long fail_cell; int fail_code;   /* first failing source cell (row-major index in padded domain) */
} orc_stats;

int orc_num_moments(int dim) { return dim == 1 ? 6 : (dim == 2 ? 11 : -1); }

/* ------------------------------------------------------------------------ */
/* Equilibrium raw moments, Eqs. (IIB7a-d) with M0 = rho and Ma = rho u_a     */
/* (App. A, Eqs. A3a-b, A3g, A7a-b).                                          */
/* ------------------------------------------------------------------------ */
static void eq_moments(int dim, double K, double rho, double ux, double uy, double RT, double *m)
{
    if (dim == 1) {
        m[0] = rho;
        m[1] = rho * ux;
        m[2] = rho * (ux * ux + RT);
        m[3] = rho * (ux * ux + 3.0 * RT) * ux;          /* |u|^2 + (D+2) RT, D = 1 */
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
        m[6] = rho * (uu + 4.0 * RT) * ux;               /* D + 2 = 4 */
        m[7] = rho * (uu + 4.0 * RT) * uy;
        m[8] = rho * K * RT;
        m[9] = rho * K * RT * ux;
        m[10] = rho * K * RT * uy;
    }
}

int orc_moments_from_primitives(int dim, double K, long n, const double *rho, const double *ux,
                                const double *uy, const double *RT, double *out)
{
    int nm = orc_num_moments(dim);
    if (nm < 0 || n < 0) return ORC_EINVAL;
    for (long i = 0; i < n; i++) {
        double m[11];
        eq_moments(dim, K, rho[i], ux[i], dim == 2 ? uy[i] : 0.0, RT[i], m);
        for (int k = 0; k < nm; k++) out[(long)k * n + i] = m[k];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Collision: moments of one cell -> normalised post-collision central        */
/* moment targets for the fluon (m) and phonon (n) reconstructions.           */
/*                                                                            */
/* Basis order (relative velocity c~ = c - u):                                */
/*   2D fluon : 1, x, y, xx, xy, yy, xxx, xxy, xyy, yyy   (10)                */
/*   2D phonon: 1, x, y, xx, xy, yy                       (6)                 */
/*   1D fluon : 1, x, xx, xxx                             (4)                 */
/*   1D phonon: 1, x, xx                                  (3)                 */
/* Third-order fluon constraints are the per-axis pieces M~_{aa|g} of         */
/* Eq. (IIB14): xxx = M~_{xx|x}, xxy = M~_{xx|y}, xyy = M~_{yy|x},            */
/* yyy = M~_{yy|y}.  The phonon second-order constraint is Eq. (IIB17), which */
/* fixes the off-diagonal xy component to zero.                               */
/*                                                                            */
/* Knudsen number, Eq. (D2), read with numerators normalised by rho only so   */
/* that both ratios are dimensionless; the sums are L1 norms over all D^2     */
/* (a,b) pairs and over g.  Limiter, Eq. (D3): frequencies are unchanged for  */
/* Kn < 10^kn_lo, set to omega_H above 10^kn_hi, and linear in log10 Kn in     */
/* between (the wording after Eq. (D3b); the printed cases are swapped).      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double rho, u[2], RT;
    double rho_post;                     /* zeroth post-collision moment (rho plus a mass source) */
    double Pneq[2][2], Q[2], g0, h[2];   /* non-equilibrium central moments */
    double kn, om_f, om_b, om_h;
    int limited;
    double m[10], n[6];
    int nf, ng;
} orc_cell;

static double limit_omega(double kn, double om, const orc_params *p)
{
    double lo = pow(10.0, p->kn_lo), hi = pow(10.0, p->kn_hi);
    if (kn < lo) return om;
    if (kn > hi) return p->omega_H;
    double k = log10(kn);
    return (p->omega_H - om) / (p->kn_hi - p->kn_lo) * (k - p->kn_lo) + om;
}

/* src: mass added to the cell in this step, Delta t times the rate of the  */
/* source (Eq. VC1), 0 elsewhere.  Its central moments (Eqs. VC6-VC7) are   */
/* those of a Maxwellian at rest in the cell's frame at the cell's RT: mass */
/* src, no first or third moments, second moments src RT delta, phonon     */
/* energy src K RT with second moments src K RT RT delta.  Added to the     */
/* post-collision moments (Eq. VC8), they leave RT and the frame unchanged  */
/* and raise the zeroth moment to rho + src, which the targets are          */
/* normalised by (Eq. IIB18) and the moment fractions scaled by.            */
static int collide_src(const orc_params *p, const double *mom, double src, orc_cell *c)
{
    int D = p->dim;
    double K = p->K;
    memset(c, 0, sizeof(*c));
    /* Eq. (IIB6) */
    double rho = mom[0];
    if (!(rho > 0.0) || !isfinite(rho)) return ORC_EEPR;
    double ux, uy = 0.0, Mxx, Mxy = 0.0, Myy = 0.0, MDx, MDy = 0.0, G0, Gx, Gy = 0.0, Mx, My = 0.0;
    if (D == 1) {
        Mx = mom[1]; Mxx = mom[2]; MDx = mom[3]; G0 = mom[4]; Gx = mom[5];
    } else {
        Mx = mom[1]; My = mom[2]; Mxx = mom[3]; Mxy = mom[4]; Myy = mom[5];
        MDx = mom[6]; MDy = mom[7]; G0 = mom[8]; Gx = mom[9]; Gy = mom[10];
    }
    ux = Mx / rho;
    if (D == 2) uy = My / rho;
    double uu = ux * ux + uy * uy;
    double RT = ((Mxx + Myy + G0) / rho - uu) / (D + K);
    if (!(RT > 0.0) || !isfinite(RT)) return ORC_EEPR;
    c->rho = rho; c->u[0] = ux; c->u[1] = uy; c->RT = RT;
    double rp = rho + src;
    if (!(rp > 0.0)) return ORC_EEPR;
    c->rho_post = rp;

    /* Eq. (IIB9a): P_ab = M_ab - rho (u_a u_b + RT delta_ab) */
    double P[2][2] = {{0, 0}, {0, 0}};
    P[0][0] = Mxx - rho * (ux * ux + RT);
    if (D == 2) {
        P[0][1] = P[1][0] = Mxy - rho * (ux * uy);
        P[1][1] = Myy - rho * (uy * uy + RT);
    }
    /* Eq. (IIB9b): Q_g = M_Dg - 2 u_a P_ag - u_g P_aa - rho (|u|^2 + (D+2) RT) u_g */
    double u[2] = {ux, uy};
    double MD[2] = {MDx, MDy};
    double trP = P[0][0] + P[1][1];
    double Q[2] = {0, 0};
    for (int g = 0; g < D; g++) {
        double s = 0.0;
        for (int a = 0; a < D; a++) s += u[a] * P[a][g];
        Q[g] = MD[g] - 2.0 * s - u[g] * trP - rho * (uu + (D + 2) * RT) * u[g];
    }
    /* Eqs. (IIB9c-d) */
    double g0 = G0 - rho * K * RT;
    double Gv[2] = {Gx, Gy};
    double h[2] = {0, 0};
    for (int g = 0; g < D; g++) h[g] = Gv[g] - u[g] * G0;

    for (int a = 0; a < 2; a++) {
        for (int b = 0; b < 2; b++) c->Pneq[a][b] = P[a][b];
        c->Q[a] = Q[a]; c->h[a] = h[a];
    }
    c->g0 = g0;

    /* Knudsen number, Eq. (D2) */
    double sP = 0.0, sQ = 0.0;
    for (int a = 0; a < D; a++) {
        for (int b = 0; b < D; b++) sP += fabs(P[a][b]);
        sQ += fabs(Q[a]) + fabs(h[a]);
    }
    double knA = (sP + fabs(g0)) / (rho * (D + K) * RT);
    double knB = sQ / (rho * (D + K + 2.0) * pow(RT, 1.5));
    double kn = knA > knB ? knA : knB;
    c->kn = kn;
    double of = p->omega_f, ob = p->omega_b, oh = p->omega_h;
    if (p->kn_limiter) {
        of = limit_omega(kn, p->omega_f, p);
        ob = limit_omega(kn, p->omega_b, p);
        oh = limit_omega(kn, p->omega_h, p);
        c->limited = (of != p->omega_f) || (ob != p->omega_b) || (oh != p->omega_h);
    }
    c->om_f = of; c->om_b = ob; c->om_h = oh;

    /* Eqs. (IIB10-11): bulk = -(g0/D) delta, shear = P - bulk */
    double bulk[2][2] = {{0, 0}, {0, 0}}, shear[2][2];
    for (int a = 0; a < D; a++) bulk[a][a] = -g0 / D;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) shear[a][b] = P[a][b] - bulk[a][b];
    /* Eq. (IIB14): t_{a|g} = (1 + 2 delta_ag)/(D+2) Q_g */
    double t[2][2];
    for (int a = 0; a < 2; a++)
        for (int g = 0; g < 2; g++) t[a][g] = (1.0 + 2.0 * (a == g)) / (D + 2) * Q[g];

    /* Eqs. (IIB16a-d) normalised by rho (Eq. IIB18), with a mass source by  */
    /* rho + src: (rho RT delta + neq + src RT delta) / (rho + src)          */
    double mab[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            mab[a][b] = RT * (a == b) + ((1.0 - of) * shear[a][b] + (1.0 - ob) * bulk[a][b]) / rp;
    double rKT = rp * K * RT;
    if (D == 1) {
        c->nf = 4; c->ng = 3;
        c->m[0] = 1.0; c->m[1] = 0.0; c->m[2] = mab[0][0];
        c->m[3] = (1.0 - oh) * t[0][0] / rp;
        /* Eqs. (IIB16e-f, IIB17) normalised by rho K RT */
        c->n[0] = 1.0 + (1.0 - ob) * g0 / rKT;
        c->n[1] = (1.0 - oh) * h[0] / rKT;
        c->n[2] = RT;
    } else {
        c->nf = 10; c->ng = 6;
        c->m[0] = 1.0; c->m[1] = 0.0; c->m[2] = 0.0;
        c->m[3] = mab[0][0]; c->m[4] = mab[0][1]; c->m[5] = mab[1][1];
        c->m[6] = (1.0 - oh) * t[0][0] / rp;    /* xxx = M~_{xx|x} */
        c->m[7] = (1.0 - oh) * t[0][1] / rp;    /* xxy = M~_{xx|y} */
        c->m[8] = (1.0 - oh) * t[1][0] / rp;    /* xyy = M~_{yy|x} */
        c->m[9] = (1.0 - oh) * t[1][1] / rp;    /* yyy = M~_{yy|y} */
        c->n[0] = 1.0 + (1.0 - ob) * g0 / rKT;
        c->n[1] = (1.0 - oh) * h[0] / rKT;
        c->n[2] = (1.0 - oh) * h[1] / rKT;
        c->n[3] = RT; c->n[4] = 0.0; c->n[5] = RT;
    }
    return ORC_OK;
}

int orc_collide(const orc_params *p, const double *mom, orc_cell *c) { return collide_src(p, mom, 0.0, c); }

/* Flat export of orc_collide for the tests: out = [rho, ux, uy, RT, kn,
 * om_f, om_b, om_h, limited, Pxx, Pxy, Pyy, Qx, Qy, g0, hx, hy, m[10], n[6]] */
int orc_collide_flat(const orc_params *p, const double *mom, double *out)
{
    orc_cell c;
    int st = orc_collide(p, mom, &c);
    double v[] = {c.rho, c.u[0], c.u[1], c.RT, c.kn, c.om_f, c.om_b, c.om_h, (double)c.limited,
                  c.Pneq[0][0], c.Pneq[0][1], c.Pneq[1][1], c.Q[0], c.Q[1], c.g0, c.h[0], c.h[1]};
    int k = 0;
    for (unsigned i = 0; i < sizeof(v) / sizeof(v[0]); i++) out[k++] = v[i];
    for (int i = 0; i < 10; i++) out[k++] = c.m[i];
    for (int i = 0; i < 6; i++) out[k++] = c.n[i];
    return st;
}

/* As orc_collide_flat, with a mass source of src in the cell. */
int orc_collide_src_flat(const orc_params *p, const double *mom, double src, double *out)
{
    orc_cell c;
    int st = collide_src(p, mom, src, &c);
    double v[] = {c.rho, c.u[0], c.u[1], c.RT, c.kn, c.om_f, c.om_b, c.om_h, (double)c.limited,
                  c.Pneq[0][0], c.Pneq[0][1], c.Pneq[1][1], c.Q[0], c.Q[1], c.g0, c.h[0], c.h[1]};
    int k = 0;
    for (unsigned i = 0; i < sizeof(v) / sizeof(v[0]); i++) out[k++] = v[i];
    for (int i = 0; i < 10; i++) out[k++] = c.m[i];
    for (int i = 0; i < 6; i++) out[k++] = c.n[i];
    return st;
}

/* ------------------------------------------------------------------------ */
/* Lagrangian acoustic stencil, Sec. II.C.                                    */
/*                                                                            */
/* Readings (they reproduce both worked examples the paper prints: 284 points */
/* for RT = 5, u = (13.7, 14.1) and 41 refined points for RT = 0.2,           */
/* u = (3.7, 4.1)):                                                           */
/*   R = max([n sqrt(RT)], r_min) with [x] = floor(x + 1/2)        Eq. (IIC6) */
/*   base points: integer c with |c - u| <= R + 1/2 (unrounded u), dC = 1     */
/*   N_r = [1 / (3 sqrt(RT))]                                      Eq. (IIC9) */
/*   for Lvl = 1..N_r every point of spacing h = 2^(1-Lvl) with               */
/*   |c - u| <= 3 * 2^-Lvl is replaced by its 2^D children c + (+-h/4, ...),  */
/*   each with dC * 2^-D                                   Eqs. (IIC10-11)    */
/*   every descendant lands in the cell of its integer ancestor.              */
/* Base points are enumerated row by row (c_y outer, c_x inner); children     */
/* replace their parent in place, in the sign order (-,-), (+,-), (-,+),      */
/* (+,+) (x fastest).                                                         */
/* ------------------------------------------------------------------------ */
static double round_half_up(double x) { return floor(x + 0.5); }

int orc_las_radius(double RT, double n_conf, int r_min)
{
    int R = (int)round_half_up(n_conf * sqrt(RT));
    return R > r_min ? R : r_min;
}

int orc_las_levels(double RT) { return (int)round_half_up(1.0 / (3.0 * sqrt(RT))); }

static double dist_u(int dim, const double *c, const double *u)
{
    double dx = c[0] - u[0];
    if (dim == 1) return fabs(dx);
    double dy = c[1] - u[1];
    return sqrt(dx * dx + dy * dy);
}

/* Fills c[2*i], dC[i], d[2*i] for i < q and returns q, or -q_needed if cap is
 * too small. */
int orc_las(int dim, const double *u, double RT, double n_conf, int r_min, int cap, double *c, double *dC,
            int *d, double *spacing)
{
    int R = orc_las_radius(RT, n_conf, r_min);
    int Nr = orc_las_levels(RT);
    double rr = R + 0.5;
    /* base disk */
    int q = 0;
    int ylo = dim == 2 ? (int)floor(u[1] - rr) - 1 : 0, yhi = dim == 2 ? (int)ceil(u[1] + rr) + 1 : 0;
    int xlo = (int)floor(u[0] - rr) - 1, xhi = (int)ceil(u[0] + rr) + 1;
    int nmax = (xhi - xlo + 1) * (yhi - ylo + 1);
    for (int l = 0; l < Nr; l++) nmax *= (dim == 2 ? 4 : 2);
    double *tc = malloc(sizeof(double) * 2 * nmax), *tdc = malloc(sizeof(double) * nmax), *th = malloc(sizeof(double) * nmax);
    int *td = malloc(sizeof(int) * 2 * nmax);
    double *nc = malloc(sizeof(double) * 2 * nmax), *ndc = malloc(sizeof(double) * nmax), *nh = malloc(sizeof(double) * nmax);
    int *nd = malloc(sizeof(int) * 2 * nmax);
    if (!tc || !tdc || !th || !td || !nc || !ndc || !nh || !nd) {
        free(tc); free(tdc); free(th); free(td); free(nc); free(ndc); free(nh); free(nd);
        return 0;
    }
    for (int cy = ylo; cy <= yhi; cy++) {
        for (int cx = xlo; cx <= xhi; cx++) {
            double cc[2] = {cx, cy};
            double dxv = cc[0] - u[0];
            double inside;
            if (dim == 1) inside = dxv * dxv <= rr * rr;
            else {
                double dyv = cc[1] - u[1];
                inside = dxv * dxv + dyv * dyv <= rr * rr;
            }
            if (!inside) continue;
            tc[2 * q] = cx; tc[2 * q + 1] = dim == 2 ? cy : 0.0;
            tdc[q] = 1.0; th[q] = 1.0;
            td[2 * q] = cx; td[2 * q + 1] = dim == 2 ? cy : 0;
            q++;
        }
    }
    for (int lvl = 1; lvl <= Nr; lvl++) {
        double thr = 3.0 * pow(0.5, lvl);
        int m = 0;
        for (int i = 0; i < q; i++) {
            if (dist_u(dim, &tc[2 * i], u) <= thr) {
                double h = th[i];
                int nchild = dim == 2 ? 4 : 2;
                for (int k = 0; k < nchild; k++) {
                    double sx = (k & 1) ? 1.0 : -1.0;
                    double sy = (k & 2) ? 1.0 : -1.0;
                    nc[2 * m] = tc[2 * i] + sx * h / 4.0;
                    nc[2 * m + 1] = dim == 2 ? tc[2 * i + 1] + sy * h / 4.0 : 0.0;
                    ndc[m] = tdc[i] * (dim == 2 ? 0.25 : 0.5);
                    nh[m] = h / 2.0;
                    nd[2 * m] = td[2 * i]; nd[2 * m + 1] = td[2 * i + 1];
                    m++;
                }
            } else {
                nc[2 * m] = tc[2 * i]; nc[2 * m + 1] = tc[2 * i + 1];
                ndc[m] = tdc[i]; nh[m] = th[i];
                nd[2 * m] = td[2 * i]; nd[2 * m + 1] = td[2 * i + 1];
                m++;
            }
        }
        double *sw;
        int *swi;
        sw = tc; tc = nc; nc = sw;
        sw = tdc; tdc = ndc; ndc = sw;
        sw = th; th = nh; nh = sw;
        swi = td; td = nd; nd = swi;
        q = m;
    }
    int ret = q;
    if (q > cap) ret = -q;
    else {
        for (int i = 0; i < q; i++) {
            c[2 * i] = tc[2 * i]; c[2 * i + 1] = tc[2 * i + 1];
            dC[i] = tdc[i];
            d[2 * i] = td[2 * i]; d[2 * i + 1] = td[2 * i + 1];
            if (spacing) spacing[i] = th[i];
        }
    }
    free(tc); free(tdc); free(th); free(td); free(nc); free(ndc); free(nh); free(nd);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* Entropic population reconstruction, Sec. II.D.                             */
/*                                                                            */
/* Populations f_i = dC_i exp(-(1 + sum_j lambda_j T_j(c~_i)))     Eq. (IID7) */
/* Newton: A dl = sum_k T f_k - M', A_ij = sum_k T_i f_k T_j,                 */
/*         lambda += dl                                      Eqs. (IID8-11)  */
/* solved by Cholesky (Sec. II.D), started from Eq. (IID13).                  */
/*                                                                            */
/* Readings: the residual test is max_j |r_j| / RT^(k_j/2) <= tol, where k_j   */
/* is the polynomial order of basis function j (a scale-free form of the      */
/* 1e-12 residual of Sec. II.D).  After the test passes, one more Newton      */
/* update is applied (a polishing step that brings the conserved moments to   */
/* rounding level), and the populations are evaluated at the polished        */
/* multipliers.  Safeguard: while the Newton decrement r.dl exceeds 1e-8, a   */
/* step must lower the convex dual Phi = sum_i f_i + lambda.M' by the Armijo  */
/* fraction 1e-4, else it is halved (at most 30 times).  A residual that is  */
/* below 1e-10 and did not decrease at the last update has reached the       */
/* rounding floor of the sums (large, badly conditioned stencils stall just  */
/* above 1e-12): the solve is taken as converged there.  Failure (Cholesky    */
/* breakdown, non-finite values, line search or iteration cap exhausted)      */
/* returns ORC_EEPR.                                                          */
/* ------------------------------------------------------------------------ */
static void basis(int dim, int nb, const double *ct, double *T, int *order)
{
    double x = ct[0];
    if (dim == 1) {
        double v[4] = {1.0, x, x * x, x * x * x};
        int o[4] = {0, 1, 2, 3};
        for (int j = 0; j < nb; j++) { T[j] = v[j]; if (order) order[j] = o[j]; }
    } else {
        double y = ct[1];
        double v[10] = {1.0, x, y, x * x, x * y, y * y, x * x * x, x * x * y, x * y * y, y * y * y};
        int o[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
        for (int j = 0; j < nb; j++) { T[j] = v[j]; if (order) order[j] = o[j]; }
    }
}

/* One pass at multipliers lam: populations, dual value, residual, Hessian. */
static int epr_eval(int dim, int nb, int q, const double *c, const double *dC, const double *u,
                    const double *lam, const double *target, double *pop, double *phi, double *r, double *A)
{
    double s[10] = {0};
    for (int i = 0; i < nb * nb; i++) A[i] = 0.0;
    double sum = 0.0;
    for (int i = 0; i < q; i++) {
        double ct[2] = {c[2 * i] - u[0], dim == 2 ? c[2 * i + 1] - u[1] : 0.0};
        double T[10];
        basis(dim, nb, ct, T, NULL);
        double e = 0.0;
        for (int j = 0; j < nb; j++) e += lam[j] * T[j];
        double f = dC[i] * exp(-(1.0 + e));
        pop[i] = f;
        sum += f;
        for (int j = 0; j < nb; j++) s[j] += T[j] * f;
        for (int j = 0; j < nb; j++)
            for (int k = 0; k < nb; k++) A[j * nb + k] += T[j] * f * T[k];
    }
    double lm = 0.0;
    for (int j = 0; j < nb; j++) { r[j] = s[j] - target[j]; lm += lam[j] * target[j]; }
    *phi = sum + lm;
    if (!isfinite(*phi)) return ORC_ENONFINITE;
    for (int j = 0; j < nb; j++) if (!isfinite(r[j])) return ORC_ENONFINITE;
    return ORC_OK;
}

/* Cholesky solve of the SPD system A x = b (A is nb x nb, row-major). */
static int cholesky_solve(int nb, const double *A, const double *b, double *x)
{
    double L[100] = {0};
    for (int i = 0; i < nb; i++) {
        for (int j = 0; j <= i; j++) {
            double s = A[i * nb + j];
            for (int k = 0; k < j; k++) s -= L[i * nb + k] * L[j * nb + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return ORC_EEPR;
                L[i * nb + i] = sqrt(s);
            } else {
                L[i * nb + j] = s / L[j * nb + j];
            }
        }
    }
    double y[10];
    for (int i = 0; i < nb; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= L[i * nb + k] * y[k];
        y[i] = s / L[i * nb + i];
    }
    for (int i = nb - 1; i >= 0; i--) {
        double s = y[i];
        for (int k = i + 1; k < nb; k++) s -= L[k * nb + i] * x[k];
        x[i] = s / L[i * nb + i];
    }
    return ORC_OK;
}

/* Initial guess, Eq. (IID13). */
void orc_epr_initial(int dim, int nb, double RT, double *lam)
{
    for (int j = 0; j < nb; j++) lam[j] = 0.0;
    lam[0] = -1.0 + 0.5 * dim * log(2.0 * M_PI * RT);
    if (dim == 1) lam[2] = 1.0 / (2.0 * RT);
    else { lam[3] = 1.0 / (2.0 * RT); lam[5] = 1.0 / (2.0 * RT); }
}

/* lam: in = initial multipliers (if use_init) / out = converged multipliers.
 * Returns ORC_OK and the number of Newton updates in *iters. */
int orc_epr(int dim, int nb, int q, const double *c, const double *dC, const double *u, double RT,
            const double *target, int use_init, double *lam, double tol, int maxit, double *pop, int *iters)
{
    double r[10], A[100], phi, dl[10], lt[10], rt[10], At[100], phit;
    int order[10];
    double Tdummy[10], zero[2] = {0, 0};
    basis(dim, nb, zero, Tdummy, order);
    if (!use_init) orc_epr_initial(dim, nb, RT, lam);
    double *popt = malloc(sizeof(double) * (q > 0 ? q : 1));
    if (!popt) return ORC_ENOMEM;
    int st = epr_eval(dim, nb, q, c, dC, u, lam, target, pop, &phi, r, A);
    int nit = 0;
    double res_prev = INFINITY;
    if (st != ORC_OK) { free(popt); return ORC_EEPR; }
    for (;;) {
        double res = 0.0;
        for (int j = 0; j < nb; j++) {
            double v = fabs(r[j]) / pow(RT, 0.5 * order[j]);
            if (v > res) res = v;
        }
        if (res <= tol) break;
        if (nit > 0 && res <= ORC_STALL_RES && !(res < res_prev)) break;
        res_prev = res;
        if (nit >= maxit) { free(popt); return ORC_EEPR; }
        if (cholesky_solve(nb, A, r, dl) != ORC_OK) { free(popt); return ORC_EEPR; }
        double dec = 0.0;
        for (int j = 0; j < nb; j++) dec += r[j] * dl[j];
        double t = 1.0;
        int ok = 0;
        for (int ls = 0; ls <= 30; ls++) {
            for (int j = 0; j < nb; j++) lt[j] = lam[j] + t * dl[j];
            int s2 = epr_eval(dim, nb, q, c, dC, u, lt, target, popt, &phit, rt, At);
            if (s2 == ORC_OK && (dec <= 1e-8 || phit <= phi - 1e-4 * t * dec)) { ok = 1; break; }
            t *= 0.5;
        }
        if (!ok) { free(popt); return ORC_EEPR; }
        for (int j = 0; j < nb; j++) { lam[j] = lt[j]; r[j] = rt[j]; }
        for (int j = 0; j < nb * nb; j++) A[j] = At[j];
        for (int i = 0; i < q; i++) pop[i] = popt[i];
        phi = phit;
        nit++;
    }
    /* polishing update */
    if (cholesky_solve(nb, A, r, dl) != ORC_OK) { free(popt); return ORC_EEPR; }
    for (int j = 0; j < nb; j++) lam[j] += dl[j];
    nit++;
    st = epr_eval(dim, nb, q, c, dC, u, lam, target, pop, &phi, r, A);
    free(popt);
    if (st != ORC_OK) return ORC_EEPR;
    *iters = nit;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One time step.                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int status, q, it_f, it_g, limited;
    double rho, RT, u[2], kn;
    double *c, *wf, *wg;
    int *d;
    /* no-slip walls: per real point, the wall face it crosses (2 low, 3
     * high) or -1; per face the image populations that leave it (count,
     * velocities before the reflection, landing displacements, scaled
     * weights), or fallback[face] = 1: the absorbed points are reflected
     * specularly instead (no image population crosses the face) */
    signed char *wall;
    int qi[2];
    double *ci[2], *wfi[2], *wgi[2];
    int *di[2];
    int fallback[2];
} cell_out;

static int pad_w(const orc_params *p, int face)
{
    int b = p->bc[face];
    return (b == ORC_BC_OUTFLOW || b == ORC_BC_INFLOW) ? p->pad : 0;
}

/* Moments of source cell (sx, sy) of the padded domain (Sec. III.A): interior
 * cells read the state; a pad cell takes the inflow equilibrium if one of its
 * pad faces is an inflow, else a copy of the nearest interior cell
 * (zero-gradient outflow, non-equilibrium kept). */
static void source_moments(const orc_params *p, const double *in, int sx, int sy, double *m)
{
    int nx = p->nx, ny = p->ny, nm = orc_num_moments(p->dim);
    long n = (long)nx * ny;
    int inflow = 0;
    if (sx < 0 && p->bc[0] == ORC_BC_INFLOW) inflow = 1;
    if (sx >= nx && p->bc[1] == ORC_BC_INFLOW) inflow = 1;
    if (sy < 0 && p->bc[2] == ORC_BC_INFLOW) inflow = 1;
    if (sy >= ny && p->bc[3] == ORC_BC_INFLOW) inflow = 1;
    if (inflow) {
        eq_moments(p->dim, p->K, p->in_rho, p->in_u[0], p->in_u[1], p->in_RT, m);
        return;
    }
    int ix = sx < 0 ? 0 : (sx >= nx ? nx - 1 : sx);
    int iy = sy < 0 ? 0 : (sy >= ny ? ny - 1 : sy);
    for (int k = 0; k < nm; k++) m[k] = in[(long)k * n + (long)iy * nx + ix];
}

static int has_walls(const orc_params *p)
{
    return p->dim == 2 && (p->bc[2] == ORC_BC_WALL || p->bc[3] == ORC_BC_WALL);
}

/* ------------------------------------------------------------------------ */
/* Extended bounce-back at the no-slip walls of the y faces, Sec. III.B.      */
/*                                                                            */
/* A real population whose straight path crosses a wall face n is absorbed:   */
/* its moment fractions add to the imbalances Delta m_n (fluons) and          */
/* Delta g_n (phonons) of its source (Eq. IIIB8) instead of streaming.  For   */
/* each face with Delta m_n > 0 the source reconstructs image populations     */
/* with the same normalised post-collision targets (non-equilibrium part of   */
/* the cell, Eqs. IIIB9-10; RT unchanged: adiabatic) on the acoustic stencil  */
/* of the image velocity u_n = u - 2 u_w (Eq. IIIB11; u_w along x, no slip    */
/* direction) (Eq. IIIB13), streams them with -c_i, and keeps those whose     */
/* path crosses face n (the last wall they touch: one reflection, the channel */
/* being wider than the reach); their sum is Delta m'_n (Eq. IIIB14).  They   */
/* land at the mirror image of x - d_i across the face with velocity          */
/* (-c_x, c_y), scaled by Delta m_n / Delta m'_n (Eq. IIIB15).                */
/* Readings: phonons are scaled by their own ratio Delta g_n / Delta g'_n, so */
/* the wall returns the internal energy of the extra degrees of freedom it    */
/* absorbed as it returns the mass; when no image population crosses the     */
/* face (flow toward the wall faster than the image stencil reaches back),    */
/* the absorbed populations are reflected specularly instead.  A stencil that */
/* crosses both faces, a refined stencil that crosses one, and a population  */
/* that would land only after a second reflection are reported (ORC_EREACH). */
/* ------------------------------------------------------------------------ */
static int wall_images(const orc_params *p, int sx, int sy, const orc_cell *cl, cell_out *co,
                       const double *dm, const double *dg)
{
    for (int f = 0; f < 2; f++) {
        co->qi[f] = 0; co->ci[f] = NULL; co->wfi[f] = NULL; co->wgi[f] = NULL; co->di[f] = NULL; co->fallback[f] = 0;
    }
    for (int f = 0; f < 2; f++) {
        if (!(dm[f] > 0.0)) continue;
        double un[2] = {cl->u[0] - 2.0 * p->wall_u[2 + f], cl->u[1]};
        int cap = 64, q;
        double *c = NULL, *dC = NULL;
        int *d = NULL;
        for (;;) {
            c = malloc(sizeof(double) * 2 * cap); dC = malloc(sizeof(double) * cap); d = malloc(sizeof(int) * 2 * cap);
            q = orc_las(2, un, cl->RT, p->n_conf, p->r_min, cap, c, dC, d, NULL);
            if (q >= 0) break;
            free(c); free(dC); free(d);
            cap = -q;
        }
        double *pf = malloc(sizeof(double) * q), *pg = malloc(sizeof(double) * q);
        double lf[10], lg[10];
        int itf = 0, itg = 0;
        int s1 = orc_epr(2, cl->nf, q, c, dC, un, cl->RT, cl->m, 0, lf, p->newton_tol, p->newton_max_it, pf, &itf);
        int s2 = orc_epr(2, cl->ng, q, c, dC, un, cl->RT, cl->n, 0, lg, p->newton_tol, p->newton_max_it, pg, &itg);
        free(dC);
        if (s1 != ORC_OK || s2 != ORC_OK) { free(c); free(d); free(pf); free(pg); return ORC_EEPR; }
        double sg = cl->rho_post * p->K * cl->RT;
        double dmi = 0.0, dgi = 0.0;
        int keep = 0;
        for (int i = 0; i < q; i++) {
            pf[i] *= cl->rho_post; pg[i] *= sg;
            int yu = sy - d[2 * i + 1];                       /* unfolded end of the -c_i path */
            int cross = f == 0 ? yu < 0 : yu > p->ny - 1;
            if (!cross) continue;
            int ly = f == 0 ? -1 - yu : 2 * p->ny - 1 - yu;    /* mirror image across the face */
            if (ly < 0 || ly > p->ny - 1) { free(c); free(d); free(pf); free(pg); return ORC_EREACH; }
            dmi += pf[i]; dgi += pg[i];
            c[2 * keep] = c[2 * i]; c[2 * keep + 1] = c[2 * i + 1];
            d[2 * keep] = d[2 * i]; d[2 * keep + 1] = d[2 * i + 1];
            pf[keep] = pf[i]; pg[keep] = pg[i];
            keep++;
        }
        if (!(dmi > 0.0) || !(dgi > 0.0)) {
            co->fallback[f] = 1;
            free(c); free(d); free(pf); free(pg);
            continue;
        }
        for (int i = 0; i < keep; i++) { pf[i] *= dm[f] / dmi; pg[i] *= dg[f] / dgi; }
        co->qi[f] = keep; co->ci[f] = c; co->di[f] = d; co->wfi[f] = pf; co->wgi[f] = pg;
    }
    return ORC_OK;
}

static void process_cell(const orc_params *p, const double *mom, double src, int sx, int sy, cell_out *co)
{
    orc_cell cl;
    memset(co, 0, sizeof(*co));
    int st = collide_src(p, mom, src, &cl);
    if (st != ORC_OK) { co->status = st; return; }
    co->rho = cl.rho; co->RT = cl.RT; co->u[0] = cl.u[0]; co->u[1] = cl.u[1];
    co->kn = cl.kn; co->limited = cl.limited;
    int cap = 64;
    double *c = NULL, *dC = NULL;
    int *d = NULL;
    int q;
    for (;;) {
        c = malloc(sizeof(double) * 2 * cap); dC = malloc(sizeof(double) * cap); d = malloc(sizeof(int) * 2 * cap);
        q = orc_las(p->dim, cl.u, cl.RT, p->n_conf, p->r_min, cap, c, dC, d, NULL);
        if (q >= 0) break;
        free(c); free(dC); free(d);
        cap = -q;
    }
    double *pf = malloc(sizeof(double) * q), *pg = malloc(sizeof(double) * q);
    double lf[10], lg[10];
    int itf = 0, itg = 0;
    int s1 = orc_epr(p->dim, cl.nf, q, c, dC, cl.u, cl.RT, cl.m, 0, lf, p->newton_tol, p->newton_max_it, pf, &itf);
    int s2 = orc_epr(p->dim, cl.ng, q, c, dC, cl.u, cl.RT, cl.n, 0, lg, p->newton_tol, p->newton_max_it, pg, &itg);
    free(dC);
    if (s1 != ORC_OK || s2 != ORC_OK) {
        co->status = ORC_EEPR;
        free(c); free(d); free(pf); free(pg);
        return;
    }
    /* moment fractions, Eq. (IIE3a): rho f' and rho K RT g' (rho plus the  */
    /* source's mass at the source cell)                                     */
    double sg = cl.rho_post * p->K * cl.RT;
    for (int i = 0; i < q; i++) { pf[i] *= cl.rho_post; pg[i] *= sg; }
    co->q = q; co->c = c; co->d = d; co->wf = pf; co->wg = pg;
    co->it_f = itf; co->it_g = itg;
    co->status = ORC_OK;
    if (has_walls(p)) {
        co->wall = malloc((size_t)(q > 0 ? q : 1));
        double dm[2] = {0.0, 0.0}, dg[2] = {0.0, 0.0};
        for (int i = 0; i < q; i++) {
            int yu = sy + d[2 * i + 1];
            int f = -1;
            if (p->bc[2] == ORC_BC_WALL && yu < 0) f = 0;
            else if (p->bc[3] == ORC_BC_WALL && yu > p->ny - 1) f = 1;
            co->wall[i] = (signed char)f;
            if (f >= 0) { dm[f] += pf[i]; dg[f] += pg[i]; }
        }
        if ((dm[0] > 0.0 && dm[1] > 0.0) || ((dm[0] > 0.0 || dm[1] > 0.0) && orc_las_levels(cl.RT) > 0)) {
            co->status = ORC_EREACH;
            return;
        }
        int st2 = wall_images(p, sx, sy, &cl, co, dm, dg);
        if (st2 != ORC_OK) { co->status = st2; return; }
        /* a face that reflects its absorbed points specularly: each lands   */
        /* after a single reflection, or the stencil reaches too far         */
        for (int i = 0; i < q; i++) {
            int f = co->wall[i];
            if (f < 0 || !co->fallback[f]) continue;
            int yu = sy + d[2 * i + 1];
            int ly = f == 0 ? -1 - yu : 2 * p->ny - 1 - yu;
            if (ly < 0 || ly > p->ny - 1) { co->status = ORC_EREACH; return; }
        }
    }
}

/* Moment fraction deposit, Eq. (IIE3b), with absolute velocity c. */
static void deposit(int dim, double *acc, double cx, double cy, double wf, double wg)
{
    if (dim == 1) {
        acc[0] += wf;
        acc[1] += cx * wf;
        acc[2] += cx * cx * wf;
        acc[3] += cx * cx * cx * wf;
        acc[4] += wg;
        acc[5] += cx * wg;
    } else {
        double cc = cx * cx + cy * cy;
        acc[0] += wf;
        acc[1] += cx * wf;
        acc[2] += cy * wf;
        acc[3] += cx * cx * wf;
        acc[4] += cx * cy * wf;
        acc[5] += cy * cy * wf;
        acc[6] += cc * cx * wf;
        acc[7] += cc * cy * wf;
        acc[8] += wg;
        acc[9] += cx * wg;
        acc[10] += cy * wg;
    }
}

/* ------------------------------------------------------------------------ */
/* Path of one population, Sec. III.B.                                        */
/*                                                                            */
/* The population leaves the centre of cell (x, y) of the padded domain with  */
/* integer displacement (dx, dy).  Its straight path crosses the grid lines   */
/* x = const |dx| times and y = const |dy| times; the k-th crossing of the x  */
/* lines happens at path parameter (2k - 1) / (2|dx|), likewise for y.  The   */
/* crossings are taken in order of that parameter (compared exactly in        */
/* integers), an x crossing before a y crossing at the same parameter (the    */
/* path through a cell corner).  A crossing into a blocker -- a solid cell or */
/* the far side of a slip wall -- reverses that velocity component (specular  */
/* reflection) and the path stays in its cell; otherwise the path enters the  */
/* neighbouring cell.  Periodic axes wrap.  Reflection keeps |c| per          */
/* component, so mass and energy are exact.                                   */
/* Reading: the paper reflects paths at slip boundaries without fixing the     */
/* order of the two crossings at a corner; x first is our choice.  The walk   */
/* is reversible (undone by the same walk from the end with the velocity      */
/* reversed and y first at corners), so every (cell, velocity) pair is        */
/* reached by exactly one path.                                                */
/* ------------------------------------------------------------------------ */
static int blocked(const orc_params *p, int x, int y)
{
    if (x < 0 && p->bc[0] == ORC_BC_SLIPWALL) return 1;
    if (x >= p->nx && p->bc[1] == ORC_BC_SLIPWALL) return 1;
    if (p->dim == 2 && y < 0 && p->bc[2] == ORC_BC_SLIPWALL) return 1;
    if (p->dim == 2 && y >= p->ny && p->bc[3] == ORC_BC_SLIPWALL) return 1;
    if (p->solid && x >= 0 && x < p->nx && y >= 0 && y < p->ny && p->solid[(long)y * p->nx + x]) return 1;
    return 0;
}

static int wrap(int v, int n) { v %= n; return v < 0 ? v + n : v; }

static void walk_path(const orc_params *p, int x, int y, int dx, int dy, int *ex, int *ey, int *sgx, int *sgy)
{
    int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
    int sx = dx < 0 ? -1 : 1, sy = dy < 0 ? -1 : 1;
    int kx = 0, ky = 0;
    int perx = p->bc[0] == ORC_BC_PERIODIC, pery = p->dim == 2 && p->bc[2] == ORC_BC_PERIODIC;
    while (kx < ax || ky < ay) {
        /* next crossing: x if its parameter (2kx+1)/(2ax) is not larger */
        int takex;
        if (kx >= ax) takex = 0;
        else if (ky >= ay) takex = 1;
        else takex = (long)(2 * kx + 1) * ay <= (long)(2 * ky + 1) * ax;
        if (takex) {
            int nx_ = x + sx;
            if (perx) nx_ = wrap(nx_, p->nx);
            if (blocked(p, nx_, y)) sx = -sx; else x = nx_;
            kx++;
        } else {
            int ny_ = y + sy;
            if (pery) ny_ = wrap(ny_, p->ny);
            if (blocked(p, x, ny_)) sy = -sy; else y = ny_;
            ky++;
        }
    }
    *ex = x; *ey = y;
    *sgx = (dx == 0 || (sx < 0) == (dx < 0)) ? 1 : -1;
    *sgy = (dy == 0 || (sy < 0) == (dy < 0)) ? 1 : -1;
}

/* Exported for the tests: final cell and component signs of one path. */
void orc_walk(const orc_params *p, int x, int y, int dx, int dy, int *out)
{
    walk_path(p, x, y, dx, dy, &out[0], &out[1], &out[2], &out[3]);
}

/* ------------------------------------------------------------------------ */
/* Pad width, Sec. III (Fig. 5): the pads of an outflow or inflow face must   */
/* hold every source whose populations can land in the interior.  The cells   */
/* beyond a pad would be in the pad's own state (a zero-gradient copy of the  */
/* same interior cell, or the inflow equilibrium), so if a pad cell's stencil */
/* can reach farther toward the interior than the pad is wide, arrivals from  */
/* outside the padded domain are missing.  Reading: the reach toward the      */
/* interior is bounded by the stencil's box around the rounded velocity of    */
/* Eq. (IIC6), [u] + R (every base point has |c - u| <= R + 1/2, so          */
/* c <= [u] + R componentwise, and refined children land with their parent); */
/* a pad of width W must have [u_n] + R <= W, u_n the velocity component     */
/* toward the interior.  Returns 1 if source (sx, sy) breaks this.            */
/* ------------------------------------------------------------------------ */
static int pad_reach_exceeded(const orc_params *p, int sx, int sy, const double *u, double RT)
{
    int R = orc_las_radius(RT, p->n_conf, p->r_min);
    int bx = (int)round_half_up(u[0]), by = p->dim == 2 ? (int)round_half_up(u[1]) : 0;
    int wl = pad_w(p, 0), wr = pad_w(p, 1);
    int wb = p->dim == 2 ? pad_w(p, 2) : 0, wt = p->dim == 2 ? pad_w(p, 3) : 0;
    if (sx < 0 && bx + R > wl) return 1;
    if (sx >= p->nx && R - bx > wr) return 1;
    if (sy < 0 && by + R > wb) return 1;
    if (sy >= p->ny && R - by > wt) return 1;
    return 0;
}

int orc_step(const orc_params *p, const double *in, double *out, orc_stats *st)
{
    int D = p->dim, nx = p->nx, ny = p->ny;
    if ((D != 1 && D != 2) || nx <= 0 || ny <= 0 || (D == 1 && ny != 1) || !(p->K > 0.0)) return ORC_EINVAL;
    for (int ax = 0; ax < D; ax++) {
        int a = p->bc[2 * ax], b = p->bc[2 * ax + 1];
        if ((a == ORC_BC_PERIODIC) != (b == ORC_BC_PERIODIC)) return ORC_EINVAL;
    }
    for (int f = 0; f < 4; f++)
        if (p->bc[f] == ORC_BC_WALL && (D != 2 || f < 2)) return ORC_EINVAL;   /* walls: y faces, 2D */
    if (has_walls(p) && p->solid) return ORC_EINVAL;
    if (has_walls(p))
        for (int f = 0; f < 4; f++)
            if (p->bc[f] == ORC_BC_SLIPWALL) return ORC_EINVAL;   /* no-slip walls with slip walls: not supported */
    if (p->solid) {
        /* solids are 2D, and may not touch a pad face (its cells copy the
         * nearest interior cell) */
        if (D != 2) return ORC_EINVAL;
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                if (!p->solid[(long)y * nx + x]) continue;
                if ((x == 0 && pad_w(p, 0)) || (x == nx - 1 && pad_w(p, 1)) || (y == 0 && pad_w(p, 2)) ||
                    (y == ny - 1 && pad_w(p, 3)))
                    return ORC_EINVAL;
            }
    }
    int nm = orc_num_moments(D);
    long n = (long)nx * ny;
    int wl = pad_w(p, 0), wr = pad_w(p, 1);
    int wb = D == 2 ? pad_w(p, 2) : 0, wt = D == 2 ? pad_w(p, 3) : 0;
    int sxn = nx + wl + wr, syn = ny + wb + wt;
    long ns = (long)sxn * syn;
    double *acc = calloc((size_t)nm * n, sizeof(double));
    if (!acc) return ORC_ENOMEM;
    long chunk = 4096;
    cell_out *co = malloc(sizeof(cell_out) * chunk);
    if (!co) { free(acc); return ORC_ENOMEM; }
    orc_stats s;
    memset(&s, 0, sizeof(s));
    s.q_min = 1 << 30; s.rt_min = INFINITY; s.fail_cell = -1;
    int status = ORC_OK;
    for (long c0 = 0; c0 < ns && status == ORC_OK; c0 += chunk) {
        long c1 = c0 + chunk < ns ? c0 + chunk : ns;
        #pragma omp parallel for schedule(dynamic, 16)
        for (long k = c0; k < c1; k++) {
            int sx = (int)(k % sxn) - wl, sy = (int)(k / sxn) - wb;
            if (p->solid && sx >= 0 && sx < nx && sy >= 0 && sy < ny && p->solid[(long)sy * nx + sx]) {
                memset(&co[k - c0], 0, sizeof(cell_out));
                co[k - c0].status = 1;   /* no population */
                continue;
            }
            double m[11];
            source_moments(p, in, sx, sy, m);
            /* Eq. (VC1) at the time of this step's collision, Delta t = 1 */
            double src = 0.0;
            if (p->src_rate != 0.0 && sx == p->src_x && sy == p->src_y) src = p->src_rate * sin(p->src_omega * p->src_t);
            process_cell(p, m, src, sx, sy, &co[k - c0]);
        }
        /* serial, source-major deposit */
        for (long k = c0; k < c1; k++) {
            cell_out *o = &co[k - c0];
            if (o->status == 1) continue;   /* solid cell */
            int sx = (int)(k % sxn) - wl, sy = (int)(k / sxn) - wb;
            if (o->status == ORC_OK && pad_reach_exceeded(p, sx, sy, o->u, o->RT)) o->status = ORC_EREACH;
            if (o->status != ORC_OK) {
                if (status == ORC_OK) { status = o->status; s.fail_cell = k; s.fail_code = o->status; }
                continue;
            }
            s.cells++;
            s.it_sum_f += o->it_f; s.it_sum_g += o->it_g;
            if (o->it_f > s.it_max_f) s.it_max_f = o->it_f;
            if (o->it_g > s.it_max_g) s.it_max_g = o->it_g;
            s.q_sum += o->q;
            if (o->q < s.q_min) s.q_min = o->q;
            if (o->q > s.q_max) s.q_max = o->q;
            if (o->RT < s.rt_min) s.rt_min = o->RT;
            if (o->kn > s.kn_max) s.kn_max = o->kn;
            s.limited += o->limited;
            double umag = D == 2 ? sqrt(o->u[0] * o->u[0] + o->u[1] * o->u[1]) : fabs(o->u[0]);
            double colat = umag + orc_las_radius(o->RT, p->n_conf, p->r_min);   /* Eq. (IIC7) */
            if (colat > s.colat_max) s.colat_max = colat;
            for (int i = 0; i < o->q; i++) {
                /* the path of the (base) point, Sec. III.B; refined children
                 * follow their parent's path and flips */
                int lx, ly, fx, fy;
                if (o->wall && o->wall[i] >= 0) {
                    /* crosses a no-slip wall: absorbed, unless the face falls
                     * back to a specular reflection for this source */
                    int f = o->wall[i];
                    if (!o->fallback[f]) continue;
                    int yu = sy + o->d[2 * i + 1];
                    lx = sx + o->d[2 * i];
                    if (p->bc[0] == ORC_BC_PERIODIC) lx = wrap(lx, nx);
                    ly = f == 0 ? -1 - yu : 2 * ny - 1 - yu;
                    fx = 1; fy = -1;
                } else {
                    walk_path(p, sx, sy, o->d[2 * i], D == 2 ? o->d[2 * i + 1] : 0, &lx, &ly, &fx, &fy);
                }
                double cx = fx * o->c[2 * i], cy = fy * o->c[2 * i + 1];
                /* arrivals in pads are discarded (Sec. III.A) */
                if (lx < 0 || lx >= nx || ly < 0 || ly >= ny) continue;
                double a[11] = {0};
                deposit(D, a, cx, cy, o->wf[i], o->wg[i]);
                long dst = (long)ly * nx + lx;
                for (int mm = 0; mm < nm; mm++) acc[(long)mm * n + dst] += a[mm];
            }
            /* image populations of the no-slip walls: streamed with -c_i and
             * reflected by their face, velocity (-c_x, c_y) */
            for (int f = 0; f < 2; f++) {
                for (int i = 0; o->wall && i < o->qi[f]; i++) {
                    int yu = sy - o->di[f][2 * i + 1];
                    int lx = sx - o->di[f][2 * i];
                    if (p->bc[0] == ORC_BC_PERIODIC) lx = wrap(lx, nx);
                    int ly = f == 0 ? -1 - yu : 2 * ny - 1 - yu;
                    if (lx < 0 || lx >= nx) continue;
                    double a[11] = {0};
                    deposit(D, a, -o->ci[f][2 * i], o->ci[f][2 * i + 1], o->wfi[f][i], o->wgi[f][i]);
                    long dst = (long)ly * nx + lx;
                    for (int mm = 0; mm < nm; mm++) acc[(long)mm * n + dst] += a[mm];
                }
            }
        }
        for (long k = c0; k < c1; k++) {
            cell_out *o = &co[k - c0];
            free(o->c); free(o->d); free(o->wf); free(o->wg); free(o->wall);
            for (int f = 0; f < 2; f++) { free(o->ci[f]); free(o->di[f]); free(o->wfi[f]); free(o->wgi[f]); }
        }
    }
    if (status == ORC_OK) memcpy(out, acc, sizeof(double) * nm * n);
    free(acc);
    free(co);
    if (s.q_min == (1 << 30)) s.q_min = 0;
    if (st) *st = s;
    return status;
}

/* nsteps steps; on failure the state of the last completed step is left in
 * out and *done holds the number of completed steps. */
int orc_run(const orc_params *p, const double *in, double *out, int nsteps, orc_stats *st, int *done)
{
    int nm = orc_num_moments(p->dim);
    long n = (long)p->nx * p->ny;
    if (nm < 0 || n <= 0) return ORC_EINVAL;
    double *tmp = malloc(sizeof(double) * nm * n);
    if (!tmp) return ORC_ENOMEM;
    memcpy(out, in, sizeof(double) * nm * n);
    orc_stats acc;
    memset(&acc, 0, sizeof(acc));
    acc.q_min = 1 << 30; acc.rt_min = INFINITY; acc.fail_cell = -1;
    int status = ORC_OK, k;
    orc_params pk = *p;
    for (k = 0; k < nsteps; k++) {
        orc_stats s;
        pk.src_t = p->src_t + k;
        status = orc_step(&pk, out, tmp, &s);
        if (status != ORC_OK) { acc.fail_cell = s.fail_cell; acc.fail_code = s.fail_code; break; }
        memcpy(out, tmp, sizeof(double) * nm * n);
        acc.cells += s.cells; acc.it_sum_f += s.it_sum_f; acc.it_sum_g += s.it_sum_g;
        if (s.it_max_f > acc.it_max_f) acc.it_max_f = s.it_max_f;
        if (s.it_max_g > acc.it_max_g) acc.it_max_g = s.it_max_g;
        acc.q_sum += s.q_sum;
        if (s.q_min < acc.q_min) acc.q_min = s.q_min;
        if (s.q_max > acc.q_max) acc.q_max = s.q_max;
        acc.limited += s.limited;
        if (s.rt_min < acc.rt_min) acc.rt_min = s.rt_min;
        if (s.kn_max > acc.kn_max) acc.kn_max = s.kn_max;
        if (s.colat_max > acc.colat_max) acc.colat_max = s.colat_max;
    }
    free(tmp);
    if (acc.q_min == (1 << 30)) acc.q_min = 0;
    if (st) *st = acc;
    if (done) *done = k;
    return status;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
