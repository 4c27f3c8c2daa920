/*
 * Plain FP64 CPU oracle of one LELBM time step in three dimensions
 * (arXiv 2508.06911) -- TEST INFRASTRUCTURE ONLY, like lelbm_oracle.c: the
 * GPU library never links, loads or calls it.
 *
 * The method is the one of the 1D/2D oracle with D = 3, written out on its
 * own so that each stage can be read against the paper with D = 3:
 *   - macroscopic variables ............ Eq. (IIB6a-c)
 *   - non-equilibrium central moments .. Eqs. (IIB9a-d)
 *   - bulk/shear split ................. Eqs. (IIB10-11)
 *   - third-order per-axis split ....... Eq. (IIB14)
 *   - Knudsen limiter .................. App. D, Eqs. (D2-D3) (the wording
 *                                        after Eq. (D3b))
 *   - post-collision central moments ... Eqs. (IIB16a-f, IIB17), normalised
 *                                        by Eq. (IIB18)
 *   - Lagrangian acoustic stencil ...... Eq. (IIC6): integer c in the ball
 *                                        |c - u| <= R + 1/2
 *   - entropic reconstruction .......... Eqs. (IID7-11, IID13)
 *   - moment streaming ................. Eqs. (IIE3a-b)
 *
 * Stored values per cell (Sec. II.E: 13 + 4 in 3D), SoA [moment][z][y][x]:
 *   M0 Mx My Mz Mxx Mxy Mxz Myy Myz Mzz MDx MDy MDz G0 Gx Gy Gz
 * Fluon constraints (19), relative velocity c~ = c - u:
 *   1, x, y, z, xx, xy, xz, yy, yz, zz,
 *   xxx, xxy, xxz, xyy, yyy, yyz, xzz, yzz, zzz
 * the third-order ones being the per-axis pieces M~_{aa|g} of Eq. (IIB14)
 * in the order (xx|x), (xx|y), (xx|z), (yy|x), (yy|y), (yy|z), (zz|x), (zz|y),
 * (zz|z).  Phonon constraints (10): the first ten; the second-order ones are
 * RT delta_ab (Eq. IIB17).
 *
 * Scope: fully periodic boxes, or an open box (a window cut out of a larger
 * domain: it has no sources outside, and populations landing outside it are
 * dropped; only cells farther than the reach from its faces see the step of
 * the larger domain).  Stencils are refined as in 2D (Eqs. IIC9-11 with 2^3
 * children per refined point); more than 3 levels (RT < 0.0123) or radii
 * above 64 are reported as ORC3_EREACH.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC3_STALL_RES 1e-10
#define ORC3_NF 19
#define ORC3_NG 10
#define ORC3_NMOM 17

enum { ORC3_OK = 0, ORC3_EINVAL = -1, ORC3_ENOMEM = -2, ORC3_EEPR = -4, ORC3_ENONFINITE = -5, ORC3_EREACH = -6 };

/* Parameters of one 3D run.  Mirrored by the Python wrapper. */
typedef struct {
    int nx, ny, nz;
    double K;
    double omega_f, omega_b, omega_h;
    double n_conf;
    int r_min;
    double newton_tol;
    int newton_max_it;
    int kn_limiter;
    double kn_lo, kn_hi, omega_H;
    int open;            /* 0: periodic box; 1: open box (window, see above) */
} orc3_params;

typedef struct {
    long cells;
    long it_sum_f, it_sum_g;
    int it_max_f, it_max_g;
    long q_sum; int q_min, q_max;
    long limited;
    double rt_min, kn_max;
    long fail_cell; int fail_code;
} orc3_stats;

/* ------------------------------------------------------------------------ */
/* Equilibrium raw moments (App. A, Eqs. A3a-d, A7a-b) with D = 3:            */
/* M0 = rho, M_a = rho u_a, M_ab = rho (u_a u_b + RT delta_ab),               */
/* M_Dg = rho (|u|^2 + 5 RT) u_g, G0 = rho K RT, G_g = rho K RT u_g.          */
/* ------------------------------------------------------------------------ */
static void eq_moments3(double K, double rho, const double *u, double RT, double *m)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    m[0] = rho;
    for (int a = 0; a < 3; a++) m[1 + a] = rho * u[a];
    int k = 4;
    for (int a = 0; a < 3; a++)
        for (int b = a; b < 3; b++) m[k++] = rho * (u[a] * u[b] + (a == b ? RT : 0.0));
    for (int g = 0; g < 3; g++) m[10 + g] = rho * (uu + 5.0 * RT) * u[g];
    m[13] = rho * K * RT;
    for (int g = 0; g < 3; g++) m[14 + g] = rho * K * RT * u[g];
}

int orc3_moments_from_primitives(double K, long n, const double *rho, const double *ux, const double *uy,
                                 const double *uz, const double *RT, double *out)
{
    if (n < 0) return ORC3_EINVAL;
    for (long i = 0; i < n; i++) {
        double m[ORC3_NMOM], u[3] = {ux[i], uy[i], uz[i]};
        eq_moments3(K, rho[i], u, RT[i], m);
        for (int k = 0; k < ORC3_NMOM; k++) out[(long)k * n + i] = m[k];
    }
    return ORC3_OK;
}

/* ------------------------------------------------------------------------ */
/* Collision, Eqs. (IIB6-IIB18) with D = 3 and the Knudsen limiter of App. D  */
/* (same readings as the 2D oracle: Eq. (D2) numerators over rho, L1 sums over */
/* all components; limiter as worded after Eq. (D3b)).                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double rho, u[3], RT;
    double P[3][3], Q[3], g0, h[3];
    double kn, om_f, om_b, om_h;
    int limited;
    double m[ORC3_NF], n[ORC3_NG];
} orc3_cell;

static double limit_omega3(double kn, double om, const orc3_params *p)
{
    double lo = pow(10.0, p->kn_lo), hi = pow(10.0, p->kn_hi);
    if (kn < lo) return om;
    if (kn > hi) return p->omega_H;
    return (p->omega_H - om) / (p->kn_hi - p->kn_lo) * (log10(kn) - p->kn_lo) + om;
}

/* index of M_ab in the stored layout (4 + upper-triangle position) */
static int sec_idx(int a, int b)
{
    static const int t[3][3] = {{4, 5, 6}, {5, 7, 8}, {6, 8, 9}};
    return t[a][b];
}

static int collide3(const orc3_params *p, const double *mom, orc3_cell *c)
{
    const int D = 3;
    double K = p->K;
    memset(c, 0, sizeof(*c));
    double rho = mom[0];
    if (!(rho > 0.0) || !isfinite(rho)) return ORC3_EEPR;
    double u[3], uu = 0.0;
    for (int a = 0; a < 3; a++) { u[a] = mom[1 + a] / rho; uu += u[a] * u[a]; }
    double G0 = mom[13];
    double RT = ((mom[4] + mom[7] + mom[9] + G0) / rho - uu) / (D + K);
    if (!(RT > 0.0) || !isfinite(RT)) return ORC3_EEPR;
    c->rho = rho; c->RT = RT;
    for (int a = 0; a < 3; a++) c->u[a] = u[a];
    /* Eq. (IIB9a) */
    double P[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) P[a][b] = mom[sec_idx(a, b)] - rho * (u[a] * u[b] + (a == b ? RT : 0.0));
    /* Eq. (IIB9b) */
    double trP = P[0][0] + P[1][1] + P[2][2];
    double Q[3];
    for (int g = 0; g < 3; g++) {
        double s = 0.0;
        for (int a = 0; a < 3; a++) s += u[a] * P[a][g];
        Q[g] = mom[10 + g] - 2.0 * s - u[g] * trP - rho * (uu + (D + 2) * RT) * u[g];
    }
    /* Eqs. (IIB9c-d) */
    double g0 = G0 - rho * K * RT, h[3];
    for (int g = 0; g < 3; g++) h[g] = mom[14 + g] - u[g] * G0;
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) c->P[a][b] = P[a][b];
        c->Q[a] = Q[a]; c->h[a] = h[a];
    }
    c->g0 = g0;
    /* Eq. (D2) */
    double sP = 0.0, sQ = 0.0;
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) sP += fabs(P[a][b]);
        sQ += fabs(Q[a]) + fabs(h[a]);
    }
    double knA = (sP + fabs(g0)) / (rho * (D + K) * RT);
    double knB = sQ / (rho * (D + K + 2.0) * pow(RT, 1.5));
    double kn = knA > knB ? knA : knB;
    c->kn = kn;
    double of = p->omega_f, ob = p->omega_b, oh = p->omega_h;
    if (p->kn_limiter) {
        of = limit_omega3(kn, p->omega_f, p);
        ob = limit_omega3(kn, p->omega_b, p);
        oh = limit_omega3(kn, p->omega_h, p);
        c->limited = (of != p->omega_f) || (ob != p->omega_b) || (oh != p->omega_h);
    }
    c->om_f = of; c->om_b = ob; c->om_h = oh;
    /* Eqs. (IIB10-11, IIB14) */
    double bulk[3][3] = {{0}}, shear[3][3], t[3][3];
    for (int a = 0; a < 3; a++) bulk[a][a] = -g0 / D;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) shear[a][b] = P[a][b] - bulk[a][b];
    for (int a = 0; a < 3; a++)
        for (int g = 0; g < 3; g++) t[a][g] = (1.0 + 2.0 * (a == g)) / (D + 2) * Q[g];
    /* Eqs. (IIB16-18) */
    c->m[0] = 1.0;
    for (int a = 0; a < 3; a++) c->m[1 + a] = 0.0;
    int k = 4;
    for (int a = 0; a < 3; a++)
        for (int b = a; b < 3; b++)
            c->m[k++] = RT * (a == b) + ((1.0 - of) * shear[a][b] + (1.0 - ob) * bulk[a][b]) / rho;
    for (int a = 0; a < 3; a++)
        for (int g = 0; g < 3; g++) c->m[10 + 3 * a + g] = (1.0 - oh) * t[a][g] / rho;
    double rKT = rho * K * RT;
    c->n[0] = 1.0 + (1.0 - ob) * g0 / rKT;
    for (int g = 0; g < 3; g++) c->n[1 + g] = (1.0 - oh) * h[g] / rKT;
    k = 4;
    for (int a = 0; a < 3; a++)
        for (int b = a; b < 3; b++) c->n[k++] = a == b ? RT : 0.0;
    return ORC3_OK;
}

/* Flat export for the tests: [rho, ux, uy, uz, RT, kn, om_f, om_b, om_h,
 * limited, P (9, row-major), Q (3), g0, h (3), m (19), n (10)] */
int orc3_collide_flat(const orc3_params *p, const double *mom, double *out)
{
    orc3_cell c;
    int st = collide3(p, mom, &c);
    int k = 0;
    out[k++] = c.rho;
    for (int a = 0; a < 3; a++) out[k++] = c.u[a];
    out[k++] = c.RT; out[k++] = c.kn; out[k++] = c.om_f; out[k++] = c.om_b; out[k++] = c.om_h;
    out[k++] = (double)c.limited;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) out[k++] = c.P[a][b];
    for (int a = 0; a < 3; a++) out[k++] = c.Q[a];
    out[k++] = c.g0;
    for (int a = 0; a < 3; a++) out[k++] = c.h[a];
    for (int j = 0; j < ORC3_NF; j++) out[k++] = c.m[j];
    for (int j = 0; j < ORC3_NG; j++) out[k++] = c.n[j];
    return st;
}

/* ------------------------------------------------------------------------ */
/* Stencil, Eqs. (IIC6, IIC9): R = max([n sqrt(RT)], r_min), [x] = floor(x +  */
/* 1/2); the points are the integer c with |c - u| <= R + 1/2, enumerated     */
/* z-major, then y, then x.  Returns q (or -needed if cap is too small), or   */
/* ORC3_EREACH for a stencil that would be refined (N_r > 0) or R > 64.       */
/* ------------------------------------------------------------------------ */
static double rhu(double x) { return floor(x + 0.5); }

int orc3_las_radius(double RT, double n_conf, int r_min)
{
    int R = (int)rhu(n_conf * sqrt(RT));
    return R > r_min ? R : r_min;
}

int orc3_las_levels(double RT) { return (int)rhu(1.0 / (3.0 * sqrt(RT))); }

/* Fills c[3i] (velocity), dC[i] (velocity volume) and d[3i] (landing      */
/* displacement: the integer ancestor) for i < q and returns q, -q_needed if */
/* cap is too small, or ORC3_EREACH.  Refinement (Eqs. IIC10-11, the 2D      */
/* readings with D = 3): for Lvl = 1..N_r every point whose distance to u is  */
/* at most 3 2^-Lvl is replaced by its 8 children at c + (+-h/4, +-h/4,     */
/* +-h/4) (h its spacing), each with a volume of 1/8 of the parent's; the  */
/* children follow the parent in the order (-,-,-), (+,-,-), (-,+,-), ...   */
/* (x fastest).                                                             */
int orc3_las(const double *u, double RT, double n_conf, int r_min, int cap, double *c, double *dC, int *d)
{
    int Nr = orc3_las_levels(RT);
    int R = orc3_las_radius(RT, n_conf, r_min);
    if (Nr > 3 || R > 64) return ORC3_EREACH;
    double rr = R + 0.5;
    int b[3];
    for (int a = 0; a < 3; a++) b[a] = (int)rhu(u[a]);
    int nbase = 0;
    for (int cz = b[2] - R - 1; cz <= b[2] + R + 1; cz++)
        for (int cy = b[1] - R - 1; cy <= b[1] + R + 1; cy++)
            for (int cx = b[0] - R - 1; cx <= b[0] + R + 1; cx++) {
                double ex = cx - u[0], ey = cy - u[1], ez = cz - u[2];
                if (ex * ex + ey * ey + ez * ez <= rr * rr) nbase++;
            }
    int nmax = nbase;
    for (int l = 0; l < Nr; l++) nmax *= 8;
    double *tc = malloc(sizeof(double) * 3 * nmax), *tdc = malloc(sizeof(double) * nmax);
    double *th = malloc(sizeof(double) * nmax), *nc = malloc(sizeof(double) * 3 * nmax);
    double *ndc = malloc(sizeof(double) * nmax), *nh = malloc(sizeof(double) * nmax);
    int *td = malloc(sizeof(int) * 3 * nmax), *nd = malloc(sizeof(int) * 3 * nmax);
    int q = 0;
    if (tc && tdc && th && nc && ndc && nh && td && nd) {
        for (int cz = b[2] - R - 1; cz <= b[2] + R + 1; cz++)
            for (int cy = b[1] - R - 1; cy <= b[1] + R + 1; cy++)
                for (int cx = b[0] - R - 1; cx <= b[0] + R + 1; cx++) {
                    double ex = cx - u[0], ey = cy - u[1], ez = cz - u[2];
                    if (ex * ex + ey * ey + ez * ez > rr * rr) continue;
                    tc[3 * q] = cx; tc[3 * q + 1] = cy; tc[3 * q + 2] = cz;
                    td[3 * q] = cx; td[3 * q + 1] = cy; td[3 * q + 2] = cz;
                    tdc[q] = 1.0; th[q] = 1.0;
                    q++;
                }
        for (int lvl = 1; lvl <= Nr; lvl++) {
            double thr = 3.0 * pow(0.5, lvl);
            int m = 0;
            for (int i = 0; i < q; i++) {
                double ex = tc[3 * i] - u[0], ey = tc[3 * i + 1] - u[1], ez = tc[3 * i + 2] - u[2];
                if (sqrt(ex * ex + ey * ey + ez * ez) <= thr) {
                    double h = th[i];
                    for (int k = 0; k < 8; k++) {
                        double sg[3] = {(k & 1) ? 1.0 : -1.0, (k & 2) ? 1.0 : -1.0, (k & 4) ? 1.0 : -1.0};
                        for (int a = 0; a < 3; a++) {
                            nc[3 * m + a] = tc[3 * i + a] + sg[a] * h / 4.0;
                            nd[3 * m + a] = td[3 * i + a];
                        }
                        ndc[m] = tdc[i] / 8.0;
                        nh[m] = h / 2.0;
                        m++;
                    }
                } else {
                    for (int a = 0; a < 3; a++) { nc[3 * m + a] = tc[3 * i + a]; nd[3 * m + a] = td[3 * i + a]; }
                    ndc[m] = tdc[i]; nh[m] = th[i];
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
    }
    int ret = q <= cap ? q : -q;
    if (q <= cap)
        for (int i = 0; i < q; i++) {
            for (int a = 0; a < 3; a++) { c[3 * i + a] = tc[3 * i + a]; d[3 * i + a] = td[3 * i + a]; }
            dC[i] = tdc[i];
        }
    free(tc); free(tdc); free(th); free(nc); free(ndc); free(nh); free(td); free(nd);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* Entropic reconstruction, Eqs. (IID7-11, IID13), as in the 2D oracle:        */
/* f_i = exp(-(1 + sum_j lambda_j T_j(c~_i))), Newton on the convex dual with  */
/* Cholesky, Armijo backtracking while the decrement exceeds 1e-8, the scaled  */
/* residual max_j |r_j| / RT^(k_j/2) as the stop test, the stalled-residual    */
/* rule below 1e-10, and one polishing update after the stop.                  */
/* ------------------------------------------------------------------------ */
static void basis3(int nb, const double *ct, double *T, int *order)
{
    double x = ct[0], y = ct[1], z = ct[2];
    double v[ORC3_NF] = {1.0, x, y, z, x * x, x * y, x * z, y * y, y * z, z * z,
                         x * x * x, x * x * y, x * x * z, x * y * y, y * y * y, y * y * z, x * z * z, y * z * z,
                         z * z * z};
    static const int o[ORC3_NF] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3};
    for (int j = 0; j < nb; j++) { T[j] = v[j]; if (order) order[j] = o[j]; }
}

static int epr3_eval(int nb, int q, const double *c, const double *dC, const double *u, const double *lam,
                     const double *target, double *pop, double *phi, double *r, double *A)
{
    double s[ORC3_NF] = {0};
    for (int i = 0; i < nb * nb; i++) A[i] = 0.0;
    double sum = 0.0;
    for (int i = 0; i < q; i++) {
        double ct[3] = {c[3 * i] - u[0], c[3 * i + 1] - u[1], c[3 * i + 2] - u[2]};
        double T[ORC3_NF];
        basis3(nb, ct, T, NULL);
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
    if (!isfinite(*phi)) return ORC3_ENONFINITE;
    for (int j = 0; j < nb; j++) if (!isfinite(r[j])) return ORC3_ENONFINITE;
    return ORC3_OK;
}

static int chol3(int nb, const double *A, const double *b, double *x)
{
    double L[ORC3_NF * ORC3_NF] = {0}, y[ORC3_NF];
    for (int i = 0; i < nb; i++)
        for (int j = 0; j <= i; j++) {
            double s = A[i * nb + j];
            for (int k = 0; k < j; k++) s -= L[i * nb + k] * L[j * nb + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return ORC3_EEPR;
                L[i * nb + i] = sqrt(s);
            } else {
                L[i * nb + j] = s / L[j * nb + j];
            }
        }
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
    return ORC3_OK;
}

/* Eq. (IID13) with D = 3: lambda_0 = -1 + (3/2) log(2 pi RT), lambda_aa = 1/(2 RT) */
void orc3_epr_initial(int nb, double RT, double *lam)
{
    for (int j = 0; j < nb; j++) lam[j] = 0.0;
    lam[0] = -1.0 + 1.5 * log(2.0 * M_PI * RT);
    lam[4] = lam[7] = lam[9] = 1.0 / (2.0 * RT);
}

int orc3_epr(int nb, int q, const double *c, const double *dC, const double *u, double RT, const double *target,
             int use_init, double *lam, double tol, int maxit, double *pop, int *iters)
{
    double r[ORC3_NF], A[ORC3_NF * ORC3_NF], dl[ORC3_NF], lt[ORC3_NF], rt[ORC3_NF], At[ORC3_NF * ORC3_NF];
    double phi, phit, Tz[ORC3_NF], zero[3] = {0, 0, 0};
    int order[ORC3_NF];
    basis3(nb, zero, Tz, order);
    if (!use_init) orc3_epr_initial(nb, RT, lam);
    double *popt = malloc(sizeof(double) * (q > 0 ? q : 1));
    if (!popt) return ORC3_ENOMEM;
    if (epr3_eval(nb, q, c, dC, u, lam, target, pop, &phi, r, A) != ORC3_OK) { free(popt); return ORC3_EEPR; }
    int nit = 0;
    double res_prev = INFINITY;
    for (;;) {
        double res = 0.0;
        for (int j = 0; j < nb; j++) {
            double v = fabs(r[j]) / pow(RT, 0.5 * order[j]);
            if (v > res) res = v;
        }
        if (res <= tol) break;
        if (nit > 0 && res <= ORC3_STALL_RES && !(res < res_prev)) break;
        res_prev = res;
        if (nit >= maxit || chol3(nb, A, r, dl) != ORC3_OK) { free(popt); return ORC3_EEPR; }
        double dec = 0.0;
        for (int j = 0; j < nb; j++) dec += r[j] * dl[j];
        double t = 1.0;
        int ok = 0;
        for (int ls = 0; ls <= 30; ls++) {
            for (int j = 0; j < nb; j++) lt[j] = lam[j] + t * dl[j];
            int s2 = epr3_eval(nb, q, c, dC, u, lt, target, popt, &phit, rt, At);
            if (s2 == ORC3_OK && (dec <= 1e-8 || phit <= phi - 1e-4 * t * dec)) { ok = 1; break; }
            t *= 0.5;
        }
        if (!ok) { free(popt); return ORC3_EEPR; }
        for (int j = 0; j < nb; j++) { lam[j] = lt[j]; r[j] = rt[j]; }
        for (int j = 0; j < nb * nb; j++) A[j] = At[j];
        phi = phit;
        nit++;
    }
    if (chol3(nb, A, r, dl) != ORC3_OK) { free(popt); return ORC3_EEPR; }
    for (int j = 0; j < nb; j++) lam[j] += dl[j];
    nit++;
    int st = epr3_eval(nb, q, c, dC, u, lam, target, pop, &phi, r, A);
    free(popt);
    if (st != ORC3_OK) return ORC3_EEPR;
    *iters = nit;
    return ORC3_OK;
}

/* ------------------------------------------------------------------------ */
/* One step: every cell collides, reconstructs both species on its stencil   */
/* and deposits the moment fractions rho f' and rho K RT g' (Eq. IIE3a) of   */
/* each point at x + c (wrapped on a periodic box, dropped outside an open    */
/* one) with velocity c (Eq. IIE3b).  Serial, source-major deposit.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int status, q, it_f, it_g, limited;
    double RT, kn;
    int *d;              /* landing displacements (integer ancestors) */
    double *c;           /* exact velocities */
    double *wf, *wg;
} cell3_out;

static void process_cell3(const orc3_params *p, const double *mom, cell3_out *co)
{
    orc3_cell cl;
    memset(co, 0, sizeof(*co));
    int st = collide3(p, mom, &cl);
    if (st != ORC3_OK) { co->status = st; return; }
    co->RT = cl.RT; co->kn = cl.kn; co->limited = cl.limited;
    int cap = 512, q;
    int *d = NULL;
    double *c = NULL, *dC = NULL;
    for (;;) {
        d = malloc(sizeof(int) * 3 * cap);
        c = malloc(sizeof(double) * 3 * cap);
        dC = malloc(sizeof(double) * cap);
        if (!d || !c || !dC) { free(d); free(c); free(dC); co->status = ORC3_ENOMEM; return; }
        q = orc3_las(cl.u, cl.RT, p->n_conf, p->r_min, cap, c, dC, d);
        if (q >= 0 || q == ORC3_EREACH) break;
        free(d); free(c); free(dC);
        cap = -q;
    }
    if (q == ORC3_EREACH) { free(d); free(c); free(dC); co->status = ORC3_EREACH; return; }
    double *pf = malloc(sizeof(double) * q), *pg = malloc(sizeof(double) * q);
    double lf[ORC3_NF], lg[ORC3_NG];
    int itf = 0, itg = 0;
    int s1 = orc3_epr(ORC3_NF, q, c, dC, cl.u, cl.RT, cl.m, 0, lf, p->newton_tol, p->newton_max_it, pf, &itf);
    int s2 = orc3_epr(ORC3_NG, q, c, dC, cl.u, cl.RT, cl.n, 0, lg, p->newton_tol, p->newton_max_it, pg, &itg);
    free(dC);
    if (s1 != ORC3_OK || s2 != ORC3_OK) {
        free(d); free(c); free(pf); free(pg);
        co->status = ORC3_EEPR;
        return;
    }
    double sg = cl.rho * p->K * cl.RT;
    for (int i = 0; i < q; i++) { pf[i] *= cl.rho; pg[i] *= sg; }
    co->q = q; co->d = d; co->c = c; co->wf = pf; co->wg = pg; co->it_f = itf; co->it_g = itg;
    co->status = ORC3_OK;
}

static int wrap3(int v, int n) { v %= n; return v < 0 ? v + n : v; }

int orc3_step(const orc3_params *p, const double *in, double *out, orc3_stats *st)
{
    int nx = p->nx, ny = p->ny, nz = p->nz;
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(p->K > 0.0)) return ORC3_EINVAL;
    long n = (long)nx * ny * nz;
    double *acc = calloc((size_t)ORC3_NMOM * n, sizeof(double));
    if (!acc) return ORC3_ENOMEM;
    long chunk = 2048;
    cell3_out *co = malloc(sizeof(cell3_out) * chunk);
    if (!co) { free(acc); return ORC3_ENOMEM; }
    orc3_stats s;
    memset(&s, 0, sizeof(s));
    s.q_min = 1 << 30; s.rt_min = INFINITY; s.fail_cell = -1;
    int status = ORC3_OK;
    for (long c0 = 0; c0 < n && status == ORC3_OK; c0 += chunk) {
        long c1 = c0 + chunk < n ? c0 + chunk : n;
        #pragma omp parallel for schedule(dynamic, 8)
        for (long k = c0; k < c1; k++) {
            double m[ORC3_NMOM];
            for (int j = 0; j < ORC3_NMOM; j++) m[j] = in[(long)j * n + k];
            process_cell3(p, m, &co[k - c0]);
        }
        for (long k = c0; k < c1; k++) {
            cell3_out *o = &co[k - c0];
            if (o->status != ORC3_OK) {
                if (status == ORC3_OK) { status = o->status; s.fail_cell = k; s.fail_code = o->status; }
                continue;
            }
            int sx = (int)(k % nx), sy = (int)((k / nx) % ny), sz = (int)(k / ((long)nx * ny));
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
            for (int i = 0; i < o->q; i++) {
                /* lands in the cell of its integer ancestor, with its exact velocity */
                int tx = sx + o->d[3 * i], ty = sy + o->d[3 * i + 1], tz = sz + o->d[3 * i + 2];
                if (p->open && (tx < 0 || tx >= nx || ty < 0 || ty >= ny || tz < 0 || tz >= nz)) continue;
                long dst = ((long)wrap3(tz, nz) * ny + wrap3(ty, ny)) * nx + wrap3(tx, nx);
                double c[3] = {o->c[3 * i], o->c[3 * i + 1], o->c[3 * i + 2]};
                double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
                double wf = o->wf[i], wg = o->wg[i];
                double a[ORC3_NMOM];
                a[0] = wf;
                for (int g = 0; g < 3; g++) a[1 + g] = c[g] * wf;
                int kk = 4;
                for (int g = 0; g < 3; g++)
                    for (int h = g; h < 3; h++) a[kk++] = c[g] * c[h] * wf;
                for (int g = 0; g < 3; g++) a[10 + g] = cc * c[g] * wf;
                a[13] = wg;
                for (int g = 0; g < 3; g++) a[14 + g] = c[g] * wg;
                for (int j = 0; j < ORC3_NMOM; j++) acc[(long)j * n + dst] += a[j];
            }
        }
        for (long k = c0; k < c1; k++) {
            free(co[k - c0].d); free(co[k - c0].c); free(co[k - c0].wf); free(co[k - c0].wg);
        }
    }
    if (status == ORC3_OK) memcpy(out, acc, sizeof(double) * ORC3_NMOM * n);
    free(acc);
    free(co);
    if (s.q_min == (1 << 30)) s.q_min = 0;
    if (st) *st = s;
    return status;
}

int orc3_run(const orc3_params *p, const double *in, double *out, int nsteps, orc3_stats *st, int *done)
{
    long n = (long)p->nx * p->ny * p->nz;
    if (n <= 0) return ORC3_EINVAL;
    double *tmp = malloc(sizeof(double) * ORC3_NMOM * n);
    if (!tmp) return ORC3_ENOMEM;
    memcpy(out, in, sizeof(double) * ORC3_NMOM * n);
    orc3_stats acc;
    memset(&acc, 0, sizeof(acc));
    acc.q_min = 1 << 30; acc.rt_min = INFINITY; acc.fail_cell = -1;
    int status = ORC3_OK, k;
    for (k = 0; k < nsteps; k++) {
        orc3_stats s;
        status = orc3_step(p, out, tmp, &s);
        if (status != ORC3_OK) { acc.fail_cell = s.fail_cell; acc.fail_code = s.fail_code; break; }
        memcpy(out, tmp, sizeof(double) * ORC3_NMOM * n);
        acc.cells += s.cells; acc.it_sum_f += s.it_sum_f; acc.it_sum_g += s.it_sum_g;
        if (s.it_max_f > acc.it_max_f) acc.it_max_f = s.it_max_f;
        if (s.it_max_g > acc.it_max_g) acc.it_max_g = s.it_max_g;
        acc.q_sum += s.q_sum;
        if (s.q_min < acc.q_min) acc.q_min = s.q_min;
        if (s.q_max > acc.q_max) acc.q_max = s.q_max;
        acc.limited += s.limited;
        if (s.rt_min < acc.rt_min) acc.rt_min = s.rt_min;
        if (s.kn_max > acc.kn_max) acc.kn_max = s.kn_max;
    }
    free(tmp);
    if (acc.q_min == (1 << 30)) acc.q_min = 0;
    if (st) *st = acc;
    if (done) *done = k;
    return status;
}
