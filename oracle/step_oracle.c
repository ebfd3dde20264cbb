/*
 * FP64 CPU oracle of one two-phase time step of arXiv 2401.06755, Sec. 2.4
 * (Stages 1-4), with linear (p = 1) filters on a uniform grid.
 *
 * TEST INFRASTRUCTURE ONLY (see nn4mg_oracle.c).  Every operator is a filter
 * sum f(C; w) over a halo-padded tensor (Sec. 2.2.2); the filters are the
 * tensor products of the 1D linear-element vectors
 *     K = [-1, 2, -1] / h,  M = h [1, 4, 1] / 6,  G = [-1, 0, 1] / 2,
 * w_x = G (x) M (x) M (the printed w_x of Sec. 2.2.3), w_m = M (x) M (x) M,
 * w_lap = K M M + M K M + M M K, w_xx^PG = K (x) M (x) M.
 *
 * Readings where the paper is silent, garbled or inconsistent:
 *  - Psi_x inside the Petrov-Galerkin formulas (Eqs. k-abs, k-square, a_psi,
 *    normalisation, negativek) is in derivative units, f(Psi; w_x) / m_l;
 *    the residuals (Eqs. Petrov, Petrov-Cs, ph_disc, ph_disc2) use the filters
 *    as printed (volume-integrated);
 *  - mu = C mu_l + (1 - C) mu_g (same blend as Eq. rho); absorption sigma = 0;
 *  - halo rules per field on the tank box (free-slip side and bottom walls,
 *    outlet on top, Sec. 3.1): C, rho, mu, k and derived scalars +mirror on all
 *    faces; velocity component d: -mirror on the walls normal to d (not the
 *    top), +mirror elsewhere; vector fields made from grad C (normals,
 *    surface-tension force): -mirror on faces normal to the component, +mirror
 *    elsewhere; mass fluxes rho q_d follow q_d; p_nh and dp_nh: +mirror except
 *    -mirror on top; p_hs: +mirror on sides, -mirror on top, and on the bottom
 *    the affine halo p(-1) = p(0) + g h rho(0) (Sec. 2.3.3), whose constant
 *    part is moved to the right-hand side so the multigrid sees homogeneous
 *    rules;
 *  - the isotropic coefficient of Eq. k_Psi-n is used for the velocities; the
 *    volume fraction uses the anisotropic compressive coefficients of
 *    Sec. 2.3.5 (linear detectors Eqs. Sx-lin..Sz-lin); the two maxima are kept
 *    apart (k_max of Eq. max-k vs the clamp k_max of Eq. alpha_min_and_max);
 *  - the VOF step uses the latest velocity u^{n+1} in all its coefficients;
 *  - Eqs. ph_disc and surface-tension-k are followed as printed; the
 *    surface-tension source of the momentum residual (Eq. Petrov) takes the
 *    sign for which the Stage-1 pressure balances it, as Eq. hydro-pressure
 *    states (printed, the two signs disagree: the pressure of Eq. ph_disc has
 *    the physical Laplace jump, so its gradient is -s_t, and the printed
 *    -f(s_t; w_m) would double the force at a static drop).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* halo rules */
enum { R_EVEN = 0, R_ODD = 1, R_AFFINE = 2 };

typedef struct {
    double rho_l, rho_g, mu_l, mu_g, g, sigma_t, dt;
    int mg_cycles, n_corr, n_vel_iter;
    int mg_cycles_nh; /* cycles of each correction solve (the j of the i-j strategies, Sec. 3.2); 0: mg_cycles */
    int order;        /* 1 (or 0): linear filters throughout; 2: quadratic ConvFEM for the momentum, interface
                         and volume-fraction advection terms, linear volume-fraction diffusion and pressure
                         equations (Table disc_combinations, "linear/quadratic") */
} or_step_params;

typedef struct {
    double relres[8];
    int solves;
} or_step_info;

/* from nn4mg_oracle.c */
typedef struct or_hier or_hier;
or_hier *or_setup(int nx, int ny, int nz, double h, const int bc[6], const double *k, double omega, int nu_post,
                  int min_coarse, int harmonic);
void or_free(or_hier *H);
int or_solve(or_hier *H, const double *b, double *x, double rtol, int max_cycles, int fixed, double *hist,
             int *cycles_out);
void or_q1_filter(double h, double w[27]);

static int NX, NY, NZ;
static double H;
/* Test-only periodic box: when set, every halo wraps (no walls, no affine
 * bottom halo) and the pressure solves are periodic.  The tank rules above are
 * the default. */
static int WRAP = 0;

static size_t pid(int i, int j, int k) { return (size_t)(i + 1) + (size_t)(NX + 2) * ((size_t)(j + 1) + (size_t)(NY + 2) * (size_t)(k + 1)); }
static size_t cid(int i, int j, int k) { return (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * (size_t)k); }
static size_t ncell(void) { return (size_t)NX * NY * NZ; }
static double *alloc(void) { return (double *)calloc(ncell(), sizeof(double)); }
static double *palloc(void) { return (double *)calloc((size_t)(NX + 2) * (NY + 2) * (NZ + 2), sizeof(double)); }

static double halo(int rule, double mirror, double lift) {
    if (rule == R_ODD) return -mirror;
    if (rule == R_AFFINE) return mirror + lift;
    return mirror;
}

/* Pad u with per-face rules, axis by axis.  lift (may be NULL) is the padded
 * field whose value at the mirror cell times lift_scale is added on R_AFFINE
 * faces.  In the periodic test mode every face takes the opposite interior
 * value instead. */
static void pad(const double *u, const int rule[6], const double *liftp, double lift_scale, double *up)
{
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) up[pid(i, j, k)] = u[cid(i, j, k)];
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j) {
            if (WRAP) {
                up[pid(-1, j, k)] = up[pid(NX - 1, j, k)];
                up[pid(NX, j, k)] = up[pid(0, j, k)];
                continue;
            }
            up[pid(-1, j, k)] = halo(rule[0], up[pid(0, j, k)], liftp ? lift_scale * liftp[pid(0, j, k)] : 0.0);
            up[pid(NX, j, k)] = halo(rule[1], up[pid(NX - 1, j, k)], liftp ? lift_scale * liftp[pid(NX - 1, j, k)] : 0.0);
        }
    for (int k = 0; k < NZ; ++k)
        for (int i = -1; i <= NX; ++i) {
            if (WRAP) {
                up[pid(i, -1, k)] = up[pid(i, NY - 1, k)];
                up[pid(i, NY, k)] = up[pid(i, 0, k)];
                continue;
            }
            up[pid(i, -1, k)] = halo(rule[2], up[pid(i, 0, k)], liftp ? lift_scale * liftp[pid(i, 0, k)] : 0.0);
            up[pid(i, NY, k)] = halo(rule[3], up[pid(i, NY - 1, k)], liftp ? lift_scale * liftp[pid(i, NY - 1, k)] : 0.0);
        }
    for (int j = -1; j <= NY; ++j)
        for (int i = -1; i <= NX; ++i) {
            if (WRAP) {
                up[pid(i, j, -1)] = up[pid(i, j, NZ - 1)];
                up[pid(i, j, NZ)] = up[pid(i, j, 0)];
                continue;
            }
            up[pid(i, j, -1)] = halo(rule[4], up[pid(i, j, 0)], liftp ? lift_scale * liftp[pid(i, j, 0)] : 0.0);
            up[pid(i, j, NZ)] = halo(rule[5], up[pid(i, j, NZ - 1)], liftp ? lift_scale * liftp[pid(i, j, NZ - 1)] : 0.0);
        }
}

/* f(C; w) on the interior from a padded tensor; w[(c+1)*9+(b+1)*3+(a+1)]. */
static void filt(const double *up, const double w[27], double *out)
{
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double s = 0.0;
                for (int c = -1; c <= 1; ++c)
                    for (int b = -1; b <= 1; ++b)
                        for (int a = -1; a <= 1; ++a) s += w[(c + 1) * 9 + (b + 1) * 3 + (a + 1)] * up[pid(i + a, j + b, k + c)];
                out[cid(i, j, k)] = s;
            }
}

/* f(u; w) with the rules of u. */
static void apply(const double *u, const int rule[6], const double w[27], double *out)
{
    double *up = palloc();
    pad(u, rule, NULL, 0.0, up);
    filt(up, w, out);
    free(up);
}

/* Eq. (k-Txx): 1/2 [ f(k.C; w) + k.f(C; w) - C.f(k; w) ], halos of k.C = product of halos. */
static void fdiff(const double *C, const int ruleC[6], const double *k, const int ruleK[6], const double w[27],
                  double *out)
{
    size_t n = ncell(), np = (size_t)(NX + 2) * (NY + 2) * (NZ + 2);
    double *Cp = palloc(), *kp = palloc(), *kCp = palloc();
    double *a = alloc(), *b = alloc(), *c = alloc();
    pad(C, ruleC, NULL, 0.0, Cp);
    pad(k, ruleK, NULL, 0.0, kp);
    for (size_t p = 0; p < np; ++p) kCp[p] = kp[p] * Cp[p];
    filt(kCp, w, a);
    filt(Cp, w, b);
    filt(kp, w, c);
    for (size_t p = 0; p < n; ++p) out[p] = 0.5 * (a[p] + k[p] * b[p] - C[p] * c[p]);
    free(Cp); free(kp); free(kCp); free(a); free(b); free(c);
}

/* ---------------------------------------------- two-layer halos (quadratic) */

/* Quadratic ConvFEM filters reach two cells (Sec. 2.2.3, 5 x 5 x 5 filters),
 * so their fields carry a two-cell halo (Sec. 2.3.3: two nodes thick).  Halo
 * cell -1-m takes the value of interior cell m (the same reflection about the
 * wall as the one-cell halo), with the field's sign; the affine rule adds
 * (2m + 1) lift (the wall-normal distance between the two cells is (2m + 1) h,
 * so the value extrapolated with the specified gradient); periodic wraps. */
static size_t pid2(int i, int j, int k)
{
    return (size_t)(i + 2) + (size_t)(NX + 4) * ((size_t)(j + 2) + (size_t)(NY + 4) * (size_t)(k + 2));
}
static double *palloc2(void) { return (double *)calloc((size_t)(NX + 4) * (NY + 4) * (NZ + 4), sizeof(double)); }

static double halo2(int rule, double mirror, double lift, int m)
{
    if (rule == R_ODD) return -mirror;
    if (rule == R_AFFINE) return mirror + (double)(2 * m + 1) * lift;
    return mirror;
}

static void pad2(const double *u, const int rule[6], const double *liftp2, double lift_scale, double *up)
{
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) up[pid2(i, j, k)] = u[cid(i, j, k)];
    for (int m = 0; m < 2; ++m) {
        for (int k = 0; k < NZ; ++k)
            for (int j = 0; j < NY; ++j) {
                int lo = -1 - m, hi = NX + m, ml = m, mh = NX - 1 - m;
                if (WRAP) {
                    up[pid2(lo, j, k)] = up[pid2(NX + lo, j, k)];
                    up[pid2(hi, j, k)] = up[pid2(hi - NX, j, k)];
                    continue;
                }
                up[pid2(lo, j, k)] = halo2(rule[0], up[pid2(ml, j, k)], liftp2 ? lift_scale * liftp2[pid2(ml, j, k)] : 0.0, m);
                up[pid2(hi, j, k)] = halo2(rule[1], up[pid2(mh, j, k)], liftp2 ? lift_scale * liftp2[pid2(mh, j, k)] : 0.0, m);
            }
    }
    for (int m = 0; m < 2; ++m)
        for (int k = 0; k < NZ; ++k)
            for (int i = -2; i <= NX + 1; ++i) {
                int lo = -1 - m, hi = NY + m, ml = m, mh = NY - 1 - m;
                if (WRAP) {
                    up[pid2(i, lo, k)] = up[pid2(i, NY + lo, k)];
                    up[pid2(i, hi, k)] = up[pid2(i, hi - NY, k)];
                    continue;
                }
                up[pid2(i, lo, k)] = halo2(rule[2], up[pid2(i, ml, k)], liftp2 ? lift_scale * liftp2[pid2(i, ml, k)] : 0.0, m);
                up[pid2(i, hi, k)] = halo2(rule[3], up[pid2(i, mh, k)], liftp2 ? lift_scale * liftp2[pid2(i, mh, k)] : 0.0, m);
            }
    for (int m = 0; m < 2; ++m)
        for (int j = -2; j <= NY + 1; ++j)
            for (int i = -2; i <= NX + 1; ++i) {
                int lo = -1 - m, hi = NZ + m, ml = m, mh = NZ - 1 - m;
                if (WRAP) {
                    up[pid2(i, j, lo)] = up[pid2(i, j, NZ + lo)];
                    up[pid2(i, j, hi)] = up[pid2(i, j, hi - NZ)];
                    continue;
                }
                up[pid2(i, j, lo)] = halo2(rule[4], up[pid2(i, j, ml)], liftp2 ? lift_scale * liftp2[pid2(i, j, ml)] : 0.0, m);
                up[pid2(i, j, hi)] = halo2(rule[5], up[pid2(i, j, mh)], liftp2 ? lift_scale * liftp2[pid2(i, j, mh)] : 0.0, m);
            }
}

/* f(C; w) for a 5 x 5 x 5 filter, w[(c+2)*25 + (b+2)*5 + (a+2)]. */
static void filt5(const double *up, const double w[125], double *out)
{
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double s = 0.0;
                for (int c = -2; c <= 2; ++c)
                    for (int b = -2; b <= 2; ++b)
                        for (int a = -2; a <= 2; ++a)
                            s += w[(c + 2) * 25 + (b + 2) * 5 + (a + 2)] * up[pid2(i + a, j + b, k + c)];
                out[cid(i, j, k)] = s;
            }
}

static void apply5(const double *u, const int rule[6], const double w[125], double *out)
{
    double *up = palloc2();
    pad2(u, rule, NULL, 0.0, up);
    filt5(up, w, out);
    free(up);
}

/* Eq. (k-Txx) with a 5 x 5 x 5 filter. */
static void fdiff5(const double *C, const int ruleC[6], const double *k, const int ruleK[6], const double w[125],
                   double *out)
{
    size_t n = ncell(), np = (size_t)(NX + 4) * (NY + 4) * (NZ + 4);
    double *Cp = palloc2(), *kp = palloc2(), *kCp = palloc2();
    double *a = alloc(), *b = alloc(), *c = alloc();
    pad2(C, ruleC, NULL, 0.0, Cp);
    pad2(k, ruleK, NULL, 0.0, kp);
    for (size_t p = 0; p < np; ++p) kCp[p] = kp[p] * Cp[p];
    filt5(kCp, w, a);
    filt5(Cp, w, b);
    filt5(kp, w, c);
    for (size_t p = 0; p < n; ++p) out[p] = 0.5 * (a[p] + k[p] * b[p] - C[p] * c[p]);
    free(Cp); free(kp); free(kCp); free(a); free(b); free(c);
}

/* ------------------------------------------------------------- filters */

static void outer3(const double x[3], const double y[3], const double z[3], double w[27])
{
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) w[c * 9 + b * 3 + a] = x[a] * y[b] * z[c];
}

static double WD[3][27];   /* w_x, w_y, w_z */
static double WM[27];      /* consistent mass w_m */
static double WMA[27];     /* w_m / m_l - E (the residual filter of Eq. a_psi) */
static double WLAP[27];    /* w_lap */
static double WPG[3][27];  /* w_xx^PG, w_yy^PG, w_zz^PG */
/* quadratic ConvFEM: w_x, w_y, w_z, w_m, w_m / m_l - E, w_lap (5 x 5 x 5) */
static double QD[3][125], QM[125], QMA[125], QLAP[125];
static int ORDER = 1;

static void outer5(const double x[5], const double y[5], const double z[5], double w[125])
{
    for (int c = 0; c < 5; ++c)
        for (int b = 0; b < 5; ++b)
            for (int a = 0; a < 5; ++a) w[c * 25 + b * 5 + a] = x[a] * y[b] * z[c];
}

/* The 1D quadratic ConvFEM vectors (Sec. 2.2.3: the stencils of the node
 * types summed and averaged).  A quadratic element of length 2h has nodes at
 * 0, h, 2h with element matrices (Lagrange basis)
 *   mass (2h/30) [[4, 2, -1], [2, 16, 2], [-1, 2, 4]],
 *   stiffness (1/(6h)) [[7, -8, 1], [-8, 16, -8], [1, -8, 7]],
 *   derivative int N_a N_b' = [[-1/2, 2/3, -1/6], [-2/3, 0, 2/3], [1/6, -2/3, 1/2]].
 * A vertex node collects the last row of the element on its left and the
 * first row of the one on its right (offsets -2..2); a mid node the middle
 * row (offsets -1..1).  Their average over the two node types is
 *   M2 = (h/30) [-1, 4, 24, 4, -1],  K2 = (1/(12h)) [1, -16, 30, -16, 1],
 *   G2 = (1/12) [1, -8, 0, 8, -1],
 * and the 3D filters are their tensor products, as for the linear ones. */
static void quad_vectors(double h, double M2[5], double K2[5], double G2[5])
{
    const double m[5] = {-1.0, 4.0, 24.0, 4.0, -1.0}, k[5] = {1.0, -16.0, 30.0, -16.0, 1.0},
                 g[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
    for (int q = 0; q < 5; ++q) {
        M2[q] = h * m[q] / 30.0;
        K2[q] = k[q] / (12.0 * h);
        G2[q] = g[q] / 12.0;
    }
}

static void build_filters(double h)
{
    const double K[3] = {-1.0 / h, 2.0 / h, -1.0 / h};
    const double M[3] = {h / 6.0, 4.0 * h / 6.0, h / 6.0};
    const double G[3] = {-0.5, 0.0, 0.5};
    outer3(G, M, M, WD[0]);
    outer3(M, G, M, WD[1]);
    outer3(M, M, G, WD[2]);
    outer3(M, M, M, WM);
    const double ml = h * h * h;
    for (int q = 0; q < 27; ++q) WMA[q] = WM[q] / ml - (q == 13 ? 1.0 : 0.0);
    outer3(K, M, M, WPG[0]);
    outer3(M, K, M, WPG[1]);
    outer3(M, M, K, WPG[2]);
    or_q1_filter(h, WLAP);
    double M2[5], K2[5], G2[5], t[125];
    quad_vectors(h, M2, K2, G2);
    outer5(G2, M2, M2, QD[0]);
    outer5(M2, G2, M2, QD[1]);
    outer5(M2, M2, G2, QD[2]);
    outer5(M2, M2, M2, QM);
    for (int q = 0; q < 125; ++q) QMA[q] = QM[q] / ml - (q == 62 ? 1.0 : 0.0);
    outer5(K2, M2, M2, QLAP);
    outer5(M2, K2, M2, t);
    for (int q = 0; q < 125; ++q) QLAP[q] += t[q];
    outer5(M2, M2, K2, t);
    for (int q = 0; q < 125; ++q) QLAP[q] += t[q];
}

/* f(u; w) with the filter of the step's order for the terms that take it
 * (w1: 3 x 3 x 3, w2: 5 x 5 x 5). */
static void applyO(const double *u, const int rule[6], const double *w1, const double *w2, double *out)
{
    if (ORDER == 2) apply5(u, rule, w2, out);
    else apply(u, rule, w1, out);
}

static void set_grid(int nx, int ny, int nz, double h)
{
    NX = nx; NY = ny; NZ = nz; H = h;
    build_filters(h);
}

/* ------------------------------------------------------------- rules */

static const int RULE_EVEN[6] = {R_EVEN, R_EVEN, R_EVEN, R_EVEN, R_EVEN, R_EVEN};
/* velocity component d on the tank: free-slip walls except the top outlet */
static void rule_vel(int d, int r[6])
{
    for (int f = 0; f < 6; ++f) r[f] = R_EVEN;
    if (d == 0) r[0] = r[1] = R_ODD;
    if (d == 1) r[2] = r[3] = R_ODD;
    if (d == 2) r[4] = R_ODD;
}
/* component d of a vector made from grad C (C even on every face) */
static void rule_grad(int d, int r[6])
{
    for (int f = 0; f < 6; ++f) r[f] = R_EVEN;
    r[2 * d] = r[2 * d + 1] = R_ODD;
}
static const int RULE_PNH[6] = {R_EVEN, R_EVEN, R_EVEN, R_EVEN, R_EVEN, R_ODD};
static const int RULE_PHS[6] = {R_EVEN, R_EVEN, R_EVEN, R_EVEN, R_AFFINE, R_ODD};

/* the pressure hierarchy: Neumann except zero on top (periodic in the test mode) */
static or_hier *pressure_hierarchy(void)
{
    const int bcT[6] = {1, 1, 1, 1, 1, 0}, bcW[6] = {2, 2, 2, 2, 2, 2};
    return or_setup(NX, NY, NZ, H, WRAP ? bcW : bcT, NULL, 2.0 / 3.0, 2, 4, 0);
}

/* ------------------------------------------------------------- PG pieces */

/* a_Psi = alpha_a f(u Psi_x + v Psi_y + w Psi_z; w_m/m_l - E), Psi_d in derivative units. */
static void adv_residual(const double *u, const double *v, const double *w, const double *Pd[3], double alpha_a,
                         double *adv, double *a)
{
    size_t n = ncell();
    for (size_t p = 0; p < n; ++p) adv[p] = u[p] * Pd[0][p] + v[p] * Pd[1][p] + w[p] * Pd[2][p];
    applyO(adv, RULE_EVEN, WMA, QMA, a);
    for (size_t p = 0; p < n; ++p) a[p] *= alpha_a;
}

/* Eq. k_Psi-n with Eqs. efficient-kabs-special-case, k-square (h_Psi = h), max-k. */
static void pg_isotropic(const double *u, const double *v, const double *w, const double *Pd[3], const double *a,
                         const double *rho, const double *mu, double *kout)
{
    const double eps_k = 1e-7, a_kabs = 1.0 / 16.0, a_ksq = 4.0;
    size_t n = ncell();
    for (size_t p = 0; p < n; ++p) {
        double G = fabs(Pd[0][p]) + fabs(Pd[1][p]) + fabs(Pd[2][p]);
        double kabs = a_kabs * H * fabs(a[p]) / (eps_k + G / 3.0);
        double g2 = Pd[0][p] * Pd[0][p] + Pd[1][p] * Pd[1][p] + Pd[2][p] * Pd[2][p];
        double adv = fabs(u[p] * Pd[0][p]) + fabs(v[p] * Pd[1][p]) + fabs(w[p] * Pd[2][p]);
        double ksq = a_ksq * a[p] * a[p] * H / (eps_k + adv / 3.0 * g2);
        double kmax = H * (fabs(u[p]) + fabs(v[p]) + fabs(w[p]));
        double m = kmax;
        if (kabs < m) m = kabs;
        if (ksq < m) m = ksq;
        kout[p] = rho[p] * m + mu[p];
    }
}

/* ------------------------------------------------------------- stages */

/* grad C in derivative units (Cd), the normals, the curvature of
 * Eq. surface-tension-k and the surface-tension vectors of
 * Eq. surface-tension-uvw. */
static void surface(const double *C, double sigma_t, double *Cd[3], double *nrm[3], double *kappa, double *st[3],
                    double *tmp)
{
    size_t n = ncell();
    const double ml = H * H * H;
    int rg[3][6];
    for (int d = 0; d < 3; ++d) rule_grad(d, rg[d]);
    for (int d = 0; d < 3; ++d) {
        applyO(C, RULE_EVEN, WD[d], QD[d], Cd[d]);
        for (size_t p = 0; p < n; ++p) Cd[d][p] /= ml;
    }
    const double eps_t = 1e-7 / H;
    for (size_t p = 0; p < n; ++p) {
        double l = sqrt(Cd[0][p] * Cd[0][p] + Cd[1][p] * Cd[1][p] + Cd[2][p] * Cd[2][p]);
        for (int d = 0; d < 3; ++d) nrm[d][p] = Cd[d][p] / (eps_t + l);
    }
    for (size_t p = 0; p < n; ++p) kappa[p] = 0.0;
    for (int d = 0; d < 3; ++d) {
        applyO(nrm[d], rg[d], WD[d], QD[d], tmp);
        for (size_t p = 0; p < n; ++p) kappa[p] += tmp[p];
    }
    for (size_t p = 0; p < n; ++p) {
        kappa[p] /= ml;
        for (int d = 0; d < 3; ++d) st[d][p] = sigma_t * kappa[p] * Cd[d][p];
    }
}

static void solve_pressure(or_hier *Hr, const double *b, double *x, int cycles, or_step_info *info)
{
    double hist[1024];
    int cyc = 0;
    or_solve(Hr, b, x, 0.0, cycles, 1, hist, &cyc);
    if (info && info->solves < 8) info->relres[info->solves++] = hist[cyc];
}

/* Stage 3: n_corr solves of Eq. ph_disc2 for dp_nh with the corrections of
 * Eq. vel-cor applied to q (the Stage-2 estimate in, q^{n+1} out) and
 * p_nh += dp_nh. */
static void correct(const or_step_params *P, or_hier *Hr, const double *rho, double *q[3], double *p_nh,
                    or_step_info *info)
{
    size_t n = ncell();
    const double ml = H * H * H, dt = P->dt;
    int rv[3][6];
    for (int d = 0; d < 3; ++d) rule_vel(d, rv[d]);
    double *b = alloc(), *tmp = alloc(), *tmp2 = alloc(), *dp = alloc();
    for (int it = 0; it < P->n_corr; ++it) {
        for (size_t p = 0; p < n; ++p) b[p] = 0.0;
        for (int d = 0; d < 3; ++d) {
            for (size_t p = 0; p < n; ++p) tmp2[p] = rho[p] * q[d][p];
            apply(tmp2, rv[d], WD[d], tmp);
            for (size_t p = 0; p < n; ++p) b[p] -= tmp[p] / dt;
            apply(rho, RULE_EVEN, WD[d], tmp);
            for (size_t p = 0; p < n; ++p) b[p] += q[d][p] * tmp[p] / dt;
        }
        for (size_t p = 0; p < n; ++p) dp[p] = 0.0;
        solve_pressure(Hr, b, dp, P->mg_cycles_nh > 0 ? P->mg_cycles_nh : P->mg_cycles, info);
        for (int d = 0; d < 3; ++d) {
            apply(dp, RULE_PNH, WD[d], tmp);
            for (size_t p = 0; p < n; ++p) q[d][p] += -dt * (tmp[p] / ml) / rho[p];
        }
        for (size_t p = 0; p < n; ++p) p_nh[p] += dp[p];
    }
    free(b); free(tmp); free(tmp2); free(dp);
}

/* Stage 4 coefficients: the anisotropic compressive diffusivities of
 * Sec. 2.3.5 (detectors Eqs. Sx-lin..Sz-lin with the 0.05/0.95 override,
 * weights w+ and w-, k- of Eqs. negativek and normalisation, k+ of
 * Eq. positivek, clamps of Eq. alpha_min_and_max).  Cd = grad C in
 * derivative units; a receives the advection residual of Eq. a_psi. */
static void vof_coefs(const double *C, const double *u, const double *v, const double *w, double *const Cd[3],
                      double dt, double *kd[3], double *a)
{
    const double Kp = 300.0, Km = 300.0, beta = 0.1, eps_x = 1e-4, Kpos = 3.0, eps_k = 1e-7;
    const double h = H, kmin = 1e-4 / dt * h * h, kclamp = 0.05 / dt * h * h;
    const double *Pd[3] = {Cd[0], Cd[1], Cd[2]};
    double *adv = alloc();
    adv_residual(u, v, w, Pd, 2.0, adv, a);
    free(adv);
    double *Cp = palloc2();
    pad2(C, RULE_EVEN, NULL, 0.0, Cp);
    for (int kk = 0; kk < NZ; ++kk)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t p = cid(i, j, kk);
                double c0 = Cp[pid2(i, j, kk)];
                double S[3];
                for (int d = 0; d < 3; ++d) {
                    /* value at offset s along direction d */
                    double c[5];
                    for (int o = -2; o <= 2; ++o)
                        c[o + 2] = Cp[pid2(i + (d == 0 ? o : 0), j + (d == 1 ? o : 0), kk + (d == 2 ? o : 0))];
                    /* Eqs. Sx-lin..Sz-lin; with the quadratic filters Eqs. Sx-quad..Sz-quad (the
                     * smallest of the three products of successive differences) */
                    S[d] = (c[2] - c[1]) * (c[3] - c[2]);
                    if (ORDER == 2) {
                        double s1 = (c[1] - c[0]) * (c[2] - c[1]), s3 = (c[3] - c[2]) * (c[4] - c[3]);
                        if (s1 < S[d]) S[d] = s1;
                        if (s3 < S[d]) S[d] = s3;
                    }
                }
                if (c0 > 0.95 || c0 < 0.05) S[0] = S[1] = S[2] = -1.0;
                double cx = Cd[0][p], cy = Cd[1][p], cz = Cd[2][p];
                double g2 = cx * cx + cy * cy + cz * cz;
                double proj = (u[p] * cx + v[p] * cy + w[p] * cz) / (eps_x + g2);
                double us = cx * proj, vs = cy * proj, ws = cz * proj;
                double kneg = -beta * (u[p] * u[p] + v[p] * v[p] + w[p] * w[p]) /
                              (eps_x + g2 * (fabs(us) + fabs(vs) + fabs(ws)) / 3.0);
                double G = fabs(cx) + fabs(cy) + fabs(cz);
                double kabs = (1.0 / 16.0) * h * fabs(a[p]) / (eps_k + G / 3.0);
                for (int d = 0; d < 3; ++d) {
                    double wp = -fmax(-1.0, fmin(0.0, Kp * S[d]));
                    double wm = fmin(1.0, fmax(0.0, Km * S[d]));
                    double kk2 = wp * (Kpos * kabs) + wm * (kneg / h);
                    kd[d][p] = fmax(-kmin, fmin(kclamp, kk2));
                }
            }
    free(Cp);
}

/* Stage 4: C^{n+1} = C^n - dt f(s_C; w_ml^-1) (Eq. transport-indicator-1)
 * with s_C = m_l (u C_x + v C_y + w C_z) + sum_d f_diff(C, k_d; w_dd^PG)
 * (Eq. Petrov-C). */
static void vof_update(double *C, const double *u, const double *v, const double *w, double *const Cd[3], double dt)
{
    size_t n = ncell();
    const double ml = H * H * H;
    double *a = alloc(), *tmp = alloc(), *kd[3];
    for (int d = 0; d < 3; ++d) kd[d] = alloc();
    vof_coefs(C, u, v, w, Cd, dt, kd, a);
    double *sC = alloc();
    for (size_t p = 0; p < n; ++p) sC[p] = ml * (u[p] * Cd[0][p] + v[p] * Cd[1][p] + w[p] * Cd[2][p]);
    for (int d = 0; d < 3; ++d) {
        fdiff(C, RULE_EVEN, kd[d], RULE_EVEN, WPG[d], tmp);
        for (size_t p = 0; p < n; ++p) sC[p] += tmp[p];
    }
    for (size_t p = 0; p < n; ++p) C[p] = C[p] - dt * sC[p] / ml;
    for (int d = 0; d < 3; ++d) free(kd[d]);
    free(sC); free(a); free(tmp);
}

/* ------------------------------------------------------------- the step */

int or_step(int nx, int ny, int nz, double h, const or_step_params *P, double *C, double *u, double *v,
            double *w, double *p_hs, double *p_nh, or_step_info *info)
{
    set_grid(nx, ny, nz, h);
    if (info) memset(info, 0, sizeof(*info));
    if (P->order != 0 && P->order != 1 && P->order != 2) return -1;
    if (P->order == 2 && (nx < 2 || ny < 2 || nz < 2)) return -1;
    ORDER = P->order == 2 ? 2 : 1;
    const size_t n = ncell();
    const double ml = h * h * h, dt = P->dt;
    double *q[3] = {u, v, w};
    int rv[3][6], rg[3][6];
    for (int d = 0; d < 3; ++d) { rule_vel(d, rv[d]); rule_grad(d, rg[d]); }

    double *rho = alloc(), *mu = alloc(), *Cd[3], *nrm[3], *st[3];
    for (int d = 0; d < 3; ++d) { Cd[d] = alloc(); nrm[d] = alloc(); st[d] = alloc(); }
    double *tmp = alloc(), *tmp2 = alloc(), *b = alloc();

    /* density and viscosity, Eq. rho */
    for (size_t p = 0; p < n; ++p) {
        rho[p] = P->rho_l * C[p] + P->rho_g * (1.0 - C[p]);
        mu[p] = P->mu_l * C[p] + P->mu_g * (1.0 - C[p]);
    }
    /* grad C (derivative units), normals, curvature, surface tension */
    double *kappa = alloc();
    surface(C, P->sigma_t, Cd, nrm, kappa, st, tmp);

    or_hier *Hr = pressure_hierarchy();
    if (!Hr) return -1;

    /* ---- Stage 1: hydrostatic + surface-tension pressure, Eq. ph_disc ---- */
    for (size_t p = 0; p < n; ++p) b[p] = 0.0;
    for (int d = 0; d < 3; ++d) {
        apply(st[d], rg[d], WD[d], tmp);
        for (size_t p = 0; p < n; ++p) b[p] += tmp[p];
    }
    for (size_t p = 0; p < n; ++p) tmp2[p] = P->g * rho[p];
    apply(tmp2, RULE_EVEN, WD[2], tmp);
    for (size_t p = 0; p < n; ++p) b[p] += tmp[p];
    /* lift of the affine bottom halo: A applied to the halo constants alone */
    if (!WRAP) {
        double *zero = alloc(), *liftp = palloc(), *rhop = palloc();
        pad(rho, RULE_EVEN, NULL, 0.0, rhop);
        pad(zero, RULE_PHS, rhop, P->g * h, liftp);
        filt(liftp, WLAP, tmp);
        for (size_t p = 0; p < n; ++p) b[p] -= tmp[p];
        free(zero); free(liftp); free(rhop);
    }
    solve_pressure(Hr, b, p_hs, P->mg_cycles, info);

    /* ---- Stage 2: velocity predictor, Eqs. Petrov, velocity-1 ---- */
    double *qn[3], *qh[3], *qt[3], *Qd[3][3], *kq[3];
    for (int c = 0; c < 3; ++c) {
        qn[c] = alloc(); qh[c] = alloc(); qt[c] = alloc(); kq[c] = alloc();
        memcpy(qn[c], q[c], n * sizeof(double));
        memcpy(qh[c], q[c], n * sizeof(double));
        for (int d = 0; d < 3; ++d) Qd[c][d] = alloc();
    }
    double *adv = alloc(), *a = alloc(), *gp = alloc(), *src = alloc();
    for (int it = 0; it < P->n_vel_iter; ++it) {
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
                applyO(qh[c], rv[c], WD[d], QD[d], Qd[c][d]);
                for (size_t p = 0; p < n; ++p) Qd[c][d][p] /= ml;
            }
        for (int c = 0; c < 3; ++c) {
            const double *Pd[3] = {Qd[c][0], Qd[c][1], Qd[c][2]};
            adv_residual(qh[0], qh[1], qh[2], Pd, 2.0, adv, a);
            pg_isotropic(qh[0], qh[1], qh[2], Pd, a, rho, mu, kq[c]);
            /* s = rho (u q_x + v q_y + w q_z) m_l + f_lap(q, k_q) + f(p_hs + p_nh; w_c) - f(s_q + s_t; w_m) */
            if (ORDER == 2) fdiff5(qh[c], rv[c], kq[c], RULE_EVEN, QLAP, tmp);
            else fdiff(qh[c], rv[c], kq[c], RULE_EVEN, WLAP, tmp);
            if (ORDER == 2) {   /* p_hs with its affine bottom halo, two cells */
                double *pp = palloc2(), *rp = palloc2();
                pad2(rho, RULE_EVEN, NULL, 0.0, rp);
                pad2(p_hs, RULE_PHS, rp, P->g * h, pp);
                filt5(pp, QD[c], gp);
                free(pp); free(rp);
            } else {   /* p_hs with its affine bottom halo */
                double *pp = palloc(), *rp = palloc();
                pad(rho, RULE_EVEN, NULL, 0.0, rp);
                pad(p_hs, RULE_PHS, rp, P->g * h, pp);
                filt(pp, WD[c], gp);
                free(pp); free(rp);
            }
            for (size_t p = 0; p < n; ++p) tmp[p] += gp[p];
            applyO(p_nh, RULE_PNH, WD[c], QD[c], gp);
            for (size_t p = 0; p < n; ++p) tmp[p] += gp[p];
            /* the surface-tension source with the sign that the Stage-1
             * pressure balances (Eq. hydro-pressure): p_hs of Eq. ph_disc has
             * gradient -s_t for kappa = +div n, so s_t enters as +f(s_t; w_m) */
            applyO(st[c], rg[c], WM, QM, gp);
            for (size_t p = 0; p < n; ++p) tmp[p] += gp[p];
            if (c == 2) {
                for (size_t p = 0; p < n; ++p) src[p] = -P->g * rho[p];
                applyO(src, RULE_EVEN, WM, QM, gp);
                for (size_t p = 0; p < n; ++p) tmp[p] -= gp[p];
            }
            for (size_t p = 0; p < n; ++p) {
                double s = rho[p] * ml * adv[p] + tmp[p];
                qt[c][p] = (-s / ml + rho[p] * qn[c][p] / dt) / (rho[p] / dt);
            }
        }
        for (int c = 0; c < 3; ++c)
            for (size_t p = 0; p < n; ++p) qh[c][p] = 0.5 * (qn[c][p] + qt[c][p]);
    }

    /* ---- Stage 3: non-hydrostatic correction, Eqs. ph_disc2, vel-cor ---- */
    correct(P, Hr, rho, qt, p_nh, info);
    for (int c = 0; c < 3; ++c) memcpy(q[c], qt[c], n * sizeof(double));

    /* ---- Stage 4: volume fraction, Eqs. Petrov-C, transport-indicator-1 ---- */
    vof_update(C, u, v, w, Cd, dt);

    or_free(Hr);
    for (int c = 0; c < 3; ++c) {
        free(qn[c]); free(qh[c]); free(qt[c]); free(kq[c]);
        for (int d = 0; d < 3; ++d) free(Qd[c][d]);
    }
    for (int d = 0; d < 3; ++d) { free(Cd[d]); free(nrm[d]); free(st[d]); }
    free(rho); free(mu); free(tmp); free(tmp2); free(b); free(kappa); free(adv); free(a); free(gp); free(src);
    ORDER = 1;
    return 0;
}

/* ------------------------------------------------------------- pieces for the pins */

void or_step_filters(double h, double *wx, double *wm, double *wpgx, double *wlap)
{
    build_filters(h);
    memcpy(wx, WD[0], sizeof(WD[0]));
    memcpy(wm, WM, sizeof(WM));
    memcpy(wpgx, WPG[0], sizeof(WPG[0]));
    memcpy(wlap, WLAP, sizeof(WLAP));
}

/* 1: every halo wraps and the pressure solves are periodic; 0: the tank. */
void or_step_set_periodic(int on) { WRAP = on ? 1 : 0; }

/* Filter order of the stage pieces below (or_step sets its own from the
 * parameters): 1 linear, 2 quadratic ConvFEM for the terms that take it. */
void or_step_set_order(int order) { ORDER = order == 2 ? 2 : 1; }

/* The quadratic ConvFEM filters (5 x 5 x 5, [(c+2)*25 + (b+2)*5 + (a+2)]). */
void or_step_filters_quadratic(double h, double *wx, double *wm, double *wlap)
{
    build_filters(h);
    memcpy(wx, QD[0], sizeof(QD[0]));
    memcpy(wm, QM, sizeof(QM));
    memcpy(wlap, QLAP, sizeof(QLAP));
}

/* f(u; w) of a 5 x 5 x 5 filter with the two-cell halo of a rule given per
 * face (0 even, 1 odd), for the pins of the two-cell halo. */
void or_step_apply5(int nx, int ny, int nz, double h, const int rule[6], const double *w, const double *u, double *out)
{
    set_grid(nx, ny, nz, h);
    apply5(u, rule, w, out);
}

/* Curvature and surface-tension vectors of C (Eqs. surface-tension-k,
 * surface-tension-uvw) and grad C in derivative units. */
void or_step_surface(int nx, int ny, int nz, double h, double sigma_t, const double *C, double *Cx, double *Cy,
                     double *Cz, double *kappa, double *stx, double *sty, double *stz)
{
    set_grid(nx, ny, nz, h);
    double *Cd[3] = {Cx, Cy, Cz}, *st[3] = {stx, sty, stz}, *nrm[3], *tmp = alloc();
    for (int d = 0; d < 3; ++d) nrm[d] = alloc();
    surface(C, sigma_t, Cd, nrm, kappa, st, tmp);
    for (int d = 0; d < 3; ++d) free(nrm[d]);
    free(tmp);
}

/* Velocity diffusivity of component comp (0..2) as Stage 2 forms it from the
 * velocity (u, v, w): a = advection residual (Eq. a_psi), k = Eq. k_Psi-n. */
void or_step_pg_velocity(int nx, int ny, int nz, double h, int comp, const double *u, const double *v,
                         const double *w, const double *rho, const double *mu, double *a, double *k)
{
    set_grid(nx, ny, nz, h);
    const double *q[3] = {u, v, w};
    const double ml = h * h * h;
    size_t n = ncell();
    int rv[6];
    rule_vel(comp, rv);
    double *Pd[3], *adv = alloc();
    for (int d = 0; d < 3; ++d) {
        Pd[d] = alloc();
        applyO(q[comp], rv, WD[d], QD[d], Pd[d]);
        for (size_t p = 0; p < n; ++p) Pd[d][p] /= ml;
    }
    const double *cPd[3] = {Pd[0], Pd[1], Pd[2]};
    adv_residual(u, v, w, cPd, 2.0, adv, a);
    pg_isotropic(u, v, w, cPd, a, rho, mu, k);
    for (int d = 0; d < 3; ++d) free(Pd[d]);
    free(adv);
}

/* Stage-4 diffusivities (kx, ky, kz) and the advection residual a of C. */
void or_step_vof_coefs(int nx, int ny, int nz, double h, double dt, const double *C, const double *u,
                       const double *v, const double *w, double *kx, double *ky, double *kz, double *a)
{
    set_grid(nx, ny, nz, h);
    const double ml = h * h * h;
    size_t n = ncell();
    double *Cd[3], *kd[3] = {kx, ky, kz};
    for (int d = 0; d < 3; ++d) {
        Cd[d] = alloc();
        applyO(C, RULE_EVEN, WD[d], QD[d], Cd[d]);
        for (size_t p = 0; p < n; ++p) Cd[d][p] /= ml;
    }
    vof_coefs(C, u, v, w, Cd, dt, kd, a);
    for (int d = 0; d < 3; ++d) free(Cd[d]);
}

/* Stage 4 alone: C updated in place with the velocity (u, v, w). */
void or_step_vof(int nx, int ny, int nz, double h, double dt, double *C, const double *u, const double *v,
                 const double *w)
{
    set_grid(nx, ny, nz, h);
    const double ml = h * h * h;
    size_t n = ncell();
    double *Cd[3];
    for (int d = 0; d < 3; ++d) {
        Cd[d] = alloc();
        applyO(C, RULE_EVEN, WD[d], QD[d], Cd[d]);
        for (size_t p = 0; p < n; ++p) Cd[d][p] /= ml;
    }
    vof_update(C, u, v, w, Cd, dt);
    for (int d = 0; d < 3; ++d) free(Cd[d]);
}

/* Stage 3 alone: n_corr corrections of the velocity estimate (u, v, w) in
 * place with rho from C (Eq. rho), p_nh += dp_nh. */
int or_step_correct(int nx, int ny, int nz, double h, const or_step_params *P, const double *C, double *u,
                    double *v, double *w, double *p_nh, or_step_info *info)
{
    set_grid(nx, ny, nz, h);
    if (info) memset(info, 0, sizeof(*info));
    size_t n = ncell();
    double *rho = alloc(), *q[3] = {u, v, w};
    for (size_t p = 0; p < n; ++p) rho[p] = P->rho_l * C[p] + P->rho_g * (1.0 - C[p]);
    or_hier *Hr = pressure_hierarchy();
    if (!Hr) { free(rho); return -1; }
    correct(P, Hr, rho, q, p_nh, info);
    or_free(Hr);
    free(rho);
    return 0;
}
