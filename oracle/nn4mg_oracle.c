/*
 * FP64 CPU oracle for the pressure solve of Chen, Heaney, Gomes, Matar, Pain,
 * "Solving the discretised multiphase flow equations with interface capturing
 * on structured grids using machine learning libraries" (arXiv 2401.06755).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no source,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * Plain loops in double precision, in the order the paper states the method:
 * every field is padded with a one-cell halo (Sec. 2.2.1, Fig. 1; Sec. 2.3.3),
 * every operator is the filter sum f(C; w) of Sec. 2.2.2 over that padded
 * tensor, and the variable-coefficient operator is the three-filter identity
 * of Eq. (k-T) in Sec. 2.2.4. No blocking, no fusion, no reordering.
 *
 * Readings where the paper is silent:
 *  - cell-centred nodes, x_i = (i + 1/2) h (Fig. 1 caption);
 *  - Dirichlet-zero halo = minus the mirrored interior value, so the boundary
 *    sits on the cell face at every level (Sec. 2.3.3 / Fig. bc-applied:
 *    halo chosen so the interpolated boundary value is the prescribed one);
 *    zero-normal-derivative halo = copy of the nearest interior value
 *    (Sec. 2.3.3); periodic = wrap (test-only);
 *    halos filled axis by axis, so edge/corner halo cells carry the product
 *    of the per-axis signs;
 *  - the linear-element Laplacian filter has centre 8h/3, face 0, edge -h/6,
 *    corner -h/12 (tensor-product Q1 stiffness, the same convention that
 *    gives the printed first-derivative filter w_x of Sec. 2.2.3);
 *  - sawtooth V(0, nu) cycle: restriction of the residual on the way down
 *    (U-Net encoder), exact dense solve at the bottom, trilinear
 *    prolongation + nu weighted-Jacobi sweeps on the way up (decoder),
 *    Fig. multi-grid / Sec. 2.4;
 *  - restriction = sum of the 8 children (the residuals are volume
 *    integrated), coarse operators re-discretised at h_l = 2^l h with the
 *    coefficient averaged over the 8 children (BCs at every level, Sec. 2.3.3);
 *  - Jacobi diagonal = the filter centre (times the coefficient form below),
 *    i.e. the interior diagonal, not the halo-folded one;
 *  - all-Neumann/periodic (singular) problems: b projected to zero mean, x
 *    projected to zero mean after every cycle, coarsest matrix shifted by
 *    mean(diag) * 11^T / n before the Cholesky factorisation.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { OR_BC_DIRICHLET0 = 0, OR_BC_NEUMANN0 = 1, OR_BC_PERIODIC = 2 };

/* ------------------------------------------------------------------------ */
/* Padded tensors (Sec. 2.2.2: size (Nx+2l) x (Ny+2l) x (Nz+2l), here l = 1) */
/* ------------------------------------------------------------------------ */

static size_t pidx(int nx, int ny, int i, int j, int k)
{
    return (size_t)(i + 1) + (size_t)(nx + 2) * ((size_t)(j + 1) + (size_t)(ny + 2) * (size_t)(k + 1));
}

static size_t cidx(int nx, int ny, int i, int j, int k)
{
    return (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * (size_t)k);
}

/* Value of one halo cell from its mirror (nearest interior cell) and its
 * periodic image.  `coef` selects the rule for material coefficients, which
 * are always continued by a zero-derivative copy. */
static double halo_value(int bc, int coef, double mirror, double image)
{
    if (bc == OR_BC_PERIODIC) return image;
    if (coef) return mirror;
    if (bc == OR_BC_DIRICHLET0) return -mirror;
    return mirror; /* OR_BC_NEUMANN0 */
}

/* Copy u into the interior of up and fill the one-cell halo, x then y then z. */
void or_pad(const double *u, int nx, int ny, int nz, const int bc[6], int coef, double *up)
{
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                up[pidx(nx, ny, i, j, k)] = u[cidx(nx, ny, i, j, k)];
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            up[pidx(nx, ny, -1, j, k)] = halo_value(bc[0], coef, up[pidx(nx, ny, 0, j, k)], up[pidx(nx, ny, nx - 1, j, k)]);
            up[pidx(nx, ny, nx, j, k)] = halo_value(bc[1], coef, up[pidx(nx, ny, nx - 1, j, k)], up[pidx(nx, ny, 0, j, k)]);
        }
    for (int k = 0; k < nz; ++k)
        for (int i = -1; i <= nx; ++i) {
            up[pidx(nx, ny, i, -1, k)] = halo_value(bc[2], coef, up[pidx(nx, ny, i, 0, k)], up[pidx(nx, ny, i, ny - 1, k)]);
            up[pidx(nx, ny, i, ny, k)] = halo_value(bc[3], coef, up[pidx(nx, ny, i, ny - 1, k)], up[pidx(nx, ny, i, 0, k)]);
        }
    for (int j = -1; j <= ny; ++j)
        for (int i = -1; i <= nx; ++i) {
            up[pidx(nx, ny, i, j, -1)] = halo_value(bc[4], coef, up[pidx(nx, ny, i, j, 0)], up[pidx(nx, ny, i, j, nz - 1)]);
            up[pidx(nx, ny, i, j, nz)] = halo_value(bc[5], coef, up[pidx(nx, ny, i, j, nz - 1)], up[pidx(nx, ny, i, j, 0)]);
        }
}

static double *pad_alloc(int nx, int ny, int nz)
{
    return (double *)malloc(sizeof(double) * (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2));
}

/* ------------------------------------------------------------------------ */
/* Filters                                                                   */
/* ------------------------------------------------------------------------ */

/* w[(c+1)*9 + (b+1)*3 + (a+1)] is the weight of offset (a, b, c) = (x, y, z).
 * Linear-element Laplacian: centre 8h/3, faces 0, edges -h/6, corners -h/12. */
void or_q1_filter(double h, double w[27])
{
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
                int m = abs(a) + abs(b) + abs(c);
                double v = 0.0;
                if (m == 0) v = 8.0 * h / 3.0;
                else if (m == 1) v = 0.0;
                else if (m == 2) v = -h / 6.0;
                else v = -h / 12.0;
                w[(c + 1) * 9 + (b + 1) * 3 + (a + 1)] = v;
            }
}

/* f(C; w) at every interior node (Sec. 2.2.2): the sum over the 27 offsets of
 * weight times padded value. */
void or_filter_apply(const double *up, int nx, int ny, int nz, const double w[27], double *out)
{
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int c = -1; c <= 1; ++c)
                    for (int b = -1; b <= 1; ++b)
                        for (int a = -1; a <= 1; ++a)
                            s += w[(c + 1) * 9 + (b + 1) * 3 + (a + 1)] * up[pidx(nx, ny, i + a, j + b, k + c)];
                out[cidx(nx, ny, i, j, k)] = s;
            }
}

/* ------------------------------------------------------------------------ */
/* The pressure operator                                                     */
/* ------------------------------------------------------------------------ */

/* y = A x.  Constant coefficient (k == NULL): y = f(x; w_lap), Eq. (ph_disc).
 * Nodal coefficient k: Eq. (k-T),
 *     y = 1/2 [ f(k.x; w) + k.f(x; w) - x.f(k; w) ],
 * with the halo of the product k.x equal to the product of the halos. */
void or_apply(int nx, int ny, int nz, double h, const int bc[6], const double *k, const double *x, double *y)
{
    double w[27];
    or_q1_filter(h, w);
    size_t n = (size_t)nx * ny * nz, np = (size_t)(nx + 2) * (ny + 2) * (nz + 2);
    double *xp = pad_alloc(nx, ny, nz);
    or_pad(x, nx, ny, nz, bc, 0, xp);
    if (!k) {
        or_filter_apply(xp, nx, ny, nz, w, y);
        free(xp);
        return;
    }
    double *kp = pad_alloc(nx, ny, nz), *kxp = pad_alloc(nx, ny, nz);
    double *f_kx = (double *)malloc(sizeof(double) * n), *f_x = (double *)malloc(sizeof(double) * n),
           *f_k = (double *)malloc(sizeof(double) * n);
    or_pad(k, nx, ny, nz, bc, 1, kp);
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (size_t p = 0; p < np; ++p) kxp[p] = kp[p] * xp[p];
    or_filter_apply(kxp, nx, ny, nz, w, f_kx);
    or_filter_apply(xp, nx, ny, nz, w, f_x);
    or_filter_apply(kp, nx, ny, nz, w, f_k);
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (size_t p = 0; p < n; ++p) y[p] = 0.5 * (f_kx[p] + k[p] * f_x[p] - x[p] * f_k[p]);
    free(xp); free(kp); free(kxp); free(f_kx); free(f_x); free(f_k);
}

/* Jacobi diagonal: the coefficient of x_i in A x when halo values are treated
 * as separate unknowns.  Constant: the filter centre.  Eq. (k-T):
 * 1/2 (w0 k_i + k_i w0 - f(k; w)_i). */
void or_diag(int nx, int ny, int nz, double h, const int bc[6], const double *k, double *d)
{
    double w[27];
    or_q1_filter(h, w);
    double w0 = w[13];
    size_t n = (size_t)nx * ny * nz;
    if (!k) {
        for (size_t p = 0; p < n; ++p) d[p] = w0;
        return;
    }
    double *kp = pad_alloc(nx, ny, nz), *f_k = (double *)malloc(sizeof(double) * n);
    or_pad(k, nx, ny, nz, bc, 1, kp);
    or_filter_apply(kp, nx, ny, nz, w, f_k);
    for (size_t p = 0; p < n; ++p) d[p] = 0.5 * (2.0 * w0 * k[p] - f_k[p]);
    free(kp); free(f_k);
}

/* r = b - A x (the residual forced to zero in Eqs. ph_disc / ph_disc2). */
void or_residual(int nx, int ny, int nz, double h, const int bc[6], const double *k, const double *b, const double *x,
                 double *r)
{
    size_t n = (size_t)nx * ny * nz;
    double *ax = (double *)malloc(sizeof(double) * n);
    or_apply(nx, ny, nz, h, bc, k, x, ax);
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (size_t p = 0; p < n; ++p) r[p] = b[p] - ax[p];
    free(ax);
}

/* nsweeps of weighted Jacobi, y <- y + omega (b - A y) / D (Sec. 1.2, Jacobi
 * smoothing inside the U-Net). */
void or_jacobi(int nx, int ny, int nz, double h, const int bc[6], const double *k, const double *b, double *y,
               double omega, int nsweeps)
{
    size_t n = (size_t)nx * ny * nz;
    double *d = (double *)malloc(sizeof(double) * n), *r = (double *)malloc(sizeof(double) * n);
    or_diag(nx, ny, nz, h, bc, k, d);
    for (int s = 0; s < nsweeps; ++s) {
        or_residual(nx, ny, nz, h, bc, k, b, y, r);
        #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
        for (size_t p = 0; p < n; ++p) y[p] += omega * r[p] / d[p];
    }
    free(d); free(r);
}

/* ------------------------------------------------------------------------ */
/* Grid transfers (U-Net encoder / decoder, Fig. multi-grid)                 */
/* ------------------------------------------------------------------------ */

/* rc(I,J,K) = sum of r over the 8 fine cells (2I+a, 2J+b, 2K+c). */
void or_restrict(int nx, int ny, int nz, const double *r, double *rc)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) s += r[cidx(nx, ny, 2 * I + a, 2 * J + b, 2 * K + c)];
                rc[cidx(cx, cy, I, J, K)] = s;
            }
}

/* ef = P ec, cell-centred trilinear interpolation.  Per axis the fine cell
 * 2I+a lies a quarter cell from coarse centre I towards I-1 (a = 0) or I+1
 * (a = 1): weight 3/4 on I and 1/4 on that neighbour; coarse halos follow the
 * (homogeneous) boundary conditions of the level. */
void or_prolong(int cx, int cy, int cz, const int bc[6], const double *ec, double *ef)
{
    int nx = 2 * cx, ny = 2 * cy, nz = 2 * cz;
    double *ep = pad_alloc(cx, cy, cz);
    or_pad(ec, cx, cy, cz, bc, 0, ep);
    const double wt[2] = {0.75, 0.25};
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int I = i / 2, J = j / 2, K = k / 2;
                int ox = (i % 2) ? 1 : -1, oy = (j % 2) ? 1 : -1, oz = (k % 2) ? 1 : -1;
                double s = 0.0;
                for (int r = 0; r < 2; ++r)
                    for (int q = 0; q < 2; ++q)
                        for (int p = 0; p < 2; ++p)
                            s += wt[p] * wt[q] * wt[r] * ep[pidx(cx, cy, I + p * ox, J + q * oy, K + r * oz)];
                ef[cidx(nx, ny, i, j, k)] = s;
            }
    free(ep);
}

/* Coarse coefficient: mean of the 8 children (harmonic = 8 / sum(1/k)). */
void or_coarsen_k(int nx, int ny, int nz, const double *k, double *kc, int harmonic)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    #pragma omp parallel for  /* timing build only (-fopenmp); ignored by the parity build */
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            double v = k[cidx(nx, ny, 2 * I + a, 2 * J + b, 2 * K + c)];
                            s += harmonic ? 1.0 / v : v;
                        }
                kc[cidx(cx, cy, I, J, K)] = harmonic ? 8.0 / s : s / 8.0;
            }
}

/* ------------------------------------------------------------------------ */
/* Coarsest level: dense matrix and Cholesky factorisation                   */
/* ------------------------------------------------------------------------ */

/* A (row-major n x n) with column j = A e_j. */
void or_dense(int nx, int ny, int nz, double h, const int bc[6], const double *k, double *A)
{
    size_t n = (size_t)nx * ny * nz;
    double *e = (double *)calloc(n, sizeof(double)), *col = (double *)malloc(sizeof(double) * n);
    for (size_t j = 0; j < n; ++j) {
        e[j] = 1.0;
        or_apply(nx, ny, nz, h, bc, k, e, col);
        for (size_t i = 0; i < n; ++i) A[i * n + j] = col[i];
        e[j] = 0.0;
    }
    free(e); free(col);
}

/* In-place lower Cholesky A = L L^T (row-major, lower triangle used).
 * Returns 0, or -1 on a non-positive pivot. */
int or_cholesky(int n, double *A)
{
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) s -= A[(size_t)j * n + p] * A[(size_t)j * n + p];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        A[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int p = 0; p < j; ++p) t -= A[(size_t)i * n + p] * A[(size_t)j * n + p];
            A[(size_t)i * n + j] = t / ljj;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = 0.0;
    return 0;
}

/* Solve L L^T x = b. */
void or_chol_solve(int n, const double *L, const double *b, double *x)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int p = 0; p < i; ++p) s -= L[(size_t)i * n + p] * x[p];
        x[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < n; ++p) s -= L[(size_t)p * n + i] * x[p];
        x[i] = s / L[(size_t)i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* Hierarchy and the sawtooth V-cycle (Fig. multi-grid, Sec. 2.4)            */
/* ------------------------------------------------------------------------ */

#define OR_MAX_LEVELS 16
#define OR_MAX_COARSE 4096

typedef struct {
    int L;
    int nx[OR_MAX_LEVELS], ny[OR_MAX_LEVELS], nz[OR_MAX_LEVELS];
    double h[OR_MAX_LEVELS];
    double *k[OR_MAX_LEVELS]; /* NULL for constant coefficient */
    double *b[OR_MAX_LEVELS]; /* level right-hand sides (b[0] unused) */
    double *e[OR_MAX_LEVELS]; /* level corrections */
    int bc[6];
    int singular;
    int nu_post;
    double omega;
    int nc;
    double *chol; /* nc x nc lower factor */
} or_hier;

int or_num_levels(int nx, int ny, int nz, int min_coarse)
{
    int L = 1;
    while (nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0) {
        int m = nx < ny ? nx : ny;
        m = m < nz ? m : nz;
        if (m <= min_coarse) break;
        nx /= 2; ny /= 2; nz /= 2;
        ++L;
        if (L == OR_MAX_LEVELS) break;
    }
    return L;
}

void or_free(or_hier *H)
{
    if (!H) return;
    for (int l = 0; l < H->L; ++l) {
        if (l > 0 && H->k[l]) free(H->k[l]);
        free(H->b[l]);
        free(H->e[l]);
    }
    free(H->chol);
    free(H);
}

/* Build the level chain.  k (may be NULL) is copied for level 0 only by
 * reference: the caller keeps it alive while the hierarchy is used. */
or_hier *or_setup(int nx, int ny, int nz, double h, const int bc[6], const double *k, double omega, int nu_post,
                  int min_coarse, int harmonic)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || nu_post < 1) return NULL;
    or_hier *H = (or_hier *)calloc(1, sizeof(or_hier));
    H->L = or_num_levels(nx, ny, nz, min_coarse);
    memcpy(H->bc, bc, sizeof(int) * 6);
    H->singular = 1;
    for (int f = 0; f < 6; ++f)
        if (bc[f] == OR_BC_DIRICHLET0) H->singular = 0;
    H->omega = omega;
    H->nu_post = nu_post;
    for (int l = 0; l < H->L; ++l) {
        H->nx[l] = nx >> l; H->ny[l] = ny >> l; H->nz[l] = nz >> l;
        H->h[l] = h * (double)(1 << l);
        size_t n = (size_t)H->nx[l] * H->ny[l] * H->nz[l];
        H->b[l] = (double *)calloc(n, sizeof(double));
        H->e[l] = (double *)calloc(n, sizeof(double));
        if (k) {
            if (l == 0) H->k[0] = (double *)k;
            else {
                H->k[l] = (double *)malloc(sizeof(double) * n);
                or_coarsen_k(H->nx[l - 1], H->ny[l - 1], H->nz[l - 1], H->k[l - 1], H->k[l], harmonic);
            }
        }
    }
    int c = H->L - 1;
    size_t nc = (size_t)H->nx[c] * H->ny[c] * H->nz[c];
    if (nc > OR_MAX_COARSE) { or_free(H); return NULL; }
    H->nc = (int)nc;
    H->chol = (double *)malloc(sizeof(double) * nc * nc);
    or_dense(H->nx[c], H->ny[c], H->nz[c], H->h[c], bc, H->k[c], H->chol);
    if (H->singular) {
        double cbar = 0.0;
        for (size_t i = 0; i < nc; ++i) cbar += H->chol[i * nc + i];
        cbar /= (double)nc;
        for (size_t i = 0; i < nc * nc; ++i) H->chol[i] += cbar / (double)nc;
    }
    if (or_cholesky((int)nc, H->chol) != 0) { or_free(H); return NULL; }
    return H;
}

int or_levels(const or_hier *H) { return H->L; }
int or_coarse_n(const or_hier *H) { return H->nc; }
/* Copy the level-l coefficient (for tests). */
void or_level_k(const or_hier *H, int l, double *out)
{
    size_t n = (size_t)H->nx[l] * H->ny[l] * H->nz[l];
    memcpy(out, H->k[l], sizeof(double) * n);
}

static void subtract_mean(size_t n, double *v)
{
    double s = 0.0;
    for (size_t p = 0; p < n; ++p) s += v[p];
    s /= (double)n;
    for (size_t p = 0; p < n; ++p) v[p] -= s;
}

static void coarsest_solve(or_hier *H, const double *bc_rhs, double *e)
{
    or_chol_solve(H->nc, H->chol, bc_rhs, e);
    if (H->singular) subtract_mean((size_t)H->nc, e);
}

/* One sawtooth V(0, nu_post) cycle on x for A x = b at level 0. */
void or_vcycle(or_hier *H, double *x, const double *b)
{
    int L = H->L;
    size_t n0 = (size_t)H->nx[0] * H->ny[0] * H->nz[0];
    double *r = (double *)malloc(sizeof(double) * n0);
    or_residual(H->nx[0], H->ny[0], H->nz[0], H->h[0], H->bc, H->k[0], b, x, r);
    if (L == 1) {
        coarsest_solve(H, r, H->e[0]);
        for (size_t p = 0; p < n0; ++p) x[p] += H->e[0][p];
        free(r);
        return;
    }
    /* encoder: restrict the residual down to the coarsest level; the coarse
     * initial guesses are zero, so each coarse residual is its right-hand side */
    or_restrict(H->nx[0], H->ny[0], H->nz[0], r, H->b[1]);
    for (int l = 1; l + 1 < L; ++l) or_restrict(H->nx[l], H->ny[l], H->nz[l], H->b[l], H->b[l + 1]);
    coarsest_solve(H, H->b[L - 1], H->e[L - 1]);
    /* decoder: prolongate, add, smooth */
    for (int l = L - 2; l >= 0; --l) {
        double *y = (l == 0) ? x : H->e[l];
        size_t n = (size_t)H->nx[l] * H->ny[l] * H->nz[l];
        double *pe = (double *)malloc(sizeof(double) * n);
        or_prolong(H->nx[l + 1], H->ny[l + 1], H->nz[l + 1], H->bc, H->e[l + 1], pe);
        if (l == 0)
            for (size_t p = 0; p < n; ++p) y[p] += pe[p];
        else
            for (size_t p = 0; p < n; ++p) y[p] = pe[p];
        free(pe);
        or_jacobi(H->nx[l], H->ny[l], H->nz[l], H->h[l], H->bc, H->k[l], (l == 0) ? b : H->b[l], y, H->omega,
                  H->nu_post);
    }
    free(r);
}

static double norm2(size_t n, const double *v)
{
    double s = 0.0;
    for (size_t p = 0; p < n; ++p) s += v[p] * v[p];
    return sqrt(s);
}

/* Stationary solve: relres_c = ||b - A x_c|| / ||b|| before each cycle;
 * stops when relres <= rtol (unless fixed) or after max_cycles cycles.
 * hist receives relres_0 .. relres_cycles (max_cycles + 1 entries).
 * Returns 0 converged/fixed, -4 not converged, -5 breakdown (non-finite). */
int or_solve(or_hier *H, const double *b_in, double *x, double rtol, int max_cycles, int fixed, double *hist,
             int *cycles_out)
{
    size_t n0 = (size_t)H->nx[0] * H->ny[0] * H->nz[0];
    double *b = (double *)malloc(sizeof(double) * n0), *r = (double *)malloc(sizeof(double) * n0);
    memcpy(b, b_in, sizeof(double) * n0);
    if (H->singular) subtract_mean(n0, b);
    double nb = norm2(n0, b);
    int status = 0, c = 0;
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * n0);
        if (hist) hist[0] = 0.0;
        if (cycles_out) *cycles_out = 0;
        free(b); free(r);
        return 0;
    }
    if (H->singular) subtract_mean(n0, x);
    for (c = 0;; ++c) {
        or_residual(H->nx[0], H->ny[0], H->nz[0], H->h[0], H->bc, H->k[0], b, x, r);
        double rel = norm2(n0, r) / nb;
        if (hist) hist[c] = rel;
        if (!isfinite(rel)) { status = -5; break; }
        if (!fixed && rel <= rtol) break;
        if (c == max_cycles) {
            if (!fixed) status = -4;
            break;
        }
        or_vcycle(H, x, b);
        if (H->singular) subtract_mean(n0, x);
    }
    if (cycles_out) *cycles_out = c;
    free(b); free(r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Flexible conjugate gradients around the cycle                             */
/* ------------------------------------------------------------------------ */

static double dot(size_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t p = 0; p < n; ++p) s += a[p] * b[p];
    return s;
}

/* FCG(1), flexible conjugate gradients with one direction kept (Notay,
 * SIAM J. Sci. Comput. 22, 2000), preconditioned by one sawtooth cycle from a
 * zero guess (precond = 1) or by the identity (precond = 0, plain CG).  The
 * paper repeats the cycle on its own; this outer iteration is the library's
 * addition around the same cycle, written as the plain recurrence:
 *   r = b - A x, z = M r, p = z, rho = z.r;  then per iteration
 *   t = A p, alpha = rho / p.t, x += alpha p, r -= alpha t,
 *   z = M r, beta = -(z.t) / (p.t), rho = z.r, p = z + beta p.
 * hist[c] = ||r_c|| / ||b|| with the recursively updated r, before iteration
 * c; the stopping rule and the return codes are those of or_solve.  Singular
 * problems: b projected to zero mean, x projected once at the end. */
int or_fcg(or_hier *H, const double *b_in, double *x, double rtol, int max_iter, int fixed, int precond,
           double *hist, int *iters_out)
{
    size_t n = (size_t)H->nx[0] * H->ny[0] * H->nz[0];
    double *b = (double *)malloc(sizeof(double) * n), *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n), *p = (double *)malloc(sizeof(double) * n);
    double *t = (double *)malloc(sizeof(double) * n);
    memcpy(b, b_in, sizeof(double) * n);
    if (H->singular) subtract_mean(n, b);
    double nb = norm2(n, b);
    int status = 0, c = 0;
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * n);
        if (hist) hist[0] = 0.0;
        if (iters_out) *iters_out = 0;
        free(b); free(r); free(z); free(p); free(t);
        return 0;
    }
    or_residual(H->nx[0], H->ny[0], H->nz[0], H->h[0], H->bc, H->k[0], b, x, r);
    if (precond) {
        memset(z, 0, sizeof(double) * n);
        or_vcycle(H, z, r);
    } else {
        memcpy(z, r, sizeof(double) * n);
    }
    memcpy(p, z, sizeof(double) * n);
    double rho = dot(n, z, r);
    for (c = 0;; ++c) {
        double rel = norm2(n, r) / nb;
        if (hist) hist[c] = rel;
        if (!isfinite(rel)) { status = -5; break; }
        if (!fixed && rel <= rtol) break;
        if (c == max_iter) {
            if (!fixed) status = -4;
            break;
        }
        or_apply(H->nx[0], H->ny[0], H->nz[0], H->h[0], H->bc, H->k[0], p, t);
        double pt = dot(n, p, t), alpha = rho / pt;
        for (size_t q = 0; q < n; ++q) x[q] += alpha * p[q];
        for (size_t q = 0; q < n; ++q) r[q] -= alpha * t[q];
        if (precond) {
            memset(z, 0, sizeof(double) * n);
            or_vcycle(H, z, r);
        } else {
            memcpy(z, r, sizeof(double) * n);
        }
        double beta = -dot(n, z, t) / pt;
        rho = dot(n, z, r);
        for (size_t q = 0; q < n; ++q) p[q] = z[q] + beta * p[q];
    }
    if (H->singular) subtract_mean(n, x);
    if (iters_out) *iters_out = c;
    free(b); free(r); free(z); free(p); free(t);
    return status;
}
