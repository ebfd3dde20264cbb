// Host side of the nn4mg library: level hierarchy, coarsest-level inverse,
// cycle driver and the C-ABI declared in include/nn4mg.h.
//
// The solve runs the sawtooth cycle of Fig. multi-grid (arXiv 2401.06755,
// Sec. 2.4): the residual of the finest level is restricted to every coarser
// level (the coarse initial guesses are zero, so their residuals are their
// right-hand sides), solved exactly at the bottom, then prolongated, added and
// smoothed by nu_post weighted-Jacobi sweeps on the way up.  The residual norm
// and the stopping rule are evaluated on the device after every cycle; kernels
// of later cycles exit at once when the rule has fired, so the host only
// synchronises once per batch of cycles.
#include "../../include/nn4mg.h"
#include "mg_async.h"
#include "mg_internal.h"

#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace nn4mg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(NN4MG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxLevels = 16;
constexpr int kMaxCoarse = 512;
constexpr int kDefaultZc = 16;

struct Level {
    int nx = 0, ny = 0, nz = 0;
    double h = 0.0;
    size_t n = 0;
    double *b = nullptr, *e = nullptr, *t = nullptr;  // FP64 cycle buffers
    double *k = nullptr;                              // FP64 coefficient
    float *b32 = nullptr, *e32 = nullptr, *t32 = nullptr, *t32b = nullptr;  // FP32 cycle buffers
    void *ks = nullptr;                               // FP32 / FP16 smoothing coefficient
    TileShape tiles[3]{};  // launch shape per kernel class (NN4MG_KCLASS_*)
    bool block2 = false;   // both sweeps as 8^3 blocks instead of the z-marching kernel
};

// Default launch shape of a level: the tile width that pads the x-y plane
// least (ties: the wider tile, for longer coalesced rows), and the longest
// z-chunk that still gives >= 1024 workgroups.  (Used for the single-sweep
// classes; the shapes below are what the autotuner picks on large levels.)
TileShape default_tiles(int nx, int ny, int nz, int zmul = 1)
{
    int best_tx = 64;
    double best_area = 1e300;
    for (int tx : {64, 32, 16}) {
        const int ty = 512 / tx;
        const double area = (double)((nx + tx - 1) / tx * tx) * (double)((ny + ty - 1) / ty * ty);
        if (area < best_area) {
            best_area = area;
            best_tx = tx;
        }
    }
    int zc = kDefaultZc;
    while (zc > 2 && (double)nx * ny * nz * zmul / (512.0 * zc) < 1024.0) zc /= 2;
    return make_tiles(nx, ny, nz, zc, best_tx);
}

// Longest z-chunk (power of two, at most 64) that keeps >= 512 workgroups
// (two per compute unit) for a tile of tx x ty cells.
int zchunk_for(int nx, int ny, int nz, int tx, int ty)
{
    const long tiles = (long)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
    int zc = 64;
    while (zc > 2 && tiles * ((nz + zc - 1) / zc) < 512) zc /= 2;
    return zc;
}

// Default shape per kernel class: the residual in 64-wide tiles of 2 rows per
// thread; with the two-sweep pass (nu_post == 2) the first-sweep class in
// 32-wide tiles, 2 rows per thread in FP64 and 1 with FP32 smoothing (the FP64
// run state of 64-wide tiles leaves one wave per SIMD).  zmul: the launches
// cover that many copies of the level (a batched group), so the z-chunk is
// chosen for zmul times the workgroups.
TileShape default_tiles_for(int nx, int ny, int nz, int kclass, bool mixed, bool fused, int zmul = 1)
{
    if (kclass == NN4MG_KCLASS_FINE_RESID && nx >= 64)
        return make_tiles(nx, ny, nz, zchunk_for(nx, ny, nz * zmul, 64, 8), 64, 2);
    if (kclass == NN4MG_KCLASS_FINE_SWEEP_PROLONG && fused && nx >= 32) {
        const int ry = mixed ? 1 : 2;
        return make_tiles(nx, ny, nz, zchunk_for(nx, ny, nz * zmul, 32, 8 * ry), 32, ry);
    }
    return default_tiles(nx, ny, nz, zmul);
}

int count_levels(int nx, int ny, int nz, int min_coarse)
{
    int L = 1;
    while (nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0) {
        int m = nx < ny ? nx : ny;
        m = m < nz ? m : nz;
        if (m <= min_coarse) break;
        nx /= 2;
        ny /= 2;
        nz /= 2;
        ++L;
        if (L == kMaxLevels) break;
    }
    return L;
}

int validate(const nn4mg_config *c)
{
    if (!c) return fail(NN4MG_EINVAL, "config is NULL");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1 || c->nx > 65536 || c->ny > 65536 || c->nz > 65536)
        return fail(NN4MG_EINVAL, "grid dims must be in [1, 65536]");
    if ((double)c->nx * c->ny * c->nz > 8.0e9) return fail(NN4MG_EINVAL, "grid too large");
    if (!(c->h > 0.0) || !std::isfinite(c->h)) return fail(NN4MG_EINVAL, "h must be positive");
    for (int f = 0; f < 6; ++f)
        if (c->bc[f] < 0 || c->bc[f] > 2) return fail(NN4MG_EINVAL, "unknown boundary rule");
    for (int a = 0; a < 3; ++a)
        if ((c->bc[2 * a] == NN4MG_BC_PERIODIC) != (c->bc[2 * a + 1] == NN4MG_BC_PERIODIC))
            return fail(NN4MG_EINVAL, "periodic must be set on both faces of an axis");
    if (c->coef_mode != NN4MG_COEF_CONST && c->coef_mode != NN4MG_COEF_NODAL)
        return fail(NN4MG_EINVAL, "unknown coef_mode");
    if (c->precision < 0 || c->precision > 2) return fail(NN4MG_EINVAL, "unknown precision");
    if (c->precision == NN4MG_PREC_FP16_COEF && c->coef_mode != NN4MG_COEF_NODAL)
        return fail(NN4MG_EINVAL, "FP16 coefficient storage needs a nodal coefficient");
    if (c->nu_post < 1 || c->nu_post > 64) return fail(NN4MG_EINVAL, "nu_post must be in [1, 64]");
    if (!(c->omega > 0.0 && c->omega < 2.0)) return fail(NN4MG_EINVAL, "omega must be in (0, 2)");
    if (c->min_coarse < 1) return fail(NN4MG_EINVAL, "min_coarse must be >= 1");
    if (c->outer != NN4MG_OUTER_STATIONARY && c->outer != NN4MG_OUTER_FCG)
        return fail(NN4MG_EINVAL, "unknown outer iteration");
    if (c->coarse_avg != 0 && c->coarse_avg != 1) return fail(NN4MG_EINVAL, "coarse_avg must be 0 or 1");
    for (int i = 0; i < 7; ++i)
        if (c->reserved[i] != 0) return fail(NN4MG_EINVAL, "reserved fields must be zero");
    const int L = count_levels(c->nx, c->ny, c->nz, c->min_coarse);
    const double nc = (double)(c->nx >> (L - 1)) * (c->ny >> (L - 1)) * (c->nz >> (L - 1));
    if (nc > kMaxCoarse) return fail(NN4MG_EINVAL, "coarsest level has more than 512 cells (dims not divisible enough)");
    if (c->outer == NN4MG_OUTER_FCG && L < 2) return fail(NN4MG_EINVAL, "the FCG outer iteration needs two levels or more");
    return NN4MG_OK;
}

// ---------------------------------------------------------------- host operator
// Link form of Eq. (k-T): (A x)_i = sum_{s in edges, corners} c_s (k_i + k_s)(x_i - x_s)
// with c_edge = h/12, c_corner = h/24; k == NULL: the constant-coefficient filter.
int hfold(int i, int n, int lo, int hi, int &s)
{
    if (i < 0) {
        if (lo == BC_P) return i + n;
        if (lo == BC_D) s = -s;
        return -1 - i;
    }
    if (i >= n) {
        if (hi == BC_P) return i - n;
        if (hi == BC_D) s = -s;
        return 2 * n - 1 - i;
    }
    return i;
}

void host_apply(int nx, int ny, int nz, double h, const int bc[6], const double *k, const double *x, double *y)
{
    for (int kk = 0; kk < nz; ++kk)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = (size_t)i + (size_t)nx * (j + (size_t)ny * kk);
                double acc = 0.0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int m = std::abs(dx) + std::abs(dy) + std::abs(dz);
                            if (m < 2) continue;
                            const double cs = (m == 2) ? h / 12.0 : h / 24.0;
                            int s = 1;
                            const int fi = hfold(i + dx, nx, bc[0], bc[1], s);
                            const int fj = hfold(j + dy, ny, bc[2], bc[3], s);
                            const int fk = hfold(kk + dz, nz, bc[4], bc[5], s);
                            const size_t q = (size_t)fi + (size_t)nx * (fj + (size_t)ny * fk);
                            const double kl = k ? 0.5 * (k[c] + k[q]) : 1.0;
                            acc += 2.0 * cs * kl * (x[c] - s * x[q]);
                        }
                y[c] = acc;
            }
}

// Dense coarsest matrix, rank-one shift if singular, Cholesky, explicit inverse.
int coarse_inverse(int nx, int ny, int nz, double h, const int bc[6], const double *k, int singular,
                   std::vector<double> &inv)
{
    const int n = nx * ny * nz;
    std::vector<double> A((size_t)n * n), e(n, 0.0), col(n);
    for (int j = 0; j < n; ++j) {
        e[j] = 1.0;
        host_apply(nx, ny, nz, h, bc, k, e.data(), col.data());
        for (int i = 0; i < n; ++i) A[(size_t)i * n + j] = col[i];
        e[j] = 0.0;
    }
    if (singular) {
        double cbar = 0.0;
        for (int i = 0; i < n; ++i) cbar += A[(size_t)i * n + i];
        cbar /= n;
        for (auto &v : A) v += cbar / n;
    }
    // Cholesky A = L L^T (lower, in place)
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) s -= A[(size_t)j * n + p] * A[(size_t)j * n + p];
        if (!(s > 0.0)) return fail(NN4MG_EINVAL, "coarsest matrix is not positive definite");
        const double d = std::sqrt(s);
        A[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int p = 0; p < j; ++p) t -= A[(size_t)i * n + p] * A[(size_t)j * n + p];
            A[(size_t)i * n + j] = t / d;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> y(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int p = 0; p < i; ++p) s -= A[(size_t)i * n + p] * y[p];
            y[i] = s / A[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int p = i + 1; p < n; ++p) s -= A[(size_t)p * n + i] * y[p];
            y[i] = s / A[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[(size_t)c * n + i] = y[i];
    }
    // symmetrise (the kernel reads column i as row i)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double v = 0.5 * (inv[(size_t)i * n + j] + inv[(size_t)j * n + i]);
            inv[(size_t)i * n + j] = inv[(size_t)j * n + i] = v;
        }
    return NN4MG_OK;
}

}  // namespace

struct nn4mg_hier {
    nn4mg_config cfg{};
    hipStream_t stream = nullptr;
    int L = 0;
    Level lv[kMaxLevels];
    int tail = 0;           // first level of the one-workgroup coarse end (0: none)
    void *ktail = nullptr;  // padded coefficients of the tail levels (nodal; FP64, or FP32 when mixed)
    bool fused = false;     // both post-sweeps of a level in one pass (nu_post == 2)
    int singular = 0;
    int mixed = 0;
    int kt64 = KT_NONE;     // coefficient type of FP64 launches
    int kts = KT_NONE;      // coefficient type of FP32 smoothing launches
    int nc = 0;
    double *ainv = nullptr;
    SolveState *st = nullptr;
    SolveState *st_host = nullptr;
    double *partials = nullptr;
    int max_partials = 0;
    double *scal = nullptr;  // device scalars: [0] sum, [1] mean of x, [2..7] spare
    int *flag = nullptr;
    double *fcg = nullptr;   // FCG vectors r, z, p, t = -A p at level 0, FP64
    double *fcg_part = nullptr;  // FCG dot-product partials
    size_t bytes = 0;
    // Device fields are carved from one arena: dalloc records each field and
    // its offset, place_fields makes one allocation of ncopy identical copies
    // (bstride bytes apart) and points every field into copy 0.  A batched
    // hierarchy (ncopy > 1) launches each cycle kernel once over all copies;
    // a view (view_of != nullptr) is copy c of one, with its own pointers and
    // single launches, owning nothing.
    struct Field {
        void **ptr;
        size_t off;
    };
    std::vector<Field> fields;
    size_t arena_used = 0;
    void *arena = nullptr;
    int ncopy = 1;
    long long bstride = 0;
    bool group = false;  // the server's batched form (per-copy fields, launched through batch_enqueue_cycles)
    int cap = 1;         // group: copies allocated (ncopy is the count a launch covers)
    std::vector<hipGraphExec_t> bgraph;  // group: captured cycle over copies 0 .. k - 1, by k
    const nn4mg_hier *view_of = nullptr;
    double *bw = nullptr, *xw = nullptr;  // batched: per-copy right-hand side and iterate
    std::vector<void *> allocs;
    // captured hipGraphs of one stationary iteration (body + residual + stopping
    // rule), from x into lv[0].t and back (one graph unless the finest sweeps
    // take the direct form)
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    const double *graph_b = nullptr;
    double *graph_x = nullptr;
    bool graphs_ok = true;  // cleared after a capture failure
    int tiles_epoch = 0, graph_epoch = -1;
    // async solve bookkeeping
    double solve_rtol = 0.0;
    int solve_max = 0, solve_fixed = 0, solve_enqueued = 0, solve_planned = 0;
    double solve_prev_last = -1.0;
    std::chrono::steady_clock::time_point solve_t0;
    // kernel timing (nn4mg_profile)
    bool prof_on = false;
    int cur_tag = 0;
    size_t prof_solve_begin = 0;
    std::vector<hipEvent_t> prof_ev;  // 2 per record
    std::vector<int> prof_cls, prof_tag, prof_valid, prof_lvl;
};

namespace {

constexpr size_t kArenaAlign = 256;
// Running copies a group's default launch shapes are chosen for.
constexpr int kGroupTileCopies = 4;

size_t arena_round(size_t v) { return (v + kArenaAlign - 1) & ~(kArenaAlign - 1); }

// Reserve a field of `bytes` in the arena; *p is set by place_fields.
int dalloc_bytes(nn4mg_hier *H, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 1;
    const size_t off = arena_round(H->arena_used);
    H->arena_used = off + bytes;
    H->fields.push_back({p, off});
    *p = nullptr;
    return NN4MG_OK;
}

template <typename P>
int dalloc(nn4mg_hier *H, P **p, size_t count)
{
    static_assert(sizeof(P *) == sizeof(void *), "pointer field");
    return dalloc_bytes(H, reinterpret_cast<void **>(p), (count ? count : 1) * sizeof(P));
}

// One allocation for every reserved field, ncopy times.
int place_fields(nn4mg_hier *H)
{
    const size_t A = arena_round(H->arena_used);
    void *q = nullptr;
    if (hipMalloc(&q, A * (size_t)H->ncopy) != hipSuccess) {
        (void)hipGetLastError();
        return fail(NN4MG_ENOMEM, "hipMalloc failed");
    }
    H->arena = q;
    H->allocs.push_back(q);
    H->bstride = (long long)A;
    H->bytes = A * (size_t)H->ncopy;
    for (const nn4mg_hier::Field &f : H->fields) *f.ptr = (char *)q + f.off;
    return NN4MG_OK;
}

void release(nn4mg_hier *H)
{
    if (H->view_of) return;  // a view owns nothing
    if (H->stream) (void)hipStreamSynchronize(H->stream);
    for (hipGraphExec_t &g : H->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (hipGraphExec_t &g : H->bgraph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (hipEvent_t e : H->prof_ev) (void)hipEventDestroy(e);
    H->prof_ev.clear();
    for (void *p : H->allocs) (void)hipFree(p);
    H->allocs.clear();
    if (H->st_host) (void)hipHostFree(H->st_host);
    H->st_host = nullptr;
}

size_t bytes_for(const nn4mg_config *c)
{
    const int L = count_levels(c->nx, c->ny, c->nz, c->min_coarse);
    const bool mixed = c->precision != NN4MG_PREC_FP64;
    const bool nodal = c->coef_mode == NN4MG_COEF_NODAL;
    const size_t ks = c->precision == NN4MG_PREC_FP16_COEF ? 2 : 4;
    size_t b = 0;
    size_t maxblk = 1024;
    for (int l = 0; l < L; ++l) {
        const size_t n = (size_t)(c->nx >> l) * (c->ny >> l) * (c->nz >> l);
        for (int tx : {64, 32, 16}) {
            const TileShape t = make_tiles(c->nx >> l, c->ny >> l, c->nz >> l, 2, tx);
            if ((size_t)t.blocks() > maxblk) maxblk = t.blocks();
        }
        if (nodal) b += 8 * n;
        // padded coefficient copy of a possible tail level
        if (nodal && n <= 1024) b += 8 * (size_t)((c->nx >> l) + 2) * ((c->ny >> l) + 2) * ((c->nz >> l) + 2);
        if (!mixed) {
            b += (l == 0) ? 8 * n : 24 * n;
        } else {
            b += (l == 0) ? 8 * n : 12 * n;
            if (l == 0 && c->nu_post > 2) b += 4 * n;
            if (nodal) b += ks * n;
        }
    }
    const size_t nc = (size_t)(c->nx >> (L - 1)) * (c->ny >> (L - 1)) * (c->nz >> (L - 1));
    b += 8 * nc * nc + sizeof(SolveState) + 8 * maxblk + 64 + 4;
    b += kArenaAlign * (size_t)(5 * L + 12);  // alignment of each field in the arena
    if (c->outer == NN4MG_OUTER_FCG) b += 4 * 8 * (size_t)c->nx * c->ny * c->nz + 8 * (size_t)fcg_partials_needed();
    return b;
}

// The coarse end of the cycle runs in one workgroup from the first level whose
// fields (right-hand side and two iterates per level, down to the coarsest)
// fit the LDS budget.
constexpr size_t kTailLdsBudget = 128 * 1024;
// One compute unit sweeps a 16^3 level slower than the whole chip does including
// its launch; up to about a thousand cells the single workgroup wins.
constexpr size_t kTailMaxCells = 1024;
int choose_tail(const nn4mg_hier *H)
{
    if (H->L < 2) return 0;
    const size_t elt = H->mixed ? 4 : 8;
    const int nodal = H->cfg.coef_mode == NN4MG_COEF_NODAL;
    const Level &C = H->lv[H->L - 1];
    if ((size_t)(C.nx + 2) * (C.ny + 2) * (C.nz + 2) > 2 * kTailMaxCells) return 0;  // no tail
    for (int T = 1; T < H->L; ++T) {
        if (H->L - T > kTailMaxLevels) continue;
        int nx[kTailMaxLevels], ny[kTailMaxLevels], nz[kTailMaxLevels];
        bool fits = true;
        for (int l = T; l < H->L; ++l) {
            nx[l - T] = H->lv[l].nx;
            ny[l - T] = H->lv[l].ny;
            nz[l - T] = H->lv[l].nz;
            // the workgroup covers at most two padded cells per thread
            fits = fits && (size_t)(nx[l - T] + 2) * (ny[l - T] + 2) * (nz[l - T] + 2) <= 2 * kTailMaxCells;
        }
        if (!fits) continue;
        const size_t cells = tail_field_cells(nx, ny, nz, H->L - T, nodal);
        if (cells * elt + 48 * 1024 <= kTailLdsBudget && H->lv[T].n <= kTailMaxCells) return T;
    }
    return H->lv[H->L - 1].n <= kTailMaxCells ? H->L - 1 : 0;
}

// The coarse levels' coefficients from lv[0].k (nodal): coarsening, the
// smoothing copies, the tail's padded copy.
int enqueue_coef_kernels(nn4mg_hier *H)
{
    hipStream_t s = H->stream;
    const nn4mg_config &c = H->cfg;
    const bool nodal = c.coef_mode == NN4MG_COEF_NODAL;
    if (nodal) {
        for (int l = 1; l < H->L; ++l)
            HIP_TRY(launch_coarsen_k(H->lv[l - 1].k, H->lv[l].k, H->lv[l - 1].nx, H->lv[l - 1].ny, H->lv[l - 1].nz,
                                     c.coarse_avg, s));
        if (H->mixed)
            for (int l = 0; l < H->L; ++l) HIP_TRY(launch_cast_k(H->lv[l].k, H->lv[l].ks, H->lv[l].n, H->kts, s));
        if (H->ktail) {
            size_t off = 0;
            const size_t elt = H->mixed ? sizeof(float) : sizeof(double);
            for (int l = H->tail; l < H->L; ++l) {
                const Level &V = H->lv[l];
                HIP_TRY(launch_tail_kpad(H->mixed ? 0 : 1, H->mixed ? H->kts : KT_F64,
                                         H->mixed ? V.ks : (const void *)V.k, V.nx, V.ny, V.nz, c.bc,
                                         (char *)H->ktail + off * elt, s));
                off += (size_t)(V.nx + 2) * (V.ny + 2) * (V.nz + 2);
            }
        }
    }
    return NN4MG_OK;
}

int rebuild_coefficients(nn4mg_hier *H)
{
    hipStream_t s = H->stream;
    const nn4mg_config &c = H->cfg;
    const bool nodal = c.coef_mode == NN4MG_COEF_NODAL;
    int rc0 = enqueue_coef_kernels(H);
    if (rc0) return rc0;
    const Level &C = H->lv[H->L - 1];
    std::vector<double> hk;
    if (nodal) {
        hk.resize(C.n);
        HIP_TRY(hipMemcpyAsync(hk.data(), C.k, C.n * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    std::vector<double> inv;
    int rc = coarse_inverse(C.nx, C.ny, C.nz, C.h, c.bc, nodal ? hk.data() : nullptr, H->singular, inv);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(H->ainv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return NN4MG_OK;
}

int load_k(nn4mg_hier *H, const double *k_dev)
{
    hipStream_t s = H->stream;
    Level &F = H->lv[0];
    HIP_TRY(hipMemcpyAsync(F.k, k_dev, F.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(H->flag, 0, sizeof(int), s));
    HIP_TRY(launch_check_positive(F.k, F.n, H->flag, s));
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, H->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) return fail(NN4MG_EINVAL, "coefficient k must be positive and finite");
    return rebuild_coefficients(H);
}

constexpr size_t kProfMax = 3 * 4096;

// Open a timing record for a launch of class cls; returns its index or -1.
long prof_begin(nn4mg_hier *H, int cls, int level = 0)
{
    if (!H->prof_on) return -1;
    const size_t i = H->prof_cls.size();
    if (i >= kProfMax) return -1;
    if (H->prof_ev.size() < 2 * (i + 1)) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return -1;
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return -1;
        }
        H->prof_ev.push_back(e0);
        H->prof_ev.push_back(e1);
    }
    if (hipEventRecord(H->prof_ev[2 * i], H->stream) != hipSuccess) return -1;
    H->prof_cls.push_back(cls);
    H->prof_lvl.push_back(level);
    H->prof_tag.push_back(H->cur_tag);
    H->prof_valid.push_back(1);
    return (long)i;
}

void prof_end(nn4mg_hier *H, long i)
{
    if (i < 0) return;
    if (hipEventRecord(H->prof_ev[2 * i + 1], H->stream) != hipSuccess) H->prof_valid[i] = 0;
}

// After a solve that ran `cycles` iterations: launches tagged with a later
// iteration exited early and are dropped.
void prof_close_solve(nn4mg_hier *H, int cycles, bool ran)
{
    for (size_t i = H->prof_solve_begin; i < H->prof_cls.size(); ++i)
        if (!ran || H->prof_tag[i] > cycles) H->prof_valid[i] = 0;
    H->prof_solve_begin = H->prof_cls.size();
}

StencilArgs base_args(const nn4mg_hier *H, int l, int kclass)
{
    StencilArgs a;
    std::memset(&a, 0, sizeof(a));
    const Level &V = H->lv[l];
    a.g.nx = V.nx;
    a.g.ny = V.ny;
    a.g.nz = V.nz;
    for (int f = 0; f < 6; ++f) a.g.bc[f] = H->cfg.bc[f];
    a.t = V.tiles[kclass];
    a.h = V.h;
    a.omega = H->cfg.omega;
    a.ncopy = H->ncopy;
    a.bstride = H->bstride;
    if (l + 1 < H->L) {
        a.cnx = H->lv[l + 1].nx;
        a.cny = H->lv[l + 1].ny;
        a.cnz = H->lv[l + 1].nz;
    }
    return a;
}

// Finest-level FP64 residual r = (b - bmean) - A x.  r_full / r_coarse select
// the outputs (FP32 when the handle is mixed and to_f32 is set).
int enqueue_resid(nn4mg_hier *H, const double *x, const double *b, const double *bmean, void *r_full,
                  void *r_coarse, bool to_f32, bool partials, const int *done)
{
    StencilArgs a = base_args(H, 0, NN4MG_KCLASS_FINE_RESID);
    a.yin = x;
    a.b = b;
    a.k = H->lv[0].k;
    a.bmean = bmean;
    a.r = r_full;
    a.rc = r_coarse;
    a.partials = partials ? H->partials : nullptr;
    a.done = done;
    const long pr = prof_begin(H, NN4MG_KCLASS_FINE_RESID);
    HIP_TRY(launch_stencil(1, H->kt64, IN_PLAIN, OUT_RESID, to_f32 ? 1 : 0, a, H->stream));
    prof_end(H, pr);
    return NN4MG_OK;
}

// Launch shape of the two-sweep kernel at level l: the first-sweep class's
// shape when the kernel has an instance for it.
TileShape sweep2_tiles(const nn4mg_hier *H, int l)
{
    const Level &V = H->lv[l];
    TileShape t = V.tiles[NN4MG_KCLASS_FINE_SWEEP_PROLONG];
    if (!sweep2_supports(t.tx, t.ry)) t = make_tiles(V.nx, V.ny, V.nz, t.zc, t.tx == 16 ? 16 : t.tx, t.tx == 16 ? 2 : 1);
    return t;
}

// Both sweeps of level l from P e_{l+1} against the right-hand side b:
// out_mode OUT_STORE into y, or OUT_ADD64 into x64.  With xin (FP64, marching
// form only): from xin + P e_{l+1} against b - bmean, stored into y != xin.
int enqueue_sweep2(nn4mg_hier *H, int l, const void *b, void *y, double *x64, int out_mode, const int *done,
                   const double *xin = nullptr, const double *bmean = nullptr)
{
    const bool f64 = !H->mixed;
    StencilArgs a = base_args(H, l, NN4MG_KCLASS_FINE_SWEEP_PROLONG);
    a.t = sweep2_tiles(H, l);
    a.b = b;
    a.k = f64 ? (const void *)H->lv[l].k : H->lv[l].ks;
    a.ec = f64 ? (const void *)H->lv[l + 1].e : (const void *)H->lv[l + 1].e32;
    a.yin = xin;
    a.bmean = bmean;
    a.yout = y;
    a.x64 = x64;
    a.done = done;
    const long pr = prof_begin(H, NN4MG_KCLASS_FINE_SWEEP_PROLONG, l);
    if (xin)
        HIP_TRY(launch_sweep2(1, H->kt64, IN_PROLONG_ADD, OUT_STORE, a, H->stream));
    else if (H->lv[l].block2)
        HIP_TRY(launch_sweep2_block(f64 ? 1 : 0, f64 ? H->kt64 : H->kts, out_mode, a, H->stream));
    else
        HIP_TRY(launch_sweep2(f64 ? 1 : 0, f64 ? H->kt64 : H->kts, IN_PROLONG, out_mode, a, H->stream));
    prof_end(H, pr);
    return NN4MG_OK;
}

// Largest coarse level that defaults to the 8^3 block form of the two sweeps.
constexpr size_t kBlock2MaxCells = 64 * 64 * 64;

bool level_fusable(const nn4mg_hier *H, int l)
{
    const Level &V = H->lv[l];
    return H->fused && V.nx >= 4 && V.ny >= 4 && V.nz >= 4;
}

// FP64 cycles whose finest sweeps run in the marching two-sweep pass take the
// direct form x' = S S (x + P e_1) against b - bmean: the finest residual
// kernel then writes only R r and the norm partials (no full r), and the pass
// reads x on its two-cell ring, so x' goes to a second buffer (lv[0].t) and
// successive cycles alternate between x and lv[0].t.
bool direct_fine(const nn4mg_hier *H)
{
    // batched hierarchies and their views keep the correction form: the copies
    // of a batch run from different cycle counts, so no common buffer order
    if (H->group || H->view_of) return false;
    return !H->mixed && H->L > 1 && level_fusable(H, 0) && !H->lv[0].block2;
}

// nu_post Jacobi sweeps at level l >= 1 (first input: P e_{l+1}); result in e.
int enqueue_coarse_sweeps(nn4mg_hier *H, int l, const int *done)
{
    if (level_fusable(H, l)) {
        Level &V = H->lv[l];
        const bool f64 = !H->mixed;
        return enqueue_sweep2(H, l, f64 ? (const void *)V.b : (const void *)V.b32,
                              f64 ? (void *)V.e : (void *)V.e32, nullptr, OUT_STORE, done);
    }
    Level &V = H->lv[l];
    const int nu = H->cfg.nu_post;
    const bool f64 = !H->mixed;
    void *buf[2] = {f64 ? (void *)V.t : (void *)V.t32, f64 ? (void *)V.e : (void *)V.e32};
    int cur = (nu % 2 == 1) ? 1 : 0;  // the last sweep must land in e
    const void *in = nullptr;
    for (int s = 0; s < nu; ++s) {
        StencilArgs a = base_args(H, l, s == 0 ? NN4MG_KCLASS_FINE_SWEEP_PROLONG : NN4MG_KCLASS_FINE_SWEEP);
        a.b = f64 ? (const void *)V.b : (const void *)V.b32;
        a.k = f64 ? (const void *)V.k : V.ks;
        a.yout = buf[cur];
        a.done = done;
        int in_mode = IN_PLAIN;
        if (s == 0) {
            in_mode = IN_PROLONG;
            a.ec = f64 ? (const void *)H->lv[l + 1].e : (const void *)H->lv[l + 1].e32;
        } else {
            a.yin = in;
        }
        const long pr = prof_begin(H, s == 0 ? NN4MG_KCLASS_FINE_SWEEP_PROLONG : NN4MG_KCLASS_FINE_SWEEP, l);
        HIP_TRY(launch_stencil(f64 ? 1 : 0, f64 ? H->kt64 : H->kts, in_mode, OUT_STORE, 0, a, H->stream));
        prof_end(H, pr);
        in = buf[cur];
        cur ^= 1;
    }
    return NN4MG_OK;
}

// Finest-level sweeps: FP64: x <- smooth(x + P e_1) (x_zero: smooth(P e_1), x
// not read; direct form: the result goes to x_out); mixed: x += smooth(P e_1).
int enqueue_fine_sweeps(nn4mg_hier *H, const double *b, const double *bmean, double *x, const int *done,
                        bool x_zero = false, double *x_out = nullptr)
{
    Level &F = H->lv[0];
    const int nu = H->cfg.nu_post;
    if (level_fusable(H, 0)) {
        if (H->mixed) return enqueue_sweep2(H, 0, F.b32, nullptr, x, OUT_ADD64, done);
        if (x_zero) return enqueue_sweep2(H, 0, b, x, nullptr, OUT_STORE, done);
        if (direct_fine(H)) {
            if (!x_out || x_out == x) return fail(NN4MG_EINVAL, "direct finest sweeps need a second buffer");
            return enqueue_sweep2(H, 0, b, x_out, nullptr, OUT_STORE, done, x, bmean);
        }
        // the 8^3 block form: the correction is smoothed against the full
        // residual the residual kernel wrote into F.t
        return enqueue_sweep2(H, 0, F.t, nullptr, x, OUT_ADD64, done);
    }
    if (!H->mixed) {
        void *buf[2] = {F.t, x};
        int cur = 0;
        const void *in = nullptr;
        for (int s = 0; s < nu; ++s) {
            StencilArgs a = base_args(H, 0, s == 0 ? NN4MG_KCLASS_FINE_SWEEP_PROLONG : NN4MG_KCLASS_FINE_SWEEP);
            a.b = b;
            a.bmean = bmean;
            a.k = F.k;
            a.yout = buf[cur];
            a.done = done;
            int in_mode = IN_PLAIN;
            if (s == 0) {
                in_mode = x_zero ? IN_PROLONG : IN_PROLONG_ADD;
                a.yin = x_zero ? nullptr : x;
                a.ec = H->lv[1].e;
            } else {
                a.yin = in;
            }
            const long pr = prof_begin(H, s == 0 ? NN4MG_KCLASS_FINE_SWEEP_PROLONG : NN4MG_KCLASS_FINE_SWEEP);
            HIP_TRY(launch_stencil(1, H->kt64, in_mode, OUT_STORE, 0, a, H->stream));
            prof_end(H, pr);
            in = buf[cur];
            cur ^= 1;
        }
        if (nu % 2 == 1) HIP_TRY(launch_copy(x, F.t, F.n, done, H->stream));
        return NN4MG_OK;
    }
    float *buf[2] = {F.t32, F.t32b};
    int cur = 0;
    const void *in = nullptr;
    for (int s = 0; s < nu; ++s) {
        const bool last = (s == nu - 1);
        StencilArgs a = base_args(H, 0, s == 0 ? NN4MG_KCLASS_FINE_SWEEP_PROLONG : NN4MG_KCLASS_FINE_SWEEP);
        a.b = F.b32;
        a.k = F.ks;
        a.done = done;
        int in_mode = IN_PLAIN;
        if (s == 0) {
            in_mode = IN_PROLONG;
            a.ec = H->lv[1].e32;
        } else {
            a.yin = in;
        }
        if (last) {
            a.x64 = x;
        } else {
            a.yout = buf[cur];
        }
        const long pr = prof_begin(H, s == 0 ? NN4MG_KCLASS_FINE_SWEEP_PROLONG : NN4MG_KCLASS_FINE_SWEEP);
        HIP_TRY(launch_stencil(0, H->kts, in_mode, last ? OUT_ADD64 : OUT_STORE, 0, a, H->stream));
        prof_end(H, pr);
        if (!last) {
            in = buf[cur];
            cur ^= 1;
        }
    }
    return NN4MG_OK;
}

int resid_blocks(const nn4mg_hier *H) { return H->lv[0].tiles[NN4MG_KCLASS_FINE_RESID].blocks(); }

// Everything of one cycle after the finest residual has been restricted to
// level 1 (FP64: lv[1].b; mixed: lv[1].b32 and the FP32 finest residual in
// lv[0].b32).
// stop_np > 0: the first restriction-chain launch also applies the stopping
// rule to the stop_np norm partials in H->partials.
// x_out: where the direct form of the finest sweeps puts the new iterate.
int enqueue_cycle_body(nn4mg_hier *H, const double *b, const double *bmean, double *x, const int *done,
                       bool x_zero = false, int stop_np = 0, double *x_out = nullptr)
{
    const bool f64 = !H->mixed;
    const int L = H->L;
    hipStream_t s = H->stream;
    int rc;
    if (H->tail > 0) {
        const int T = H->tail;
        // right-hand sides of levels 2 .. T - 1, up to three levels per launch
        for (int l = 1; l + 1 < T; l += 3) {
            const int depth = std::min(3, T - 1 - l);
            Level &V = H->lv[l];
            auto bof = [&](int m) -> void * {
                if (m > l + depth) return nullptr;
                return f64 ? (void *)H->lv[m].b : (void *)H->lv[m].b32;
            };
            // the first launch may also run the stopping rule (on the residual
            // the previous stationary cycle ended with, or on FCG's updated r)
            const bool stop_here = stop_np > 0 && l == 1;
            HIP_TRY(launch_restrict_chain(f64 ? 1 : 0, f64 ? (void *)V.b : (void *)V.b32, bof(l + 1), bof(l + 2),
                                          bof(l + 3), V.nx, V.ny, V.nz, depth, done, s, stop_here ? H->st : nullptr,
                                          stop_here ? H->partials : nullptr, stop_here ? stop_np : 0, H->ncopy,
                                          H->bstride));
        }
        TailArgs ta;
        std::memset(&ta, 0, sizeof(ta));
        ta.levels = L - T;
        for (int l = T; l < L; ++l) {
            const Level &V = H->lv[l];
            ta.nx[l - T] = V.nx;
            ta.ny[l - T] = V.ny;
            ta.nz[l - T] = V.nz;
            ta.h[l - T] = V.h;
        }
        ta.kpad = H->ktail;
        if (T >= 2)
            ta.b_above = f64 ? (const void *)H->lv[T - 1].b : (const void *)H->lv[T - 1].b32;
        else
            ta.b_first = f64 ? (const void *)H->lv[T].b : (const void *)H->lv[T].b32;
        ta.e_first = f64 ? (void *)H->lv[T].e : (void *)H->lv[T].e32;
        ta.ainv = H->ainv;
        ta.ainv_in_lds = (size_t)H->nc * H->nc * 8 <= 48 * 1024;
        ta.singular = H->singular;
        for (int f = 0; f < 6; ++f) ta.bc[f] = H->cfg.bc[f];
        ta.omega = H->cfg.omega;
        ta.nu = H->cfg.nu_post;
        ta.done = done;
        ta.ncopy = H->ncopy;
        ta.bstride = H->bstride;
        HIP_TRY(launch_tail(f64 ? 1 : 0, f64 ? H->kt64 : H->kts, ta, s));
        for (int l = T - 1; l >= 1; --l)
            if ((rc = enqueue_coarse_sweeps(H, l, done))) return rc;
        return enqueue_fine_sweeps(H, b, bmean, x, done, x_zero, x_out);
    }
    for (int l = 1; l + 1 < L; ++l) {
        Level &V = H->lv[l];
        HIP_TRY(launch_restrict(f64 ? 1 : 0, f64 ? (void *)V.b : (void *)V.b32,
                                f64 ? (void *)H->lv[l + 1].b : (void *)H->lv[l + 1].b32, V.nx, V.ny, V.nz, done, s));
    }
    Level &C = H->lv[L - 1];
    HIP_TRY(launch_coarse_solve(f64 ? 1 : 0, f64 ? (void *)C.b : (void *)C.b32, f64 ? (void *)C.e : (void *)C.e32,
                                H->ainv, H->nc, H->singular, done, s));
    for (int l = L - 2; l >= 1; --l)
        if ((rc = enqueue_coarse_sweeps(H, l, done))) return rc;
    return enqueue_fine_sweeps(H, b, bmean, x, done, x_zero, x_out);
}

// One outer iteration starting with the finest residual.  For a single-level
// hierarchy the whole problem is the coarsest one.
int enqueue_resid_for_cycle(nn4mg_hier *H, const double *b, const double *x, const double *bmean, bool with_norm,
                            const int *done)
{
    if (H->L == 1) {
        Level &F = H->lv[0];
        return enqueue_resid(H, x, b, bmean, H->mixed ? (void *)F.b32 : (void *)F.b, nullptr, H->mixed, with_norm,
                             done);
    }
    if (H->mixed)
        return enqueue_resid(H, x, b, bmean, H->lv[0].b32, H->lv[1].b32, true, with_norm, done);
    // the 8^3 block form of the finest sweeps smooths the correction against
    // the full residual; the direct form needs none
    const bool full = H->fused && !direct_fine(H);
    return enqueue_resid(H, x, b, bmean, full ? H->lv[0].t : nullptr, H->lv[1].b, false, with_norm, done);
}

int enqueue_single_level_body(nn4mg_hier *H, double *x, const int *done)
{
    Level &F = H->lv[0];
    hipStream_t s = H->stream;
    if (!H->mixed) {
        HIP_TRY(launch_coarse_solve(1, F.b, F.e, H->ainv, H->nc, H->singular, done, s));
        HIP_TRY(launch_add(x, F.e, 0, F.n, done, s));
    } else {
        HIP_TRY(launch_coarse_solve(0, F.b32, F.e32, H->ainv, H->nc, H->singular, done, s));
        HIP_TRY(launch_add(x, F.e32, 1, F.n, done, s));
    }
    return NN4MG_OK;
}

// The stationary solve's stopping rule runs inside the cycle's first
// restriction-chain launch when there is one (levels between the finest and
// the coarse end); otherwise as its own launch after each residual.
bool stop_in_chain(const nn4mg_hier *H) { return H->L > 1 && H->tail > 2; }

// One cycle body from x; the new iterate is in x, or (direct_fine) in x_out.
int enqueue_body(nn4mg_hier *H, const double *b, const double *bmean, double *x, const int *done,
                 bool with_stop = false, double *x_out = nullptr)
{
    if (H->L == 1) return enqueue_single_level_body(H, x, done);
    return enqueue_cycle_body(H, b, bmean, x, done, false, with_stop && stop_in_chain(H) ? resid_blocks(H) : 0,
                              x_out);
}

// One cycle (finest residual, then the body) from x back into x, as the
// one-cycle entry point and the autotuner's trials run it.  The direct form
// goes through lv[0].t; `par` selects the way round (the autotuner alternates
// and ends on x).
int enqueue_cycle_inplace(nn4mg_hier *H, const double *b, double *x, int par = -1)
{
    int rc;
    if (!direct_fine(H)) {
        if ((rc = enqueue_resid_for_cycle(H, b, x, nullptr, false, nullptr))) return rc;
        return enqueue_body(H, b, nullptr, x, nullptr);
    }
    double *t = H->lv[0].t;
    double *src = par == 1 ? t : x, *dst = par == 1 ? x : t;
    if ((rc = enqueue_resid_for_cycle(H, b, src, nullptr, false, nullptr))) return rc;
    if ((rc = enqueue_body(H, b, nullptr, src, nullptr, false, dst))) return rc;
    if (par < 0) HIP_TRY(launch_copy(x, t, H->lv[0].n, nullptr, H->stream));
    return NN4MG_OK;
}

}  // namespace

// ============================================================================ C-ABI

extern "C" {

void nn4mg_config_default(nn4mg_config *cfg, int nx, int ny, int nz, double h)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->nx = nx;
    cfg->ny = ny;
    cfg->nz = nz;
    cfg->h = h;
    for (int f = 0; f < 6; ++f) cfg->bc[f] = NN4MG_BC_DIRICHLET0;
    cfg->coef_mode = NN4MG_COEF_CONST;
    cfg->precision = NN4MG_PREC_FP64;
    cfg->nu_post = 2;
    cfg->omega = 2.0 / 3.0;
    cfg->min_coarse = 4;
    cfg->outer = NN4MG_OUTER_STATIONARY;
    cfg->coarse_avg = 0;
}

size_t nn4mg_bytes_required(const nn4mg_config *cfg)
{
    if (validate(cfg) != NN4MG_OK) return 0;
    return bytes_for(cfg);
}

const char *nn4mg_last_error(void) { return g_err.c_str(); }


int nn4mg_destroy(nn4mg_t h)
{
    if (!h) return NN4MG_OK;
    release(h);
    delete h;
    return NN4MG_OK;
}

int nn4mg_setup(const nn4mg_config *cfg, const double *k_dev, void *hip_stream, nn4mg_t *out)
{
    if (!out) return fail(NN4MG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    if (cfg->coef_mode == NN4MG_COEF_NODAL && !k_dev) return fail(NN4MG_EINVAL, "nodal coefficient requires k");
    return nn4mg::setup_hier(cfg, k_dev, (hipStream_t)hip_stream, 1, out);
}

}  // extern "C"

// A hierarchy of ncopy identical copies (validated cfg).  With one copy the
// coefficient is set up from k_dev; a batched hierarchy gets its per-copy
// right-hand side and iterate fields, and each copy's coefficient is set up
// through its view.
int nn4mg::setup_hier(const nn4mg_config *cfg, const double *k_dev, hipStream_t stream, int ncopy, nn4mg_hier **out,
                      bool group)
{
    *out = nullptr;
    if (ncopy < 1 || (ncopy > 1 && !group)) return fail(NN4MG_EINVAL, "several copies are a batched group");
    const bool nodal = cfg->coef_mode == NN4MG_COEF_NODAL;
    nn4mg_hier *H = new nn4mg_hier();
    H->cfg = *cfg;
    H->stream = stream;
    H->ncopy = ncopy;
    H->cap = ncopy;
    H->group = group;
    if (group) H->bgraph.assign((size_t)ncopy + 1, nullptr);
    H->L = count_levels(cfg->nx, cfg->ny, cfg->nz, cfg->min_coarse);
    H->mixed = cfg->precision != NN4MG_PREC_FP64;
    H->singular = 1;
    for (int f = 0; f < 6; ++f)
        if (cfg->bc[f] == NN4MG_BC_DIRICHLET0) H->singular = 0;
    H->kt64 = nodal ? KT_F64 : KT_NONE;
    H->kts = !nodal ? KT_NONE : (cfg->precision == NN4MG_PREC_FP16_COEF ? KT_F16 : KT_F32);
    int maxblk = 1024;
#define TRY(x)                    \
    do {                          \
        int r_ = (x);             \
        if (r_) {                 \
            nn4mg_destroy(H);     \
            return r_;            \
        }                         \
    } while (0)
    for (int l = 0; l < H->L; ++l) {
        Level &V = H->lv[l];
        V.nx = cfg->nx >> l;
        V.ny = cfg->ny >> l;
        V.nz = cfg->nz >> l;
        V.h = cfg->h * (double)(1 << l);
        V.n = (size_t)V.nx * V.ny * V.nz;
        // a group's launches usually cover several running copies (the same
        // shapes whatever the group's size, so a request's result does not
        // depend on the group it runs in)
        const int zmul = group ? kGroupTileCopies : 1;
        for (int c = 0; c < 3; ++c)
            V.tiles[c] = default_tiles_for(V.nx, V.ny, V.nz, c, H->mixed, cfg->nu_post == 2 && H->L >= 2, zmul);
        if (V.tiles[0].blocks() > maxblk) maxblk = V.tiles[0].blocks();
        if (nodal) TRY(dalloc(H, &V.k, V.n));
        const bool single = (H->L == 1);
        if (!H->mixed) {
            TRY(dalloc(H, &V.t, V.n));
            if (l > 0 || single) {
                TRY(dalloc(H, &V.b, V.n));
                TRY(dalloc(H, &V.e, V.n));
            }
        } else {
            TRY(dalloc(H, &V.b32, V.n));
            TRY(dalloc(H, &V.t32, V.n));
            if (l > 0 || single) TRY(dalloc(H, &V.e32, V.n));
            if (l == 0 && cfg->nu_post > 2) TRY(dalloc(H, &V.t32b, V.n));
            if (nodal) TRY(dalloc_bytes(H, &V.ks, V.n * (H->kts == KT_F16 ? sizeof(__half) : sizeof(float))));
        }
    }
    for (int l = 0; l < H->L; ++l)
        for (int tx : {64, 32, 16}) {
            const int nb = make_tiles(H->lv[l].nx, H->lv[l].ny, H->lv[l].nz, 2, tx, 2).blocks();
            if (nb > maxblk) maxblk = nb;
        }
    const Level &C = H->lv[H->L - 1];
    H->nc = (int)C.n;
    H->tail = choose_tail(H);
    H->fused = cfg->nu_post == 2 && H->L >= 2;
    if (group && (H->L < 2 || H->tail == 0 || !H->fused || cfg->outer != NN4MG_OUTER_STATIONARY)) {
        nn4mg_destroy(H);
        return fail(NN4MG_EINVAL, "no batched form: needs the stationary cycle, two post-sweeps and a one-workgroup "
                                  "coarse end");
    }
    // coarse levels of up to 64^3 cells: the block form of the two sweeps is
    // shorter than a march over z (the autotuner re-decides per level)
    for (int l = 1; l < H->L; ++l) H->lv[l].block2 = level_fusable(H, l) && H->lv[l].n <= kBlock2MaxCells;
    if (nodal && H->tail > 0) {
        size_t cells = 0;
        for (int l = H->tail; l < H->L; ++l)
            cells += (size_t)(H->lv[l].nx + 2) * (H->lv[l].ny + 2) * (H->lv[l].nz + 2);
        TRY(dalloc_bytes(H, &H->ktail, cells * (H->mixed ? sizeof(float) : sizeof(double))));
    }
    TRY(dalloc(H, &H->ainv, (size_t)H->nc * H->nc));
    TRY(dalloc(H, &H->st, 1));
    TRY(dalloc(H, &H->partials, (size_t)maxblk));
    H->max_partials = maxblk;
    TRY(dalloc(H, &H->scal, 8));
    TRY(dalloc(H, &H->flag, 1));
    if (cfg->outer == NN4MG_OUTER_FCG) {
        TRY(dalloc(H, &H->fcg, 4 * H->lv[0].n));
        TRY(dalloc(H, &H->fcg_part, (size_t)fcg_partials_needed()));
    }
    if (group) {
        TRY(dalloc(H, &H->bw, H->lv[0].n));
        TRY(dalloc(H, &H->xw, H->lv[0].n));
    }
    TRY(place_fields(H));
    if (hipHostMalloc((void **)&H->st_host, sizeof(SolveState) * (size_t)ncopy, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        nn4mg_destroy(H);
        return fail(NN4MG_ENOMEM, "pinned host allocation failed");
    }
    if (!group) {
        if (nodal)
            TRY(load_k(H, k_dev));
        else
            TRY(rebuild_coefficients(H));
    }
#undef TRY
    *out = H;
    return NN4MG_OK;
}

extern "C" {

int nn4mg_update_coef(nn4mg_t H, const double *k_dev)
{
    if (!H) return fail(NN4MG_EINVAL, "handle is NULL");
    if (H->cfg.coef_mode != NN4MG_COEF_NODAL) return fail(NN4MG_EINVAL, "handle has a constant coefficient");
    if (!k_dev) return fail(NN4MG_EINVAL, "k is NULL");
    return load_k(H, k_dev);
}

int nn4mg_levels(nn4mg_t H, int *levels, int *dims, int max_levels)
{
    if (!H) return fail(NN4MG_EINVAL, "handle is NULL");
    if (levels) *levels = H->L;
    if (dims)
        for (int l = 0; l < H->L && l < max_levels; ++l) {
            dims[3 * l] = H->lv[l].nx;
            dims[3 * l + 1] = H->lv[l].ny;
            dims[3 * l + 2] = H->lv[l].nz;
        }
    return NN4MG_OK;
}

size_t nn4mg_bytes_held(nn4mg_t H) { return H ? H->bytes : 0; }

int nn4mg_residual(nn4mg_t H, const double *x, const double *b, double *r, double *norm2_out)
{
    if (!H || !x || !b) return fail(NN4MG_EINVAL, "NULL argument");
    StencilArgs a = base_args(H, 0, NN4MG_KCLASS_FINE_RESID);
    a.yin = x;
    a.b = b;
    a.k = H->lv[0].k;
    a.r = r;
    a.partials = norm2_out ? H->partials : nullptr;
    HIP_TRY(launch_stencil(1, H->kt64, IN_PLAIN, OUT_RESID, 0, a, H->stream));
    if (norm2_out) {
        HIP_TRY(launch_reduce(H->partials, resid_blocks(H), 1.0, H->scal, H->stream));
        double s = 0.0;
        HIP_TRY(hipMemcpyAsync(&s, H->scal, sizeof(double), hipMemcpyDeviceToHost, H->stream));
        HIP_TRY(hipStreamSynchronize(H->stream));
        *norm2_out = std::sqrt(s);
    }
    return NN4MG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free residual
// Device memory of nn4mg_residual_noalloc: the residual kernel's per-workgroup
// sums of r^2 and the reduced sum.  Each GPU holds its own copy for the life
// of the process; calls on one GPU share it.
constexpr int kStaticPartials = 1 << 18;                 // workgroups of one residual launch, at most
constexpr int kStaticDoubles = kStaticPartials + 32;     // + the reduced sum (own 256-byte line)
static __device__ __align__(256) double scratch[kStaticDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current; the host-side name is not a device address).
int static_scratch(double **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NN4MG_EDEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(NN4MG_EDEVICE, "hipGetSymbolAddress returned NULL for the static scratch");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return NN4MG_OK;
}

}  // namespace

extern "C" {

int nn4mg_residual_noalloc(const nn4mg_config *cfg, const double *k_dev, const double *x_dev, const double *b_dev,
                           double *r_dev, double *norm2_out, void *hip_stream)
{
    int rc;
    if ((rc = validate(cfg))) return rc;
    if (!x_dev || !b_dev) return fail(NN4MG_EINVAL, "NULL argument");
    const bool nodal = cfg->coef_mode == NN4MG_COEF_NODAL;
    if (nodal && !k_dev) return fail(NN4MG_EINVAL, "nodal coefficient mode needs k");
    const int L = count_levels(cfg->nx, cfg->ny, cfg->nz, cfg->min_coarse);
    const bool mixed = cfg->precision != NN4MG_PREC_FP64;
    StencilArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g.nx = cfg->nx;
    a.g.ny = cfg->ny;
    a.g.nz = cfg->nz;
    for (int f = 0; f < 6; ++f) a.g.bc[f] = cfg->bc[f];
    // the launch shape nn4mg_setup gives the finest residual of this config
    a.t = default_tiles_for(cfg->nx, cfg->ny, cfg->nz, NN4MG_KCLASS_FINE_RESID, mixed, cfg->nu_post == 2 && L >= 2);
    a.h = cfg->h;
    a.omega = cfg->omega;
    a.yin = x_dev;
    a.b = b_dev;
    a.k = nodal ? k_dev : nullptr;
    a.r = r_dev;
    const int nblk = a.t.blocks();
    if (norm2_out && nblk > kStaticPartials)
        return fail(NN4MG_EINVAL, "grid needs " + std::to_string(nblk) + " residual workgroups; the static scratch holds " +
                                      std::to_string(kStaticPartials));
    double *ptr = nullptr;
    if (norm2_out && (rc = static_scratch(&ptr))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    a.partials = norm2_out ? ptr : nullptr;
    HIP_TRY(launch_stencil(1, nodal ? KT_F64 : KT_NONE, IN_PLAIN, OUT_RESID, 0, a, st));
    if (norm2_out) {
        // every workgroup writes its partial, so nothing needs clearing first
        HIP_TRY(launch_reduce(ptr, nblk, 1.0, ptr + kStaticPartials, st));
        double sum = 0.0;
        HIP_TRY(hipMemcpyAsync(&sum, ptr + kStaticPartials, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *norm2_out = std::sqrt(sum);
    }
    return NN4MG_OK;
}

}  // extern "C"

namespace {

struct StateHeader {
    double nb, bmean, rtol;
    int max_cycles, fixed, nres, done, status, pad_;
    double last;
};
static_assert(sizeof(StateHeader) == offsetof(SolveState, hist), "state header layout");

int read_header(nn4mg_hier *H, StateHeader *hd)
{
    HIP_TRY(hipMemcpyAsync(H->st_host, H->st, sizeof(StateHeader), hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    std::memcpy(hd, H->st_host, sizeof(StateHeader));
    return NN4MG_OK;
}

// ||b - mean|| (mean only for singular problems) into st->nb, st->bmean.
int enqueue_b_norm(nn4mg_hier *H, const double *b)
{
    const size_t n = H->lv[0].n;
    hipStream_t s = H->stream;
    if (H->singular) {
        HIP_TRY(launch_sum_partials(b, n, nullptr, 1, H->partials, s));
        HIP_TRY(launch_reduce(H->partials, sum_blocks(n), 1.0 / (double)n, &H->st->bmean, s));
    }
    HIP_TRY(launch_sum_partials(b, n, H->singular ? &H->st->bmean : nullptr, 2, H->partials, s));
    HIP_TRY(launch_reduce(H->partials, sum_blocks(n), 1.0, H->scal, s));
    HIP_TRY(launch_set_nb(H->st, H->scal, s));
    return NN4MG_OK;
}

// Iteration `par` (0 or 1, the parity of its index in the solve): with the
// direct finest sweeps, even iterations take x to lv[0].t and odd ones back.
int enqueue_stationary_iteration(nn4mg_hier *H, const double *b, double *x, int par)
{
    int rc;
    H->cur_tag += 1;
    const int *done = &H->st->done;
    const double *bmean = H->singular ? &H->st->bmean : nullptr;
    double *src = x, *dst = x;
    if (direct_fine(H)) {
        src = par ? H->lv[0].t : x;
        dst = par ? x : H->lv[0].t;
    }
    if ((rc = enqueue_body(H, b, bmean, src, done, true, dst))) return rc;
    if ((rc = enqueue_resid_for_cycle(H, b, dst, bmean, true, done))) return rc;
    // with the rule in the next cycle's chain, the residual is judged there
    // (or by the stand-alone launch that ends each batch)
    if (!stop_in_chain(H))
        HIP_TRY(launch_finish_norm(H->st, H->partials, resid_blocks(H), H->stream, 0, H->ncopy, H->bstride));
    return NN4MG_OK;
}

// ---- flexible CG outer iteration: one sawtooth cycle from zero is the
// preconditioner M.  Vectors (level 0, FP64): r, z, p, t = -A p.
struct FcgVec {
    double *r, *z, *p, *t;
};
FcgVec fcg_vec(nn4mg_hier *H)
{
    const size_t n = H->lv[0].n;
    return FcgVec{H->fcg, H->fcg + n, H->fcg + 2 * n, H->fcg + 3 * n};
}

// z = M r.  FP64: the cycle's right-hand side is r itself; mixed: the FP32
// copy of r already sits in lv[0].b32 and the cycle adds its correction to z.
// stop_np > 0: the cycle's first restriction-chain launch applies the
// stopping rule to that many norm partials (the caller checked stop_in_chain).
int enqueue_precondition(nn4mg_hier *H, const double *r, double *z, const int *done, int stop_np = 0)
{
    Level &F = H->lv[0];
    hipStream_t s = H->stream;
    if (!H->mixed) {
        HIP_TRY(launch_restrict(1, r, H->lv[1].b, F.nx, F.ny, F.nz, done, s));
        return enqueue_cycle_body(H, r, nullptr, z, done, true, stop_np);
    }
    HIP_TRY(launch_restrict(0, F.b32, H->lv[1].b32, F.nx, F.ny, F.nz, done, s));
    HIP_TRY(launch_zero(z, F.n, done, s));
    return enqueue_cycle_body(H, nullptr, nullptr, z, done, false, stop_np);
}

// Start: r = (b - mean) - A x, its norm (stopping rule), z = M r, rho = z.r, p = z.
int enqueue_fcg_start(nn4mg_hier *H, const double *b, double *x)
{
    const FcgVec v = fcg_vec(H);
    const size_t n = H->lv[0].n;
    hipStream_t s = H->stream;
    const int *done = &H->st->done;
    int rc;
    if ((rc = enqueue_resid(H, x, b, H->singular ? &H->st->bmean : nullptr, v.r, nullptr, false, true, done)))
        return rc;
    HIP_TRY(launch_finish_norm(H->st, H->partials, resid_blocks(H), s));
    if (H->mixed) HIP_TRY(launch_cast_f32(v.r, H->lv[0].b32, n, done, s));
    if ((rc = enqueue_precondition(H, v.r, v.z, done))) return rc;
    HIP_TRY(launch_fcg_dots(v.z, v.r, nullptr, n, H->fcg_part, H->st, 0, s));
    HIP_TRY(launch_copy(v.p, v.z, n, done, s));
    return NN4MG_OK;
}

// One FCG(1) iteration: t = -A p, alpha, x and r update with the stopping
// rule on ||r||, z = M r, beta, p = z + beta p.
int enqueue_fcg_iteration(nn4mg_hier *H, double *x)
{
    const FcgVec v = fcg_vec(H);
    const size_t n = H->lv[0].n;
    hipStream_t s = H->stream;
    const int *done = &H->st->done;
    int rc;
    H->cur_tag += 1;
    {   // t = -A p with per-block partials of p.t, then alpha
        StencilArgs a = base_args(H, 0, NN4MG_KCLASS_FINE_RESID);
        a.yin = v.p;
        a.b = nullptr;  // t = 0 - A p
        a.k = H->lv[0].k;
        a.r = v.t;
        a.partials = H->partials;
        a.dot_x = 1;
        a.done = done;
        const long pr = prof_begin(H, NN4MG_KCLASS_FINE_RESID);
        HIP_TRY(launch_stencil(1, H->kt64, IN_PLAIN, OUT_RESID, 0, a, s));
        prof_end(H, pr);
        HIP_TRY(launch_fcg_alpha_partials(H->partials, resid_blocks(H), H->st, s));
    }
    HIP_TRY(launch_fcg_update(H->st, x, v.p, v.r, v.t, H->mixed ? H->lv[0].b32 : nullptr, n, H->partials, s));
    // the stopping rule on ||r|| runs in the preconditioning cycle's first
    // chain launch when it has one (the restriction before it runs regardless)
    const bool fold = stop_in_chain(H);
    if (!fold) HIP_TRY(launch_finish_norm(H->st, H->partials, fcg_update_blocks(n), s));
    if ((rc = enqueue_precondition(H, v.r, v.z, done, fold ? fcg_update_blocks(n) : 0))) return rc;
    HIP_TRY(launch_fcg_dots(v.z, v.r, v.t, n, H->fcg_part, H->st, 2, s));
    HIP_TRY(launch_fcg_direction(H->st, v.z, v.p, n, s));
    return NN4MG_OK;
}

int enqueue_iteration(nn4mg_hier *H, const double *b, double *x, int par)
{
    if (H->cfg.outer == NN4MG_OUTER_FCG) return enqueue_fcg_iteration(H, x);
    return enqueue_stationary_iteration(H, b, x, par);
}

// Parity of iteration `index` of a solve: which graph (and buffer order) it uses.
int iteration_parity(const nn4mg_hier *H, int index)
{
    return (H->cfg.outer != NN4MG_OUTER_FCG && direct_fine(H)) ? (index & 1) : 0;
}

// The end of a solve in two halves.  enqueue: from the state header hd (the
// solve is over), move the iterate into x if the last direct-form cycle left
// it in lv[0].t, zero it for a zero right-hand side or remove its mean for a
// singular problem, and copy the whole state to H->st_host.  complete (once
// that copy has arrived): the status and info.
int finish_enqueue(nn4mg_hier *H, double *x, const StateHeader &hd)
{
    hipStream_t s = H->stream;
    const size_t n = H->lv[0].n;
    // an odd number of direct-form cycles leaves the iterate in lv[0].t
    if (iteration_parity(H, hd.nres > 0 ? hd.nres - 1 : 0)) HIP_TRY(launch_copy(x, H->lv[0].t, n, nullptr, s));
    if (hd.nb == 0.0) {
        HIP_TRY(launch_fill(x, n, 0.0, s));
    } else if (H->singular && hd.status != -5) {
        HIP_TRY(launch_sum_partials(x, n, nullptr, 1, H->partials, s));
        HIP_TRY(launch_reduce(H->partials, sum_blocks(n), 1.0 / (double)n, H->scal + 1, s));
        HIP_TRY(launch_sub_scalar(x, n, H->scal + 1, s));
    }
    HIP_TRY(hipMemcpyAsync(H->st_host, H->st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
    return NN4MG_OK;
}

int finish_complete(nn4mg_hier *H, nn4mg_info *info, std::chrono::steady_clock::time_point t0)
{
    const SolveState &S = *H->st_host;
    prof_close_solve(H, S.nres - 1, S.nb > 0.0);
    int status = NN4MG_OK;
    if (S.status == -4) status = fail(NN4MG_ENOTCONV, "max_cycles reached before rtol");
    if (S.status == -5)
        status = fail(NN4MG_EBREAKDOWN, "breakdown: non-finite residual, residual grown past 1e3 times the first, "
                                         "or a non-positive p.Ap in flexible CG");
    if (info) {
        info->cycles = S.nres > 0 ? S.nres - 1 : 0;
        info->status = status;
        info->relres0 = S.hist[0];
        info->relres = S.last;
        info->hist_len = S.nres < NN4MG_HIST_MAX ? S.nres : NN4MG_HIST_MAX;
        for (int i = 0; i < info->hist_len; ++i) info->hist[i] = S.hist[i];
        info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int finish_solve(nn4mg_hier *H, double *x, nn4mg_info *info, std::chrono::steady_clock::time_point t0)
{
    StateHeader hd;
    int rc;
    if ((rc = read_header(H, &hd))) return rc;
    if ((rc = finish_enqueue(H, x, hd))) return rc;
    HIP_TRY(hipStreamSynchronize(H->stream));
    return finish_complete(H, info, t0);
}

// Capture one stationary iteration of parity `par` on the handle's stream as
// a graph bound to (b, x).  Returns false (and launches nothing) if capture is
// not possible.
bool capture_iteration(nn4mg_hier *H, const double *b, double *x, int par)
{
    if (!H->graphs_ok || H->stream == nullptr || H->prof_on) return false;
    if (H->graph_b != b || H->graph_x != x || H->graph_epoch != H->tiles_epoch) {
        for (hipGraphExec_t &ge : H->graph)
            if (ge) {
                (void)hipGraphExecDestroy(ge);
                ge = nullptr;
            }
        H->graph_b = b;
        H->graph_x = x;
        H->graph_epoch = H->tiles_epoch;
    }
    if (H->graph[par]) return true;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(H->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        H->graphs_ok = false;
        return false;
    }
    const int saved_tag = H->cur_tag;
    const int rc = enqueue_iteration(H, b, x, par);
    H->cur_tag = saved_tag;
    const hipError_t e = hipStreamEndCapture(H->stream, &g);
    if (rc != NN4MG_OK || e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        H->graphs_ok = false;
        return false;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        (void)hipGetLastError();
        H->graphs_ok = false;
        return false;
    }
    H->graph[par] = ex;
    return true;
}

}  // namespace

namespace nn4mg {

// ---- asynchronous solve pieces (used by nn4mg_solve and the server) ----

int solve_begin(nn4mg_hier *H, const double *b, double *x, double rtol, int max_cycles, int fixed)
{
    hipStream_t s = H->stream;
    int rc;
    H->solve_t0 = std::chrono::steady_clock::now();
    H->solve_rtol = rtol;
    H->solve_max = max_cycles;
    H->solve_fixed = fixed;
    H->solve_enqueued = 0;
    H->solve_prev_last = -1.0;
    H->solve_planned = fixed ? max_cycles : (max_cycles < 4 ? max_cycles : 4);
    HIP_TRY(launch_init_state(H->st, rtol, max_cycles, fixed, s));
    H->cur_tag = 0;
    H->prof_solve_begin = H->prof_cls.size();
    if ((rc = enqueue_b_norm(H, b))) return rc;
    if (H->cfg.outer == NN4MG_OUTER_FCG) return enqueue_fcg_start(H, b, x);
    if ((rc = enqueue_resid_for_cycle(H, b, x, H->singular ? &H->st->bmean : nullptr, true, &H->st->done))) return rc;
    HIP_TRY(launch_finish_norm(H->st, H->partials, resid_blocks(H), s, stop_in_chain(H) ? 1 : 0));
    return NN4MG_OK;
}

// Enqueue the next planned batch of cycles (as graph launches when possible).
int solve_enqueue_next(nn4mg_hier *H, const double *b, double *x)
{
    int rc;
    const int n = H->solve_planned;
    if (n <= 0) return NN4MG_OK;
    const int p0 = iteration_parity(H, H->solve_enqueued), p1 = iteration_parity(H, H->solve_enqueued + 1);
    if (capture_iteration(H, b, x, p0) && (n == 1 || capture_iteration(H, b, x, p1))) {
        for (int c = 0; c < n; ++c)
            HIP_TRY(hipGraphLaunch(H->graph[iteration_parity(H, H->solve_enqueued + c)], H->stream));
        H->cur_tag += n;
    } else {
        for (int c = 0; c < n; ++c)
            if ((rc = enqueue_iteration(H, b, x, iteration_parity(H, H->solve_enqueued + c)))) return rc;
    }
    // the last residual of the batch is judged before the host reads the state
    if (H->cfg.outer != NN4MG_OUTER_FCG && stop_in_chain(H))
        HIP_TRY(launch_finish_norm(H->st, H->partials, resid_blocks(H), H->stream, 1));
    H->solve_enqueued += n;
    return NN4MG_OK;
}

int solve_header_async(nn4mg_hier *H, hipEvent_t ev)
{
    HIP_TRY(hipMemcpyAsync(H->st_host, H->st, sizeof(StateHeader), hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipEventRecord(ev, H->stream));
    return NN4MG_OK;
}

// After the header copy completed: 1 if the solve is finished, else plan the
// next batch from the observed convergence rate and return 0.
int solve_after_header(nn4mg_hier *H)
{
    StateHeader hd;
    std::memcpy(&hd, H->st_host, sizeof(StateHeader));
    if (hd.done || H->solve_enqueued >= H->solve_max) return 1;
    const int remaining = H->solve_max - H->solve_enqueued;
    int need = 4;
    if (H->solve_prev_last > 0.0 && hd.last > 0.0 && hd.last < H->solve_prev_last) {
        const double rate = std::pow(hd.last / H->solve_prev_last, 1.0 / (H->solve_planned > 0 ? H->solve_planned : 1));
        if (rate > 0.0 && rate < 1.0) need = (int)std::ceil(std::log(H->solve_rtol / hd.last) / std::log(rate));
    }
    if (need < 1) need = 1;
    if (need > 64) need = 64;
    H->solve_prev_last = hd.last;
    H->solve_planned = need < remaining ? need : remaining;
    return 0;
}

int solve_finish(nn4mg_hier *H, double *x, nn4mg_info *info) { return finish_solve(H, x, info, H->solve_t0); }

size_t solve_header_bytes() { return sizeof(StateHeader); }

int solve_fixed_enqueue(nn4mg_hier *H, const double *b, double *x, int cycles, void *host_hdr)
{
    if (!H || !b || !x || !host_hdr || cycles < 1) return fail(NN4MG_EINVAL, "bad fixed-count solve arguments");
    if (H->singular || H->cfg.outer == NN4MG_OUTER_FCG || H->group || H->view_of || H->L < 1)
        return fail(NN4MG_EINVAL, "fixed-count solve without host round trip: stationary, non-singular hierarchies only");
    int rc;
    if ((rc = solve_begin(H, b, x, 0.0, cycles, 1))) return rc;
    if ((rc = solve_enqueue_next(H, b, x))) return rc;  // all `cycles`, as planned for a fixed count
    HIP_TRY(launch_finish_fixed(x, H->lv[0].t, H->lv[0].n, H->st, direct_fine(H) ? 1 : 0, H->stream));
    HIP_TRY(hipMemcpyAsync(host_hdr, H->st, sizeof(StateHeader), hipMemcpyDeviceToHost, H->stream));
    return NN4MG_OK;
}

int solve_fixed_result(const void *host_hdr, double *relres)
{
    StateHeader hd;
    std::memcpy(&hd, host_hdr, sizeof(hd));
    if (relres) *relres = hd.last;
    if (hd.status == -5)
        return fail(NN4MG_EBREAKDOWN, "breakdown: non-finite residual or residual grown past 1e3 times the first");
    return NN4MG_OK;  // status -4 is the end of the fixed count
}

int hier_set_stream(nn4mg_hier *H, hipStream_t s)
{
    if (H->stream) HIP_TRY(hipStreamSynchronize(H->stream));
    H->stream = s;
    return NN4MG_OK;
}

void hier_use_stream(nn4mg_hier *H, hipStream_t s) { H->stream = s; }

int solve_header_copy(nn4mg_hier *H)
{
    HIP_TRY(hipMemcpyAsync(H->st_host, H->st, sizeof(StateHeader), hipMemcpyDeviceToHost, H->stream));
    return NN4MG_OK;
}

// ---- batched hierarchies ----

int view_create(nn4mg_hier *G, int c, nn4mg_hier **out)
{
    *out = nullptr;
    if (!G || !G->group || c < 0 || c >= G->cap) return fail(NN4MG_EINVAL, "view: not a batched hierarchy copy");
    nn4mg_hier *V = new nn4mg_hier(*G);
    V->view_of = G;
    V->group = false;
    V->ncopy = 1;
    V->arena = nullptr;
    V->allocs.clear();
    V->fields.clear();
    V->graph[0] = V->graph[1] = nullptr;
    V->bgraph.clear();
    V->cap = 1;
    V->graph_b = nullptr;
    V->graph_x = nullptr;
    V->prof_on = false;
    V->prof_ev.clear();
    V->prof_cls.clear();
    V->prof_tag.clear();
    V->prof_valid.clear();
    V->prof_lvl.clear();
    V->bytes = 0;
    V->st_host = G->st_host + c;
    const long long off = (long long)c * G->bstride;
    for (const nn4mg_hier::Field &f : G->fields) {
        const size_t at = (size_t)((const char *)f.ptr - (const char *)G);
        if (at + sizeof(void *) > sizeof(nn4mg_hier)) {
            delete V;
            return fail(NN4MG_EINVAL, "view: field outside the hierarchy");
        }
        void **pv = reinterpret_cast<void **>(reinterpret_cast<char *>(V) + at);
        *pv = copy_ptr(*pv, off);
    }
    *out = V;
    return NN4MG_OK;
}

void view_destroy(nn4mg_hier *V)
{
    if (!V || !V->view_of) return;
    V->st_host = nullptr;
    delete V;
}

double *hier_bw(nn4mg_hier *H) { return H->bw; }
double *hier_xw(nn4mg_hier *H) { return H->xw; }

int hier_load_coef(nn4mg_hier *H, const double *k_dev)
{
    if (H->cfg.coef_mode == NN4MG_COEF_NODAL) {
        if (!k_dev) return fail(NN4MG_EINVAL, "nodal coefficient requires k");
        return load_k(H, k_dev);
    }
    return rebuild_coefficients(H);
}

// The batched cycle over copies 0 .. k - 1, captured once per k.
hipGraphExec_t batch_graph(nn4mg_hier *G, int k)
{
    if (G->bgraph[k]) return G->bgraph[k];
    if (!G->graphs_ok || G->prof_on) return nullptr;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(G->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        G->graphs_ok = false;
        return nullptr;
    }
    const int rc = enqueue_iteration(G, G->bw, G->xw, 0);
    const hipError_t e = hipStreamEndCapture(G->stream, &g);
    hipGraphExec_t ex = nullptr;
    if (rc == NN4MG_OK && e == hipSuccess && g && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
        G->bgraph[k] = ex;
    } else {
        (void)hipGetLastError();
        G->graphs_ok = false;
        ex = nullptr;
    }
    if (g) (void)hipGraphDestroy(g);
    return ex;
}

int batch_enqueue_cycles(nn4mg_hier *G, int n, int k)
{
    if (!G->group || k < 1 || k > G->cap) return fail(NN4MG_EINVAL, "batch: copy count outside the group");
    if (n <= 0) return NN4MG_OK;
    // launches below cover copies 0 .. k - 1 (the later ones have no solve)
    G->ncopy = k;
    int rc = NN4MG_OK;
    if (hipGraphExec_t ex = batch_graph(G, k)) {
        for (int c = 0; c < n && !rc; ++c)
            if (hipGraphLaunch(ex, G->stream) != hipSuccess) rc = fail(NN4MG_EDEVICE, "hipGraphLaunch failed");
    } else {
        for (int c = 0; c < n && !rc; ++c) rc = enqueue_iteration(G, G->bw, G->xw, 0);
    }
    // the last residual of the batch is judged before the host reads the states
    if (!rc && stop_in_chain(G) &&
        launch_finish_norm(G->st, G->partials, resid_blocks(G), G->stream, 1, G->ncopy, G->bstride) != hipSuccess)
        rc = fail(NN4MG_EDEVICE, "batch: stopping-rule launch failed");
    G->ncopy = G->cap;
    return rc;
}

// A copy with no solve: its stopping flag set, so the batched launches skip it.
int hier_mark_idle(nn4mg_hier *H)
{
    static const int one = 1;
    HIP_TRY(launch_init_state(H->st, 0.0, 0, 1, H->stream));
    HIP_TRY(hipMemcpyAsync(&H->st->done, &one, sizeof(int), hipMemcpyHostToDevice, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    return NN4MG_OK;
}

int hier_coarse_cells(const nn4mg_hier *H) { return H->nc; }

int coef_begin(nn4mg_hier *H, const double *k_dev, double *hk, int *bad)
{
    hipStream_t s = H->stream;
    const Level &F = H->lv[0];
    const Level &C = H->lv[H->L - 1];
    HIP_TRY(hipMemcpyAsync(F.k, k_dev, F.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(H->flag, 0, sizeof(int), s));
    HIP_TRY(launch_check_positive(F.k, F.n, H->flag, s));
    HIP_TRY(hipMemcpyAsync(bad, H->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    const int rc = enqueue_coef_kernels(H);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(hk, C.k, C.n * sizeof(double), hipMemcpyDeviceToHost, s));
    return NN4MG_OK;
}

int coef_end(nn4mg_hier *H, const double *hk, const int *bad, double *inv)
{
    if (*bad) return fail(NN4MG_EINVAL, "coefficient k must be positive and finite");
    const Level &C = H->lv[H->L - 1];
    std::vector<double> v;
    const int rc = coarse_inverse(C.nx, C.ny, C.nz, C.h, H->cfg.bc, hk, H->singular, v);
    if (rc) return rc;
    std::memcpy(inv, v.data(), v.size() * sizeof(double));
    HIP_TRY(hipMemcpyAsync(H->ainv, inv, v.size() * sizeof(double), hipMemcpyHostToDevice, H->stream));
    return NN4MG_OK;
}

int solve_finish_enqueue(nn4mg_hier *H, double *x)
{
    StateHeader hd;
    std::memcpy(&hd, H->st_host, sizeof(StateHeader));
    return finish_enqueue(H, x, hd);
}

int solve_finish_complete(nn4mg_hier *H, nn4mg_info *info) { return finish_complete(H, info, H->solve_t0); }

int hier_planned(const nn4mg_hier *H) { return H->solve_planned; }
int hier_started(const nn4mg_hier *H) { return H->solve_enqueued > 0; }

void hier_note_enqueued(nn4mg_hier *H, int n)
{
    H->solve_enqueued += n;
    H->solve_planned = n;
}

}  // namespace nn4mg

namespace {

int solve_stationary(nn4mg_hier *H, const double *b, double *x, double rtol, int max_cycles, int fixed,
                     nn4mg_info *info)
{
    int rc;
    if ((rc = nn4mg::solve_begin(H, b, x, rtol, max_cycles, fixed))) return rc;
    StateHeader hd;
    while (true) {
        if ((rc = nn4mg::solve_enqueue_next(H, b, x))) return rc;
        if ((rc = read_header(H, &hd))) return rc;
        if (nn4mg::solve_after_header(H)) break;
    }
    // the header just read is the final one (nothing was enqueued since): finish without reading it again
    if ((rc = finish_enqueue(H, x, hd))) return rc;
    HIP_TRY(hipStreamSynchronize(H->stream));
    return finish_complete(H, info, H->solve_t0);
}

}  // namespace

extern "C" {

int nn4mg_profile(nn4mg_t H, int enable)
{
    if (!H) return fail(NN4MG_EINVAL, "handle is NULL");
    HIP_TRY(hipStreamSynchronize(H->stream));
    if (enable) {
        H->prof_cls.clear();
        H->prof_lvl.clear();
        H->prof_tag.clear();
        H->prof_valid.clear();
        H->prof_solve_begin = 0;
    }
    H->prof_on = enable != 0;
    return NN4MG_OK;
}

int nn4mg_profile_read_level(nn4mg_t H, int level, int kclass, int *launches, double *total_ms)
{
    if (!H) return fail(NN4MG_EINVAL, "handle is NULL");
    if (kclass < 0 || kclass >= NN4MG_KCLASS_COUNT) return fail(NN4MG_EINVAL, "unknown kernel class");
    if (level < 0 || level >= H->L) return fail(NN4MG_EINVAL, "bad level");
    HIP_TRY(hipStreamSynchronize(H->stream));
    int n = 0;
    double tot = 0.0;
    for (size_t i = 0; i < H->prof_cls.size(); ++i) {
        if (H->prof_cls[i] != kclass || H->prof_lvl[i] != level || !H->prof_valid[i]) continue;
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, H->prof_ev[2 * i], H->prof_ev[2 * i + 1]));
        tot += ms;
        ++n;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = tot;
    return NN4MG_OK;
}

int nn4mg_profile_read(nn4mg_t H, int kclass, int *launches, double *total_ms)
{
    return nn4mg_profile_read_level(H, 0, kclass, launches, total_ms);
}

int nn4mg_set_tiles(nn4mg_t H, int level, int kclass, int tx, int ry, int zc)
{
    if (!H) return fail(NN4MG_EINVAL, "handle is NULL");
    if (level < 0 || level >= H->L) return fail(NN4MG_EINVAL, "bad level");
    if (kclass < -1 || kclass >= NN4MG_KCLASS_COUNT) return fail(NN4MG_EINVAL, "bad kernel class");
    if (tx == 8) {
        // both post-sweeps as 8^3 blocks: a shape of the first-sweep class of a fused level only
        if (kclass != NN4MG_KCLASS_FINE_SWEEP_PROLONG || ry != 8 || zc != 8)
            return fail(NN4MG_EINVAL, "the 8^3 block shape is (8, 8, 8) for the first-sweep class only");
        if (!level_fusable(H, level))
            return fail(NN4MG_EINVAL, "the 8^3 block shape needs nu_post == 2 and a level of at least 4^3");
        HIP_TRY(hipStreamSynchronize(H->stream));
        H->lv[level].block2 = true;
        H->tiles_epoch++;
        return NN4MG_OK;
    }
    if ((tx != 64 && tx != 32 && tx != 16) || (ry != 1 && ry != 2 && ry != 4) || (tx == 16 && ry == 4) || zc < 2 ||
        (zc & 1))
        return fail(NN4MG_EINVAL, "bad tile shape");
    if (ry == 1 && kclass == NN4MG_KCLASS_FINE_RESID)
        return fail(NN4MG_EINVAL, "the residual kernel needs an even number of rows per thread");
    Level &V = H->lv[level];
    const TileShape t = make_tiles(V.nx, V.ny, V.nz, zc, tx, ry);
    if (t.blocks() > H->max_partials && (kclass < 0 || kclass == NN4MG_KCLASS_FINE_RESID))
        return fail(NN4MG_EINVAL, "tile shape needs too many workgroups");
    HIP_TRY(hipStreamSynchronize(H->stream));
    for (int c = 0; c < NN4MG_KCLASS_COUNT; ++c) {
        if (ry == 1 && c == NN4MG_KCLASS_FINE_RESID) continue;  // kclass -1: sweeps only
        if (kclass < 0 || kclass == c) V.tiles[c] = t;
    }
    if (kclass < 0 || kclass == NN4MG_KCLASS_FINE_SWEEP_PROLONG) V.block2 = false;
    H->tiles_epoch++;
    return NN4MG_OK;
}

int nn4mg_get_tiles(nn4mg_t H, int level, int kclass, int *tx, int *ry, int *zc)
{
    if (!H) return fail(NN4MG_EINVAL, "handle is NULL");
    if (level < 0 || level >= H->L) return fail(NN4MG_EINVAL, "bad level");
    if (kclass < 0 || kclass >= NN4MG_KCLASS_COUNT) return fail(NN4MG_EINVAL, "bad kernel class");
    const TileShape &t = H->lv[level].tiles[kclass];
    const bool blk = kclass == NN4MG_KCLASS_FINE_SWEEP_PROLONG && H->lv[level].block2;
    if (tx) *tx = blk ? 8 : t.tx;
    if (ry) *ry = blk ? 8 : t.ry;
    if (zc) *zc = blk ? 8 : t.zc;
    return NN4MG_OK;
}

int nn4mg_autotune(nn4mg_t H, const double *b, double *x, int *tiles_out, int max_levels)
{
    if (!H || !b || !x) return fail(NN4MG_EINVAL, "NULL argument");
    const int L = H->L;
    constexpr int NT_SHAPES = 8;
    const int txs[NT_SHAPES] = {64, 64, 32, 32, 16, 64, 32, 16};
    const int rys[NT_SHAPES] = {2, 4, 2, 4, 2, 1, 1, 1};
    constexpr int NZC = 6;
    const int zcs[NZC] = {2, 4, 8, 16, 32, 64};
    const int reps = 3;
    constexpr int NC = NN4MG_KCLASS_COUNT;
    std::vector<double> best((size_t)L * NC, 1e300);
    std::vector<TileShape> best_t((size_t)L * NC);
    for (int l = 0; l < L; ++l)
        for (int c = 0; c < NC; ++c) best_t[(size_t)l * NC + c] = H->lv[l].tiles[c];
    for (int l = 0; l < L; ++l) H->lv[l].block2 = false;  // the marching shapes are timed first
    const bool saved_on = H->prof_on;
    auto clear = [&]() {
        H->prof_cls.clear();
        H->prof_lvl.clear();
        H->prof_tag.clear();
        H->prof_valid.clear();
        H->prof_solve_begin = 0;
    };
    int rc;
    for (int ti = 0; ti < NT_SHAPES; ++ti)
        for (int zi = 0; zi < NZC; ++zi) {
            std::vector<bool> used(L, false);
            for (int l = 0; l < L; ++l) {
                Level &V = H->lv[l];
                if (zcs[zi] > V.nz + (V.nz & 1)) continue;
                const TileShape t = make_tiles(V.nx, V.ny, V.nz, zcs[zi], txs[ti], rys[ti]);
                // one row per thread: sweep classes only; the residual keeps its best shape so far
                if (rys[ti] == 1) {
                    V.tiles[NN4MG_KCLASS_FINE_RESID] = best_t[(size_t)l * NC + NN4MG_KCLASS_FINE_RESID];
                    for (int c = 0; c < NC; ++c)
                        if (c != NN4MG_KCLASS_FINE_RESID) V.tiles[c] = t;
                } else {
                    if (t.blocks() > H->max_partials) continue;
                    for (int c = 0; c < NC; ++c) V.tiles[c] = t;
                }
                used[l] = true;
            }
            HIP_TRY(hipStreamSynchronize(H->stream));
            H->prof_on = true;
            clear();
            H->cur_tag = 0;
            for (int r = 0; r < reps + 1; ++r) {
                if (r == 1) {  // the first cycle warms caches and code; drop it
                    HIP_TRY(hipStreamSynchronize(H->stream));
                    clear();
                }
                if ((rc = enqueue_cycle_inplace(H, b, x, r & 1))) return rc;
            }
            H->prof_on = false;
            for (int l = 0; l < L; ++l) {
                if (!used[l]) continue;
                for (int c = 0; c < NC; ++c) {
                    double ms = 0.0;
                    int n = 0;
                    if ((rc = nn4mg_profile_read_level(H, l, c, &n, &ms))) return rc;
                    if (n > 0 && ms < best[(size_t)l * NC + c]) {
                        best[(size_t)l * NC + c] = ms;
                        best_t[(size_t)l * NC + c] = H->lv[l].tiles[c];
                    }
                }
            }
        }
    for (int l = 0; l < L; ++l)
        for (int c = 0; c < NC; ++c) H->lv[l].tiles[c] = best_t[(size_t)l * NC + c];
    // the 8^3 block kernel against the best marching shape, per fused level
    {
        constexpr int C1 = NN4MG_KCLASS_FINE_SWEEP_PROLONG;
        std::vector<bool> cand(L, false);
        bool any = false;
        for (int l = 0; l < L; ++l) {
            H->lv[l].block2 = false;
            if (level_fusable(H, l)) cand[l] = any = true;
        }
        if (any) {
            for (int l = 0; l < L; ++l) H->lv[l].block2 = cand[l];
            HIP_TRY(hipStreamSynchronize(H->stream));
            H->prof_on = true;
            clear();
            H->cur_tag = 0;
            for (int r = 0; r < reps + 1; ++r) {
                if (r == 1) {
                    HIP_TRY(hipStreamSynchronize(H->stream));
                    clear();
                }
                if ((rc = enqueue_cycle_inplace(H, b, x, r & 1))) return rc;
            }
            H->prof_on = false;
            for (int l = 0; l < L; ++l) {
                if (!cand[l]) continue;
                double ms = 0.0;
                int n = 0;
                if ((rc = nn4mg_profile_read_level(H, l, C1, &n, &ms))) return rc;
                H->lv[l].block2 = n > 0 && ms < best[(size_t)l * NC + C1];
            }
        }
    }
    H->tiles_epoch++;
    H->prof_on = saved_on;
    clear();
    if (tiles_out)
        for (int l = 0; l < L && l < max_levels; ++l)
            for (int c = 0; c < NC; ++c) {
                const TileShape &t = best_t[(size_t)l * NC + c];
                const bool blk = c == NN4MG_KCLASS_FINE_SWEEP_PROLONG && H->lv[l].block2;
                tiles_out[9 * l + 3 * c] = blk ? 8 : t.tx;
                tiles_out[9 * l + 3 * c + 1] = blk ? 8 : t.ry;
                tiles_out[9 * l + 3 * c + 2] = blk ? 8 : t.zc;
            }
    return NN4MG_OK;
}

int nn4mg_vcycle(nn4mg_t H, const double *b, double *x)
{
    if (!H || !b || !x) return fail(NN4MG_EINVAL, "NULL argument");
    return enqueue_cycle_inplace(H, b, x);
}

int nn4mg_solve(nn4mg_t H, const double *b, double *x, double rtol, int max_cycles, int fixed_cycles,
                nn4mg_info *info)
{
    if (!H || !b || !x) return fail(NN4MG_EINVAL, "NULL argument");
    if (max_cycles < 0) return fail(NN4MG_EINVAL, "max_cycles must be >= 0");
    if (!(rtol >= 0.0)) return fail(NN4MG_EINVAL, "rtol must be >= 0");
    return solve_stationary(H, b, x, rtol, max_cycles, fixed_cycles ? 1 : 0, info);
}

}  // extern "C"

int nn4mg::set_error(int code, const char *msg) { return fail(code, msg ? msg : ""); }
