// Internal declarations of the nn4mg HIP library (not part of the C-ABI).
#pragma once

#include "../../include/nn4mg.h"

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stddef.h>
#include <stdint.h>

namespace nn4mg {

enum Bc { BC_D = 0, BC_N = 1, BC_P = 2 };

// Coefficient storage of a stencil launch.
enum KType { KT_NONE = 0, KT_F64 = 1, KT_F32 = 2, KT_F16 = 3 };

// How a stencil kernel forms the field it smooths, per loaded cell.
enum InMode {
    IN_PLAIN = 0,       // y = yin
    IN_PROLONG = 1,     // y = P ec
    IN_PROLONG_ADD = 2  // y = yin + P ec
};

// What a stencil kernel writes.
enum OutMode {
    OUT_STORE = 0,  // yout = y + omega (b - A y) / D
    OUT_ADD64 = 1,  // x64 += y + omega (b - A y) / D
    OUT_RESID = 2   // r = (b - bmean) - A y, optional restriction R r, per-block sum of r^2
};

// Launch shape of the z-marching stencil kernels: a workgroup of 256 threads
// (tx along x, 256/tx along y, ry rows per thread) owns a tx x (ry*256/tx)
// column of cells and marches `zc` planes along z.
struct TileShape {
    int tx;  // cells per tile along x: 64, 32 or 16
    int ry;  // cell rows per thread: 2 or 4 (tile is tx x ry*256/tx)
    int tiles_x, tiles_y, chunks_z, zc;
    int blocks() const { return tiles_x * tiles_y * chunks_z; }
};

TileShape make_tiles(int nx, int ny, int nz, int zc, int tx, int ry = 2);

struct Geom {
    int nx, ny, nz;
    int bc[6];
};

// Argument block of one stencil launch.  Pointers are device pointers; the
// element types follow the template instance chosen by the launcher.
struct StencilArgs {
    Geom g;
    TileShape t;
    double h, omega;
    const void *yin;     // IN_PLAIN input / IN_PROLONG_ADD addend (type T)
    const void *ec;      // coarse correction (type T), dims cnx x cny x cnz
    int cnx, cny, cnz;
    const void *b;       // right-hand side (type T); NULL for zero (residual mode)
    const void *k;       // coefficient (KType), NULL for constant
    void *yout;          // OUT_STORE destination (type T)
    double *x64;         // OUT_ADD64 destination
    const double *bmean; // subtracted from b if not NULL (projected right-hand side)
    void *r;             // OUT_RESID: full residual (type OT), may be NULL
    void *rc;            // OUT_RESID: restricted residual (type OT), may be NULL
    double *partials;    // OUT_RESID: one sum of r^2 per block (x.r with dot_x), may be NULL
    int dot_x;           // OUT_RESID: partials of x.r instead of r.r
    const int *done;     // skip the launch when *done != 0 (may be NULL)
    // batched launch: the same level of ncopy identical hierarchies whose
    // fields lie bstride bytes apart (ncopy 0 or 1: one hierarchy)
    int ncopy;
    int bnb;             // blocks per copy (set by the launcher)
    long long bstride;
};

// Move a field pointer to the copy `off` bytes further on (NULL stays NULL).
// Byte-pointer arithmetic, not integer casts: the compiler then still knows
// that the result points to global memory and keeps global (not flat) loads.
template <typename P>
__host__ __device__ __forceinline__ P *copy_ptr(P *p, long long off)
{
    using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    return p ? (P *)((B *)p + off) : p;
}

// Block lb (after the XCD remap) of a batched launch works on copy lb / bnb:
// move every field pointer of a to that copy and return the block's index
// within the copy.
__device__ __forceinline__ int enter_copy(StencilArgs &a, int lb)
{
    if (a.ncopy <= 1) return lb;
    const int c = lb / a.bnb;
    const long long off = (long long)c * a.bstride;
    a.yin = copy_ptr(a.yin, off);
    a.ec = copy_ptr(a.ec, off);
    a.b = copy_ptr(a.b, off);
    a.k = copy_ptr(a.k, off);
    a.yout = copy_ptr(a.yout, off);
    a.x64 = copy_ptr(a.x64, off);
    a.bmean = copy_ptr(a.bmean, off);
    a.r = copy_ptr(a.r, off);
    a.rc = copy_ptr(a.rc, off);
    a.partials = copy_ptr(a.partials, off);
    a.done = copy_ptr(a.done, off);
    return lb - c * a.bnb;
}

// The launch grid of a with nb blocks per copy; sets a.bnb.
inline unsigned batched_grid(StencilArgs &a, int nb)
{
    a.bnb = nb;
    return (unsigned)nb * (unsigned)(a.ncopy > 1 ? a.ncopy : 1);
}

// Device-resident state of a solve; the host polls a copy of it.
struct SolveState {
    double nb;       // ||b - bmean||
    double bmean;    // mean of b (singular problems), else 0
    double rtol;
    int max_cycles;
    int fixed;
    int nres;        // residual norms recorded
    int done;        // 1 once the stopping rule fired
    int status;      // 0, -4 (max cycles), -5 (non-finite)
    int taken;       // 1: a stand-alone stopping-rule launch already took the latest residual
    double last;     // last relative residual
    double hist[512];
    // flexible CG scalars
    double fcg_rho, fcg_alpha, fcg_beta, fcg_pq_prev;
};

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error.

// Stencil kernel: T in {double, float}; kt selects the coefficient type
// (KT_F64 requires T = double or float; KT_F32/KT_F16 require T = float);
// for OUT_RESID, T must be double and out_f32 selects float outputs r/rc.
hipError_t launch_stencil(int T_is_f64, int kt, int in_mode, int out_mode, int out_f32, const StencilArgs &a,
                          hipStream_t s);

// depth (1..3) successive restrictions from the level of dims nx x ny x nz into c1, c2, c3 (one launch).
// With st, one extra workgroup applies the stopping rule to the np residual
// partials (skipped when a stand-alone launch marked them taken).
hipError_t launch_restrict_chain(int T_is_f64, const void *fine, void *c1, void *c2, void *c3, int nx, int ny, int nz,
                                 int depth, const int *done, hipStream_t s, SolveState *st = nullptr,
                                 const double *partials = nullptr, int np = 0, int ncopy = 1,
                                 long long bstride = 0);
hipError_t launch_restrict(int T_is_f64, const void *fine, void *coarse, int nx, int ny, int nz, const int *done,
                           hipStream_t s);
hipError_t launch_coarsen_k(const double *kf, double *kc, int nx, int ny, int nz, int harmonic, hipStream_t s);
hipError_t launch_cast_k(const double *k, void *out, size_t n, int kt, hipStream_t s);
hipError_t launch_check_positive(const double *k, size_t n, int *bad, hipStream_t s);

// Sums (fixed order, deterministic): partials[blk] = sum over the block's
// slice of (v - shift)^p (p = 1 or 2; shift may be NULL).
int sum_blocks(size_t n);
hipError_t launch_sum_partials(const double *v, size_t n, const double *shift, int power, double *partials,
                               hipStream_t s);
// out[0] = scale * sum(partials[0..n))  (single workgroup, fixed tree)
hipError_t launch_reduce(const double *partials, int n, double scale, double *out, hipStream_t s);
// Reset the solve state; set_nb: nb = sqrt(*sumsq), and done at once if nb == 0.
hipError_t launch_init_state(SolveState *st, double rtol, int max_cycles, int fixed, hipStream_t s);
hipError_t launch_set_nb(SolveState *st, const double *sumsq, hipStream_t s);
// Stopping rule after a residual: consumes partials of r^2.
// Stopping rule on the residual partials; mark_taken = 1 tells the stopping
// workgroup of the next restriction chain that this residual is done.
hipError_t launch_finish_norm(SolveState *st, const double *partials, int n, hipStream_t s, int mark_taken = 0,
                              int ncopy = 1, long long bstride = 0);

hipError_t launch_coarse_solve(int T_is_f64, const void *bc, void *ec, const double *ainv, int n, int singular,
                               const int *done, hipStream_t s);
hipError_t launch_sub_scalar(double *x, size_t n, const double *val, hipStream_t s);
hipError_t launch_fill(double *x, size_t n, double v, hipStream_t s);
hipError_t launch_copy(double *dst, const double *src, size_t n, const int *done, hipStream_t s);
// x += e (e FP64, or FP32 when e_f32)
hipError_t launch_add(double *x, const void *e, int e_f32, size_t n, const int *done, hipStream_t s);

// ---- asynchronous solve pieces over a hierarchy (mg_api.hip) ----
// begin: reset the device state, b-norm, first residual; enqueue_next: the next
// planned batch of cycles (graph launches when the stream allows capture);
// header_async: copy the state header to pinned host memory and record ev;
// after_header (once ev completed): 1 when finished, else plans the next batch;
// finish: projection / zero fill, full state read-back (synchronous).
int solve_begin(nn4mg_hier *H, const double *b, double *x, double rtol, int max_cycles, int fixed);
int solve_enqueue_next(nn4mg_hier *H, const double *b, double *x);
int solve_header_async(nn4mg_hier *H, hipEvent_t ev);
int solve_after_header(nn4mg_hier *H);
int solve_finish(nn4mg_hier *H, double *x, nn4mg_info *info);
int hier_set_stream(nn4mg_hier *H, hipStream_t s);
// the stream of later work on H, with no wait for work already enqueued
void hier_use_stream(nn4mg_hier *H, hipStream_t s);
// copy the state header to pinned host memory (no event)
int solve_header_copy(nn4mg_hier *H);

// ---- batched hierarchies (mg_api.hip) ----
// setup_hier: a hierarchy of a validated cfg (group false: one copy, as
// nn4mg_setup), or a batched group of ncopy identical copies (the stationary
// cycle with two post-sweeps and a one-workgroup coarse end, else
// NN4MG_EINVAL) that launches every cycle kernel once over all copies; copy c is
// driven through its view (the solve pieces above, single launches).  Each
// copy has its own right-hand side and iterate fields (hier_bw / hier_xw) and
// coefficient (hier_load_coef on its view).  batch_enqueue_cycles: n cycles of
// every copy whose stopping rule has not fired, then the batch-end rule
// (hier_mark_idle: set a copy's stopping flag, for copies with no solve).
// hier_note_enqueued: record on a view that n cycles were enqueued for it.
int setup_hier(const nn4mg_config *cfg, const double *k_dev, hipStream_t stream, int ncopy, nn4mg_hier **out,
               bool group = false);
int view_create(nn4mg_hier *G, int c, nn4mg_hier **out);
void view_destroy(nn4mg_hier *V);
double *hier_bw(nn4mg_hier *H);
double *hier_xw(nn4mg_hier *H);
int hier_load_coef(nn4mg_hier *H, const double *k_dev);
// Asynchronous halves of the nodal coefficient set-up and of a solve's end
// (no host wait; the caller waits for the enqueued work in between).
// coef_begin: copy of k, its positivity check (flag into *bad, pinned), the
// coarse levels' coefficients and the coarsest level's k into hk (pinned,
// hier_coarse_cells doubles); coef_end (after those arrived): the flag, the
// coarsest inverse formed on the host into inv (pinned, cells^2 doubles) and
// its upload.  solve_finish_enqueue (the header in host memory says the solve
// is over): the iterate's projection or zero fill and the copy of the whole
// state to host memory; solve_finish_complete (after it arrived): info and
// status, as solve_finish.
int hier_coarse_cells(const nn4mg_hier *H);
int coef_begin(nn4mg_hier *H, const double *k_dev, double *hk, int *bad);
int coef_end(nn4mg_hier *H, const double *hk, const int *bad, double *inv);
int solve_finish_enqueue(nn4mg_hier *H, double *x);
int solve_finish_complete(nn4mg_hier *H, nn4mg_info *info);
int hier_mark_idle(nn4mg_hier *H);
int batch_enqueue_cycles(nn4mg_hier *G, int n, int k);  // over copies 0 .. k - 1
int hier_planned(const nn4mg_hier *H);
int hier_started(const nn4mg_hier *H);  // cycles have been enqueued for it
void hier_note_enqueued(nn4mg_hier *H, int n);

// ---- flexible CG vector kernels (mg_fcg.hip); t = -A p, q = A p = -t ----
// dots: rho = z.r (mode 0), or rho = z.r and beta = -(z.q)/(p.q) (mode 2);
// alpha: alpha = rho / (p.q) (breakdown if p.q <= 0); update: x += alpha p,
// r -= alpha q, r32 = (float) r if r32 != NULL, per-block r^2 partials
// (fcg_update_blocks of them, for launch_finish_norm); direction: p = z + beta p.
int fcg_partials_needed();
int fcg_update_blocks(size_t n);
hipError_t launch_fcg_dots(const double *z, const double *r, const double *t, size_t n, double *partials,
                           SolveState *st, int mode, hipStream_t s);
hipError_t launch_fcg_alpha(const double *p, const double *t, size_t n, double *partials, SolveState *st,
                            hipStream_t s);
// alpha from nblk per-block partials of p.t (t = -A p) written by the residual kernel
hipError_t launch_fcg_alpha_partials(const double *partials, int nblk, SolveState *st, hipStream_t s);
hipError_t launch_fcg_update(SolveState *st, double *x, const double *p, double *r, const double *t, float *r32,
                             size_t n, double *partials, hipStream_t s);
hipError_t launch_fcg_direction(SolveState *st, const double *z, double *p, size_t n, hipStream_t s);
hipError_t launch_cast_f32(const double *src, float *dst, size_t n, const int *done, hipStream_t s);
hipError_t launch_zero(double *x, size_t n, const int *done, hipStream_t s);

// ---- both post-smoothing sweeps in one pass (mg_fused.hip) ----
// in_mode IN_PROLONG: input P e (a.ec), right-hand side a.b (no bmean),
// coefficient a.k; out_mode OUT_STORE (a.yout) or OUT_ADD64 (a.x64 += e).
// in_mode IN_PROLONG_ADD (FP64, OUT_STORE only): input a.yin + P e,
// right-hand side a.b - a.bmean, result in a.yout != a.yin.
bool sweep2_supports(int tx, int ry);
hipError_t launch_sweep2(int T_is_f64, int kt, int in_mode, int out_mode, const StencilArgs &a, hipStream_t s);

// ---- the same two sweeps as independent 8^3 blocks (mg_block.hip) ----
// Same arguments and result as launch_sweep2 (a.t is not used); one
// workgroup per 8^3 block of the level, for levels whose marching chain of
// planes, not their bytes, sets the time.
int block2_blocks(int nx, int ny, int nz);
hipError_t launch_sweep2_block(int T_is_f64, int kt, int out_mode, const StencilArgs &a, hipStream_t s);

// ---- coarse end of the cycle in one workgroup (mg_tail.hip) ----
constexpr int kTailMaxLevels = 8;
struct TailArgs {
    int levels;                         // tail levels, finest first; the last is the coarsest
    int nx[kTailMaxLevels], ny[kTailMaxLevels], nz[kTailMaxLevels];
    double h[kTailMaxLevels];
    const void *kpad;                   // coefficient of every tail level on its padded cells (type T), finest
                                        // first, built by launch_tail_kpad; NULL if constant
    const void *b_above;                // right-hand side of the level above the first tail level, or NULL
    const void *b_first;                // right-hand side of the first tail level (when b_above is NULL)
    void *e_first;                      // out: correction of the first tail level
    const double *ainv;                 // coarsest inverse (FP64, symmetric)
    int ainv_in_lds;                    // stage the inverse in LDS (it fits)
    int singular;
    int bc[6];
    double omega;
    int nu;
    const int *done;                    // skip when *done != 0 (may be NULL)
    int ncopy;                          // batched: one workgroup per copy, fields bstride bytes apart
    long long bstride;
};
// LDS elements of the tail levels' fields: right-hand side, two iterates and
// (nodal) the coefficient per level, the last three with a one-cell halo.
size_t tail_field_cells(const int *nx, const int *ny, const int *nz, int levels, int nodal);
size_t tail_lds_bytes(const TailArgs &a, int t_is_f64, int nodal);
// Padded copy (one-cell halo by the +mirror rule) of a level's coefficient k
// (storage type kt) as type T (double if T_is_f64, else float), for the tail.
hipError_t launch_tail_kpad(int T_is_f64, int kt, const void *k, int nx, int ny, int nz, const int *bc, void *out,
                            hipStream_t s);
hipError_t launch_tail(int T_is_f64, int kt, const TailArgs &a, hipStream_t s);

// Record the message returned by nn4mg_last_error() on this thread; returns code.
int set_error(int code, const char *msg);

}  // namespace nn4mg
