// Grid-transfer, coefficient, reduction and coarsest-level kernels of the
// multigrid solve (gfx950).  The stencil kernel lives in mg_stencil.hip.
#include "mg_async.h"
#include "mg_internal.h"

#include <type_traits>

namespace nn4mg {

namespace {

// ------------------------------------------------------------------ transfers

template <typename T>
__global__ __launch_bounds__(256) void restrict_kernel(const T *f, T *c, int nx, int ny, int nz, const int *done)
{
    if (done && *done) return;
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const size_t nc = (size_t)cx * cy * cz, sy = (size_t)nx, sz = (size_t)nx * ny;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < nc; id += (size_t)gridDim.x * blockDim.x) {
        const int I = (int)(id % cx);
        const size_t t = id / cx;
        const int J = (int)(t % cy), K = (int)(t / cy);
        const size_t g = 2 * (size_t)I + sy * 2 * (size_t)J + sz * 2 * (size_t)K;
        c[id] = ((f[g] + f[g + 1]) + (f[g + sy] + f[g + sy + 1])) +
                ((f[g + sz] + f[g + sz + 1]) + (f[g + sz + sy] + f[g + sz + sy + 1]));
    }
}

// The stopping rule on the latest residual norm (thread 0 of one workgroup):
// record the relative residual and set done / status.  A non-finite residual,
// or one that has grown past kDivergence times the first, is a breakdown: a
// convergent cycle never grows the residual by that much, so the iteration
// diverges (a smoother weight past its stability bound, a coarse operator the
// cycle cannot use) and further cycles only overflow.
constexpr double kDivergence = 1.0e3;

__device__ void stop_rule(SolveState *st, double sumsq)
{
    const double rel = sqrt(sumsq) / st->nb;
    const int idx = st->nres;
    if (idx < 512) st->hist[idx] = rel;
    st->last = rel;
    st->nres = idx + 1;
    if (!isfinite(rel) || (idx > 0 && rel > kDivergence * st->hist[0])) {
        st->done = 1;
        st->status = -5;
    } else if (!st->fixed && rel <= st->rtol) {
        st->done = 1;
        st->status = 0;
    } else if (idx >= st->max_cycles) {
        st->done = 1;
        st->status = st->fixed ? 0 : -4;
    }
}

// Sum of n partials by a 512-thread workgroup, fixed order; thread 0 holds it.
__device__ double reduce_512(const double *p, int n, double *red)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 512) acc += p[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < 8; ++w) s += red[w];
    return s;
}

// Up to three successive restrictions (sum of the 8 children) in one launch:
// each workgroup owns a 16^3 block of the input level and writes the 8^3, 4^3
// and 2^3 blocks of the next levels under it.  A coarse cell depends only on
// its own children, so no workgroup waits for another.  Sums in the order of
// restrict_kernel (x pairs, then y, then z), so the results are the same.
template <typename T>
__global__ __launch_bounds__(512) void restrict_chain_kernel(const T *f, T *c1, T *c2, T *c3, int nx, int ny, int nz,
                                                             int depth, const int *done, SolveState *st,
                                                             const double *partials, int np, int nbc,
                                                             long long bstride)
{
    // batched (nbc > 0): workgroup g works on copy g / nbc, whose fields lie
    // bstride bytes further on per copy
    int g = (int)blockIdx.x;
    if (nbc > 0) {
        const int c = g / nbc;
        g -= c * nbc;
        const long long off = (long long)c * bstride;
        f = copy_ptr(f, off);
        c1 = copy_ptr(c1, off);
        c2 = copy_ptr(c2, off);
        c3 = copy_ptr(c3, off);
        done = copy_ptr(done, off);
        st = copy_ptr(st, off);
        partials = copy_ptr(partials, off);
    }
    if (done && *done) return;
    if (st && g == 0) {
        // the extra first workgroup (dispatched first, so its reduction is off
        // the chain's critical path): stopping rule of the residual the
        // previous cycle ended with, unless a stand-alone launch already took it
        __shared__ double red[8];
        __shared__ int taken;
        // one thread reads and clears the flag; every thread branches on the
        // shared copy, so no wave can read it after the clear
        if (threadIdx.x == 0) {
            taken = st->taken;
            st->taken = 0;
        }
        __syncthreads();
        if (taken) return;  // uniform
        const double s = reduce_512(partials, np, red);
        if (threadIdx.x == 0) stop_rule(st, s);
        return;
    }
    __shared__ T s1[512];  // the 8^3 block of the first coarse level
    __shared__ T s2[64];   // the 4^3 block of the second
    const int bxn = (nx + 15) / 16, byn = (ny + 15) / 16;
    const int bid = st ? g - 1 : g;
    const int bx = bid % bxn, rest = bid / bxn;
    const int by = rest % byn, bz = rest / byn;
    const int t = threadIdx.x;
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    {
        const int I = bx * 8 + (t & 7), J = by * 8 + ((t >> 3) & 7), K = bz * 8 + (t >> 6);
        T v = (T)0;
        if (I < cx && J < cy && K < cz) {
            const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
            const size_t g = 2 * (size_t)I + sy * 2 * (size_t)J + sz * 2 * (size_t)K;
            v = ((f[g] + f[g + 1]) + (f[g + sy] + f[g + sy + 1])) +
                ((f[g + sz] + f[g + sz + 1]) + (f[g + sz + sy] + f[g + sz + sy + 1]));
            c1[(size_t)I + (size_t)cx * ((size_t)J + (size_t)cy * (size_t)K)] = v;
        }
        s1[t] = v;
    }
    if (depth < 2) return;  // uniform
    __syncthreads();
    const int dx = cx >> 1, dy = cy >> 1, dz = cz >> 1;
    if (t < 64) {
        const int mi = t & 3, mj = (t >> 2) & 3, mk = t >> 4;
        const int I = bx * 4 + mi, J = by * 4 + mj, K = bz * 4 + mk;
        T v = (T)0;
        if (I < dx && J < dy && K < dz) {
            const int o = 2 * mi + 16 * mj + 128 * mk;
            v = ((s1[o] + s1[o + 1]) + (s1[o + 8] + s1[o + 9])) + ((s1[o + 64] + s1[o + 65]) + (s1[o + 72] + s1[o + 73]));
            c2[(size_t)I + (size_t)dx * ((size_t)J + (size_t)dy * (size_t)K)] = v;
        }
        s2[t] = v;
    }
    if (depth < 3) return;
    __syncthreads();
    const int ex = dx >> 1, ey = dy >> 1, ez = dz >> 1;
    if (t < 8) {
        const int ni = t & 1, nj = (t >> 1) & 1, nk = t >> 2;
        const int I = bx * 2 + ni, J = by * 2 + nj, K = bz * 2 + nk;
        if (I < ex && J < ey && K < ez) {
            const int o = 2 * ni + 8 * nj + 32 * nk;
            c3[(size_t)I + (size_t)ex * ((size_t)J + (size_t)ey * (size_t)K)] =
                ((s2[o] + s2[o + 1]) + (s2[o + 4] + s2[o + 5])) + ((s2[o + 16] + s2[o + 17]) + (s2[o + 20] + s2[o + 21]));
        }
    }
}

__global__ __launch_bounds__(256) void coarsen_k_kernel(const double *f, double *c, int nx, int ny, int nz,
                                                        int harmonic)
{
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const size_t nc = (size_t)cx * cy * cz, sy = (size_t)nx, sz = (size_t)nx * ny;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < nc; id += (size_t)gridDim.x * blockDim.x) {
        const int I = (int)(id % cx);
        const size_t t = id / cx;
        const int J = (int)(t % cy), K = (int)(t / cy);
        const size_t g = 2 * (size_t)I + sy * 2 * (size_t)J + sz * 2 * (size_t)K;
        const size_t o[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
        double s = 0.0;
        for (int q = 0; q < 8; ++q) s += harmonic ? 1.0 / f[g + o[q]] : f[g + o[q]];
        c[id] = harmonic ? 8.0 / s : s * 0.125;
    }
}

__global__ __launch_bounds__(256) void cast_k_f32(const double *k, float *o, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        o[i] = (float)k[i];
}

__global__ __launch_bounds__(256) void cast_k_f16(const double *k, __half *o, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        o[i] = __float2half((float)k[i]);
}

__global__ __launch_bounds__(256) void check_positive_kernel(const double *k, size_t n, int *bad)
{
    bool b = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double v = k[i];
        if (!(v > 0.0) || !isfinite(v)) b = true;
    }
    if (b) *bad = 1;
}

// ----------------------------------------------------------------- reductions

constexpr int kSumBlocks = 1024;

__device__ __forceinline__ double block_sum_256(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
    return s;
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double *v, size_t n, const double *shift, int power,
                                                           double *partials)
{
    __shared__ double red[4];
    const double sh = shift ? *shift : 0.0;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double d = v[i] - sh;
        acc += (power == 2) ? d * d : d;
    }
    const double s = block_sum_256(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__device__ double reduce_1024(const double *p, int n, double *red)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += p[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < 16; ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(1024) void reduce_kernel(const double *p, int n, double scale, double *out)
{
    __shared__ double red[16];
    const double s = reduce_1024(p, n, red);
    if (threadIdx.x == 0) out[0] = scale * s;
}

__global__ __launch_bounds__(1024) void finish_norm_kernel(SolveState *st, const double *p, int n, int mark,
                                                          long long bstride)
{
    __shared__ double red[16];
    // batched: workgroup c judges copy c
    st = copy_ptr(st, (long long)blockIdx.x * bstride);
    p = copy_ptr(p, (long long)blockIdx.x * bstride);
    if (st->done) return;
    const double s = reduce_1024(p, n, red);
    if (threadIdx.x == 0) {
        stop_rule(st, s);
        if (mark) st->taken = 1;
    }
}

__global__ void init_state_kernel(SolveState *st, double rtol, int max_cycles, int fixed)
{
    st->nb = 0.0;
    st->bmean = 0.0;
    st->rtol = rtol;
    st->max_cycles = max_cycles;
    st->fixed = fixed;
    st->nres = 0;
    st->done = 0;
    st->status = 0;
    st->taken = 0;
    st->last = 0.0;
    st->fcg_rho = st->fcg_alpha = st->fcg_beta = st->fcg_pq_prev = 0.0;
}

__global__ void set_nb_kernel(SolveState *st, const double *sumsq)
{
    const double nb = sqrt(*sumsq);
    st->nb = nb;
    if (!isfinite(nb)) {
        // a non-finite right-hand side: breakdown before any cycle, x untouched
        st->done = 1;
        st->status = -5;
        st->hist[0] = nb;
        st->last = nb;
        st->nres = 1;
    } else if (!(nb > 0.0)) {
        st->done = 1;
        st->hist[0] = 0.0;
        st->last = 0.0;
        st->nres = 1;
    }
}

// -------------------------------------------------------------- coarsest level

// e = A_c^{-1} b with the symmetric FP64 inverse (column i read by thread i,
// coalesced); singular problems: subtract the mean of e.
template <typename T>
__global__ __launch_bounds__(512) void coarse_solve_kernel(const T *bc, T *ec, const double *ainv, int n,
                                                           int singular, const int *done)
{
    if (done && *done) return;
    __shared__ double sb[512];
    __shared__ double red[8];
    for (int j = threadIdx.x; j < n; j += 512) sb[j] = (double)bc[j];
    __syncthreads();
    double e = 0.0;
    const int i = threadIdx.x;
    if (i < n) {
        for (int j = 0; j < n; ++j) e += ainv[(size_t)j * n + i] * sb[j];
    }
    if (singular) {
        double v = (i < n) ? e : 0.0;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double s = 0.0;
        for (int w = 0; w < 8; ++w) s += red[w];
        e -= s / (double)n;
    }
    if (i < n) ec[i] = (T)e;
}

__global__ __launch_bounds__(256) void sub_scalar_kernel(double *x, size_t n, const double *val)
{
    const double v = *val;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] -= v;
}

__global__ __launch_bounds__(256) void fill_kernel(double *x, size_t n, double v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ __launch_bounds__(256) void copy_kernel(double *d, const double *s, size_t n, const int *done)
{
    if (done && *done) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

template <typename E>
__global__ __launch_bounds__(256) void add_kernel(double *x, const E *e, size_t n, const int *done)
{
    if (done && *done) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] += (double)e[i];
}

int stream_blocks(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

hipError_t launch_restrict(int T_is_f64, const void *fine, void *coarse, int nx, int ny, int nz, const int *done,
                           hipStream_t s)
{
    const size_t nc = (size_t)(nx / 2) * (ny / 2) * (nz / 2);
    if (T_is_f64)
        hipLaunchKernelGGL(restrict_kernel<double>, dim3(stream_blocks(nc)), dim3(256), 0, s, (const double *)fine,
                           (double *)coarse, nx, ny, nz, done);
    else
        hipLaunchKernelGGL(restrict_kernel<float>, dim3(stream_blocks(nc)), dim3(256), 0, s, (const float *)fine,
                           (float *)coarse, nx, ny, nz, done);
    return hipGetLastError();
}

hipError_t launch_restrict_chain(int T_is_f64, const void *fine, void *c1, void *c2, void *c3, int nx, int ny, int nz,
                                 int depth, const int *done, hipStream_t s, SolveState *st, const double *partials,
                                 int np, int ncopy, long long bstride)
{
    if (depth < 1 || depth > 3) return hipErrorInvalidValue;
    if (st && (!partials || np < 1)) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)(((nx + 15) / 16) * ((ny + 15) / 16) * ((nz + 15) / 16));
    const unsigned per = st ? nb + 1 : nb;
    const bool batched = ncopy > 1;
    const dim3 grid(batched ? per * (unsigned)ncopy : per);
    const int nbc = batched ? (int)per : 0;
    if (T_is_f64)
        hipLaunchKernelGGL(restrict_chain_kernel<double>, grid, dim3(512), 0, s, (const double *)fine, (double *)c1,
                           (double *)c2, (double *)c3, nx, ny, nz, depth, done, st, partials, np, nbc, bstride);
    else
        hipLaunchKernelGGL(restrict_chain_kernel<float>, grid, dim3(512), 0, s, (const float *)fine, (float *)c1,
                           (float *)c2, (float *)c3, nx, ny, nz, depth, done, st, partials, np, nbc, bstride);
    return hipGetLastError();
}

hipError_t launch_coarsen_k(const double *kf, double *kc, int nx, int ny, int nz, int harmonic, hipStream_t s)
{
    const size_t nc = (size_t)(nx / 2) * (ny / 2) * (nz / 2);
    hipLaunchKernelGGL(coarsen_k_kernel, dim3(stream_blocks(nc)), dim3(256), 0, s, kf, kc, nx, ny, nz, harmonic);
    return hipGetLastError();
}

hipError_t launch_cast_k(const double *k, void *out, size_t n, int kt, hipStream_t s)
{
    if (kt == KT_F32)
        hipLaunchKernelGGL(cast_k_f32, dim3(stream_blocks(n)), dim3(256), 0, s, k, (float *)out, n);
    else if (kt == KT_F16)
        hipLaunchKernelGGL(cast_k_f16, dim3(stream_blocks(n)), dim3(256), 0, s, k, (__half *)out, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_check_positive(const double *k, size_t n, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(check_positive_kernel, dim3(stream_blocks(n)), dim3(256), 0, s, k, n, bad);
    return hipGetLastError();
}

int sum_blocks(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > (size_t)kSumBlocks) b = kSumBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_sum_partials(const double *v, size_t n, const double *shift, int power, double *partials,
                               hipStream_t s)
{
    hipLaunchKernelGGL(sum_partials_kernel, dim3(sum_blocks(n)), dim3(256), 0, s, v, n, shift, power, partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int n, double scale, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, s, partials, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_init_state(SolveState *st, double rtol, int max_cycles, int fixed, hipStream_t s)
{
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, s, st, rtol, max_cycles, fixed);
    return hipGetLastError();
}

hipError_t launch_set_nb(SolveState *st, const double *sumsq, hipStream_t s)
{
    hipLaunchKernelGGL(set_nb_kernel, dim3(1), dim3(1), 0, s, st, sumsq);
    return hipGetLastError();
}

hipError_t launch_finish_norm(SolveState *st, const double *partials, int n, hipStream_t s, int mark_taken,
                              int ncopy, long long bstride)
{
    hipLaunchKernelGGL(finish_norm_kernel, dim3(ncopy > 1 ? ncopy : 1), dim3(1024), 0, s, st, partials, n, mark_taken,
                       ncopy > 1 ? bstride : 0LL);
    return hipGetLastError();
}

hipError_t launch_coarse_solve(int T_is_f64, const void *bc, void *ec, const double *ainv, int n, int singular,
                               const int *done, hipStream_t s)
{
    if (n > 512) return hipErrorInvalidValue;
    if (T_is_f64)
        hipLaunchKernelGGL(coarse_solve_kernel<double>, dim3(1), dim3(512), 0, s, (const double *)bc, (double *)ec,
                           ainv, n, singular, done);
    else
        hipLaunchKernelGGL(coarse_solve_kernel<float>, dim3(1), dim3(512), 0, s, (const float *)bc, (float *)ec,
                           ainv, n, singular, done);
    return hipGetLastError();
}

hipError_t launch_sub_scalar(double *x, size_t n, const double *val, hipStream_t s)
{
    hipLaunchKernelGGL(sub_scalar_kernel, dim3(stream_blocks(n)), dim3(256), 0, s, x, n, val);
    return hipGetLastError();
}

hipError_t launch_fill(double *x, size_t n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(stream_blocks(n)), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(double *dst, const double *src, size_t n, const int *done, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel, dim3(stream_blocks(n)), dim3(256), 0, s, dst, src, n, done);
    return hipGetLastError();
}

hipError_t launch_add(double *x, const void *e, int e_f32, size_t n, const int *done, hipStream_t s)
{
    if (e_f32)
        hipLaunchKernelGGL(add_kernel<float>, dim3(stream_blocks(n)), dim3(256), 0, s, x, (const float *)e, n, done);
    else
        hipLaunchKernelGGL(add_kernel<double>, dim3(stream_blocks(n)), dim3(256), 0, s, x, (const double *)e, n, done);
    return hipGetLastError();
}


namespace {

// The device side of a fixed-count solve's finish (see launch_finish_fixed).
__global__ __launch_bounds__(256) void finish_fixed_kernel(double *x, const double *t, size_t n, const SolveState *st,
                                                           int direct)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (st->nb == 0.0) {
        x[i] = 0.0;
        return;
    }
    const int nres = st->nres;
    if (direct && nres > 0 && ((nres - 1) & 1)) x[i] = t[i];
}

}  // namespace

hipError_t launch_finish_fixed(double *x, const double *t, size_t n, const SolveState *st, int direct, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(finish_fixed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, t, n, st, direct);
    return hipGetLastError();
}

}  // namespace nn4mg
