// Vector kernels of the flexible conjugate-gradient outer iteration (gfx950).
//
// The outer iteration keeps r, z = M r (one sawtooth cycle from zero), the
// search direction p and t = -A p (the residual kernel run on p against a zero
// right-hand side) in FP64 at the finest level, and runs FCG(1):
// alpha = (z.r)/(p.q), x += alpha p, r -= alpha q, then beta = -(z'.q)/(p.q),
// p = z' + beta p, with q = A p = -t.  All scalars
// live in the device solve state, so a batch of iterations runs with no host
// round trip; every kernel returns at once when the stopping rule has fired.
// Dot products are reduced in a fixed order (per-block partials, then one
// workgroup), so results are bitwise repeatable.
#include "mg_internal.h"

namespace nn4mg {

namespace {

constexpr int kDotBlocks = 1024;

int dot_blocks(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > kDotBlocks) b = kDotBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

// Sum over a 256-thread block, result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Sum of p[0..n) by one 1024-thread workgroup, result valid in thread 0.
__device__ double reduce_partials(const double *p, int n, double *red)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += p[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < 16; ++w) s += red[w];
    return s;
}

// partials[blk] = sum z r; partials[nblk + blk] = sum z q = -sum z t (0 if t is NULL).
__global__ __launch_bounds__(256) void dots_kernel(const double *z, const double *r, const double *t, size_t n,
                                                   double *partials, const int *done)
{
    if (*done) return;
    __shared__ double red[8];
    double a = 0.0, b = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double zi = z[i];
        a += zi * r[i];
        if (t) b -= zi * t[i];
    }
    const double sa = block_sum(a, red);
    const double sb = block_sum(b, red + 4);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = sa;
        partials[gridDim.x + blockIdx.x] = sb;
    }
}

// partials[blk] = -sum p t = p . A p
__global__ __launch_bounds__(256) void pq_kernel(const double *p, const double *t, size_t n, double *partials,
                                                 const int *done)
{
    if (*done) return;
    __shared__ double red[4];
    double a = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        a -= p[i] * t[i];
    }
    const double s = block_sum(a, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// mode 0: rho = sum z r (start);  mode 1: alpha = rho / (p.q) from partials of p.q;
// mode 3: the same from partials of p.t = -p.q;  mode 2: beta = -(z.q) / (p.q), rho = z.r.
__global__ __launch_bounds__(1024) void scalar_kernel(SolveState *st, const double *partials, int nblk, int mode)
{
    __shared__ double red[16];
    if (st->done) return;
    if (mode == 1 || mode == 3) {
        const double pq = (mode == 3 ? -1.0 : 1.0) * reduce_partials(partials, nblk, red);
        if (threadIdx.x == 0) {
            st->fcg_pq_prev = pq;
            if (!(pq > 0.0) || !isfinite(pq)) {
                // p . A p must be positive for an SPD (or semidefinite, on the range) operator
                st->fcg_alpha = 0.0;
                st->done = 1;
                st->status = -5;
            } else {
                st->fcg_alpha = st->fcg_rho / pq;
            }
        }
        return;
    }
    const double zr = reduce_partials(partials, nblk, red);
    __syncthreads();
    const double zq = (mode == 2) ? reduce_partials(partials + nblk, nblk, red) : 0.0;
    if (threadIdx.x == 0) {
        st->fcg_rho = zr;
        st->fcg_beta = (mode == 2) ? -zq / st->fcg_pq_prev : 0.0;
    }
}

// x += alpha p; r -= alpha q (= r + alpha t); r32 = (float) r (if given); partials of r^2.
__global__ __launch_bounds__(256) void update_kernel(const SolveState *st, double *x, const double *p, double *r,
                                                     const double *t, float *r32, size_t n, double *partials)
{
    if (st->done) return;
    __shared__ double red[4];
    const double alpha = st->fcg_alpha;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const double ri = r[i] + alpha * t[i];
        r[i] = ri;
        if (r32) r32[i] = (float)ri;
        acc += ri * ri;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = z + beta p
__global__ __launch_bounds__(256) void direction_kernel(const SolveState *st, const double *z, double *p, size_t n)
{
    if (st->done) return;
    const double beta = st->fcg_beta;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(256) void cast_f32_kernel(const double *src, float *dst, size_t n, const int *done)
{
    if (*done) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

__global__ __launch_bounds__(256) void zero_kernel(double *x, size_t n, const int *done)
{
    if (*done) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

int grid_blocks(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int fcg_partials_needed() { return 2 * kDotBlocks; }

hipError_t launch_fcg_dots(const double *z, const double *r, const double *t, size_t n, double *partials,
                           SolveState *st, int mode, hipStream_t s)
{
    const int nb = dot_blocks(n);
    hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(256), 0, s, z, r, t, n, partials, &st->done);
    hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(1024), 0, s, st, (const double *)partials, nb, mode);
    return hipGetLastError();
}

hipError_t launch_fcg_alpha(const double *p, const double *t, size_t n, double *partials, SolveState *st,
                            hipStream_t s)
{
    const int nb = dot_blocks(n);
    hipLaunchKernelGGL(pq_kernel, dim3(nb), dim3(256), 0, s, p, t, n, partials, &st->done);
    hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(1024), 0, s, st, (const double *)partials, nb, 1);
    return hipGetLastError();
}

hipError_t launch_fcg_alpha_partials(const double *partials, int nblk, SolveState *st, hipStream_t s)
{
    hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(1024), 0, s, st, partials, nblk, 3);
    return hipGetLastError();
}

int fcg_update_blocks(size_t n) { return dot_blocks(n); }

hipError_t launch_fcg_update(SolveState *st, double *x, const double *p, double *r, const double *t, float *r32,
                             size_t n, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(update_kernel, dim3(dot_blocks(n)), dim3(256), 0, s, (const SolveState *)st, x, p, r, t, r32,
                       n, partials);
    return hipGetLastError();
}

hipError_t launch_fcg_direction(SolveState *st, const double *z, double *p, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(direction_kernel, dim3(grid_blocks(n)), dim3(256), 0, s, (const SolveState *)st, z, p, n);
    return hipGetLastError();
}

hipError_t launch_cast_f32(const double *src, float *dst, size_t n, const int *done, hipStream_t s)
{
    hipLaunchKernelGGL(cast_f32_kernel, dim3(grid_blocks(n)), dim3(256), 0, s, src, dst, n, done);
    return hipGetLastError();
}

hipError_t launch_zero(double *x, size_t n, const int *done, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel, dim3(grid_blocks(n)), dim3(256), 0, s, x, n, done);
    return hipGetLastError();
}

}  // namespace nn4mg
