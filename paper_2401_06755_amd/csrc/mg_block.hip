// Both post-smoothing sweeps of a small level as independent 8 x 8 x 8 blocks (gfx950).
//
// The sawtooth cycle of Fig. multi-grid (arXiv 2401.06755, Sec. 2.4) ends each
// level with the prolongation of the coarser correction and nu_post = 2
// weighted-Jacobi sweeps.  On the coarse levels the z-marching two-sweep kernel
// takes about as long as its chain of plane steps (loads, LDS commits and
// barriers, one plane after another), whatever the level size.  Here each
// workgroup owns one E^3 output block (E = 8; 4 on levels with too few 8^3
// blocks to fill the chip) and stages everything it needs at once:
//   * the coarse correction under the block ((E/2 + 4)^3 coarse cells, halos
//     by the boundary rules) and, for a nodal coefficient, k on the block plus
//     a two-cell ring ((E + 4)^3), in one round of global loads;
//   * P e on the (E + 4)^3 region, cell-centred trilinear from the staged coarse cells;
//   * the first sweep on the block plus a one-cell ring ((E + 2)^3);
//   * the second sweep on the block, written out.
// Ring cells outside the grid are computed from halo-synthesised inputs like
// any other cell: the sweep commutes with the boundary reflections, so they
// hold the halo values of the first sweep's output (as in the marching kernel).
// Operator and sweep are those of the stencil kernels: with the plane sums D
// (corners) and X (crosses) of the 3x3 neighbourhood,
//   S = 2 D(z) + 2 (X(z-1) + X(z+1)) + D(z-1) + D(z+1),
//   constant coefficient  A y = (-h/12) (S[y] - 32 y),
//   nodal coefficient     A_k y = (h/24) [(32 k + S[k]) y - k S[y] - S[k y]] (Eq. k-T).
#include "mg_device.h"
#include "mg_internal.h"

namespace nn4mg {

namespace {

// Corner and cross sums of the 3x3 neighbourhood of o in a plane with row stride W.
template <typename T, int W>
__device__ __forceinline__ T dsum(const T *v, int o)
{
    return (v[o - W - 1] + v[o - W + 1]) + (v[o + W - 1] + v[o + W + 1]);
}
template <typename T, int W>
__device__ __forceinline__ T xsum(const T *v, int o)
{
    return (v[o - W] + v[o + W]) + (v[o - 1] + v[o + 1]);
}
// The same for the product k v, k with its own strides.
template <typename T, int W, int WK>
__device__ __forceinline__ T dprod(const T *v, int o, const T *k, int ok)
{
    return (k[ok - WK - 1] * v[o - W - 1] + k[ok - WK + 1] * v[o - W + 1]) +
           (k[ok + WK - 1] * v[o + W - 1] + k[ok + WK + 1] * v[o + W + 1]);
}
template <typename T, int W, int WK>
__device__ __forceinline__ T xprod(const T *v, int o, const T *k, int ok)
{
    return (k[ok - WK] * v[o - W] + k[ok + WK] * v[o + W]) + (k[ok - 1] * v[o - 1] + k[ok + 1] * v[o + 1]);
}

// One Jacobi update of the cell at c of field v (row stride W, plane stride WP);
// the coefficient at ck of k (strides WK, WKP).  Sums in the order of the
// marching kernels: 2 D(z) + (2 X(z-1) + D(z-1)), then + (2 X(z+1) + D(z+1)).
template <typename T, bool HK, int W, int WP, int WK, int WKP>
__device__ __forceinline__ T jacobi_at(const T *v, int c, const T *k, int ck, T bb, T cw, T om_w0, T om, T icv)
{
    const T y0 = v[c];
    const T Dz = dsum<T, W>(v, c);
    const T Sx = (Dz + Dz + fma((T)2, xsum<T, W>(v, c - WP), dsum<T, W>(v, c - WP))) +
                 fma((T)2, xsum<T, W>(v, c + WP), dsum<T, W>(v, c + WP));
    if constexpr (!HK) {
        return y0 + om_w0 * (bb - cw * (Sx - (T)32 * y0));
    } else {
        const T kc = k[ck];
        const T Dk = dsum<T, WK>(k, ck);
        const T Sk = (Dk + Dk + fma((T)2, xsum<T, WK>(k, ck - WKP), dsum<T, WK>(k, ck - WKP))) +
                     fma((T)2, xsum<T, WK>(k, ck + WKP), dsum<T, WK>(k, ck + WKP));
        const T Dp = dprod<T, W, WK>(v, c, k, ck);
        const T Sp = (Dp + Dp + fma((T)2, xprod<T, W, WK>(v, c - WP, k, ck - WKP),
                                    dprod<T, W, WK>(v, c - WP, k, ck - WKP))) +
                     fma((T)2, xprod<T, W, WK>(v, c + WP, k, ck + WKP), dprod<T, W, WK>(v, c + WP, k, ck + WKP));
        const T Dg = fma((T)32, kc, Sk);
        const T Ays = Dg * y0 - kc * Sx - Sp;
        return y0 + om * (bb * icv - Ays) * recip(Dg);
    }
}

// Shape of a single-level block pass: output block edge E (8, or 4 for levels
// with too few 8^3 blocks to fill the chip), NT threads.  Every output cell's
// arithmetic is the same whatever E, so both edges give identical results.
template <int E>
struct BlockShape {
    static constexpr int NT = E == 8 ? 512 : 256;
    static constexpr int PE = E + 4, PN = PE * PE * PE;      // staged input region (two-cell ring)
    static constexpr int QE = E + 2, QN = QE * QE * QE;      // first-sweep region (one-cell ring)
    static constexpr int CE = E / 2 + 4, CN = CE * CE * CE;  // coarse footprint
    static constexpr int ON = E * E * E;                     // output cells
    static constexpr int NP = (PN + NT - 1) / NT;
    static constexpr int NQ = (QN + NT - 1) / NT;
    static_assert(CN <= NT && ON <= NT, "one coarse cell and at most one output cell per thread");
};

template <typename T, typename KT, int OUT, int E>
__global__ __launch_bounds__(BlockShape<E>::NT) void sweep2_block_kernel(const StencilArgs a_)
{
    using S = BlockShape<E>;
    constexpr int NT = S::NT, PE = S::PE, PN = S::PN, QE = S::QE, QN = S::QN, CE = S::CE, CN = S::CN;
    constexpr int NP = S::NP, NQ = S::NQ;
    StencilArgs a = a_;
    const int lb = enter_copy(a, xcd_remap(blockIdx.x, gridDim.x));
    constexpr bool HK = HasK<KT>::value;
    constexpr bool ADD = OUT == OUT_ADD64;
    __shared__ T sx[PN];                // P e on the staged region
    __shared__ T sk[HK ? PN : 1];       // coefficient on the staged region
    __shared__ T sy[QN];                // first-sweep output
    __shared__ T sc[CN];                // coarse footprint

    // the stopping flag is read with the first loads and tested before any write
    const int stop = a.done ? *a.done : 0;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int bxn = (nx + E - 1) / E, byn = (ny + E - 1) / E;
    const int bx = lb % bxn, rest = lb / bxn;
    const int by = rest % byn, bz = rest / byn;
    const int i0 = bx * E, j0 = by * E, k0 = bz * E;
    const int t = threadIdx.x;

    const T h = (T)a.h, om = (T)a.omega;
    const T cw = -h / (T)12, cv = h / (T)24;
    const T om_w0 = om / ((T)(8.0 / 3.0) * h);
    const T icv = (T)1 / cv;

    const T *bp = (const T *)a.b;
    const KT *kp = (const KT *)a.k;

    // one round of global loads: coarse footprint, coefficient, right-hand sides
    T cval;
    {
        const int ct = min(t, CN - 1);
        const int cx = ct % CE, cy = (ct / CE) % CE, cz = ct / (CE * CE);
        int s = 1;
        const int fI = fold((i0 >> 1) - 2 + cx, a.cnx, a.g.bc[0], a.g.bc[1], s);
        const int fJ = fold((j0 >> 1) - 2 + cy, a.cny, a.g.bc[2], a.g.bc[3], s);
        const int fK = fold((k0 >> 1) - 2 + cz, a.cnz, a.g.bc[4], a.g.bc[5], s);
        const T v = ((const T *)a.ec)[(size_t)fI + (size_t)a.cnx * ((size_t)fJ + (size_t)a.cny * (size_t)fK)];
        cval = s < 0 ? -v : v;
    }
    typename KStore<T, KT>::type kr[HK ? NP : 1];
    if constexpr (HK) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int idx = min(q * NT + t, PN - 1);
            const int px = idx % PE, py = (idx / PE) % PE, pz = idx / (PE * PE);
            int s = 1;
            const int fi = fold(i0 + px - 2, nx, a.g.bc[0], a.g.bc[1], s);
            const int fj = fold(j0 + py - 2, ny, a.g.bc[2], a.g.bc[3], s);
            const int fk = fold(k0 + pz - 2, nz, a.g.bc[4], a.g.bc[5], s);
            kr[q] = kp[(size_t)fi + (size_t)nx * ((size_t)fj + (size_t)ny * (size_t)fk)];
        }
    }
    T bq[NQ];  // first-sweep right-hand side, signed by the halo rule
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int idx = min(q * NT + t, QN - 1);
        const int qx = idx % QE, qy = (idx / QE) % QE, qz = idx / (QE * QE);
        int s = 1;
        const int fi = fold(i0 + qx - 1, nx, a.g.bc[0], a.g.bc[1], s);
        const int fj = fold(j0 + qy - 1, ny, a.g.bc[2], a.g.bc[3], s);
        const int fk = fold(k0 + qz - 1, nz, a.g.bc[4], a.g.bc[5], s);
        const T v = bp[(size_t)fi + (size_t)nx * ((size_t)fj + (size_t)ny * (size_t)fk)];
        bq[q] = s < 0 ? -v : v;
    }
    // this thread's output cell (threads beyond the block's cells only stage)
    const int ot = min(t, S::ON - 1);
    const int ox = ot % E, oy = (ot / E) % E, oz = ot / (E * E);
    const int gi = i0 + ox, gj = j0 + oy, gk = k0 + oz;
    const bool valid = t < S::ON && gi < nx && gj < ny && gk < nz;
    const size_t g = (size_t)min(gi, nx - 1) + (size_t)nx * ((size_t)min(gj, ny - 1) + (size_t)ny * (size_t)min(gk, nz - 1));
    const T b2 = bp[g];
    double xo = 0.0;
    if constexpr (ADD) xo = a.x64[g];
    if (stop) return;  // uniform over the workgroup

    if (t < CN) sc[t] = cval;
    if constexpr (HK) {
#pragma unroll
        for (int q = 0; q < NP; ++q)
            if (q * NT + t < PN) sk[q * NT + t] = kconv<T, KT>(kr[q]);
    }
    __syncthreads();

    // P e on the staged region: z first, then the x-y bilinear weights
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int idx = q * NT + t;
        if (idx < PN) {
            const int px = idx % PE, py = (idx / PE) % PE, pz = idx / (PE * PE);
            const int ui = i0 + px - 2, uj = j0 + py - 2, uk = k0 + pz - 2;  // unfolded fine position
            const int I = (ui >> 1) - ((i0 >> 1) - 2), J = (uj >> 1) - ((j0 >> 1) - 2);
            const int K = (uk >> 1) - ((k0 >> 1) - 2);
            const int dI = (ui & 1) ? 1 : -1, dJ = (uj & 1) ? CE : -CE, dK = (uk & 1) ? CE * CE : -CE * CE;
            const T w3 = (T)0.75, wq = (T)0.25;
            const int c00 = I + CE * J + CE * CE * K;
            const T z00 = w3 * sc[c00] + wq * sc[c00 + dK];
            const T z01 = w3 * sc[c00 + dI] + wq * sc[c00 + dI + dK];
            const T z10 = w3 * sc[c00 + dJ] + wq * sc[c00 + dJ + dK];
            const T z11 = w3 * sc[c00 + dJ + dI] + wq * sc[c00 + dJ + dI + dK];
            sx[idx] = w3 * (w3 * z00 + wq * z01) + wq * (w3 * z10 + wq * z11);
        }
    }
    __syncthreads();

    // first sweep on the block plus its one-cell ring
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int idx = q * NT + t;
        if (idx < QN) {
            const int qx = idx % QE, qy = (idx / QE) % QE, qz = idx / (QE * QE);
            const int c = (qz + 1) * PE * PE + (qy + 1) * PE + (qx + 1);
            sy[idx] = jacobi_at<T, HK, PE, PE * PE, PE, PE * PE>(sx, c, sk, c, bq[q], cw, om_w0, om, icv);
        }
    }
    __syncthreads();

    // second sweep on the block
    if (valid) {
        const int cyy = (oz + 1) * QE * QE + (oy + 1) * QE + (ox + 1);
        const int ckk = (oz + 2) * PE * PE + (oy + 2) * PE + (ox + 2);
        const T y = jacobi_at<T, HK, QE, QE * QE, PE, PE * PE>(sy, cyy, sk, ckk, b2, cw, om_w0, om, icv);
        if constexpr (ADD)
            a.x64[g] = xo + (double)y;
        else
            ((T *)a.yout)[g] = y;
    }
}

// Launches with fewer 8^3 blocks than this (over all copies) use 4^3 blocks:
// a block pass is bound by its workgroup's LDS reads, so a level that leaves
// most compute units idle runs faster as more, smaller blocks.
constexpr int kSmallBlockBelow = 256;

template <typename T, typename KT, int OUT>
hipError_t goB(const StencilArgs &a_, hipStream_t s)
{
    StencilArgs a = a_;
    const int nb8 = block2_blocks(a.g.nx, a.g.ny, a.g.nz);
    if ((long long)nb8 * (a.ncopy > 1 ? a.ncopy : 1) < kSmallBlockBelow) {
        const int nb4 = ((a.g.nx + 3) / 4) * ((a.g.ny + 3) / 4) * ((a.g.nz + 3) / 4);
        const unsigned grid = batched_grid(a, nb4);
        hipLaunchKernelGGL((sweep2_block_kernel<T, KT, OUT, 4>), dim3(grid), dim3(BlockShape<4>::NT), 0, s, a);
    } else {
        const unsigned grid = batched_grid(a, nb8);
        hipLaunchKernelGGL((sweep2_block_kernel<T, KT, OUT, 8>), dim3(grid), dim3(BlockShape<8>::NT), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

int block2_blocks(int nx, int ny, int nz)
{
    return ((nx + 7) / 8) * ((ny + 7) / 8) * ((nz + 7) / 8);
}

hipError_t launch_sweep2_block(int T_is_f64, int kt, int out_mode, const StencilArgs &a, hipStream_t s)
{
    if (a.g.nx < 2 || a.g.ny < 2 || a.g.nz < 2) return hipErrorInvalidValue;
    if (a.bmean || !a.ec || !a.b) return hipErrorInvalidValue;
    if (T_is_f64) {
        if (out_mode == OUT_STORE) {
            if (kt == KT_NONE) return goB<double, NoK, OUT_STORE>(a, s);
            if (kt == KT_F64) return goB<double, double, OUT_STORE>(a, s);
        }
        if (out_mode == OUT_ADD64) {
            if (kt == KT_NONE) return goB<double, NoK, OUT_ADD64>(a, s);
            if (kt == KT_F64) return goB<double, double, OUT_ADD64>(a, s);
        }
        return hipErrorInvalidValue;
    }
    if (out_mode == OUT_STORE) {
        if (kt == KT_NONE) return goB<float, NoK, OUT_STORE>(a, s);
        if (kt == KT_F32) return goB<float, float, OUT_STORE>(a, s);
        if (kt == KT_F16) return goB<float, __half, OUT_STORE>(a, s);
    }
    if (out_mode == OUT_ADD64) {
        if (kt == KT_NONE) return goB<float, NoK, OUT_ADD64>(a, s);
        if (kt == KT_F32) return goB<float, float, OUT_ADD64>(a, s);
        if (kt == KT_F16) return goB<float, __half, OUT_ADD64>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace nn4mg
