// Device helpers shared by the z-marching stencil kernels (not part of the C-ABI).
#pragma once

#include "mg_internal.h"

#include <type_traits>

namespace nn4mg {
namespace {

struct NoK {};

template <typename KT>
struct HasK {
    static constexpr bool value = true;
};
template <>
struct HasK<NoK> {
    static constexpr bool value = false;
};

// Storage type of a prefetched coefficient value (the value as loaded).
template <typename T, typename KT>
struct KStore {
    using type = KT;
};
template <typename T>
struct KStore<T, NoK> {
    using type = T;
};

template <typename T, typename KT>
__device__ __forceinline__ T kconv(typename KStore<T, KT>::type v)
{
    if constexpr (std::is_same<KT, __half>::value)
        return (T)__half2float(v);
    else if constexpr (std::is_same<KT, NoK>::value)
        return (T)0;
    else
        return (T)v;
}

// 1/d: hardware reciprocal refined by Newton steps (two in FP64).
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ float recip(float d)
{
    float r = __builtin_amdgcn_rcpf(d);
    return fmaf(fmaf(-d, r, 1.0f), r, r);
}

// Halo index -> interior index, flipping the sign across a Dirichlet-zero
// wall.  Indices beyond the one-cell halo (ragged tiles) are clamped into
// range; their values are never used by a valid output.
__device__ __forceinline__ int fold(int i, int n, int lo, int hi, int &sgn)
{
    if (i < 0) {
        if (lo == BC_P) {
            i += n;
            return i < 0 ? 0 : i;
        }
        if (lo == BC_D) sgn = -sgn;
        i = -1 - i;
        return i < n ? i : n - 1;
    }
    if (i >= n) {
        if (hi == BC_P) {
            i -= n;
            return i < n ? i : n - 1;
        }
        if (hi == BC_D) sgn = -sgn;
        i = 2 * n - 1 - i;
        return i >= 0 ? i : 0;
    }
    return i;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8).
// Give each XCD a contiguous range of tiles so neighbouring tiles, which share
// halo lines, share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, k = b >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

}  // namespace
}  // namespace nn4mg
