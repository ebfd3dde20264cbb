// The coarse end of the sawtooth cycle in one workgroup (gfx950).
//
// Below a few thousand cells a level is too small to fill the chip, and each
// of its kernels costs mostly launch and ramp-up time.  This kernel runs the
// whole coarse end of the cycle of Fig. multi-grid (arXiv 2401.06755, Sec.
// 2.4) in one 1024-thread workgroup with every field in LDS: restriction of
// the right-hand side down to the coarsest level (sum of the 8 children), the
// exact coarsest solve with the FP64 inverse (mean removed for singular
// problems), and on the way up the cell-centred trilinear prolongation and
// nu_post weighted-Jacobi sweeps per level.  The operator is the same
// linear-element filter as the z-marching kernel, written through the edge and
// corner sums of the 27-point neighbourhood:
//     S[v] = 2 (sum over the 12 edge neighbours) + (sum over the 8 corners),
//     constant coefficient  A y = (-h/12) (S[y] - 32 y),  D = 8h/3,
//     nodal coefficient     A y = (h/24) [(32 k + S[k]) y - k S[y] - S[k y]],
//                           D = (h/24) (32 k + S[k])   (Eq. k-T, link form),
// with halos from the boundary rules of Sec. 2.3.3 (the coefficient always
// +mirror).  Input: the right-hand side of the first tail level, or of the
// level above it (then restricted here); output: the correction of the first
// tail level, in HBM, for the prolongation into the next finer level.
#include "mg_internal.h"

#include <type_traits>

namespace nn4mg {

namespace {

constexpr int TT = 1024;

struct NoK {};

// Halo index -> interior index with the sign of a Dirichlet-zero wall (the
// same rules as the z-marching kernel; indices are at most one cell outside).
__device__ __forceinline__ int tfold(int i, int n, int lo, int hi, int &sgn)
{
    if (i < 0) {
        if (lo == BC_P) return i + n;
        if (lo == BC_D) sgn = -sgn;
        return -1 - i;
    }
    if (i >= n) {
        if (hi == BC_P) return i - n;
        if (hi == BC_D) sgn = -sgn;
        return 2 * n - 1 - i;
    }
    return i;
}

template <typename T, typename KT>
__device__ __forceinline__ T kval(const KT *k, int g)
{
    if constexpr (std::is_same<KT, __half>::value)
        return (T)__half2float(k[g]);
    else
        return (T)k[g];
}

// One tail level: dims, spacing and the offsets of its LDS fields (elements
// of the shared array): right-hand side, two iterates and the coefficient.
struct Lv {
    int nx, ny, nz, n;
    double h;
    int ob, oya, oyb, ok;
};

// out = y + omega (b - A y) / D over the level; every field in LDS.
template <typename T, bool HK>
__device__ __forceinline__ void sweep(T *sm, const Lv &L, int oy, int oo, const int *bc, T omega)
{
    const T h = (T)L.h;
    const T cw = -h / (T)12, icv = (T)24 / h;
    const T om_w0 = omega / ((T)(8.0 / 3.0) * h);
    const T *y = sm + oy;
    const T *kk = sm + L.ok;
    const T *b = sm + L.ob;
    T *out = sm + oo;
    for (int c = threadIdx.x; c < L.n; c += TT) {
        const int i = c % L.nx, t = c / L.nx;
        const int j = t % L.ny, kz = t / L.ny;
        T Sy = 0, Sk = 0, Sp = 0;
        const T y0 = y[c];
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            int sz = 1;
            const int fz = tfold(kz + dz, L.nz, bc[4], bc[5], sz);
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                int sy = sz;
                const int fy = tfold(j + dy, L.ny, bc[2], bc[3], sy);
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int nzc = (dx != 0) + (dy != 0) + (dz != 0);
                    if (nzc < 2) continue;  // centre and faces carry no weight
                    int s = sy;
                    const int fx = tfold(i + dx, L.nx, bc[0], bc[1], s);
                    const int g = fx + L.nx * (fy + L.ny * fz);
                    const T w = (nzc == 2) ? (T)2 : (T)1;
                    const T v = (s < 0) ? -y[g] : y[g];
                    Sy += w * v;
                    if constexpr (HK) {
                        const T kv = kk[g];
                        Sk += w * kv;
                        Sp += w * kv * v;
                    }
                }
            }
        }
        T r;
        if constexpr (!HK) {
            r = y0 + om_w0 * (b[c] - cw * (Sy - (T)32 * y0));
        } else {
            const T k0 = kk[c];
            const T Dg = (T)32 * k0 + Sk;
            const T Ays = Dg * y0 - k0 * Sy - Sp;
            r = y0 + omega * (b[c] * icv - Ays) / Dg;
        }
        out[c] = r;
    }
}

// y = P e of the coarser level (cell-centred trilinear, coarse halos by the
// boundary rules), interior cells; both fields in LDS.
template <typename T>
__device__ __forceinline__ void prolong(T *sm, const Lv &F, int oy, const Lv &C, int oe, const int *bc)
{
    const T *ec = sm + oe;
    T *y = sm + oy;
    const int cx = C.nx, cy = C.ny, cz = C.nz;
    for (int c = threadIdx.x; c < F.n; c += TT) {
        const int i = c % F.nx, t = c / F.nx;
        const int j = t % F.ny, kz = t / F.ny;
        int I[2], J[2], K[2];
        int sI[2] = {1, 1}, sJ[2] = {1, 1}, sK[2] = {1, 1};
        I[0] = tfold(i >> 1, cx, bc[0], bc[1], sI[0]);
        I[1] = tfold((i >> 1) + ((i & 1) ? 1 : -1), cx, bc[0], bc[1], sI[1]);
        J[0] = tfold(j >> 1, cy, bc[2], bc[3], sJ[0]);
        J[1] = tfold((j >> 1) + ((j & 1) ? 1 : -1), cy, bc[2], bc[3], sJ[1]);
        K[0] = tfold(kz >> 1, cz, bc[4], bc[5], sK[0]);
        K[1] = tfold((kz >> 1) + ((kz & 1) ? 1 : -1), cz, bc[4], bc[5], sK[1]);
        const T w[2] = {(T)0.75, (T)0.25};
        T acc = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            T pl = 0;
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                T row = 0;
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const int s = sI[d] * sJ[b2] * sK[a];
                    const T v = ec[I[d] + cx * (J[b2] + cy * K[a])];
                    row += w[d] * (s < 0 ? -v : v);
                }
                pl += w[b2] * row;
            }
            acc += w[a] * pl;
        }
        y[c] = acc;
    }
}

// out[c] = sum of the 8 children of coarse cell c; in has dims (2cx, 2cy, 2cz).
template <typename T, typename S>
__device__ __forceinline__ void restrict_to(const S *in, int cx, int cy, int cz, T *out)
{
    const int n = cx * cy * cz, fx = 2 * cx, fy = 2 * cy;
    const int sy = fx, sz = fx * fy;
    for (int c = threadIdx.x; c < n; c += TT) {
        const int I = c % cx, t = c / cx;
        const int J = t % cy, K = t / cy;
        const int g = 2 * I + fx * (2 * J + fy * 2 * K);
        const T v0 = (T)in[g], v1 = (T)in[g + 1], v2 = (T)in[g + sy], v3 = (T)in[g + sy + 1];
        const T v4 = (T)in[g + sz], v5 = (T)in[g + sz + 1], v6 = (T)in[g + sz + sy], v7 = (T)in[g + sz + sy + 1];
        out[c] = ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7));
    }
}

template <typename T, typename KT>
__global__ __launch_bounds__(TT) void tail_kernel(const TailArgs a)
{
    if (a.done && *a.done) return;
    constexpr bool HK = !std::is_same<KT, NoK>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    T *sm = (T *)smem;
    __shared__ double red[TT / 64];
    __shared__ Lv lv[kTailMaxLevels];
    __shared__ int s_total;
    const int nl = a.levels;
    if (threadIdx.x == 0) {
        int off = 0;
#pragma unroll
        for (int l = 0; l < kTailMaxLevels; ++l) {
            if (l < nl) {
                const int n = a.nx[l] * a.ny[l] * a.nz[l];
                lv[l].nx = a.nx[l];
                lv[l].ny = a.ny[l];
                lv[l].nz = a.nz[l];
                lv[l].n = n;
                lv[l].h = a.h[l];
                lv[l].ob = off;
                lv[l].oya = off + n;
                lv[l].oyb = off + 2 * n;
                lv[l].ok = HK ? off + 3 * n : 0;
                off += (HK ? 4 : 3) * n;
            }
        }
        s_total = off;
    }
    __syncthreads();
    const T om = (T)a.omega;
    const Lv &C = lv[nl - 1];
    const int nc = C.n;
    // FP64 inverse in LDS after the fields when it fits (8-byte aligned)
    double *ainv_s = (double *)(smem + (((size_t)s_total * sizeof(T) + 7) & ~(size_t)7));

    // every HBM read up front, all in flight together: the first level's
    // right-hand side (restricted from the level above if given), the
    // coefficient of every tail level and the coarsest inverse
    if (a.b_above)
        restrict_to<T, T>((const T *)a.b_above, lv[0].nx, lv[0].ny, lv[0].nz, sm + lv[0].ob);
    else
        for (int c = threadIdx.x; c < lv[0].n; c += TT) sm[lv[0].ob + c] = ((const T *)a.b_first)[c];
    if constexpr (HK) {
        for (int l = 0; l < nl; ++l) {
            const KT *kp = (const KT *)a.k[l];
            for (int c = threadIdx.x; c < lv[l].n; c += TT) sm[lv[l].ok + c] = kval<T, KT>(kp, c);
        }
    }
    if (a.ainv_in_lds)
        for (int c = threadIdx.x; c < nc * nc; c += TT) ainv_s[c] = a.ainv[c];
    __syncthreads();
    for (int l = 0; l + 1 < nl; ++l) {
        restrict_to<T, T>(sm + lv[l].ob, lv[l + 1].nx, lv[l + 1].ny, lv[l + 1].nz, sm + lv[l + 1].ob);
        __syncthreads();
    }

    // coarsest: e = A_c^{-1} b (symmetric inverse), mean removed if singular
    {
        const T *bc = sm + C.ob;
        const int i = threadIdx.x;
        double e = 0.0;
        if (i < nc) {
            if (a.ainv_in_lds) {
                for (int j = 0; j < nc; ++j) e += ainv_s[j * nc + i] * (double)bc[j];
            } else {
#pragma unroll 8
                for (int j = 0; j < nc; ++j) e += a.ainv[(size_t)j * nc + i] * (double)bc[j];
            }
        }
        if (a.singular) {
            double part = (i < nc) ? e : 0.0;
            for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
            __syncthreads();
            double sum = 0.0;
            for (int w = 0; w < TT / 64; ++w) sum += red[w];
            e -= sum / (double)nc;
        }
        if (i < nc) sm[C.oya + i] = (T)e;
        __syncthreads();
    }

    // up: y = P e_{l+1}, then nu_post sweeps; the prolongation goes to the
    // buffer that makes the last sweep land in ya
    for (int l = nl - 2; l >= 0; --l) {
        const Lv &V = lv[l];
        int src = (a.nu % 2 == 0) ? V.oya : V.oyb;
        prolong<T>(sm, V, src, lv[l + 1], lv[l + 1].oya, a.bc);
        __syncthreads();
        for (int s = 0; s < a.nu; ++s) {
            const int o = (src == V.oya) ? V.oyb : V.oya;
            sweep<T, HK>(sm, V, src, o, a.bc, om);
            __syncthreads();
            src = o;
        }
    }

    // the first tail level's correction back to HBM
    T *e_out = (T *)a.e_first;
    for (int c = threadIdx.x; c < lv[0].n; c += TT) e_out[c] = sm[lv[0].oya + c];
}

}  // namespace

size_t tail_lds_bytes(const TailArgs &a, int t_is_f64, int nodal)
{
    size_t n = 0;
    for (int l = 0; l < a.levels; ++l) n += (size_t)a.nx[l] * a.ny[l] * a.nz[l];
    size_t b = (nodal ? 4 : 3) * n * (t_is_f64 ? 8 : 4);
    b = (b + 7) & ~(size_t)7;
    if (a.ainv_in_lds) {
        const int l = a.levels - 1;
        const size_t nc = (size_t)a.nx[l] * a.ny[l] * a.nz[l];
        b += 8 * nc * nc;
    }
    return b;
}

hipError_t launch_tail(int T_is_f64, int kt, const TailArgs &a, hipStream_t s)
{
    if (a.levels < 1 || a.levels > kTailMaxLevels) return hipErrorInvalidValue;
    const size_t lds = tail_lds_bytes(a, T_is_f64, kt != KT_NONE);
    auto go = [&](auto kernel) -> hipError_t {
        hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kernel, dim3(1), dim3(TT), lds, s, a);
        return hipGetLastError();
    };
    if (T_is_f64) {
        if (kt == KT_NONE) return go(tail_kernel<double, NoK>);
        if (kt == KT_F64) return go(tail_kernel<double, double>);
        return hipErrorInvalidValue;
    }
    if (kt == KT_NONE) return go(tail_kernel<float, NoK>);
    if (kt == KT_F32) return go(tail_kernel<float, float>);
    if (kt == KT_F16) return go(tail_kernel<float, __half>);
    return hipErrorInvalidValue;
}

}  // namespace nn4mg
