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

struct Bc6 {
    int v[6];
};

template <typename T, typename KT>
__device__ __forceinline__ T kval(const KT *k, int g)
{
    if constexpr (std::is_same<KT, __half>::value)
        return (T)__half2float(k[g]);
    else
        return (T)k[g];
}

// One tail level: dims, spacing and the offsets of its LDS fields (elements
// of the shared array).  The right-hand side is stored without a halo; the two
// iterates and the coefficient carry a one-cell halo (padded dims px = nx + 2,
// ...), so stencils read fixed offsets.
struct Lv {
    int nx, ny, nz, n;
    int px, pxy, pn;   // padded row, plane and cell counts
    double h;
    int ob, oya, oyb, ok;
};

// The padded cells of a level a thread owns (p = thread + r * 1024, r < 2):
// the interior cell each holds (the folded one for a halo cell), its padded
// index and the sign of the boundary rule across the fold.  Computed once per
// level and shared by the prolongation and the sweeps.
struct PCell {
    int c, q, i, j, k, sg;  // c < 0: no cell
};

__device__ __forceinline__ void padded_cells(const Lv &V, const int *bc, PCell (&pc)[2])
{
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int p = (int)threadIdx.x + r * TT;
        if (p < V.pn) {
            // p / pxy and rem / px through FP32 reciprocals: (p + 0.5) / pxy lies at
            // least 0.5 / pxy from an integer, far above the rounding error while
            // pn < 2^21 (here pn <= 2 * 1024); FP32 keeps this off the slower FP64
            // conversions, which cost the most in this one-workgroup kernel
            const float rpxy = __builtin_amdgcn_rcpf((float)V.pxy), rpx = __builtin_amdgcn_rcpf((float)V.px);
            const int pk = (int)(((float)p + 0.5f) * rpxy);
            const int rem = p - pk * V.pxy;
            const int pj = (int)(((float)rem + 0.5f) * rpx);
            const int pi = rem - pj * V.px;
            int sg = 1;
            const int i = tfold(pi - 1, V.nx, bc[0], bc[1], sg);
            const int j = tfold(pj - 1, V.ny, bc[2], bc[3], sg);
            const int k = tfold(pk - 1, V.nz, bc[4], bc[5], sg);
            pc[r] = {i + V.nx * (j + V.ny * k), (k + 1) * V.pxy + (j + 1) * V.px + (i + 1), i, j, k, sg};
        } else {
            pc[r] = {-1, 0, 0, 0, 0, 1};
        }
    }
}

__device__ __forceinline__ int padded_of(const Lv &V, int c)
{
    // c / nx and t / ny through FP32 reciprocals, exact for these indices (as in padded_cells)
    const int t = (int)(((float)c + 0.5f) * __builtin_amdgcn_rcpf((float)V.nx));
    const int i = c - t * V.nx;
    const int k = (int)(((float)t + 0.5f) * __builtin_amdgcn_rcpf((float)V.ny));
    const int j = t - k * V.ny;
    return (k + 1) * V.pxy + (j + 1) * V.px + (i + 1);
}

__device__ __forceinline__ double trecip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    return fma(fma(-d, r, 1.0), r, r);
}
__device__ __forceinline__ float trecip(float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(fmaf(-d, r, 1.0f), r, r);
}

// Corner (D) and cross (X) sums of the 3x3 neighbourhood of o in a plane of row stride W.
template <typename T>
__device__ __forceinline__ T dsum(const T *v, int o, int W)
{
    return (v[o - W - 1] + v[o - W + 1]) + (v[o + W - 1] + v[o + W + 1]);
}
template <typename T>
__device__ __forceinline__ T xsum(const T *v, int o, int W)
{
    return (v[o - W] + v[o + W]) + (v[o - 1] + v[o + 1]);
}
template <typename T>
__device__ __forceinline__ T dprod(const T *v, const T *k, int o, int W)
{
    return (k[o - W - 1] * v[o - W - 1] + k[o - W + 1] * v[o - W + 1]) +
           (k[o + W - 1] * v[o + W - 1] + k[o + W + 1] * v[o + W + 1]);
}
template <typename T>
__device__ __forceinline__ T xprod(const T *v, const T *k, int o, int W)
{
    return (k[o - W] * v[o - W] + k[o + W] * v[o + W]) + (k[o - 1] * v[o - 1] + k[o + 1] * v[o + 1]);
}

// out = y + omega (b - A y) / D at every padded cell (halo cells take the
// signed value of the interior cell they mirror, so out is halo-complete):
// S = 2 D(z) + 2 (X(z-1) + X(z+1)) + D(z-1) + D(z+1) for y, k and k y.
template <typename T, bool HK>
__device__ __forceinline__ void sweep(T *sm, const Lv &L, const PCell (&pc)[2], int oy, int oo, T omega)
{
    const T h = (T)L.h;
    const T cw = -h / (T)12, icv = (T)24 / h;
    const T om_w0 = omega / ((T)(8.0 / 3.0) * h);
    const T *y = sm + oy;
    const T *kk = sm + L.ok;
    const T *b = sm + L.ob;
    T *out = sm + oo;
    const int W = L.px, WP = L.pxy;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (pc[r].c < 0) continue;
        const int c = pc[r].c, q = pc[r].q;
        const T y0 = y[q];
        const T Dz = dsum(y, q, W);
        const T Sy = (Dz + Dz + fma((T)2, xsum(y, q - WP, W), dsum(y, q - WP, W))) +
                     fma((T)2, xsum(y, q + WP, W), dsum(y, q + WP, W));
        T v;
        if constexpr (!HK) {
            v = y0 + om_w0 * (b[c] - cw * (Sy - (T)32 * y0));
        } else {
            const T Dk = dsum(kk, q, W);
            const T Sk = (Dk + Dk + fma((T)2, xsum(kk, q - WP, W), dsum(kk, q - WP, W))) +
                         fma((T)2, xsum(kk, q + WP, W), dsum(kk, q + WP, W));
            const T Dp = dprod(y, kk, q, W);
            const T Sp = (Dp + Dp + fma((T)2, xprod(y, kk, q - WP, W), dprod(y, kk, q - WP, W))) +
                         fma((T)2, xprod(y, kk, q + WP, W), dprod(y, kk, q + WP, W));
            const T k0 = kk[q];
            const T Dg = fma((T)32, k0, Sk);
            const T Ays = Dg * y0 - k0 * Sy - Sp;
            v = y0 + omega * (b[c] * icv - Ays) * trecip(Dg);
        }
        out[(int)threadIdx.x + r * TT] = pc[r].sg < 0 ? -v : v;
    }
}

// y = P e of the coarser level at every padded cell of F (cell-centred
// trilinear; the coarse field is halo-complete, so no folding is needed).
template <typename T>
__device__ __forceinline__ void prolong(T *sm, const PCell (&pc)[2], int oy, const Lv &C, int oe)
{
    const T *ec = sm + oe;
    T *y = sm + oy;
    const int CW = C.px, CP = C.pxy;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (pc[r].c < 0) continue;
        const int i = pc[r].i, j = pc[r].j, kz = pc[r].k;
        const int q = ((kz >> 1) + 1) * CP + ((j >> 1) + 1) * CW + ((i >> 1) + 1);
        const int dI = (i & 1) ? 1 : -1, dJ = (j & 1) ? CW : -CW, dK = (kz & 1) ? CP : -CP;
        const T w3 = (T)0.75, wq = (T)0.25;
        const T z00 = w3 * ec[q] + wq * ec[q + dK];
        const T z01 = w3 * ec[q + dI] + wq * ec[q + dI + dK];
        const T z10 = w3 * ec[q + dJ] + wq * ec[q + dJ + dK];
        const T z11 = w3 * ec[q + dJ + dI] + wq * ec[q + dJ + dI + dK];
        const T v = w3 * (w3 * z00 + wq * z01) + wq * (w3 * z10 + wq * z11);
        y[(int)threadIdx.x + r * TT] = pc[r].sg < 0 ? -v : v;
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

// Padded coefficient cells and coarsest-inverse entries a thread stages with its first loads.
constexpr int kTailKRegs = 3;
constexpr int kTailARegs = 4;

template <typename T, typename KT>
__global__ __launch_bounds__(TT) void tail_kernel(const TailArgs a)
{
    // batched: workgroup c runs copy c (its fields bstride bytes further on)
    const long long coff = a.ncopy > 1 ? (long long)blockIdx.x * a.bstride : 0;
    const int *done_p = copy_ptr(a.done, coff);
    const T *kpad_p = copy_ptr((const T *)a.kpad, coff);
    const T *b_above_p = copy_ptr((const T *)a.b_above, coff);
    const T *b_first_p = copy_ptr((const T *)a.b_first, coff);
    const double *ainv_p = copy_ptr(a.ainv, coff);
    T *e_first_p = copy_ptr((T *)a.e_first, coff);
    constexpr bool HK = !std::is_same<KT, NoK>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    T *sm = (T *)smem;
    __shared__ double red[TT / 64];
    __shared__ Lv lv[kTailMaxLevels];
    __shared__ int s_total;
    const int nl = a.levels;
    // the stopping flag is read with the first loads and tested before any write
    const int stop = done_p ? *done_p : 0;
    if (threadIdx.x == 0) {
        int off = 0;
#pragma unroll
        for (int l = 0; l < kTailMaxLevels; ++l) {
            if (l < nl) {
                const int n = a.nx[l] * a.ny[l] * a.nz[l];
                const int pn = (a.nx[l] + 2) * (a.ny[l] + 2) * (a.nz[l] + 2);
                lv[l].nx = a.nx[l];
                lv[l].ny = a.ny[l];
                lv[l].nz = a.nz[l];
                lv[l].n = n;
                lv[l].px = a.nx[l] + 2;
                lv[l].pxy = (a.nx[l] + 2) * (a.ny[l] + 2);
                lv[l].pn = pn;
                lv[l].h = a.h[l];
                lv[l].ob = off;
                lv[l].oya = off + n;
                lv[l].oyb = off + n + pn;
                off += n + 2 * pn;
            }
        }
        // the padded coefficients of all levels follow, contiguous as in kpad
        int ko = off;
#pragma unroll
        for (int l = 0; l < kTailMaxLevels; ++l) {
            if (l < nl) {
                lv[l].ok = HK ? ko : 0;
                if (HK) ko += lv[l].pn;
            }
        }
        s_total = ko;
    }

    // every HBM read up front, all in flight together: the first level's
    // right-hand side (restricted from the level above if given), the
    // coefficient of every tail level on its padded cells (the halo by the
    // +mirror rule) and the coarsest inverse
    const int n0 = a.nx[0] * a.ny[0] * a.nz[0];
    T rb = (T)0;
    if ((int)threadIdx.x < n0) {
        const int c = threadIdx.x;
        if (b_above_p) {
            const int cx = a.nx[0], cy = a.ny[0];
            const int I = c % cx, t = c / cx;
            const int J = t % cy, K = t / cy;
            const int fx = 2 * cx, fy = 2 * cy, sy = fx, sz = fx * fy;
            const T *in = b_above_p;
            const int g = 2 * I + fx * (2 * J + fy * 2 * K);
            const T v0 = in[g], v1 = in[g + 1], v2 = in[g + sy], v3 = in[g + sy + 1];
            const T v4 = in[g + sz], v5 = in[g + sz + 1], v6 = in[g + sz + sy], v7 = in[g + sz + sy + 1];
            rb = ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7));
        } else {
            rb = b_first_p[c];
        }
    }
    // padded coefficients (contiguous) and the coarsest inverse, first parts in registers
    int ktot = 0, kbase = 0;
#pragma unroll
    for (int l = 0; l < kTailMaxLevels; ++l) {
        if (l < nl) {
            kbase += a.nx[l] * a.ny[l] * a.nz[l] + 2 * (a.nx[l] + 2) * (a.ny[l] + 2) * (a.nz[l] + 2);
            if (HK) ktot += (a.nx[l] + 2) * (a.ny[l] + 2) * (a.nz[l] + 2);
        }
    }
    T kr[HK ? kTailKRegs : 1];
    if constexpr (HK) {
#pragma unroll
        for (int q = 0; q < kTailKRegs; ++q) {
            const int f = (int)threadIdx.x + q * TT;
            kr[q] = f < ktot ? kpad_p[f] : (T)0;
        }
    }
    const int ncl = a.nx[nl - 1] * a.ny[nl - 1] * a.nz[nl - 1];
    double ar[kTailARegs];
#pragma unroll
    for (int q = 0; q < kTailARegs; ++q) {
        const int f = (int)threadIdx.x + q * TT;
        ar[q] = (a.ainv_in_lds && f < ncl * ncl) ? ainv_p[f] : 0.0;
    }
    if (stop) return;  // uniform over the workgroup
    __syncthreads();   // level table

    const T om = (T)a.omega;
    const Lv &C = lv[nl - 1];
    const int nc = C.n;
    // FP64 inverse in LDS after the fields when it fits (8-byte aligned)
    double *ainv_s = (double *)(smem + (((size_t)s_total * sizeof(T) + 7) & ~(size_t)7));
    if ((int)threadIdx.x < n0) sm[lv[0].ob + threadIdx.x] = rb;
    if constexpr (HK) {
#pragma unroll
        for (int q = 0; q < kTailKRegs; ++q) {
            const int f = (int)threadIdx.x + q * TT;
            if (f < ktot) sm[kbase + f] = kr[q];
        }
        for (int f = threadIdx.x + kTailKRegs * TT; f < ktot; f += TT) sm[kbase + f] = kpad_p[f];
    }
    if (a.ainv_in_lds) {
#pragma unroll
        for (int q = 0; q < kTailARegs; ++q) {
            const int f = (int)threadIdx.x + q * TT;
            if (f < nc * nc) ainv_s[f] = ar[q];
        }
        for (int c = threadIdx.x + kTailARegs * TT; c < nc * nc; c += TT) ainv_s[c] = ainv_p[c];
    }
    __syncthreads();
    for (int l = 0; l + 1 < nl; ++l) {
        restrict_to<T, T>(sm + lv[l].ob, lv[l + 1].nx, lv[l + 1].ny, lv[l + 1].nz, sm + lv[l + 1].ob);
        __syncthreads();
    }

    // coarsest: e = A_c^{-1} b (symmetric inverse), mean removed if singular,
    // at every padded cell (halo cells from the cell they mirror; at most two
    // padded cells per thread)
    {
        const T *bc = sm + C.ob;
        double e[2] = {0.0, 0.0};
        int sg[2] = {1, 1};
        double part = 0.0;
        PCell pc[2];
        padded_cells(C, a.bc, pc);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int p = threadIdx.x + r * TT;
            if (pc[r].c >= 0) {
                const int i = pc[r].c;
                sg[r] = pc[r].sg;
                // four interleaved partial sums keep the loads in flight
                double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
                const double *col = a.ainv_in_lds ? (const double *)ainv_s : ainv_p;
                int j = 0;
                if (a.ainv_in_lds) {
                    for (; j + 3 < nc; j += 4) {
                        acc0 += ainv_s[j * nc + i] * (double)bc[j];
                        acc1 += ainv_s[(j + 1) * nc + i] * (double)bc[j + 1];
                        acc2 += ainv_s[(j + 2) * nc + i] * (double)bc[j + 2];
                        acc3 += ainv_s[(j + 3) * nc + i] * (double)bc[j + 3];
                    }
                } else {
                    for (; j + 3 < nc; j += 4) {
                        acc0 += col[(size_t)j * nc + i] * (double)bc[j];
                        acc1 += col[(size_t)(j + 1) * nc + i] * (double)bc[j + 1];
                        acc2 += col[(size_t)(j + 2) * nc + i] * (double)bc[j + 2];
                        acc3 += col[(size_t)(j + 3) * nc + i] * (double)bc[j + 3];
                    }
                }
                for (; j < nc; ++j) acc0 += col[(size_t)j * nc + i] * (double)bc[j];
                e[r] = (acc0 + acc1) + (acc2 + acc3);
                if (pc[r].q == p) part += e[r];
            }
        }
        if (a.singular) {
            for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
            __syncthreads();
            double sum = 0.0;
            for (int w = 0; w < TT / 64; ++w) sum += red[w];
            e[0] -= sum / (double)nc;
            e[1] -= sum / (double)nc;
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int p = threadIdx.x + r * TT;
            if (p < C.pn) sm[C.oya + p] = (T)(sg[r] < 0 ? -e[r] : e[r]);
        }
        __syncthreads();
    }

    // up: y = P e_{l+1}, then nu_post sweeps; the prolongation goes to the
    // buffer that makes the last sweep land in ya
    for (int l = nl - 2; l >= 0; --l) {
        const Lv &V = lv[l];
        PCell pc[2];
        padded_cells(V, a.bc, pc);
        int src = (a.nu % 2 == 0) ? V.oya : V.oyb;
        prolong<T>(sm, pc, src, lv[l + 1], lv[l + 1].oya);
        __syncthreads();
        for (int s = 0; s < a.nu; ++s) {
            const int o = (src == V.oya) ? V.oyb : V.oya;
            sweep<T, HK>(sm, V, pc, src, o, om);
            __syncthreads();
            src = o;
        }
    }

    // the first tail level's correction back to HBM
    T *e_out = e_first_p;
    for (int c = threadIdx.x; c < lv[0].n; c += TT) e_out[c] = sm[lv[0].oya + padded_of(lv[0], c)];
}

}  // namespace

size_t tail_field_cells(const int *nx, const int *ny, const int *nz, int levels, int nodal)
{
    size_t n = 0;
    for (int l = 0; l < levels; ++l) {
        const size_t pn = (size_t)(nx[l] + 2) * (ny[l] + 2) * (nz[l] + 2);
        n += (size_t)nx[l] * ny[l] * nz[l] + (nodal ? 3 : 2) * pn;
    }
    return n;
}

size_t tail_lds_bytes(const TailArgs &a, int t_is_f64, int nodal)
{
    size_t b = tail_field_cells(a.nx, a.ny, a.nz, a.levels, nodal) * (t_is_f64 ? 8 : 4);
    b = (b + 7) & ~(size_t)7;
    if (a.ainv_in_lds) {
        const int l = a.levels - 1;
        const size_t nc = (size_t)a.nx[l] * a.ny[l] * a.nz[l];
        b += 8 * nc * nc;
    }
    return b;
}

namespace {

template <typename T, typename KT>
__global__ __launch_bounds__(256) void kpad_kernel(const KT *k, int nx, int ny, int nz, Bc6 bc, T *out)
{
    const int pn = (nx + 2) * (ny + 2) * (nz + 2);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pn) return;
    const int px = nx + 2, pi = p % px, t = p / px;
    const int pj = t % (ny + 2), pk = t / (ny + 2);
    int sg = 1;
    const int i = tfold(pi - 1, nx, bc.v[0], bc.v[1], sg);
    const int j = tfold(pj - 1, ny, bc.v[2], bc.v[3], sg);
    const int kk = tfold(pk - 1, nz, bc.v[4], bc.v[5], sg);
    out[p] = kval<T, KT>(k, i + nx * (j + ny * kk));  // the coefficient's halo is +mirror
}

}  // namespace

hipError_t launch_tail_kpad(int T_is_f64, int kt, const void *k, int nx, int ny, int nz, const int *bc, void *out,
                            hipStream_t s)
{
    Bc6 b;
    for (int f = 0; f < 6; ++f) b.v[f] = bc[f];
    const int pn = (nx + 2) * (ny + 2) * (nz + 2);
    const dim3 grid((pn + 255) / 256), block(256);
    if (T_is_f64) {
        if (kt != KT_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((kpad_kernel<double, double>), grid, block, 0, s, (const double *)k, nx, ny, nz, b,
                           (double *)out);
    } else if (kt == KT_F32) {
        hipLaunchKernelGGL((kpad_kernel<float, float>), grid, block, 0, s, (const float *)k, nx, ny, nz, b,
                           (float *)out);
    } else if (kt == KT_F16) {
        hipLaunchKernelGGL((kpad_kernel<float, __half>), grid, block, 0, s, (const __half *)k, nx, ny, nz, b,
                           (float *)out);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tail(int T_is_f64, int kt, const TailArgs &a, hipStream_t s)
{
    if (a.levels < 1 || a.levels > kTailMaxLevels) return hipErrorInvalidValue;
    if (a.nx[0] * a.ny[0] * a.nz[0] > TT) return hipErrorInvalidValue;
    for (int l = 0; l < a.levels; ++l)
        if ((a.nx[l] + 2) * (a.ny[l] + 2) * (a.nz[l] + 2) > 2 * TT) return hipErrorInvalidValue;
    if (kt != KT_NONE && !a.kpad) return hipErrorInvalidValue;
    const size_t lds = tail_lds_bytes(a, T_is_f64, kt != KT_NONE);
    auto go = [&](auto kernel) -> hipError_t {
        hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kernel, dim3(a.ncopy > 1 ? a.ncopy : 1), dim3(TT), lds, s, a);
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
