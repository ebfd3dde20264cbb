// HIP kernels for gfx950 (MI355X) of the sawtooth multigrid pressure solve of
// arXiv 2401.06755 (Sec. 2.4, Fig. multi-grid).
//
// The hot kernel is one z-marching stencil kernel.  A workgroup of 256 threads
// (one wave per 64-cell row, two rows per thread) owns a 64 x 8 column of cells
// and marches a chunk of z-planes.  Each plane is staged once in LDS with its
// one-cell halo; the halo is synthesised at load time from the boundary rules
// of Sec. 2.3.3 (Dirichlet: -mirror, Neumann: +mirror, periodic: wrap; the
// coefficient always +mirror), so no padded copies exist in HBM.  From LDS each
// thread keeps, per plane, the centre plus the "diagonal" (4 corners of the
// 3x3) and "cross" (4 edge midpoints) sums; the 27-point linear-element filter
// needs only those, because its face weights are zero:
//     A x = w0 x + we (D_0 + X_-1 + X_+1) + wc (D_-1 + D_+1),
// with w0 = 8h/3, we = -h/6 (12 edge neighbours), wc = -h/12 (8 corners).
// For a nodal coefficient k, Eq. (k-T) of Sec. 2.2.4 is evaluated in the
// equivalent link form
//     A_k x = D x_i - k_i S[x] - S[k x],  D = (4h/3) k_i + S[k],
// S[v] = sum_s c_s v_s with c_s = -w_s / 2 over the 20 edge/corner offsets,
// so the plane sums of x, k and k.x are all the kernel needs.
//
// The same kernel body produces a Jacobi sweep (optionally reading its input
// as x + P e_coarse, the U-Net decoder's upsample-and-add) or a residual with
// the 2x restriction (U-Net encoder) and a per-block sum of r^2 fused in.
#include "mg_internal.h"

#include <type_traits>

namespace nn4mg {

namespace {

constexpr int NT = 256;
constexpr int TX = kTileX;  // 64 cells along x per tile (one wave row)
constexpr int TY = kTileY;  // 8 cells along y per tile (4 thread rows x 2)
constexpr int PX = TX + 2;  // LDS plane with halo
constexpr int PY = TY + 2;
constexpr int PN = PX * PY;

struct NoK {};

template <typename KT>
struct HasK {
    static constexpr bool value = true;
};
template <>
struct HasK<NoK> {
    static constexpr bool value = false;
};

template <typename T, typename KT>
__device__ __forceinline__ T kload(const KT *k, size_t g)
{
    if constexpr (std::is_same<KT, __half>::value)
        return (T)__half2float(k[g]);
    else
        return (T)k[g];
}

// Map a (possibly halo) index to an interior index and flip the sign for a
// Dirichlet-zero wall.  Indices beyond the one-cell halo (ragged tiles) are
// clamped into range; their values are never used by a valid output.
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

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Give each XCD a contiguous range of logical tiles so neighbouring
// tiles (which share halo cache lines) share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, k = b >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Cell-centred trilinear prolongation at fine interior cell (fi, fj, fk):
// per axis 3/4 of the parent and 1/4 of the parent's neighbour on the side of
// the child; coarse halos follow the boundary rules.
template <typename T>
__device__ __forceinline__ T prolong_at(const StencilArgs &a, int fi, int fj, int fk)
{
    const T *e = (const T *)a.ec;
    const int cnx = a.cnx, cny = a.cny, cnz = a.cnz;
    const int I = fi >> 1, J = fj >> 1, K = fk >> 1;
    int sI = 1, sJ = 1, sK = 1;
    const int I1 = fold(I + ((fi & 1) ? 1 : -1), cnx, a.g.bc[0], a.g.bc[1], sI);
    const int J1 = fold(J + ((fj & 1) ? 1 : -1), cny, a.g.bc[2], a.g.bc[3], sJ);
    const int K1 = fold(K + ((fk & 1) ? 1 : -1), cnz, a.g.bc[4], a.g.bc[5], sK);
    const T w3 = (T)0.75;
    const T wx = (T)(0.25 * sI), wy = (T)(0.25 * sJ), wz = (T)(0.25 * sK);
    const size_t sy = (size_t)cnx, sz = (size_t)cnx * cny;
    const size_t r00 = J * sy + K * sz, r10 = J1 * sy + K * sz, r01 = J * sy + K1 * sz, r11 = J1 * sy + K1 * sz;
    const T p00 = w3 * e[r00 + I] + wx * e[r00 + I1];
    const T p10 = w3 * e[r10 + I] + wx * e[r10 + I1];
    const T p01 = w3 * e[r01 + I] + wx * e[r01 + I1];
    const T p11 = w3 * e[r11 + I] + wx * e[r11 + I1];
    return w3 * (w3 * p00 + wy * p10) + wz * (w3 * p01 + wy * p11);
}

// Stage plane z (with its halo ring) of the smoothed field and of k in LDS.
template <typename T, typename KT, int IN>
__device__ __forceinline__ void load_plane(T *sx, T *sk, const StencilArgs &a, int i0, int j0, int z)
{
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    int sz = 1;
    const int fk = fold(z, nz, a.g.bc[4], a.g.bc[5], sz);
    const T *yin = (const T *)a.yin;
    const KT *kp = (const KT *)a.k;
    for (int idx = threadIdx.x; idx < PN; idx += NT) {
        const int py = idx / PX;
        const int px = idx - py * PX;
        int s = sz;
        const int fi = fold(i0 + px - 1, nx, a.g.bc[0], a.g.bc[1], s);
        const int fj = fold(j0 + py - 1, ny, a.g.bc[2], a.g.bc[3], s);
        const size_t g = (size_t)fi + (size_t)nx * ((size_t)fj + (size_t)ny * (size_t)fk);
        T v;
        if constexpr (IN == IN_PLAIN) {
            v = yin[g];
        } else {
            v = prolong_at<T>(a, fi, fj, fk);
            if constexpr (IN == IN_PROLONG_ADD) v += yin[g];
        }
        sx[idx] = (s < 0) ? -v : v;
        if constexpr (HasK<KT>::value) sk[idx] = kload<T, KT>(kp, g);
    }
}

template <typename T>
struct Summ {
    T c, D, X;       // centre, corner sum, cross sum of the field
    T kc, kD, kX;    // same for k
    T pD, pX;        // corner / cross sums of k.x
};

// Plane sums for the two cells (rows 2*ly and 2*ly+1) of this thread.
template <typename T, bool HK>
__device__ __forceinline__ void summarize(const T *sx, const T *sk, int lx, int ly, Summ<T> out[2])
{
    T v[4][3];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) v[rr][cc] = sx[(2 * ly + rr) * PX + lx + cc];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        out[r].c = v[r + 1][1];
        out[r].D = (v[r][0] + v[r][2]) + (v[r + 2][0] + v[r + 2][2]);
        out[r].X = (v[r][1] + v[r + 2][1]) + (v[r + 1][0] + v[r + 1][2]);
    }
    if constexpr (HK) {
        T k[4][3], p[4][3];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                k[rr][cc] = sk[(2 * ly + rr) * PX + lx + cc];
                p[rr][cc] = k[rr][cc] * v[rr][cc];
            }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            out[r].kc = k[r + 1][1];
            out[r].kD = (k[r][0] + k[r][2]) + (k[r + 2][0] + k[r + 2][2]);
            out[r].kX = (k[r][1] + k[r + 2][1]) + (k[r + 1][0] + k[r + 1][2]);
            out[r].pD = (p[r][0] + p[r][2]) + (p[r + 2][0] + p[r + 2][2]);
            out[r].pX = (p[r][1] + p[r + 2][1]) + (p[r + 1][0] + p[r + 1][2]);
        }
    }
}

// A y and the Jacobi diagonal at the centre of (P, C, N) = planes z-1, z, z+1.
template <typename T, bool HK>
__device__ __forceinline__ void apply_op(const Summ<T> &P, const Summ<T> &C, const Summ<T> &N, T h, T &Ay, T &Dg)
{
    if constexpr (!HK) {
        const T w0 = (T)(8.0 / 3.0) * h, we = -h / (T)6, wc = -h / (T)12;
        Ay = w0 * C.c + we * (C.D + P.X + N.X) + wc * (P.D + N.D);
        Dg = w0;
    } else {
        const T ce = h / (T)12, cc = h / (T)24, c4 = (T)(4.0 / 3.0) * h;
        const T Sx = ce * (C.D + P.X + N.X) + cc * (P.D + N.D);
        const T Sk = ce * (C.kD + P.kX + N.kX) + cc * (P.kD + N.kD);
        const T Sp = ce * (C.pD + P.pX + N.pX) + cc * (P.pD + N.pD);
        Dg = c4 * C.kc + Sk;
        Ay = Dg * C.c - C.kc * Sx - Sp;
    }
}

template <typename T, typename KT, int IN, int OUT, typename OT>
__global__ __launch_bounds__(NT) void stencil_kernel(const StencilArgs a)
{
    if (a.done && *a.done) return;
    constexpr bool HK = HasK<KT>::value;
    __shared__ T sx[2][PN];
    __shared__ T sk[2][HK ? PN : 1];
    __shared__ double red[NT / 64];

    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int tile_x = lb % a.t.tiles_x;
    const int rest = lb / a.t.tiles_x;
    const int tile_y = rest % a.t.tiles_y;
    const int cz = rest / a.t.tiles_y;
    const int i0 = tile_x * TX, j0 = tile_y * TY;
    const int z0 = cz * a.t.zc;
    const int z1 = min(z0 + a.t.zc, nz);
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int gi = i0 + lx, gj = j0 + 2 * ly;
    const bool valid[2] = {gi < nx && gj < ny, gi < nx && gj + 1 < ny};
    const T h = (T)a.h, om = (T)a.omega;
    const T *b = (const T *)a.b;
    const size_t plane = (size_t)nx * ny;

    Summ<T> sp[2], sc[2], sn[2];
    load_plane<T, KT, IN>(sx[0], sk[0], a, i0, j0, z0 - 1);
    __syncthreads();
    summarize<T, HK>(sx[0], sk[0], lx, ly, sp);
    load_plane<T, KT, IN>(sx[1], sk[1], a, i0, j0, z0);
    __syncthreads();
    summarize<T, HK>(sx[1], sk[1], lx, ly, sc);

    double nacc = 0.0, zacc = 0.0;
    const double bm = a.bmean ? *a.bmean : 0.0;
    const T bmT = (T)bm;
    int buf = 0;
    for (int z = z0; z < z1; ++z) {
        load_plane<T, KT, IN>(sx[buf], sk[buf], a, i0, j0, z + 1);
        __syncthreads();
        summarize<T, HK>(sx[buf], sk[buf], lx, ly, sn);
        buf ^= 1;
        double rsum = 0.0;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            T Ay, Dg;
            apply_op<T, HK>(sp[r], sc[r], sn[r], h, Ay, Dg);
            const size_t g = (size_t)gi + (size_t)nx * (size_t)(gj + r) + plane * (size_t)z;
            if constexpr (OUT == OUT_RESID) {
                double rv = 0.0;
                if (valid[r]) rv = ((double)b[g] - bm) - (double)Ay;
                if (a.r && valid[r]) ((OT *)a.r)[g] = (OT)rv;
                nacc += rv * rv;
                rsum += rv;
            } else {
                if (valid[r]) {
                    const T y = sc[r].c + om * ((b[g] - bmT) - Ay) / Dg;
                    if constexpr (OUT == OUT_STORE)
                        ((T *)a.yout)[g] = y;
                    else
                        a.x64[g] += (double)y;
                }
            }
        }
        if constexpr (OUT == OUT_RESID) {
            if (a.rc) {
                rsum += __shfl_xor(rsum, 1);
                zacc += rsum;
                if (z & 1) {
                    if (!(lx & 1) && valid[0]) {
                        const int cx = nx >> 1, cy = ny >> 1;
                        ((OT *)a.rc)[(size_t)(gi >> 1) + (size_t)cx * ((size_t)(gj >> 1) + (size_t)cy * (size_t)(z >> 1))] =
                            (OT)zacc;
                    }
                    zacc = 0.0;
                }
            }
        }
        sp[0] = sc[0]; sp[1] = sc[1];
        sc[0] = sn[0]; sc[1] = sn[1];
    }
    if constexpr (OUT == OUT_RESID) {
        if (a.partials) {
            for (int off = 32; off > 0; off >>= 1) nacc += __shfl_down(nacc, off);
            if (lx == 0) red[ly] = nacc;
            __syncthreads();
            if (threadIdx.x == 0) a.partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
        }
    }
}

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

__global__ __launch_bounds__(1024) void finish_norm_kernel(SolveState *st, const double *p, int n)
{
    __shared__ double red[16];
    if (st->done) return;
    const double s = reduce_1024(p, n, red);
    if (threadIdx.x == 0) {
        const double rel = sqrt(s) / st->nb;
        const int idx = st->nres;
        if (idx < 512) st->hist[idx] = rel;
        st->last = rel;
        st->nres = idx + 1;
        if (!isfinite(rel)) {
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
    st->last = 0.0;
    st->fcg_rho = st->fcg_alpha = st->fcg_beta = st->fcg_pq_prev = 0.0;
}

__global__ void set_nb_kernel(SolveState *st, const double *sumsq)
{
    const double nb = sqrt(*sumsq);
    st->nb = nb;
    if (!(nb > 0.0)) {
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

template <typename T, typename KT, int IN, int OUT, typename OT>
hipError_t go(const StencilArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT>), dim3(a.t.blocks()), dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T, typename KT, int OUT, typename OT>
hipError_t go_in(int in_mode, const StencilArgs &a, hipStream_t s)
{
    switch (in_mode) {
    case IN_PLAIN: return go<T, KT, IN_PLAIN, OUT, OT>(a, s);
    case IN_PROLONG: return go<T, KT, IN_PROLONG, OUT, OT>(a, s);
    case IN_PROLONG_ADD: return go<T, KT, IN_PROLONG_ADD, OUT, OT>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

TileShape make_tiles(int nx, int ny, int nz, int zc)
{
    if (zc < 2) zc = 2;
    zc &= ~1;
    TileShape t;
    t.tiles_x = (nx + kTileX - 1) / kTileX;
    t.tiles_y = (ny + kTileY - 1) / kTileY;
    t.zc = zc;
    t.chunks_z = (nz + zc - 1) / zc;
    return t;
}

hipError_t launch_stencil(int T_is_f64, int kt, int in_mode, int out_mode, int out_f32, const StencilArgs &a,
                          hipStream_t s)
{
    if (T_is_f64) {
        if (out_mode == OUT_RESID) {
            if (in_mode != IN_PLAIN) return hipErrorInvalidValue;
            if (kt == KT_NONE)
                return out_f32 ? go<double, NoK, IN_PLAIN, OUT_RESID, float>(a, s)
                               : go<double, NoK, IN_PLAIN, OUT_RESID, double>(a, s);
            if (kt == KT_F64)
                return out_f32 ? go<double, double, IN_PLAIN, OUT_RESID, float>(a, s)
                               : go<double, double, IN_PLAIN, OUT_RESID, double>(a, s);
            return hipErrorInvalidValue;
        }
        if (out_mode == OUT_STORE) {
            if (kt == KT_NONE) return go_in<double, NoK, OUT_STORE, double>(in_mode, a, s);
            if (kt == KT_F64) return go_in<double, double, OUT_STORE, double>(in_mode, a, s);
        }
        if (out_mode == OUT_ADD64) {
            if (kt == KT_NONE) return go_in<double, NoK, OUT_ADD64, double>(in_mode, a, s);
            if (kt == KT_F64) return go_in<double, double, OUT_ADD64, double>(in_mode, a, s);
        }
        return hipErrorInvalidValue;
    }
    if (out_mode == OUT_STORE) {
        if (kt == KT_NONE) return go_in<float, NoK, OUT_STORE, float>(in_mode, a, s);
        if (kt == KT_F32) return go_in<float, float, OUT_STORE, float>(in_mode, a, s);
        if (kt == KT_F16) return go_in<float, __half, OUT_STORE, float>(in_mode, a, s);
    }
    if (out_mode == OUT_ADD64) {
        if (kt == KT_NONE) return go_in<float, NoK, OUT_ADD64, float>(in_mode, a, s);
        if (kt == KT_F32) return go_in<float, float, OUT_ADD64, float>(in_mode, a, s);
        if (kt == KT_F16) return go_in<float, __half, OUT_ADD64, float>(in_mode, a, s);
    }
    return hipErrorInvalidValue;
}

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

hipError_t launch_finish_norm(SolveState *st, const double *partials, int n, hipStream_t s)
{
    hipLaunchKernelGGL(finish_norm_kernel, dim3(1), dim3(1024), 0, s, st, partials, n);
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

}  // namespace nn4mg
