// The z-marching stencil kernel of the multigrid solve (gfx950).
//
// One workgroup of 256 threads owns a TX x TY column of cells (TX in {64, 32,
// 16} cells along x, TY = RY * 256 / TX along y, RY in {2, 4} y-rows per
// thread) and marches a chunk of z-planes.  Per plane:
//   1. a plane prefetched into registers two planes earlier is written to
//      LDS with its one-cell halo ring, and the slot is refilled at once, so
//      two planes of HBM loads stay in flight behind the LDS work.  Halo
//      cells come from the boundary rules of Sec. 2.3.3 of arXiv 2401.06755
//      (Dirichlet -mirror, Neumann +mirror, periodic wrap; the coefficient
//      always +mirror) through addresses and signs computed once per
//      workgroup, so no padded copy exists in HBM;
//   2. each thread forms, for its RY cells, the corner sum D and the cross
//      sum X of the 3x3 neighbourhood in this plane.  The linear-element
//      Laplacian filter has zero face weights and its edge weight is twice
//      its corner weight (-h/6 and -h/12), so with S = 2 D(z) + 2 (X(z-1) +
//      X(z+1)) + D(z-1) + D(z+1),
//          A x = (-h/12) (S[x] - 32 x),
//      and only one running partial sum per cell is kept across planes.  A
//      nodal coefficient k uses the link form of Eq. (k-T),
//          A_k x = (h/24) [ (32 k + S[k]) x - k S[x] - S[k x] ],
//      built from the same plane sums of x, k and k.x, with the Jacobi
//      diagonal (h/24)(32 k + S[k]).
// Input modes: the smoothed field is the input array, or P e_coarse, or the
// input plus P e_coarse (the U-Net decoder's upsample-and-add).  For those the
// coarse correction is interpolated along z while it is prefetched, staged in
// LDS for the tile's footprint, and interpolated in x and y from there
// (separable cell-centred trilinear weights 3/4, 1/4).  Halo cells of P e are
// evaluated at their own position with coarse halos, which equals the fine
// boundary rule applied to P e for all three rules.
// Output modes: a weighted-Jacobi sweep y + omega (b - A y) / D stored, or
// added into an FP64 field; or the residual r = b - A y with the 2x
// restriction (sum of the 8 children) and a per-block sum of r^2.
#include "mg_device.h"
#include "mg_internal.h"

#include <type_traits>

namespace nn4mg {

namespace {

constexpr int NT = 256;

template <int TX, int RY>
struct Tile {
    static constexpr int TYT = NT / TX;  // thread rows
    static constexpr int TY = RY * TYT;  // cell rows (RY per thread)
    static constexpr int PX = TX + 2, PY = TY + 2, PN = PX * PY;
    static constexpr int NPRE = (PN + NT - 1) / NT;
    static constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2, CN = CX * CY;  // coarse footprint
    static constexpr int NPREC = (CN + NT - 1) / NT;
};

// Per-thread, plane-invariant geometry of the staged cells: in-plane offset
// and halo sign of each fine slot, and for the prolongation modes the coarse
// footprint slot plus the four LDS taps of the x-y interpolation.
template <int TX, int RY, bool PRO>
struct Geo {
    int off[Tile<TX, RY>::NPRE];
    bool neg[Tile<TX, RY>::NPRE];
    int coff[PRO ? Tile<TX, RY>::NPREC : 1];
    bool cneg[PRO ? Tile<TX, RY>::NPREC : 1];
    int tap[PRO ? Tile<TX, RY>::NPRE : 1];  // LDS index of the (I, J) tap
    int tdx[PRO ? Tile<TX, RY>::NPRE : 1];  // offset to the x neighbour tap
    int tdy[PRO ? Tile<TX, RY>::NPRE : 1];  // offset to the y neighbour tap
};

template <int TX, int RY, bool PRO>
__device__ __forceinline__ void make_geo(Geo<TX, RY, PRO> &G, const StencilArgs &a, int i0, int j0)
{
    using TL = Tile<TX, RY>;
#pragma unroll
    for (int q = 0; q < TL::NPRE; ++q) {
        const int idx = min((int)threadIdx.x + q * NT, TL::PN - 1);
        const int py = idx / TL::PX;
        const int px = idx - py * TL::PX;
        int s = 1;
        const int fi = fold(i0 + px - 1, a.g.nx, a.g.bc[0], a.g.bc[1], s);
        const int fj = fold(j0 + py - 1, a.g.ny, a.g.bc[2], a.g.bc[3], s);
        G.off[q] = fi + a.g.nx * fj;
        G.neg[q] = s < 0;
        if constexpr (PRO) {
            const int ci0 = (i0 >> 1) - 1, cj0 = (j0 >> 1) - 1;
            const int ui = i0 + px - 1, uj = j0 + py - 1;  // unfolded
            const int I = ui >> 1, J = uj >> 1;
            const int li0 = min(max(I - ci0, 0), TL::CX - 1);
            const int li1 = min(max(I + ((ui & 1) ? 1 : -1) - ci0, 0), TL::CX - 1);
            const int lj0 = min(max(J - cj0, 0), TL::CY - 1);
            const int lj1 = min(max(J + ((uj & 1) ? 1 : -1) - cj0, 0), TL::CY - 1);
            G.tap[q] = lj0 * TL::CX + li0;
            G.tdx[q] = li1 - li0;
            G.tdy[q] = (lj1 - lj0) * TL::CX;
        }
    }
    if constexpr (PRO) {
        const int ci0 = (i0 >> 1) - 1, cj0 = (j0 >> 1) - 1;
#pragma unroll
        for (int q = 0; q < TL::NPREC; ++q) {
            const int idx = min((int)threadIdx.x + q * NT, TL::CN - 1);
            const int cy = idx / TL::CX;
            const int cx = idx - cy * TL::CX;
            int s = 1;
            const int fI = fold(ci0 + cx, a.cnx, a.g.bc[0], a.g.bc[1], s);
            const int fJ = fold(cj0 + cy, a.cny, a.g.bc[2], a.g.bc[3], s);
            G.coff[q] = fI + a.cnx * fJ;
            G.cneg[q] = s < 0;
        }
    }
}

// Registers of one prefetched plane, holding the values exactly as loaded:
// halo signs, the z-interpolation of the coarse correction and coefficient
// conversions are applied when the plane is committed to LDS, so no load
// result is consumed before then and every load of the plane stays in flight.
template <typename T, typename KT, int TX, int RY, bool PRO, bool ADD>
struct Prefetch {
    T x[Tile<TX, RY>::NPRE];
    typename KStore<T, KT>::type k[HasK<KT>::value ? Tile<TX, RY>::NPRE : 1];
    T c1[PRO ? Tile<TX, RY>::NPREC : 1];  // coarse plane nearest to z
    T c2[PRO ? Tile<TX, RY>::NPREC : 1];  // the other coarse plane
    T bo[RY];                 // right-hand side of the output plane one below
    double xo[ADD ? RY : 1];  // FP64 field of that plane (OUT_ADD64)
    bool zneg;                // the plane is a -mirror halo plane
    T wK, wK2;                // z-interpolation weights with halo signs
};

// Issue the loads of fine plane z (field and k), of the two coarse planes of
// its z-interpolation (prolongation modes) and of the output-plane values of
// z - 1.  Every address is in range (slots past the tile repeat the last
// cell; rows past the grid read a clamped row), so the loads need no guards.
// The output-plane values (right-hand side and FP64 field of plane z - 1) are
// a part of their own: the step consumes them after it has issued the next
// plane's field loads, so they are reloaded at the end of the step, into the
// registers just read (see step below).
template <typename T, typename KT, int TX, int RY, bool PRO, bool ADD>
__device__ __forceinline__ void fetch_out(Prefetch<T, KT, TX, RY, PRO, ADD> &p, const StencilArgs &a, int z,
                                          const size_t *gb)
{
    const size_t plane = (size_t)a.g.nx * a.g.ny;
    const T *b = (const T *)a.b;  // NULL: a zero right-hand side
    const size_t pl = plane * (size_t)(z - 1);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        p.bo[r] = b ? b[gb[r] + pl] : (T)0;
        if constexpr (ADD) p.xo[r] = a.x64[gb[r] + pl];
    }
}

template <typename T, typename KT, int IN, int TX, int RY, bool ADD>
__device__ __forceinline__ void fetch_in(Prefetch<T, KT, TX, RY, IN != IN_PLAIN, ADD> &p,
                                         const Geo<TX, RY, IN != IN_PLAIN> &G, const StencilArgs &a, int z)
{
    using TL = Tile<TX, RY>;
    const size_t plane = (size_t)a.g.nx * a.g.ny;
    int sz = 1;
    const int fk = fold(z, a.g.nz, a.g.bc[4], a.g.bc[5], sz);
    p.zneg = sz < 0;
    const size_t pz = plane * (size_t)fk;
    const T *yin = (const T *)a.yin;
    const KT *kp = (const KT *)a.k;
#pragma unroll
    for (int q = 0; q < TL::NPRE; ++q) {
        const size_t g = pz + (size_t)G.off[q];
        if constexpr (IN != IN_PROLONG) p.x[q] = yin[g];
        if constexpr (HasK<KT>::value) p.k[q] = kp[g];
    }
    if constexpr (IN != IN_PLAIN) {
        const T *e = (const T *)a.ec;
        const int K = z >> 1;
        int sK = 1, sK2 = 1;
        const int fK = fold(K, a.cnz, a.g.bc[4], a.g.bc[5], sK);
        const int fK2 = fold(K + ((z & 1) ? 1 : -1), a.cnz, a.g.bc[4], a.g.bc[5], sK2);
        p.wK = (T)(0.75 * sK);
        p.wK2 = (T)(0.25 * sK2);
        const size_t cpl = (size_t)a.cnx * a.cny;
        const size_t p1 = cpl * (size_t)fK, p2 = cpl * (size_t)fK2;
#pragma unroll
        for (int q = 0; q < TL::NPREC; ++q) {
            const size_t g = (size_t)G.coff[q];
            p.c1[q] = e[g + p1];
            p.c2[q] = e[g + p2];
        }
    }
}

template <typename T, typename KT, int IN, int TX, int RY, bool ADD>
__device__ __forceinline__ void fetch(Prefetch<T, KT, TX, RY, IN != IN_PLAIN, ADD> &p,
                                      const Geo<TX, RY, IN != IN_PLAIN> &G, const StencilArgs &a, int z, int z0,
                                      const size_t *gb)
{
    if (z - 1 >= z0) fetch_out<T, KT, TX, RY, IN != IN_PLAIN, ADD>(p, a, z, gb);
    fetch_in<T, KT, IN, TX, RY, ADD>(p, G, a, z);
}

// Write a prefetched plane to LDS (forming x + P e for the prolongation modes).
template <typename T, typename KT, int IN, int TX, int RY, bool ADD>
__device__ __forceinline__ void commit(const Prefetch<T, KT, TX, RY, IN != IN_PLAIN, ADD> &p,
                                       const Geo<TX, RY, IN != IN_PLAIN> &G, T *sx, T *sk, T *scoarse)
{
    using TL = Tile<TX, RY>;
    constexpr bool HK = HasK<KT>::value;
    if constexpr (IN != IN_PLAIN) {
#pragma unroll
        for (int q = 0; q < TL::NPREC; ++q)
            if (q * NT + (int)threadIdx.x < TL::CN) {
                const T v = p.wK * p.c1[q] + p.wK2 * p.c2[q];
                scoarse[q * NT + threadIdx.x] = G.cneg[q] ? -v : v;
            }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < TL::NPRE; ++q) {
        const int idx = q * NT + threadIdx.x;
        if (idx < TL::PN) {
            if constexpr (IN == IN_PLAIN) {
                sx[idx] = (G.neg[q] != p.zneg) ? -p.x[q] : p.x[q];
            } else {
                const T w3 = (T)0.75, w1 = (T)0.25;
                const int t0 = G.tap[q], t1 = t0 + G.tdy[q];
                T v = w3 * (w3 * scoarse[t0] + w1 * scoarse[t0 + G.tdx[q]]) +
                      w1 * (w3 * scoarse[t1] + w1 * scoarse[t1 + G.tdx[q]]);
                if constexpr (IN == IN_PROLONG_ADD) v += (G.neg[q] != p.zneg) ? -p.x[q] : p.x[q];
                sx[idx] = v;
            }
            if constexpr (HK) sk[idx] = kconv<T, KT>(p.k[q]);
        }
    }
    __syncthreads();
}

// Per plane and cell: a = 2 D (own plane) and o = 2 X + D (neighbour planes)
// for the field, k and k.x.
template <typename T>
struct PlaneSums {
    T xc, xa, xo;
    T kc, ka, ko;
    T pa, po;
};

template <typename T, bool HK, int TX, int RY>
__device__ __forceinline__ void plane_sums(const T *sx, const T *sk, int lx, int ly, PlaneSums<T> out[RY])
{
    using TL = Tile<TX, RY>;
    const int base = RY * ly * TL::PX + lx;
    T v[RY + 2][3];
#pragma unroll
    for (int rr = 0; rr < RY + 2; ++rr)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) v[rr][cc] = sx[base + rr * TL::PX + cc];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const T D = (v[r][0] + v[r][2]) + (v[r + 2][0] + v[r + 2][2]);
        const T X = (v[r][1] + v[r + 2][1]) + (v[r + 1][0] + v[r + 1][2]);
        out[r].xc = v[r + 1][1];
        out[r].xa = D + D;
        out[r].xo = fma((T)2, X, D);
    }
    if constexpr (HK) {
        T k[RY + 2][3], p[RY + 2][3];
#pragma unroll
        for (int rr = 0; rr < RY + 2; ++rr)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                k[rr][cc] = sk[base + rr * TL::PX + cc];
                p[rr][cc] = k[rr][cc] * v[rr][cc];
            }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const T Dk = (k[r][0] + k[r][2]) + (k[r + 2][0] + k[r + 2][2]);
            const T Xk = (k[r][1] + k[r + 2][1]) + (k[r + 1][0] + k[r + 1][2]);
            const T Dp = (p[r][0] + p[r][2]) + (p[r + 2][0] + p[r + 2][2]);
            const T Xp = (p[r][1] + p[r + 2][1]) + (p[r + 1][0] + p[r + 1][2]);
            out[r].kc = k[r + 1][1];
            out[r].ka = Dk + Dk;
            out[r].ko = fma((T)2, Xk, Dk);
            out[r].pa = Dp + Dp;
            out[r].po = fma((T)2, Xp, Dp);
        }
    }
}

// Running partial sums of one cell across planes: q = a(z) + o(z-1) waits for
// o(z+1); o is the newest plane's neighbour contribution.
template <typename T>
struct Run {
    T qx, ox, qk, ok, qp, op, xc, kc;
};

#ifndef NN4MG_MIN_WAVES
#define NN4MG_MIN_WAVES 1
#endif

template <typename T, typename KT, int IN, int OUT, typename OT, int TX, int RY>
__global__ __launch_bounds__(NT, NN4MG_MIN_WAVES) void stencil_kernel(const StencilArgs a_)
{
    StencilArgs a = a_;
    const int lb = enter_copy(a, xcd_remap(blockIdx.x, gridDim.x));
    if (a.done && *a.done) return;
    using TL = Tile<TX, RY>;
    constexpr bool HK = HasK<KT>::value;
    constexpr bool PRO = IN != IN_PLAIN;
    constexpr bool ADD = OUT == OUT_ADD64;
    constexpr int RP = RY / 2;  // restriction row pairs per thread
    __shared__ T sx[2][TL::PN];
    __shared__ T sk[2][HK ? TL::PN : 1];
    __shared__ T sc[PRO ? TL::CN : 1];
    __shared__ double red[NT / 64];

    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int tile_x = lb % a.t.tiles_x;
    const int rest = lb / a.t.tiles_x;
    const int tile_y = rest % a.t.tiles_y;
    const int cz = rest / a.t.tiles_y;
    const int i0 = tile_x * TX, j0 = tile_y * TL::TY;
    const int z0 = cz * a.t.zc;
    const int z1 = min(z0 + a.t.zc, nz);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int gi = i0 + lx, gj = j0 + RY * ly;
    bool valid[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) valid[r] = gi < nx && gj + r < ny;
    const size_t plane = (size_t)nx * ny;
    const size_t g0 = (size_t)gi + (size_t)nx * (size_t)gj;  // (gi, gj, 0); row r adds r * nx
    size_t gb[RY];  // load offsets of the thread's rows, clamped into the grid
#pragma unroll
    for (int r = 0; r < RY; ++r) gb[r] = (size_t)min(gi, nx - 1) + (size_t)nx * (size_t)min(gj + r, ny - 1);

    // Scaled filter constants: constant coefficient A y = cw (S - 32 y) with
    // cw = -h/12; nodal A y = cv [(32 k + S[k]) y - k S[y] - S[k y]], cv = h/24.
    const T h = (T)a.h, om = (T)a.omega;
    const T cw = -h / (T)12, cv = h / (T)24;
    const T om_w0 = om / ((T)(8.0 / 3.0) * h);  // omega / (8h/3)
    const T icv = (T)1 / cv;
    const double bm = a.bmean ? *a.bmean : 0.0;
    const T bmT = (T)bm;

    Geo<TX, RY, PRO> G;
    make_geo<TX, RY, PRO>(G, a, i0, j0);
    Prefetch<T, KT, TX, RY, PRO, ADD> pA, pB;
    PlaneSums<T> ps[RY];
    Run<T> run[RY];

    auto absorb = [&](bool first) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            run[r].qx = first ? ps[r].xa : ps[r].xa + run[r].ox;
            run[r].ox = ps[r].xo;
            run[r].xc = ps[r].xc;
            if constexpr (HK) {
                run[r].qk = first ? ps[r].ka : ps[r].ka + run[r].ok;
                run[r].qp = first ? ps[r].pa : ps[r].pa + run[r].op;
                run[r].ok = ps[r].ko;
                run[r].op = ps[r].po;
                run[r].kc = ps[r].kc;
            }
        }
    };

    double nacc = 0.0, zacc[RP > 0 ? RP : 1];
#pragma unroll
    for (int q = 0; q < RP; ++q) zacc[q] = 0.0;

    // One output plane: commit plane z + 1 from slot p, refill the slot with
    // plane z + 3 (two planes stay in flight), then finish plane z and load
    // the output values of plane z + 2 into the registers it just read.
    // The steady form (ST; PAR = z & 1 known) runs on tiles inside the grid
    // with the restricted residual output present (mode 1: and the full
    // residual, mode 2: without it): it issues the same loads and stores on
    // every path, so the compiler's wait counts keep the next planes' loads in
    // flight instead of waiting for every outstanding load.
    int buf = 0;
    auto step = [&](auto st_tag, auto par_tag, Prefetch<T, KT, TX, RY, PRO, ADD> &p, int z) {
        constexpr int MODE = decltype(st_tag)::value;
        constexpr bool ST = MODE != 0;
        constexpr int PAR = decltype(par_tag)::value;
        commit<T, KT, IN, TX, RY, ADD>(p, G, sx[buf], sk[buf], sc);
        if (ST || z + 3 <= z1) fetch_in<T, KT, IN, TX, RY, ADD>(p, G, a, z + 3);
        plane_sums<T, HK, TX, RY>(sx[buf], sk[buf], lx, ly, ps);
        buf ^= 1;
        double rrow[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const size_t g = g0 + (size_t)r * nx + plane * (size_t)z;
            const T y0 = run[r].xc;
            const T bb = p.bo[r] - bmT;
            T y = (T)0, Ay = (T)0;
            if constexpr (!HK) {
                const T S = run[r].qx + ps[r].xo;
                if constexpr (OUT == OUT_RESID)
                    Ay = cw * (S - (T)32 * y0);
                else
                    y = y0 + om_w0 * (bb - cw * (S - (T)32 * y0));
            } else {
                const T Sx = run[r].qx + ps[r].xo;
                const T Sk = run[r].qk + ps[r].ko;
                const T Sp = run[r].qp + ps[r].po;
                const T Dg = fma((T)32, run[r].kc, Sk);
                const T Ays = Dg * y0 - run[r].kc * Sx - Sp;  // A y / cv
                if constexpr (OUT == OUT_RESID)
                    Ay = cv * Ays;
                else
                    y = y0 + om * (bb * icv - Ays) * recip(Dg);
            }
            rrow[r] = 0.0;
            if constexpr (OUT == OUT_RESID) {
                double rv = 0.0;
                if (ST || valid[r]) rv = ((double)p.bo[r] - bm) - (double)Ay;
                if (MODE == 1 || (MODE == 0 && a.r && valid[r])) ((OT *)a.r)[g] = (OT)rv;
                nacc += a.dot_x ? (double)y0 * rv : rv * rv;
                rrow[r] = rv;
            } else if (ST || valid[r]) {
                if constexpr (OUT == OUT_STORE)
                    ((T *)a.yout)[g] = y;
                else
                    a.x64[g] = p.xo[r] + (double)y;
            }
        }
        absorb(false);
        if constexpr (OUT == OUT_RESID) {
            if (ST || a.rc) {
                const int cx = nx >> 1, cy = ny >> 1;
#pragma unroll
                for (int q = 0; q < RP; ++q) {
                    double rs = rrow[2 * q] + rrow[2 * q + 1];
                    rs += __shfl_xor(rs, 1);
                    zacc[q] += rs;
                    if (ST ? (PAR == 1) : (z & 1)) {
                        // both lanes of an x pair hold the same sum: in the steady form
                        // both store it (one store instruction on every path)
                        if (ST || (!(lx & 1) && valid[2 * q]))
                            ((OT *)a.rc)[(size_t)(gi >> 1) +
                                         (size_t)cx * ((size_t)((gj >> 1) + q) + (size_t)cy * (size_t)(z >> 1))] =
                                (OT)zacc[q];
                        zacc[q] = 0.0;
                    }
                }
            }
        }
        // output values of plane z + 2 (its step comes two steps later)
        if (ST || z + 3 <= z1) fetch_out<T, KT, TX, RY, PRO, ADD>(p, a, z + 3, gb);
    };

    // prologue: planes z0 - 1 and z0 into the running sums; planes z0 + 1 and
    // z0 + 2 (with the right-hand sides of planes z0 and z0 + 1) in flight
    fetch<T, KT, IN, TX, RY, ADD>(pA, G, a, z0 - 1, z0, gb);
    commit<T, KT, IN, TX, RY, ADD>(pA, G, sx[0], sk[0], sc);
    fetch<T, KT, IN, TX, RY, ADD>(pA, G, a, z0, z0, gb);
    plane_sums<T, HK, TX, RY>(sx[0], sk[0], lx, ly, ps);
    absorb(true);
    commit<T, KT, IN, TX, RY, ADD>(pA, G, sx[1], sk[1], sc);
    fetch<T, KT, IN, TX, RY, ADD>(pA, G, a, z0 + 1, z0, gb);
    // plane z0 + 2 is fetched even when the chunk is shorter (its values are
    // then unused; fold keeps the field plane in range and the output plane
    // is clamped into the chunk), so that every path into the march below
    // has the same loads in flight
    fetch_out<T, KT, TX, RY, PRO, ADD>(pB, a, min(z0 + 2, z1), gb);
    fetch_in<T, KT, IN, TX, RY, ADD>(pB, G, a, z0 + 2);
    plane_sums<T, HK, TX, RY>(sx[1], sk[1], lx, ly, ps);
    absorb(false);

    const std::integral_constant<int, 0> gen{};
    const std::integral_constant<int, 1> steady{};
    const std::integral_constant<int, 2> steady_rc{};
    const std::integral_constant<int, -1> anypar{};
    const std::integral_constant<int, 0> even{};
    const std::integral_constant<int, 1> odd{};
    // the steady march: tiles inside the grid, chunks starting on an even plane
    // (so the A steps are the even planes), the restricted residual output
    // present (the full residual is optional: its own form of the march)
    const bool inside = i0 + TX <= nx && j0 + TL::TY <= ny && !(z0 & 1) && (OUT != OUT_RESID || a.rc != nullptr);
    int z = z0;
    if (OUT != OUT_RESID || a.r != nullptr) {
        for (; inside && z + 4 <= z1; z += 2) {
            step(steady, even, pA, z);
            step(steady, odd, pB, z + 1);
        }
    } else {
        if constexpr (OUT == OUT_RESID) {
            for (; inside && z + 4 <= z1; z += 2) {
                step(steady_rc, even, pA, z);
                step(steady_rc, odd, pB, z + 1);
            }
        }
    }
    for (; z < z1; z += 2) {
        step(gen, anypar, pA, z);
        if (z + 1 < z1) step(gen, anypar, pB, z + 1);
    }

    if constexpr (OUT == OUT_RESID) {
        if (a.partials) {
            for (int off = 32; off > 0; off >>= 1) nacc += __shfl_down(nacc, off);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nacc;
            __syncthreads();
            // slot = the tile's index within its copy, so a batched launch
            // sums each copy's partials in the order of a single launch
            if (threadIdx.x == 0) a.partials[lb] = (red[0] + red[1]) + (red[2] + red[3]);
        }
    }
}

template <typename T, typename KT, int IN, int OUT, typename OT>
hipError_t go(const StencilArgs &a_, hipStream_t s)
{
    StencilArgs a = a_;
    const dim3 grid(batched_grid(a, a.t.blocks())), block(NT);
    const int key = a.t.tx * 10 + a.t.ry;
    if constexpr (OUT != OUT_RESID) {  // one row per thread: sweeps only (the restriction pairs rows)
        switch (key) {
        case 641: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 64, 1>), grid, block, 0, s, a); return hipGetLastError();
        case 321: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 32, 1>), grid, block, 0, s, a); return hipGetLastError();
        case 161: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 16, 1>), grid, block, 0, s, a); return hipGetLastError();
        default: break;
        }
    }
    switch (key) {
    case 642: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 64, 2>), grid, block, 0, s, a); break;
    case 644: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 64, 4>), grid, block, 0, s, a); break;
    case 322: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 32, 2>), grid, block, 0, s, a); break;
    case 324: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 32, 4>), grid, block, 0, s, a); break;
    case 162: hipLaunchKernelGGL((stencil_kernel<T, KT, IN, OUT, OT, 16, 2>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
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

TileShape make_tiles(int nx, int ny, int nz, int zc, int tx, int ry)
{
    if (tx != 64 && tx != 32 && tx != 16) tx = 64;
    if (ry != 1 && ry != 2 && ry != 4) ry = 2;
    if (tx == 16 && ry == 4) ry = 2;
    if (zc < 2) zc = 2;
    zc &= ~1;
    TileShape t;
    t.tx = tx;
    t.ry = ry;
    const int ty = (256 / tx) * ry;
    t.tiles_x = (nx + tx - 1) / tx;
    t.tiles_y = (ny + ty - 1) / ty;
    t.zc = zc;
    t.chunks_z = (nz + zc - 1) / zc;
    return t;
}

hipError_t launch_stencil(int T_is_f64, int kt, int in_mode, int out_mode, int out_f32, const StencilArgs &a,
                          hipStream_t s)
{
    if (a.t.blocks() <= 0) return hipErrorInvalidValue;
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

}  // namespace nn4mg
