// Both post-smoothing sweeps of a level in one z-marching pass (gfx950).
//
// The sawtooth cycle of Fig. multi-grid (arXiv 2401.06755, Sec. 2.4) ends
// each level with the prolongation of the coarser correction and nu_post = 2
// weighted-Jacobi sweeps.  Run as two kernels, the second sweep re-reads from
// HBM the first one's output, the right-hand side and the coefficient.  Here
// one workgroup keeps both sweeps in flight, one plane apart:
//   * the first sweep is computed on the workgroup's TX x TY output tile plus
//     a one-cell ring (the second sweep's stencil reaches one cell out), from
//     input planes staged in LDS with a two-cell ring;
//   * its output plane goes to LDS and feeds the second sweep, whose running
//     plane sums lag one plane behind.
// Ring cells that lie outside the grid are computed like any other cell from
// halo-synthesised inputs: the sweep commutes with the boundary reflections
// (Dirichlet -mirror, Neumann +mirror, periodic wrap), so they hold the halo
// values of the first sweep's output.
// The input of the first sweep is the prolongated correction P e of the
// coarser level, so the pair computes the correction of this level for the
// right-hand side b: with b = r = b - A x and x += e this is exactly
// x <- S S (x + P e), since the Jacobi sweep is affine.  Output: the
// correction stored (coarse levels, preconditioner z) or added into an FP64
// field (mixed precision at the finest level).  In the XIN form (FP64 finest
// level) the input is x + P e itself, x staged with the same two-cell ring,
// against b - mean(b), and the new iterate is stored into a second buffer:
// the finest residual kernel then has no full residual to write.
// Each thread of the first sweep walks a vertical strip of cells and the
// second sweep its RY output rows: every row of the 3-wide neighbourhood is
// read from LDS once and reduced to the pair sum of its side cells and its
// centre, which the two or three cells of the strip that reach it share.
// Operator and sweep are those of the single-sweep kernel: with the plane
// sums D (corners) and X (crosses) of the 3x3 neighbourhood,
//   S = 2 D(z) + 2 (X(z-1) + X(z+1)) + D(z-1) + D(z+1),
//   constant coefficient  A y = (-h/12) (S[y] - 32 y),
//   nodal coefficient     A_k y = (h/24) [(32 k + S[k]) y - k S[y] - S[k y]] (Eq. k-T).
#include "mg_device.h"
#include "mg_internal.h"

#include <type_traits>

namespace nn4mg {

namespace {

constexpr int FT = 256;

// Smallest strip height whose strips over a QX x QY region fit one per thread.
constexpr int strip_rows(int qx, int qy)
{
    int r = 1;
    while (((qy + r - 1) / r) * qx > FT) ++r;
    return r;
}

template <int TX, int RY>
struct FTile {
    static constexpr int TYT = FT / TX;                             // thread rows
    static constexpr int TY = RY * TYT;                             // output rows
    static constexpr int QX = TX + 2, QY = TY + 2, QN = QX * QY;    // first-sweep region
    static constexpr int PX = TX + 4, PY = TY + 4, PN = PX * PY;    // input region
    static constexpr int NPRE = (PN + FT - 1) / FT;                 // input slots per thread
    // first sweep: one vertical strip of R1 cells per thread, NST strips per column
    static constexpr int R1 = strip_rows(QX, QY);
    static constexpr int NST = (QY + R1 - 1) / R1;
    static constexpr int NT1 = NST * QX;                            // threads with a strip
    static constexpr int CX = TX / 2 + 4, CY = TY / 2 + 4, CN = CX * CY;  // coarse footprint
    static constexpr int NPREC = (CN + FT - 1) / FT;
};

// Plane-invariant geometry of a thread's slots.
template <int TX, int RY>
struct FGeo {
    using TL = FTile<TX, RY>;
    int off[TL::NPRE];    // folded in-plane offset of each input slot (coefficient, fine field)
    bool xneg[TL::NPRE];  // the fine field's halo sign of each input slot
    int tap[TL::NPRE];    // prolongation: LDS tap | x-neighbour bit << 16 | y-neighbour bit << 17
    int coff[TL::NPREC];  // folded in-plane offset of each coarse slot
    bool cneg[TL::NPREC];
    int boff[TL::R1];     // folded in-plane offset of each first-sweep strip cell (right-hand side)
    bool bneg[TL::R1];
};

template <int TX, int RY>
__device__ __forceinline__ void make_fgeo(FGeo<TX, RY> &G, const StencilArgs &a, int i0, int j0)
{
    using TL = FTile<TX, RY>;
    const int ci0 = (i0 >> 1) - 2, cj0 = (j0 >> 1) - 2;
#pragma unroll
    for (int q = 0; q < TL::NPRE; ++q) {
        const int idx = min((int)threadIdx.x + q * FT, TL::PN - 1);
        const int py = idx / TL::PX, px = idx - py * TL::PX;
        const int ui = i0 + px - 2, uj = j0 + py - 2;  // unfolded fine position
        int s = 1;
        G.off[q] = fold(ui, a.g.nx, a.g.bc[0], a.g.bc[1], s) + a.g.nx * fold(uj, a.g.ny, a.g.bc[2], a.g.bc[3], s);
        G.xneg[q] = s < 0;
        const int I = ui >> 1, J = uj >> 1;  // floor
        const int t0 = (J - cj0) * TL::CX + (I - ci0);
        G.tap[q] = t0 | ((ui & 1) << 16) | ((uj & 1) << 17);
    }
#pragma unroll
    for (int q = 0; q < TL::NPREC; ++q) {
        const int idx = min((int)threadIdx.x + q * FT, TL::CN - 1);
        const int cy = idx / TL::CX, cx = idx - cy * TL::CX;
        int s = 1;
        const int fI = fold(ci0 + cx, a.cnx, a.g.bc[0], a.g.bc[1], s);
        const int fJ = fold(cj0 + cy, a.cny, a.g.bc[2], a.g.bc[3], s);
        G.coff[q] = fI + a.cnx * fJ;
        G.cneg[q] = s < 0;
    }
    const int t1 = min((int)threadIdx.x, TL::NT1 - 1);
    const int sq = t1 / TL::QX, qx = t1 - sq * TL::QX;
#pragma unroll
    for (int q = 0; q < TL::R1; ++q) {
        const int qy = min(sq * TL::R1 + q, TL::QY - 1);  // rows past the region: any valid cell
        int s = 1;
        const int fi = fold(i0 + qx - 1, a.g.nx, a.g.bc[0], a.g.bc[1], s);
        const int fj = fold(j0 + qy - 1, a.g.ny, a.g.bc[2], a.g.bc[3], s);
        G.boff[q] = fi + a.g.nx * fj;
        G.bneg[q] = s < 0;
    }
}

// Loads of one input plane zi, as loaded (signs and weights applied later):
// coefficient, coarse correction (and fine field, XIN) of plane zi,
// first-sweep right-hand side of plane zi - 1 and (ADD) the FP64 field of
// zi - 2.  The second sweep takes its right-hand side from LDS, where the
// first sweep left it one plane earlier.
template <typename T, typename KT, int TX, int RY, bool ADD, bool XIN>
struct FPre {
    using TL = FTile<TX, RY>;
    typename KStore<T, KT>::type k[HasK<KT>::value ? TL::NPRE : 1];
    T xs[XIN ? TL::NPRE : 1];
    T c1[TL::NPREC], c2[TL::NPREC];
    T b1[TL::R1];
    double xo[ADD ? RY : 1];
};

template <typename T>
struct PS {
    T xc, xa, xo, kc, ka, ko, pa, po;
};

template <typename T>
struct Run {
    T qx, ox, qk, ok, qp, op, xc, kc;
};

// One row of a 3-wide neighbourhood: the pair sum of its two side cells and
// its centre, for the field v, the coefficient k and the product k v.
template <typename T>
struct Row {
    T h, m, kh, km, ph, pm;
};

template <typename T, bool HK>
__device__ __forceinline__ Row<T> row_at(const T *v, int c, const T *k, int ck)
{
    Row<T> o;
    const T vl = v[c - 1], vm = v[c], vr = v[c + 1];
    o.h = vl + vr;
    o.m = vm;
    if constexpr (HK) {
        const T kl = k[ck - 1], km = k[ck], kr = k[ck + 1];
        o.kh = kl + kr;
        o.km = km;
        o.ph = kl * vl + kr * vr;
        o.pm = km * vm;
    }
    return o;
}

// Plane sums of the centre row b of three consecutive rows a, b, c.
template <typename T, bool HK>
__device__ __forceinline__ PS<T> col_sums(const Row<T> &a, const Row<T> &b, const Row<T> &c)
{
    PS<T> o;
    const T D = a.h + c.h;
    const T X = (a.m + c.m) + b.h;
    o.xc = b.m;
    o.xa = D + D;
    o.xo = fma((T)2, X, D);
    if constexpr (HK) {
        const T Dk = a.kh + c.kh;
        const T Xk = (a.km + c.km) + b.kh;
        const T Dp = a.ph + c.ph;
        const T Xp = (a.pm + c.pm) + b.ph;
        o.kc = b.km;
        o.ka = Dk + Dk;
        o.ko = fma((T)2, Xk, Dk);
        o.pa = Dp + Dp;
        o.po = fma((T)2, Xp, Dp);
    }
    return o;
}

template <typename T, bool HK>
__device__ __forceinline__ void absorb(Run<T> &r, const PS<T> &p, bool first)
{
    r.qx = first ? p.xa : p.xa + r.ox;
    r.ox = p.xo;
    r.xc = p.xc;
    if constexpr (HK) {
        r.qk = first ? p.ka : p.ka + r.ok;
        r.qp = first ? p.pa : p.pa + r.op;
        r.ok = p.ko;
        r.op = p.po;
        r.kc = p.kc;
    }
}

// One Jacobi update of the cell whose plane sums complete with plane p.
template <typename T, bool HK>
__device__ __forceinline__ T jacobi(const Run<T> &r, const PS<T> &p, T bb, T cw, T om_w0, T om, T icv)
{
    const T y0 = r.xc;
    if constexpr (!HK) {
        const T S = r.qx + p.xo;
        return y0 + om_w0 * (bb - cw * (S - (T)32 * y0));
    } else {
        const T Sx = r.qx + p.xo, Sk = r.qk + p.ko, Sp = r.qp + p.po;
        const T Dg = fma((T)32, r.kc, Sk);
        const T Ays = Dg * y0 - r.kc * Sx - Sp;
        return y0 + om * (bb * icv - Ays) * recip(Dg);
    }
}

// XIN: the first sweep's input is x + P e (x = a.yin, the right-hand side
// b - bmean, output stored into a.yout, which must not alias a.yin).
template <typename T, typename KT, int OUT, bool XIN, int TX, int RY>
__global__ __launch_bounds__(FT) __attribute__((amdgpu_waves_per_eu(2))) void sweep2_kernel(const StencilArgs a_)
{
    StencilArgs a = a_;
    const int lb = enter_copy(a, xcd_remap(blockIdx.x, gridDim.x));
    if (a.done && *a.done) return;
    using TL = FTile<TX, RY>;
    constexpr bool HK = HasK<KT>::value;
    constexpr bool ADD = OUT == OUT_ADD64;
    static_assert(!(XIN && ADD), "the x + P e input form stores its result");
    __shared__ T sx[3][TL::PN];            // input planes (P e), three in rotation
    __shared__ T sk[3][HK ? TL::PN : 1];   // coefficient planes
    __shared__ T sy[2][TL::QN];            // first-sweep output planes
    __shared__ T sb[2][TL::QN];            // first-sweep right-hand sides (signed), same planes
    __shared__ T sc[2][TL::CN];            // coarse footprint of the next plane to commit (by plane parity)

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
    size_t gb[RY];  // in-plane offsets of the thread's output rows, clamped into the grid
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        valid[r] = gi < nx && gj + r < ny;
        gb[r] = (size_t)min(gi, nx - 1) + (size_t)nx * (size_t)min(gj + r, ny - 1);
    }
    const size_t plane = (size_t)nx * ny;
    const size_t cplane = (size_t)a.cnx * a.cny;

    const T h = (T)a.h, om = (T)a.omega;
    const T cw = -h / (T)12, cv = h / (T)24;
    const T om_w0 = om / ((T)(8.0 / 3.0) * h);
    const T icv = (T)1 / cv;

    FGeo<TX, RY> G;
    make_fgeo<TX, RY>(G, a, i0, j0);
    FPre<T, KT, TX, RY, ADD, XIN> pA, pB;
    Run<T> r1[TL::R1], r2[RY];
    const bool act1 = (int)threadIdx.x < TL::NT1;
    const int s1q = min((int)threadIdx.x, TL::NT1 - 1) / TL::QX;   // strip of this thread
    const int s1x = min((int)threadIdx.x, TL::NT1 - 1) - s1q * TL::QX;

    const T *bp = (const T *)a.b;
    const T *ep = (const T *)a.ec;
    const KT *kp = (const KT *)a.k;
    const T *xp = (const T *)a.yin;
    const T bm = (XIN && a.bmean) ? (T)*a.bmean : (T)0;

    // Loads of plane zi in two parts.  The coefficient and the coarse values
    // are consumed by the LDS commit at the start of the step that uses them,
    // so the next plane's loads can reuse their registers right after it; the
    // right-hand sides (and the FP64 field) are consumed by the sweeps, so
    // they are reloaded at the end of the step.  Either way no register still
    // holding a load in flight is copied at the loop's back edge (a copy would
    // wait for every outstanding load and undo the two-plane prefetch).
    // (coarse values first: they are staged one step before the rest)
    auto fetch_kc = [&](FPre<T, KT, TX, RY, ADD, XIN> &p, int zi) {
        const int K = zi >> 1;
        int s1 = 1, s2 = 1;
        const size_t p1 = cplane * (size_t)fold(K, a.cnz, a.g.bc[4], a.g.bc[5], s1);
        const size_t p2 = cplane * (size_t)fold(K + ((zi & 1) ? 1 : -1), a.cnz, a.g.bc[4], a.g.bc[5], s2);
#pragma unroll
        for (int q = 0; q < TL::NPREC; ++q) {
            p.c1[q] = ep[p1 + (size_t)G.coff[q]];
            p.c2[q] = ep[p2 + (size_t)G.coff[q]];
        }
        int sk_ = 1;
        const size_t pz = plane * (size_t)fold(zi, nz, a.g.bc[4], a.g.bc[5], sk_);
        if constexpr (HK) {
#pragma unroll
            for (int q = 0; q < TL::NPRE; ++q) p.k[q] = kp[pz + (size_t)G.off[q]];
        }
        if constexpr (XIN) {
#pragma unroll
            for (int q = 0; q < TL::NPRE; ++q) p.xs[q] = xp[pz + (size_t)G.off[q]];
        }
    };
    // MODE 0: general (every load conditional on the planes of the chunk);
    // 1 (steady) and 2 (the first steps when the steady march follows): the
    // loads are issued unconditionally, mode 2 clamping the planes into the
    // chunk (values it loads for planes without an output are never used).
    auto fetch_b = [&](auto mode_tag, FPre<T, KT, TX, RY, ADD, XIN> &p, int zi) {
        constexpr int MODE = decltype(mode_tag)::value;
        if (MODE != 0 || (zi - 1 >= z0 - 1 && zi - 1 <= z1)) {
            const int zb = MODE == 2 ? min(max(zi - 1, z0 - 1), z1) : zi - 1;
            int sb = 1;
            const size_t pb = plane * (size_t)fold(zb, nz, a.g.bc[4], a.g.bc[5], sb);
#pragma unroll
            for (int q = 0; q < TL::R1; ++q) p.b1[q] = bp[pb + (size_t)G.boff[q]];
        }
        if constexpr (ADD) {
            if (MODE != 0 || (zi - 2 >= z0 && zi - 2 < z1)) {
                const int zo = MODE == 2 ? min(max(zi - 2, z0), z1 - 1) : zi - 2;
                const size_t pl = plane * (size_t)zo;
#pragma unroll
                for (int r = 0; r < RY; ++r) p.xo[r] = a.x64[pl + gb[r]];
            }
        }
    };
    auto fetch = [&](FPre<T, KT, TX, RY, ADD, XIN> &p, int zi) {
        fetch_kc(p, zi);
        fetch_b(std::integral_constant<int, 0>{}, p, zi);
    };

    // The coarse footprint of plane zi, interpolated in z, into sc[zi & 1].
    // Staged one step ahead (before the barrier that precedes the second
    // sweep), so the commit needs no barrier of its own before reading it.
    auto stage_c = [&](const FPre<T, KT, TX, RY, ADD, XIN> &p, int zi) {
        const int K = zi >> 1;
        int s1 = 1, s2 = 1;
        (void)fold(K, a.cnz, a.g.bc[4], a.g.bc[5], s1);
        (void)fold(K + ((zi & 1) ? 1 : -1), a.cnz, a.g.bc[4], a.g.bc[5], s2);
        const T w1 = (T)(0.75 * s1), w2 = (T)(0.25 * s2);
#pragma unroll
        for (int q = 0; q < TL::NPREC; ++q)
            if (q * FT + (int)threadIdx.x < TL::CN) {
                const T v = w1 * p.c1[q] + w2 * p.c2[q];
                sc[zi & 1][q * FT + threadIdx.x] = G.cneg[q] ? -v : v;
            }
    };

    // P e (plus x, XIN) of plane zi into sx[buf] from its staged coarse
    // footprint, the coefficient into sk[buf].
    auto commit = [&](const FPre<T, KT, TX, RY, ADD, XIN> &p, int zi, int buf) {
        int sz = 1;
        if constexpr (XIN) (void)fold(zi, nz, a.g.bc[4], a.g.bc[5], sz);
        const T *scp = sc[zi & 1];
#pragma unroll
        for (int q = 0; q < TL::NPRE; ++q) {
            const int idx = q * FT + threadIdx.x;
            if (idx < TL::PN) {
                const int t0 = G.tap[q] & 0xffff;
                const int tdx = ((G.tap[q] >> 16) & 1) ? 1 : -1;
                const int tdy = ((G.tap[q] >> 17) & 1) ? TL::CX : -TL::CX;
                const T w3 = (T)0.75, wq = (T)0.25;
                const int t1 = t0 + tdy;
                const T pe = w3 * (w3 * scp[t0] + wq * scp[t0 + tdx]) + wq * (w3 * scp[t1] + wq * scp[t1 + tdx]);
                if constexpr (XIN)
                    sx[buf][idx] = ((G.xneg[q] != (sz < 0)) ? -p.xs[q] : p.xs[q]) + pe;
                else
                    sx[buf][idx] = pe;
                if constexpr (HK) sk[buf][idx] = kconv<T, KT>(p.k[q]);
            }
        }
        __syncthreads();
    };

    int buf = 0;  // sx/sk buffer of the plane being committed (rotates through 3)
    // One plane step.  The steady form (ST: planes z0 + 2 .. z1 - 2 of a tile
    // that lies inside the grid) issues the same loads and stores on every
    // path, so the compiler's wait counts let the loads of the next two planes
    // stay in flight; the general form serves the first and last steps of the
    // march and tiles that cross the grid's edge.
    // pn: the other prefetch set, holding plane zi + 1's loads.
    auto step = [&](auto mode_tag, FPre<T, KT, TX, RY, ADD, XIN> &p, const FPre<T, KT, TX, RY, ADD, XIN> &pn,
                    int zi) {
        constexpr int MODE = decltype(mode_tag)::value;
        constexpr bool ST = MODE == 1;  // steady: every condition below holds
        constexpr bool FX = MODE != 0;  // fixed loads
        commit(p, zi, buf);
        bool bzneg = false;
        {
            int sb = 1;
            (void)fold(zi - 1, nz, a.g.bc[4], a.g.bc[5], sb);
            bzneg = sb < 0;
        }
        if (FX || zi + 2 <= z1 + 1) fetch_kc(p, zi + 2);

        // first sweep: absorb plane zi down the thread's strip, completing y1(zi - 1)
        const int yb = (zi - 1) & 1;
        if (act1) {
            // window rows j = 0 .. R1 + 1 of the input plane (region rows
            // s1q R1 - 1 .. s1q R1 + R1), clamped into the staged plane
            auto wrow = [&](int j) {
                const int py = min(s1q * TL::R1 + j, TL::PY - 1);
                const int c = py * TL::PX + (s1x + 1);
                return row_at<T, HK>(sx[buf], c, sk[buf], c);
            };
            Row<T> w0 = wrow(0), w1 = wrow(1);
#pragma unroll
            for (int q = 0; q < TL::R1; ++q) {
                const Row<T> w2 = wrow(q + 2);
                const PS<T> ps = col_sums<T, HK>(w0, w1, w2);
                const int qy = s1q * TL::R1 + q;
                const T bv = XIN ? p.b1[q] - bm : p.b1[q];
                const T bq = (G.bneg[q] != bzneg) ? -bv : bv;
                if (qy < TL::QY) sb[yb][qy * TL::QX + s1x] = bq;
                if ((ST || zi >= z0) && qy < TL::QY)
                    sy[yb][qy * TL::QX + s1x] = jacobi<T, HK>(r1[q], ps, bq, cw, om_w0, om, icv);
                absorb<T, HK>(r1[q], ps, zi == z0 - 2);
                w0 = w1;
                w1 = w2;
            }
        }
        // the next plane's coarse footprint (its commit reads it after the barrier below)
        if (FX || zi + 1 <= z1 + 1) stage_c(pn, zi + 1);
        __syncthreads();
        if (ST || zi >= z0) {
            // second sweep: absorb y1(zi - 1) with the coefficient plane zi - 1,
            // completing the output plane zi - 2
            const int kb = (buf + 2) % 3;
            // window rows j = 0 .. RY + 1 of the first-sweep plane (rows RY ly + j),
            // coefficient one row and column further in the input region
            auto wrow = [&](int j) {
                const int yy = RY * ly + j;
                return row_at<T, HK>(sy[yb], yy * TL::QX + (lx + 1), sk[kb], (yy + 1) * TL::PX + (lx + 2));
            };
            Row<T> w0 = wrow(0), w1 = wrow(1);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const Row<T> w2 = wrow(r + 2);
                const PS<T> ps = col_sums<T, HK>(w0, w1, w2);
                w0 = w1;
                w1 = w2;
                if (ST || (MODE == 0 && zi >= z0 + 2)) {  // mode 2 steps have no output plane
                    // right-hand side of output plane zi - 2, left by the previous step's first sweep
                    const T bo = sb[yb ^ 1][(RY * ly + r + 1) * TL::QX + (lx + 1)];
                    const T y = jacobi<T, HK>(r2[r], ps, bo, cw, om_w0, om, icv);
                    const size_t g = gb[r] + plane * (size_t)(zi - 2);
                    if (ST || valid[r]) {  // the steady march runs only on tiles inside the grid
                        if constexpr (ADD)
                            a.x64[g] = p.xo[r] + (double)y;
                        else
                            ((T *)a.yout)[g] = y;
                    }
                }
                absorb<T, HK>(r2[r], ps, zi == z0);
            }
        }
        // right-hand sides of plane zi + 2's step, into the registers just consumed
        if (FX || zi + 2 <= z1 + 1) fetch_b(mode_tag, p, zi + 2);
        buf = (buf + 1) % 3;
    };

    fetch(pA, z0 - 2);
    fetch(pB, z0 - 1);
    stage_c(pA, z0 - 2);
    __syncthreads();
    const std::integral_constant<int, 0> gen{};
    const std::integral_constant<int, 1> steady{};
    const std::integral_constant<int, 2> first{};
    int zi = z0 - 2;
    // Tiles inside the grid with at least four planes in the chunk run the
    // first four steps (no output plane yet) with fixed loads and then the
    // steady march, both steps of a pair with all their loads and stores
    // (zi >= z0 + 2 stores; zi + 3 <= z1 + 1 keeps every fetched plane in the
    // chunk); every path into the steady loop then has the same loads in
    // flight.  Other tiles, and the last steps, take the general form.
    const bool inside = i0 + TX <= nx && j0 + TL::TY <= ny && z1 - z0 >= 4;  // uniform over the workgroup
    if (inside) {
        for (; zi < z0 + 2; zi += 2) {
            step(first, pA, pB, zi);
            step(first, pB, pA, zi + 1);
        }
        for (; zi + 3 <= z1 + 1; zi += 2) {
            step(steady, pA, pB, zi);
            step(steady, pB, pA, zi + 1);
        }
    }
    for (; zi <= z1 + 1; zi += 2) {
        step(gen, pA, pB, zi);
        if (zi + 1 <= z1 + 1) step(gen, pB, pA, zi + 1);
    }
}

template <typename T, typename KT, int OUT, bool XIN = false>
hipError_t go2(const StencilArgs &a_, hipStream_t s)
{
    StencilArgs a = a_;
    const dim3 grid(batched_grid(a, a.t.blocks())), block(FT);
    switch (a.t.tx * 10 + a.t.ry) {
    case 642: hipLaunchKernelGGL((sweep2_kernel<T, KT, OUT, XIN, 64, 2>), grid, block, 0, s, a); break;
    case 641: hipLaunchKernelGGL((sweep2_kernel<T, KT, OUT, XIN, 64, 1>), grid, block, 0, s, a); break;
    case 322: hipLaunchKernelGGL((sweep2_kernel<T, KT, OUT, XIN, 32, 2>), grid, block, 0, s, a); break;
    case 321: hipLaunchKernelGGL((sweep2_kernel<T, KT, OUT, XIN, 32, 1>), grid, block, 0, s, a); break;
    case 162: hipLaunchKernelGGL((sweep2_kernel<T, KT, OUT, XIN, 16, 2>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool sweep2_supports(int tx, int ry) { return (tx == 64 && ry <= 2) || (tx == 32 && ry <= 2) || (tx == 16 && ry == 2); }

hipError_t launch_sweep2(int T_is_f64, int kt, int in_mode, int out_mode, const StencilArgs &a, hipStream_t s)
{
    if (a.t.blocks() <= 0 || (a.t.zc & 1)) return hipErrorInvalidValue;
    if (!a.ec || !a.b) return hipErrorInvalidValue;
    if (in_mode == IN_PROLONG_ADD) {
        // FP64 only; the pass reads x on a two-cell ring that other
        // workgroups' outputs cover, so the output must be another buffer
        if (!T_is_f64 || out_mode != OUT_STORE || !a.yin || !a.yout || a.yin == a.yout) return hipErrorInvalidValue;
        if (kt == KT_NONE) return go2<double, NoK, OUT_STORE, true>(a, s);
        if (kt == KT_F64) return go2<double, double, OUT_STORE, true>(a, s);
        return hipErrorInvalidValue;
    }
    if (in_mode != IN_PROLONG || a.bmean) return hipErrorInvalidValue;
    if (T_is_f64) {
        if (out_mode == OUT_STORE) {
            if (kt == KT_NONE) return go2<double, NoK, OUT_STORE>(a, s);
            if (kt == KT_F64) return go2<double, double, OUT_STORE>(a, s);
        }
        if (out_mode == OUT_ADD64) {
            if (kt == KT_NONE) return go2<double, NoK, OUT_ADD64>(a, s);
            if (kt == KT_F64) return go2<double, double, OUT_ADD64>(a, s);
        }
        return hipErrorInvalidValue;
    }
    if (out_mode == OUT_STORE) {
        if (kt == KT_NONE) return go2<float, NoK, OUT_STORE>(a, s);
        if (kt == KT_F32) return go2<float, float, OUT_STORE>(a, s);
        if (kt == KT_F16) return go2<float, __half, OUT_STORE>(a, s);
    }
    if (out_mode == OUT_ADD64) {
        if (kt == KT_NONE) return go2<float, NoK, OUT_ADD64>(a, s);
        if (kt == KT_F32) return go2<float, float, OUT_ADD64>(a, s);
        if (kt == KT_F16) return go2<float, __half, OUT_ADD64>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace nn4mg
