// One two-phase time step of arXiv 2401.06755, Sec. 2.4 (Stages 1-4), with
// linear (p = 1) filters, or quadratic ConvFEM filters (p = 2) for the terms
// that the paper's linear/quadratic combination gives them, on gfx950.
//
// Every operator of the step is a 3x3x3 filter sum f(u; w) (Sec. 2.2.2) over a
// field whose halo is synthesised at load time from that field's boundary
// rule: a mirror with sign +1 or -1 per face, and for the hydrostatic pressure
// a bottom halo that adds g h rho (Sec. 2.3.3).  The filters are tensor
// products of the 1D linear-element vectors
//     M = h [1, 4, 1] / 6 (mass),  G = [-1, 0, 1] / 2 (first derivative),
//     K = [-1, 2, -1] / h (stiffness),
// so each is evaluated separably on a 27-value neighbourhood held in
// registers.  One thread owns one cell; the neighbourhoods of adjacent threads
// overlap in L1/L2, which carries the re-reads (the momentum predictor, with
// twelve fields the heaviest, stages its planes in LDS instead).  This explicit part moves
// about a kilobyte per cell per step; the three pressure solves, run by the
// multigrid hierarchy of this library with a fixed cycle count, dominate.
//
// Boundary rules on the tank box (Sec. 3.1: free-slip side and bottom walls,
// an outlet with zero pressure on top):
//   C, rho, mu, k and the scalars made from them: +mirror on all faces;
//   velocity component d: -mirror on the walls normal to d, except the top;
//   component d of a vector made from grad C: -mirror on both faces normal to d;
//   p_nh and its increment: +mirror, -mirror on top;
//   p_hs: +mirror on the sides, -mirror on top, mirror + g h rho on the bottom.
// In the Petrov-Galerkin formulas (Eqs. k-abs special case, k-square, a_psi,
// the normalisation and Eq. negativek) the gradient Psi_x is taken in
// derivative units, f(Psi; w_x) / m_l; the residuals use the filters as
// printed.  mu blends like Eq. rho.  The velocities take the isotropic
// coefficient of Eq. k_Psi-n; the volume fraction the anisotropic compressive
// coefficients of Sec. 2.3.5 with the linear detectors, evaluated with the
// new velocity.  The surface-tension source of the momentum residual takes the
// sign that the Stage-1 pressure balances (Eq. hydro-pressure): with the
// curvature div n of Eq. surface-tension-k, the pressure of Eq. ph_disc has the
// physical Laplace jump across a drop and gradient -s_t, so s_t enters the
// predictor as +f(s_t; w_m).
#include "mg_async.h"
#include "mg_internal.h"

#include <cmath>
#include <cstring>
#include <string>

using namespace nn4mg;

namespace {

struct Grid {
    int nx, ny, nz;
    double h;
    size_t n;
};

// Face bits of a boundary rule: bit f set = -mirror on face f
// (xlo, xhi, ylo, yhi, zlo, zhi); clear = +mirror.
constexpr unsigned kEven = 0u;
constexpr unsigned kOddTop = 32u;  // p_nh, its increment, p_hs above
__host__ __device__ constexpr unsigned rule_vel(int d) { return d == 0 ? 3u : (d == 1 ? 12u : 16u); }
__host__ __device__ constexpr unsigned rule_grad(int d) { return 3u << (2 * d); }

__device__ inline size_t at(const Grid &g, int i, int j, int k)
{
    return (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * (size_t)k);
}

// Value of the padded field at (i, j, k), each index at most one cell outside.
__device__ inline double tap(const double *u, unsigned odd, const Grid &g, int i, int j, int k)
{
    double s = 1.0;
    if (i < 0) {
        i = 0;
        if (odd & 1u) s = -s;
    } else if (i >= g.nx) {
        i = g.nx - 1;
        if (odd & 2u) s = -s;
    }
    if (j < 0) {
        j = 0;
        if (odd & 4u) s = -s;
    } else if (j >= g.ny) {
        j = g.ny - 1;
        if (odd & 8u) s = -s;
    }
    if (k < 0) {
        k = 0;
        if (odd & 16u) s = -s;
    } else if (k >= g.nz) {
        k = g.nz - 1;
        if (odd & 32u) s = -s;
    }
    return s * u[at(g, i, j, k)];
}

// 27 values around a cell: v[(c+1)*9 + (b+1)*3 + (a+1)] at (i+a, j+b, k+c).
struct Nb {
    double v[27];
    __device__ double mid() const { return v[13]; }
};

__device__ inline void load(Nb &n, const double *u, unsigned odd, const Grid &g, int i, int j, int k)
{
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) n.v[c * 9 + b * 3 + a] = tap(u, odd, g, i + a - 1, j + b - 1, k + c - 1);
}

struct V3 {
    double m, z, p;  // weights at offsets -1, 0, +1
};

// f(u; X (x) Y (x) Z), X along i.
__device__ inline double sep(const Nb &n, const V3 &X, const V3 &Y, const V3 &Z)
{
    double out = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double pl = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double *r = &n.v[c * 9 + b * 3];
            const double row = X.m * r[0] + X.z * r[1] + X.p * r[2];
            pl += (b == 0 ? Y.m : (b == 1 ? Y.z : Y.p)) * row;
        }
        out += (c == 0 ? Z.m : (c == 1 ? Z.z : Z.p)) * pl;
    }
    return out;
}

// f(k C; X (x) Y (x) Z) with the products formed on the fly (no third neighbourhood).
__device__ inline double sepp(const Nb &k, const Nb &n, const V3 &X, const V3 &Y, const V3 &Z)
{
    double out = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double pl = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double *r = &n.v[c * 9 + b * 3];
            const double *kr = &k.v[c * 9 + b * 3];
            const double row = X.m * (kr[0] * r[0]) + X.z * (kr[1] * r[1]) + X.p * (kr[2] * r[2]);
            pl += (b == 0 ? Y.m : (b == 1 ? Y.z : Y.p)) * row;
        }
        out += (c == 0 ? Z.m : (c == 1 ? Z.z : Z.p)) * pl;
    }
    return out;
}

struct Filt {
    V3 M, G, K, m;  // m = M / h
    double ml;      // lumped mass h^3
    __device__ explicit Filt(double h)
    {
        M = {h / 6.0, 4.0 * h / 6.0, h / 6.0};
        G = {-0.5, 0.0, 0.5};
        K = {-1.0 / h, 2.0 / h, -1.0 / h};
        m = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
        ml = h * h * h;
    }
    // w_d = G along d, M across (the printed w_x of Sec. 2.2.3 for d = 0)
    __device__ double d(const Nb &n, int dir) const
    {
        return dir == 0 ? sep(n, G, M, M) : (dir == 1 ? sep(n, M, G, M) : sep(n, M, M, G));
    }
    // w_dd^PG = K along d, M across
    __device__ double pg(const Nb &n, int dir) const
    {
        return dir == 0 ? sep(n, K, M, M) : (dir == 1 ? sep(n, M, K, M) : sep(n, M, M, K));
    }
    __device__ double lap(const Nb &n) const { return sep(n, K, M, M) + sep(n, M, K, M) + sep(n, M, M, K); }
    __device__ double mass(const Nb &n) const { return sep(n, M, M, M); }
    // w_m / m_l - E: the residual filter of Eq. a_psi
    __device__ double mass_resid(const Nb &n) const { return sep(n, m, m, m) - n.mid(); }
};

// Eq. k-Txx: 1/2 [f(k C; w) + k f(C; w) - C f(k; w)] with the product of the
// padded values as the halo of k C.  which: 0..2 = w_dd^PG, 3 = w_lap.
__device__ inline double fdiff(const Filt &F, const Nb &Cn, const Nb &kn, int which)
{
    double fk;  // f(k C; w)
    if (which == 3)
        fk = sepp(kn, Cn, F.K, F.M, F.M) + sepp(kn, Cn, F.M, F.K, F.M) + sepp(kn, Cn, F.M, F.M, F.K);
    else if (which == 0)
        fk = sepp(kn, Cn, F.K, F.M, F.M);
    else if (which == 1)
        fk = sepp(kn, Cn, F.M, F.K, F.M);
    else
        fk = sepp(kn, Cn, F.M, F.M, F.K);
    if (which == 3) return 0.5 * (fk + kn.mid() * F.lap(Cn) - Cn.mid() * F.lap(kn));
    return 0.5 * (fk + kn.mid() * F.pg(Cn, which) - Cn.mid() * F.pg(kn, which));
}

struct Phys {
    double rho_l, rho_g, mu_l, mu_g, g, sigma, dt;
};

template <typename F>
__device__ inline bool cell_of(const Grid &g, F &&body)
{
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.n) return false;
    const int i = (int)(id % (size_t)g.nx);
    const size_t t = id / (size_t)g.nx;
    body(id, i, (int)(t % (size_t)g.ny), (int)(t / (size_t)g.ny));
    return true;
}

struct F3 {
    double *p[3];
};
struct C3 {
    const double *p[3];
};

// ------------------------------------------------------------------ kernels

// ---- one workgroup per 8^3 block ----
// For kernels that filter several fields per cell (the advection and the PG
// diffusivity of the three components) each field is staged once in LDS on
// the block plus a one-cell halo (10^3 cells, the field's boundary rule
// applied as tap() applies it), and each thread gathers its cell's 27 values
// from there into an Nb: the values load() gives, with one global load per
// staged cell instead of 27 per cell.  Two staging buffers alternate, one
// barrier per field: a thread stages field f only after the barrier of field
// f - 1, which every thread reaches after gathering f - 2.  (For the kernels
// that filter one or two fields, and the plane-marching momentum kernel, the
// per-cell gathers through L1/L2 measured faster.)
constexpr int SB = 8;                // block edge
constexpr int SBT = SB * SB * SB;    // threads: one cell each
constexpr int SL = SB + 2;           // staged edge
constexpr int SLN = SL * SL * SL;    // staged cells

// This thread's cell of the workgroup's block (the block at (i0, j0, k0)); a
// ragged block's threads beyond the grid work on their cell clamped into it
// and write nothing.
struct BCell {
    int i0, j0, k0, i, j, k;
    bool valid;
    size_t id;
};
__device__ inline BCell bcell(const Grid &g)
{
    BCell c;
    const int bxn = (g.nx + SB - 1) / SB, byn = (g.ny + SB - 1) / SB;
    const int lb = blockIdx.x, t = threadIdx.x;
    c.i0 = (lb % bxn) * SB;
    c.j0 = ((lb / bxn) % byn) * SB;
    c.k0 = (lb / bxn / byn) * SB;
    const int i = c.i0 + t % SB, j = c.j0 + (t / SB) % SB, k = c.k0 + t / (SB * SB);
    c.valid = i < g.nx && j < g.ny && k < g.nz;
    c.i = min(i, g.nx - 1);
    c.j = min(j, g.ny - 1);
    c.k = min(k, g.nz - 1);
    c.id = at(g, c.i, c.j, c.k);
    return c;
}

unsigned blocks_of(const Grid &g)
{
    return (unsigned)(((g.nx + SB - 1) / SB) * ((g.ny + SB - 1) / SB) * ((g.nz + SB - 1) / SB));
}

// Neighbourhoods from LDS: load_nb(nb, u, odd) stages field u (rule odd) into
// the next buffer, waits for the workgroup and gathers this thread's 27 values.
struct LNb {
    double (*buf)[SLN];
    const Grid &g;
    const BCell &X;
    int next;
    template <typename V>
    __device__ void stage_gather(Nb &n, const V &val)
    {
        double *b = buf[next];
        next ^= 1;
        const int t = threadIdx.x;
#pragma unroll
        for (int r = 0; r < (SLN + SBT - 1) / SBT; ++r) {
            const int idx = t + r * SBT;
            if (idx < SLN) {
                const int x = idx % SL, y = (idx / SL) % SL, z = idx / (SL * SL);
                b[idx] = val(X.i0 + x - 1, X.j0 + y - 1, X.k0 + z - 1);
            }
        }
        __syncthreads();
        const int tx = t % SB, ty = (t / SB) % SB, tz = t / (SB * SB);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                for (int a = 0; a < 3; ++a) n.v[c * 9 + bb * 3 + a] = b[(tx + a) + SL * ((ty + bb) + SL * (tz + c))];
    }
    __device__ void operator()(Nb &n, const double *u, unsigned odd)
    {
        const Grid &gg = g;
        stage_gather(n, [&](int i, int j, int k) { return tap(u, odd, gg, i, j, k); });
    }
};

// rho, mu (Eq. rho), grad C in derivative units, unit normals.
__global__ __launch_bounds__(256) void props_kernel(Grid g, Phys P, const double *C, double *rho, double *mu, F3 Cd,
                                                    F3 nrm)
{
    cell_of(g, [&](size_t id, int i, int j, int k) {
        const Filt F(g.h);
        Nb c;
        load(c, C, kEven, g, i, j, k);
        const double c0 = c.mid();
        rho[id] = P.rho_l * c0 + P.rho_g * (1.0 - c0);
        mu[id] = P.mu_l * c0 + P.mu_g * (1.0 - c0);
        double gd[3];
        for (int d = 0; d < 3; ++d) gd[d] = F.d(c, d) / F.ml;
        const double l = sqrt(gd[0] * gd[0] + gd[1] * gd[1] + gd[2] * gd[2]);
        const double eps = 1e-7 / g.h;
        for (int d = 0; d < 3; ++d) {
            Cd.p[d][id] = gd[d];
            nrm.p[d][id] = gd[d] / (eps + l);
        }
    });
}

// Curvature kappa = div n (Eq. curvature) and the surface-tension force
// sigma kappa grad C (Eq. surface-tension-k).
__global__ __launch_bounds__(256) void surface_kernel(Grid g, double sigma, C3 nrm, C3 Cd, F3 st)
{
    cell_of(g, [&](size_t id, int i, int j, int k) {
        const Filt F(g.h);
        double kap = 0.0;
        for (int d = 0; d < 3; ++d) {
            Nb n;
            load(n, nrm.p[d], rule_grad(d), g, i, j, k);
            kap += F.d(n, d);
        }
        kap /= F.ml;
        for (int d = 0; d < 3; ++d) st.p[d][id] = sigma * kap * Cd.p[d][id];
    });
}

// Right-hand side of Eq. ph_disc: sum_d f(s_t,d; w_d) + f(g rho; w_z), minus
// the Laplacian filter applied to the affine part of p_hs's bottom halo, so the
// solve sees homogeneous rules.
__global__ __launch_bounds__(256) void rhs_hydrostatic_kernel(Grid g, double grav, C3 st, const double *rho,
                                                              double *b)
{
    cell_of(g, [&](size_t id, int i, int j, int k) {
        const Filt F(g.h);
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            Nb n;
            load(n, st.p[d], rule_grad(d), g, i, j, k);
            s += F.d(n, d);
        }
        Nb r, lift;
        load(r, rho, kEven, g, i, j, k);
        // the halo plane below k = 0 carries g h rho(i, j, 0); everything else is zero
        const double gh = grav * g.h;
        for (int q = 0; q < 27; ++q) lift.v[q] = (k == 0 && q < 9) ? gh * r.v[q] : 0.0;
        for (int q = 0; q < 27; ++q) r.v[q] *= grav;
        s += F.d(r, 2);
        if (k == 0) s -= F.lap(lift);
        b[id] = s;
    });
}

// Advection of each velocity component by the iterate: adv_c = q . grad q_c.
__global__ __launch_bounds__(SBT) void advection_kernel(Grid g, C3 q, F3 adv)
{
    __shared__ double sb[2][SLN];
    const BCell X = bcell(g);
    LNb load_nb{sb, g, X, 0};
    const Filt F(g.h);
    const size_t id = X.id;
    const double q0[3] = {q.p[0][id], q.p[1][id], q.p[2][id]};
    for (int c = 0; c < 3; ++c) {
        Nb n;
        load_nb(n, q.p[c], rule_vel(c));
        double a = 0.0;
        for (int d = 0; d < 3; ++d) a += q0[d] * (F.d(n, d) / F.ml);
        if (X.valid) adv.p[c][id] = a;
    }
}

// Isotropic Petrov-Galerkin diffusivity of each component (Eq. k_Psi-n with
// Eqs. efficient-kabs-special-case, k-square with h_Psi = h, max-k and the
// residual a_Psi of Eq. a_psi, alpha_a = 2): k_c = rho min(k_max, k_abs, k_sq) + mu.
__global__ __launch_bounds__(SBT) void pg_velocity_kernel(Grid g, C3 q, C3 adv, const double *rho,
                                                          const double *mu, F3 kq)
{
    __shared__ double sb[2][SLN];
    const BCell X = bcell(g);
    LNb load_nb{sb, g, X, 0};
    const Filt F(g.h);
    const size_t id = X.id;
    const double eps_k = 1e-7, a_kabs = 1.0 / 16.0, a_ksq = 4.0, h = g.h;
    const double u = q.p[0][id], v = q.p[1][id], w = q.p[2][id];
    for (int c = 0; c < 3; ++c) {
        Nb n;
        load_nb(n, q.p[c], rule_vel(c));
        const double px = F.d(n, 0) / F.ml, py = F.d(n, 1) / F.ml, pz = F.d(n, 2) / F.ml;
        Nb an;
        load_nb(an, adv.p[c], kEven);
        const double a = 2.0 * F.mass_resid(an);
        const double G = fabs(px) + fabs(py) + fabs(pz);
        const double kabs = a_kabs * h * fabs(a) / (eps_k + G / 3.0);
        const double g2 = px * px + py * py + pz * pz;
        const double advabs = fabs(u * px) + fabs(v * py) + fabs(w * pz);
        const double ksq = a_ksq * a * a * h / (eps_k + advabs / 3.0 * g2);
        const double kmax = h * (fabs(u) + fabs(v) + fabs(w));
        const double m = fmin(kmax, fmin(kabs, ksq));
        if (X.valid) kq.p[c][id] = rho[id] * m + mu[id];
    }
}

// One predictor iteration (Eqs. Petrov, velocity-1): the momentum residual
// s_c = rho m_l adv_c + f_lap(q_c, k_c) + f(p_hs + p_nh; w_c) - f(s_t,c; w_m)
// [- f(-g rho; w_m) for c = z] gives q~_c = (-s_c / m_l + rho q^n_c / dt) / (rho / dt),
// and the next iterate is (q^n + q~) / 2.
// Its twelve input fields are staged in LDS: one workgroup owns an MT_X x MT_Y
// column of cells and marches MT_Z planes; each plane of every field is loaded
// once, with its halo rule (and the lifted bottom halo of p_hs), into a
// three-plane rotation, and each cell's 27-value neighbourhoods are gathered
// from LDS in the order load() builds them (the same arithmetic as the
// per-cell form).  The neighbourhood re-reads that would go through L1/L2
// (324 loads per cell) become LDS reads.
constexpr int MT_X = 16, MT_Y = 8, MT_Z = 8;
constexpr int MP_X = MT_X + 2, MP_N = (MT_X + 2) * (MT_Y + 2);
constexpr int M_NF = 12;  // p_hs, p_nh, rho, q0..2, kq0..2, st0..2

struct MomIn {
    const double *u[M_NF];
};

__device__ inline unsigned mom_rule(int f)
{
    return f <= 1 ? kOddTop : (f == 2 ? kEven : (f <= 5 ? rule_vel(f - 3) : (f <= 8 ? kEven : rule_grad(f - 9))));
}

__device__ inline void gather(Nb &n, const double *sf, const int (&slot)[3], int li, int lj)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double *pl = sf + slot[c] * MP_N;
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) n.v[c * 9 + b * 3 + a] = pl[(lj + b) * MP_X + (li + a)];
    }
}

__global__ __launch_bounds__(MT_X * MT_Y) void momentum_lds_kernel(Grid g, Phys P, C3 qn, MomIn in, C3 adv,
                                                                   F3 qt, F3 qnext)
{
    __shared__ double sm[M_NF][3][MP_N];
    const int tx = (g.nx + MT_X - 1) / MT_X, ty = (g.ny + MT_Y - 1) / MT_Y;
    const int bx = blockIdx.x % tx, rest = blockIdx.x / tx;
    const int by = rest % ty, bz = rest / ty;
    const int i0 = bx * MT_X, j0 = by * MT_Y, z0 = bz * MT_Z;
    const int z1 = min(z0 + MT_Z, g.nz);
    const int li = threadIdx.x % MT_X, lj = threadIdx.x / MT_X;
    const int i = i0 + li, j = j0 + lj;
    const bool valid = i < g.nx && j < g.ny;
    const double gh = P.g * g.h;

    // plane z of every field into slot (z + 3) % 3: clamped addresses and the
    // faces crossed first, then every load in flight, then the signs of each
    // field's rule (the product over the crossed faces, as tap() forms it)
    constexpr int NR = (MP_N + MT_X * MT_Y - 1) / (MT_X * MT_Y);
    auto stage = [&](int z) {
        const int sl = (z + 3) % 3;
        const int zc = z < 0 ? 0 : (z >= g.nz ? g.nz - 1 : z);
        const unsigned zbit = z < 0 ? 16u : (z >= g.nz ? 32u : 0u);
        size_t off[NR];
        unsigned bits[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int c = min((int)threadIdx.x + r * MT_X * MT_Y, MP_N - 1);
            const int py = c / MP_X, px = c - py * MP_X;
            const int gi = i0 + px - 1, gj = j0 + py - 1;
            const int ci = gi < 0 ? 0 : (gi >= g.nx ? g.nx - 1 : gi);
            const int cj = gj < 0 ? 0 : (gj >= g.ny ? g.ny - 1 : gj);
            bits[r] = zbit | (gi < 0 ? 1u : (gi >= g.nx ? 2u : 0u)) | (gj < 0 ? 4u : (gj >= g.ny ? 8u : 0u));
            off[r] = at(g, ci, cj, zc);
        }
        double v[M_NF][NR];
#pragma unroll
        for (int f = 0; f < M_NF; ++f)
#pragma unroll
            for (int r = 0; r < NR; ++r) v[f][r] = in.u[f][off[r]];
#pragma unroll
        for (int f = 0; f < M_NF; ++f) {
            const unsigned rule = mom_rule(f);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int c = (int)threadIdx.x + r * MT_X * MT_Y;
                if (c < MP_N) {
                    double x = (__popc(bits[r] & rule) & 1) ? -v[f][r] : v[f][r];
                    if (f == 0 && z == -1) x += gh * v[2][r];  // lifted bottom halo of p_hs (rho +mirror)
                    sm[f][sl][c] = x;
                }
            }
        }
    };
    stage(z0 - 1);
    stage(z0);
    for (int k = z0; k < z1; ++k) {
        stage(k + 1);
        __syncthreads();
        const int slot[3] = {(k + 2) % 3, k % 3, (k + 1) % 3};  // planes k - 1, k, k + 1
        if (valid) {
            const size_t id = at(g, i, j, k);
            const Filt F(g.h);
            const double r0 = in.u[2][id];
            double ghs[3], gnh[3], buoy;
            {
                Nb p;
                gather(p, &sm[0][0][0], slot, li, lj);
                for (int c = 0; c < 3; ++c) ghs[c] = F.d(p, c);
            }
            {
                Nb p;
                gather(p, &sm[1][0][0], slot, li, lj);
                for (int c = 0; c < 3; ++c) gnh[c] = F.d(p, c);
            }
            {
                Nb r;
                gather(r, &sm[2][0][0], slot, li, lj);
                for (int e = 0; e < 27; ++e) r.v[e] *= -P.g;
                buoy = F.mass(r);
            }
            for (int c = 0; c < 3; ++c) {
                double s;
                {
                    Nb qv, kv;
                    gather(qv, &sm[3 + c][0][0], slot, li, lj);
                    gather(kv, &sm[6 + c][0][0], slot, li, lj);
                    s = fdiff(F, qv, kv, 3);
                }
                s += ghs[c];
                s += gnh[c];
                {   // surface tension with the sign the Stage-1 pressure balances
                    Nb t;
                    gather(t, &sm[9 + c][0][0], slot, li, lj);
                    s += F.mass(t);
                }
                if (c == 2) s -= buoy;
                s += r0 * F.ml * adv.p[c][id];
                const double qnc = qn.p[c][id];
                const double t = (-s / F.ml + r0 * qnc / P.dt) / (r0 / P.dt);
                qt.p[c][id] = t;
                qnext.p[c][id] = 0.5 * (qnc + t);
            }
        }
        __syncthreads();
    }
}

// Right-hand side of Eq. ph_disc2 for the pressure increment:
// -(1/dt) sum_d f(rho q~_d; w_d) + (1/dt) sum_d q~_d f(rho; w_d).
__global__ __launch_bounds__(256) void rhs_nonhydrostatic_kernel(Grid g, double dt, C3 qt, const double *rho,
                                                                 double *b)
{
    cell_of(g, [&](size_t id, int i, int j, int k) {
        const Filt F(g.h);
        Nb r;
        load(r, rho, kEven, g, i, j, k);
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            Nb m;
            load(m, qt.p[d], rule_vel(d), g, i, j, k);
            for (int e = 0; e < 27; ++e) m.v[e] *= r.v[e];
            s -= F.d(m, d) / dt;
            s += qt.p[d][id] * F.d(r, d) / dt;
        }
        b[id] = s;
    });
}

// Eq. vel-cor: q~_d -= dt f(dp; w_d) / (m_l rho); p_nh += dp.
__global__ __launch_bounds__(256) void correct_kernel(Grid g, double dt, const double *dp, const double *rho, C3 qin,
                                                      F3 qout, double *p_nh)
{
    cell_of(g, [&](size_t id, int i, int j, int k) {
        const Filt F(g.h);
        Nb n;
        load(n, dp, kOddTop, g, i, j, k);
        const double r0 = rho[id];
        for (int d = 0; d < 3; ++d) qout.p[d][id] = qin.p[d][id] + -dt * (F.d(n, d) / F.ml) / r0;
        p_nh[id] += n.mid();
    });
}

// u . grad C with the new velocity (input of the residual of Eq. a_psi for C).
__global__ __launch_bounds__(256) void advection_c_kernel(Grid g, C3 q, C3 Cd, double *out)
{
    cell_of(g, [&](size_t id, int, int, int) {
        out[id] = q.p[0][id] * Cd.p[0][id] + q.p[1][id] * Cd.p[1][id] + q.p[2][id] * Cd.p[2][id];
    });
}

// Anisotropic compressive diffusivities of the volume fraction (Sec. 2.3.5):
// linear interface detectors S_d, weights w+ and w-, k+ = 3 k_abs and the
// negative (compressive) k- of Eq. negativek with its normalisation, clamped
// to [-alpha_min h^2 / dt, alpha_max h^2 / dt] (Eq. alpha_min_and_max).
__global__ __launch_bounds__(256) void pg_volume_fraction_kernel(Grid g, double dt, const double *C, C3 Cd, C3 q,
                                                                 const double *advc, F3 kd)
{
    cell_of(g, [&](size_t id, int i, int j, int k) {
        const Filt F(g.h);
        const double Kp = 300.0, Km = 300.0, beta = 0.1, eps_x = 1e-4, Kpos = 3.0, eps_k = 1e-7, h = g.h;
        const double kmin = 1e-4 / dt * h * h, kclamp = 0.05 / dt * h * h;
        Nb an;
        load(an, advc, kEven, g, i, j, k);
        const double a = 2.0 * F.mass_resid(an);
        const double c0 = C[id];
        double S[3];
        S[0] = (c0 - tap(C, kEven, g, i - 1, j, k)) * (tap(C, kEven, g, i + 1, j, k) - c0);
        S[1] = (c0 - tap(C, kEven, g, i, j - 1, k)) * (tap(C, kEven, g, i, j + 1, k) - c0);
        S[2] = (c0 - tap(C, kEven, g, i, j, k - 1)) * (tap(C, kEven, g, i, j, k + 1) - c0);
        if (c0 > 0.95 || c0 < 0.05) S[0] = S[1] = S[2] = -1.0;
        const double cx = Cd.p[0][id], cy = Cd.p[1][id], cz = Cd.p[2][id];
        const double u = q.p[0][id], v = q.p[1][id], w = q.p[2][id];
        const double g2 = cx * cx + cy * cy + cz * cz;
        const double proj = (u * cx + v * cy + w * cz) / (eps_x + g2);
        const double us = cx * proj, vs = cy * proj, ws = cz * proj;
        const double kneg = -beta * (u * u + v * v + w * w) / (eps_x + g2 * (fabs(us) + fabs(vs) + fabs(ws)) / 3.0);
        const double G = fabs(cx) + fabs(cy) + fabs(cz);
        const double kabs = (1.0 / 16.0) * h * fabs(a) / (eps_k + G / 3.0);
        for (int d = 0; d < 3; ++d) {
            const double wp = -fmax(-1.0, fmin(0.0, Kp * S[d]));
            const double wm = fmin(1.0, fmax(0.0, Km * S[d]));
            const double kk = wp * (Kpos * kabs) + wm * (kneg / h);
            kd.p[d][id] = fmax(-kmin, fmin(kclamp, kk));
        }
    });
}

// Eqs. Petrov-C, transport-indicator-1: C^{n+1} = C - dt s_C / m_l with
// s_C = m_l u . grad C + sum_d f_d(C, k_d; w_dd^PG).
__global__ __launch_bounds__(256) void volume_fraction_kernel(Grid g, double dt, const double *C, C3 kd, C3 q, C3 Cd,
                                                              double *Cnew)
{
    cell_of(g, [&](size_t id, int i, int j, int k) {
        const Filt F(g.h);
        double s = F.ml * (q.p[0][id] * Cd.p[0][id] + q.p[1][id] * Cd.p[1][id] + q.p[2][id] * Cd.p[2][id]);
        Nb cn;
        load(cn, C, kEven, g, i, j, k);
        for (int d = 0; d < 3; ++d) {
            Nb kn;
            load(kn, kd.p[d], kEven, g, i, j, k);
            s += fdiff(F, cn, kn, d);
        }
        Cnew[id] = cn.mid() - dt * s / F.ml;
    });
}

__global__ __launch_bounds__(256) void copy3_kernel(size_t n, C3 src, F3 dst)
{
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    for (int d = 0; d < 3; ++d) dst.p[d][id] = src.p[d][id];
}

// ------------------------------------------------ quadratic ConvFEM (order 2)
// The 5 x 5 x 5 filters of the quadratic ConvFEM (Sec. 2.2.3: the stencils of
// the vertex and mid nodes of quadratic Lagrange elements summed and
// averaged) are tensor products of
//     M2 = h [-1, 4, 24, 4, -1] / 30,  G2 = [1, -8, 0, 8, -1] / 12,
//     K2 = [1, -16, 30, -16, 1] / (12 h),
// applied with two-cell halos (Sec. 2.3.3): halo cell -1-m takes interior
// cell m with the field's sign, and the bottom halo of p_hs adds
// (2m + 1) g h rho (the gradient -rho g extrapolated over (2m + 1) h).  They
// serve the momentum terms, the interface geometry and the volume-fraction
// advection (Table disc_combinations, "linear/quadratic"); the volume-fraction
// diffusion and the two pressure equations keep the linear filters.
//
// Each kernel runs one workgroup per 8^3 block of cells.  A filter factors
// into three 5-tap passes, along x, then y, then z, so the block stages a
// field once on its cells plus the two-cell halo (12^3, the field's boundary
// rule applied while staging) and runs the passes through LDS: about 5 fused
// multiply-adds per tap and output instead of 15, and one global load per
// staged cell instead of one per tap.  Every sum keeps the x-then-y-then-z
// order with the same weights.

struct V5 {
    double w[5];
};

// Index up to two cells outside folded onto the cell it mirrors; s flips on a
// crossed face whose bit is set in odd.
__device__ inline int fold2(int i, int n, unsigned odd, unsigned lo_bit, unsigned hi_bit, double &s)
{
    if (i < 0) {
        if (odd & lo_bit) s = -s;
        return -1 - i;
    }
    if (i >= n) {
        if (odd & hi_bit) s = -s;
        return 2 * n - 1 - i;
    }
    return i;
}

// Padded value of u at (i, j, k) with the two-cell halo of rule odd.
struct Tap2 {
    const double *u;
    unsigned odd;
    Grid g;
    __device__ double operator()(int i, int j, int k) const
    {
        double s = 1.0;
        i = fold2(i, g.nx, odd, 1u, 2u, s);
        j = fold2(j, g.ny, odd, 4u, 8u, s);
        k = fold2(k, g.nz, odd, 16u, 32u, s);
        return s * u[at(g, i, j, k)];
    }
};


constexpr int QB = SB;                // output block edge
constexpr int QT = SBT;               // threads: one output cell each
constexpr int QS = QB + 4;            // staged edge
constexpr int QSN = QS * QS * QS;     // staged cells
constexpr int QRN = QB * QS * QS;     // x-pass outputs per filter (8 x 12 x 12)
constexpr int QPN = QB * QB * QS;     // y-pass outputs per filter (8 x 8 x 12)

// The 1D weights of the quadratic filters and the mass of a cell, computed on
// the host and passed by value so they stay in scalar registers.
struct QW {
    V5 M, G, K;
    double ml;
};
QW quad_weights(double h)
{
    const double m[5] = {-1.0, 4.0, 24.0, 4.0, -1.0}, gw[5] = {1.0, -8.0, 0.0, 8.0, -1.0},
                 kw[5] = {1.0, -16.0, 30.0, -16.0, 1.0};
    QW w;
    for (int q = 0; q < 5; ++q) {
        w.M.w[q] = h * m[q] / 30.0;
        w.G.w[q] = gw[q] / 12.0;
        w.K.w[q] = kw[q] / (12.0 * h);
    }
    w.ml = h * h * h;
    return w;
}

struct QLds {
    double s[QSN];    // the staged field
    double r[2][QRN]; // x pass: the derivative (or K) filter and M
    double p[3][QPN]; // y pass: M on r[0], the derivative (or K) filter on r[1], M on r[1]
};

// Index up to two cells outside folded as fold2; indices further out (the
// halo of a ragged block's cells beyond the grid, which feed no output) are
// clamped into range.
__device__ inline int qfold(int i, int n, unsigned odd, unsigned lo_bit, unsigned hi_bit, double &s)
{
    const int f = fold2(i, n, odd, lo_bit, hi_bit, s);
    return min(max(f, 0), n - 1);
}

// A field at unfolded (i, j, k) with the two-cell halo of rule odd.
// Each staging functor splits into fetch (the global loads and the sign or
// halo case of an unfolded (i, j, k)) and value (the staged value from the
// fetched raw data), so the loads of the next field can be in flight while
// the current field's passes run.
struct QTap {
    const double *u;
    unsigned odd;
    Grid g;
    struct Raw {
        double v;
        bool neg;
    };
    __device__ Raw fetch(int i, int j, int k) const
    {
        double s = 1.0;
        const int fi = qfold(i, g.nx, odd, 1u, 2u, s);
        const int fj = qfold(j, g.ny, odd, 4u, 8u, s);
        const int fk = qfold(k, g.nz, odd, 16u, 32u, s);
        return {u[at(g, fi, fj, fk)], s < 0.0};
    }
    __device__ double value(const Raw &r) const { return r.neg ? -r.v : r.v; }
    __device__ double operator()(int i, int j, int k) const { return value(fetch(i, j, k)); }
};

// p_hs at unfolded (i, j, k): +mirror on the sides, -mirror on top, and below
// the bottom the mirror plus (2m + 1) g h rho of the mirrored cell (rho +mirror
// on the sides).
struct QPhs {
    const double *p, *rho;
    Grid g;
    double gh;
    struct Raw {
        double p, r;
        int m;  // below the bottom: the mirror distance m (>= 0); -1 inside; -2 above the top
    };
    __device__ Raw fetch(int i, int j, int k) const
    {
        double s = 1.0;
        const int fi = qfold(i, g.nx, 0u, 1u, 2u, s);
        const int fj = qfold(j, g.ny, 0u, 4u, 8u, s);
        const int fk = qfold(k, g.nz, 0u, 16u, 32u, s);
        const size_t idx = at(g, fi, fj, fk);
        Raw o;
        o.p = p[idx];
        o.r = k < 0 ? rho[idx] : 0.0;
        o.m = k < 0 ? -1 - k : (k >= g.nz ? -2 : -1);
        return o;
    }
    __device__ double value(const Raw &o) const
    {
        if (o.m >= 0) return o.p + (double)(2 * o.m + 1) * gh * o.r;
        return o.m == -2 ? -o.p : o.p;
    }
    __device__ double operator()(int i, int j, int k) const { return value(fetch(i, j, k)); }
};

template <typename A, typename B>
struct QMul {
    A a;
    B b;
    struct Raw {
        typename A::Raw a;
        typename B::Raw b;
    };
    __device__ Raw fetch(int i, int j, int k) const { return {a.fetch(i, j, k), b.fetch(i, j, k)}; }
    __device__ double value(const Raw &r) const { return a.value(r.a) * b.value(r.b); }
    __device__ double operator()(int i, int j, int k) const { return value(fetch(i, j, k)); }
};

// The next field's staging in registers: fetch issues its loads, commit
// writes the staged values to LDS (after the current field's passes; the x
// pass, the only reader of the staged field, is then done on every thread).
template <typename V>
struct QNext {
    static constexpr int NR = (QSN + QT - 1) / QT;
    typename V::Raw r[NR];
    __device__ void fetch(const V &v, int i0, int j0, int k0)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int idx = min(t + q * QT, QSN - 1);
            const int x = idx % QS, y = (idx / QS) % QS, z = idx / (QS * QS);
            r[q] = v.fetch(i0 + x - 2, j0 + y - 2, k0 + z - 2);
        }
    }
    __device__ void commit(QLds &L, const V &v) const
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int idx = t + q * QT;
            if (idx < QSN) L.s[idx] = v.value(r[q]);
        }
    }
};

// Stage field v on the block at (i0, j0, k0) plus its two-cell halo.
template <typename V>
__device__ inline void qstage(QLds &L, const V &v, int i0, int j0, int k0)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < (QSN + QT - 1) / QT; ++r) {
        const int idx = t + r * QT;
        if (idx < QSN) {
            const int x = idx % QS, y = (idx / QS) % QS, z = idx / (QS * QS);
            L.s[idx] = v(i0 + x - 2, j0 + y - 2, k0 + z - 2);
        }
    }
}

// The x and y passes of the staged field: wa is G (derivatives) or K
// (Laplacian); DER: also the passes only the derivatives or the Laplacian
// need (else the mass filter alone).  Barrier before each pass.
template <bool DER>
__device__ inline void qpasses(QLds &L, const V5 &wa, const V5 &wm)
{
    const int t = threadIdx.x;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (QRN + QT - 1) / QT; ++r) {
        const int idx = t + r * QT;
        if (idx < QRN) {
            const int x = idx % QB, yz = idx / QB;  // y + QS z
            const double *row = L.s + x + QS * yz;
            double ra = 0.0, rm = 0.0;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const double v = row[a];
                if (DER) ra += wa.w[a] * v;
                rm += wm.w[a] * v;
            }
            if (DER) L.r[0][idx] = ra;
            L.r[1][idx] = rm;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (QPN + QT - 1) / QT; ++r) {
        const int idx = t + r * QT;
        if (idx < QPN) {
            const int x = idx % QB, y = (idx / QB) % QB, z = idx / (QB * QB);
            const int o = x + QB * (y + QS * z);
            double p0 = 0.0, p1 = 0.0, p2 = 0.0;
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                if (DER) {
                    p0 += wm.w[b] * L.r[0][o + QB * b];
                    p1 += wa.w[b] * L.r[1][o + QB * b];
                }
                p2 += wm.w[b] * L.r[1][o + QB * b];
            }
            if (DER) {
                L.p[0][idx] = p0;
                L.p[1][idx] = p1;
            }
            L.p[2][idx] = p2;
        }
    }
    __syncthreads();
}

// The derivative filters d[0..2] = f(u; w_x, w_y, w_z) (DER) and the mass
// filter d[3] = f(u; w_m) of the staged field at this thread's cell.
template <bool DER>
__device__ inline void qderiv(QLds &L, const QW &F, double d[4])
{
    qpasses<DER>(L, F.G, F.M);
    const int t = threadIdx.x;
    const int o = (t % QB) + QB * ((t / QB) % QB + QB * (t / (QB * QB)));  // z-plane stride QB * QB
    double dx = 0.0, dy = 0.0, dz = 0.0, mm = 0.0;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const int q = o + QB * QB * c;
        const double Mc = F.M.w[c];
        if (DER) {
            dx += Mc * L.p[0][q];
            dy += Mc * L.p[1][q];
            dz += F.G.w[c] * L.p[2][q];
        }
        mm += Mc * L.p[2][q];
    }
    d[0] = dx;
    d[1] = dy;
    d[2] = dz;
    d[3] = mm;
}

// f(u; w_lap) = f(u; K M M + M K M + M M K) of the staged field at this thread's cell.
__device__ inline double qlap(QLds &L, const QW &F)
{
    qpasses<true>(L, F.K, F.M);
    const int t = threadIdx.x;
    const int o = (t % QB) + QB * ((t / QB) % QB + QB * (t / (QB * QB)));
    double out = 0.0;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const int q = o + QB * QB * c;
        out += F.M.w[c] * (L.p[0][q] + L.p[1][q]) + F.K.w[c] * L.p[2][q];
    }
    return out;
}

// rho, mu, grad C in derivative units and the unit normals, quadratic filters.
__global__ __launch_bounds__(QT) void props2_kernel(Grid g, Phys P, const QW F, const double *C, double *rho,
                                                    double *mu, F3 Cd, F3 nrm)
{
    __shared__ QLds L;
    const BCell X = bcell(g);
    const size_t id = X.id;
    double d[4];
    qstage(L, QTap{C, kEven, g}, X.i0, X.j0, X.k0);
    qderiv<true>(L, F, d);
    if (!X.valid) return;
    const double c0 = C[id];
    rho[id] = P.rho_l * c0 + P.rho_g * (1.0 - c0);
    mu[id] = P.mu_l * c0 + P.mu_g * (1.0 - c0);
    double gd[3];
    for (int e = 0; e < 3; ++e) gd[e] = d[e] / F.ml;
    const double l = sqrt(gd[0] * gd[0] + gd[1] * gd[1] + gd[2] * gd[2]);
    const double eps = 1e-7 / g.h;
    for (int e = 0; e < 3; ++e) {
        Cd.p[e][id] = gd[e];
        nrm.p[e][id] = gd[e] / (eps + l);
    }
}

// Curvature div n and the surface-tension vectors, quadratic filters.
__global__ __launch_bounds__(QT) void surface2_kernel(Grid g, const QW F, double sigma, C3 nrm, C3 Cd, F3 st)
{
    __shared__ QLds L;
    const BCell X = bcell(g);
    double kap = 0.0;
    for (int e = 0; e < 3; ++e) {
        double d[4];
        qstage(L, QTap{nrm.p[e], rule_grad(e), g}, X.i0, X.j0, X.k0);
        qderiv<true>(L, F, d);
        kap += d[e];
    }
    kap /= F.ml;
    if (!X.valid) return;
    for (int e = 0; e < 3; ++e) st.p[e][X.id] = sigma * kap * Cd.p[e][X.id];
}

// adv_c = q . grad q_c, quadratic filters.
__global__ __launch_bounds__(QT) void advection2_kernel(Grid g, const QW F, C3 q, F3 adv)
{
    __shared__ QLds L;
    const BCell X = bcell(g);
    const size_t id = X.id;
    const double q0[3] = {q.p[0][id], q.p[1][id], q.p[2][id]};
    for (int c = 0; c < 3; ++c) {
        double d[4];
        qstage(L, QTap{q.p[c], rule_vel(c), g}, X.i0, X.j0, X.k0);
        qderiv<true>(L, F, d);
        if (X.valid) adv.p[c][id] = q0[0] * (d[0] / F.ml) + q0[1] * (d[1] / F.ml) + q0[2] * (d[2] / F.ml);
    }
}

// Isotropic PG diffusivity of each component, quadratic filters (the residual
// filter of Eq. a_psi is w_m / m_l - E with the quadratic mass).
__global__ __launch_bounds__(QT) void pg_velocity2_kernel(Grid g, const QW F, C3 q, C3 adv, const double *rho,
                                                          const double *mu, F3 kq)
{
    __shared__ QLds L;
    const BCell X = bcell(g);
    const size_t id = X.id;
    const double eps_k = 1e-7, a_kabs = 1.0 / 16.0, a_ksq = 4.0, h = g.h;
    const double u = q.p[0][id], v = q.p[1][id], w = q.p[2][id];
    for (int c = 0; c < 3; ++c) {
        double d[4], am[4];
        qstage(L, QTap{q.p[c], rule_vel(c), g}, X.i0, X.j0, X.k0);
        qderiv<true>(L, F, d);
        const double px = d[0] / F.ml, py = d[1] / F.ml, pz = d[2] / F.ml;
        qstage(L, QTap{adv.p[c], kEven, g}, X.i0, X.j0, X.k0);
        qderiv<false>(L, F, am);
        const double a = 2.0 * (am[3] / F.ml - adv.p[c][id]);
        const double G = fabs(px) + fabs(py) + fabs(pz);
        const double kabs = a_kabs * h * fabs(a) / (eps_k + G / 3.0);
        const double g2 = px * px + py * py + pz * pz;
        const double advabs = fabs(u * px) + fabs(v * py) + fabs(w * pz);
        const double ksq = a_ksq * a * a * h / (eps_k + advabs / 3.0 * g2);
        const double kmax = h * (fabs(u) + fabs(v) + fabs(w));
        const double m = fmin(kmax, fmin(kabs, ksq));
        if (X.valid) kq.p[c][id] = rho[id] * m + mu[id];
    }
}

// One predictor iteration with the quadratic filters: s_c = rho m_l adv_c +
// f_lap(q_c, k_c) + f(p_hs + p_nh; w_c) + f(s_t,c; w_m) [- f(-g rho; w_m) for
// c = z], the same residual as momentum_lds_kernel; 15 filters per cell.
__global__ __launch_bounds__(QT) void momentum2_kernel(Grid g, Phys P, const QW F, C3 qn, const double *p_hs,
                                                       const double *p_nh, const double *rho, C3 qh, C3 kq, C3 st,
                                                       C3 adv, F3 qt, F3 qnext)
{
    __shared__ QLds L;
    const BCell X = bcell(g);
    const size_t id = X.id;
    const int i0 = X.i0, j0 = X.j0, k0 = X.k0;
    const double r0 = rho[id];
    double ghs[4], gnh[4], rm[4];
    // each field's loads are issued before the previous field's passes
    const QPhs fphs{p_hs, rho, g, P.g * g.h};
    const QTap fnh{p_nh, kOddTop, g}, frho{rho, kEven, g};
    {
        QNext<QPhs> n0;
        n0.fetch(fphs, i0, j0, k0);
        n0.commit(L, fphs);
    }
    {
        QNext<QTap> n1;
        n1.fetch(fnh, i0, j0, k0);
        qderiv<true>(L, F, ghs);
        n1.commit(L, fnh);
    }
    {
        QNext<QTap> n2;
        n2.fetch(frho, i0, j0, k0);
        qderiv<true>(L, F, gnh);
        n2.commit(L, frho);
    }
    using TM = QMul<QTap, QTap>;
    {
        const TM m0{QTap{kq.p[0], kEven, g}, QTap{qh.p[0], rule_vel(0), g}};
        QNext<TM> n3;
        n3.fetch(m0, i0, j0, k0);
        qderiv<false>(L, F, rm);
        n3.commit(L, m0);
    }
    const double buoy = -P.g * rm[3];  // f(-g rho; w_m)
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        const QTap tq{qh.p[c], rule_vel(c), g}, tk{kq.p[c], kEven, g}, ts{st.p[c], rule_grad(c), g};
        const double q0 = qh.p[c][id], kc = kq.p[c][id];
        // Eq. k-T: 1/2 [f(k q; w) + k f(q; w) - q f(k; w)]; f(k q) is staged
        double lkq, lq, lk;
        {
            QNext<QTap> n;
            n.fetch(tq, i0, j0, k0);
            lkq = qlap(L, F);
            n.commit(L, tq);
        }
        {
            QNext<QTap> n;
            n.fetch(tk, i0, j0, k0);
            lq = qlap(L, F);
            n.commit(L, tk);
        }
        {
            QNext<QTap> n;
            n.fetch(ts, i0, j0, k0);
            lk = qlap(L, F);
            n.commit(L, ts);
        }
        double s = 0.5 * (lkq + kc * lq - q0 * lk);
        s += ghs[c];
        s += gnh[c];
        double t4[4];
        {
            // the next component's product field
            const int cn = c < 2 ? c + 1 : c;
            const TM mn{QTap{kq.p[cn], kEven, g}, QTap{qh.p[cn], rule_vel(cn), g}};
            QNext<TM> n;
            if (c < 2) n.fetch(mn, i0, j0, k0);
            qderiv<false>(L, F, t4);
            if (c < 2) n.commit(L, mn);
        }
        s += t4[3];
        if (c == 2) s -= buoy;
        s += r0 * F.ml * adv.p[c][id];
        const double qnc = qn.p[c][id];
        const double tt = (-s / F.ml + r0 * qnc / P.dt) / (r0 / P.dt);
        if (X.valid) {
            qt.p[c][id] = tt;
            qnext.p[c][id] = 0.5 * (qnc + tt);
        }
    }
}

// Volume-fraction diffusivities with the quadratic advection residual and the
// detectors of Eqs. Sx-quad..Sz-quad (the smallest of three products of
// successive differences along each axis).
__global__ __launch_bounds__(QT) void pg_volume_fraction2_kernel(Grid g, const QW F, double dt, const double *C,
                                                                 C3 Cd, C3 q, const double *advc, F3 kd)
{
    __shared__ QLds L;
    const BCell X = bcell(g);
    const size_t id = X.id;
    const int i = X.i, j = X.j, k = X.k;
    const double Kp = 300.0, Km = 300.0, beta = 0.1, eps_x = 1e-4, Kpos = 3.0, eps_k = 1e-7, h = g.h;
    const double kmin = 1e-4 / dt * h * h, kclamp = 0.05 / dt * h * h;
    double am[4];
    qstage(L, QTap{advc, kEven, g}, X.i0, X.j0, X.k0);
    qderiv<false>(L, F, am);
    if (!X.valid) return;
    const double a = 2.0 * (am[3] / F.ml - advc[id]);
    const Tap2 tc{C, kEven, g};
    const double c0 = C[id];
    double S[3];
    for (int d = 0; d < 3; ++d) {
        double c[5];
        for (int o = -2; o <= 2; ++o)
            c[o + 2] = tc(i + (d == 0 ? o : 0), j + (d == 1 ? o : 0), k + (d == 2 ? o : 0));
        S[d] = (c[2] - c[1]) * (c[3] - c[2]);
        const double s1 = (c[1] - c[0]) * (c[2] - c[1]), s3 = (c[3] - c[2]) * (c[4] - c[3]);
        if (s1 < S[d]) S[d] = s1;
        if (s3 < S[d]) S[d] = s3;
    }
    if (c0 > 0.95 || c0 < 0.05) S[0] = S[1] = S[2] = -1.0;
    const double cx = Cd.p[0][id], cy = Cd.p[1][id], cz = Cd.p[2][id];
    const double u = q.p[0][id], v = q.p[1][id], w = q.p[2][id];
    const double g2 = cx * cx + cy * cy + cz * cz;
    const double proj = (u * cx + v * cy + w * cz) / (eps_x + g2);
    const double us = cx * proj, vs = cy * proj, ws = cz * proj;
    const double kneg = -beta * (u * u + v * v + w * w) / (eps_x + g2 * (fabs(us) + fabs(vs) + fabs(ws)) / 3.0);
    const double G = fabs(cx) + fabs(cy) + fabs(cz);
    const double kabs = (1.0 / 16.0) * h * fabs(a) / (eps_k + G / 3.0);
    for (int d = 0; d < 3; ++d) {
        const double wp = -fmax(-1.0, fmin(0.0, Kp * S[d]));
        const double wm = fmin(1.0, fmax(0.0, Km * S[d]));
        const double kk = wp * (Kpos * kabs) + wm * (kneg / h);
        kd.p[d][id] = fmax(-kmin, fmin(kclamp, kk));
    }
}

C3 c3(double *const p[3]) { return C3{{p[0], p[1], p[2]}}; }
F3 f3(double *const p[3]) { return F3{{p[0], p[1], p[2]}}; }

}  // namespace

// ------------------------------------------------------------------ host side

struct nn4mg_stepper {
    Grid g{};
    nn4mg_step_params p{};
    hipStream_t s = nullptr;
    nn4mg_t P = nullptr;       // constant-coefficient pressure hierarchy
    double *mem = nullptr;     // all work fields, one allocation
    double *rho, *mu, *Cd[3], *nrm[3], *st[3], *b, *px, *qa[3], *qb[3], *qt[3], *adv[3], *kq[3], *tmp;
    double *red = nullptr;     // per-block partials of sum C, then the volume (last entry)
    int nred = 0;
    hipEvent_t ev[4]{};        // step start / end, solve start / end
    // the step's solves are enqueued without waiting: per solve a start/end
    // event pair and a pinned slot for its state header, read after the step
    static constexpr int kSolves = 8;  // 1 + n_corr <= 8
    hipEvent_t sev[2 * kSolves]{};
    unsigned char *hdr = nullptr;
    bool pending[kSolves]{};
};

namespace {

constexpr int kFields = 29;

int hip_fail(hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(NN4MG_EDEVICE, m.c_str());
}

#define STEP_TRY(expr, what)                          \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

dim3 cells_grid(const Grid &g) { return dim3((unsigned)((g.n + 255) / 256)); }
dim3 mom_grid(const Grid &g)
{
    return dim3((unsigned)(((g.nx + MT_X - 1) / MT_X) * ((g.ny + MT_Y - 1) / MT_Y) * ((g.nz + MT_Z - 1) / MT_Z)));
}

// Fixed-cycle solve of A x = b on the pressure hierarchy; the work pair
// (b, px) is the same for every solve, so a captured cycle stays valid.  The
// solve is enqueued with nothing waited for on the host (its status, residual
// and time are read by collect_solves after the step); hierarchies that need
// the host inside the solve (singular ones) take the synchronous solve.
int pressure_solve(nn4mg_stepper *S, int slot, int cycles, nn4mg_step_info *info, float *ms_mg)
{
    STEP_TRY(hipEventRecord(S->sev[2 * slot], S->s), "hipEventRecord");
    int rc = solve_fixed_enqueue(S->P, S->b, S->px, cycles, S->hdr + (size_t)slot * solve_header_bytes());
    if (rc == NN4MG_OK) {
        STEP_TRY(hipEventRecord(S->sev[2 * slot + 1], S->s), "hipEventRecord");
        S->pending[slot] = true;
        if (info) info->solves = slot + 1;
        return NN4MG_OK;
    }
    if (rc != NN4MG_EINVAL) return rc;
    nn4mg_info si;
    rc = nn4mg_solve(S->P, S->b, S->px, 0.0, cycles, 1, &si);
    if (rc != NN4MG_OK && rc != NN4MG_ENOTCONV) return rc;
    STEP_TRY(hipEventRecord(S->sev[2 * slot + 1], S->s), "hipEventRecord");
    STEP_TRY(hipEventSynchronize(S->sev[2 * slot + 1]), "hipEventSynchronize");
    float ms = 0.0f;
    STEP_TRY(hipEventElapsedTime(&ms, S->sev[2 * slot], S->sev[2 * slot + 1]), "hipEventElapsedTime");
    *ms_mg += ms;
    if (info) {
        info->relres[slot] = si.relres;
        info->solves = slot + 1;
    }
    return NN4MG_OK;
}

// After the step's stream has drained: the status, final residual and device
// time of every solve enqueued without waiting.
int collect_solves(nn4mg_stepper *S, nn4mg_step_info *info, float *ms_mg)
{
    int status = NN4MG_OK;
    for (int slot = 0; slot < nn4mg_stepper::kSolves; ++slot) {
        if (!S->pending[slot]) continue;
        S->pending[slot] = false;
        double relres = 0.0;
        const int rc = solve_fixed_result(S->hdr + (size_t)slot * solve_header_bytes(), &relres);
        if (rc != NN4MG_OK && status == NN4MG_OK) status = rc;
        float ms = 0.0f;
        STEP_TRY(hipEventElapsedTime(&ms, S->sev[2 * slot], S->sev[2 * slot + 1]), "hipEventElapsedTime");
        *ms_mg += ms;
        if (info) info->relres[slot] = relres;
    }
    return status;
}

// sum C h^3 over the grid into S->red[S->nred] (fixed-order block partials)
int enqueue_volume(nn4mg_stepper *S, const double *C)
{
    const double h = S->g.h;
    STEP_TRY(launch_sum_partials(C, S->g.n, nullptr, 1, S->red, S->s), "sum partials");
    STEP_TRY(launch_reduce(S->red, S->nred, h * h * h, S->red + S->nred, S->s), "reduce");
    return NN4MG_OK;
}

int check_params(const nn4mg_step_params *p)
{
    if (!p) return set_error(NN4MG_EINVAL, "params is NULL");
    if (!(p->rho_l > 0.0) || !(p->rho_g > 0.0)) return set_error(NN4MG_EINVAL, "densities must be > 0");
    if (!(p->mu_l >= 0.0) || !(p->mu_g >= 0.0)) return set_error(NN4MG_EINVAL, "viscosities must be >= 0");
    if (!(p->dt > 0.0)) return set_error(NN4MG_EINVAL, "dt must be > 0");
    if (!std::isfinite(p->g) || !std::isfinite(p->sigma_t)) return set_error(NN4MG_EINVAL, "g, sigma_t must be finite");
    if (p->mg_cycles < 1 || p->mg_cycles > 511) return set_error(NN4MG_EINVAL, "mg_cycles must be in [1, 511]");
    if (p->mg_cycles_nh < 0 || p->mg_cycles_nh > 511) return set_error(NN4MG_EINVAL, "mg_cycles_nh must be in [0, 511]");
    if (p->order < 0 || p->order > 2) return set_error(NN4MG_EINVAL, "order must be 0, 1 or 2");
    for (int i = 0; i < 3; ++i)
        if (p->reserved[i] != 0) return set_error(NN4MG_EINVAL, "reserved fields must be zero");
    if (p->n_corr < 0 || p->n_corr > 7) return set_error(NN4MG_EINVAL, "n_corr must be in [0, 7]");
    if (p->n_vel_iter < 1 || p->n_vel_iter > 64) return set_error(NN4MG_EINVAL, "n_vel_iter must be in [1, 64]");
    return NN4MG_OK;
}

}  // namespace

extern "C" {

void nn4mg_step_params_default(nn4mg_step_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->rho_l = 1000.0;
    p->rho_g = 1.0;
    p->mu_l = 1e-3;
    p->mu_g = 1.8e-5;
    p->g = 9.81;
    p->sigma_t = 0.07;
    p->dt = 1e-4;
    p->mg_cycles = 20;
    p->n_corr = 2;
    p->n_vel_iter = 2;
}

int nn4mg_step_destroy(nn4mg_step_t S)
{
    if (!S) return NN4MG_OK;
    if (S->s) (void)hipStreamSynchronize(S->s);
    else (void)hipDeviceSynchronize();
    if (S->P) nn4mg_destroy(S->P);
    if (S->mem) (void)hipFree(S->mem);
    if (S->red) (void)hipFree(S->red);
    for (auto &e : S->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : S->sev)
        if (e) (void)hipEventDestroy(e);
    if (S->hdr) (void)hipHostFree(S->hdr);
    delete S;
    return NN4MG_OK;
}

int nn4mg_step_create(int nx, int ny, int nz, double h, const nn4mg_step_params *p, void *hip_stream,
                      nn4mg_step_t *out)
{
    if (!out) return set_error(NN4MG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    if (nx < 4 || ny < 4 || nz < 4) return set_error(NN4MG_EINVAL, "grid dims must be >= 4");
    // the quadratic filters index a cell's neighbourhood with 32-bit offsets
    if ((double)nx * ny * nz >= 2147483648.0) return set_error(NN4MG_EINVAL, "grid must have fewer than 2^31 cells");
    if (!(h > 0.0)) return set_error(NN4MG_EINVAL, "h must be > 0");
    // pressure: zero-normal-derivative walls, zero pressure on the top outlet
    nn4mg_config cfg;
    nn4mg_config_default(&cfg, nx, ny, nz, h);
    for (int f = 0; f < 5; ++f) cfg.bc[f] = NN4MG_BC_NEUMANN0;
    cfg.bc[5] = NN4MG_BC_DIRICHLET0;
    nn4mg_stepper *S = new nn4mg_stepper();
    S->g = Grid{nx, ny, nz, h, (size_t)nx * ny * nz};
    S->p = *p;
    S->s = (hipStream_t)hip_stream;
    if ((rc = nn4mg_setup(&cfg, nullptr, hip_stream, &S->P))) {
        S->P = nullptr;
        nn4mg_step_destroy(S);
        return rc;
    }
    const size_t n = S->g.n;
    hipError_t e = hipMalloc((void **)&S->mem, (size_t)kFields * n * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        S->mem = nullptr;
        nn4mg_step_destroy(S);
        return set_error(NN4MG_ENOMEM, "step work fields: hipMalloc failed");
    }
    double *q = S->mem;
    auto take = [&]() {
        double *r = q;
        q += n;
        return r;
    };
    S->rho = take();
    S->mu = take();
    for (int d = 0; d < 3; ++d) S->Cd[d] = take();
    for (int d = 0; d < 3; ++d) S->nrm[d] = take();
    for (int d = 0; d < 3; ++d) S->st[d] = take();
    S->b = take();
    S->px = take();
    for (int d = 0; d < 3; ++d) S->qa[d] = take();
    for (int d = 0; d < 3; ++d) S->qb[d] = take();
    for (int d = 0; d < 3; ++d) S->qt[d] = take();
    for (int d = 0; d < 3; ++d) S->adv[d] = take();
    for (int d = 0; d < 3; ++d) S->kq[d] = take();
    S->tmp = take();
    S->nred = sum_blocks(n);
    if ((e = hipMalloc((void **)&S->red, (size_t)(S->nred + 1) * sizeof(double))) != hipSuccess) {
        (void)hipGetLastError();
        S->red = nullptr;
        nn4mg_step_destroy(S);
        return set_error(NN4MG_ENOMEM, "step reduction buffer: hipMalloc failed");
    }
    for (auto &ev : S->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) {
            ev = nullptr;
            nn4mg_step_destroy(S);
            return hip_fail(e, "hipEventCreate");
        }
    for (auto &ev : S->sev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) {
            ev = nullptr;
            nn4mg_step_destroy(S);
            return hip_fail(e, "hipEventCreate");
        }
    if ((e = hipHostMalloc((void **)&S->hdr, nn4mg_stepper::kSolves * solve_header_bytes(), hipHostMallocDefault)) !=
        hipSuccess) {
        (void)hipGetLastError();
        S->hdr = nullptr;
        nn4mg_step_destroy(S);
        return set_error(NN4MG_ENOMEM, "step solve headers: hipHostMalloc failed");
    }
    // launch shapes of the pressure hierarchy, tuned once for this grid on the
    // stepper's own (zeroed) solve pair; every solve of the stepper uses them
    if ((e = launch_fill(S->b, n, 0.0, (hipStream_t)hip_stream)) != hipSuccess ||
        (e = launch_fill(S->px, n, 0.0, (hipStream_t)hip_stream)) != hipSuccess) {
        nn4mg_step_destroy(S);
        return hip_fail(e, "fill");
    }
    if ((rc = nn4mg_autotune(S->P, S->b, S->px, nullptr, 0))) {
        nn4mg_step_destroy(S);
        return rc;
    }
    *out = S;
    return NN4MG_OK;
}

int nn4mg_step(nn4mg_step_t S, double *C, double *u, double *v, double *w, double *p_hs, double *p_nh,
               nn4mg_step_info *info)
{
    if (!S || !C || !u || !v || !w || !p_hs || !p_nh) return set_error(NN4MG_EINVAL, "NULL argument");
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->volume = std::nan("");  // until the step completes
    }
    const Grid g = S->g;
    const nn4mg_step_params &p = S->p;
    const Phys P{p.rho_l, p.rho_g, p.mu_l, p.mu_g, p.g, p.sigma_t, p.dt};
    const hipStream_t s = S->s;
    const dim3 grid = cells_grid(g), blk(256);
    // the block-staged kernels: one workgroup per 8^3 block
    const dim3 bgrid(blocks_of(g)), bblk(SBT);
    const QW qw = quad_weights(g.h);
    double *q[3] = {u, v, w};
    float ms_mg = 0.0f;
    int rc;

    const bool quad = p.order == 2;
    for (bool &pend : S->pending) pend = false;  // nothing left over from a step that failed midway
    STEP_TRY(hipEventRecord(S->ev[0], s), "hipEventRecord");
    if (quad) {
        hipLaunchKernelGGL(props2_kernel, bgrid, bblk, 0, s, g, P, qw, (const double *)C, S->rho, S->mu,
                           f3(S->Cd), f3(S->nrm));
        hipLaunchKernelGGL(surface2_kernel, bgrid, bblk, 0, s, g, qw, p.sigma_t, c3(S->nrm), c3(S->Cd),
                           f3(S->st));
    } else {
        hipLaunchKernelGGL(props_kernel, grid, blk, 0, s, g, P, (const double *)C, S->rho, S->mu, f3(S->Cd),
                           f3(S->nrm));
        hipLaunchKernelGGL(surface_kernel, grid, blk, 0, s, g, p.sigma_t, c3(S->nrm), c3(S->Cd), f3(S->st));
    }

    // Stage 1: hydrostatic + surface-tension pressure, warm-started from p_hs
    hipLaunchKernelGGL(rhs_hydrostatic_kernel, grid, blk, 0, s, g, p.g, c3(S->st), (const double *)S->rho, S->b);
    STEP_TRY(hipGetLastError(), "step kernels");
    STEP_TRY(hipMemcpyAsync(S->px, p_hs, g.n * sizeof(double), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
    if ((rc = pressure_solve(S, 0, p.mg_cycles, info, &ms_mg))) return rc;
    STEP_TRY(hipMemcpyAsync(p_hs, S->px, g.n * sizeof(double), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");

    // Stage 2: velocity predictor iterations, q^ from q^n
    double **cur = S->qa, **nxt = S->qb;
    hipLaunchKernelGGL(copy3_kernel, grid, blk, 0, s, g.n, c3(q), f3(cur));
    for (int it = 0; it < p.n_vel_iter; ++it) {
        if (quad) {
            hipLaunchKernelGGL(advection2_kernel, bgrid, bblk, 0, s, g, qw, c3(cur), f3(S->adv));
            hipLaunchKernelGGL(pg_velocity2_kernel, bgrid, bblk, 0, s, g, qw, c3(cur), c3(S->adv),
                               (const double *)S->rho,
                               (const double *)S->mu, f3(S->kq));
            hipLaunchKernelGGL(momentum2_kernel, bgrid, bblk, 0, s, g, P, qw, c3(q), (const double *)p_hs,
                               (const double *)p_nh, (const double *)S->rho, c3(cur), c3(S->kq), c3(S->st),
                               c3(S->adv), f3(S->qt), f3(nxt));
            double **t = cur;
            cur = nxt;
            nxt = t;
            continue;
        }
        hipLaunchKernelGGL(advection_kernel, bgrid, bblk, 0, s, g, c3(cur), f3(S->adv));
        hipLaunchKernelGGL(pg_velocity_kernel, bgrid, bblk, 0, s, g, c3(cur), c3(S->adv), (const double *)S->rho,
                           (const double *)S->mu, f3(S->kq));
        {
            MomIn in;
            in.u[0] = p_hs;
            in.u[1] = p_nh;
            in.u[2] = S->rho;
            for (int c = 0; c < 3; ++c) {
                in.u[3 + c] = cur[c];
                in.u[6 + c] = S->kq[c];
                in.u[9 + c] = S->st[c];
            }
            hipLaunchKernelGGL(momentum_lds_kernel, mom_grid(g), dim3(MT_X * MT_Y), 0, s, g, P, c3(q), in,
                               c3(S->adv), f3(S->qt), f3(nxt));
        }
        double **t = cur;
        cur = nxt;
        nxt = t;
    }
    STEP_TRY(hipGetLastError(), "step kernels");

    // Stage 3: non-hydrostatic corrections; the corrected velocity lands in q
    double **qin = S->qt;
    for (int it = 0; it < p.n_corr; ++it) {
        hipLaunchKernelGGL(rhs_nonhydrostatic_kernel, grid, blk, 0, s, g, p.dt, c3(qin), (const double *)S->rho,
                           S->b);
        STEP_TRY(launch_fill(S->px, g.n, 0.0, s), "fill");
        if ((rc = pressure_solve(S, 1 + it, p.mg_cycles_nh > 0 ? p.mg_cycles_nh : p.mg_cycles, info, &ms_mg)))
            return rc;
        hipLaunchKernelGGL(correct_kernel, grid, blk, 0, s, g, p.dt, (const double *)S->px, (const double *)S->rho,
                           c3(qin), f3(q), p_nh);
        qin = q;
    }
    if (p.n_corr == 0) hipLaunchKernelGGL(copy3_kernel, grid, blk, 0, s, g.n, c3(S->qt), f3(q));

    // Stage 4: volume fraction with the new velocity
    hipLaunchKernelGGL(advection_c_kernel, grid, blk, 0, s, g, c3(q), c3(S->Cd), S->tmp);
    if (quad)
        hipLaunchKernelGGL(pg_volume_fraction2_kernel, bgrid, bblk, 0, s, g, qw, p.dt, (const double *)C,
                           c3(S->Cd), c3(q), (const double *)S->tmp, f3(S->kq));
    else
        hipLaunchKernelGGL(pg_volume_fraction_kernel, grid, blk, 0, s, g, p.dt, (const double *)C, c3(S->Cd), c3(q),
                           (const double *)S->tmp, f3(S->kq));
    hipLaunchKernelGGL(volume_fraction_kernel, grid, blk, 0, s, g, p.dt, (const double *)C, c3(S->kq), c3(q),
                       c3(S->Cd), S->b);
    STEP_TRY(hipMemcpyAsync(C, S->b, g.n * sizeof(double), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
    STEP_TRY(hipGetLastError(), "step kernels");
    STEP_TRY(hipEventRecord(S->ev[1], s), "hipEventRecord");
    // the volume of fluid after the step, sum C h^3 (the integral of C^{n+1})
    double vol = 0.0;
    if ((rc = enqueue_volume(S, C))) return rc;
    STEP_TRY(hipMemcpyAsync(&vol, S->red + S->nred, sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    STEP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    if ((rc = collect_solves(S, info, &ms_mg))) return rc;
    if (info) {
        float ms = 0.0f;
        STEP_TRY(hipEventElapsedTime(&ms, S->ev[0], S->ev[1]), "hipEventElapsedTime");
        info->ms_total = ms;
        info->ms_mg = ms_mg;
        info->volume = vol;
    }
    if (!std::isfinite(vol)) return set_error(NN4MG_EBREAKDOWN, "non-finite volume fraction after the step");
    return NN4MG_OK;
}

int nn4mg_step_run(nn4mg_step_t S, int nsteps, double *C, double *u, double *v, double *w, double *p_hs, double *p_nh,
                   double *volume, int *steps_done, nn4mg_step_info *info)
{
    if (!S || !C || !u || !v || !w || !p_hs || !p_nh) return set_error(NN4MG_EINVAL, "NULL argument");
    if (nsteps < 0) return set_error(NN4MG_EINVAL, "nsteps must be >= 0");
    if (steps_done) *steps_done = 0;
    int rc;
    if (volume) {
        if ((rc = enqueue_volume(S, C))) return rc;
        STEP_TRY(hipMemcpyAsync(volume, S->red + S->nred, sizeof(double), hipMemcpyDeviceToHost, S->s),
                 "hipMemcpyAsync");
        STEP_TRY(hipStreamSynchronize(S->s), "hipStreamSynchronize");
    }
    nn4mg_step_info si;
    for (int n = 0; n < nsteps; ++n) {
        rc = nn4mg_step(S, C, u, v, w, p_hs, p_nh, &si);
        if (info) *info = si;
        if (volume && (rc == NN4MG_OK || rc == NN4MG_EBREAKDOWN)) volume[n + 1] = si.volume;  // NaN if it stopped early
        if (rc) return rc;
        if (steps_done) *steps_done = n + 1;
    }
    return NN4MG_OK;
}

}  // extern "C"
