"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them re-types the oracle's own formula:
they use values printed in the paper (tests/golden/), closed forms, invariants,
brute force on tiny grids and library routines on independently assembled
matrices (tests/indep.py).
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from paper_2401_06755_amd import inputs
from tests import indep

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
D, N, P = 0, 1, 2


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def _grid_coords(shape_xyz, h):
    nx, ny, nz = shape_xyz
    x = ((np.arange(nx) + 0.5) * h)[None, None, :]
    y = ((np.arange(ny) + 0.5) * h)[None, :, None]
    z = ((np.arange(nz) + 0.5) * h)[:, None, None]
    return np.broadcast_arrays(x, y, z)


# --------------------------------------------------------------------------
# P1: filter weights and the tensor-product convention
# --------------------------------------------------------------------------

def test_p1_printed_wx_is_derivative_times_mass_times_mass():
    """The printed linear w_x (Sec. 2.2.3) equals (1/2)[-1,0,1] (x) M (x) M with
    M = (h/6)[1,4,1], in units m_l/(72 dx) = h^2/72."""
    g = _read_golden("wx_linear_filter.txt").reshape(3, 3, 3)  # [z][y][x]
    h = 0.37
    M = np.array([1.0, 4.0, 1.0]) * h / 6.0
    Dx = np.array([-1.0, 0.0, 1.0]) / 2.0
    built = np.einsum("c,b,a->cba", M, M, Dx)
    np.testing.assert_allclose(built, g * h ** 2 / 72.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("h", [1.0, 1 / 64, 0.3])
def test_p1_q1_laplacian_equals_tensor_product_stiffness(h):
    w = oracle.q1_filter(h)
    np.testing.assert_allclose(w, indep.q1_tensor_filter(h), rtol=1e-15, atol=1e-15 * h)
    assert abs(w.sum()) < 1e-15


def test_fig1_worked_example_orientation():
    """Fig. 1: Y33 = 4 C33 - (C32 + C34 + C23 + C43) with the 2D FD filter;
    pins the offset convention of the filter sum f(C; w)."""
    fd = _read_golden("fig1_fd_example.txt")
    w = np.zeros((3, 3, 3))
    w[1] = fd  # the 2D filter in the z = 0 slice
    rng = np.random.default_rng(0)
    C = rng.standard_normal((7, 7))  # C[j][i], i, j = 0..6 incl. halo
    up = np.zeros((3, 7, 7))
    up[1] = C
    Y = oracle.filter_apply(up, w)[0]  # interior 5x5, Y[j-1][i-1]
    expect = 4 * C[3, 3] - (C[2, 3] + C[4, 3] + C[3, 2] + C[3, 4])
    assert abs(Y[2, 2] - expect) < 1e-14
    # an asymmetric filter to pin the direction of each offset
    w2 = np.zeros((3, 3, 3))
    w2[1, 1, 2] = 1.0  # +x neighbour
    w2[1, 0, 1] = 10.0  # -y neighbour
    w2[2, 1, 1] = 100.0  # +z neighbour
    up3 = rng.standard_normal((5, 6, 7))
    Y3 = oracle.filter_apply(up3, w2)
    k, j, i = 1, 2, 3
    assert abs(Y3[k, j, i] - (up3[k + 1, j + 1, i + 2] + 10 * up3[k + 1, j, i + 1] + 100 * up3[k + 2, j + 1, i + 1])) < 1e-13


# --------------------------------------------------------------------------
# P2: polynomial exactness away from the boundary
# --------------------------------------------------------------------------

def test_p2_polynomials_interior():
    n, h = 12, 1.0 / 12
    X, Y, Z = _grid_coords((n, n, n), h)
    bc = (D,) * 6
    inner = (slice(1, -1),) * 3

    def A(u):
        return oracle.apply(u, h, bc)[inner]

    assert np.max(np.abs(A(np.ones((n, n, n))))) < 1e-15
    assert np.max(np.abs(A(X))) < 1e-15
    assert np.max(np.abs(A(X * Y * Z))) < 1e-15
    np.testing.assert_allclose(A(X ** 2), -2 * h ** 3, rtol=1e-10)
    np.testing.assert_allclose(A(Z ** 2), -2 * h ** 3, rtol=1e-10)
    got = A(X ** 2 * Y ** 2)
    want = (-2 * h ** 3 * (X ** 2 + Y ** 2) - 4 * h ** 5 / 3)[inner]
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-18)


# --------------------------------------------------------------------------
# P3: closed-form eigenpairs with the halo boundary rules
# --------------------------------------------------------------------------

KIND = {D: "DD", N: "NN", P: "PP"}


@pytest.mark.parametrize("axes,modes", [
    (("DD", "DD", "DD"), (1, 1, 1)),
    (("DD", "DD", "DD"), (3, 2, 5)),
    (("NN", "NN", "NN"), (1, 0, 2)),
    (("PP", "PP", "PP"), (1, 2, 3)),
    (("DN", "NN", "DD"), (0, 1, 2)),
    (("DD", "PP", "DN"), (2, 1, 1)),
])
def test_p3_eigenpairs(axes, modes):
    n = 16
    h = 1.0 / n
    lohi = {"DD": (D, D), "NN": (N, N), "PP": (P, P), "DN": (D, N)}
    bc = lohi[axes[0]] + lohi[axes[1]] + lohi[axes[2]]
    ux, tx = indep.eig1d(axes[0], modes[0], n)
    uy, ty = indep.eig1d(axes[1], modes[1], n)
    uz, tz = indep.eig1d(axes[2], modes[2], n)
    u = uz[:, None, None] * uy[None, :, None] * ux[None, None, :]
    lam = indep.q1_eigenvalue(h, (tx, ty, tz))
    np.testing.assert_allclose(oracle.apply(u, h, bc), lam * u, rtol=0, atol=1e-14 * max(lam, h))


def test_p3_eigenvalue_values():
    """Closed-form values at the sizes used in the parity/benchmark cases."""
    lam64 = indep.q1_eigenvalue(1 / 64, [np.pi / 64] * 3)
    assert abs(lam64 - 1.1283531611073057e-4) < 1e-18
    u, t = indep.eig1d("DD", 1, 64)
    U = u[:, None, None] * u[None, :, None] * u[None, None, :]
    AU = oracle.apply(U, 1 / 64, (D,) * 6)
    np.testing.assert_allclose(AU, lam64 * U, atol=1e-15)
    # checkerboard (theta = pi on each axis): lambda = 4h/3
    assert abs(indep.q1_eigenvalue(0.25, [np.pi] * 3) - 4 * 0.25 / 3) < 1e-15


# --------------------------------------------------------------------------
# P4: whole operator incl. boundary folding, brute force on tiny grids
# --------------------------------------------------------------------------

BCS_TINY = [
    (D, D, D, D, D, D),
    (N, N, N, N, N, N),
    (P, P, P, P, P, P),
    (D, N, N, D, P, P),
    (N, N, N, N, N, D),
]


@pytest.mark.parametrize("bc", BCS_TINY)
@pytest.mark.parametrize("dims", [(3, 4, 2), (4, 4, 4)])
def test_p4_dense_equals_fe_assembly(bc, dims):
    nx, ny, nz = dims
    h = 0.25
    A_or = oracle.dense(dims, h, bc)
    A_fe = indep.fe_assembled_matrix(nx, ny, nz, h, bc)
    np.testing.assert_allclose(A_or, A_fe, rtol=0, atol=1e-15)
    np.testing.assert_allclose(A_or, A_or.T, atol=1e-16)
    ev = np.linalg.eigvalsh(A_or)
    if any(b == D for b in bc):
        assert ev.min() > 0
    else:
        assert abs(ev.min()) < 1e-14 and ev[1] > 1e-6
        np.testing.assert_allclose(A_or @ np.ones(A_or.shape[0]), 0, atol=1e-15)


@pytest.mark.parametrize("bc", BCS_TINY)
def test_p4_kron_construction_matches(bc):
    dims = (5, 4, 6)
    h = 0.2
    A_or = oracle.dense(dims, h, bc)
    A_kr = indep.kron_matrix(*dims, h, bc).toarray()
    np.testing.assert_allclose(A_or, A_kr, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# P5: variable coefficient, Eq. (k-T)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bc", BCS_TINY)
def test_p5_kT_equals_link_form(bc):
    rng = np.random.default_rng(5)
    shape = (5, 4, 6)  # (nz, ny, nx)
    k = np.exp(rng.uniform(-3, 3, size=shape))
    x = rng.standard_normal(shape)
    h = 0.125
    got = oracle.apply(x, h, bc, k)
    want = (indep.link_matrix(k, h, bc) @ x.reshape(-1)).reshape(shape)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())


def test_p5_constant_k_and_nullspace_and_symmetry():
    rng = np.random.default_rng(6)
    shape = (4, 3, 5)
    h = 0.5
    x = rng.standard_normal(shape)
    bc = (N, N, D, N, P, P)
    np.testing.assert_allclose(oracle.apply(x, h, bc, np.full(shape, 3.5)), 3.5 * oracle.apply(x, h, bc),
                               rtol=1e-13, atol=1e-14)
    k = np.exp(rng.uniform(-2, 2, size=shape))
    bcn = (N,) * 6
    np.testing.assert_allclose(oracle.apply(np.ones(shape), h, bcn, k), 0, atol=1e-14)
    A = oracle.dense((5, 3, 4), h, bc, k)
    np.testing.assert_allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0


def test_p5_linear_coefficient_closed_form():
    """k = a + beta x, u = x: -div(k grad u) = -beta, volume-integrated -beta h^3
    (interior cells); k = a + beta y, u = x gives 0."""
    n, h = 10, 0.1
    X, Y, _ = _grid_coords((n, n, n), h)
    inner = (slice(1, -1),) * 3
    a, beta = 2.0, 0.7
    y1 = oracle.apply(np.ascontiguousarray(X), h, (D,) * 6, np.ascontiguousarray(a + beta * X))[inner]
    np.testing.assert_allclose(y1, -beta * h ** 3, rtol=1e-9)
    y2 = oracle.apply(np.ascontiguousarray(X), h, (D,) * 6, np.ascontiguousarray(a + beta * Y))[inner]
    assert np.max(np.abs(y2)) < 1e-15


# --------------------------------------------------------------------------
# P6: weighted Jacobi
# --------------------------------------------------------------------------

def test_p6_jacobi_mode_decay():
    n = 64
    h = 1.0 / n
    u, t = indep.eig1d("DD", 1, n)
    U = u[:, None, None] * u[None, :, None] * u[None, None, :]
    lam = indep.q1_eigenvalue(h, [t] * 3)
    factor = 1 - (2 / 3) * lam / (8 * h / 3)
    assert abs(factor - 0.9981946349422283) < 1e-15
    y = oracle.jacobi(np.zeros_like(U), U, h, (D,) * 6, nsweeps=2)
    np.testing.assert_allclose(y, factor ** 2 * U, atol=1e-14)


def test_p6_jacobi_checkerboard_and_variable_diag():
    n = 8
    h = 1.0 / n
    i = np.arange(n)
    cb = (-1.0) ** (i[:, None, None] + i[None, :, None] + i[None, None, :])
    y = oracle.jacobi(np.zeros_like(cb), cb, h, (P,) * 6, nsweeps=1)
    np.testing.assert_allclose(y, (2 / 3) * cb, atol=1e-14)
    d = oracle.diag((n, n, n), h, (P,) * 6, np.full((n, n, n), 2.5))
    np.testing.assert_allclose(d, 2.5 * 8 * h / 3, rtol=1e-14)


# --------------------------------------------------------------------------
# P7 / P8: grid transfers
# --------------------------------------------------------------------------

def test_p7_restriction_sum_and_ones():
    rng = np.random.default_rng(7)
    r = rng.standard_normal((6, 4, 8))
    rc = oracle.restrict(r)
    assert rc.shape == (3, 2, 4)
    assert abs(rc.sum() - r.sum()) < 1e-12
    np.testing.assert_array_equal(oracle.restrict(np.ones((4, 4, 4))), 8.0)
    # one fine cell lands in exactly its parent
    z = np.zeros((4, 6, 8))
    z[3, 2, 5] = 1.0
    rz = oracle.restrict(z)
    assert rz[1, 1, 2] == 1.0 and rz.sum() == 1.0


def test_p8_prolongation_constants_and_linears():
    c = np.full((3, 4, 5), 2.0)
    np.testing.assert_allclose(oracle.prolong(c, (N,) * 6), 2.0, atol=1e-15)
    np.testing.assert_allclose(oracle.prolong(c, (P,) * 6), 2.0, atol=1e-15)
    H = 0.2
    Xc, Yc, Zc = _grid_coords((5, 4, 3), H)
    lin = 1.0 + 2 * Xc - Yc + 0.5 * Zc
    Xf, Yf, Zf = _grid_coords((10, 8, 6), H / 2)
    pf = oracle.prolong(np.ascontiguousarray(lin), (D,) * 6)
    want = 1.0 + 2 * Xf - Yf + 0.5 * Zf
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(pf[inner], want[inner], atol=1e-14)


def test_p8_prolongation_of_sine_mode_closed_form():
    """Per axis: fine cell 2I+a sits at X_I - H/4 (a=0) or X_I + H/4 (a=1); the
    interpolant of sin(f X) is sin(f X_I)(3/4 + cos(fH)/4) -/+ cos(f X_I) sin(fH)/4.
    Exact at the walls too, since the Dirichlet halo continues the sine oddly."""
    nc = 8
    H = 1.0 / nc
    m = (1, 3, 2)
    Xc = (np.arange(nc) + 0.5) * H
    per_axis = []
    for mm in m:
        f = mm * np.pi
        sgn = np.array([-1.0, 1.0])
        v = (np.sin(f * Xc)[:, None] * (0.75 + 0.25 * np.cos(f * H))
             + sgn[None, :] * np.cos(f * Xc)[:, None] * np.sin(f * H) / 4)
        per_axis.append(v.reshape(-1))  # fine index 2I + a
    ux, uy, uz = (np.sin(mm * np.pi * Xc) for mm in m)
    ec = uz[:, None, None] * uy[None, :, None] * ux[None, None, :]
    want = per_axis[2][:, None, None] * per_axis[1][None, :, None] * per_axis[0][None, None, :]
    np.testing.assert_allclose(oracle.prolong(ec, (D,) * 6), want, atol=1e-14)


def test_coarsen_k_invariants():
    rng = np.random.default_rng(8)
    k = np.exp(rng.uniform(-3, 3, size=(4, 6, 8)))
    kc = oracle.coarsen_k(k)
    assert abs(8 * kc.sum() - k.sum()) < 1e-10 * k.sum()
    np.testing.assert_allclose(oracle.coarsen_k(np.full((2, 2, 2), 3.0)), 3.0)
    np.testing.assert_allclose(oracle.coarsen_k(np.full((2, 2, 2), 3.0), harmonic=True), 3.0)
    kh = oracle.coarsen_k(k, harmonic=True)
    assert np.all(kh <= kc * (1 + 1e-14))  # harmonic <= arithmetic mean


# --------------------------------------------------------------------------
# P9: coarsest solve
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bc", [(D,) * 6, (N, N, N, N, N, D)])
def test_p9_cholesky_solve_matches_numpy(bc):
    A = indep.fe_assembled_matrix(4, 4, 4, 0.25, bc)
    rng = np.random.default_rng(9)
    b = rng.standard_normal(64)
    L = oracle.cholesky(A)
    x = oracle.chol_solve(L, b)
    np.testing.assert_allclose(L @ L.T, A, atol=1e-14)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11, atol=1e-12)
    assert np.linalg.norm(A @ x - b) <= 1e-13 * np.linalg.norm(b)


# --------------------------------------------------------------------------
# P10-P12: the whole solve
# --------------------------------------------------------------------------

def test_p10_sine_rhs_closed_form_solution():
    n = 32
    h = 1.0 / n
    u, t = indep.eig1d("DD", 1, n)
    U = u[:, None, None] * u[None, :, None] * u[None, None, :]
    lam = indep.q1_eigenvalue(h, [t] * 3)
    H = oracle.Hierarchy((n, n, n), h, (D,) * 6)
    assert H.levels == 4 and H.coarse_n == 64
    x, hist, st = H.solve(U, rtol=1e-12, max_cycles=60)
    assert st == 0 and hist[-1] <= 1e-12
    np.testing.assert_allclose(x, U / lam, rtol=0, atol=1e-11 * np.abs(U / lam).max())


@pytest.mark.parametrize("bc", [(D,) * 6, (N, N, N, N, N, D), (D, N, P, P, N, D)])
def test_p10_solve_matches_sparse_direct(bc):
    n = 16
    h = 1.0 / n
    b = inputs.poisson_sine_noise(n, seed=3)["b"]
    H = oracle.Hierarchy((n, n, n), h, bc)
    x, hist, st = H.solve(b, rtol=1e-13, max_cycles=80)
    assert st == 0
    A = indep.kron_matrix(n, n, n, h, bc)
    xd = spla.spsolve(A.tocsc(), b.reshape(-1)).reshape(b.shape)
    np.testing.assert_allclose(x, xd, rtol=0, atol=1e-10 * np.abs(xd).max())


def test_p10_variable_solve_matches_sparse_direct():
    n = 16
    w = inputs.dense_sphere(n, seed=4, radius=0.3)
    bc = (N, N, N, N, N, D)
    H = oracle.Hierarchy(w["shape"], w["h"], bc, k=w["k"])
    x, hist, st = H.solve(w["b"], rtol=1e-12, max_cycles=400)
    assert st == 0
    A = indep.link_matrix(w["k"], w["h"], bc)
    xd = spla.spsolve(A.tocsc(), w["b"].reshape(-1)).reshape(x.shape)
    np.testing.assert_allclose(x, xd, rtol=0, atol=1e-8 * np.abs(xd).max())


def test_p11_cycle_convergence_guard():
    """Regression guard (not a paper value): asymptotic factor of V(0,2) with
    omega = 2/3 on the 32^3 sine+noise Dirichlet problem stays below 0.5."""
    w = inputs.poisson_sine_noise(32, seed=1)
    H = oracle.Hierarchy(w["shape"], w["h"], w["bc"])
    x, hist, st = H.solve(w["b"], rtol=1e-10, max_cycles=60)
    assert st == 0
    rates = hist[1:] / hist[:-1]
    assert np.max(rates[3:]) < 0.5
    assert len(hist) - 1 <= 40


def test_p12_nullspace_zero_mean():
    n = 16
    rng = np.random.default_rng(12)
    k = np.exp(rng.uniform(-2, 2, size=(n, n, n)))
    b = rng.standard_normal((n, n, n)) + 5.0  # non-zero mean: projected away
    H = oracle.Hierarchy((n, n, n), 1.0 / n, (N,) * 6, k=k)
    x, hist, st = H.solve(b, rtol=1e-11, max_cycles=300)
    assert st == 0
    assert abs(x.mean()) <= 1e-14 * np.abs(x).max()
    r = (b - b.mean()) - oracle.apply(x, 1.0 / n, (N,) * 6, k)
    assert np.linalg.norm(r) <= 1.01e-11 * np.linalg.norm(b - b.mean())


def test_fixed_cycle_mode_and_zero_rhs():
    w = inputs.poisson_sine_noise(16, seed=1)
    H = oracle.Hierarchy(w["shape"], w["h"], w["bc"])
    x, hist, st = H.solve(w["b"], max_cycles=5, fixed=True)
    assert st == 0 and len(hist) == 6
    x0, hist0, st0 = H.solve(np.zeros_like(w["b"]), x0=np.ones_like(w["b"]))
    assert st0 == 0 and np.all(x0 == 0) and len(hist0) == 1
    _, histn, stn = H.solve(w["b"], rtol=1e-14, max_cycles=2)
    assert stn == -4 and len(histn) == 3


# --------------------------------------------------------------------------
# Nodal Jacobi diagonal, coefficient coarsening map, the whole V-cycle as
# matrices assembled here from independent pieces
# --------------------------------------------------------------------------

def _pad_coef(k, bc):
    """One-cell halo of a coefficient: nearest interior value (wrap on periodic
    axes), axis by axis; independent of the oracle's padding."""
    out = k
    for ax, (lo, hi) in zip((2, 1, 0), ((bc[0], bc[1]), (bc[2], bc[3]), (bc[4], bc[5]))):
        mode = "wrap" if (lo == P and hi == P) else "edge"
        width = [(0, 0)] * 3
        width[ax] = (1, 1)
        out = np.pad(out, width, mode=mode)
    return out


def _link_diagonal(k, h, bc):
    """Interior Jacobi diagonal of the link form: the sum over the 26 links of
    (-w_s)(k_i + k_{i+s})/2, with the coefficient continued past the walls
    (nodes not folded into the diagonal: the convolutional reading)."""
    nz, ny, nx = k.shape
    kp = _pad_coef(k, bc)
    w = indep.q1_tensor_filter(h)
    d = np.zeros_like(k)
    for c in (-1, 0, 1):
        for b in (-1, 0, 1):
            for a in (-1, 0, 1):
                if (a, b, c) == (0, 0, 0):
                    continue
                kn = kp[1 + c:1 + c + nz, 1 + b:1 + b + ny, 1 + a:1 + a + nx]
                d += -w[c + 1, b + 1, a + 1] * 0.5 * (k + kn)
    return d


@pytest.mark.parametrize("bc", BCS_TINY)
def test_nodal_jacobi_diagonal(bc):
    """The nodal diagonal (Eq. k-T's coefficient of x_i): at cells away from
    every wall it is the diagonal of the link-form matrix; at every cell it is
    the link sum with the coefficient halo.  Dropping or mis-scaling the
    neighbour-k term fails both."""
    rng = np.random.default_rng(61)
    shape = (6, 5, 7)
    h = 0.2
    k = np.exp(rng.uniform(-2, 2, size=shape))
    d = oracle.diag((7, 5, 6), h, bc, k)
    ad = indep.link_matrix(k, h, bc).diagonal().reshape(shape)
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(d[inner], ad[inner], rtol=1e-14)
    np.testing.assert_allclose(d, _link_diagonal(k, h, bc), rtol=1e-14)
    assert np.max(np.abs(d - 8 * h / 3 * k)) > 1e-3 * np.abs(d).max()  # the neighbour term matters


@pytest.mark.parametrize("child", [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)])
def test_coarsen_k_parent_map_single_spike(child):
    """A spike in one fine cell changes exactly its parent: the mean of the
    eight children, or their harmonic mean."""
    a, b, c = child
    k = np.ones((6, 4, 8))
    I, J, K = 2, 1, 1
    k[2 * K + c, 2 * J + b, 2 * I + a] = 9.0
    want = np.ones((3, 2, 4))
    want[K, J, I] = (7.0 + 9.0) / 8.0
    np.testing.assert_array_equal(oracle.coarsen_k(k), want)
    want[K, J, I] = 8.0 / (7.0 + 1.0 / 9.0)
    np.testing.assert_allclose(oracle.coarsen_k(k, harmonic=True), want, rtol=1e-15)


def _agg_matrix(nx, ny, nz):
    """R: coarse cell I collects its 8 children (0/1 entries)."""
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    rows, cols = [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                rows.append(i // 2 + cx * (j // 2 + cy * (k // 2)))
                cols.append(i + nx * (j + ny * k))
    import scipy.sparse as sp
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(cx * cy * cz, nx * ny * nz))


def _prolong1d(nc, lo, hi):
    """1D cell-centred linear interpolation: fine 2I+a takes 3/4 of coarse I and
    1/4 of I-1 (a = 0) or I+1 (a = 1), the neighbour folded by the wall rule."""
    Pm = np.zeros((2 * nc, nc))
    for I in range(nc):
        for a in (0, 1):
            f = 2 * I + a
            Pm[f, I] += 0.75
            m, s = indep._fold_axis(I + (1 if a else -1), nc, lo, hi)
            Pm[f, m] += 0.25 * s
    return Pm


def _vcycle_by_matrices(x, b, dims, h, bc, k, nu, omega=2.0 / 3.0):
    """Sawtooth V(0, nu) written with explicit matrices: restriction of the
    residual down every level, exact coarsest solve (minimum-norm for a
    singular operator), then per level upwards prolongation (+ x at the
    finest) and nu weighted-Jacobi sweeps against the level's right-hand side."""
    import scipy.sparse as sp
    nx, ny, nz = dims
    L = oracle.num_levels(nx, ny, nz)
    A, D, R, Pm, dd = [], [], [], [], []
    kl = k
    for l in range(L):
        d = (nx >> l, ny >> l, nz >> l)
        hl = h * 2 ** l
        dd.append(d)
        if k is None:
            A.append(indep.kron_matrix(*d, hl, bc))
            D.append(np.full(d[0] * d[1] * d[2], 8 * hl / 3))
        else:
            A.append(indep.link_matrix(kl, hl, bc))
            D.append(_link_diagonal(kl, hl, bc).reshape(-1))
            if l + 1 < L:
                kl = kl.reshape(d[2] // 2, 2, d[1] // 2, 2, d[0] // 2, 2).mean(axis=(1, 3, 5))
        if l + 1 < L:
            R.append(_agg_matrix(*d))
            c = (d[0] // 2, d[1] // 2, d[2] // 2)
            Pm.append(sp.csr_matrix(np.kron(_prolong1d(c[2], bc[4], bc[5]),
                                            np.kron(_prolong1d(c[1], bc[2], bc[3]), _prolong1d(c[0], bc[0], bc[1])))))
    xv, bv = x.reshape(-1), b.reshape(-1)
    rhs = [None] * L
    rhs[0] = bv
    if L > 1:
        rhs[1] = R[0] @ (bv - A[0] @ xv)
        for l in range(1, L - 1):
            rhs[l + 1] = R[l] @ rhs[l]
    Ac = A[L - 1].toarray()
    if L == 1:
        return x + (np.linalg.pinv(Ac) @ (bv - A[0] @ xv)).reshape(x.shape)
    e = np.linalg.pinv(Ac) @ rhs[L - 1]
    for l in range(L - 2, -1, -1):
        y = Pm[l] @ e + (xv if l == 0 else 0.0)
        for _ in range(nu):
            y = y + omega * (rhs[l] - A[l] @ y) / D[l]
        e = y
    return e.reshape(x.shape)


@pytest.mark.parametrize("dims,bc,nodal,nu", [
    ((8, 8, 8), (D,) * 6, False, 2),
    ((8, 8, 8), (N, N, N, N, N, D), True, 2),
    ((16, 16, 16), (D, N, P, P, N, D), True, 2),
    ((16, 16, 16), (N,) * 6, True, 2),
    ((24, 16, 16), (D,) * 6, False, 3),
    ((16, 8, 16), (P, P, D, D, N, N), True, 1),
])
def test_vcycle_equals_matrix_cycle(dims, bc, nodal, nu):
    """One oracle V-cycle equals the cycle written with matrices assembled here
    (aggregation R, Kronecker 3/4-1/4 prolongation with wall folding, weighted
    Jacobi with the interior diagonal, exact coarsest solve) at two and three
    levels.  Pre-smoothing, a skipped level, a wrong prolongation target or
    right-hand side fails this."""
    nx, ny, nz = dims
    h = 1.0 / nx
    rng = np.random.default_rng(sum(dims) + nu)
    shape = (nz, ny, nx)
    k = np.exp(rng.uniform(-1, 1, size=shape)) if nodal else None
    x = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    if all(v != D for v in bc):
        b -= b.mean()  # singular operator: a consistent right-hand side
    H = oracle.Hierarchy(dims, h, bc, k=k, nu_post=nu)
    assert H.levels in (2, 3)
    got = H.vcycle(x, b)
    want = _vcycle_by_matrices(x, b, dims, h, bc, k, nu)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


# --------------------------------------------------------------------------
# The FCG(1) outer iteration
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nodal", [False, True])
def test_fcg_identity_preconditioner_is_cg(nodal):
    """With the identity as preconditioner FCG(1) is conjugate gradients: its
    iterates equal scipy's CG iterates on the independently assembled matrix."""
    import scipy.sparse.linalg as spla_

    n = 16
    h = 1.0 / n
    bc = (D, N, N, N, N, D)
    rng = np.random.default_rng(21)
    shape = (n, n, n)
    k = np.exp(rng.uniform(-1, 1, size=shape)) if nodal else None
    b = rng.standard_normal(shape)
    A = indep.link_matrix(k, h, bc) if nodal else indep.kron_matrix(n, n, n, h, bc)
    H = oracle.Hierarchy((n, n, n), h, bc, k=k)
    xs = []
    spla_.cg(A, b.reshape(-1), x0=np.zeros(n ** 3), rtol=0.0, atol=0.0, maxiter=8,
             callback=lambda xk: xs.append(xk.copy()))
    for it in (1, 4, 8):
        x, hist, st = H.fcg(b, max_iter=it, fixed=True, precond=False)
        assert st == 0 and len(hist) == it + 1
        np.testing.assert_allclose(x.reshape(-1), xs[it - 1], rtol=0, atol=1e-11 * np.abs(xs[it - 1]).max())
        r = b.reshape(-1) - A @ x.reshape(-1)
        assert abs(np.linalg.norm(r) / np.linalg.norm(b) - hist[-1]) <= 1e-10 * hist[-1]


@pytest.mark.parametrize("bc", [(D,) * 6, (N,) * 6])
def test_fcg_converges_to_sparse_direct_solution(bc):
    """FCG(1) with the cycle as preconditioner reaches the sparse direct
    solution of the independently assembled system, in fewer iterations than
    the stationary cycle needs."""
    n = 16
    w = inputs.dense_sphere(n, seed=4, radius=0.3)
    b = w["b"] - (w["b"].mean() if bc == (N,) * 6 else 0.0)
    H = oracle.Hierarchy(w["shape"], w["h"], bc, k=w["k"])
    x, hist, st = H.fcg(b, rtol=1e-12, max_iter=200)
    assert st == 0 and hist[-1] <= 1e-12
    _, hs, sts = H.solve(b, rtol=1e-12, max_cycles=2000)
    assert sts == 0 and len(hist) < len(hs)
    A = indep.link_matrix(w["k"], w["h"], bc)
    if bc == (N,) * 6:
        Ad = A.toarray()
        xd = np.linalg.lstsq(Ad, b.reshape(-1), rcond=None)[0]
        xd -= xd.mean()
    else:
        xd = spla.spsolve(A.tocsc(), b.reshape(-1))
    xd = xd.reshape(x.shape)
    np.testing.assert_allclose(x, xd, rtol=0, atol=1e-8 * np.abs(xd).max())
