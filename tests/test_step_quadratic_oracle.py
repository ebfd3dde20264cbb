"""Pins of the quadratic ConvFEM step oracle (Sec. 2.2.3 filters of 5 x 5 x 5,
two-cell halos of Sec. 2.3.3, Table disc_combinations "linear/quadratic":
quadratic filters for the momentum, interface and volume-fraction advection
terms, linear ones for the volume-fraction diffusion; the pressure equations
keep the linear operator of the multigrid).

* The 1D vectors are the average of the assembled rows of the two node types
  of quadratic Lagrange elements, assembled here by Gauss quadrature
  (independent of the oracle's printed values), and the 3D filters their
  tensor products.
* Polynomial exactness in the interior: the derivative filter is exact on
  quartics, the Laplacian filter on quintics, the mass filter on cubics.
* The two-cell halo: a numpy convolution over a field padded by reflection
  (sign per face) reproduces the oracle's filter at every cell.
* Step invariants at order 2: the hydrostatic rest state in closed form (the
  two-cell affine halo of p_hs is exact), y-independence with v = 0, and on a
  periodic box q = 0 leaves C unchanged, a uniform velocity conserves sum C,
  and a periodic shift commutes with the step.
"""
import numpy as np
import pytest

import oracle


def element_matrices(h):
    """Quadratic Lagrange element on [0, 2h] (nodes 0, h, 2h): mass, stiffness,
    and D[a][b] = int N_a N_b' dx, by 4-point Gauss quadrature (exact here)."""
    L = 2 * h
    xg, wg = np.polynomial.legendre.leggauss(4)
    x = (xg + 1) * L / 2
    w = wg * L / 2
    nodes = np.array([0.0, h, 2 * h])
    N, dN = [], []
    for a in range(3):
        others = [nodes[b] for b in range(3) if b != a]
        den = np.prod([nodes[a] - o for o in others])
        N.append((x - others[0]) * (x - others[1]) / den)
        dN.append(((x - others[0]) + (x - others[1])) / den)
    M = np.array([[np.sum(w * N[a] * N[b]) for b in range(3)] for a in range(3)])
    K = np.array([[np.sum(w * dN[a] * dN[b]) for b in range(3)] for a in range(3)])
    D = np.array([[np.sum(w * N[a] * dN[b]) for b in range(3)] for a in range(3)])
    return M, K, D


def convfem_vector(E):
    """Average over the vertex node (last row of the left element at offsets
    -2..0 plus first row of the right element at 0..2) and the mid node
    (middle row at -1..1) of the assembled stencil."""
    vertex = np.zeros(5)
    vertex[0:3] += E[2]
    vertex[2:5] += E[0]
    mid = np.zeros(5)
    mid[1:4] += E[1]
    return 0.5 * (vertex + mid)


@pytest.mark.parametrize("h", [1.0, 0.1, 1 / 48])
def test_quadratic_filters_are_averaged_element_rows(h):
    M, K, D = element_matrices(h)
    M2, K2, G2 = convfem_vector(M), convfem_vector(K), convfem_vector(D)
    wx, wm, wlap = oracle.step_filters_quadratic(h)
    outer = lambda a, b, c: np.einsum("c,b,a->cba", c, b, a)  # x fastest: filter[c, b, a]
    np.testing.assert_allclose(wx, outer(G2, M2, M2), rtol=0, atol=1e-14 * np.abs(wx).max())
    np.testing.assert_allclose(wm, outer(M2, M2, M2), rtol=0, atol=1e-14 * np.abs(wm).max())
    lap = outer(K2, M2, M2) + outer(M2, K2, M2) + outer(M2, M2, K2)
    np.testing.assert_allclose(wlap, lap, rtol=0, atol=1e-14 * np.abs(lap).max())
    # the averaged rows: h/30 [-1 4 24 4 -1], [1 -16 30 -16 1]/(12 h), [1 -8 0 8 -1]/12
    np.testing.assert_allclose(M2, h * np.array([-1, 4, 24, 4, -1]) / 30, rtol=1e-13)
    np.testing.assert_allclose(K2, np.array([1, -16, 30, -16, 1]) / (12 * h), rtol=1e-13)
    np.testing.assert_allclose(G2, np.array([1, -8, 0, 8, -1]) / 12, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_quadratic_derivative_exact_on_quartics(deg):
    n, h = 16, 1.0 / 16
    x = (np.arange(n) + 0.5) * h
    shape = (5, 5, n)
    u = np.ascontiguousarray(np.broadcast_to((x ** deg)[None, None, :], shape))
    wx, wm, wlap = oracle.step_filters_quadratic(h)
    inner = (slice(None), slice(None), slice(2, n - 2))
    ml = h ** 3
    du = oracle.step_apply5(u, h, (0,) * 6, wx) / ml
    want = deg * x ** (deg - 1) if deg > 0 else np.zeros(n)
    np.testing.assert_allclose(du[inner], np.broadcast_to(want, shape)[inner], rtol=0, atol=1e-11)
    # mass: f(u; w_m) = m_l u on cubics (its second and third moments vanish)
    if deg <= 3:
        np.testing.assert_allclose(oracle.step_apply5(u, h, (0,) * 6, wm)[inner] / ml, u[inner], rtol=0, atol=1e-12)


@pytest.mark.parametrize("deg", [2, 3, 4, 5])
def test_quadratic_laplacian_exact_on_quintics(deg):
    n, h = 16, 1.0 / 16
    z = (np.arange(n) + 0.5) * h
    shape = (n, 5, 5)
    u = np.ascontiguousarray(np.broadcast_to((z ** deg)[:, None, None], shape))
    _, _, wlap = oracle.step_filters_quadratic(h)
    lap = -oracle.step_apply5(u, h, (0,) * 6, wlap) / h ** 3
    want = deg * (deg - 1) * z ** (deg - 2)
    np.testing.assert_allclose(lap[2:n - 2], np.broadcast_to(want[:, None, None], shape)[2:n - 2], rtol=0,
                               atol=1e-9)


def _pad_reflect(u, rule):
    """Two-cell halo by reflection about each wall (cell -1-m mirrors cell m),
    negated on faces with rule 1, axis by axis (x, y, z)."""
    p = u
    for ax, (lo, hi) in zip((2, 1, 0), ((rule[0], rule[1]), (rule[2], rule[3]), (rule[4], rule[5]))):
        n = p.shape[ax]
        lo_part = np.flip(np.take(p, [0, 1], axis=ax), axis=ax) * (-1.0 if lo else 1.0)
        hi_part = np.flip(np.take(p, [n - 2, n - 1], axis=ax), axis=ax) * (-1.0 if hi else 1.0)
        p = np.concatenate([lo_part, p, hi_part], axis=ax)
    return p


@pytest.mark.parametrize("rule", [(0,) * 6, (1, 1, 0, 0, 1, 0), (0, 1, 1, 0, 0, 1)])
def test_two_cell_halo_against_numpy_convolution(rule):
    rng = np.random.default_rng(5)
    nz, ny, nx = 7, 6, 9
    h = 0.3
    u = rng.standard_normal((nz, ny, nx))
    w = rng.standard_normal((5, 5, 5))
    up = _pad_reflect(u, rule)
    want = np.zeros_like(u)
    for c in range(5):
        for b in range(5):
            for a in range(5):
                want += w[c, b, a] * up[c:c + nz, b:b + ny, a:a + nx]
    got = oracle.step_apply5(u, h, rule, w)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


def _state(n, ny=None, nz=None):
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    return {k: np.zeros((nz, ny, n)) for k in ("C", "u", "v", "w", "p_hs", "p_nh")}


def test_quadratic_hydrostatic_rest_state():
    n = 16
    h = 1.0 / n
    st = _state(n)
    st["C"][:] = 1.0
    oracle.step(st, h, oracle.step_params(mg_cycles=40, order=2))
    z = (np.arange(n) + 0.5) * h
    exact = 1000.0 * 9.81 * (1.0 - z)[:, None, None] * np.ones((n, n, n))
    np.testing.assert_allclose(st["p_hs"], exact, rtol=0, atol=1e-9 * exact.max())
    for q in ("u", "v", "w"):
        assert np.abs(st[q]).max() < 1e-9
    assert np.array_equal(st["C"], np.ones((n, n, n)))


def test_quadratic_y_independence_and_v_zero():
    from paper_2401_06755_amd import inputs

    h, st = inputs.water_block(16, 6, 16)
    oracle.step(st, h, oracle.step_params(rho_g=500.0, mg_cycles=20, order=2))
    for k in ("C", "u", "w", "p_hs", "p_nh"):
        f = st[k]
        assert np.max(np.abs(f - f[:, :1, :])) <= 1e-12 * max(np.abs(f).max(), 1e-300), k
    vel = max(np.abs(st["u"]).max(), np.abs(st["w"]).max())
    assert np.abs(st["v"]).max() <= 1e-12 * vel and vel > 0


def _blob(n):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - 0.45) ** 2 + (Y - 0.5) ** 2 + (Z - 0.55) ** 2)
    C = np.clip(0.5 - (r - 0.25) / (2 * h), 0.0, 1.0).transpose(2, 1, 0)
    return h, np.ascontiguousarray(C)


def test_quadratic_vof_zero_velocity_and_uniform_velocity_conservation():
    n = 16
    h, C = _blob(n)
    z = np.zeros_like(C)
    with oracle.periodic_step(), oracle.step_order(2):
        C1 = oracle.step_vof(C, z, z, z, h, 1e-3)
        assert np.array_equal(C1, C)
        U = (0.3, -0.2, 0.1)
        C2 = oracle.step_vof(C, *[np.full_like(C, u) for u in U], h, 1e-3)
    assert abs(C2.sum() - C.sum()) <= 1e-12 * C.sum()
    assert np.abs(C2 - C).max() > 1e-4  # the field did move


def test_quadratic_full_step_periodic_shift_commutes():
    n = 16
    h, C = _blob(n)
    st = _state(n)
    st["C"] = C
    rng = np.random.default_rng(3)
    for q in ("u", "v", "w"):
        st[q] = 0.05 * rng.standard_normal(C.shape)
    sh = {k: np.ascontiguousarray(np.roll(v, (1, 2, 3), axis=(0, 1, 2))) for k, v in st.items()}
    p = oracle.step_params(rho_l=2.0, rho_g=1.0, mu_l=1e-2, mu_g=1e-2, mg_cycles=80, order=2)
    with oracle.periodic_step():
        oracle.step(st, h, p)
        oracle.step(sh, h, p)
    for k in st:
        np.testing.assert_allclose(np.roll(st[k], (1, 2, 3), axis=(0, 1, 2)), sh[k], rtol=0,
                                   atol=1e-9 * max(np.abs(st[k]).max(), 1e-30))


def test_quadratic_detectors_on_a_kinked_profile():
    """The detector of Eqs. Sx-quad is the smallest of the three products of
    successive differences: a profile with a kink two cells away is flagged
    (S < 0) where Eq. Sx-lin is not, and only there does w- vanish."""
    n, dt = 24, 1e-3
    h = 1.0 / n
    c1 = np.linspace(0.1, 0.9, n)
    c1[12] = c1[11] - 0.01  # a local dip: products next to it change sign
    shape = (4, 4, n)
    C = np.ascontiguousarray(np.broadcast_to(c1[None, None, :], shape))
    z = np.zeros(shape)
    U = np.full(shape, 0.5)
    with oracle.step_order(1):
        k_lin = oracle.step_vof_coefs(C, U, z, z, h, dt)[0][0, 0]
    with oracle.step_order(2):
        k_quad = oracle.step_vof_coefs(C, U, z, z, h, dt)[0][0, 0]
    d = np.diff(c1)
    s_lin = d[:-1] * d[1:]  # at cells 1 .. n-2
    i = np.arange(3, n - 3)
    s_quad = np.minimum(np.minimum(s_lin[i - 2], s_lin[i - 1]), s_lin[i])
    flagged = (s_quad < 0) & (s_lin[i - 1] >= 0)
    assert flagged.any()
    # where only the quadratic detector flags, the diffusivity switches to positive (k+)
    assert np.all(k_quad[i][flagged] >= 0) and np.any(k_lin[i][flagged] < 0)
