"""Pins of the time-step oracle (Sec. 2.4, Stages 1-4) against closed forms and
symmetries.  Paper figures are not numeric, so parity vs the paper itself is
unpinned; these pins fix the oracle's pieces independently."""
import numpy as np
import pytest

import oracle
from tests import indep


def water_block(nx, ny, nz, x1=0.25, z1=0.5):
    h = 1.0 / nx
    x = (np.arange(nx) + 0.5) * h
    z = (np.arange(nz) + 0.5) * h
    C = ((x[None, None, :] <= x1) & (z[:, None, None] <= z1)).astype(np.float64)
    C = np.ascontiguousarray(np.broadcast_to(C, (nz, ny, nx)))
    zero = np.zeros((nz, ny, nx))
    return h, dict(C=C, u=zero.copy(), v=zero.copy(), w=zero.copy(), p_hs=zero.copy(), p_nh=zero.copy())


def test_step_filters_are_tensor_products():
    h = 0.1
    wx, wm, wpgx, wlap = oracle.step_filters(h)
    M = np.array([1.0, 4.0, 1.0]) * h / 6
    # printed w_x (Sec. 2.2.3): (m_l / (72 dx)) [-1 0 1] x [1 4 1] x [1 4 1]
    g = np.einsum("c,b,a->cba", np.array([1, 4, 1.0]), np.array([1, 4, 1.0]), np.array([-1, 0, 1.0]))
    np.testing.assert_allclose(wx, g * h ** 2 / 72, atol=1e-16)
    np.testing.assert_allclose(wm.sum(), h ** 3, rtol=1e-14)  # consistent mass integrates to the cell volume
    np.testing.assert_allclose(wm, np.einsum("c,b,a->cba", M, M, M), atol=1e-18)
    # w_xx + w_yy + w_zz = w_lap; w_xx^PG = K (x) M (x) M
    np.testing.assert_allclose(wpgx + wpgx.transpose(0, 2, 1) + wpgx.transpose(2, 1, 0), wlap, atol=1e-15)
    np.testing.assert_allclose(wlap, indep.q1_tensor_filter(h), atol=1e-15)


def test_hydrostatic_rest_state():
    """Single fluid at rest: p_hs = rho g (1 - z) (Q1 is exact on linears and the
    affine bottom halo is exact), the velocity stays zero to solver tolerance,
    and C is unchanged exactly."""
    nx = ny = nz = 16
    h = 1.0 / nx
    st = {k: np.zeros((nz, ny, nx)) for k in ("u", "v", "w", "p_hs", "p_nh")}
    st["C"] = np.ones((nz, ny, nx))
    C0 = st["C"].copy()
    res = oracle.step(st, h, oracle.step_params(sigma_t=0.07, mg_cycles=40))
    z = (np.arange(nz) + 0.5) * h
    exact = 1000.0 * 9.81 * (1.0 - z)[:, None, None] * np.ones((nz, ny, nx))
    np.testing.assert_allclose(st["p_hs"], exact, rtol=0, atol=1e-9 * exact.max())
    for q in ("u", "v", "w"):
        assert np.abs(st[q]).max() < 1e-9
    assert np.array_equal(st["C"], C0)
    assert len(res) == 3


def test_y_independence_and_v_zero():
    """The block spans all of y and the rules are y-symmetric: every field stays
    independent of y and v stays zero (to rounding)."""
    h, st = water_block(16, 6, 16)
    oracle.step(st, h, oracle.step_params(mg_cycles=20))
    for k in ("C", "u", "w", "p_hs", "p_nh"):
        f = st[k]
        assert np.max(np.abs(f - f[:, :1, :])) <= 1e-10 * max(np.abs(f).max(), 1e-30), k
    assert np.abs(st["v"]).max() <= 1e-10 * np.abs(st["u"]).max()


def test_x_mirror_symmetry():
    """A block centred in x stays mirror-symmetric: C, w, p even in x, u odd."""
    nx, ny, nz = 16, 4, 16
    h = 1.0 / nx
    x = (np.arange(nx) + 0.5) * h
    z = (np.arange(nz) + 0.5) * h
    C = ((np.abs(x - 0.5)[None, None, :] <= 0.25) & (z[:, None, None] <= 0.5)).astype(np.float64)
    C = np.ascontiguousarray(np.broadcast_to(C, (nz, ny, nx)))
    st = dict(C=C, **{k: np.zeros((nz, ny, nx)) for k in ("u", "v", "w", "p_hs", "p_nh")})
    oracle.step(st, h, oracle.step_params(mg_cycles=20))
    flip = lambda f: f[:, :, ::-1]
    for k in ("C", "w", "p_hs", "p_nh"):
        scale = max(np.abs(st[k]).max(), 1e-30)
        assert np.max(np.abs(st[k] - flip(st[k]))) <= 1e-9 * scale, k
    assert np.max(np.abs(st["u"] + flip(st["u"]))) <= 1e-9 * np.abs(st["u"]).max()
    assert np.abs(st["u"]).max() > 0


def test_collapsing_column_predictor_direction():
    """Predictor only (no correction): the column's weight drives water outwards
    at its foot and downwards at its top corner; the three pressure solves of
    a full step converge to solver accuracy."""
    h, st = water_block(24, 8, 24)
    oracle.step(st, h, oracle.step_params(mg_cycles=20, n_corr=0))
    assert st["u"].max() > 0
    assert st["w"].min() < 0
    h, st = water_block(24, 8, 24)
    res = oracle.step(st, h, oracle.step_params(mg_cycles=20))
    assert len(res) == 3 and all(r < 1e-6 for r in res)


def test_layered_rest_state_hydrostatic_profile():
    """Water below z = 1/2, air above, at rest: Stage 1 gives the piecewise
    linear hydrostatic column away from the interface (slopes rho_l g and
    rho_g g), and the predictor leaves the velocity tangential to the layers
    (u, v = 0)."""
    n = 24
    h = 1.0 / n
    z = (np.arange(n) + 0.5) * h
    C = np.ascontiguousarray(np.broadcast_to((z[:, None, None] <= 0.5).astype(float), (n, 8, n)))
    st = dict(C=C.copy(), **{k: np.zeros((n, 8, n)) for k in ("u", "v", "w", "p_hs", "p_nh")})
    oracle.step(st, h, oracle.step_params(mg_cycles=40, sigma_t=0.0, n_corr=0))
    col = st["p_hs"][:, 0, 0]
    slope_w = (col[1:9] - col[0:8]) / h
    slope_a = (col[16:23] - col[15:22]) / h
    np.testing.assert_allclose(slope_w, -1000 * 9.81, rtol=1e-6)
    np.testing.assert_allclose(slope_a, -1 * 9.81, rtol=1e-5)
    assert np.abs(st["u"]).max() < 1e-12 and np.abs(st["v"]).max() < 1e-12


# --------------------------------------------------------------------------
# Stage 4 (volume fraction): P15 (ii)-(iv) on a test-only periodic box
# --------------------------------------------------------------------------

def _blob(n, ny=None, centre=(0.45, 0.5, 0.55), radius=0.27):
    ny = ny or n
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    y = (np.arange(ny) + 0.5) / ny
    d = np.sqrt((x[None, None, :] - centre[0]) ** 2 + (y[None, :, None] - centre[1]) ** 2
                + (x[:, None, None] - centre[2]) ** 2) - radius
    return h, np.ascontiguousarray(np.clip(0.5 - d / (2 * h), 0.0, 1.0))


def test_vof_zero_velocity_keeps_C_and_zero_coefficients():
    """q = 0: the advection residual, k_abs and k- all vanish, so every
    Stage-4 diffusivity is zero and C^{n+1} = C^n bit for bit (Sec. 2.3.5,
    Eq. transport-indicator-1)."""
    h, C = _blob(16)
    z = np.zeros_like(C)
    kx, ky, kz, a = oracle.step_vof_coefs(C, z, z, z, h, 1e-4)
    for f in (kx, ky, kz, a):
        assert np.all(f == 0.0)
    assert np.array_equal(oracle.step_vof(C, z, z, z, h, 1e-4), C)
    rho = 1000 * C + (1 - C)
    mu = 1e-3 * C + 1.8e-5 * (1 - C)
    for comp in range(3):  # velocity diffusivity = mu alone (Eq. k_Psi-n, min = k_max = 0)
        a, k = oracle.step_pg_velocity(comp, z, z, z, rho, mu, h)
        assert np.all(a == 0.0) and np.array_equal(k, mu)


@pytest.mark.parametrize("U", [(0.3, -0.2, 0.1), (1.0, 0.0, 0.0)])
def test_vof_uniform_velocity_conserves_volume_periodic(U):
    """Uniform velocity on a periodic box: sum C is conserved to rounding (the
    first-derivative filter is antisymmetric and the Eq. k-T form of each
    compressive diffusion term sums to zero for a symmetric filter), whatever
    the diffusivities, which are non-zero here."""
    h, C = _blob(16)
    uu = [np.full_like(C, c) for c in U]
    with oracle.periodic_step():
        kx, ky, kz, _ = oracle.step_vof_coefs(C, *uu, h, 1e-3)
        C1 = oracle.step_vof(C, *uu, h, 1e-3)
    assert max(np.abs(kx).max(), np.abs(ky).max(), np.abs(kz).max()) > 0
    assert (kx < 0).any() and (kx > 0).any()  # both compressive and positive diffusion act
    assert np.abs(C1 - C).max() > 1e-6
    assert abs(C1.sum() - C.sum()) <= 1e-12 * C.sum()


def test_vof_periodic_shift_commutes():
    """A one-cell periodic shift commutes with Stage 4 (every operator is the
    same filter at every cell)."""
    h, C = _blob(16)
    rng = np.random.default_rng(3)
    uu = [np.ascontiguousarray(0.3 * rng.standard_normal(C.shape)) for _ in range(3)]
    sh = lambda f: np.ascontiguousarray(np.roll(f, (1, -1, 1), axis=(0, 1, 2)))
    with oracle.periodic_step():
        a = oracle.step_vof(C, *uu, h, 1e-3)
        b = oracle.step_vof(sh(C), *[sh(u) for u in uu], h, 1e-3)
    np.testing.assert_allclose(b, sh(a), rtol=0, atol=1e-15)


def test_full_step_periodic_shift_commutes():
    """The whole step on a periodic box (density ratio 2, surface tension on)
    commutes with a one-cell shift up to the pressure solves' convergence."""
    n = 16
    h, C = _blob(n)
    rng = np.random.default_rng(4)
    st = dict(C=C, u=0.05 * rng.standard_normal(C.shape), v=0.05 * rng.standard_normal(C.shape),
              w=0.05 * rng.standard_normal(C.shape), p_hs=np.zeros_like(C), p_nh=np.zeros_like(C))
    sh = lambda f: np.ascontiguousarray(np.roll(f, 1, axis=2))
    p = oracle.step_params(rho_l=2.0, rho_g=1.0, mu_l=1e-2, mu_g=1e-2, mg_cycles=80)
    a = {k: np.ascontiguousarray(v).copy() for k, v in st.items()}
    b = {k: sh(v) for k, v in st.items()}
    with oracle.periodic_step():
        oracle.step(a, h, p)
        oracle.step(b, h, p)
    for k in a:
        scale = np.abs(a[k]).max()
        assert np.max(np.abs(b[k] - sh(a[k]))) <= 1e-10 * scale, k


# --------------------------------------------------------------------------
# Petrov-Galerkin coefficients against fields whose derivatives are known
# --------------------------------------------------------------------------

@pytest.mark.parametrize("V0,W0", [(0.0, 0.0), (0.2, -0.1)])
def test_pg_velocity_coefficients_closed_form(V0, W0):
    """u = c (x^2 - x0^2) along x, v and w constant.  The derivative filter is
    exact on quadratics, so u_x = 2 c x; u u_x = 2 c^2 (x^3 - x0^2 x), on which
    the mixed-mass residual filter w_m/m_l - E (Eq. a_psi) gives h^2 times the
    x^3 coefficient: a = alpha_a 2 c^2 h^2 x with alpha_a = 2.  Then
    Eqs. efficient-kabs-special-case, k-square (h_Psi = h), max-k and k_Psi-n
    (alpha_kabs = 1/16, alpha_ksquare = 4 at p = 1, eps_k = 1e-7)."""
    n, c = 32, 1.0
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    x0 = x[20]
    shape = (6, 5, n)
    X = np.broadcast_to(x[None, None, :], shape)
    u = np.ascontiguousarray(c * (X ** 2 - x0 ** 2))
    v, w = np.full(shape, V0), np.full(shape, W0)
    rng = np.random.default_rng(9)
    rho = rng.uniform(1.0, 1000.0, size=shape)
    mu = rng.uniform(1e-5, 1e-3, size=shape)
    a, k = oracle.step_pg_velocity(0, u, v, w, rho, mu, h)
    ux = 2 * c * X
    a_want = 2.0 * 2 * c ** 2 * h ** 2 * X
    kabs = (1 / 16) * h * np.abs(a_want) / (1e-7 + np.abs(ux) / 3)
    ksq = 4 * a_want ** 2 * h / (1e-7 + np.abs(u * ux) / 3 * ux ** 2)
    kmax = h * (np.abs(u) + abs(V0) + abs(W0))
    k_want = rho * np.minimum(kmax, np.minimum(kabs, ksq)) + mu
    inner = (slice(None), slice(None), slice(2, n - 2))  # two cells off the x walls
    np.testing.assert_allclose(a[inner], a_want[inner], rtol=1e-9, atol=1e-12 * np.abs(a_want).max())
    np.testing.assert_allclose(k[inner], k_want[inner], rtol=1e-9)
    # the closed form exercises more than one branch of the minimum
    which = np.argmin(np.stack([kmax, kabs, ksq]), axis=0)[inner]
    assert len(np.unique(which)) >= 2


def test_vof_coefficients_on_tanh_profile():
    """C = (1 + tanh((x - 1/2) / (2h))) / 2 moving with u = U along x: the
    gradient is the central difference of C (the transverse mass filters sum to
    the cell area), S_y = S_z = 0, S_x is Eq. Sx-lin, cells with C > 0.95 or
    C < 0.05 take S = -1 in every direction; then w+, w-, k- with its
    normalisation (beta = 0.1, eps_x = 1e-4), k+ = 3 k_abs and the clamps of
    Eq. alpha_min_and_max (Sec. 2.3.5)."""
    n, U, dt = 32, 0.7, 1e-3
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    c1 = 0.5 * (1 + np.tanh((x - 0.5) / (2 * h)))
    shape = (4, 4, n)
    C = np.ascontiguousarray(np.broadcast_to(c1[None, None, :], shape))
    z = np.zeros(shape)
    kx, ky, kz, a = oracle.step_vof_coefs(C, np.full(shape, U), z, z, h, dt)
    i = np.arange(2, n - 2)
    cx = (c1[i + 1] - c1[i - 1]) / (2 * h)
    adv = lambda j: U * (c1[j + 1] - c1[j - 1]) / (2 * h)
    a_w = 2.0 * ((adv(i - 1) + 4 * adv(i) + adv(i + 1)) / 6 - adv(i))
    S = (c1[i] - c1[i - 1]) * (c1[i + 1] - c1[i])
    bulk = (c1[i] > 0.95) | (c1[i] < 0.05)
    Sx = np.where(bulk, -1.0, S)
    Syz = np.where(bulk, -1.0, 0.0)
    us = cx * (U * cx / (1e-4 + cx ** 2))
    kneg = -0.1 * U ** 2 / (1e-4 + cx ** 2 * np.abs(us) / 3)
    kabs = (1 / 16) * h * np.abs(a_w) / (1e-7 + np.abs(cx) / 3)
    kmin, kmax = 1e-4 / dt * h * h, 0.05 / dt * h * h

    def kd(Sd):
        wp = -np.maximum(-1, np.minimum(0, 300 * Sd))
        wm = np.minimum(1, np.maximum(0, 300 * Sd))
        return np.maximum(-kmin, np.minimum(kmax, wp * 3 * kabs + wm * kneg / h))

    np.testing.assert_allclose(a[0, 0, i], a_w, rtol=1e-10, atol=1e-13 * np.abs(a_w).max())
    np.testing.assert_allclose(kx[0, 0, i], kd(Sx), rtol=1e-10, atol=1e-16)
    np.testing.assert_allclose(ky[0, 0, i], kd(Syz), rtol=1e-10, atol=1e-16)
    np.testing.assert_allclose(kz[0, 0, i], kd(Syz), rtol=1e-10, atol=1e-16)
    assert (kx[0, 0, i] < 0).any() and (kx[0, 0, i] > 0).any()


# --------------------------------------------------------------------------
# Stage 3 (Eqs. ph_disc2, vel-cor)
# --------------------------------------------------------------------------

def _wd(q, d, h):
    """f(q; w_d) on a periodic box: (1/2)[-1, 0, 1] along d, h[1, 4, 1]/6 across."""
    out = q
    for ax, dd in ((2, 0), (1, 1), (0, 2)):
        if dd == d:
            out = 0.5 * (np.roll(out, -1, axis=ax) - np.roll(out, 1, axis=ax))
        else:
            out = h * (np.roll(out, 1, axis=ax) + 4 * out + np.roll(out, -1, axis=ax)) / 6
    return out


def test_stage3_fourier_mode_divergence_factor():
    """Constant density on a periodic box, the Stage-2 velocity one Fourier
    mode: every filter is diagonal, so one correction multiplies the discrete
    divergence sum_d f(q_d; w_d) by 1 - S / (m_l lambda), with
    S = sum_d sin^2(t_d) prod_{e != d} M_e^2, M = h (2 + cos t) / 3, and lambda
    the Q1 eigenvalue; the pressure increment is -rho D / (dt lambda).  Two
    corrections give the factor squared."""
    n = 16
    h = 1.0 / n
    m = (1, 2, 3)
    t = [2 * np.pi * mm / n for mm in m]
    i = np.arange(n)
    phase = (t[2] * i[:, None, None] + t[1] * i[None, :, None] + t[0] * i[None, None, :]) + 0.3
    amp = (0.7, -0.4, 0.25)
    q = [np.ascontiguousarray(a * np.cos(phase)) for a in amp]
    C = np.full((n, n, n), 0.4)
    params = oracle.step_params(rho_l=1000.0, rho_g=1.0, dt=1e-3, mg_cycles=60, n_corr=1)
    rho = 0.4 * 1000.0 + 0.6
    Mh = [h * (2 + np.cos(tt)) / 3 for tt in t]
    lam = indep.q1_eigenvalue(h, t)
    S = sum(np.sin(t[d]) ** 2 * np.prod([Mh[e] ** 2 for e in range(3) if e != d]) for d in range(3))
    fac = 1 - S / (h ** 3 * lam)
    D0 = sum(_wd(q[d], d, h) for d in range(3))
    with oracle.periodic_step():
        u1, v1, w1, pnh1, _ = oracle.step_correct(C, *q, np.zeros_like(C), h, params)
        params.n_corr = 2
        u2, v2, w2, pnh2, _ = oracle.step_correct(C, *q, np.zeros_like(C), h, params)
    D1 = sum(_wd(f, d, h) for d, f in enumerate((u1, v1, w1)))
    D2 = sum(_wd(f, d, h) for d, f in enumerate((u2, v2, w2)))
    sc = np.abs(D0).max()
    assert 0.05 < fac < 0.95
    np.testing.assert_allclose(D1, fac * D0, rtol=0, atol=1e-10 * sc)
    np.testing.assert_allclose(D2, fac ** 2 * D0, rtol=0, atol=1e-10 * sc)
    dp1 = -rho * D0 / (1e-3 * lam)
    np.testing.assert_allclose(pnh1, dp1, rtol=0, atol=1e-10 * np.abs(dp1).max())
    np.testing.assert_allclose(pnh2, dp1 * (1 + fac), rtol=0, atol=1e-10 * np.abs(dp1).max())


def test_stage3_uniform_velocity_is_a_fixed_point():
    """A uniform velocity has a zero right-hand side in Eq. ph_disc2 for any
    density field (f(rho U; w_d) = U f(rho; w_d)), so the corrections leave it
    unchanged up to rounding, at density ratio 1000."""
    h, C = _blob(16)
    U = (0.3, -0.2, 0.1)
    q = [np.full_like(C, c) for c in U]
    with oracle.periodic_step():
        u1, v1, w1, pnh, _ = oracle.step_correct(C, *q, np.zeros_like(C), h, oracle.step_params(mg_cycles=20))
    for f, c in zip((u1, v1, w1), U):
        assert np.abs(f - c).max() <= 1e-9 * abs(c)


# --------------------------------------------------------------------------
# Stages 1-3 on the layered rest state: where the printed scheme's interface
# velocities come from
# --------------------------------------------------------------------------

def _layered(n, ny=4):
    h = 1.0 / n
    z = (np.arange(n) + 0.5) * h
    C = np.ascontiguousarray(np.broadcast_to((z[:, None, None] <= 0.5).astype(float), (n, ny, n)))
    return h, z, dict(C=C.copy(), **{k: np.zeros((n, ny, n)) for k in ("u", "v", "w", "p_hs", "p_nh")})


def test_layered_rest_state_predictor_seed_closed_form():
    """Water below z = 1/2, air above, at rest.  Stage 1 solves
    K p = G(g rho) along z (Q1 stiffness, central derivative) exactly, so
    (p_{k+1} - p_k)/h = -g (rho_k + rho_{k+1})/2; the Stage-2 force
    f(p; w_z) + f(g rho; w_m) is then h^2 [G p + h M(g rho)/h] =
    -(g h^3 / 12)(rho_{k+1} - 2 rho_k + rho_{k-1}), non-zero only at the two
    cells beside the interface, and Eq. velocity-1 turns it into
    w = dt g (rho_{k+1} - 2 rho_k + rho_{k-1}) / (12 rho_k).  The light cell
    gets rho_l/rho_g times the heavy cell's speed."""
    n = 16
    h, z, st = _layered(n)
    p = oracle.step_params(mg_cycles=80, sigma_t=0.0, n_corr=0, n_vel_iter=1)
    oracle.step(st, h, p)
    rho = np.where(z <= 0.5, 1000.0, 1.0)
    d2 = np.zeros(n)
    d2[1:-1] = rho[2:] - 2 * rho[1:-1] + rho[:-2]
    w_want = p.dt * p.g * d2 / (12 * rho)
    col = st["w"][:, 0, 0]
    np.testing.assert_allclose(col, w_want, rtol=0, atol=1e-9 * np.abs(w_want).max())
    assert col[n // 2] > 0.08 and abs(col[n // 2 - 1]) < 1e-4
    assert np.abs(st["u"]).max() < 1e-12 and np.abs(st["v"]).max() < 1e-12


@pytest.mark.parametrize("ratio,grows", [(1000.0, True), (2.0, False)])
def test_layered_rest_state_corrections_amplify_light_phase(ratio, grows):
    """Each Stage-3 correction multiplies the light-phase interface speed by
    about (rho_l - rho_g)/(2 rho_g) at a density ratio of 1000: the term
    q~ f(rho; w_z) of Eq. ph_disc2 weights the light cell's velocity by the
    full density jump, and Eq. vel-cor divides the resulting pressure gradient
    by the light density.  At a ratio of 2 the corrections do not amplify."""
    n = 16
    peaks = []
    for nc in (0, 1, 2):
        h, z, st = _layered(n)
        oracle.step(st, h, oracle.step_params(rho_g=1000.0 / ratio, mg_cycles=60, sigma_t=0.0, n_corr=nc))
        peaks.append(np.abs(st["w"]).max())
    g1, g2 = peaks[1] / peaks[0], peaks[2] / peaks[1]
    if grows:
        assert g1 > 100 and g2 > 100
    else:
        assert g1 < 1.0 and g2 < 1.0


# --------------------------------------------------------------------------
# Surface tension (Eqs. surface-tension-k, surface-tension-uvw, ph_disc)
# --------------------------------------------------------------------------

def test_curvature_planar_and_quadratic():
    """A planar ramp has zero curvature (exactly: constant normals).  For
    C = r^2/2 the derivative filter is exact (C_x = x, ...), the normals are
    r_hat and Eq. surface-tension-k gives div(r_hat) = 2/r up to the
    second-order error of the central derivative of x/r."""
    n = 32
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y, Z = np.broadcast_arrays(x[None, None, :], x[None, :, None], x[:, None, None])
    ramp = np.ascontiguousarray(0.3 + 0.8 * X + 0.5 * Y - 0.2 * Z)
    s = oracle.step_surface(ramp, h, 0.07)
    inner = (slice(2, -2),) * 3
    assert np.abs(s["kappa"][inner]).max() < 1e-9
    np.testing.assert_allclose(s["Cx"][inner], 0.8, rtol=1e-12)
    R2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2
    bowl = np.ascontiguousarray(R2 / 2)
    s = oracle.step_surface(bowl, h, 0.07)
    r = np.sqrt(R2)
    sel = (r > 0.25) & (r < 0.4)
    np.testing.assert_allclose(s["Cx"][sel], (X - 0.5)[sel], rtol=0, atol=1e-12)
    np.testing.assert_allclose(s["kappa"][sel], 2 / r[sel], rtol=0.02)
    np.testing.assert_allclose(s["st"][2][sel], (0.07 * s["kappa"] * (Z - 0.5))[sel], rtol=1e-12)


def test_static_drop_laplace_jump_and_balance():
    """A drop (C = 1 inside r < 1/4, no gravity): Stage 1 gives the
    Young-Laplace jump p_in - p_out = 2 sigma / R, and the Stage-2 force on the
    drop nearly cancels (the surface-tension source balances the pressure it
    produced): the predicted speed stays a small fraction of dt |s_t| / rho."""
    n = 32
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    R, sigma = 0.25, 0.07
    d = np.sqrt((x[None, None, :] - 0.5) ** 2 + (x[None, :, None] - 0.5) ** 2 + (x[:, None, None] - 0.5) ** 2) - R
    C = np.ascontiguousarray(np.clip(0.5 - d / (2 * h), 0, 1))
    st = dict(C=C.copy(), **{k: np.zeros((n, n, n)) for k in ("u", "v", "w", "p_hs", "p_nh")})
    p = oracle.step_params(rho_l=2.0, rho_g=1.0, g=0.0, sigma_t=sigma, mg_cycles=60, n_corr=0)
    oracle.step(st, h, p)
    jump = st["p_hs"][n // 2, n // 2, n // 2] - st["p_hs"][n // 2, n // 2, 1]
    np.testing.assert_allclose(jump, 2 * sigma / R, rtol=0.02)
    s = oracle.step_surface(C, h, sigma)
    force = max(np.abs(f).max() for f in s["st"])
    umax = max(np.abs(st[k]).max() for k in ("u", "v", "w"))
    assert umax < 0.25 * p.dt * force / 1.0
