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
