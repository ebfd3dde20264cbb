"""Failure handling of the solve through the C-ABI.

* A diverging iteration (weighted Jacobi at omega = 1.8, past the smoother's
  stability bound) ends with EBREAKDOWN at the first residual above 1e3 times
  the first one; the residuals up to there are the oracle's (which has no
  guard and simply keeps diverging), to the fixed-count bar of 1e-10.
* A non-finite right-hand side ends with EBREAKDOWN, for the stationary and
  the flexible-CG outer iteration; a non-finite or non-positive coefficient is
  rejected at setup with EINVAL.
"""
import numpy as np
import pytest

import oracle
from paper_2401_06755_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_06755_amd import nn4mg

    nn4mg.lib()
    return nn4mg


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def test_divergence_is_a_breakdown(mg):
    outer = 0
    import torch

    n = 16
    w = inputs.dense_sphere(n, seed=2)
    om = 1.8
    cfg = mg.config_default(n, n, n, w["h"], bc=w["bc"], coef_mode=1, omega=om, outer=outer)
    H = mg.Hierarchy(cfg, dev(w["k"]))
    bd = dev(w["b"])
    xd = torch.zeros_like(bd)
    with pytest.raises(mg.Nn4mgError) as e:
        H.solve(bd, xd, rtol=1e-8, max_cycles=200)
    assert e.value.code == mg.NN4MG_EBREAKDOWN
    info = mg.Info()
    code = mg.lib().nn4mg_solve(H.handle, mg._field(bd, n ** 3, "b"), mg._field(xd.zero_(), n ** 3, "x"), 1e-8, 200,
                                0, mg.ctypes.byref(info))
    assert code == mg.NN4MG_EBREAKDOWN and info.status == mg.NN4MG_EBREAKDOWN
    hist = np.array(info.hist[: info.hist_len])
    assert hist[-1] > 1e3 * hist[0] and np.all(hist[:-1] <= 1e3 * hist[0])
    assert np.all(np.isfinite(xd.cpu().numpy()))
    OH = oracle.Hierarchy(w["shape"], w["h"], w["bc"], k=w["k"], omega=om)
    _, ohist, _ = OH.solve(w["b"], max_cycles=len(hist) + 2, fixed=True)
    m = len(hist)
    np.testing.assert_allclose(hist, ohist[:m], rtol=1e-10, atol=0)
    assert ohist[m - 1] > 1e3  # the oracle keeps going: the guard is the library's
    H.close()


def test_fcg_with_a_diverging_smoother_stagnates_without_breakdown(mg):
    """The same cycle as a preconditioner: flexible CG does not diverge (the
    oracle's FCG stagnates near 0.2 after 100 iterations), so the guard must
    not fire; the solve ends with ENOTCONV."""
    import torch

    n = 16
    w = inputs.dense_sphere(n, seed=2)
    cfg = mg.config_default(n, n, n, w["h"], bc=w["bc"], coef_mode=1, omega=1.8, outer=1)
    H = mg.Hierarchy(cfg, dev(w["k"]))
    bd = dev(w["b"])
    xd = torch.zeros_like(bd)
    info = H.solve(bd, xd, rtol=1e-8, max_cycles=30)
    assert info.status == mg.NN4MG_ENOTCONV
    hist = np.array(info.hist[: info.hist_len])
    assert hist.max() < 10.0 and np.all(np.isfinite(hist))
    H.close()


@pytest.mark.parametrize("outer", [0, 1])
def test_nan_rhs_is_a_breakdown(mg, outer):
    import torch

    n = 32
    w = inputs.dense_sphere(n, seed=2)
    b = w["b"].copy()
    b[3, 5, 7] = np.nan
    cfg = mg.config_default(n, n, n, w["h"], bc=w["bc"], coef_mode=1, outer=outer)
    H = mg.Hierarchy(cfg, dev(w["k"]))
    xd = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.Nn4mgError) as e:
        H.solve(dev(b), xd, rtol=1e-8, max_cycles=50)
    assert e.value.code == mg.NN4MG_EBREAKDOWN
    # the same hierarchy still solves a finite right-hand side afterwards
    info = H.solve(dev(w["b"]), xd.zero_(), rtol=1e-8, max_cycles=200)
    assert info.status == 0 and info.relres <= 1e-8
    H.close()


@pytest.mark.parametrize("bad", [np.nan, np.inf, 0.0, -1.0])
def test_bad_coefficient_rejected_at_setup(mg, bad):
    n = 16
    w = inputs.dense_sphere(n, seed=2)
    k = w["k"].copy()
    k[1, 2, 3] = bad
    cfg = mg.config_default(n, n, n, w["h"], bc=w["bc"], coef_mode=1)
    with pytest.raises(mg.Nn4mgError) as e:
        mg.Hierarchy(cfg, dev(k))
    assert e.value.code == mg.NN4MG_EINVAL
