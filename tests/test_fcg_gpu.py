"""Flexible-CG outer iteration (NN4MG_OUTER_FCG) on the GPU.

FCG(1) with one sawtooth V(0,2) cycle from zero as the preconditioner M:
alpha = (z.r)/(p.Ap), x += alpha p, r -= alpha Ap, z = M r,
beta = -(z.Ap)/(p.Ap), p = z + beta p.  Checks:
* the residual history of the first iterations equals the oracle's FCG(1)
  (its operator, its V-cycle, the same recurrence), to 1e-9 relative per
  entry; the 64^3 case has three levels above the one-workgroup coarse end,
  so its stopping rule runs inside the preconditioning cycle's first
  restriction-chain launch (CG amplifies rounding differences from iteration to iteration, so
  the comparison stops after a few iterations);
* converged solves satisfy the oracle's FP64 system to rtol (5% slack for
  the different summation order of the two residuals) in fewer outer
  iterations than the stationary cycle, for FP64 and FP32-smoothing cycles;
* graph replays on a side stream reproduce the direct launches bitwise.
"""
import numpy as np
import pytest

import oracle
from paper_2401_06755_amd import inputs

pytestmark = pytest.mark.gpu

D, N = 0, 1


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


def oracle_fcg_history(work, iters):
    """The oracle's FCG(1) (cycle from zero as preconditioner), fixed count."""
    OH = oracle.Hierarchy(work["shape"], work["h"], work["bc"], k=work["k"])
    x, hist, st = OH.fcg(work["b"], max_iter=iters, fixed=True)
    assert st == 0
    return hist, x


def sphere_work(shape, bc, seed):
    nx, ny, nz = shape
    h = 1.0 / nx
    frac = inputs.sphere_fraction(shape, h, (0.5, 0.5, 0.5 * nz / nx), 0.3)
    return dict(shape=shape, h=h, bc=bc, k=inputs.two_phase_k(frac, 1000.0, 1.0),
                b=inputs.gaussian(shape, seed, zero_mean=False))


@pytest.mark.parametrize("shape,bc", [((32, 32, 32), (N,) * 6), ((48, 16, 32), (N, N, N, N, N, D)),
                                      ((64, 64, 64), (N, N, N, N, N, D))])
def test_fcg_history_matches_oracle_recurrence(mg, shape, bc):
    work = sphere_work(shape, bc, seed=11)
    iters = 6
    want, xw = oracle_fcg_history(work, iters)
    cfg = mg.config_default(*shape, work["h"], bc=bc, coef_mode=1, outer=mg.OUTER_FCG)
    H = mg.Hierarchy(cfg, dev(work["k"]))
    xd = dev(np.zeros_like(work["b"]))
    info = H.solve(dev(work["b"]), xd, rtol=0.0, max_cycles=iters, fixed_cycles=True)
    got = np.array(info.history())
    assert len(got) == iters + 1
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-13)
    x = xd.cpu().numpy().reshape(work["b"].shape)
    assert np.max(np.abs(x - xw)) <= 1e-9 * np.abs(xw).max()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,bc", [((64, 64, 64), (N,) * 6), ((32, 32, 64), (N, N, N, N, N, D))])
def test_fcg_solve_reaches_tolerance_in_fewer_iterations(mg, prec, shape, bc):
    work = sphere_work(shape, bc, seed=4)
    b = work["b"]
    res = {}
    for outer in (mg.OUTER_STATIONARY, mg.OUTER_FCG):
        cfg = mg.config_default(*shape, work["h"], bc=bc, coef_mode=1, precision=prec, outer=outer)
        H = mg.Hierarchy(cfg, dev(work["k"]))
        xd = dev(np.zeros_like(b))
        info = H.solve(dev(b), xd, rtol=1e-8, max_cycles=1000)
        assert info.status == 0 and info.relres <= 1e-8
        res[outer] = (info, xd.cpu().numpy().reshape(b.shape))
    info, x = res[mg.OUTER_FCG]
    bb = b - b.mean() if all(v != D for v in bc) else b
    r = bb - oracle.apply(x, work["h"], bc, work["k"])
    assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(bb)
    assert info.cycles < res[mg.OUTER_STATIONARY][0].cycles
    if all(v != D for v in bc):
        assert abs(x.mean()) <= 1e-12 * np.abs(x).max()


def test_fcg_dense_sphere_128(mg):
    w = inputs.dense_sphere(128, seed=2)
    cfg = mg.config_default(128, 128, 128, w["h"], bc=w["bc"], coef_mode=1, outer=mg.OUTER_FCG)
    H = mg.Hierarchy(cfg, dev(w["k"]))
    xd = dev(np.zeros_like(w["b"]))
    info = H.solve(dev(w["b"]), xd, rtol=1e-8, max_cycles=500)
    assert info.status == 0 and info.relres <= 1e-8
    x = xd.cpu().numpy().reshape(w["b"].shape)
    bb = w["b"] - w["b"].mean()
    r = bb - oracle.apply(x, w["h"], w["bc"], w["k"])
    assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(bb)


def test_fcg_graph_replays_match_direct_launches(mg):
    import torch

    w = inputs.dense_sphere(48, seed=2)
    cfg = mg.config_default(48, 48, 48, w["h"], bc=w["bc"], coef_mode=1, outer=mg.OUTER_FCG)
    k, b = dev(w["k"]), dev(w["b"])
    H1 = mg.Hierarchy(cfg, k)
    x1 = dev(np.zeros_like(w["b"]))
    info1 = H1.solve(b, x1, rtol=1e-8, max_cycles=500)
    ref = x1.cpu().numpy()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    H2 = mg.Hierarchy(cfg, k, stream=s)
    for rep in range(3):
        x2 = dev(np.zeros_like(w["b"]))
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        info2 = H2.solve(b, x2, rtol=1e-8, max_cycles=500)
        torch.cuda.synchronize()
        assert info2.cycles == info1.cycles and info2.status == 0
        assert np.array_equal(x2.cpu().numpy(), ref), rep
        assert info2.history() == info1.history()
        del junk


def test_fcg_zero_rhs_and_single_level_rejected(mg):
    cfg = mg.config_default(16, 16, 16, 1 / 16, bc=(N,) * 6, outer=mg.OUTER_FCG)
    H = mg.Hierarchy(cfg)
    xd = dev(np.ones((16, 16, 16)))
    info = H.solve(dev(np.zeros((16, 16, 16))), xd, rtol=1e-8, max_cycles=10)
    assert info.status == 0 and info.cycles == 0
    assert np.all(xd.cpu().numpy() == 0.0)
    with pytest.raises(mg.Nn4mgError):
        mg.Hierarchy(mg.config_default(5, 5, 5, 1 / 5, outer=mg.OUTER_FCG))  # one level only
