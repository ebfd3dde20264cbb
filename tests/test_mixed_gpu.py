"""Mixed-precision forms against the FP64 oracle.

FP32_SMOOTH runs the V-cycle on the correction in FP32 (FP32 copy of k) with
the residual, the coarsest solve and the update x += e in FP64; FP16_COEF
stores that copy of k in FP16.  The outer residual is always the FP64
operator's, so a converged solve satisfies the FP64 system to rtol.

Tolerances:
* one outer iteration x + V32(0, b - A x) vs the oracle's x + V64(0, b - A x):
  the two corrections differ by FP32 rounding carried through ~4 levels of
  sweeps, bounded here by 2e-5 of the largest correction entry (FP32 unit
  roundoff 6e-8 times a growth factor of a few hundred), and 2e-2 for FP16
  coefficients (unit roundoff 5e-4 on k);
* solves: the oracle's FP64 residual of the returned x is <= rtol ||b||, and
  x agrees with the oracle's FP64 solve to the same rtol within the error the
  condition number allows (checked at 1e-5 relative on these sizes).
"""
import numpy as np
import pytest

import oracle
from paper_2401_06755_amd import inputs

pytestmark = pytest.mark.gpu

D, N, P = 0, 1, 2


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


def host(t, shape):
    return t.cpu().numpy().reshape(shape)


def sphere_case(shape, radius=0.3, seed=3):
    nx, ny, nz = shape
    h = 1.0 / nx
    frac = inputs.sphere_fraction(shape, h, (0.5, 0.5, 0.5 * nz / nx), radius)
    k = inputs.two_phase_k(frac, 1000.0, 1.0)
    b = inputs.gaussian(shape, seed, zero_mean=False)
    return h, k, b


@pytest.mark.parametrize("prec,tol", [(1, 2e-5), (2, 2e-2)])
@pytest.mark.parametrize("shape,bc", [((48, 48, 48), (N, N, N, N, N, D)), ((40, 12, 24), (D, N, D, D, N, N))])
def test_one_outer_iteration_matches_oracle(mg, prec, tol, shape, bc):
    h, k, b = sphere_case(shape)
    rng = np.random.default_rng(9)
    x0 = rng.standard_normal(b.shape)
    cfg = mg.config_default(*shape, h, bc=bc, coef_mode=1, precision=prec)
    H = mg.Hierarchy(cfg, dev(k))
    xd = dev(x0)
    H.vcycle(dev(b), xd)
    got = host(xd, b.shape)
    want = oracle.Hierarchy(shape, h, bc, k=k).vcycle(x0, b)
    corr = want - x0
    assert np.max(np.abs((got - x0) - corr)) <= tol * np.abs(corr).max()


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("shape,bc", [((64, 64, 64), (N,) * 6), ((32, 32, 64), (N, N, N, N, N, D))])
def test_mixed_solve_reaches_fp64_tolerance(mg, prec, shape, bc):
    h, k, b = sphere_case(shape, seed=4)
    cfg = mg.config_default(*shape, h, bc=bc, coef_mode=1, precision=prec)
    H = mg.Hierarchy(cfg, dev(k))
    xd = dev(np.zeros_like(b))
    info = H.solve(dev(b), xd, rtol=1e-8, max_cycles=1000)
    assert info.status == 0 and info.relres <= 1e-8
    x = host(xd, b.shape)
    bb = b - b.mean() if all(v != D for v in bc) else b
    r = bb - oracle.apply(x, h, bc, k)
    assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(bb)
    # FP64 GPU solve of the same system to the same tolerance
    H64 = mg.Hierarchy(mg.config_default(*shape, h, bc=bc, coef_mode=1), dev(k))
    x64d = dev(np.zeros_like(b))
    info64 = H64.solve(dev(b), x64d, rtol=1e-8, max_cycles=1000)
    x64 = host(x64d, b.shape)
    assert np.max(np.abs(x - x64)) <= 1e-5 * np.abs(x64).max()
    # the outer iteration count is governed by the FP64 residual: within a few cycles of FP64
    assert abs(info.cycles - info64.cycles) <= max(3, info64.cycles // 10)


def test_constant_coefficient_mixed(mg):
    w = inputs.poisson_sine_noise(64, seed=1)
    cfg = mg.config_default(64, 64, 64, w["h"], bc=w["bc"], precision=1)
    H = mg.Hierarchy(cfg)
    xd = dev(np.zeros_like(w["b"]))
    info = H.solve(dev(w["b"]), xd, rtol=1e-8, max_cycles=200)
    assert info.status == 0
    x = host(xd, w["b"].shape)
    r = w["b"] - oracle.apply(x, w["h"], w["bc"])
    assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(w["b"])


def test_fp16_needs_nodal(mg):
    with pytest.raises(mg.Nn4mgError):
        mg.Hierarchy(mg.config_default(16, 16, 16, 1 / 16, precision=2))


@pytest.mark.parametrize("shape,bc", [((32, 32, 32), (N, N, N, N, N, D)), ((48, 16, 32), (D, N, P, P, N, N))])
def test_fp16_storage_exact_coefficients_bitwise_fp32(mg, shape, bc):
    """k in {0.5, 1}: the means of 8 children on every coarser level are
    multiples of 2^-4, 2^-7, 2^-10 in [0.5, 1], all exact in FP16 (spacing
    2^-11 there), so the FP16-stored coefficient holds the same values as the
    FP32 copy on every level.  The FP16_COEF cycle must then equal the
    FP32_SMOOTH cycle bit for bit (one cycle and ten fixed cycles), and both
    stay within the FP32 bar of the oracle's FP64 cycle."""
    import torch

    nx, ny, nz = shape
    h = 1.0 / nx
    rng = np.random.default_rng(21)
    k = np.where(rng.random((nz, ny, nx)) < 0.5, 0.5, 1.0)
    b = inputs.gaussian((nx, ny, nz), 22, zero_mean=False)
    x0 = rng.standard_normal(b.shape)
    out = {}
    for prec in (1, 2):
        cfg = mg.config_default(nx, ny, nz, h, bc=bc, coef_mode=1, precision=prec)
        H = mg.Hierarchy(cfg, dev(k))
        assert len(H.levels()) >= 3
        xd = dev(x0)
        H.vcycle(dev(b), xd)
        xs = dev(np.zeros_like(b))
        H.solve(dev(b), xs, max_cycles=10, fixed_cycles=True)
        torch.cuda.synchronize()
        out[prec] = (host(xd, b.shape), host(xs, b.shape))
        H.close()
    np.testing.assert_array_equal(out[2][0], out[1][0])
    np.testing.assert_array_equal(out[2][1], out[1][1])
    want = oracle.Hierarchy(shape, h, bc, k=k).vcycle(x0, b)
    corr = want - x0
    assert np.max(np.abs((out[2][0] - x0) - corr)) <= 2e-5 * np.abs(corr).max()
