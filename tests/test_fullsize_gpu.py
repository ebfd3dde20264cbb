"""Full-size solves in the benchmark's launch configuration (autotuned tiles),
checked by the oracle's FP64 residual of the returned x over the whole field.

* 256^3 dense sphere (rho 1000/1, k = 1/rho, Neumann), FP64 and FP32-smoothing.
* 256 x 256 x 512 rising bubble (air in water, zero pressure on top), FP16-stored
  coefficient + FP32 smoothing + FP64 residual/refinement.
The bar is the solve tolerance itself: ||b - A x||_2 <= 1e-8 ||b||_2 with A the
oracle's FP64 operator (Eq. k-T), with 5% slack for the different summation
order of the two residual evaluations.
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


def run(mg, work, precision):
    import torch

    nx, ny, nz = work["shape"]
    cfg = mg.config_default(nx, ny, nz, work["h"], bc=work["bc"], coef_mode=1, precision=precision)
    kd = torch.from_numpy(work["k"].reshape(-1)).cuda()
    bd = torch.from_numpy(work["b"].reshape(-1)).cuda()
    xd = torch.zeros_like(bd)
    H = mg.Hierarchy(cfg, kd)
    H.autotune(bd, xd)
    xd.zero_()
    info = H.solve(bd, xd, rtol=1e-8, max_cycles=2000)
    x = xd.cpu().numpy().reshape(work["b"].shape)
    H.close()
    return info, x


def oracle_relres(work, x):
    b = work["b"]
    if all(v != 0 for v in work["bc"]):
        b = b - b.mean()
    r = b - oracle.apply(x, work["h"], work["bc"], work["k"])
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_sphere_256(mg, precision):
    work = inputs.dense_sphere(256, seed=2)
    info, x = run(mg, work, precision)
    assert info.status == 0 and info.relres <= 1e-8
    assert oracle_relres(work, x) <= 1.05e-8
    if all(v != 0 for v in work["bc"]):
        assert abs(x.mean()) <= 1e-12 * np.abs(x).max()


def test_rising_bubble_256x256x512_fp16_coefficient(mg):
    work = inputs.rising_bubble(256, seed=5)
    info, x = run(mg, work, 2)
    assert info.status == 0 and info.relres <= 1e-8
    assert oracle_relres(work, x) <= 1.05e-8
