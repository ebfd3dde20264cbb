"""nn4mg_residual_noalloc (no hierarchy, no device allocation: the norm
partials live in a static device array) against nn4mg_residual on a
hierarchy set up from the same config, through the C-ABI.  Same kernel and
launch shape on both sides, so r and the norm are expected bit for bit; the
bar written here is the residual's own (1e-13 of the largest entry, and the
norm to 1e-14 relative).  Two calls in a row share the static array, the
second on a smaller grid, and the residual is also checked against the
oracle's."""
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


def one_case(mg, shape_xyz, bc, nodal, seed):
    import torch

    nx, ny, nz = shape_xyz
    shape = (nz, ny, nx)
    h = 1.0 / nx
    rng = np.random.default_rng(seed)
    k = np.exp(rng.uniform(-2.0, 2.0, size=shape)) if nodal else None
    x = rng.standard_normal(shape)
    b = inputs.gaussian(shape, seed + 1, zero_mean=False)
    cfg = mg.config_default(nx, ny, nz, h, bc=bc, coef_mode=1 if nodal else 0)
    kd = dev(k) if nodal else None
    xd, bd = dev(x), dev(b)
    r_static = torch.full_like(xd, float("nan"))
    nrm_static = mg.residual_noalloc(cfg, xd, bd, k=kd, r=r_static)
    H = mg.Hierarchy(cfg, kd)
    r_hier = torch.full_like(xd, float("nan"))
    nrm_hier = H.residual(xd, bd, r_hier)
    torch.cuda.synchronize()
    H.close()
    rs = r_static.cpu().numpy().reshape(shape)
    rh = r_hier.cpu().numpy().reshape(shape)
    scale = np.abs(rh).max()
    np.testing.assert_allclose(rs, rh, rtol=0, atol=1e-13 * scale)
    assert abs(nrm_static - nrm_hier) <= 1e-14 * nrm_hier
    ro = oracle.residual(b, x, h, bc, k=k)
    np.testing.assert_allclose(rs, ro, rtol=0, atol=1e-13 * np.abs(ro).max())
    assert abs(nrm_static - np.linalg.norm(ro)) <= 1e-12 * np.linalg.norm(ro)
    # without a norm: r only, no synchronisation, no use of the static array
    r2 = torch.full_like(xd, float("nan"))
    assert mg.residual_noalloc(cfg, xd, bd, k=kd, r=r2, norm=False) is None
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r2.cpu().numpy().reshape(shape), rs)
    return nrm_static


CASES = [
    # (first call, second call on a smaller grid)
    (((80, 24, 40), (N, N, N, N, N, D), True), ((40, 12, 24), (N, N, N, N, N, D), True)),
    (((64, 64, 64), (D, D, D, D, D, D), False), ((5, 7, 3), (D, N, N, D, N, N), False)),
    (((96, 32, 64), (D, N, P, P, N, D), True), ((16, 8, 8), (N, N, N, N, N, N), False)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_residual_matches_hierarchy_twice(mg, first, second):
    n1 = one_case(mg, *first, seed=11)
    n2 = one_case(mg, *second, seed=12)
    assert np.isfinite(n1) and np.isfinite(n2)


def test_noalloc_residual_argument_errors(mg):
    import torch

    cfg = mg.config_default(16, 16, 16, 1 / 16, coef_mode=1)
    x = torch.zeros(16 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.Nn4mgError) as e:
        mg.residual_noalloc(cfg, x, x)  # nodal without k
    assert e.value.code == mg.NN4MG_EINVAL
    bad = mg.config_default(33, 33, 33, 1 / 33)
    y = torch.zeros(33 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.Nn4mgError):
        mg.residual_noalloc(bad, y, y)  # coarsest level too large, as nn4mg_setup rejects
