"""Launch shapes give the same cycle: every z-marching tile shape of the
two-sweep kernel, and the 8^3 block form of the same two sweeps, against the
FP64 oracle through the C-ABI.

The block kernel sums the operator in the marching kernels' order but forms
the prolongation and the products k y with its own rounding, so the bar is the
one of the V-cycle parity tests: one FP64 cycle to 1e-12 of the largest entry,
fixed-count FP64 solves to 1e-10, and the mixed forms to the tolerances of the
mixed-precision tests (2e-5 FP32, 2e-2 FP16 coefficients).  Cases cover all
three boundary rules, ragged blocks (level dims not multiples of 8), both
coefficient modes, and the block kernel at the finest level (adding into x).
"""
import numpy as np
import pytest

import oracle
from paper_2401_06755_amd import inputs

pytestmark = pytest.mark.gpu

D, N, P = 0, 1, 2
SWEEP1 = 1  # kernel class of the first sweep (the two-sweep kernel's shape)


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


def rand_k(shape, seed, spread=3.0):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(-spread, spread, size=shape))


def fusable_levels(H):
    return [l for l, (nx, ny, nz) in enumerate(H.levels()) if min(nx, ny, nz) >= 4]


def set_block(H, levels):
    for l in levels:
        H.set_tiles(l, 8, 8, 8, kclass=SWEEP1)


CASES = [
    ((64, 64, 64), (D,) * 6, False),
    ((80, 24, 40), (N, N, N, N, N, D), True),
    ((32, 48, 16), (D, N, P, P, N, D), True),
    ((40, 12, 24), (N, N, D, N, N, N), True),
    ((48, 48, 48), (N,) * 6, True),
    ((64, 32, 48), (P, P, D, N, P, P), True),
    ((24, 40, 56), (D, D, P, P, N, D), False),
]


def one_cycle(mg, shape, bc, var, shapes_fn, prec=0):
    nx, ny, nz = shape
    rng = np.random.default_rng(21)
    x0 = rng.standard_normal((nz, ny, nx))
    b = rng.standard_normal((nz, ny, nx))
    if all(v != D for v in bc):
        b -= b.mean()
    k = rand_k((nz, ny, nx), 22) if var else None
    h = 1.0 / nx
    cfg = mg.config_default(*shape, h, bc=bc, coef_mode=1 if var else 0, precision=prec)
    H = mg.Hierarchy(cfg, dev(k) if var else None)
    shapes_fn(H)
    xd = dev(x0)
    H.vcycle(dev(b), xd)
    got = host(xd, x0.shape)
    want = oracle.Hierarchy(shape, h, bc, k=k).vcycle(x0, b)
    H.close()
    return got, want, x0


@pytest.mark.parametrize("shape,bc,var", CASES)
@pytest.mark.parametrize("levels", ["coarse", "all"])
def test_block_two_sweeps_one_cycle_fp64(mg, shape, bc, var, levels):
    def shapes(H):
        fl = fusable_levels(H)
        set_block(H, [l for l in fl if l > 0] if levels == "coarse" else fl)
        for l in fusable_levels(H):
            if levels == "all" or l > 0:
                assert H.get_tiles(l, SWEEP1) == (8, 8, 8)

    got, want, _ = one_cycle(mg, shape, bc, var, shapes)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.abs(want).max()


MARCHING = [(64, 2, 16), (64, 1, 4), (32, 2, 2), (32, 1, 8), (16, 2, 4), (64, 4, 6), (32, 4, 2)]


@pytest.mark.parametrize("tile", MARCHING)
@pytest.mark.parametrize("shape,bc,var", [CASES[1], CASES[3], CASES[5]])
def test_marching_shapes_one_cycle_fp64(mg, shape, bc, var, tile):
    def shapes(H):
        for l in range(len(H.levels())):
            H.set_tiles(l, *tile, kclass=SWEEP1)

    got, want, _ = one_cycle(mg, shape, bc, var, shapes)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("prec,tol", [(1, 2e-5), (2, 2e-2)])
@pytest.mark.parametrize("shape,bc", [((48, 48, 48), (N, N, N, N, N, D)), ((40, 12, 24), (D, N, D, D, N, N))])
def test_block_two_sweeps_one_cycle_mixed(mg, prec, tol, shape, bc):
    got, want, x0 = one_cycle(mg, shape, bc, True, lambda H: set_block(H, fusable_levels(H)), prec=prec)
    corr = want - x0
    assert np.max(np.abs((got - x0) - corr)) <= tol * np.abs(corr).max()


@pytest.mark.parametrize("outer", [0, 1])
def test_block_fixed_cycle_solve_fp64(mg, outer):
    shape, bc = (40, 40, 80), (N, N, N, N, N, D)
    nx, ny, nz = shape
    b = np.random.default_rng(31).standard_normal((nz, ny, nx))
    frac = inputs.sphere_fraction(shape, 1.0 / nx, (0.5, 0.5, 0.5 * nz / nx), 0.3)
    k = inputs.two_phase_k(frac, 1000.0, 1.0)
    h = 1.0 / nx
    cfg = mg.config_default(*shape, h, bc=bc, coef_mode=1, outer=outer)
    H = mg.Hierarchy(cfg, dev(k))
    set_block(H, fusable_levels(H))
    xd = dev(np.zeros_like(b))
    if outer == 0:
        info = H.solve(dev(b), xd, max_cycles=10, fixed_cycles=True)
        xo, hist_o, st = oracle.Hierarchy(shape, h, bc, k=k).solve(b, max_cycles=10, fixed=True)
        assert info.status == 0 and st == 0
        assert np.max(np.abs(host(xd, b.shape) - xo)) <= 1e-10 * np.abs(xo).max()
    else:
        info = H.solve(dev(b), xd, rtol=1e-8, max_cycles=200)
        assert info.status == 0 and info.relres <= 1e-8
        r = b - oracle.apply(host(xd, b.shape), h, bc, k)
        assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(b)
    H.close()


def test_block_shape_rules(mg):
    shape = (32, 32, 32)
    cfg = mg.config_default(*shape, 1 / 32, bc=(D,) * 6)
    H = mg.Hierarchy(cfg)
    with pytest.raises(mg.Nn4mgError):
        H.set_tiles(0, 8, 8, 8, kclass=0)  # the residual class has no block form
    with pytest.raises(mg.Nn4mgError):
        H.set_tiles(0, 8, 8, 8, kclass=-1)
    with pytest.raises(mg.Nn4mgError):
        H.set_tiles(0, 8, 4, 8, kclass=SWEEP1)
    H.set_tiles(1, 8, 8, 8, kclass=SWEEP1)
    assert H.get_tiles(1, SWEEP1) == (8, 8, 8)
    H.set_tiles(1, 32, 2, 4, kclass=SWEEP1)  # a marching shape replaces it
    assert H.get_tiles(1, SWEEP1) == (32, 2, 4)
    H.close()
    # three post-sweeps: no two-sweep kernel, so no block form
    cfg3 = mg.config_default(*shape, 1 / 32, bc=(D,) * 6, nu_post=3)
    H3 = mg.Hierarchy(cfg3)
    with pytest.raises(mg.Nn4mgError):
        H3.set_tiles(1, 8, 8, 8, kclass=SWEEP1)
    H3.close()


def test_autotune_may_pick_block_and_stays_exact(mg):
    w = inputs.dense_sphere(64, seed=2)
    cfg = mg.config_default(*w["shape"], w["h"], bc=w["bc"], coef_mode=1)
    H = mg.Hierarchy(cfg, dev(w["k"]))
    bd, xd = dev(w["b"]), dev(np.zeros_like(w["b"]))
    tiles = H.autotune(bd, xd)
    for l, t in enumerate(tiles):
        assert t[SWEEP1] == H.get_tiles(l, SWEEP1)
    xd.zero_()
    info = H.solve(bd, xd, max_cycles=6, fixed_cycles=True)
    xo, _, _ = oracle.Hierarchy(w["shape"], w["h"], w["bc"], k=w["k"]).solve(w["b"], max_cycles=6, fixed=True)
    assert info.status == 0
    assert np.max(np.abs(host(xd, w["b"].shape) - xo)) <= 1e-10 * np.abs(xo).max()
    H.close()
