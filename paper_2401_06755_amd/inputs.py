"""Seeded synthetic inputs for the pressure solve (shared by tests, smoke and bench).

This module only draws numbers and lays out fields: it holds none of the
solver's arithmetic, and it is the one piece that the oracle side and the HIP
side both use. Arrays are numpy float64 of shape (nz, ny, nx) in C order, so x
is the fastest index, and cell centres sit at ((i + 1/2) h, (j + 1/2) h,
(k + 1/2) h).

Workloads stand in for the paper's collapsing-column and rising-bubble
pressure solves (Sec. 3): a sine mode plus noise on the unit cube, a dense
sphere in a light fluid (water drop in air), and an air bubble in water.
"""
from __future__ import annotations

import numpy as np

BC_DIRICHLET0, BC_NEUMANN0, BC_PERIODIC = 0, 1, 2

ALL_DIRICHLET = (0, 0, 0, 0, 0, 0)
ALL_NEUMANN = (1, 1, 1, 1, 1, 1)
# Neumann on the sides and the bottom, zero pressure at the top (z high):
# the boundary conditions of the paper's tank problems (Sec. 3.1).
TOP_DIRICHLET = (1, 1, 1, 1, 1, 0)


def centres(n: int, h: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def sine_mode(shape_xyz, h, modes=(1, 1, 1)) -> np.ndarray:
    """prod_d sin(m_d pi x_d) sampled at cell centres."""
    nx, ny, nz = shape_xyz
    sx = np.sin(modes[0] * np.pi * centres(nx, h))
    sy = np.sin(modes[1] * np.pi * centres(ny, h))
    sz = np.sin(modes[2] * np.pi * centres(nz, h))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def uniform_noise(shape_xyz, seed: int, amplitude: float) -> np.ndarray:
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    return amplitude * rng.uniform(-1.0, 1.0, size=(nz, ny, nx))


def gaussian(shape_xyz, seed: int, zero_mean: bool = True) -> np.ndarray:
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(size=(nz, ny, nx))
    if zero_mean:
        g -= g.mean()
    return g


def sphere_fraction(shape_xyz, h, centre, radius) -> np.ndarray:
    """Liquid fraction of a sphere with a linear ramp two cells wide:
    C = clamp(1/2 - d / (2h), 0, 1), d = signed distance (positive outside)."""
    nx, ny, nz = shape_xyz
    x = centres(nx, h)[None, None, :]
    y = centres(ny, h)[None, :, None]
    z = centres(nz, h)[:, None, None]
    d = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2) - radius
    return np.clip(0.5 - d / (2.0 * h), 0.0, 1.0)


def two_phase_k(frac: np.ndarray, rho_inside: float, rho_outside: float) -> np.ndarray:
    """Coefficient k = 1 / rho for a two-fluid density field (fraction 1 inside)."""
    rho = rho_inside * frac + rho_outside * (1.0 - frac)
    return 1.0 / rho


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def poisson_sine_noise(n: int = 64, seed: int = 1):
    """Constant-coefficient Poisson on the unit cube, zero Dirichlet walls,
    b = sin(pi x) sin(pi y) sin(pi z) + 1e-3 U[-1, 1).  (64^3 workload.)"""
    h = 1.0 / n
    shape = (n, n, n)
    b = sine_mode(shape, h) + uniform_noise(shape, seed, 1e-3)
    return dict(shape=shape, h=h, bc=ALL_DIRICHLET, k=None, b=b)


def dense_sphere(n: int = 256, seed: int = 2, radius: float = 0.15):
    """Variable-density Poisson: rho = 1000 in a sphere of radius 0.15 at the
    centre of the unit box, 1 outside, two-cell ramp; k = 1/rho; Neumann
    walls; Gaussian right-hand side projected to zero mean.  (256^3 workload.)"""
    h = 1.0 / n
    shape = (n, n, n)
    frac = sphere_fraction(shape, h, (0.5, 0.5, 0.5), radius)
    k = two_phase_k(frac, 1000.0, 1.0)
    b = gaussian(shape, seed, zero_mean=True)
    return dict(shape=shape, h=h, bc=ALL_NEUMANN, k=k, b=b)


def served_request(req_id: int, base_seed: int = 4000, edges=(32, 48, 64, 96, 128)):
    """One request of the served stream: cube edge drawn from `edges`, random
    dense sphere (centre U[0.25,0.75]^3, radius U[0.1,0.2], rho 1000/1),
    Neumann walls, zero-mean Gaussian right-hand side."""
    rng = np.random.default_rng(base_seed + req_id)
    n = int(edges[rng.integers(0, len(edges))])
    c = rng.uniform(0.25, 0.75, size=3)
    r = rng.uniform(0.1, 0.2)
    h = 1.0 / n
    shape = (n, n, n)
    frac = sphere_fraction(shape, h, tuple(c), r)
    k = two_phase_k(frac, 1000.0, 1.0)
    b = gaussian(shape, base_seed + req_id + 1_000_000, zero_mean=True)
    return dict(shape=shape, h=h, bc=ALL_NEUMANN, k=k, b=b, edge=n)


def rising_bubble(nx: int = 256, seed: int = 5, radius: float = 0.25):
    """Rising-bubble pressure solve: 256 x 256 x 512 cells on a 1 x 1 x 2 box,
    air bubble (rho 1) of radius 0.25 at (0.5, 0.5, 0.5) in water (rho 1000),
    zero pressure at the top, Neumann elsewhere, Gaussian right-hand side."""
    h = 1.0 / nx
    shape = (nx, nx, 2 * nx)
    frac = sphere_fraction(shape, h, (0.5, 0.5, 0.5), radius)
    k = two_phase_k(frac, 1.0, 1000.0)
    b = gaussian(shape, seed, zero_mean=False)
    return dict(shape=shape, h=h, bc=TOP_DIRICHLET, k=k, b=b)


def water_block(nx: int = 128, ny: int | None = None, nz: int | None = None, x1: float = 0.25, z1: float = 0.5):
    """Collapsing water column on the unit-spacing tank (Sec. 3.1 set-up): C = 1 in
    cells whose centre lies in [0, x1] x [0, 1] x [0, z1] (box units of h = 1/nx),
    else 0; fluid at rest, pressures zero.  Returns (h, dict of (nz, ny, nx) arrays)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    h = 1.0 / nx
    x = (np.arange(nx) + 0.5) * h
    z = (np.arange(nz) + 0.5) * h
    C = ((x[None, None, :] <= x1) & (z[:, None, None] <= z1)).astype(np.float64)
    C = np.ascontiguousarray(np.broadcast_to(C, (nz, ny, nx)))
    zero = np.zeros((nz, ny, nx))
    return h, dict(C=C, u=zero.copy(), v=zero.copy(), w=zero.copy(), p_hs=zero.copy(), p_nh=zero.copy())


def bubble_state(nx: int = 32, ny: int | None = None, nz: int | None = None, radius: float = 1.0 / 6.0,
                 centre_z: float = 1.0 / 3.0):
    """Rising air bubble in a water tank for the time step (Sec. 3.2 set-up,
    scaled to a box of width 1): nx x ny x nz cells of h = 1/nx (default
    1 x 1 x 2 box), water (C = 1) everywhere except a sphere of radius 1/6 at
    (1/2, 1/2, 1/3) (the paper's bubble of radius H/2 at height H in a
    3H x 3H x 6H tank), two-cell linear ramp; fluid at rest, pressures zero.
    Returns (h, dict of (nz, ny, nx) arrays)."""
    ny = nx if ny is None else ny
    nz = 2 * nx if nz is None else nz
    h = 1.0 / nx
    C = 1.0 - sphere_fraction((nx, ny, nz), h, (0.5, 0.5 * ny * h, centre_z), radius)
    zero = np.zeros((nz, ny, nx))
    return h, dict(C=np.ascontiguousarray(C), u=zero.copy(), v=zero.copy(), w=zero.copy(), p_hs=zero.copy(),
                   p_nh=zero.copy())
