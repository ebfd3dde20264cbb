"""Independent constructions used to pin the oracle (no oracle code here).

* ``fe_assembled_matrix``: the pressure matrix from an explicit trilinear
  finite-element assembly with Gauss quadrature over the dual cells of the
  cell-centred grid, halo nodes folded into the interior by the boundary rules.
* ``kron_matrix``: the same operator as a sum of Kronecker products of 1D
  stiffness/mass matrices, each folded on its own axis.
* ``link_matrix``: the variable-coefficient operator in link form,
  A_k x_i = sum_{s != 0} (-w_s) (k_i + k_{i+s}) / 2 (x_i - x_{i+s}), which is the
  algebraic rearrangement of Eq. (k-T) when the filter weights sum to zero.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

DIR, NEU, PER = 0, 1, 2


def q1_tensor_filter(h):
    """K x M x M + M x K x M + M x M x K from 1D linear elements, [z][y][x]."""
    K = np.array([-1.0, 2.0, -1.0]) / h
    M = np.array([1.0, 4.0, 1.0]) * h / 6.0
    return (np.einsum("c,b,a->cba", M, M, K) + np.einsum("c,b,a->cba", M, K, M)
            + np.einsum("c,b,a->cba", K, M, M))


def _fold_axis(idx, n, lo, hi):
    """Map a padded index (-1..n) on one axis to (interior index, sign)."""
    if 0 <= idx < n:
        return idx, 1.0
    bc = lo if idx < 0 else hi
    if bc == PER:
        return (idx + n) % n, 1.0
    mirror = 0 if idx < 0 else n - 1
    return mirror, (-1.0 if bc == DIR else 1.0)


def _element_stiffness(h):
    """Trilinear hexahedron of side h: K_e[a, b] = int grad N_a . grad N_b,
    2-point Gauss rule per axis (exact for these integrands)."""
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    corners = list(itertools.product([0, 1], repeat=3))  # (cz, cy, cx)
    Ke = np.zeros((8, 8))
    for xi, eta, zeta in itertools.product(g, g, g):
        grads = []
        for cz, cy, cx in corners:
            sx, sy, sz = (2 * cx - 1), (2 * cy - 1), (2 * cz - 1)
            nx_ = 0.5 * (1 + sx * xi)
            ny_ = 0.5 * (1 + sy * eta)
            nz_ = 0.5 * (1 + sz * zeta)
            # d/dx = (2/h) d/dxi
            grads.append(np.array([0.5 * sx * ny_ * nz_, 0.5 * sy * nx_ * nz_, 0.5 * sz * nx_ * ny_]) * (2.0 / h))
        grads = np.array(grads)
        Ke += grads @ grads.T * (h / 2.0) ** 3
    return Ke, corners


def fe_assembled_matrix(nx, ny, nz, h, bc):
    """Dense interior matrix from element assembly on the padded node set."""
    Ke, corners = _element_stiffness(h)
    px, py, pz = nx + 2, ny + 2, nz + 2
    N = px * py * pz
    G = np.zeros((N, N))

    def pid(i, j, k):
        return (i + 1) + px * ((j + 1) + py * (k + 1))

    for k in range(-1, nz):
        for j in range(-1, ny):
            for i in range(-1, nx):
                ids = [pid(i + cx, j + cy, k + cz) for cz, cy, cx in corners]
                G[np.ix_(ids, ids)] += Ke
    n = nx * ny * nz
    A = np.zeros((n, n))
    rows = [pid(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    for k in range(-1, nz + 1):
        for j in range(-1, ny + 1):
            for i in range(-1, nx + 1):
                col = pid(i, j, k)
                fi, si = _fold_axis(i, nx, bc[0], bc[1])
                fj, sj = _fold_axis(j, ny, bc[2], bc[3])
                fk, sk = _fold_axis(k, nz, bc[4], bc[5])
                m = fi + nx * (fj + ny * fk)
                A[:, m] += si * sj * sk * G[rows, col]
    return A


def _fold1d(n, h, lo, hi):
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    k1 = np.array([-1.0, 2.0, -1.0]) / h
    m1 = np.array([1.0, 4.0, 1.0]) * h / 6.0
    for i in range(n):
        for o in (-1, 0, 1):
            c, s = _fold_axis(i + o, n, lo, hi)
            K[i, c] += s * k1[o + 1]
            M[i, c] += s * m1[o + 1]
    return K, M


def kron_matrix(nx, ny, nz, h, bc):
    Kx, Mx = _fold1d(nx, h, bc[0], bc[1])
    Ky, My = _fold1d(ny, h, bc[2], bc[3])
    Kz, Mz = _fold1d(nz, h, bc[4], bc[5])
    k = sp.kron
    A = k(Mz, k(My, Kx)) + k(Mz, k(Ky, Mx)) + k(Kz, k(My, Mx))
    return sp.csr_matrix(A)


def link_matrix(k_field, h, bc):
    """Sparse A_k in link form; k halos are zero-derivative copies (periodic: wrap)."""
    nz, ny, nx = k_field.shape
    w = q1_tensor_filter(h)
    n = nx * ny * nz
    kf = k_field.reshape(-1)
    rows, cols, vals = [], [], []
    coef_bc = [PER if b == PER else NEU for b in bc]
    for kk in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = i + nx * (j + ny * kk)
                for c, b, a in itertools.product((-1, 0, 1), repeat=3):
                    if (a, b, c) == (0, 0, 0):
                        continue
                    ws = w[c + 1, b + 1, a + 1]
                    if ws == 0.0:
                        continue
                    fi, si = _fold_axis(i + a, nx, bc[0], bc[1])
                    fj, sj = _fold_axis(j + b, ny, bc[2], bc[3])
                    fk, sk = _fold_axis(kk + c, nz, bc[4], bc[5])
                    gi, _ = _fold_axis(i + a, nx, coef_bc[0], coef_bc[1])
                    gj, _ = _fold_axis(j + b, ny, coef_bc[2], coef_bc[3])
                    gk, _ = _fold_axis(kk + c, nz, coef_bc[4], coef_bc[5])
                    kn = kf[gi + nx * (gj + ny * gk)]
                    link = -ws * 0.5 * (kf[r] + kn)
                    rows += [r, r]
                    cols += [r, fi + nx * (fj + ny * fk)]
                    vals += [link, -link * si * sj * sk]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def eig1d(kind, m, n):
    """Mode and angle theta = (frequency) * h for a 1D boundary pair.
    kind: 'DD' sin(m pi x), 'NN' cos(m pi x), 'DN' sin((m+1/2) pi x),
    'PP' cos(2 pi m x)."""
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    if kind == "DD":
        f = m * np.pi
        return np.sin(f * x), f * h
    if kind == "NN":
        f = m * np.pi
        return np.cos(f * x), f * h
    if kind == "DN":
        f = (m + 0.5) * np.pi
        return np.sin(f * x), f * h
    if kind == "PP":
        f = 2 * m * np.pi
        return np.cos(f * x), f * h
    raise ValueError(kind)


def q1_eigenvalue(h, thetas):
    s = [np.sin(t / 2) ** 2 for t in thetas]
    c = [2 + np.cos(t) for t in thetas]
    return 4 * h / 9 * (s[0] * c[1] * c[2] + c[0] * s[1] * c[2] + c[0] * c[1] * s[2])
