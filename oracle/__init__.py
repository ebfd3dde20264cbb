"""FP64 CPU oracle for the multigrid pressure solve (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library never calls it, and
it shares no code with the HIP path: the C source here is compiled by gcc into
``oracle/_liboracle.so`` and wrapped with ctypes over numpy arrays.

Every routine follows a passage of arXiv 2401.06755 (cited in the C source):
the filter notation f(C; w) of Sec. 2.2.2 over halo-padded tensors (Sec. 2.3.3),
the variable-coefficient identity Eq. (k-T) of Sec. 2.2.4, and the sawtooth
multigrid (U-Net) of Sec. 2.4 / Fig. multi-grid.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "nn4mg_oracle.c"), os.path.join(_HERE, "step_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same sources, for
# the CPU test that runs the oracle's pins under the sanitizers (loaded instead
# of the plain build when NN4MG_ORACLE_SANITIZED=1, with libasan preloaded).
_SAN_PATH = os.path.join(_HERE, "_liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]

BC_DIRICHLET0, BC_NEUMANN0, BC_PERIODIC = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction: plain IEEE order)."""
    srcs = [s for s in _SRC if os.path.exists(s)]
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC",
               "-o", _LIB_PATH + ".tmp", *srcs, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def build_sanitized() -> str:
    """The oracle built with ASan and UBSan (same flags otherwise)."""
    srcs = [s for s in _SRC if os.path.exists(s)]
    cmd = ["gcc", "-O1", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC", *SAN_FLAGS,
           "-o", _SAN_PATH + ".tmp", *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SAN_PATH + ".tmp", _SAN_PATH)
    return _SAN_PATH


# OpenMP build of the same sources, used only to time the oracle on every host
# core beside the GPU (the parity build above ignores the pragmas).
_OMP_PATH = os.path.join(_HERE, "_liboracle_omp.so")


def build_timing() -> str:
    srcs = [s for s in _SRC if os.path.exists(s)]
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c99", "-shared", "-fPIC", "-o", _OMP_PATH + ".tmp", *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_OMP_PATH + ".tmp", _OMP_PATH)
    return _OMP_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if os.environ.get("NN4MG_ORACLE_SANITIZED") == "1":
            L = ctypes.CDLL(_SAN_PATH)
        elif os.environ.get("NN4MG_ORACLE_OPENMP") == "1":
            L = ctypes.CDLL(_OMP_PATH)
        else:
            if not os.path.exists(_LIB_PATH):
                build()
            L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i, d, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        sig = {
            "or_pad": (None, [dp, i, i, i, ip, i, dp]),
            "or_q1_filter": (None, [d, dp]),
            "or_filter_apply": (None, [dp, i, i, i, dp, dp]),
            "or_apply": (None, [i, i, i, d, ip, dp, dp, dp]),
            "or_diag": (None, [i, i, i, d, ip, dp, dp]),
            "or_residual": (None, [i, i, i, d, ip, dp, dp, dp, dp]),
            "or_jacobi": (None, [i, i, i, d, ip, dp, dp, dp, d, i]),
            "or_restrict": (None, [i, i, i, dp, dp]),
            "or_prolong": (None, [i, i, i, ip, dp, dp]),
            "or_coarsen_k": (None, [i, i, i, dp, dp, i]),
            "or_dense": (None, [i, i, i, d, ip, dp, dp]),
            "or_cholesky": (i, [i, dp]),
            "or_chol_solve": (None, [i, dp, dp, dp]),
            "or_num_levels": (i, [i, i, i, i]),
            "or_setup": (vp, [i, i, i, d, ip, dp, d, i, i, i]),
            "or_free": (None, [vp]),
            "or_levels": (i, [vp]),
            "or_coarse_n": (i, [vp]),
            "or_level_k": (None, [vp, i, dp]),
            "or_vcycle": (None, [vp, dp, dp]),
            "or_solve": (i, [vp, dp, dp, d, i, i, dp, ip]),
            "or_fcg": (i, [vp, dp, dp, d, i, i, i, dp, ip]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if hasattr(L, "or_step"):
            _declare_step(L)
        _lib = L
    return _lib


class StepParams(ctypes.Structure):
    """Physical constants and iteration counts of one time step (Sec. 2.4)."""
    _fields_ = [("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double), ("mu_l", ctypes.c_double),
                ("mu_g", ctypes.c_double), ("g", ctypes.c_double), ("sigma_t", ctypes.c_double),
                ("dt", ctypes.c_double), ("mg_cycles", ctypes.c_int), ("n_corr", ctypes.c_int),
                ("n_vel_iter", ctypes.c_int), ("mg_cycles_nh", ctypes.c_int), ("order", ctypes.c_int)]


class StepInfo(ctypes.Structure):
    _fields_ = [("relres", ctypes.c_double * 8), ("solves", ctypes.c_int)]


def _declare_step(L):
    dp = ctypes.POINTER(ctypes.c_double)
    L.or_step.restype = ctypes.c_int
    L.or_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(StepParams),
                          dp, dp, dp, dp, dp, dp, ctypes.POINTER(StepInfo)]
    L.or_step_filters.restype = None
    L.or_step_filters.argtypes = [ctypes.c_double, dp, dp, dp, dp]
    i, d = ctypes.c_int, ctypes.c_double
    L.or_step_set_periodic.restype = None
    L.or_step_set_periodic.argtypes = [i]
    L.or_step_surface.restype = None
    L.or_step_surface.argtypes = [i, i, i, d, d, dp, dp, dp, dp, dp, dp, dp, dp]
    L.or_step_pg_velocity.restype = None
    L.or_step_pg_velocity.argtypes = [i, i, i, d, i, dp, dp, dp, dp, dp, dp, dp]
    L.or_step_vof_coefs.restype = None
    L.or_step_vof_coefs.argtypes = [i, i, i, d, d, dp, dp, dp, dp, dp, dp, dp, dp]
    L.or_step_vof.restype = None
    L.or_step_vof.argtypes = [i, i, i, d, d, dp, dp, dp, dp]
    L.or_step_correct.restype = ctypes.c_int
    L.or_step_correct.argtypes = [i, i, i, d, ctypes.POINTER(StepParams), dp, dp, dp, dp, dp,
                                  ctypes.POINTER(StepInfo)]
    L.or_step_set_order.restype = None
    L.or_step_set_order.argtypes = [i]
    L.or_step_filters_quadratic.restype = None
    L.or_step_filters_quadratic.argtypes = [d, dp, dp, dp]
    L.or_step_apply5.restype = None
    L.or_step_apply5.argtypes = [i, i, i, d, ctypes.POINTER(ctypes.c_int), dp, dp, dp]


def step_params(rho_l=1000.0, rho_g=1.0, mu_l=1e-3, mu_g=1.8e-5, g=9.81, sigma_t=0.07, dt=1e-4, mg_cycles=20,
                n_corr=2, n_vel_iter=2, mg_cycles_nh=0, order=1):
    """mg_cycles: cycles of every pressure solve; mg_cycles_nh (if > 0) those
    of the correction solves only (the j of the i-j strategies, Sec. 3.2);
    order 2: quadratic ConvFEM filters for the momentum, interface and
    volume-fraction advection terms (linear volume-fraction diffusion and
    pressure equations)."""
    return StepParams(rho_l, rho_g, mu_l, mu_g, g, sigma_t, dt, mg_cycles, n_corr, n_vel_iter, mg_cycles_nh,
                      order)


def step_filters_quadratic(h):
    """The quadratic ConvFEM filters w_x, w_m, w_lap as (5, 5, 5) arrays indexed [c, b, a] (z, y, x)."""
    out = [np.empty(125) for _ in range(3)]
    lib().or_step_filters_quadratic(float(h), *[_d(o) for o in out])
    return [o.reshape(5, 5, 5) for o in out]


def step_apply5(u, h, rule, w):
    """f(u; w) for a 5x5x5 filter w (indexed [c, b, a]) with the two-cell halo
    of `rule` (per face: 0 even, 1 odd)."""
    u = _f64(u)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    r = (ctypes.c_int * 6)(*[int(x) for x in rule])
    lib().or_step_apply5(nx, ny, nz, float(h), r, _d(np.ascontiguousarray(w, dtype=np.float64).reshape(-1)), _d(u),
                         _d(out))
    return out


class step_order:
    """Context manager: the stage pieces (step_surface, step_pg_velocity,
    step_vof_coefs, step_vof) use the filters of this order inside it."""

    def __init__(self, order):
        self.order = order

    def __enter__(self):
        lib().or_step_set_order(int(self.order))
        return self

    def __exit__(self, *exc):
        lib().or_step_set_order(1)
        return False


def step(state, h, params=None):
    """One time step in place on a dict of (nz, ny, nx) float64 arrays
    C, u, v, w, p_hs, p_nh; returns the relative residuals of the pressure solves."""
    params = params or step_params()
    arrs = [state[k] for k in ("C", "u", "v", "w", "p_hs", "p_nh")]
    for a in arrs:
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    nz, ny, nx = arrs[0].shape
    info = StepInfo()
    rc = lib().or_step(nx, ny, nz, float(h), ctypes.byref(params), *[_d(a) for a in arrs], ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("oracle step failed")
    return [info.relres[i] for i in range(info.solves)]


class periodic_step:
    """Context manager: inside it the step oracle uses the test-only periodic
    box (every halo wraps, periodic pressure solves) instead of the tank."""

    def __enter__(self):
        lib().or_step_set_periodic(1)
        return self

    def __exit__(self, *exc):
        lib().or_step_set_periodic(0)
        return False


def step_surface(C, h, sigma_t):
    """grad C (derivative units), curvature and surface-tension vectors of C."""
    C = _f64(C)
    nx, ny, nz = _shape(C)
    out = [np.empty_like(C) for _ in range(7)]
    lib().or_step_surface(nx, ny, nz, float(h), float(sigma_t), _d(C), *[_d(a) for a in out])
    return dict(Cx=out[0], Cy=out[1], Cz=out[2], kappa=out[3], st=(out[4], out[5], out[6]))


def step_pg_velocity(comp, u, v, w, rho, mu, h):
    """Advection residual a and diffusivity k of velocity component comp."""
    u, v, w, rho, mu = (_f64(a) for a in (u, v, w, rho, mu))
    nx, ny, nz = _shape(u)
    a, k = np.empty_like(u), np.empty_like(u)
    lib().or_step_pg_velocity(nx, ny, nz, float(h), int(comp), _d(u), _d(v), _d(w), _d(rho), _d(mu), _d(a), _d(k))
    return a, k


def step_vof_coefs(C, u, v, w, h, dt):
    """Stage-4 diffusivities (kx, ky, kz) and the advection residual of C."""
    C, u, v, w = (_f64(a) for a in (C, u, v, w))
    nx, ny, nz = _shape(C)
    out = [np.empty_like(C) for _ in range(4)]
    lib().or_step_vof_coefs(nx, ny, nz, float(h), float(dt), _d(C), _d(u), _d(v), _d(w), *[_d(a) for a in out])
    return out[0], out[1], out[2], out[3]


def step_vof(C, u, v, w, h, dt):
    """Stage 4 alone: returns C^{n+1}."""
    C = _f64(C).copy()
    u, v, w = (_f64(a) for a in (u, v, w))
    nx, ny, nz = _shape(C)
    lib().or_step_vof(nx, ny, nz, float(h), float(dt), _d(C), _d(u), _d(v), _d(w))
    return C


def step_correct(C, u, v, w, p_nh, h, params):
    """Stage 3 alone on copies: returns (u, v, w, p_nh, relres list)."""
    C = _f64(C)
    u, v, w, p_nh = (_f64(a).copy() for a in (u, v, w, p_nh))
    nx, ny, nz = _shape(C)
    info = StepInfo()
    rc = lib().or_step_correct(nx, ny, nz, float(h), ctypes.byref(params), _d(C), _d(u), _d(v), _d(w), _d(p_nh),
                               ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("oracle correction failed")
    return u, v, w, p_nh, [info.relres[i] for i in range(info.solves)]


def step_filters(h):
    wx, wm, wpg, wl = (np.empty(27) for _ in range(4))
    lib().or_step_filters(float(h), _d(wx), _d(wm), _d(wpg), _d(wl))
    return wx.reshape(3, 3, 3), wm.reshape(3, 3, 3), wpg.reshape(3, 3, 3), wl.reshape(3, 3, 3)


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _bc(bc):
    arr = (ctypes.c_int * 6)(*[int(v) for v in bc])
    return arr


def _shape(a: np.ndarray):
    """Arrays are (nz, ny, nx) in C order, i.e. x fastest."""
    nz, ny, nx = a.shape
    return nx, ny, nz


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def pad(u, bc, coef=False):
    u = _f64(u)
    nx, ny, nz = _shape(u)
    out = np.empty((nz + 2, ny + 2, nx + 2))
    lib().or_pad(_d(u), nx, ny, nz, _bc(bc), int(coef), _d(out))
    return out


def q1_filter(h):
    w = np.empty(27)
    lib().or_q1_filter(float(h), _d(w))
    return w.reshape(3, 3, 3)  # [c][b][a] = (z, y, x)


def filter_apply(up, w):
    up = _f64(up)
    w = _f64(w).reshape(27)
    nz, ny, nx = up.shape[0] - 2, up.shape[1] - 2, up.shape[2] - 2
    out = np.empty((nz, ny, nx))
    lib().or_filter_apply(_d(up), nx, ny, nz, _d(w), _d(out))
    return out


def apply(x, h, bc, k=None):
    x = _f64(x)
    nx, ny, nz = _shape(x)
    y = np.empty_like(x)
    kk = _f64(k) if k is not None else None
    lib().or_apply(nx, ny, nz, float(h), _bc(bc), _d(kk) if kk is not None else None, _d(x), _d(y))
    return y


def diag(shape_xyz, h, bc, k=None):
    nx, ny, nz = shape_xyz
    d = np.empty((nz, ny, nx))
    kk = _f64(k) if k is not None else None
    lib().or_diag(nx, ny, nz, float(h), _bc(bc), _d(kk) if kk is not None else None, _d(d))
    return d


def residual(b, x, h, bc, k=None):
    b, x = _f64(b), _f64(x)
    nx, ny, nz = _shape(x)
    r = np.empty_like(x)
    kk = _f64(k) if k is not None else None
    lib().or_residual(nx, ny, nz, float(h), _bc(bc), _d(kk) if kk is not None else None, _d(b), _d(x), _d(r))
    return r


def jacobi(b, y, h, bc, k=None, omega=2.0 / 3.0, nsweeps=1):
    b = _f64(b)
    y = _f64(y).copy()
    nx, ny, nz = _shape(y)
    kk = _f64(k) if k is not None else None
    lib().or_jacobi(nx, ny, nz, float(h), _bc(bc), _d(kk) if kk is not None else None, _d(b), _d(y), float(omega),
                    int(nsweeps))
    return y


def restrict(r):
    r = _f64(r)
    nx, ny, nz = _shape(r)
    rc = np.empty((nz // 2, ny // 2, nx // 2))
    lib().or_restrict(nx, ny, nz, _d(r), _d(rc))
    return rc


def prolong(ec, bc):
    ec = _f64(ec)
    cx, cy, cz = _shape(ec)
    ef = np.empty((2 * cz, 2 * cy, 2 * cx))
    lib().or_prolong(cx, cy, cz, _bc(bc), _d(ec), _d(ef))
    return ef


def coarsen_k(k, harmonic=False):
    k = _f64(k)
    nx, ny, nz = _shape(k)
    kc = np.empty((nz // 2, ny // 2, nx // 2))
    lib().or_coarsen_k(nx, ny, nz, _d(k), _d(kc), int(harmonic))
    return kc


def dense(shape_xyz, h, bc, k=None):
    nx, ny, nz = shape_xyz
    n = nx * ny * nz
    A = np.empty((n, n))
    kk = _f64(k) if k is not None else None
    lib().or_dense(nx, ny, nz, float(h), _bc(bc), _d(kk) if kk is not None else None, _d(A))
    return A


def cholesky(A):
    L = _f64(A).copy()
    rc = lib().or_cholesky(L.shape[0], _d(L))
    if rc != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return L


def chol_solve(L, b):
    L, b = _f64(L), _f64(b)
    x = np.empty_like(b)
    lib().or_chol_solve(L.shape[0], _d(L), _d(b), _d(x))
    return x


def num_levels(nx, ny, nz, min_coarse=4):
    return lib().or_num_levels(nx, ny, nz, min_coarse)


class Hierarchy:
    """Level chain + coarsest Cholesky factor; mirrors nn4mg_setup's meaning."""

    def __init__(self, shape_xyz, h, bc, k=None, omega=2.0 / 3.0, nu_post=2, min_coarse=4, harmonic=False):
        nx, ny, nz = shape_xyz
        self.shape = (nz, ny, nx)
        self._k = _f64(k) if k is not None else None  # kept alive: level 0 is referenced
        self._ptr = lib().or_setup(nx, ny, nz, float(h), _bc(bc),
                                   _d(self._k) if self._k is not None else None, float(omega), int(nu_post),
                                   int(min_coarse), int(harmonic))
        if not self._ptr:
            raise ValueError("oracle setup rejected the configuration")
        self.levels = lib().or_levels(self._ptr)
        self.coarse_n = lib().or_coarse_n(self._ptr)

    def level_k(self, l):
        nz, ny, nx = self.shape
        out = np.empty((nz >> l, ny >> l, nx >> l))
        lib().or_level_k(self._ptr, l, _d(out))
        return out

    def vcycle(self, x, b):
        x = _f64(x).copy()
        lib().or_vcycle(self._ptr, _d(x), _d(_f64(b)))
        return x

    def solve(self, b, x0=None, rtol=1e-8, max_cycles=100, fixed=False):
        b = _f64(b)
        x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
        hist = np.zeros(max_cycles + 1)
        cyc = ctypes.c_int(0)
        st = lib().or_solve(self._ptr, _d(b), _d(x), float(rtol), int(max_cycles), int(fixed), _d(hist),
                            ctypes.byref(cyc))
        return x, hist[: cyc.value + 1].copy(), st

    def fcg(self, b, x0=None, rtol=1e-8, max_iter=100, fixed=False, precond=True):
        """FCG(1) around one cycle from zero (precond) or plain CG; returns
        (x, history of ||r|| / ||b||, status)."""
        b = _f64(b)
        x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
        hist = np.zeros(max_iter + 1)
        it = ctypes.c_int(0)
        st = lib().or_fcg(self._ptr, _d(b), _d(x), float(rtol), int(max_iter), int(fixed), int(precond), _d(hist),
                          ctypes.byref(it))
        return x, hist[: it.value + 1].copy(), st

    def __del__(self):
        p = getattr(self, "_ptr", None)
        if p:
            lib().or_free(p)
            self._ptr = None
