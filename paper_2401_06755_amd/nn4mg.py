"""Python binding of the nn4mg C-ABI (include/nn4mg.h): argument marshalling only.

Every step of the solve runs in the HIP kernels of libnn4mg.so; this module
checks tensor shapes/dtypes/devices, passes raw device pointers and the current
torch stream, and converts status codes into exceptions.  PyTorch provides the
device memory and the stream.  If the library has not been built, every entry
point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnn4mg.so")

NN4MG_OK = 0
NN4MG_EINVAL = -1
NN4MG_ENOMEM = -2
NN4MG_EDEVICE = -3
NN4MG_ENOTCONV = -4
NN4MG_EBREAKDOWN = -5
NN4MG_EBUSY = -6

BC_DIRICHLET0, BC_NEUMANN0, BC_PERIODIC = 0, 1, 2
COEF_CONST, COEF_NODAL = 0, 1
PREC_FP64, PREC_FP32_SMOOTH, PREC_FP16_COEF = 0, 1, 2
OUTER_STATIONARY, OUTER_FCG = 0, 1
KCLASS_FINE_RESID, KCLASS_FINE_SWEEP_PROLONG, KCLASS_FINE_SWEEP = 0, 1, 2
HIST_MAX = 512


class Nn4mgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nn4mg error {code}: {msg}")
        self.code = code


class NotConverged(Nn4mgError):
    pass


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("h", ctypes.c_double),
        ("bc", ctypes.c_int * 6),
        ("coef_mode", ctypes.c_int), ("precision", ctypes.c_int),
        ("nu_post", ctypes.c_int), ("omega", ctypes.c_double),
        ("min_coarse", ctypes.c_int), ("outer", ctypes.c_int), ("coarse_avg", ctypes.c_int),
        ("reserved", ctypes.c_int * 7),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int), ("status", ctypes.c_int),
        ("relres0", ctypes.c_double), ("relres", ctypes.c_double),
        ("hist_len", ctypes.c_int),
        ("hist", ctypes.c_double * HIST_MAX),
        ("solve_ms", ctypes.c_double),
    ]

    def history(self):
        return [self.hist[i] for i in range(self.hist_len)]


class Result(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_ulonglong),
        ("info", Info),
        ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
        ("bytes", ctypes.c_size_t),
    ]


class StepParams(ctypes.Structure):
    _fields_ = [
        ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
        ("mu_l", ctypes.c_double), ("mu_g", ctypes.c_double),
        ("g", ctypes.c_double), ("sigma_t", ctypes.c_double), ("dt", ctypes.c_double),
        ("mg_cycles", ctypes.c_int), ("n_corr", ctypes.c_int), ("n_vel_iter", ctypes.c_int),
        ("mg_cycles_nh", ctypes.c_int), ("order", ctypes.c_int), ("reserved", ctypes.c_int * 3),
    ]


class StepInfo(ctypes.Structure):
    _fields_ = [
        ("solves", ctypes.c_int),
        ("relres", ctypes.c_double * 8),
        ("ms_total", ctypes.c_double), ("ms_mg", ctypes.c_double), ("volume", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load libnn4mg.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"nn4mg HIP library missing at {LIB_PATH}; build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    cfgp = ctypes.POINTER(Config)
    L.nn4mg_config_default.restype = None
    L.nn4mg_config_default.argtypes = [cfgp, i, i, i, d]
    L.nn4mg_bytes_required.restype = sz
    L.nn4mg_bytes_required.argtypes = [cfgp]
    L.nn4mg_setup.restype = i
    L.nn4mg_setup.argtypes = [cfgp, vp, vp, ctypes.POINTER(vp)]
    L.nn4mg_update_coef.restype = i
    L.nn4mg_update_coef.argtypes = [vp, vp]
    L.nn4mg_residual.restype = i
    L.nn4mg_residual.argtypes = [vp, vp, vp, vp, ctypes.POINTER(d)]
    L.nn4mg_vcycle.restype = i
    L.nn4mg_residual_noalloc.restype = i
    L.nn4mg_residual_noalloc.argtypes = [cfgp, vp, vp, vp, vp, ctypes.POINTER(d), vp]
    L.nn4mg_vcycle.argtypes = [vp, vp, vp]
    L.nn4mg_solve.restype = i
    L.nn4mg_solve.argtypes = [vp, vp, vp, d, i, i, ctypes.POINTER(Info)]
    L.nn4mg_levels.restype = i
    L.nn4mg_levels.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), i]
    L.nn4mg_bytes_held.restype = sz
    L.nn4mg_bytes_held.argtypes = [vp]
    L.nn4mg_profile.restype = i
    L.nn4mg_profile.argtypes = [vp, i]
    L.nn4mg_profile_read.restype = i
    L.nn4mg_profile_read.argtypes = [vp, i, ctypes.POINTER(i), ctypes.POINTER(d)]
    L.nn4mg_profile_read_level.restype = i
    L.nn4mg_profile_read_level.argtypes = [vp, i, i, ctypes.POINTER(i), ctypes.POINTER(d)]
    L.nn4mg_set_tiles.restype = i
    L.nn4mg_set_tiles.argtypes = [vp, i, i, i, i, i]
    L.nn4mg_get_tiles.restype = i
    L.nn4mg_get_tiles.argtypes = [vp, i, i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    L.nn4mg_autotune.restype = i
    L.nn4mg_autotune.argtypes = [vp, vp, vp, ctypes.POINTER(i), i]
    L.nn4mg_server_create.restype = i
    L.nn4mg_server_create.argtypes = [sz, i, ctypes.POINTER(vp)]
    L.nn4mg_server_submit.restype = i
    L.nn4mg_server_submit.argtypes = [vp, cfgp, vp, vp, vp, d, i, ctypes.c_ulonglong]
    L.nn4mg_server_poll.restype = i
    L.nn4mg_server_poll.argtypes = [vp, ctypes.POINTER(Result), i, ctypes.POINTER(i)]
    L.nn4mg_server_drain.restype = i
    L.nn4mg_server_drain.argtypes = [vp, d]
    L.nn4mg_server_stats.restype = i
    L.nn4mg_server_stats.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(i), ctypes.POINTER(i)]
    L.nn4mg_server_destroy.restype = i
    L.nn4mg_server_destroy.argtypes = [vp]
    stp = ctypes.POINTER(StepParams)
    L.nn4mg_step_params_default.restype = None
    L.nn4mg_step_params_default.argtypes = [stp]
    L.nn4mg_step_create.restype = i
    L.nn4mg_step_create.argtypes = [i, i, i, d, stp, vp, ctypes.POINTER(vp)]
    L.nn4mg_step.restype = i
    L.nn4mg_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(StepInfo)]
    L.nn4mg_step_run.restype = i
    L.nn4mg_step_run.argtypes = [vp, i, vp, vp, vp, vp, vp, vp, ctypes.POINTER(d), ctypes.POINTER(i),
                                 ctypes.POINTER(StepInfo)]
    L.nn4mg_step_destroy.restype = i
    L.nn4mg_step_destroy.argtypes = [vp]
    L.nn4mg_destroy.restype = i
    L.nn4mg_destroy.argtypes = [vp]
    L.nn4mg_last_error.restype = ctypes.c_char_p
    L.nn4mg_last_error.argtypes = []
    _lib = L
    return L


def _check(code):
    if code == NN4MG_OK:
        return
    msg = lib().nn4mg_last_error().decode()
    if code == NN4MG_ENOTCONV:
        raise NotConverged(code, msg)
    raise Nn4mgError(code, msg)


def config_default(nx, ny, nz, h, **kw) -> Config:
    c = Config()
    lib().nn4mg_config_default(ctypes.byref(c), int(nx), int(ny), int(nz), float(h))
    for key, val in kw.items():
        if key == "bc":
            for f in range(6):
                c.bc[f] = int(val[f])
        else:
            setattr(c, key, val)
    return c


def bytes_required(cfg: Config) -> int:
    return int(lib().nn4mg_bytes_required(ctypes.byref(cfg)))


def _field(t: torch.Tensor, n: int, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def residual_noalloc(cfg: Config, x: torch.Tensor, b: torch.Tensor, k: torch.Tensor | None = None,
                     r: torch.Tensor | None = None, norm: bool = True, stream: torch.cuda.Stream | None = None):
    """r = b - A x on the finest level of cfg with no hierarchy and no device
    allocation (nn4mg_residual_noalloc), on the current torch stream."""
    n = cfg.nx * cfg.ny * cfg.nz
    st = stream if stream is not None else torch.cuda.current_stream()
    out = ctypes.c_double(0.0)
    _check(lib().nn4mg_residual_noalloc(ctypes.byref(cfg), _field(k, n, "k") if k is not None else None,
                                        _field(x, n, "x"), _field(b, n, "b"),
                                        _field(r, n, "r") if r is not None else None,
                                        ctypes.byref(out) if norm else None, ctypes.c_void_p(st.cuda_stream)))
    return out.value if norm else None


class Hierarchy:
    """A multigrid hierarchy bound to the current torch stream (nn4mg_setup)."""

    def __init__(self, cfg: Config, k: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None):
        self.cfg = cfg
        self.n = cfg.nx * cfg.ny * cfg.nz
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        kp = _field(k, self.n, "k") if k is not None else None
        h = ctypes.c_void_p()
        _check(lib().nn4mg_setup(ctypes.byref(cfg), kp, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("hierarchy destroyed")
        return self._h

    def update_coef(self, k: torch.Tensor):
        _check(lib().nn4mg_update_coef(self.handle, _field(k, self.n, "k")))

    def residual(self, x: torch.Tensor, b: torch.Tensor, r: torch.Tensor | None = None, norm: bool = True):
        out = ctypes.c_double(0.0)
        _check(lib().nn4mg_residual(self.handle, _field(x, self.n, "x"), _field(b, self.n, "b"),
                                    _field(r, self.n, "r") if r is not None else None,
                                    ctypes.byref(out) if norm else None))
        return out.value if norm else None

    def vcycle(self, b: torch.Tensor, x: torch.Tensor):
        _check(lib().nn4mg_vcycle(self.handle, _field(b, self.n, "b"), _field(x, self.n, "x")))

    def solve(self, b: torch.Tensor, x: torch.Tensor, rtol: float = 1e-8, max_cycles: int = 100,
              fixed_cycles: bool = False, raise_on_notconv: bool = False) -> Info:
        info = Info()
        code = lib().nn4mg_solve(self.handle, _field(b, self.n, "b"), _field(x, self.n, "x"), float(rtol),
                                 int(max_cycles), int(bool(fixed_cycles)), ctypes.byref(info))
        if code == NN4MG_ENOTCONV and not raise_on_notconv:
            return info
        _check(code)
        return info

    def levels(self):
        L = ctypes.c_int(0)
        dims = (ctypes.c_int * 48)()
        _check(lib().nn4mg_levels(self.handle, ctypes.byref(L), dims, 16))
        return [(dims[3 * l], dims[3 * l + 1], dims[3 * l + 2]) for l in range(L.value)]

    def profile(self, enable: bool):
        _check(lib().nn4mg_profile(self.handle, int(bool(enable))))

    def profile_read(self, kclass: int):
        n = ctypes.c_int(0)
        ms = ctypes.c_double(0.0)
        _check(lib().nn4mg_profile_read(self.handle, int(kclass), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def profile_read_level(self, level: int, kclass: int):
        n = ctypes.c_int(0)
        ms = ctypes.c_double(0.0)
        _check(lib().nn4mg_profile_read_level(self.handle, int(level), int(kclass), ctypes.byref(n),
                                              ctypes.byref(ms)))
        return n.value, ms.value

    def set_tiles(self, level: int, tx: int, ry: int, zc: int, kclass: int = -1):
        _check(lib().nn4mg_set_tiles(self.handle, int(level), int(kclass), int(tx), int(ry), int(zc)))

    def get_tiles(self, level: int, kclass: int = 0):
        tx, ry, zc = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().nn4mg_get_tiles(self.handle, int(level), int(kclass), ctypes.byref(tx), ctypes.byref(ry),
                                     ctypes.byref(zc)))
        return tx.value, ry.value, zc.value

    def autotune(self, b: torch.Tensor, x: torch.Tensor):
        """Per level, a list of (tx, ry, zc) per kernel class (resid, first sweep, later sweeps)."""
        out = (ctypes.c_int * (9 * 16))()
        _check(lib().nn4mg_autotune(self.handle, _field(b, self.n, "b"), _field(x, self.n, "x"), out, 16))
        return [[(out[9 * l + 3 * c], out[9 * l + 3 * c + 1], out[9 * l + 3 * c + 2]) for c in range(3)]
                for l in range(len(self.levels()))]

    def bytes_held(self) -> int:
        return int(lib().nn4mg_bytes_held(self.handle))

    def close(self):
        if getattr(self, "_h", None):
            lib().nn4mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (nn4mg_server_*).  Tensors passed to
    submit() must stay alive and untouched until poll() returns their tag."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4):
        h = ctypes.c_void_p()
        _check(lib().nn4mg_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, cfg: Config, b: torch.Tensor, x: torch.Tensor, k: torch.Tensor | None = None,
               rtol: float = 1e-8, max_cycles: int = 1000, tag: int = 0):
        n = cfg.nx * cfg.ny * cfg.nz
        kp = _field(k, n, "k") if k is not None else None
        # the server's slot streams are not ordered after torch's: the inputs
        # must be complete on the device before the library copies them
        torch.cuda.current_stream().synchronize()
        _check(lib().nn4mg_server_submit(self._h, ctypes.byref(cfg), kp, _field(b, n, "b"), _field(x, n, "x"),
                                         float(rtol), int(max_cycles), int(tag)))
        # tags need not be unique: per tag, the count of requests in flight and
        # the tensors of all of them
        held = self._keep.setdefault(int(tag), [0, []])
        held[0] += 1
        held[1].append((cfg, b, x, k))

    def poll(self, cap: int = 256):
        out = (Result * cap)()
        nd = ctypes.c_int(0)
        _check(lib().nn4mg_server_poll(self._h, out, cap, ctypes.byref(nd)))
        res = [out[i] for i in range(nd.value)]
        for r in res:
            tag = int(r.tag)
            held = self._keep.get(tag)
            if held is not None:
                # a result names only its tag, so the tensors of a tag are
                # released together once every request with that tag is done
                held[0] -= 1
                if held[0] <= 0:
                    del self._keep[tag]
        return res

    def drain(self, timeout_ms: float = -1.0):
        _check(lib().nn4mg_server_drain(self._h, float(timeout_ms)))

    def stats(self):
        a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
        act, q = ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().nn4mg_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(act), ctypes.byref(q)))
        return dict(bytes_in_use=a.value, peak_bytes=b.value, active=act.value, queued=q.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().nn4mg_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STEP_FIELDS = ("C", "u", "v", "w", "p_hs", "p_nh")


def step_params(**kw) -> StepParams:
    p = StepParams()
    lib().nn4mg_step_params_default(ctypes.byref(p))
    for key, val in kw.items():
        setattr(p, key, val)
    return p


class Stepper:
    """Two-phase time step (nn4mg_step_*) on an nx x ny x nz grid, bound to the
    current torch stream.  step() advances a dict of device float64 tensors
    C, u, v, w, p_hs, p_nh in place."""

    def __init__(self, nx, ny, nz, h, params: StepParams | None = None, stream: torch.cuda.Stream | None = None):
        self.params = params if params is not None else step_params()
        self.n = int(nx) * int(ny) * int(nz)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h_ = ctypes.c_void_p()
        _check(lib().nn4mg_step_create(int(nx), int(ny), int(nz), float(h), ctypes.byref(self.params),
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h_)))
        self._h = h_

    def step(self, state: dict) -> StepInfo:
        if not self._h:
            raise RuntimeError("stepper destroyed")
        ptrs = [_field(state[k], self.n, k) for k in STEP_FIELDS]
        info = StepInfo()
        _check(lib().nn4mg_step(self._h, *ptrs, ctypes.byref(info)))
        return info

    def run(self, state: dict, nsteps: int, raise_on_breakdown: bool = True):
        """nsteps steps in place (nn4mg_step_run).  Returns (volumes, steps
        done, info of the last step): volumes[n] = sum C h^3 after step n,
        volumes[0] before the first."""
        if not self._h:
            raise RuntimeError("stepper destroyed")
        ptrs = [_field(state[k], self.n, k) for k in STEP_FIELDS]
        vol = (ctypes.c_double * (int(nsteps) + 1))()
        done = ctypes.c_int(0)
        info = StepInfo()
        code = lib().nn4mg_step_run(self._h, int(nsteps), *ptrs, vol, ctypes.byref(done), ctypes.byref(info))
        if not (code == NN4MG_EBREAKDOWN and not raise_on_breakdown):
            _check(code)
        n = done.value + (1 if code == NN4MG_EBREAKDOWN else 0)
        return [vol[i] for i in range(n + 1)], done.value, info

    def close(self):
        if getattr(self, "_h", None):
            lib().nn4mg_step_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
