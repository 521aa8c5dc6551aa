"""ctypes binding of the C ABI declared in include/imexhdg.h.

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch provides the device workspace and the stream.  Importing
this module imports torch first, so that the library binds to the HIP
runtime torch has already loaded.  A missing library raises at load time.
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libimexhdg.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NOCONV, E_NONFINITE, E_STATE = 0, -1, -2, -3, -4, -5, -6
SCHEME_ARS232, SCHEME_ARS443 = 0, 1
PHYSICS_LINEARIZED, PHYSICS_NONLINEAR = 0, 1
PREC_FP64, PREC_MIXED, PREC_FP32, PREC_BF16 = 0, 1, 2, 3
LAUNCH_GRAPH, LAUNCH_HOST = 0, 1
GUESS_EXTRAPOLATE, GUESS_LAST = 0, 1
VARS_DEPTH, VARS_GEOPOTENTIAL = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1
BOUNDARY_PERIODIC, BOUNDARY_VORTEX, BOUNDARY_WALL = 0, 1, 2
PHASES = ["explicit", "condense", "trace", "recover", "other"]

EXPORTS = [
    "imexhdg_config_init", "imexhdg_validate", "imexhdg_workspace_bytes",
    "imexhdg_create", "imexhdg_destroy", "imexhdg_sizes", "imexhdg_get_nodes",
    "imexhdg_set_state", "imexhdg_set_state_device", "imexhdg_set_depth", "imexhdg_get_state",
    "imexhdg_step",
    "imexhdg_get_diag",
    "imexhdg_last_error", "imexhdg_state_device", "imexhdg_nl_residual",
    "imexhdg_linear_residual", "imexhdg_stage_solve", "imexhdg_stage_solve_noalloc",
    "imexhdg_profile",
    "imexhdg_profile_read", "imexhdg_profile_read_min", "imexhdg_kernel_name",
    "imexhdg_get_schedule",
    "imexhdg_set_schedule", "imexhdg_set_launch_geometry", "imexhdg_autotune",
    "imexhdg_ens_workspace_bytes", "imexhdg_ens_create", "imexhdg_ens_destroy",
    "imexhdg_ens_members", "imexhdg_ens_sizes", "imexhdg_ens_get_nodes",
    "imexhdg_ens_set_state", "imexhdg_ens_set_state_device", "imexhdg_ens_get_state",
    "imexhdg_ens_step",
    "imexhdg_ens_get_diag", "imexhdg_ens_get_schedule", "imexhdg_ens_set_launch_geometry",
    "imexhdg_ens_autotune",
]
KERNELS = ["nl_residual", "combine", "local_apply", "trace_rhs", "trace_residual", "bicg_init",
           "bicg_k1", "bicg_k2", "bicg_k1f", "axpy", "recover", "diag", "linear_residual"]


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
        ("degree", ctypes.c_int32),
        ("g", ctypes.c_double), ("H", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("scheme", ctypes.c_int32), ("physics", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("krylov_rtol", ctypes.c_double),
        ("krylov_max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("refine_rtol", ctypes.c_double), ("refine_max", ctypes.c_int32),
        ("launch", ctypes.c_int32), ("trace_guess", ctypes.c_int32),
        ("local_sweeps", ctypes.c_int32),
        ("boundary", ctypes.c_int32),
        ("variable_depth", ctypes.c_int32),
        ("vortex", ctypes.c_double * 5),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double * 3), ("energy", ctypes.c_double),
        ("steps", ctypes.c_int64), ("krylov_iters", ctypes.c_int64),
        ("stage_solves", ctypes.c_int64), ("refine_sweeps", ctypes.c_int64),
        ("last_relres", ctypes.c_double), ("max_relres", ctypes.c_double),
        ("nonfinite", ctypes.c_int32),
        ("graph_steps", ctypes.c_int64), ("redo_steps", ctypes.c_int64),
        ("step_ms", ctypes.c_double), ("phase_ms", ctypes.c_double * 5),
        ("depth_corrections", ctypes.c_int64),
    ]


def _diag_dict(d):
    out = {f: (list(getattr(d, f)) if f in ("mass", "phase_ms") else getattr(d, f))
           for f, _ in Diag._fields_}
    out["phase_ms"] = dict(zip(PHASES, out["phase_ms"]))
    return out


def _device_state(t, n_nodes, device):
    """(pointer, dtype code) of a contiguous (3, n_nodes) FP64 / FP32 tensor
    on the context's device; the tensor must stay alive for the call."""
    want = device.index if device.index is not None else torch.cuda.current_device()
    if not isinstance(t, torch.Tensor) or t.device.type != device.type or t.device.index != want:
        raise ValueError("device state must be a tensor on the context's device")
    if t.dtype not in (torch.float64, torch.float32):
        raise ValueError("device state must be float64 or float32")
    if not t.is_contiguous() or t.numel() != 3 * n_nodes:
        raise ValueError("device state must be a contiguous (3, n_nodes) tensor")
    return ctypes.c_void_p(t.data_ptr()), (DTYPE_F64 if t.dtype == torch.float64 else DTYPE_F32)


class ImexError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"imexhdg error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libimexhdg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1711_02751_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    cfgp = ctypes.POINTER(Config)
    sig = {
        "imexhdg_config_init": (ctypes.c_int, [cfgp]),
        "imexhdg_validate": (ctypes.c_int, [cfgp]),
        "imexhdg_workspace_bytes": (ctypes.c_int, [cfgp, ctypes.POINTER(ctypes.c_size_t)]),
        "imexhdg_create": (ctypes.c_int, [cfgp, P, P, ctypes.c_size_t, ctypes.POINTER(P)]),
        "imexhdg_destroy": (None, [P]),
        "imexhdg_sizes": (ctypes.c_int, [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "imexhdg_get_nodes": (ctypes.c_int, [P, P, P]),
        "imexhdg_set_state": (ctypes.c_int, [P, ctypes.c_int, P, P, P]),
        "imexhdg_get_state": (ctypes.c_int, [P, ctypes.c_int, P, P, P]),
        "imexhdg_set_state_device": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P]),
        "imexhdg_step": (ctypes.c_int, [P, i32]),
        "imexhdg_get_diag": (ctypes.c_int, [P, ctypes.POINTER(Diag)]),
        "imexhdg_last_error": (ctypes.c_char_p, []),
        "imexhdg_state_device": (ctypes.c_int, [P, ctypes.POINTER(P)]),
        "imexhdg_nl_residual": (ctypes.c_int, [P, P, P]),
        "imexhdg_linear_residual": (ctypes.c_int, [P, P, P, P]),
        "imexhdg_stage_solve": (ctypes.c_int, [P, P, P, P, ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "imexhdg_stage_solve_noalloc": (ctypes.c_int, [P, P, P, P, ctypes.POINTER(i32),
                                                       ctypes.POINTER(dbl)]),
        "imexhdg_profile": (ctypes.c_int, [P, i32]),
        "imexhdg_profile_read": (ctypes.c_int, [P, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl)]),
        "imexhdg_profile_read_min": (ctypes.c_int, [P, i32, dbl, ctypes.POINTER(i64),
                                                    ctypes.POINTER(dbl)]),
        "imexhdg_kernel_name": (ctypes.c_char_p, [i32]),
        "imexhdg_get_schedule": (ctypes.c_int, [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "imexhdg_set_schedule": (ctypes.c_int, [P, i32, ctypes.POINTER(i32)]),
        "imexhdg_set_launch_geometry": (ctypes.c_int, [P, i32, i32]),
        "imexhdg_ens_workspace_bytes": (ctypes.c_int, [cfgp, i32, ctypes.POINTER(ctypes.c_size_t)]),
        "imexhdg_ens_create": (ctypes.c_int, [cfgp, i32, P, P, ctypes.c_size_t,
                                              ctypes.POINTER(P)]),
        "imexhdg_ens_destroy": (None, [P]),
        "imexhdg_ens_members": (ctypes.c_int, [P, ctypes.POINTER(i32)]),
        "imexhdg_ens_sizes": (ctypes.c_int, [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "imexhdg_ens_get_nodes": (ctypes.c_int, [P, i32, P, P]),
        "imexhdg_ens_set_state": (ctypes.c_int, [P, i32, ctypes.c_int, P, P, P]),
        "imexhdg_ens_get_state": (ctypes.c_int, [P, i32, ctypes.c_int, P, P, P]),
        "imexhdg_ens_set_state_device": (ctypes.c_int, [P, i32, ctypes.c_int, ctypes.c_int, P]),
        "imexhdg_ens_step": (ctypes.c_int, [P, i32]),
        "imexhdg_ens_get_diag": (ctypes.c_int, [P, i32, ctypes.POINTER(Diag)]),
        "imexhdg_ens_get_schedule": (ctypes.c_int, [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "imexhdg_ens_set_launch_geometry": (ctypes.c_int, [P, i32, i32]),
        "imexhdg_ens_autotune": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.POINTER(i32),
                                                ctypes.POINTER(i32)]),
        "imexhdg_autotune": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.POINTER(i32),
                                            ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise ImexError(rc, load().imexhdg_last_error().decode())
    return rc


def default_config(**kw):
    cfg = Config()
    _check(load().imexhdg_config_init(ctypes.byref(cfg)))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise TypeError(f"unknown config field {k}")
        if k == "vortex":
            v = (ctypes.c_double * 5)(*[float(a) for a in v])
        setattr(cfg, k, v)
    return cfg


def validate(cfg):
    return load().imexhdg_validate(ctypes.byref(cfg))


def workspace_bytes(cfg):
    n = ctypes.c_size_t(0)
    _check(load().imexhdg_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def _ptr(a):
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


class Solver:
    """One IMEX HDG-DG context on the current CUDA (HIP) device and stream."""

    def __init__(self, cfg=None, device="cuda", **kw):
        self.lib = load()
        self.cfg = cfg if cfg is not None else default_config(**kw)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        nbytes = workspace_bytes(self.cfg)
        # torch owns the device workspace; the context borrows it
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._ctx = ctypes.c_void_p()
        _check(self.lib.imexhdg_create(ctypes.byref(self.cfg),
                                       ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.c_void_p(aligned), nbytes,
                                       ctypes.byref(self._ctx)))
        nn, nt = ctypes.c_int64(), ctypes.c_int64()
        _check(self.lib.imexhdg_sizes(self._ctx, ctypes.byref(nn), ctypes.byref(nt)))
        self.n_nodes, self.n_trace = nn.value, nt.value
        self.K = self.cfg.degree + 1
        # elements of the device layout (a bounded mesh is padded by two ghost
        # columns and rows)
        self.nel = self.n_trace // (6 * self.K)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self.lib.imexhdg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- host-side state
    def nodes(self):
        x = np.empty(self.n_nodes)
        y = np.empty(self.n_nodes)
        _check(self.lib.imexhdg_get_nodes(self._ctx, _ptr(x), _ptr(y)))
        return x, y

    def set_state(self, a, b, c, vars=VARS_DEPTH):
        arrs = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel()) for v in (a, b, c)]
        for v in arrs:
            if v.size != self.n_nodes:
                raise ValueError("state arrays must hold n_nodes values")
        _check(self.lib.imexhdg_set_state(self._ctx, vars, *[_ptr(v) for v in arrs]))

    def set_depth(self, B):
        """Nodal depth under the reference plane (variable_depth = 1),
        n_nodes values in the host state ordering."""
        b = np.ascontiguousarray(np.asarray(B, dtype=np.float64).ravel())
        if b.size != self.n_nodes:
            raise ValueError("depth must hold n_nodes values")
        _check(self.lib.imexhdg_set_depth(self._ctx, _ptr(b)))

    def set_state_device(self, t, vars=VARS_DEPTH):
        """State from a device tensor of shape (3, n_nodes) (host state
        ordering per variable), float64 or float32, without a host copy."""
        p, dt = _device_state(t, self.n_nodes, self.device)
        _check(self.lib.imexhdg_set_state_device(self._ctx, vars, dt, p))

    def get_state(self, vars=VARS_DEPTH):
        out = [np.empty(self.n_nodes) for _ in range(3)]
        _check(self.lib.imexhdg_get_state(self._ctx, vars, *[_ptr(v) for v in out]))
        return out

    def step(self, n=1, allow_noconv=False):
        return _check(self.lib.imexhdg_step(self._ctx, int(n)),
                      allow=(E_NOCONV,) if allow_noconv else ())

    def diag(self):
        d = Diag()
        _check(self.lib.imexhdg_get_diag(self._ctx, ctypes.byref(d)))
        return _diag_dict(d)

    # ---- event profiler
    def profile(self, kernel=-1):
        """kernel: class name or id; -1 all classes, -2 off."""
        if isinstance(kernel, str):
            kernel = KERNELS.index(kernel)
        _check(self.lib.imexhdg_profile(self._ctx, int(kernel)))

    def profile_read(self, kernel, min_us=0.0):
        """(launches, total ms) of a class since profile(); with min_us > 0,
        over the launches that took at least min_us only."""
        if isinstance(kernel, str):
            kernel = KERNELS.index(kernel)
        n, ms = ctypes.c_int64(), ctypes.c_double()
        if min_us > 0.0:
            _check(self.lib.imexhdg_profile_read_min(self._ctx, int(kernel), min_us / 1000.0,
                                                     ctypes.byref(n), ctypes.byref(ms)))
        else:
            _check(self.lib.imexhdg_profile_read(self._ctx, int(kernel), ctypes.byref(n),
                                                 ctypes.byref(ms)))
        return n.value, ms.value

    # ---- fixed launch schedule (LAUNCH_GRAPH)
    def schedule(self):
        """(sweeps, [inner-iteration budget per sweep]) of the captured step."""
        n = ctypes.c_int32()
        b = (ctypes.c_int32 * 8)()
        _check(self.lib.imexhdg_get_schedule(self._ctx, ctypes.byref(n), b))
        return n.value, list(b)[:n.value]

    def set_schedule(self, budgets):
        b = (ctypes.c_int32 * max(8, len(budgets)))(*[int(v) for v in budgets])
        _check(self.lib.imexhdg_set_schedule(self._ctx, len(budgets), b))

    # ---- launch geometry
    def set_launch_geometry(self, face_grid, elem_grid):
        _check(self.lib.imexhdg_set_launch_geometry(self._ctx, int(face_grid), int(elem_grid)))

    def autotune(self, cache_path=None):
        """Tune the Krylov grid caps on the current state; returns them."""
        f, e = ctypes.c_int32(), ctypes.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self.lib.imexhdg_autotune(self._ctx, path, ctypes.byref(f), ctypes.byref(e)))
        return f.value, e.value

    # ---- operator-level calls on device tensors (volume / trace device layout)
    def state_device_ptr(self):
        p = ctypes.c_void_p()
        _check(self.lib.imexhdg_state_device(self._ctx, ctypes.byref(p)))
        return p.value

    def volume_empty(self):
        return torch.empty(3 * self.n_nodes, dtype=torch.float64, device=self.device)

    def trace_zeros(self):
        return torch.zeros(self.n_trace, dtype=torch.float64, device=self.device)

    def nl_residual(self, q):
        out = self.volume_empty()
        _check(self.lib.imexhdg_nl_residual(self._ctx, _ptr(q), _ptr(out)))
        return out

    def linear_residual(self, Q, qhat):
        out = self.volume_empty()
        _check(self.lib.imexhdg_linear_residual(self._ctx, _ptr(Q), _ptr(qhat), _ptr(out)))
        return out

    def stage_solve(self, res0, qhat=None, allow_noconv=False):
        Q = self.volume_empty()
        qh = self.trace_zeros() if qhat is None else qhat.clone()
        it, rr = ctypes.c_int32(), ctypes.c_double()
        _check(self.lib.imexhdg_stage_solve(self._ctx, _ptr(res0), _ptr(Q), _ptr(qh),
                                            ctypes.byref(it), ctypes.byref(rr)),
               allow=(E_NOCONV,) if allow_noconv else ())
        return Q, qh, it.value, rr.value

    def stage_solve_noalloc(self, res0, Q, qhat, allow_noconv=False):
        """imexhdg_stage_solve_noalloc into caller-provided tensors: Q
        (3 n_nodes FP64) receives the stage state, qhat (n_trace FP64) holds
        the guess on entry and the trace on exit.  Returns (iterations,
        relative residual)."""
        it, rr = ctypes.c_int32(), ctypes.c_double()
        _check(self.lib.imexhdg_stage_solve_noalloc(self._ctx, _ptr(res0), _ptr(Q), _ptr(qhat),
                                                    ctypes.byref(it), ctypes.byref(rr)),
               allow=(E_NOCONV,) if allow_noconv else ())
        return it.value, rr.value


# ---- layout helpers (host numpy <-> device layout of the C ABI)
def volume_to_device_layout(q, nel, K):
    """q: (3, n_nodes) in host ordering [e][j*K+i] -> flat [c][node][e]."""
    q = np.asarray(q).reshape(3, nel, K * K)
    return np.ascontiguousarray(q.transpose(0, 2, 1)).ravel()


def volume_from_device_layout(v, nel, K):
    v = np.asarray(v).reshape(3, K * K, nel)
    return np.ascontiguousarray(v.transpose(0, 2, 1)).reshape(3, nel * K * K)


class Ensemble:
    """Members stepped together: every launch covers all members, one graph
    launch per step.  cfgs: list of Config that differ in nx, ny, Lx, Ly, dt
    only (LAUNCH_GRAPH)."""

    def __init__(self, cfgs, device="cuda"):
        self.lib = load()
        self.cfgs = list(cfgs)
        n = len(self.cfgs)
        self._arr = (Config * n)(*self.cfgs)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        nb = ctypes.c_size_t(0)
        _check(self.lib.imexhdg_ens_workspace_bytes(self._arr, n, ctypes.byref(nb)))
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self._ens = ctypes.c_void_p()
        _check(self.lib.imexhdg_ens_create(self._arr, n, ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.c_void_p(aligned), nb.value,
                                           ctypes.byref(self._ens)))
        self.n = n
        self.n_nodes, self.n_trace = [], []
        for m in range(n):
            nn, nt = ctypes.c_int64(), ctypes.c_int64()
            _check(self.lib.imexhdg_ens_sizes(self._ens, m, ctypes.byref(nn), ctypes.byref(nt)))
            self.n_nodes.append(nn.value)
            self.n_trace.append(nt.value)

    def close(self):
        if getattr(self, "_ens", None) and self._ens.value:
            self.lib.imexhdg_ens_destroy(self._ens)
            self._ens = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nodes(self, m):
        x = np.empty(self.n_nodes[m])
        y = np.empty(self.n_nodes[m])
        _check(self.lib.imexhdg_ens_get_nodes(self._ens, m, _ptr(x), _ptr(y)))
        return x, y

    def set_state(self, m, a, b, c, vars=VARS_DEPTH):
        arrs = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel()) for v in (a, b, c)]
        for v in arrs:
            if v.size != self.n_nodes[m]:
                raise ValueError("state arrays must hold the member's n_nodes values")
        _check(self.lib.imexhdg_ens_set_state(self._ens, m, vars, *[_ptr(v) for v in arrs]))

    def set_state_device(self, m, t, vars=VARS_DEPTH):
        p, dt = _device_state(t, self.n_nodes[m], self.device)
        _check(self.lib.imexhdg_ens_set_state_device(self._ens, m, vars, dt, p))

    def get_state(self, m, vars=VARS_DEPTH):
        out = [np.empty(self.n_nodes[m]) for _ in range(3)]
        _check(self.lib.imexhdg_ens_get_state(self._ens, m, vars, *[_ptr(v) for v in out]))
        return out

    def step(self, n=1, allow_noconv=False):
        return _check(self.lib.imexhdg_ens_step(self._ens, int(n)),
                      allow=(E_NOCONV,) if allow_noconv else ())

    def diag(self, m):
        d = Diag()
        _check(self.lib.imexhdg_ens_get_diag(self._ens, m, ctypes.byref(d)))
        return _diag_dict(d)

    def schedule(self):
        n = ctypes.c_int32()
        b = (ctypes.c_int32 * 8)()
        _check(self.lib.imexhdg_ens_get_schedule(self._ens, ctypes.byref(n), b))
        return n.value, list(b)[:n.value]

    def set_launch_geometry(self, face_grid, elem_grid):
        _check(self.lib.imexhdg_ens_set_launch_geometry(self._ens, int(face_grid),
                                                        int(elem_grid)))

    def autotune(self, cache_path=None):
        """Tune the per-member face blocks on the current state; returns
        (cap, tiles per block), the latter 0 when the blocks are capped."""
        f, t = ctypes.c_int32(), ctypes.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self.lib.imexhdg_ens_autotune(self._ens, path, ctypes.byref(f), ctypes.byref(t)))
        return f.value, t.value
