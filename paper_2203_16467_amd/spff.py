"""Thin Python binding of the spff C ABI (include/spff.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides device memory (the workspace and field buffers) and the
stream.  The functions mirror the C entry points by name; ``Problem`` is a
small convenience wrapper around them.

The library is loaded from the package directory (built in-tree by
``paper_2203_16467_amd.build``).  There is no fallback: a missing or
unloadable library raises ``SpffLibraryError``.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspff.so")

OK, WARN_NOT_CONVERGED, E_INVALID, E_NOMEM, E_DEVICE, E_NONFINITE, E_BUSY = 0, 1, -1, -2, -3, -4, -5
AT1, AT2 = 1, 2
SPLIT_NONE, SPLIT_SPECTRAL, SPLIT_VOLDEV = 0, 1, 2
CONTACT_SAME = -1
EVOL_AM, EVOL_TIME, EVOL_NEAR_EQ = 0, 1, 2
NYQ_ZERO, NYQ_FREE = 0, 1
IRR_CRACK_SET, IRR_DAMAGE = 0, 1
FP32, FP64 = 0, 1
OP_PROJECT, OP_NEG_LAPLACIAN, OP_DISPLACEMENT = 0, 1, 2
FIELD_PHI, FIELD_PHI_REF, FIELD_STRAIN, FIELD_STRESS, FIELD_PSI_PLUS, FIELD_EPS_STAR, FIELD_DISP = (
    1, 2, 4, 8, 16, 32, 64)
FIELD_PLANES = {FIELD_PHI: 1, FIELD_PHI_REF: 1, FIELD_STRAIN: 3, FIELD_STRESS: 3, FIELD_PSI_PLUS: 1,
                FIELD_EPS_STAR: 3, FIELD_DISP: 2}
FIELD_NAMES = {FIELD_PHI: "phi", FIELD_PHI_REF: "phi_ref", FIELD_STRAIN: "strain", FIELD_STRESS: "stress",
               FIELD_PSI_PLUS: "psi_plus", FIELD_EPS_STAR: "eps_star", FIELD_DISP: "disp"}


class SpffLibraryError(RuntimeError):
    pass


class SpffError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"spff status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("at", ctypes.c_int32), ("split", ctypes.c_int32),
        ("irreversibility", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("nu", ctypes.c_double), ("ell", ctypes.c_double), ("gc", ctypes.c_double),
        ("crack_set_threshold", ctypes.c_double), ("k_res", ctypes.c_double), ("eta_over_dt", ctypes.c_double),
        ("tol_mech", ctypes.c_double), ("tol_abs_mech", ctypes.c_double),
        ("tol_pf", ctypes.c_double), ("tol_abs_pf", ctypes.c_double), ("tol_am", ctypes.c_double),
        ("max_cg", ctypes.c_int32), ("max_newton", ctypes.c_int32), ("max_bccg", ctypes.c_int32),
        ("max_am", ctypes.c_int32), ("ticks_per_sync", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("floor_factor", ctypes.c_double), ("stall_iters", ctypes.c_int32),
        ("plan_rows", ctypes.c_int32), ("plan_cols", ctypes.c_int32), ("plan_threads", ctypes.c_int32),
        ("contact", ctypes.c_int32), ("evolution", ctypes.c_int32),
        ("eta", ctypes.c_double), ("dt_max", ctypes.c_double), ("dt_min", ctypes.c_double),
        ("dphi_max", ctypes.c_double), ("dphi_min", ctypes.c_double),
        ("fphi_max", ctypes.c_double), ("drive_threshold", ctypes.c_double), ("deps_max", ctypes.c_double),
        ("nyquist", ctypes.c_int32),
    ]


class StepStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("am_iters", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
        ("cg_iters", ctypes.c_int32), ("bccg_iters", ctypes.c_int32), ("ticks", ctypes.c_int32),
        ("dphi_l1", ctypes.c_double), ("mech_residual", ctypes.c_double), ("pf_residual", ctypes.c_double),
        ("F_e", ctypes.c_double), ("F_f", ctypes.c_double), ("sigma_bar", ctypes.c_double * 3),
        ("C_bar", ctypes.c_double), ("phi_max", ctypes.c_double), ("phi_mean", ctypes.c_double),
        ("crack_px", ctypes.c_int64), ("wall_ms", ctypes.c_double),
        ("dt", ctypes.c_double), ("halvings", ctypes.c_int32), ("advance", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("fphi_max", ctypes.c_double), ("eps_bar", ctypes.c_double * 3),
        ("ne_flag", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def to_dict(self):
        out = {name: getattr(self, name) for name, _ in self._fields_}
        out["sigma_bar"] = list(self.sigma_bar)
        out["eps_bar"] = list(self.eps_bar)
        return out


class Profile(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double * 4), ("launches", ctypes.c_int64 * 4),
                ("alg_bytes", ctypes.c_double * 4), ("ticks", ctypes.c_int64),
                ("kernel_span_ms", ctypes.c_double * 4)]

    KERNELS = ("rowfwd", "col", "rowinv", "ctrl")

    def to_dict(self):
        return {"kernel_ms": dict(zip(self.KERNELS, self.kernel_ms)),
                "launches": dict(zip(self.KERNELS, self.launches)),
                "alg_bytes": dict(zip(self.KERNELS, self.alg_bytes)), "ticks": self.ticks,
                "kernel_span_ms": dict(zip(self.KERNELS, self.kernel_span_ms))}


FFT_LDS, FFT_REG, FFT_REG4 = 1, 2, 3


class Plan(ctypes.Structure):
    """spff_plan: launch plan of the three FFT kernels for one bucket."""
    _fields_ = [("row_kind", ctypes.c_int32), ("rows", ctypes.c_int32), ("row_threads", ctypes.c_int32),
                ("col_kind", ctypes.c_int32), ("cols", ctypes.c_int32), ("col_threads", ctypes.c_int32)]

    def to_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        return cls(**{k: int(d[k]) for k, _ in cls._fields_})


_lib = None

# C signatures: name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "spff_default_config": (None, [ctypes.POINTER(Config)]),
    "spff_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "spff_create_batch": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P,
                                         ctypes.POINTER(_P)]),
    "spff_create_problem": (ctypes.c_int, [ctypes.POINTER(Config), _P, _P, _P, ctypes.c_size_t, _P,
                                           ctypes.POINTER(_P)]),
    "spff_load_step_batch": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(StepStats)]),
    "spff_load_step": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(StepStats)]),
    "spff_run_sequence": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(StepStats)]),
    "spff_run_evolution": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(StepStats)]),
    "spff_get_fields": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "spff_state_bytes": (ctypes.c_size_t, [_P]),
    "spff_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "spff_set_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "spff_apply_operator": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "spff_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "spff_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(Profile)]),
    "spff_server_create": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(_P)]),
    "spff_server_register": (ctypes.c_int, [_P, ctypes.POINTER(Config), _P, ctypes.POINTER(ctypes.c_int32)]),
    "spff_server_submit": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "spff_server_progress": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "spff_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(StepStats)]),
    "spff_server_get_fields": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "spff_server_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "spff_server_destroy": (ctypes.c_int, [_P]),
    "spff_problem_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "spff_destroy_problem": (ctypes.c_int, [_P]),
    "spff_plan_buckets": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "spff_get_plan": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(Plan)]),
    "spff_set_plan": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(Plan)]),
    "spff_load_step_static": (ctypes.c_int, [ctypes.POINTER(Config), _P, _P, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(StepStats), _P]),
    "spff_last_error": (ctypes.c_char_p, []),
    "spff_version": (ctypes.c_char_p, []),
}


def lib():
    """Load libspff.so from the package directory (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SpffLibraryError(f"{LIB_PATH} is missing: build it with `python -m paper_2203_16467_amd.build`")
        try:
            L = ctypes.CDLL(LIB_PATH)
        except OSError as e:  # pragma: no cover - depends on the machine
            raise SpffLibraryError(f"cannot load {LIB_PATH}: {e}") from e
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().spff_last_error().decode()


def version():
    return lib().spff_version().decode()


def _check(status):
    if status < 0:
        raise SpffError(status, last_error())
    return status


def default_config(**overrides):
    cfg = Config()
    lib().spff_default_config(ctypes.byref(cfg))
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def workspace_bytes(cfg, nbatch=1):
    out = ctypes.c_size_t(0)
    _check(lib().spff_workspace_bytes(ctypes.byref(cfg), int(nbatch), ctypes.byref(out)))
    return out.value


def _torch():
    import torch  # imported lazily: the CPU-only ABI checks do not need it
    return torch


def _real_dtype(cfg):
    torch = _torch()
    return torch.float64 if cfg.precision == FP64 else torch.float32


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _aligned_workspace(nbytes, device):
    torch = _torch()
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw.data_ptr() + off


def create_batch(cfg, E, phi_init=None, stream=None):
    """spff_create_batch: E is a device tensor [B, ny, nx] (or [ny, nx]) of the
    configuration's real type.  Returns a ``Problem``."""
    return Problem(E, cfg, phi_init=phi_init, stream=stream)


def create_problem(cfg, E, phi_init=None, stream=None):
    """spff_create_problem: single problem, E of shape [ny, nx]."""
    return Problem(E, cfg, phi_init=phi_init, stream=stream)


class Problem:
    """Owns a workspace tensor and a spff_problem handle."""

    def __init__(self, E, cfg, phi_init=None, stream=None):
        torch = _torch()
        if not E.is_cuda:
            raise ValueError("E must be a device tensor")
        dt = _real_dtype(cfg)
        E = E.to(dt)
        if E.dim() == 2:
            E = E[None]
        self.B, ny, nx = E.shape
        if (ny, nx) != (cfg.ny, cfg.nx):
            raise ValueError(f"E shape {tuple(E.shape)} does not match config {cfg.ny}x{cfg.nx}")
        self.cfg = cfg
        self.device = E.device
        self.dtype = dt
        self.stream = stream if stream is not None else torch.cuda.current_stream(E.device)
        E = E.contiguous()
        pi = None
        if phi_init is not None:
            pi = phi_init.to(device=E.device, dtype=dt)
            if pi.dim() == 2:
                pi = pi[None]
            pi = pi.expand(self.B, ny, nx).contiguous()
        nbytes = workspace_bytes(cfg, self.B)
        self._ws, ws_ptr = _aligned_workspace(nbytes, E.device)
        h = ctypes.c_void_p()
        _check(lib().spff_create_batch(ctypes.byref(cfg), self.B, ctypes.c_void_p(E.data_ptr()),
                                       ctypes.c_void_p(pi.data_ptr() if pi is not None else 0),
                                       ctypes.c_void_p(ws_ptr), nbytes, _stream_ptr(self.stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().spff_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_step(self, eps_bar):
        """spff_load_step_batch.  eps_bar: (3,) applied to every problem or
        (B, 3).  Returns (status, [stats dict per problem])."""
        eb = np.asarray(eps_bar, dtype=np.float64)
        if eb.shape == (3,):
            eb = np.broadcast_to(eb, (self.B, 3))
        eb = np.ascontiguousarray(eb, dtype=np.float64)
        if eb.shape != (self.B, 3):
            raise ValueError("eps_bar must have shape (3,) or (B, 3)")
        stats = (StepStats * self.B)()
        st = lib().spff_load_step_batch(self.handle, eb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), stats)
        _check(st)
        return st, [s.to_dict() for s in stats]

    def run_sequence(self, eps_bar):
        """spff_run_sequence.  eps_bar: (K, 3) applied to every problem or
        (B, K, 3).  Returns (status, stats) with stats[b][k] a dict."""
        eb = np.asarray(eps_bar, dtype=np.float64)
        if eb.ndim == 2:
            eb = np.broadcast_to(eb, (self.B,) + eb.shape)
        eb = np.ascontiguousarray(eb, dtype=np.float64)
        if eb.ndim != 3 or eb.shape[0] != self.B or eb.shape[2] != 3:
            raise ValueError("eps_bar must have shape (K, 3) or (B, K, 3)")
        K = eb.shape[1]
        stats = (StepStats * (self.B * K))()
        st = lib().spff_run_sequence(self.handle, K, eb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), stats)
        _check(st)
        return st, [[stats[b * K + k].to_dict() for k in range(K)] for b in range(self.B)]

    def run_evolution(self, deps, nsteps=None):
        """spff_run_evolution (Algorithm 3 or 4 on the device).  deps: (3,)
        constant increment (then nsteps is required), (K, 3) applied to
        every problem, or (B, K, 3).  Returns (status, stats)."""
        d = np.asarray(deps, dtype=np.float64)
        if d.ndim == 1:
            if nsteps is None:
                raise ValueError("nsteps is required with a constant increment")
            d = np.broadcast_to(d, (int(nsteps), 3))
        if d.ndim == 2:
            d = np.broadcast_to(d, (self.B,) + d.shape)
        d = np.ascontiguousarray(d, dtype=np.float64)
        if d.ndim != 3 or d.shape[0] != self.B or d.shape[2] != 3:
            raise ValueError("deps must have shape (3,), (K, 3) or (B, K, 3)")
        K = d.shape[1]
        stats = (StepStats * (self.B * K))()
        st = lib().spff_run_evolution(self.handle, K, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), stats)
        _check(st)
        return st, [[stats[b * K + k].to_dict() for k in range(K)] for b in range(self.B)]

    def get_fields(self, mask, index=-1):
        """spff_get_fields: returns {name: tensor}; index = -1 gives every
        problem ([B, planes, ny, nx]), else one problem ([planes, ny, nx])."""
        torch = _torch()
        outs, ptrs = {}, []
        nb = self.B if index < 0 else 1
        for bit in sorted(FIELD_PLANES):
            if mask & bit:
                t = torch.empty((nb, FIELD_PLANES[bit], self.cfg.ny, self.cfg.nx), dtype=self.dtype,
                                device=self.device)
                outs[FIELD_NAMES[bit]] = t if index < 0 else t[0]
                ptrs.append(t.data_ptr())
        arr = (ctypes.c_void_p * max(1, len(ptrs)))(*ptrs)
        _check(lib().spff_get_fields(self.handle, int(index), int(mask), arr))
        return outs

    def apply_operator(self, op, x):
        """spff_apply_operator: G (op=OP_PROJECT, x [B,3,ny,nx]), -lap_N
        (op=OP_NEG_LAPLACIAN, x [B,ny,nx]) or the displacement of a strain
        field (op=OP_DISPLACEMENT, x [B,3,ny,nx] -> [B,2,ny,nx]); returns a
        new tensor."""
        x = x.to(device=self.device, dtype=self.dtype).contiguous()
        if op == OP_DISPLACEMENT:
            if x.dim() != 4 or x.shape[1] != 3:
                raise ValueError("displacement operator needs x of shape [B, 3, ny, nx]")
            out = _torch().empty((x.shape[0], 2) + tuple(x.shape[2:]), dtype=self.dtype, device=self.device)
        else:
            out = _torch().empty_like(x)
        _check(lib().spff_apply_operator(self.handle, int(op), ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr())))
        return out

    def profile_enable(self, on=True):
        """spff_profile_enable (resets the totals)."""
        _check(lib().spff_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        """spff_profile_read -> dict of per-kernel time, launches, bytes."""
        out = Profile()
        _check(lib().spff_profile_read(self.handle, ctypes.byref(out)))
        return out.to_dict()

    def plan_buckets(self):
        """Slot counts of the launch buckets (spff_plan_buckets)."""
        n = ctypes.c_int32(0)
        _check(lib().spff_plan_buckets(self.handle, ctypes.byref(n), None))
        sizes = (ctypes.c_int32 * n.value)()
        _check(lib().spff_plan_buckets(self.handle, ctypes.byref(n), sizes))
        return list(sizes)

    def get_plan(self, bucket):
        pl = Plan()
        _check(lib().spff_get_plan(self.handle, int(bucket), ctypes.byref(pl)))
        return pl.to_dict()

    def set_plan(self, bucket, plan=None):
        """Install a plan (dict of spff_plan fields) for a bucket; None
        restores the built-in heuristic.  Returns the plan in use."""
        if plan is None:
            _check(lib().spff_set_plan(self.handle, int(bucket), None))
            return self.get_plan(bucket)
        pl = Plan.from_dict(plan)
        _check(lib().spff_set_plan(self.handle, int(bucket), ctypes.byref(pl)))
        return pl.to_dict()

    def get_state(self):
        """spff_get_state: (state tensor [B, 5, ny, nx], eps_bar (B, 3))."""
        torch = _torch()
        t = torch.empty((self.B, 5, self.cfg.ny, self.cfg.nx), dtype=self.dtype, device=self.device)
        eb = np.zeros((self.B, 3))
        _check(lib().spff_get_state(self.handle, ctypes.c_void_p(t.data_ptr()),
                                    eb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return t, eb

    def set_state(self, state, eps_bar=None):
        """spff_set_state from a tensor [B, 5, ny, nx] of the real type."""
        state = state.to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(state.shape) != (self.B, 5, self.cfg.ny, self.cfg.nx):
            raise ValueError("state shape mismatch")
        ebp = None
        if eps_bar is not None:
            eb = np.ascontiguousarray(np.broadcast_to(np.asarray(eps_bar, np.float64), (self.B, 3)))
            ebp = eb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(lib().spff_set_state(self.handle, ctypes.c_void_p(state.data_ptr()), ebp))


STATIC_SCRATCH_BYTES = 64 << 20


def load_step_static(cfg, E, state, eps_bar, stream=None):
    """spff_load_step_static: one load step of one problem whose state
    (device tensor [5, ny, nx] = eps*[3], phi, phi_ref, of the config's real
    type, contiguous) is updated in place; all solver scratch is the
    library's static device array (no allocation by the library or here).
    Returns (status, stats dict)."""
    dt = _real_dtype(cfg)
    if not (E.is_cuda and state.is_cuda) or E.dtype != dt or state.dtype != dt:
        raise ValueError("E and state must be device tensors of the configuration's real type")
    if tuple(E.shape[-2:]) != (cfg.ny, cfg.nx) or tuple(state.shape) != (5, cfg.ny, cfg.nx):
        raise ValueError("E must be [ny, nx] and state [5, ny, nx]")
    if not (E.is_contiguous() and state.is_contiguous()):
        raise ValueError("E and state must be contiguous")
    eb = (ctypes.c_double * 3)(*[float(v) for v in eps_bar])
    out = StepStats()
    st = lib().spff_load_step_static(ctypes.byref(cfg), ctypes.c_void_p(E.data_ptr()),
                                     ctypes.c_void_p(state.data_ptr()), eb, ctypes.byref(out),
                                     _stream_ptr(stream))
    _check(st)
    return st, out.to_dict()


class Server:
    """Continuous-batching server over resident problems (spff_server_*).

    arena_bytes of device memory are allocated once with torch; the library
    sub-allocates resident state and class engines from it."""

    def __init__(self, arena_bytes, scratch_budget_bytes=0, ticks_per_sync=8, use_graph=1, device="cuda:0"):
        torch = _torch()
        self.device = torch.device(device)
        self._arena, ptr = _aligned_workspace(int(arena_bytes), self.device)
        h = ctypes.c_void_p()
        _check(lib().spff_server_create(ctypes.c_void_p(ptr), int(arena_bytes), int(scratch_budget_bytes),
                                        int(ticks_per_sync), int(use_graph), ctypes.byref(h)))
        self.handle = h
        self.cfgs = []

    def close(self):
        if getattr(self, "handle", None):
            lib().spff_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def register(self, cfg, E):
        """spff_server_register: E device tensor [ny, nx] of the config's real type."""
        E = E.to(device=self.device, dtype=_real_dtype(cfg)).contiguous()
        out = ctypes.c_int32()
        _check(lib().spff_server_register(self.handle, ctypes.byref(cfg), ctypes.c_void_p(E.data_ptr()),
                                          ctypes.byref(out)))
        self.cfgs.append(cfg)
        return out.value

    def submit(self, pid, eps_bar):
        eb = (ctypes.c_double * 3)(*[float(v) for v in eps_bar])
        t = ctypes.c_uint64()
        _check(lib().spff_server_submit(self.handle, int(pid), eb, ctypes.byref(t)))
        return t.value

    def progress(self, max_rounds=1):
        c, p = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().spff_server_progress(self.handle, int(max_rounds), ctypes.byref(c), ctypes.byref(p)))
        return c.value, p.value

    def poll(self, ticket):
        """Stats dict when done, None while pending."""
        out = StepStats()
        st = lib().spff_server_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(out))
        if st == E_BUSY:
            return None
        _check(st)
        return out.to_dict()

    def get_fields(self, pid, mask):
        torch = _torch()
        cfg = self.cfgs[pid]
        outs, ptrs = {}, []
        for bit in (FIELD_PHI, FIELD_PHI_REF, FIELD_EPS_STAR):
            if mask & bit:
                t = torch.empty((FIELD_PLANES[bit], cfg.ny, cfg.nx), dtype=_real_dtype(cfg), device=self.device)
                outs[FIELD_NAMES[bit]] = t
                ptrs.append(t.data_ptr())
        arr = (ctypes.c_void_p * max(1, len(ptrs)))(*ptrs)
        _check(lib().spff_server_get_fields(self.handle, int(pid), int(mask), arr))
        return outs

    def info(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(lib().spff_server_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"classes": a.value, "slots": b.value, "arena_used": c.value}
