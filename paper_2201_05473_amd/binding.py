"""ctypes binding of liblbmpwfa (include/lbmpwfa.h).

Argument marshalling only: every step of the path runs in the library's HIP kernels.  torch
provides the device workspace (a uint8 tensor) and the stream handle.  The functions named
``lbm_*`` mirror the C entry points one to one; ``Lattice`` is a small convenience owner of a
context and its workspace.  If the library is missing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_F64, LBM_F32, LBM_F16, LBM_F16N = 0, 1, 2, 3
_STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16": LBM_F16, "f16n": LBM_F16N}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbmpwfa.so")

c_int32, c_int64, c_double, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                  ctypes.c_size_t, ctypes.c_void_p)


class LbmConfig(ctypes.Structure):
    _fields_ = [
        ("nz", c_int32), ("nr", c_int32),
        ("dz", c_double), ("dr", c_double), ("c_dt_over_dz", c_double), ("tau", c_double),
        ("storage", c_int32),
        ("moving_window", c_int32), ("periodic", c_int32), ("fields_on", c_int32), ("cyl_on", c_int32),
        ("n0", c_double),
        ("ramp_kind", c_int32),
        ("ramp_start", c_double), ("ramp_len", c_double),
        ("nb", c_double), ("sigma_z", c_double), ("sigma_r", c_double), ("zd0", c_double),
        ("n_floor", c_double),
        ("check_every", c_int32),
        ("fp64_math", c_int32),
        ("collision", c_int32),
        ("trt_magic", c_double),
        ("driver", c_int32),
        ("max_particles", c_int64),
        ("mrt_se", c_double), ("mrt_seps", c_double), ("mrt_sq", c_double), ("mrt_spi", c_double),
        ("resort_every", c_int32),
        ("bunch_streaming", c_int32),
    ]


class LbmDiag(ctypes.Structure):
    _fields_ = [
        ("charge", c_double), ("field_energy", c_double), ("gauss_max", c_double), ("umax", c_double),
        ("step", c_int64), ("shifts", c_int64), ("nonfinite", c_int32), ("reserved", c_int32),
    ]


class LbmObjective(ctypes.Structure):
    _fields_ = [("z_behind", c_double), ("row", c_int32)]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblbmpwfa error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load the HIP library (once).  Raises OSError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"{p} not found: build it with paper_2201_05473_amd/build.py (no fallback exists)")
    # torch first: the library then binds to the HIP runtime torch has loaded, so that torch's
    # device memory and stream handles are valid in it (one runtime per process)
    import torch  # noqa: F401
    lib = ctypes.CDLL(p)
    P = ctypes.POINTER
    sig = {
        "lbm_workspace_bytes": (c_int32, [P(LbmConfig), P(c_size_t)]),
        "lbm_init": (c_int32, [P(LbmConfig), c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, P(c_void_p)]),
        "lbm_step": (c_int32, [c_void_p, c_int64]),
        "lbm_moments": (c_int32, [c_void_p, c_void_p, c_int32, c_int32]),
        "lbm_fields": (c_int32, [c_void_p, c_void_p, c_int32, c_int32]),
        "lbm_get_state": (c_int32, [c_void_p, c_void_p, P(c_int64), P(c_int64)]),
        "lbm_set_state": (c_int32, [c_void_p, c_void_p, c_int64, c_int64]),
        "lbm_diagnostics": (c_int32, [c_void_p, P(LbmDiag)]),
        "lbm_diagnostics_noalloc": (c_int32, [c_void_p, P(LbmDiag)]),
        "lbm_checkpoint_bytes": (c_int32, [c_void_p, P(c_size_t)]),
        "lbm_save": (c_int32, [c_void_p, c_void_p, c_int32]),
        "lbm_load": (c_int32, [c_void_p, c_void_p, c_int32]),
        "lbm_counters": (c_int32, [c_void_p, P(c_int64), P(c_int64)]),
        "lbm_vjp_workspace_bytes": (c_int32, [P(LbmConfig), P(c_size_t)]),
        "lbm_vjp_step": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
        "lbm_vjp_init": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
        "lbm_adjoint_workspace_bytes": (c_int32, [P(LbmConfig), c_int64, c_int32, P(c_size_t)]),
        "lbm_adjoint": (c_int32, [c_void_p, P(LbmObjective), c_int64, c_int32, c_void_p, c_size_t,
                                  P(c_double), c_void_p]),
        "lbm_adjoint_revolve_workspace_bytes": (c_int32, [P(LbmConfig), c_int32, P(c_size_t)]),
        "lbm_adjoint_revolve": (c_int32, [c_void_p, P(LbmObjective), c_int64, c_int32, c_void_p, c_size_t,
                                          P(c_double), c_void_p, P(c_int64)]),
        "lbm_witness": (c_int32, [c_void_p, P(LbmObjective), P(c_double)]),
        "lbm_bubble_length": (c_int32, [c_void_p, c_int32, c_double, c_double, c_double, P(c_int64),
                                        P(c_double)]),
        "lbm_set_bunch": (c_int32, [c_void_p, c_int64, c_void_p, c_int32]),
        "lbm_get_bunch": (c_int32, [c_void_p, c_void_p, c_int64, P(c_int64)]),
        "lbm_destroy": (c_int32, [c_void_p]),
        "lbm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, lbm_last_error())


def make_config(cfg: dict) -> LbmConfig:
    """C configuration struct from a workload dictionary (extra keys are ignored)."""
    c = LbmConfig()
    for name, ctype in LbmConfig._fields_:
        v = cfg[name]
        if name == "storage" and isinstance(v, str):
            v = _STORAGE[v]
        setattr(c, name, int(v) if ctype in (c_int32, c_int64) else float(v))
    return c


# --- one-to-one wrappers of the C entry points ----------------------------------------------

def lbm_last_error() -> str:
    return load_library().lbm_last_error().decode()


def lbm_workspace_bytes(cfg: dict | LbmConfig) -> int:
    c = cfg if isinstance(cfg, LbmConfig) else make_config(cfg)
    n = c_size_t(0)
    _check(load_library().lbm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)))
    return n.value


def lbm_init(cfg: dict | LbmConfig, n_pert, p_init, workspace_ptr: int, ws_bytes: int,
             stream_handle: int) -> int:
    c = cfg if isinstance(cfg, LbmConfig) else make_config(cfg)
    npert = None if n_pert is None else np.ascontiguousarray(n_pert, dtype=np.float64)
    pinit = None if p_init is None else np.ascontiguousarray(p_init, dtype=np.float64)
    if npert is not None and npert.shape != (c.nr, c.nz):
        raise ValueError(f"n_pert must have shape {(c.nr, c.nz)}")
    if pinit is not None and pinit.shape != (2, c.nr, c.nz):
        raise ValueError(f"p_init must have shape {(2, c.nr, c.nz)}")
    ctx = c_void_p(0)
    _check(load_library().lbm_init(
        ctypes.byref(c),
        None if npert is None else npert.ctypes.data_as(c_void_p),
        None if pinit is None else pinit.ctypes.data_as(c_void_p),
        c_void_p(workspace_ptr), c_size_t(ws_bytes), c_void_p(stream_handle), ctypes.byref(ctx)))
    return ctx.value


def lbm_step(ctx: int, nsteps: int):
    _check(load_library().lbm_step(c_void_p(ctx), c_int64(nsteps)))


def lbm_moments(ctx: int, dst_ptr: int, dtype: int, on_device: bool):
    _check(load_library().lbm_moments(c_void_p(ctx), c_void_p(dst_ptr), dtype, int(on_device)))


def lbm_fields(ctx: int, dst_ptr: int, dtype: int, on_device: bool):
    _check(load_library().lbm_fields(c_void_p(ctx), c_void_p(dst_ptr), dtype, int(on_device)))


def lbm_get_state(ctx: int, nz: int, nr: int):
    out = np.empty((33, nr, nz), dtype=np.float64)
    k, s = c_int64(0), c_int64(0)
    _check(load_library().lbm_get_state(c_void_p(ctx), out.ctypes.data_as(c_void_p), ctypes.byref(k),
                                        ctypes.byref(s)))
    return out, k.value, s.value


def lbm_set_state(ctx: int, state, step: int, shifts: int):
    src = np.ascontiguousarray(state, dtype=np.float64)
    _check(load_library().lbm_set_state(c_void_p(ctx), src.ctypes.data_as(c_void_p), c_int64(step),
                                        c_int64(shifts)))


def lbm_diagnostics(ctx: int) -> dict:
    d = LbmDiag()
    _check(load_library().lbm_diagnostics(c_void_p(ctx), ctypes.byref(d)))
    return {name: getattr(d, name) for name, _ in LbmDiag._fields_ if name != "reserved"}


def lbm_diagnostics_noalloc(ctx: int) -> dict:
    d = LbmDiag()
    _check(load_library().lbm_diagnostics_noalloc(c_void_p(ctx), ctypes.byref(d)))
    return {name: getattr(d, name) for name, _ in LbmDiag._fields_ if name != "reserved"}


def lbm_checkpoint_bytes(ctx: int) -> int:
    n = c_size_t(0)
    _check(load_library().lbm_checkpoint_bytes(c_void_p(ctx), ctypes.byref(n)))
    return n.value


def lbm_save(ctx: int, dst_ptr: int, on_device: bool):
    _check(load_library().lbm_save(c_void_p(ctx), c_void_p(dst_ptr), int(on_device)))


def lbm_load(ctx: int, src_ptr: int, on_device: bool):
    _check(load_library().lbm_load(c_void_p(ctx), c_void_p(src_ptr), int(on_device)))


def lbm_vjp_workspace_bytes(cfg: dict | LbmConfig) -> int:
    c = cfg if isinstance(cfg, LbmConfig) else make_config(cfg)
    n = c_size_t(0)
    _check(load_library().lbm_vjp_workspace_bytes(ctypes.byref(c), ctypes.byref(n)))
    return n.value


def lbm_vjp_step(ctx: int, ws_ptr: int, ws_bytes: int, lam_next, nz: int, nr: int):
    src = np.ascontiguousarray(lam_next, dtype=np.float64)
    if src.shape != (33, nr, nz):
        raise ValueError(f"lam_next must have shape {(33, nr, nz)}")
    out = np.empty((33, nr, nz), dtype=np.float64)
    grad = np.zeros(4, dtype=np.float64)
    _check(load_library().lbm_vjp_step(c_void_p(ctx), c_void_p(ws_ptr), c_size_t(ws_bytes),
                                       src.ctypes.data_as(c_void_p), out.ctypes.data_as(c_void_p),
                                       grad.ctypes.data_as(c_void_p)))
    return out, grad


def lbm_vjp_init(ctx: int, ws_ptr: int, ws_bytes: int, lam0, nz: int, nr: int):
    src = np.ascontiguousarray(lam0, dtype=np.float64)
    if src.shape != (33, nr, nz):
        raise ValueError(f"lam0 must have shape {(33, nr, nz)}")
    grad = np.zeros(4, dtype=np.float64)
    _check(load_library().lbm_vjp_init(c_void_p(ctx), c_void_p(ws_ptr), c_size_t(ws_bytes),
                                       src.ctypes.data_as(c_void_p), grad.ctypes.data_as(c_void_p)))
    return grad


def lbm_adjoint_workspace_bytes(cfg: dict | LbmConfig, nsteps: int, ckpt_every: int) -> int:
    c = cfg if isinstance(cfg, LbmConfig) else make_config(cfg)
    n = c_size_t(0)
    _check(load_library().lbm_adjoint_workspace_bytes(ctypes.byref(c), c_int64(nsteps), c_int32(ckpt_every),
                                                      ctypes.byref(n)))
    return n.value


def lbm_adjoint(ctx: int, z_behind: float, row: int, nsteps: int, ckpt_every: int, ws_ptr: int,
                ws_bytes: int):
    obj = LbmObjective(float(z_behind), int(row))
    J = c_double(0.0)
    grad = np.zeros(4, dtype=np.float64)
    _check(load_library().lbm_adjoint(c_void_p(ctx), ctypes.byref(obj), c_int64(nsteps), c_int32(ckpt_every),
                                      c_void_p(ws_ptr), c_size_t(ws_bytes), ctypes.byref(J),
                                      grad.ctypes.data_as(c_void_p)))
    return J.value, grad


def lbm_witness(ctx: int, z_behind: float, row: int) -> float:
    obj = LbmObjective(float(z_behind), int(row))
    J = c_double(0.0)
    _check(load_library().lbm_witness(c_void_p(ctx), ctypes.byref(obj), ctypes.byref(J)))
    return J.value


def lbm_adjoint_revolve_workspace_bytes(cfg: dict | LbmConfig, snapshots: int) -> int:
    c = cfg if isinstance(cfg, LbmConfig) else make_config(cfg)
    n = c_size_t(0)
    _check(load_library().lbm_adjoint_revolve_workspace_bytes(ctypes.byref(c), c_int32(snapshots), ctypes.byref(n)))
    return n.value


def lbm_adjoint_revolve(ctx: int, z_behind: float, row: int, nsteps: int, snapshots: int, ws_ptr: int,
                        ws_bytes: int):
    """(J, grad, forward steps taken) with binomial checkpointing under a snapshot budget."""
    obj = LbmObjective(float(z_behind), int(row))
    J = c_double(0.0)
    adv = c_int64(0)
    grad = np.zeros(4, dtype=np.float64)
    _check(load_library().lbm_adjoint_revolve(c_void_p(ctx), ctypes.byref(obj), c_int64(nsteps),
                                              c_int32(snapshots), c_void_p(ws_ptr), c_size_t(ws_bytes),
                                              ctypes.byref(J), grad.ctypes.data_as(c_void_p), ctypes.byref(adv)))
    return J.value, grad, adv.value


def lbm_bubble_length(ctx: int, row: int = 0, n_star: float = 0.95, z_from: float = -math.inf,
                      z_to: float = math.inf):
    """(count, length) of the sites of a row below n_star times the background density."""
    n = c_int64(0)
    length = c_double(0.0)
    _check(load_library().lbm_bubble_length(c_void_p(ctx), c_int32(row), c_double(n_star), c_double(z_from),
                                            c_double(z_to), ctypes.byref(n), ctypes.byref(length)))
    return n.value, length.value


def lbm_set_bunch(ctx: int, bunch, init_fields: bool = True):
    """Upload a [7][n] macroparticle bunch (x, y, z, p_x, p_y, p_z, w); init_fields also sets the
    initial field from it (step 0 only)."""
    b = np.ascontiguousarray(np.asarray(bunch, dtype=np.float64))
    if b.ndim != 2 or b.shape[0] != 7:
        raise ValueError("bunch must have shape [7][n]")
    _check(load_library().lbm_set_bunch(c_void_p(ctx), c_int64(b.shape[1]), b.ctypes.data_as(c_void_p),
                                        c_int32(1 if init_fields else 0)))


def lbm_get_bunch(ctx: int, n_max: int):
    """The current bunch as a [7][n] float64 array (lost particles have w = 0)."""
    out = np.zeros(7 * max(n_max, 1))
    n = c_int64(0)
    _check(load_library().lbm_get_bunch(c_void_p(ctx), out.ctypes.data_as(c_void_p), c_int64(n_max), ctypes.byref(n)))
    return out[:7 * n.value].reshape(7, n.value)


def lbm_counters(ctx: int):
    k, s = c_int64(0), c_int64(0)
    _check(load_library().lbm_counters(c_void_p(ctx), ctypes.byref(k), ctypes.byref(s)))
    return k.value, s.value


def lbm_destroy(ctx: int):
    _check(load_library().lbm_destroy(c_void_p(ctx)))


# --- convenience owner ------------------------------------------------------------------------

class Lattice:
    """A context plus its device workspace (a torch uint8 tensor) on one GPU and stream."""

    def __init__(self, cfg: dict, n_pert=None, p_init=None, device="cuda", stream=None):
        import torch
        load_library()
        self.cfg = dict(cfg)
        self.nz, self.nr = int(cfg["nz"]), int(cfg["nr"])
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws_bytes = lbm_workspace_bytes(cfg)
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ctx = lbm_init(cfg, n_pert, p_init, self.ws_ptr, self.ws_bytes, self.stream.cuda_stream)

    def step(self, nsteps: int = 1):
        lbm_step(self.ctx, nsteps)

    def _out3(self, fn, dtype):
        import torch
        dt = torch.float64 if dtype == torch.float64 else torch.float32
        out = torch.empty((3, self.nr, self.nz), dtype=dt, device=self.device)
        fn(self.ctx, out.data_ptr(), LBM_F64 if dt == torch.float64 else LBM_F32, True)
        return out

    def moments(self, dtype=None):
        """[3][nr][nz] device tensor: n, J_z, J_r (stream-ordered)."""
        import torch
        return self._out3(lbm_moments, dtype or torch.float64)

    def fields(self, dtype=None):
        """[3][nr][nz] device tensor: E_z, E_r, B_theta (stream-ordered)."""
        import torch
        return self._out3(lbm_fields, dtype or torch.float64)

    def state(self):
        """(state [33][nr][nz] float64 numpy, step, shifts); synchronising."""
        return lbm_get_state(self.ctx, self.nz, self.nr)

    def set_state(self, state, step: int, shifts: int):
        lbm_set_state(self.ctx, state, step, shifts)

    def save(self, on_device: bool = False):
        """Native-format checkpoint: a uint8 numpy array (host) or torch tensor (device); with the
        particle driver it holds the bunch as well."""
        import torch
        n = lbm_checkpoint_bytes(self.ctx)
        if on_device:
            buf = torch.empty(n, dtype=torch.uint8, device=self.device)
            lbm_save(self.ctx, buf.data_ptr(), True)
        else:
            buf = np.empty(n, dtype=np.uint8)
            lbm_save(self.ctx, buf.ctypes.data, False)
        return buf

    def load(self, buf):
        if isinstance(buf, np.ndarray):
            lbm_load(self.ctx, buf.ctypes.data, False)
        else:
            lbm_load(self.ctx, buf.data_ptr(), True)

    def diagnostics(self) -> dict:
        return lbm_diagnostics(self.ctx)

    def _scratch(self, nbytes: int):
        import torch
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        return buf, (buf.data_ptr() + 255) // 256 * 256

    def vjp_step(self, lam_next):
        """(lambda^k, theta partials) of the step from the current state, for lambda^{k+1}."""
        nbytes = lbm_vjp_workspace_bytes(self.cfg)
        buf, ptr = self._scratch(nbytes)
        return lbm_vjp_step(self.ctx, ptr, nbytes, lam_next, self.nz, self.nr)

    def vjp_init(self, lam0):
        """theta partials of the initial state for lambda^0 (the context must be at step 0)."""
        nbytes = lbm_vjp_workspace_bytes(self.cfg)
        buf, ptr = self._scratch(nbytes)
        return lbm_vjp_init(self.ctx, ptr, nbytes, lam0, self.nz, self.nr)

    def adjoint(self, nsteps: int, ckpt_every: int | None = None, z_behind: float = 4.0, row: int = 0):
        """(J, dJ/d(ramp_len, n0, sigma_r, nb)) of the witness field after nsteps steps from the
        initial state; checkpoints every ckpt_every steps (default: about sqrt(nsteps))."""
        if ckpt_every is None:
            ckpt_every = max(1, int(round(nsteps ** 0.5)))
        nbytes = lbm_adjoint_workspace_bytes(self.cfg, nsteps, ckpt_every)
        buf, ptr = self._scratch(nbytes)
        return lbm_adjoint(self.ctx, z_behind, row, nsteps, ckpt_every, ptr, nbytes)

    def adjoint_revolve(self, nsteps: int, snapshots: int, z_behind: float = 4.0, row: int = 0):
        """(J, dJ/d(ramp_len, n0, sigma_r, nb), forward steps taken) with binomial checkpointing
        under a budget of `snapshots` stored states; the lattice is back at its initial state after."""
        nbytes = lbm_adjoint_revolve_workspace_bytes(self.cfg, snapshots)
        buf, ptr = self._scratch(nbytes)
        return lbm_adjoint_revolve(self.ctx, z_behind, row, nsteps, snapshots, ptr, nbytes)

    def witness(self, z_behind: float = 4.0, row: int = 0) -> float:
        """The adjoint's objective J for the current state (no gradient)."""
        return lbm_witness(self.ctx, z_behind, row)

    def bubble_length(self, row: int = 0, n_star: float = 0.95, z_from: float = -math.inf,
                      z_to: float = math.inf):
        return lbm_bubble_length(self.ctx, row, n_star, z_from, z_to)

    def set_bunch(self, bunch, init_fields: bool = True):
        lbm_set_bunch(self.ctx, bunch, init_fields)

    def bunch(self):
        return lbm_get_bunch(self.ctx, int(self.cfg.get("max_particles", 0)))

    def counters(self):
        return lbm_counters(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
