"""ctypes binding of libhawkes.so: argument marshalling only.

Every step of the likelihood runs in the HIP library; this module converts
torch tensors (device memory, streams) into the plain pointers and sizes of
the C ABI in include/hawkes.h, and raises on a non-zero status.  If the
library has not been built, loading fails loudly; there is no fallback.
"""

from __future__ import annotations

import ctypes
from pathlib import Path

import torch

LIB_PATH = Path(__file__).resolve().parent / "libhawkes.so"

HAWKES_FP64 = 0
HAWKES_FP32 = 1
HAWKES_FP32_SKIP = 2
PRECISIONS = {"fp64": HAWKES_FP64, "fp32": HAWKES_FP32, "fp32_skip": HAWKES_FP32_SKIP,
              HAWKES_FP64: HAWKES_FP64, HAWKES_FP32: HAWKES_FP32, HAWKES_FP32_SKIP: HAWKES_FP32_SKIP}

HAWKES_OK = 0
HAWKES_EORDER = -5
HAWKES_EDATA = -6

# every entry point declared in include/hawkes.h
EXPORTS = (
    "hawkes_workspace_bytes", "hawkes_workspace_min_bytes", "hawkes_loglik", "hawkes_loglik_grad", "hawkes_event_terms",
    "hawkes_loglik_batch", "hawkes_resample_locations", "hawkes_workspace_status", "hawkes_loglik_grad_noalloc",
    "hawkes_strerror", "hawkes_last_error",
    # include/hawkes_mlp.h
    "hawkes_mlp_state_bytes", "hawkes_mlp_workspace_bytes", "hawkes_mlp_load", "hawkes_mlp_store",
    "hawkes_mlp_forward", "hawkes_mlp_leapfrog", "hawkes_mlp_loss_grad", "hawkes_mlp_adam_step",
)
# hawkes_mlp_leapfrog_io: 42 doubles (z, p, grad, inv_mass, m_z, s_z: 6 each; m_y, s_y, prior_var, eps, s, status)
LEAPFROG_IO_DOUBLES = 42
# hawkes_options.symmetric_groups: the library's default and largest accepted counts
SYM_GROUPS_DEFAULT = 384
SYM_GROUPS_MAX = 1024
ROW_WGS_MAX = 65536
MLP_PARAMS = 133633


class Theta(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("mu", "tau_x", "tau_t", "xi", "h0", "omega")]


class Events(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("t", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("s", ctypes.c_void_p), ("area", ctypes.c_double)]


class Options(ctypes.Structure):
    """hawkes_options: per-call tuning and timing (all-zero = defaults)."""

    _fields_ = [("row_workgroups", ctypes.c_int64), ("symmetric_groups", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("timing_start", ctypes.c_void_p), ("timing_stop", ctypes.c_void_p)]


class HawkesError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


_lib = None


def load(path: Path | str | None = None) -> ctypes.CDLL:
    """Load libhawkes.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = Path(path) if path is not None else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is not built; run paper_2407_11349_amd.build.build_library() first")
    lib = ctypes.CDLL(str(p))
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    ev_p, th_p = ctypes.POINTER(Events), ctypes.POINTER(Theta)
    lib.hawkes_workspace_bytes.argtypes = [i64, ctypes.c_int]
    lib.hawkes_workspace_bytes.restype = ctypes.c_size_t
    lib.hawkes_workspace_min_bytes.argtypes = [i64, ctypes.c_int]
    lib.hawkes_workspace_min_bytes.restype = ctypes.c_size_t
    common = [ev_p, th_p, ctypes.c_int, i64, i64, vp, ctypes.c_size_t]
    opt_p = ctypes.POINTER(Options)
    lib.hawkes_loglik.argtypes = common + [vp, opt_p, vp]
    lib.hawkes_loglik_grad.argtypes = common + [vp, vp, opt_p, vp]
    lib.hawkes_event_terms.argtypes = common + [vp, vp, opt_p, vp]
    lib.hawkes_loglik_grad_noalloc.argtypes = [ev_p, th_p, ctypes.c_int, i64, i64, vp, vp, opt_p, vp]
    lib.hawkes_loglik_batch.argtypes = [ev_p, th_p, i64, ctypes.c_int, i64, i64, vp, ctypes.c_size_t, vp, opt_p,
                                        vp]
    lib.hawkes_resample_locations.argtypes = [i64, vp, vp, i32, u64, u64, vp, vp, vp]
    lib.hawkes_workspace_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int), vp]
    lib.hawkes_mlp_state_bytes.argtypes = []
    lib.hawkes_mlp_state_bytes.restype = ctypes.c_size_t
    lib.hawkes_mlp_workspace_bytes.argtypes = [i64]
    lib.hawkes_mlp_workspace_bytes.restype = ctypes.c_size_t
    lib.hawkes_mlp_load.argtypes = [vp, vp, vp]
    lib.hawkes_mlp_store.argtypes = [vp, vp, vp]
    lib.hawkes_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.hawkes_mlp_leapfrog.argtypes = [vp, vp, i64, vp]
    lib.hawkes_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, vp, ctypes.c_size_t, vp, vp, vp]
    lib.hawkes_mlp_adam_step.argtypes = [vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         vp]
    lib.hawkes_strerror.argtypes = [ctypes.c_int]
    lib.hawkes_strerror.restype = ctypes.c_char_p
    lib.hawkes_last_error.argtypes = []
    lib.hawkes_last_error.restype = ctypes.c_char_p
    for name in ("hawkes_loglik", "hawkes_loglik_grad", "hawkes_event_terms", "hawkes_loglik_batch",
                 "hawkes_loglik_grad_noalloc",
                 "hawkes_resample_locations",
                 "hawkes_workspace_status", "hawkes_mlp_load",
                 "hawkes_mlp_store", "hawkes_mlp_forward", "hawkes_mlp_leapfrog", "hawkes_mlp_loss_grad",
                 "hawkes_mlp_adam_step"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != HAWKES_OK:
        lib = load()
        raise HawkesError(status, where, lib.hawkes_last_error().decode() or lib.hawkes_strerror(status).decode())


def precision_code(precision) -> int:
    try:
        return PRECISIONS[precision]
    except KeyError:
        raise ValueError(f"unknown precision {precision!r}") from None


def stream_handle(stream: torch.cuda.Stream | None = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def theta_struct(theta) -> Theta:
    if isinstance(theta, torch.Tensor):
        vals = theta.detach().to("cpu", torch.float64).tolist()
    else:
        vals = [float(v) for v in theta]
    if len(vals) != 6:
        raise ValueError("theta must have 6 components (mu, tau_x, tau_t, xi, h0, omega)")
    return Theta(*vals)


def theta_array(thetas):
    """A ctypes array of Theta structs from a (K, 6) array-like of parameter vectors."""
    rows = thetas.detach().to("cpu", torch.float64).tolist() if isinstance(thetas, torch.Tensor) else list(thetas)
    if len(rows) < 1:
        raise ValueError("need at least one parameter vector")
    arr = (Theta * len(rows))()
    for k, row in enumerate(rows):
        arr[k] = theta_struct(row)
    return arr


def ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else int(t.data_ptr())


def options(row_workgroups: int = 0, symmetric_groups: int = 0, timer=None):
    """A hawkes_options struct for a call (None when every field keeps its default)."""
    if not row_workgroups and not symmetric_groups and timer is None:
        return None
    o = Options(int(row_workgroups), int(symmetric_groups), 0, None, None)
    if timer is not None:
        o.timing_start, o.timing_stop = timer.handles()
    return o


def opt_ref(o):
    return None if o is None else ctypes.byref(o)


_hip = None


def hip_runtime() -> ctypes.CDLL:
    """The HIP runtime the library and torch share (loaded once by soname), for the caller-owned
    timing events of hawkes_options."""
    global _hip
    if _hip is None:
        torch.cuda.init()
        hip = ctypes.CDLL("libamdhip64.so.7")
        vp = ctypes.c_void_p
        hip.hipEventCreate.argtypes = [ctypes.POINTER(vp)]
        hip.hipEventDestroy.argtypes = [vp]
        hip.hipEventSynchronize.argtypes = [vp]
        hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), vp, vp]
        for f in (hip.hipEventCreate, hip.hipEventDestroy, hip.hipEventSynchronize, hip.hipEventElapsedTime):
            f.restype = ctypes.c_int
        _hip = hip
    return _hip


class SweepTimer:
    """Two HIP events that a call records around its pair sweep (hawkes_options.timing_start/stop);
    elapsed_ms() waits for the stop event and returns the sweep's duration on the device."""

    def __init__(self):
        hip = hip_runtime()
        self._start, self._stop = ctypes.c_void_p(), ctypes.c_void_p()
        for e in (self._start, self._stop):
            if hip.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")

    def handles(self):
        return self._start.value, self._stop.value

    def elapsed_ms(self) -> float:
        hip = hip_runtime()
        ms = ctypes.c_float(0.0)
        if hip.hipEventSynchronize(self._stop) != 0 or hip.hipEventElapsedTime(ctypes.byref(ms), self._start,
                                                                                self._stop) != 0:
            raise RuntimeError("timing events were not recorded")
        return float(ms.value)

    def __del__(self):
        if _hip is not None:
            for e in (getattr(self, "_start", None), getattr(self, "_stop", None)):
                if e is not None and e.value:
                    _hip.hipEventDestroy(e)
