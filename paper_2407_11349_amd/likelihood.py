"""Python face of libhawkes: device event sets, workspaces, and the calls.

All arithmetic happens in the HIP library; PyTorch supplies device memory and
the current stream.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib


def _dev_f64(a, device) -> torch.Tensor:
    t = torch.as_tensor(a, dtype=torch.float64)
    return t.to(device).contiguous()


@dataclass
class DeviceEvents:
    """An event set resident in HBM (FP64 SoA: t, x, y, s).  area = 0: Gaussian spatial
    background; area > 0: the paper's spatially uniform background 1/area (km^2)."""

    t: torch.Tensor
    x: torch.Tensor
    y: torch.Tensor
    s: torch.Tensor
    area: float = 0.0

    @classmethod
    def from_arrays(cls, t, x, y, s, device="cuda", area: float = 0.0) -> "DeviceEvents":
        return cls(_dev_f64(t, device), _dev_f64(x, device), _dev_f64(y, device), _dev_f64(s, device), float(area))

    @property
    def n(self) -> int:
        return int(self.t.shape[0])

    def struct(self) -> _lib.Events:
        for a in (self.t, self.x, self.y, self.s):
            if a.dtype != torch.float64 or not a.is_cuda or not a.is_contiguous() or a.shape[0] != self.n:
                raise ValueError("event arrays must be contiguous float64 CUDA tensors of equal length")
        return _lib.Events(self.n, _lib.ptr(self.t), _lib.ptr(self.x), _lib.ptr(self.y), _lib.ptr(self.s),
                           float(self.area))


def workspace_bytes(n: int, precision="fp32") -> int:
    return int(_lib.load().hawkes_workspace_bytes(int(n), _lib.precision_code(precision)))


def workspace_min_bytes(n: int, precision="fp32") -> int:
    return int(_lib.load().hawkes_workspace_min_bytes(int(n), _lib.precision_code(precision)))


class Workspace:
    """Caller-owned device scratch for the likelihood calls (allocated once)."""

    def __init__(self, n: int, precision="fp32", device="cuda", nbytes: int | None = None):
        """nbytes: the workspace size (default hawkes_workspace_bytes; a larger one gives the sweep's
        passes more room, a smaller one below the minimum is refused by the calls)."""
        need = workspace_bytes(n, precision)
        if need == 0:
            raise ValueError(f"invalid workspace request n={n} precision={precision}")
        nbytes = need if nbytes is None else int(nbytes)
        nbytes = (nbytes + 255) // 256 * 256
        self.nbytes = nbytes
        # over-allocate so the base can be aligned to 256 bytes
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._buf.data_ptr()
        self.offset = (-base) % 256
        self.ptr = base + self.offset

    def status(self, stream=None) -> int:
        st = ctypes.c_int(0)
        _lib.check(_lib.load().hawkes_workspace_status(self.ptr, ctypes.byref(st), _lib.stream_handle(stream)),
                   "hawkes_workspace_status")
        return int(st.value)


_WS_CACHE: dict = {}


def _workspace(events: DeviceEvents, precision, ws: Workspace | None, stream=None) -> Workspace:
    """The caller's workspace, else one cached per (size, precision, device, stream): calls that share
    a workspace must not overlap, and calls on one stream never do."""
    if ws is not None:
        return ws
    key = (events.n, _lib.precision_code(precision), events.t.device, _lib.stream_handle(stream))
    w = _WS_CACHE.get(key)
    if w is None:
        if len(_WS_CACHE) >= 4:
            _WS_CACHE.clear()
        # allocated on the stream that uses it: torch's caching allocator hands a freed block back only to
        # later allocations on the same stream, which are ordered after this stream's pending calls
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            w = Workspace(events.n, precision, events.t.device)
        _WS_CACHE[key] = w
    return w


def _rows(events: DeviceEvents, rows):
    if rows is None:
        return 0, events.n
    r0, r1 = rows
    return int(r0), int(r1)


# Keyword arguments of every likelihood call, passed to the library as hawkes_options:
#   symmetric_groups  0 = default (384), 1..1024, or -1 = whole-set calls take the row sweep
#   row_workgroups    0 = default (32768), else 1..65536
#   timer             a SweepTimer whose events the call records around its pair sweep


def loglik(events: DeviceEvents, theta, precision="fp32", rows=None, ws=None, out=None, stream=None, *,
           symmetric_groups=0, row_workgroups=0, timer=None) -> torch.Tensor:
    """Log-likelihood of rows [r0, r1) as a 1-element float64 device tensor (asynchronous)."""
    lib = _lib.load()
    w = _workspace(events, precision, ws, stream)
    r0, r1 = _rows(events, rows)
    out = torch.empty(1, dtype=torch.float64, device=events.t.device) if out is None else out
    ev = events.struct()
    th = _lib.theta_struct(theta)
    o = _lib.options(row_workgroups, symmetric_groups, timer)
    _lib.check(lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), _lib.precision_code(precision), r0, r1,
                                 w.ptr, w.nbytes, _lib.ptr(out), _lib.opt_ref(o), _lib.stream_handle(stream)),
               "hawkes_loglik")
    return out


def loglik_grad(events: DeviceEvents, theta, precision="fp32", rows=None, ws=None, out=None, grad=None,
                stream=None, *, symmetric_groups=0, row_workgroups=0, timer=None):
    """(loglik (1,), gradient (6,)) float64 device tensors, gradient w.r.t. natural theta."""
    lib = _lib.load()
    w = _workspace(events, precision, ws, stream)
    r0, r1 = _rows(events, rows)
    dev = events.t.device
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    grad = torch.empty(6, dtype=torch.float64, device=dev) if grad is None else grad
    ev = events.struct()
    th = _lib.theta_struct(theta)
    o = _lib.options(row_workgroups, symmetric_groups, timer)
    _lib.check(lib.hawkes_loglik_grad(ctypes.byref(ev), ctypes.byref(th), _lib.precision_code(precision), r0, r1,
                                      w.ptr, w.nbytes, _lib.ptr(out), _lib.ptr(grad), _lib.opt_ref(o),
                                      _lib.stream_handle(stream)), "hawkes_loglik_grad")
    return out, grad


def loglik_grad_noalloc(events: DeviceEvents, theta, precision="fp32", rows=None, out=None, grad=None, stream=None,
                        *, symmetric_groups=0, row_workgroups=0, timer=None):
    """loglik_grad with the library's own static workspace (hawkes_loglik_grad_noalloc): no device memory
    is allocated for the call when out and grad are given.  Calls on one GPU must not overlap."""
    lib = _lib.load()
    r0, r1 = _rows(events, rows)
    dev = events.t.device
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    grad = torch.empty(6, dtype=torch.float64, device=dev) if grad is None else grad
    ev = events.struct()
    th = _lib.theta_struct(theta)
    o = _lib.options(row_workgroups, symmetric_groups, timer)
    _lib.check(lib.hawkes_loglik_grad_noalloc(ctypes.byref(ev), ctypes.byref(th), _lib.precision_code(precision), r0,
                                              r1, _lib.ptr(out), _lib.ptr(grad), _lib.opt_ref(o),
                                              _lib.stream_handle(stream)), "hawkes_loglik_grad_noalloc")
    return out, grad


def loglik_batch(events: DeviceEvents, thetas, precision="fp32", rows=None, ws=None, out=None,
                 stream=None, *, symmetric_groups=0, row_workgroups=0, timer=None) -> torch.Tensor:
    """Log-likelihoods of rows [r0, r1) at each of K parameter vectors (a (K, 6) array-like) as a
    K-element float64 device tensor (asynchronous); FP32 evaluates them two per pair sweep."""
    lib = _lib.load()
    w = _workspace(events, precision, ws, stream)
    r0, r1 = _rows(events, rows)
    arr = _lib.theta_array(thetas)
    k = len(arr)
    out = torch.empty(k, dtype=torch.float64, device=events.t.device) if out is None else out
    if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() < k:
        raise ValueError("out must be a contiguous float64 CUDA tensor of at least K elements")
    ev = events.struct()
    o = _lib.options(row_workgroups, symmetric_groups, timer)
    _lib.check(lib.hawkes_loglik_batch(ctypes.byref(ev), arr, k, _lib.precision_code(precision), r0, r1, w.ptr,
                                       w.nbytes, _lib.ptr(out), _lib.opt_ref(o), _lib.stream_handle(stream)),
               "hawkes_loglik_batch")
    return out


def event_terms(events: DeviceEvents, theta, precision="fp32", rows=None, ws=None, stream=None, *,
                symmetric_groups=0, row_workgroups=0, timer=None):
    """(lambda_n, Lambda_n) for the rows, float64 device tensors."""
    lib = _lib.load()
    w = _workspace(events, precision, ws, stream)
    r0, r1 = _rows(events, rows)
    dev = events.t.device
    lam = torch.empty(r1 - r0, dtype=torch.float64, device=dev)
    comp = torch.empty(r1 - r0, dtype=torch.float64, device=dev)
    ev = events.struct()
    th = _lib.theta_struct(theta)
    o = _lib.options(row_workgroups, symmetric_groups, timer)
    _lib.check(lib.hawkes_event_terms(ctypes.byref(ev), ctypes.byref(th), _lib.precision_code(precision), r0, r1,
                                      w.ptr, w.nbytes, _lib.ptr(lam), _lib.ptr(comp), _lib.opt_ref(o),
                                      _lib.stream_handle(stream)), "hawkes_event_terms")
    return lam, comp


def resample_locations(county: torch.Tensor, rect: torch.Tensor, seed: int, iteration: int,
                       x_out: torch.Tensor, y_out: torch.Tensor, stream=None) -> None:
    """Uniform within-county redraw of every location into x_out, y_out (device, in place)."""
    lib = _lib.load()
    n = int(county.shape[0])
    for a, dt in ((county, torch.int32), (rect, torch.float64), (x_out, torch.float64), (y_out, torch.float64)):
        if a.dtype != dt or not a.is_cuda or not a.is_contiguous():
            raise ValueError("resample arguments must be contiguous CUDA tensors of the documented dtypes")
    if x_out.shape[0] != n or y_out.shape[0] != n or rect.dim() != 2 or rect.shape[1] != 4:
        raise ValueError("shape mismatch in resample arguments")
    _lib.check(lib.hawkes_resample_locations(n, _lib.ptr(county), _lib.ptr(rect), int(rect.shape[0]),
                                             int(seed) & (2**64 - 1), int(iteration) & (2**64 - 1),
                                             _lib.ptr(x_out), _lib.ptr(y_out), _lib.stream_handle(stream)),
               "hawkes_resample_locations")


SweepTimer = _lib.SweepTimer


class HawkesLoglik(torch.autograd.Function):
    """l(theta) with a hand-written adjoint: forward runs the fused
    forward+adjoint sweep and keeps the gradient; backward scales it."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, events: DeviceEvents, precision="fp32", rows=None, ws=None):
        ll, g = loglik_grad(events, theta, precision=precision, rows=rows, ws=ws)
        ctx.save_for_backward(g)
        ctx.theta_device = theta.device
        return ll.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return (grad_out.to(g.device) * g).to(ctx.theta_device), None, None, None, None


def hawkes_loglik(theta: torch.Tensor, events: DeviceEvents, precision="fp32", rows=None, ws=None) -> torch.Tensor:
    return HawkesLoglik.apply(theta, events, precision, rows, ws)
