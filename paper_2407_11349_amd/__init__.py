"""MI355X-native spatiotemporal Hawkes likelihood (arXiv 2407.11349).

The O(N^2) log-likelihood, its gradient and the cut-posterior location draw
run in hand-written HIP kernels for gfx950 behind the C ABI of
include/hawkes.h (libhawkes.so); this package is the thin Python binding.
"""

from .likelihood import (DeviceEvents, HawkesLoglik, Workspace, event_terms, hawkes_loglik, last_pair_kernel_ms,
                         loglik, loglik_batch, loglik_grad, resample_locations, set_timing, workspace_bytes)

__all__ = [
    "DeviceEvents", "HawkesLoglik", "Workspace", "event_terms", "hawkes_loglik", "last_pair_kernel_ms", "loglik",
    "loglik_batch", "loglik_grad", "resample_locations", "set_timing", "workspace_bytes",
]
