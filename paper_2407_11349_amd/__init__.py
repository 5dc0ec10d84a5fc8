"""MI355X-native spatiotemporal Hawkes likelihood (arXiv 2407.11349).

The O(N^2) log-likelihood, its gradient and the cut-posterior location draw
run in hand-written HIP kernels for gfx950 behind the C ABI of
include/hawkes.h (libhawkes.so); this package is the thin Python binding.
"""

from .likelihood import (DeviceEvents, HawkesLoglik, SweepTimer, Workspace, event_terms, hawkes_loglik, loglik,
                         loglik_batch, loglik_grad, resample_locations, workspace_bytes, workspace_min_bytes)

__all__ = [
    "DeviceEvents", "HawkesLoglik", "SweepTimer", "Workspace", "event_terms", "hawkes_loglik", "loglik",
    "loglik_batch", "loglik_grad", "resample_locations", "workspace_bytes", "workspace_min_bytes",
]
