"""Samplers over the six log-parameters: HMC, delayed-acceptance HMC with a
surrogate, the paper's univariate Metropolis-Hastings, the cut-posterior driver,
and bulk-ESS / split R-hat."""

from .da_hmc import DAState, DelayedAcceptanceHMC
from .mh import UnivariateMH
from .ess import bulk_ess, ess, mcse_mean, split_rhat
from .hmc import HMC, DualAveraging, HMCState, NonFiniteStateError, accept_prob, leapfrog

__all__ = ["DAState", "DelayedAcceptanceHMC", "bulk_ess", "ess", "mcse_mean", "split_rhat", "HMC", "DualAveraging",
           "HMCState", "NonFiniteStateError", "accept_prob", "leapfrog", "UnivariateMH"]
