"""MI355X hot path of grid-based BPMF sampling (replica-exchange HMC against
precomputed receptor grids, u_kn, MBAR), after Minh, "Alchemical Grid Dock
(AlGDock)", arXiv 1507.03703.

The compute lives in libbpmf.so (hand-written HIP for gfx950, C ABI declared
in include/bpmf.h).  This module only marshals arguments: numpy arrays for
host inputs, torch CUDA tensors for device buffers, torch's caching allocator
and current stream for device memory and ordering.  There is no fallback:
importing fails if the library has not been built.
"""
from __future__ import annotations

from ._binding import (BPMFError, Context, LIB_PATH, library,  # noqa: F401
                       EXPORTED, SCHEDULE_LINEAR, SCHEDULE_SOFT,
                       detect_equilibration, protocol_adapt_dt,
                       protocol_insert, protocol_mean_pacc,
                       protocol_next_alpha, protocol_next_temperature,
                       protocol_sigmas, protocol_sir, protocol_state)

__all__ = ["BPMFError", "Context", "LIB_PATH", "library", "EXPORTED",
           "SCHEDULE_LINEAR", "SCHEDULE_SOFT", "detect_equilibration",
           "protocol_adapt_dt", "protocol_insert", "protocol_mean_pacc",
           "protocol_next_alpha", "protocol_next_temperature",
           "protocol_sigmas", "protocol_sir", "protocol_state"]
