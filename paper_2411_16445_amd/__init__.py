"""MI355X (gfx950) engine for plastic networks of multi-compartment neurons.

The simulation runs in libplasticarbor.so (hand-written HIP kernels behind
the C ABI of include/plasticarbor.h); this package only builds it and binds
it.  See ``binding.Simulation``.
"""
from .binding import (PA_BATCHED, PA_FP64, PA_MIXED, PA_PLAIN, PAError, Simulation,  # noqa: F401
                      load_library)

__all__ = ["Simulation", "PAError", "load_library", "PA_FP64", "PA_MIXED", "PA_PLAIN",
           "PA_BATCHED"]
