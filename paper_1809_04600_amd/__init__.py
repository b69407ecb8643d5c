"""Screened Epstein-Nesbet PT2 (fast SHCI perturbative step) on AMD MI355X.

The computation lives in libshci_pt2.so (HIP kernels for gfx950, C ABI in
include/shci_pt2.h); this package is its thin Python binding.
"""
from .binding import (SHCI_FP32C, SHCI_FP64, Context, ShciError, dets_numpy, dets_tensor,  # noqa: F401
                      lib)
from .autograd import (PT2Function, SemistochasticPT2Function, pt2_energy,  # noqa: F401
                       pt2_semistochastic_energy)
