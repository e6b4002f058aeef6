"""MI355X (gfx950) phase-field lattice Boltzmann hot path.

The two-distribution incompressible phase-field LB model of Li, Luo & Gao
(arXiv:1110.5004), with the switch that keeps or removes the additional
interfacial force F_a, as hand-written HIP kernels behind the C ABI of
include/lbm.h.  This package only marshals arguments (binding.py) and builds
the library (build.py).
"""
from .binding import (BF16, D2Q9, D3Q19, FORM_FUSED, FORM_THREE, FORM_TWO, FP16, FP32, PERIODIC,
                      WALL, LbmError, Simulation,
                      beta_kappa, beta_kappa_sym, copy_bw, declared_functions, encode16,
                      encode16_stochastic,
                      field_diagnostics, field_diagnostics_noalloc, lib, pull_copy_bw,
                      pull_copy_bytes, stream_words, variants)

__all__ = ["Simulation", "LbmError", "beta_kappa", "beta_kappa_sym", "lib", "stream_words", "encode16", "encode16_stochastic",
           "copy_bw", "field_diagnostics", "field_diagnostics_noalloc", "pull_copy_bw", "pull_copy_bytes", "variants", "declared_functions",
           "D2Q9", "D3Q19", "PERIODIC", "WALL", "FP32", "FP16", "BF16",
           "FORM_THREE", "FORM_FUSED", "FORM_TWO"]
