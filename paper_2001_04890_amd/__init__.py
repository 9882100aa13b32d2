"""MI355X-native two-site QC-DMRG H.psi (Brabec et al., Section 2): Python binding of libdmrg.so.

The binding only marshals arguments: every step of H.psi, Davidson and the operator preparation
runs inside the HIP library (``csrc/``). PyTorch supplies device memory and streams. There is no
CPU fallback: importing the package fails loudly when ``libdmrg.so`` is missing.
"""
from .binding import (DMRG_OK, DMRG_NOT_CONVERGED, MLP_IN, MLP_PARAMS, PREC_FP64, PREC_SPLIT2, DmrgError,
                      Hop, Mlp, block_grow, block_grow_layout, lib, lib_path, renormalize_blocks, sweep, truncate,
                      version)

__all__ = ["Hop", "Mlp", "DmrgError", "PREC_FP64", "PREC_SPLIT2", "DMRG_OK", "DMRG_NOT_CONVERGED", "MLP_IN",
           "MLP_PARAMS", "block_grow", "block_grow_layout", "lib", "lib_path", "renormalize_blocks", "sweep", "truncate",
           "version"]
