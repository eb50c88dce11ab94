"""MI355X-native selected-basis diagonalisation (SBD) hot path.

The computation lives in the HIP library ``libsbd.so`` (C ABI in
``include/sbd.h``); this package only marshals arguments to it.
"""
from ._native import (FP32, FP64, SBD_NOT_CONVERGED, SBD_OK, Basis, DavidsonOpts,
                      DavidsonReport, Excitations, Hamiltonian, SBDError, davidson, sigma_timed, SIGMA_STAGES, gram, map_vectors,
                      default_opts, last_error, load, sigma, sigma_noalloc, EXPORTED, LIB_PATH, Server,
                      serve_estimate, release_cached_memory, memory_stats, FullBasis,
                      FullHamiltonian, full_sigma, full_davidson, full_map_vectors, sqd_run,
                      occupations, full_occupations, recover_configurations)

__all__ = ["FP32", "FP64", "SBD_OK", "SBD_NOT_CONVERGED", "Basis", "Excitations",
           "Hamiltonian", "SBDError", "sigma", "sigma_noalloc", "sigma_timed", "SIGMA_STAGES", "gram", "map_vectors", "davidson", "default_opts", "DavidsonOpts",
           "DavidsonReport", "last_error", "load", "EXPORTED", "LIB_PATH", "Server", "serve_estimate",
           "release_cached_memory", "memory_stats", "FullBasis", "FullHamiltonian", "full_sigma",
           "full_davidson", "full_map_vectors", "sqd_run", "occupations", "full_occupations",
           "recover_configurations"]
