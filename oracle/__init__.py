"""FP64 CPU oracle for the double-frame differential analysis.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check of the package and
the CPU-baseline leg of the benchmark may import this package. The HIP
library never calls it, links it or falls back to it, and this package
imports nothing from the HIP library.

Every function here is pinned by CPU tests against facts that do not come
from the oracle itself (brute-force DFT, Parseval, closed forms, lattice
counts, statistical recovery of a known synthetic model). No function is
"parity unpinned".
"""
from .dda import (normalise, spectra, pair_power, bin_index, bin_counts,
                  azimuthal_average, structure_function,
                  structure_function_bins)
from .precision import (round_bf16, f16_exponent, round_f16_scaled, stored_spectra,
                        structure_function_stored, structure_function_stored_bins)
from .backward import structure_function_grad

__all__ = ["normalise", "spectra", "pair_power", "bin_index", "bin_counts",
           "azimuthal_average", "structure_function", "structure_function_bins",
           "round_bf16", "f16_exponent", "round_f16_scaled", "stored_spectra",
           "structure_function_stored", "structure_function_stored_bins",
           "structure_function_grad"]
