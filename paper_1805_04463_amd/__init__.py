"""MI355X (gfx950) causal-set interval abundances and Benincasa-Dowker action.

The compute path is libcausal.so (HIP kernels behind the C ABI in include/causal.h);
``binding`` marshals torch device tensors into it.  Importing this package does not
load the library; the first call does, and fails loudly if it is not built.
"""
from .binding import (CS_COUNT_BITSET, CS_COUNT_BITSET_DENSE, CS_COUNT_MFMA, CS_COUNT_MFMA_FP4, CS_DS2_SLAB, CS_MINK3_DIAMOND, CS_DS4_SLAB, CS_MINK2_DIAMOND,  # noqa: F401
                      CS_MINK4_DIAMOND, REGION_DIM, SYMBOLS, BatchGraph, BatchPlan, CausalError,
                      cs_action, cs_autotune, cs_causal_matrix, cs_dalembertian, cs_coord_planes, cs_degrees,
                      cs_interval_histogram, cs_interval_histogram_noalloc, cs_longest_chain,
                      cs_ld_words, cs_measure_mfma_peak, cs_sprinkle, lib)
