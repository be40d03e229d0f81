"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds inputs only -- region codes, sizes, seeds, smearing parameters and
the batch's per-instance (n, seed) draws -- and none of the method's arithmetic:
each side (GPU library, CPU oracle) sprinkles, links, counts and evaluates the
action from these inputs with its own code.

The five workloads follow the sizes and regions the thesis studies (Ch. 4 and
App. A): a 1+1 Minkowski diamond, 3+1 Minkowski diamonds at two sizes, a 3+1
de Sitter slab and an ensemble of 1+1 diamonds of uneven size.  All inputs are
synthetic sprinklings; no dataset is involved.
"""
from __future__ import annotations

import numpy as np

# Region codes, identical to the enumeration of the C ABI and the oracle.
MINK2_DIAMOND = 0
MINK4_DIAMOND = 1
DS4_SLAB = 2
DS2_SLAB = 3
MINK3_DIAMOND = 4
REGION_NAMES = {MINK2_DIAMOND: "mink2_diamond", MINK4_DIAMOND: "mink4_diamond",
                DS4_SLAB: "ds4_slab", DS2_SLAB: "ds2_slab", MINK3_DIAMOND: "mink3_diamond"}
REGION_DIM = {MINK2_DIAMOND: 2, MINK4_DIAMOND: 4, DS4_SLAB: 4, DS2_SLAB: 2, MINK3_DIAMOND: 3}
DS_ETA0 = 1.2
# The 1+1 de Sitter slab of the thesis's action benchmark: eta in [-1/2, 1/2], smearing
# eps = 2^-6, ten seeds per size, N from 2^10 to 2^17.
DS2_ETA0 = 0.5
DS2_EPS = 2.0 ** -6
DS2_SEEDS = tuple(range(100, 110))

WORKLOADS = {
    "mink2_n1024": dict(region=MINK2_DIAMOND, n=1024, seed=1, eps=(0.1,)),
    "mink4_n16384": dict(region=MINK4_DIAMOND, n=16384, seed=2, eps=(0.1,)),
    "ds4_n65536": dict(region=DS4_SLAB, n=65536, seed=3, eps=(0.1,)),
    "batch_mink2_256": dict(region=MINK2_DIAMOND, count=256, nmin=512, nmax=8192, seed=4,
                            eps=(0.1,)),
    "mink4_n131072": dict(region=MINK4_DIAMOND, n=131072, seed=5, eps=(0.05, 0.1, 0.2)),
    "mink3_n16384": dict(region=MINK3_DIAMOND, n=16384, seed=6, eps=(0.05, 0.1, 0.2)),
    "mink3_n131072": dict(region=MINK3_DIAMOND, n=131072, seed=5, eps=(0.05, 0.1, 0.2)),
    "ds2_n131072": dict(region=DS2_SLAB, n=131072, seed=DS2_SEEDS[0], eps=(DS2_EPS,),
                        eta0=DS2_ETA0),
}


def batch_instances(seed: int = 4, count: int = 256, nmin: int = 512, nmax: int = 8192):
    """Per-instance sizes, uniform integers in [nmin, nmax], and per-instance seeds,
    drawn with numpy's PCG64 from ``seed``.  Returns (n: int64[count], seeds: uint64[count])."""
    rng = np.random.default_rng(seed)
    n = rng.integers(nmin, nmax + 1, size=count, dtype=np.int64)
    seeds = rng.integers(0, 2**63 - 1, size=count, dtype=np.int64).astype(np.uint64)
    return n, seeds
