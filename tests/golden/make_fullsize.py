"""Write the stored interval abundances of the full-size Minkowski workloads.

Calls the oracle only: sprinkle (App. A, rejection into the diamond) -> causal matrix
(strict light cone, Sec. 4.1) -> the oracle's optimised tier of the interval count
(Alg. "Optimized Interval Abundance Measurement", eq. IOIs), which the CPU tests hold
equal to the definitional tier.  The Minkowski sprinkles use exact IEEE operations only
(products, sums, comparisons, no transcendental), so the stored values do not depend on
the machine that ran this script.

Usage:  python tests/golden/make_fullsize.py [workload ...]
        (default: mink4_n131072 mink3_n131072; a few minutes each on 8 cores)

Output: tests/golden/hist_<workload>.txt, a text file with
  - header lines starting with '#': provenance and the oracle source's sha256;
  - 'key value' lines: n, seed, relations (sum N_n), chains3 (sum n N_n),
    nonzero (bins with N_n > 0), hist_sha256 (sha256 of the n-1 bins as little-endian
    uint64, i.e. every bin);
  - then one 'n N_n' line per nonzero bin, in increasing n.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as orc  # noqa: E402
import workloads as W  # noqa: E402

DEFAULT = ("mink4_n131072", "mink3_n131072")


def oracle_sha256() -> str:
    with open(os.path.join(ROOT, "oracle", "causal_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def hist_sha256(hist: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(hist, dtype="<u8").tobytes()).hexdigest()


def make(name: str) -> str:
    cfg = W.WORKLOADS[name]
    region, n, seed = cfg["region"], cfg["n"], cfg["seed"]
    if region not in (W.MINK2_DIAMOND, W.MINK3_DIAMOND, W.MINK4_DIAMOND):
        raise ValueError("only the Minkowski sprinkles are machine-independent")
    t0 = time.time()
    coords = orc.sprinkle(region, n, seed)
    bits = orc.causal_matrix(region, coords)
    _, _, chains3, rel = orc.degrees(bits, n)
    hist, pairs = orc.histogram_fast(bits, n)
    del bits
    assert pairs == rel == int(hist.sum())
    assert chains3 == int((np.arange(n - 1, dtype=np.uint64) * hist).sum())
    nz = np.flatnonzero(hist)
    path = os.path.join(HERE, f"hist_{name}.txt")
    with open(path, "w") as f:
        f.write(f"# Interval abundances N_n (eq. IOIs) of the workload {name}: region "
                f"{W.REGION_NAMES[region]}, N={n}, seed {seed}.\n")
        f.write("# Written by tests/golden/make_fullsize.py from the oracle alone (sprinkle, "
                "causal matrix, optimised tier).\n")
        f.write(f"# oracle_sha256 {oracle_sha256()}\n")
        f.write(f"n {n}\nseed {seed}\nrelations {rel}\nchains3 {chains3}\n")
        f.write(f"nonzero {len(nz)}\nhist_sha256 {hist_sha256(hist)}\n")
        for k in nz:
            f.write(f"{k} {int(hist[k])}\n")
    print(f"{name}: R={rel} nonzero={len(nz)} {time.time() - t0:.1f} s -> {path}", flush=True)
    return path


def load(name: str):
    """(meta dict, hist uint64[n-1]) from tests/golden/hist_<name>.txt."""
    meta, bins = {}, []
    with open(os.path.join(HERE, f"hist_{name}.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            a, b = line.split()
            if a.isdigit():
                bins.append((int(a), int(b)))
            else:
                meta[a] = b
    n = int(meta["n"])
    hist = np.zeros(n - 1, dtype=np.uint64)
    for k, v in bins:
        hist[k] = v
    if len(bins) != int(meta["nonzero"]) or hist_sha256(hist) != meta["hist_sha256"]:
        raise ValueError(f"golden file for {name} is damaged")
    return meta, hist


if __name__ == "__main__":
    for name in sys.argv[1:] or DEFAULT:
        make(name)
