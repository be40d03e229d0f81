"""The stored oracle abundances of the full-size Minkowski workloads (tests/golden,
written by tests/golden/make_fullsize.py from the oracle alone), held to the oracle.

Every bin is covered by the file's sha256 of the n-1 bins; the zeroth and first moments,
sum N_n = R (relations) and sum n N_n = sum_k indeg(k) outdeg(k) (3-chains i ≺ k ≺ j), are
recomputed here from the oracle's own sprinkle and causal matrix in O(N^2 / 64) word
operations, so a stale or damaged file, or an oracle whose sprinkle or relation changed,
fails here without the minutes of the full count."""
import importlib.util
import os

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
NAMES = ("mink4_n131072", "mink3_n131072")


def load(name):
    spec = importlib.util.spec_from_file_location(
        "make_fullsize", os.path.join(HERE, "golden", "make_fullsize.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load(name)


@pytest.mark.parametrize("name", NAMES)
def test_golden_self_consistent(name):
    meta, hist = load(name)            # checks the bin count and the sha256 of every bin
    cfg = W.WORKLOADS[name]
    n = int(meta["n"])
    assert n == cfg["n"] and int(meta["seed"]) == cfg["seed"] and len(hist) == n - 1
    assert int(hist.sum()) == int(meta["relations"])
    assert int((np.arange(n - 1, dtype=np.uint64) * hist).sum()) == int(meta["chains3"])
    assert hist[0] > 0 and hist[-1] == 0  # links exist; no pair has every element inside


@pytest.mark.slow
@pytest.mark.parametrize("name", NAMES)
def test_golden_matches_oracle_matrix(orc, name):
    meta, _ = load(name)
    cfg = W.WORKLOADS[name]
    coords = orc.sprinkle(cfg["region"], cfg["n"], cfg["seed"])
    bits = orc.causal_matrix(cfg["region"], coords)
    _, _, chains3, rel = orc.degrees(bits, cfg["n"])
    assert rel == int(meta["relations"])
    assert chains3 == int(meta["chains3"])
