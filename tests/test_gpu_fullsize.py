"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

3+1 diamond N = 16384: the whole path from the seed, bit-exact against the oracle
(coordinates, matrix, N_n from the oracle's optimised tier) and actions to 1e-12.
de Sitter slab N = 65536: the matrix from the oracle's coordinates, bit-exact against
the oracle's full matrix; N_n of every counter bin by bin against the oracle's optimised
tier, computed in the test.
3+1 diamond N = 131072 (the benchmark's workload): coordinates and the whole matrix
bit-exact against the oracle's; N_n of every counter bin by bin against the abundances
the oracle stored in tests/golden (tests/golden/make_fullsize.py).
Inputs flow from the oracle to the GPU, never back: no device result enters an oracle call.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_04463_amd as cs
    cs.lib()
    return cs


def host_u64(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def load_golden(name: str):
    """(meta, N_n) stored by tests/golden/make_fullsize.py from the oracle alone."""
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "make_fullsize.py")
    spec = importlib.util.spec_from_file_location("make_fullsize", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load(name)


def degree_moments(bits: np.ndarray, n: int):
    """(relations, sum_i indeg(i) * outdeg(i)) of a symmetric packed matrix, in chunks."""
    rel = 0
    c3 = 0
    for r0 in range(0, n, 4096):
        blk = bits[r0:min(n, r0 + 4096)]
        rows = np.arange(r0, r0 + blk.shape[0])
        pc = np.bitwise_count(blk).astype(np.int32)
        cum = np.cumsum(pc, axis=1, dtype=np.int64)
        wi, b = rows >> 6, rows & 63
        before = np.where(wi > 0, cum[np.arange(len(rows)), np.maximum(wi - 1, 0)], 0)
        word = blk[np.arange(len(rows)), wi]
        low = np.bitwise_count(word & ((np.uint64(1) << b.astype(np.uint64)) - np.uint64(1)))
        indeg = before + low.astype(np.int64)
        outdeg = cum[:, -1] - indeg
        rel += int(outdeg.sum())
        c3 += int((indeg * outdeg).sum())
    return rel, c3


def test_mink4_n16384_whole_path(cs, orc):
    cfg = W.WORKLOADS["mink4_n16384"]
    n, seed = cfg["n"], cfg["seed"]
    coords, bits, hist, acts = orc.pipeline(W.MINK4_DIAMOND, n, seed, eps_list=cfg["eps"],
                                            fast=True)
    c = cs.cs_sprinkle(W.MINK4_DIAMOND, n, seed)
    assert np.array_equal(c.cpu().numpy(), coords)
    b = cs.cs_causal_matrix(W.MINK4_DIAMOND, c)
    assert np.array_equal(host_u64(b), bits)
    for counter in (cs.CS_COUNT_MFMA, cs.CS_COUNT_BITSET, cs.CS_COUNT_MFMA_FP4):
        h = cs.cs_interval_histogram(b, n, counter)
        assert np.array_equal(host_u64(h), hist)
        for eps, want in acts.items():
            got = cs.cs_action(h, n, 4, eps).item()
            assert abs(got - want) <= 1e-12 * abs(want)


def test_ds4_n65536(cs, orc):
    """The matrix from the oracle's coordinates against the oracle's matrix; N_n of every
    counter bin by bin against the oracle's optimised tier over that matrix (computed
    here: the slab's sprinkle uses libm, so no stored value is machine-independent)."""
    cfg = W.WORKLOADS["ds4_n65536"]
    n, seed = cfg["n"], cfg["seed"]
    coords = orc.sprinkle(W.DS4_SLAB, n, seed, eta0=W.DS_ETA0)
    want = orc.causal_matrix(W.DS4_SLAB, coords)
    b = cs.cs_causal_matrix(W.DS4_SLAB, torch.from_numpy(coords).cuda())
    assert np.array_equal(host_u64(b), want)
    hist, pairs = orc.histogram_fast(want, n)
    del want
    assert pairs == int(hist.sum())
    for counter in (cs.CS_COUNT_MFMA, cs.CS_COUNT_BITSET, cs.CS_COUNT_MFMA_FP4):
        h = cs.cs_interval_histogram(b, n, counter)
        assert np.array_equal(host_u64(h), hist), counter
    for eps in (0.0, 0.1):
        want_s, _ = orc.action(hist, n, 4, eps)
        got = cs.cs_action(h, n, 4, eps).item()
        assert abs(got - want_s) <= 1e-12 * abs(want_s), (eps, got, want_s)
    # the GPU sprinkle from the same seed agrees to a few ulps
    g = cs.cs_sprinkle(W.DS4_SLAB, n, seed, eta0=W.DS_ETA0).cpu().numpy()
    assert np.allclose(g, coords, rtol=4e-15, atol=4e-16)


def fullsize_parity(cs, orc, name: str, counters):
    """A Minkowski workload at N = 131072 from the seed: coordinates and the whole matrix
    bit-exact against the oracle's; N_n of every counter bin by bin against the stored
    oracle abundances; actions against the oracle's actions of those abundances."""
    cfg = W.WORKLOADS[name]
    region, n, seed = cfg["region"], cfg["n"], cfg["seed"]
    dim = W.REGION_DIM[region]
    meta, hist = load_golden(name)
    assert int(meta["n"]) == n and int(meta["seed"]) == seed
    coords = orc.sprinkle(region, n, seed)
    c = cs.cs_sprinkle(region, n, seed)
    assert np.array_equal(c.cpu().numpy(), coords)
    b = cs.cs_causal_matrix(region, c)
    got = host_u64(b)
    want = orc.causal_matrix(region, coords)
    assert np.array_equal(got, want)
    del got, want
    for counter in counters:
        print(f"{name}: counter {counter}", flush=True)
        h = cs.cs_interval_histogram(b, n, counter)
        assert np.array_equal(host_u64(h), hist), counter
    assert int(hist.sum()) == int(meta["relations"])
    for eps in tuple(cfg["eps"]) + (0.0,):
        want_s, _ = orc.action(hist, n, dim, eps)
        got_s = cs.cs_action(h, n, dim, eps).item()
        assert abs(got_s - want_s) <= 1e-12 * max(abs(want_s), 1.0), (eps, got_s, want_s)
    return meta


def test_mink4_n131072(cs, orc):
    meta = fullsize_parity(cs, orc, "mink4_n131072",
                           (cs.CS_COUNT_MFMA, cs.CS_COUNT_BITSET, cs.CS_COUNT_MFMA_FP4))
    n = int(meta["n"])
    # ordering fraction of the 3+1 diamond is 1/10 (sd of R/(N(N-1)/2) at this N is ~1e-3)
    assert abs(int(meta["relations"]) / (n * (n - 1) / 2) - 0.1) < 0.01
