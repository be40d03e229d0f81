"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

3+1 diamond N = 16384: the whole path from the seed, bit-exact against the oracle
(coordinates, matrix, N_n from the oracle's optimised tier) and actions to 1e-12.
de Sitter slab N = 65536: the matrix from the oracle's coordinates, bit-exact against
the oracle's full matrix; N_n checked by exact invariants against the oracle's
relation count and 3-chain count, and MFMA == bitset.
3+1 diamond N = 131072: coordinates bit-exact; matrix rows sampled against the
oracle's rows; N_n by the invariants sum N_n = R and sum n N_n = sum indeg*outdeg
(both from the matrix, any size) and MFMA == bitset.
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
    cfg = W.WORKLOADS["ds4_n65536"]
    n, seed = cfg["n"], cfg["seed"]
    coords = orc.sprinkle(W.DS4_SLAB, n, seed, eta0=W.DS_ETA0)
    want = orc.causal_matrix(W.DS4_SLAB, coords)
    _, _, chains3, rel = orc.degrees(want, n)
    b = cs.cs_causal_matrix(W.DS4_SLAB, torch.from_numpy(coords).cuda())
    assert np.array_equal(host_u64(b), want)
    del want
    hm = host_u64(cs.cs_interval_histogram(b, n, cs.CS_COUNT_MFMA)).copy()
    hb = host_u64(cs.cs_interval_histogram(b, n, cs.CS_COUNT_BITSET)).copy()
    hf = host_u64(cs.cs_interval_histogram(b, n, cs.CS_COUNT_MFMA_FP4)).copy()
    assert np.array_equal(hm, hb) and np.array_equal(hm, hf)
    assert int(hm.sum()) == rel
    assert int((np.arange(n - 1, dtype=np.uint64) * hm).sum()) == chains3
    h = cs.cs_interval_histogram(b, n, cs.CS_COUNT_MFMA_FP4)
    for eps in (0.0, 0.1):
        want, _ = orc.action(hm, n, 4, eps)
        got = cs.cs_action(h, n, 4, eps).item()
        assert abs(got - want) <= 1e-12 * abs(want), (eps, got, want)
    # the GPU sprinkle from the same seed agrees to a few ulps
    g = cs.cs_sprinkle(W.DS4_SLAB, n, seed, eta0=W.DS_ETA0).cpu().numpy()
    assert np.allclose(g, coords, rtol=4e-15, atol=4e-16)


def test_mink4_n131072(cs, orc):
    cfg = W.WORKLOADS["mink4_n131072"]
    n, seed = cfg["n"], cfg["seed"]
    coords = orc.sprinkle(W.MINK4_DIAMOND, n, seed)
    c = cs.cs_sprinkle(W.MINK4_DIAMOND, n, seed)
    assert np.array_equal(c.cpu().numpy(), coords)
    b = cs.cs_causal_matrix(W.MINK4_DIAMOND, c)
    got = host_u64(b)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.arange(64), rng.integers(0, n, 192), np.arange(n - 64, n)]))
    assert np.array_equal(got[rows], orc.causal_rows(W.MINK4_DIAMOND, coords, rows))
    rel, c3 = degree_moments(got, n)
    del got
    hm = host_u64(cs.cs_interval_histogram(b, n, cs.CS_COUNT_MFMA)).copy()
    hb = host_u64(cs.cs_interval_histogram(b, n, cs.CS_COUNT_BITSET)).copy()
    hf = host_u64(cs.cs_interval_histogram(b, n, cs.CS_COUNT_MFMA_FP4)).copy()
    assert np.array_equal(hm, hb) and np.array_equal(hm, hf)
    assert int(hm.sum()) == rel
    assert int((np.arange(n - 1, dtype=np.uint64) * hm).sum()) == c3
    # ordering fraction of the 3+1 diamond is 1/10 (sd of R/(N(N-1)/2) at this N is ~1e-3)
    assert abs(rel / (n * (n - 1) / 2) - 0.1) < 0.01
    # local and smeared actions from the counted abundances, against the oracle's sums
    h = cs.cs_interval_histogram(b, n, cs.CS_COUNT_MFMA_FP4)
    for eps in cfg["eps"] + (0.0,):
        want, _ = orc.action(hm, n, 4, eps)
        got = cs.cs_action(h, n, 4, eps).item()
        assert abs(got - want) <= 1e-12 * abs(want), (eps, got, want)
