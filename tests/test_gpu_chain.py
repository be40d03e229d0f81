"""GPU parity of the longest chains through Alexandroff sets (Sec. 2.5.2, algorithm
"Maximal Chain Length") and of the degree vectors, against the oracle.

Lengths and heights are integers: bit-exact.  Small cases span several 64-element words
and 256-word scan steps with ragged tails, on every region, with pairs that include the
virtual ends (-1, n), unrelated pairs, empty Alexandroff sets and many pairs per call.
The 1+1 profile case takes every (minimal, maximal) pair of a 16384-element diamond,
the chain-representation candidates of Sec. 2.2.  At the 131072-element 3+1 bench size,
heights of sampled elements are checked one by one against the oracle, and every
sampled height against its definition (one more than the largest height among the
element's past, from the matrix rows); degrees are checked in full against a numpy
popcount of the matrix.
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def pairs_for(n, rng, extra=12):
    lo = [-1, 0, -1, n - 2, n - 1, -1]
    hi = [n, n, n - 1, n - 1, n, 0]
    for _ in range(extra):
        a = int(rng.integers(-1, n - 1))
        b = int(rng.integers(a + 1, n + 1))
        lo.append(a)
        hi.append(b)
    return lo, hi


REGIONS = [(W.MINK2_DIAMOND, {}), (W.MINK4_DIAMOND, {}), (W.MINK3_DIAMOND, {}),
           (W.DS2_SLAB, {"eta0": W.DS2_ETA0})]


@pytest.mark.parametrize("region,kw", REGIONS, ids=["mink2", "mink4", "mink3", "ds2"])
@pytest.mark.parametrize("n", [2, 3, 65, 130, 700, 4097])
def test_chain_parity(cs, orc, region, kw, n):
    rng = np.random.default_rng(n * 7 + region)
    coords = orc.sprinkle(region, n, 30 + n, **kw)
    bits = orc.causal_matrix(region, coords)
    b = torch.from_numpy(bits.view(np.int64)).cuda()
    lo, hi = pairs_for(n, rng)
    want_l, want_h = orc.longest_chain(bits, n, lo, hi, heights=True)
    got_l, got_h = cs.cs_longest_chain(b, n, lo, hi, heights=True)
    assert np.array_equal(host(got_l), want_l)
    assert np.array_equal(host(got_h), want_h)
    # lengths alone (no height output) agree too
    only, none = cs.cs_longest_chain(b, n, lo, hi)
    assert none is None and np.array_equal(host(only), want_l)
    ind, outd, _, _ = orc.degrees(bits, n)
    gi, go = cs.cs_degrees(b, n)
    assert np.array_equal(host(gi), ind) and np.array_equal(host(go), outd)


def test_many_pairs_one_call(cs, orc):
    n = 1500
    coords = orc.sprinkle(W.MINK4_DIAMOND, n, 44)
    bits = orc.causal_matrix(W.MINK4_DIAMOND, coords)
    rng = np.random.default_rng(45)
    lo, hi = pairs_for(n, rng, extra=400)
    want, _ = orc.longest_chain(bits, n, lo, hi)
    got, _ = cs.cs_longest_chain(torch.from_numpy(bits.view(np.int64)).cuda(), n, lo, hi)
    assert np.array_equal(host(got), want)
    assert (want == 0).any() and (want > 3).any()


def test_many_related_pairs_one_call(cs, orc):
    """6000 pairs in one call (grid rows and long-scan queues far beyond the other cases):
    related pairs drawn from the matrix, pairs from the virtual bottom and to the virtual top,
    and unrelated pairs, on a 1+1 diamond (long chains) of 2048 points."""
    n = 2048
    coords = orc.sprinkle(W.MINK2_DIAMOND, n, 48)
    bits = orc.causal_matrix(W.MINK2_DIAMOND, coords)
    rng = np.random.default_rng(49)
    rows = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)
    I, J = np.nonzero(np.triu(rows, 1))
    pick = rng.choice(len(I), 3000, replace=False)
    lo = list(I[pick]) + [-1] * 1000 + list(rng.integers(0, n, 1000)) + list(rng.integers(0, n - 1, 1000))
    hi = list(J[pick]) + list(rng.integers(0, n, 1000)) + [n] * 1000
    hi += [int(rng.integers(a + 1, n)) for a in lo[len(hi):]]
    want, _ = orc.longest_chain(bits, n, lo, hi)
    got, _ = cs.cs_longest_chain(torch.from_numpy(bits.view(np.int64)).cuda(), n, lo, hi)
    assert np.array_equal(host(got), want)
    assert (want[:3000] >= 1).all() and want.max() > 40


def test_profile_pairs_mink2_n16384(cs, orc):
    """Every (minimal, maximal) pair of a 1+1 diamond at the boundary chapter's size."""
    n = 16384
    c = cs.cs_sprinkle(W.MINK2_DIAMOND, n, 46)
    b = cs.cs_causal_matrix(W.MINK2_DIAMOND, c)
    bits = host(b).view(np.uint64)
    assert np.array_equal(bits, orc.causal_matrix(W.MINK2_DIAMOND, host(c)))
    gi, go = cs.cs_degrees(b, n)
    ind, outd, _, _ = orc.degrees(bits, n)
    assert np.array_equal(host(gi), ind) and np.array_equal(host(go), outd)
    P, F = np.flatnonzero(ind == 0), np.flatnonzero(outd == 0)
    lo = np.repeat(P, len(F))
    hi = np.tile(F, len(P))
    keep = lo < hi
    lo, hi = lo[keep], hi[keep]
    want, _ = orc.longest_chain(bits, n, lo, hi)
    got, _ = cs.cs_longest_chain(b, n, lo, hi)
    assert np.array_equal(host(got), want)
    # the whole order: the longest chain of a 1+1 diamond is about 2 sqrt(N)
    whole, _ = cs.cs_longest_chain(b, n, [-1], [n])
    h = int(host(whole)[0]) - 1
    assert h == int(want.max()) + 1
    assert 0.8 * 2 * np.sqrt(n) < h < 2 * np.sqrt(n)


def degree_vectors(bits, n):
    ind = np.empty(n, dtype=np.int64)
    outd = np.empty(n, dtype=np.int64)
    for r0 in range(0, n, 4096):
        blk = bits[r0:min(n, r0 + 4096)]
        rows = np.arange(r0, r0 + blk.shape[0])
        cum = np.cumsum(np.bitwise_count(blk).astype(np.int32), axis=1, dtype=np.int64)
        wi, bi = rows >> 6, rows & 63
        before = np.where(wi > 0, cum[np.arange(len(rows)), np.maximum(wi - 1, 0)], 0)
        word = blk[np.arange(len(rows)), wi]
        low = np.bitwise_count(word & ((np.uint64(1) << bi.astype(np.uint64)) - np.uint64(1)))
        ind[rows] = before + low.astype(np.int64)
        outd[rows] = cum[:, -1] - ind[rows]
    return ind, outd


def test_heights_mink4_n131072(cs, orc):
    cfg = W.WORKLOADS["mink4_n131072"]
    n, seed = cfg["n"], cfg["seed"]
    c = cs.cs_sprinkle(W.MINK4_DIAMOND, n, seed)
    b = cs.cs_causal_matrix(W.MINK4_DIAMOND, c)
    length, height = cs.cs_longest_chain(b, n, [-1], [n], heights=True)
    gi, go = cs.cs_degrees(b, n)
    length, height, gi, go = int(host(length)[0]), host(height)[0], host(gi), host(go)
    bits = host(b).view(np.uint64)
    del b
    ind, outd = degree_vectors(bits, n)
    assert np.array_equal(gi, ind) and np.array_equal(go, outd)
    assert length == int(height.max()) + 1 and np.all(height >= 1)
    assert np.array_equal(height == 1, ind == 0)           # minimal elements
    rng = np.random.default_rng(47)
    ks = np.unique(np.concatenate([[n - 1, int(np.argmax(height))], rng.integers(0, n, 6)]))
    want, _ = orc.longest_chain(bits, n, [-1] * len(ks), ks)
    assert np.array_equal(height[ks], want)
    for k in np.unique(np.concatenate([ks, rng.integers(0, n, 200)])):
        row = np.unpackbits(bits[k].view(np.uint8), bitorder="little")[:k].astype(bool)
        past = np.flatnonzero(row)
        assert height[k] == (1 + int(height[past].max()) if len(past) else 1), k
