"""Pins for the oracle's interval abundances (CPU only).

N_n is the number of related pairs whose Alexandroff set holds n elements
(eq. IOIs; the thesis's n_m is N_{m-1}).  Pinned by brute-force enumeration of
every 2D order on up to 6 elements, closed forms (chain, antichain, disjoint
chains), exact invariants, the numpy C@C special case, relabelling invariance,
the naive/optimised algorithm agreement and the 2D expectation E[N_n] by
quadrature.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import brute


def _hist_from_coords(orc, region, coords, naive=True):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[1]
    bits = orc.causal_matrix(region, coords)
    h = orc.histogram_naive(bits, n) if naive else orc.histogram_fast(bits, n)[0]
    return bits, h


def _sorted2d(u, v):
    order = np.lexsort((u, np.add(u, v)))
    return np.array([np.asarray(u, float)[order], np.asarray(v, float)[order]])


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_all_2d_orders_brute_force(orc, n):
    for u, v in brute.all_2d_orders(n):
        c = _sorted2d([x + 1.0 for x in u], [x + 1.0 for x in v])
        _, h = _hist_from_coords(orc, W.MINK2_DIAMOND, c)
        rel = brute.order_from_dominance(list(c[0]), list(c[1]))
        want = brute.abundances(n, rel)
        assert list(h) == want, (u, v)


@pytest.mark.parametrize("n", [2, 7, 64, 65, 130])
def test_chain_and_antichain(orc, n):
    k = np.arange(1, n + 1, dtype=float)
    _, h = _hist_from_coords(orc, W.MINK2_DIAMOND, [k, k])
    assert list(h) == [n - 1 - m for m in range(n - 1)]
    _, h = _hist_from_coords(orc, W.MINK2_DIAMOND, _sorted2d(k, k[::-1]))
    assert not h.any()
    t = np.zeros((4, n))
    t[0] = k / (n + 1)
    _, h4 = _hist_from_coords(orc, W.MINK4_DIAMOND, t, naive=False)
    assert list(h4) == [n - 1 - m for m in range(n - 1)]


def test_disjoint_chains(orc):
    # three chains, mutually unrelated: block-diagonal staircase in (u, v)
    lens = [5, 9, 3]
    u, v = [], []
    base_u, base_v = 0.0, 100.0
    for L in lens:
        for q in range(L):
            u.append(base_u + q)
            v.append(base_v + q)
        base_u += L
        base_v -= 50
    c = _sorted2d(u, v)
    n = len(u)
    _, h = _hist_from_coords(orc, W.MINK2_DIAMOND, c)
    want = np.zeros(n - 1, dtype=np.int64)
    for L in lens:
        for m in range(L - 1):
            want[m] += L - 1 - m
    assert np.array_equal(h.astype(np.int64), want)


@pytest.mark.parametrize("region,n", [(W.MINK2_DIAMOND, 1024), (W.MINK4_DIAMOND, 1500),
                                      (W.DS4_SLAB, 1200)])
def test_invariants_and_numpy_product(orc, region, n):
    c = orc.sprinkle(region, n, seed=41)
    bits, h = _hist_from_coords(orc, region, c)
    _, _, chains3, rel = orc.degrees(bits, n)
    assert int(h.sum()) == rel
    assert int((np.arange(n - 1, dtype=np.uint64) * h).sum()) == chains3
    S = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)
    C = np.triu(S, 1).astype(np.float64)
    P = C @ C                               # exact: entries < 2^53
    want = np.bincount(P[C > 0].astype(np.int64), minlength=n - 1)
    assert np.array_equal(h.astype(np.int64), want)


@pytest.mark.parametrize("region,n", [(W.MINK2_DIAMOND, 1024), (W.MINK4_DIAMOND, 2048),
                                      (W.DS4_SLAB, 2048), (W.MINK2_DIAMOND, 577)])
def test_naive_equals_optimised(orc, region, n):
    c = orc.sprinkle(region, n, seed=43)
    bits = orc.causal_matrix(region, c)
    a = orc.histogram_naive(bits, n)
    b, pairs = orc.histogram_fast(bits, n)
    assert np.array_equal(a, b)
    assert pairs == int(a.sum())


def test_row_restricted_fast_tier_adds_up(orc):
    n = 900
    c = orc.sprinkle(W.MINK4_DIAMOND, n, seed=44)
    bits = orc.causal_matrix(W.MINK4_DIAMOND, c)
    full, _ = orc.histogram_fast(bits, n)
    parts = sum(orc.histogram_fast(bits, n, a, b)[0].astype(np.int64)
                for a, b in [(0, 100), (100, 517), (517, n)])
    assert np.array_equal(parts, full.astype(np.int64))


def test_relabelling_invariance(orc):
    """Sorting by u alone is another natural labelling of a 2D order."""
    n = 800
    c = orc.sprinkle(W.MINK2_DIAMOND, n, seed=45)
    _, h1 = _hist_from_coords(orc, W.MINK2_DIAMOND, c)
    order = np.lexsort((c[1], c[0]))
    _, h2 = _hist_from_coords(orc, W.MINK2_DIAMOND, c[:, order])
    assert np.array_equal(h1, h2)


@pytest.mark.slow
def test_mink2_expected_abundances(orc):
    """E[N_n] = N(N-1) C(N-2,n) ∫∫ (1-a)(1-b)(ab)^n (1-ab)^(N-2-n) da db for the
    1+1 diamond (a, b: the light-cone extents of a pair), against the mean over seeds."""
    n, seeds = 64, range(1000, 1400)
    hs = np.array([_hist_from_coords(orc, W.MINK2_DIAMOND,
                                     orc.sprinkle(W.MINK2_DIAMOND, n, seed=s))[1]
                   for s in seeds], dtype=np.float64)
    mean, se = hs.mean(0), hs.std(0, ddof=1) / math.sqrt(len(seeds))
    for m in (0, 1, 2, 5, 12):
        f = lambda a, b: (1 - a) * (1 - b) * (a * b) ** m * (1 - a * b) ** (n - 2 - m)
        val, _ = integrate.dblquad(f, 0, 1, 0, 1, epsabs=1e-13, epsrel=1e-10)
        exp = n * (n - 1) * math.comb(n - 2, m) * val
        assert abs(mean[m] - exp) < 5 * se[m] + 1e-9, (m, mean[m], exp, se[m])
    assert abs(hs.sum(1).mean() - n * (n - 1) / 4) < 5 * hs.sum(1).std() / math.sqrt(len(seeds))


def test_element_restricted_naive_tier_adds_up(orc):
    """The definitional tier over disjoint sets of elements j adds up to the whole count,
    and each element's part holds exactly its past's size in pairs (sum over i ≺ j)."""
    n = 700
    c = orc.sprinkle(W.MINK4_DIAMOND, n, seed=46)
    bits = orc.causal_matrix(W.MINK4_DIAMOND, c)
    full = orc.histogram_naive(bits, n)
    rng = np.random.default_rng(3)
    perm = rng.permutation(n)
    parts = [orc.histogram_naive_elems(bits, n, perm[a:b]) for a, b in [(0, 50), (50, 333), (333, n)]]
    assert np.array_equal(sum(p.astype(np.int64) for p in parts), full.astype(np.int64))
    ind, _, _, _ = orc.degrees(bits, n)
    assert int(parts[0].sum()) == int(ind[perm[:50]].sum())
    with pytest.raises(ValueError):
        orc.histogram_naive_elems(bits, n, [n])
