"""Pins for the oracle's longest chains (Sec. 2.5.2, algorithm "Maximal Chain Length").

Lengths count links; -1 and n are virtual elements below and above everything.
Pinned by:
  * 2D orders: a 1+1 diamond is the order u_i < u_j and v_i < v_j, so the longest chain
    through a set of points is the longest strictly increasing subsequence of v taken in
    u order (patience sorting, a textbook routine); the longest chain between i and j
    is one link more than that of the points strictly inside their (u, v) rectangle, and
    the height of k is the longest increasing subsequence ending at k;
  * brute force over every path of the relation on tiny 3D and 4D orders;
  * closed forms: a total order, an antichain, disjoint unions of chains;
  * Mirsky's theorem on a 3+1 sprinkling: removing minimal elements layer by layer
    (numpy) takes exactly as many rounds as the longest chain has elements, and the
    heights are constant on those layers;
  * the recursion entered from either end gives the same lengths.
The degree vectors, used to find minimal and maximal elements, are pinned by quadrant
counts of a 2D order and by a total order.
"""
import bisect

import numpy as np
import pytest

import workloads as W


def pack(rel):
    """Packed symmetric bitset rows of a boolean relation matrix (rel[i, j]: i ≺ j)."""
    n = rel.shape[0]
    S = rel | rel.T
    ld = ((n + 511) // 512) * 8
    b = np.zeros((n, ld * 64), dtype=np.uint8)
    b[:, :n] = S
    return np.packbits(b, axis=1, bitorder="little").view(np.uint64).copy()


def order_2d(u, v):
    """i ≺ j iff u_i < u_j and v_i < v_j, labelled by increasing u."""
    idx = np.argsort(u, kind="stable")
    u, v = u[idx], v[idx]
    rel = (u[:, None] < u[None, :]) & (v[:, None] < v[None, :])
    return rel, u, v


def lis_ending(v):
    """For each k, the longest strictly increasing subsequence of v ending at k."""
    tails, out = [], []
    for x in v:
        p = bisect.bisect_left(tails, x)
        if p == len(tails):
            tails.append(x)
        else:
            tails[p] = x
        out.append(p + 1)
    return np.array(out)


def lis(v):
    return int(lis_ending(v).max()) if len(v) else 0


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (50, 2), (2000, 3)])
def test_2d_whole_order_is_lis(orc, n, seed):
    rng = np.random.default_rng(seed)
    rel, u, v = order_2d(rng.random(n), rng.random(n))
    length, h = orc.longest_chain(pack(rel), n, [-1], [n], heights=True)
    assert length[0] == lis(v) + 1
    assert np.array_equal(h[0], lis_ending(v))


def test_2d_pairs_are_lis_of_rectangles(orc):
    rng = np.random.default_rng(4)
    n = 70
    rel, u, v = order_2d(rng.random(n), rng.random(n))
    bits = pack(rel)
    pairs = [(i, j) for i in range(-1, n) for j in range(i + 1, n + 1)]
    lo = [p[0] for p in pairs]
    hi = [p[1] for p in pairs]
    length, _ = orc.longest_chain(bits, n, lo, hi)
    for (i, j), got in zip(pairs, length):
        vi = -np.inf if i < 0 else v[i]
        vj = np.inf if j == n else v[j]
        if i >= 0 and j < n and not rel[i, j]:
            assert got == 0, (i, j)
            continue
        inside = [v[m] for m in range(i + 1, j) if vi < v[m] < vj]
        assert got == lis(inside) + 1, (i, j)


def test_2d_sprinkle_is_lis(orc):
    n = 3000
    c = orc.sprinkle(W.MINK2_DIAMOND, n, 21)
    u, v = c[0], c[1]
    bits = orc.causal_matrix(W.MINK2_DIAMOND, c)
    length, h = orc.longest_chain(bits, n, [-1], [n], heights=True)
    # labels are in time order; the chain is the increasing subsequence of v in u order
    order = np.argsort(u, kind="stable")
    assert length[0] == lis(v[order]) + 1
    ending = np.empty(n, dtype=np.int64)
    ending[order] = lis_ending(v[order])
    assert np.array_equal(h[0], ending)


def brute_longest(rel, a, b):
    """Longest path (links) from a to b over the relation, by trying every path."""
    n = rel.shape[0]

    def succ(x):
        if x == -1:
            return range(n)
        return [y for y in range(n) if rel[x, y]]

    def ends(x):
        return b == n or (x == -1 and b < n) or (x >= 0 and rel[x, b])

    best = 0

    def walk(x, links):
        nonlocal best
        if ends(x):
            best = max(best, links + 1)
        for y in succ(x):
            if b == n or rel[y, b]:
                walk(y, links + 1)
    if a == -1 or b == n or rel[a, b]:
        walk(a, 0)
    return best


@pytest.mark.parametrize("dim,seed", [(3, 5), (4, 6), (4, 7)])
def test_tiny_orders_brute_force(orc, dim, seed):
    rng = np.random.default_rng(seed)
    n = 9
    t = np.sort(rng.random(n))
    x = rng.random((n, dim - 1)) - 0.5
    dt = t[None, :] - t[:, None]
    d2 = ((x[None, :, :] - x[:, None, :]) ** 2).sum(-1)
    rel = (dt > 0) & (dt * dt > d2)
    pairs = [(i, j) for i in range(-1, n) for j in range(i + 1, n + 1)]
    length, h = orc.longest_chain(pack(rel), n, [p[0] for p in pairs], [p[1] for p in pairs],
                                  heights=True)
    for s, (i, j) in enumerate(pairs):
        assert length[s] == brute_longest(rel, i, j), (i, j)
        for k in range(n):
            inside = (i == -1 or rel[i, k]) and (k == j or j == n or rel[k, j])
            want = brute_longest(rel, i, k) if inside else 0
            assert h[s, k] == want, (i, j, k)


def test_closed_forms(orc):
    n = 40
    chain = np.triu(np.ones((n, n), dtype=bool), 1)
    length, h = orc.longest_chain(pack(chain), n, [-1, 0, 3, 5], [n, n - 1, 4, 30], heights=True)
    assert list(length) == [n + 1, n - 1, 1, 25]
    assert np.array_equal(h[0], np.arange(1, n + 1))
    anti = np.zeros((n, n), dtype=bool)
    length, h = orc.longest_chain(pack(anti), n, [-1, 0, -1, 7], [n, 1, 9, n], heights=True)
    assert list(length) == [2, 0, 1, 1]
    assert np.array_equal(h[0], np.ones(n)) and not h[1].any()
    assert h[2, 9] == 1 and h[2].sum() == 1
    # disjoint union of chains of sizes 5, 11, 3 (interleaved labels)
    sizes = [5, 11, 3]
    label = np.concatenate([np.full(s, c) for c, s in enumerate(sizes)])
    perm = np.random.default_rng(8).permutation(len(label))
    lab = label[perm]
    m = len(lab)
    rel = (lab[:, None] == lab[None, :]) & np.triu(np.ones((m, m), dtype=bool), 1)
    length, _ = orc.longest_chain(pack(rel), m, [-1], [m])
    assert length[0] == max(sizes) + 1


def test_mirsky_layers_4d(orc):
    n = 1500
    c = orc.sprinkle(W.MINK4_DIAMOND, n, 9)
    bits = orc.causal_matrix(W.MINK4_DIAMOND, c)
    S = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)
    past = np.tril(S, -1)                      # past[k, i]: i ≺ k
    length, h = orc.longest_chain(bits, n, [-1], [n], heights=True)
    remaining = np.ones(n, dtype=bool)
    rounds = 0
    while remaining.any():
        minimal = remaining & ~(past & remaining[None, :]).any(1)
        rounds += 1
        assert np.all(h[0][minimal] == rounds)
        remaining &= ~minimal
    assert length[0] == rounds + 1
    assert rounds > 5


def test_both_ends_agree(orc):
    n = 400
    c = orc.sprinkle(W.MINK3_DIAMOND, n, 10)
    bits = orc.causal_matrix(W.MINK3_DIAMOND, c)
    for lo, hi in [(-1, n), (3, n), (-1, 350), (2, 390)]:
        length, h = orc.longest_chain(bits, n, [lo], [hi], heights=True)
        ks = np.flatnonzero(h[0])
        got, _ = orc.longest_chain(bits, n, [lo] * len(ks), ks)
        assert np.array_equal(got, h[0][ks])
        if hi < n and length[0]:
            assert h[0][hi] == length[0]


def test_bad_pairs_rejected(orc):
    n = 10
    bits = pack(np.zeros((n, n), dtype=bool))
    for lo, hi in [(3, 3), (5, 2), (-2, 4), (0, n + 1), (n, n + 1)]:
        with pytest.raises(ValueError):
            orc.longest_chain(bits, n, [lo], [hi])


def test_degrees(orc):
    """Past and future degrees (the degree vectors of Sec. 3.2): counts of points in the
    lower-left and upper-right quadrants of a 2D order; i and n-1-i on a total order."""
    rng = np.random.default_rng(11)
    n = 600
    rel, u, v = order_2d(rng.random(n), rng.random(n))
    ind, outd, _, r = orc.degrees(pack(rel), n)
    below = ((u[None, :] < u[:, None]) & (v[None, :] < v[:, None])).sum(1)
    above = ((u[None, :] > u[:, None]) & (v[None, :] > v[:, None])).sum(1)
    assert np.array_equal(ind, below) and np.array_equal(outd, above) and r == rel.sum()
    m = 77
    ind, outd, _, _ = orc.degrees(pack(np.triu(np.ones((m, m), dtype=bool), 1)), m)
    assert np.array_equal(ind, np.arange(m)) and np.array_equal(outd, m - 1 - np.arange(m))
