"""Pins for the oracle's causal matrix (CPU only).

The relation is timelike separation (Ch. 4 introduction), strict on the light
cone, stored as the symmetric packed matrix P + P^T of Sec. 3.2.  Pinned by:
partial-order axioms, geometric special cases with exactly representable
coordinates, and the ordering fractions of the diamonds (1/2 of pairs in 1+1,
8/35 in 2+1 and 1/10 in 3+1 -- the Myrheim-Meyer fraction Γ(d+1)Γ(d/2)/(2Γ(3d/2)) at
d = 2, 3, 4).
"""
import math

import numpy as np
import pytest

import workloads as W


def unpack(bits, n):
    b = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")
    return b[:, :n].astype(bool), b[:, n:]


@pytest.mark.parametrize("region", [W.MINK2_DIAMOND, W.MINK4_DIAMOND, W.DS4_SLAB,
                                    W.MINK3_DIAMOND])
def test_matrix_is_a_partial_order(orc, region):
    n = 700
    c = orc.sprinkle(region, n, seed=21)
    bits = orc.causal_matrix(region, c)
    S, pad = unpack(bits, n)
    assert not pad.any()
    assert np.array_equal(S, S.T)
    assert not S.diagonal().any()
    C = np.triu(S, 1)
    # transitivity: i ≺ k ≺ j  =>  i ≺ j
    two = (C.astype(np.int64) @ C.astype(np.int64)) > 0
    assert not (two & ~C).any()
    assert C.sum() > 0


def _mat(orc, region, pts):
    c = np.ascontiguousarray(np.array(pts, dtype=np.float64).T)
    return unpack(orc.causal_matrix(region, c), c.shape[1])[0]


def test_mink4_special_cases(orc):
    # time axis: a chain
    S = _mat(orc, W.MINK4_DIAMOND, [(0.1 * k, 0, 0, 0) for k in range(1, 6)])
    assert np.triu(S, 1).sum() == 10
    # one time slice: an antichain
    S = _mat(orc, W.MINK4_DIAMOND, [(0.5, 0.01 * k, 0, 0) for k in range(5)])
    assert not S.any()
    # exactly null separated (all values dyadic): unrelated; just inside: related
    pts = [(0.25, 0, 0, 0), (0.5, 0.25, 0, 0), (0.5, 0, 0.125, 0.125), (0.5, 0.0, 0.0, 0.24)]
    S = _mat(orc, W.MINK4_DIAMOND, pts)
    assert not S[0, 1]                     # dt = dx = 1/4
    assert S[0, 2]                         # dt^2 = 1/16 > 1/32
    assert S[0, 3]                         # dt = 0.25 > 0.24
    pts = [(0.25, 0, 0, 0), (0.5, 0.125, 0.125, 0.125 * math.sqrt(2))]
    S = _mat(orc, W.MINK4_DIAMOND, pts)
    assert S[0, 1] == (0.0625 > (0.015625 + 0.015625) + (0.125 * math.sqrt(2)) ** 2)


def test_mink2_special_cases(orc):
    S = _mat(orc, W.MINK2_DIAMOND, [(0.1, 0.1), (0.1, 0.5), (0.2, 0.6), (0.3, 0.05)])
    assert not S[0, 1]          # equal u: null separated
    assert S[0, 2] and S[1, 2]
    assert not S[0, 3] and not S[2, 3]


def test_ds4_special_cases(orc):
    def pt(eta, nvec):
        x = math.tan(eta)
        c = 1 / math.sqrt(1 + x * x)
        return (x, c, x * c, *nvec)
    e = (1.0, 0.0, 0.0, 0.0)
    anti = (-1.0, 0.0, 0.0, 0.0)
    side = (0.0, 1.0, 0.0, 0.0)   # 90 degrees from e
    pts = [pt(-1.0, e), pt(1.0, e), pt(1.1, anti), pt(0.6, side), pt(0.5, side)]
    S = _mat(orc, W.DS4_SLAB, pts)
    assert S[0, 1]             # same point of S^3, later
    assert not S[0, 2]         # antipodal: angle pi > 2.1
    assert S[0, 3]             # d eta = 1.6 > pi/2
    assert not S[0, 4]         # d eta = 1.5 < pi/2
    assert not S[3, 4]         # same spatial point, earlier one second: eta decreasing


def _ordering_fraction(orc, region, n, seeds):
    fr = []
    for s in seeds:
        c = orc.sprinkle(region, n, seed=s)
        S, _ = unpack(orc.causal_matrix(region, c), n)
        fr.append(np.triu(S, 1).sum() / (n * (n - 1) / 2))
    return np.mean(fr), np.std(fr, ddof=1) / math.sqrt(len(fr))


def test_mink2_ordering_fraction_is_half(orc):
    m, se = _ordering_fraction(orc, W.MINK2_DIAMOND, 400, range(100, 130))
    assert abs(m - 0.5) < 5 * se + 1e-3


def test_mink3_ordering_fraction(orc):
    target = math.gamma(4) * math.gamma(1.5) / (2 * math.gamma(4.5))
    assert abs(target - 8 / 35) < 1e-15
    m, se = _ordering_fraction(orc, W.MINK3_DIAMOND, 600, range(300, 330))
    assert abs(m - target) < 4 * se


def test_mink4_ordering_fraction_is_tenth(orc):
    g = math.gamma
    target = g(5) * g(2) / (2 * g(6))
    assert abs(target - 0.1) < 1e-15
    m, se = _ordering_fraction(orc, W.MINK4_DIAMOND, 600, range(200, 230))
    assert abs(m - target) < 5 * se + 1e-3


@pytest.mark.parametrize("region", [W.MINK2_DIAMOND, W.MINK4_DIAMOND, W.DS4_SLAB,
                                    W.MINK3_DIAMOND])
def test_matrix_against_vectorised_predicate(orc, region):
    """Cross-check of the C indexing against a numpy evaluation of the same predicate."""
    n = 333
    c = orc.sprinkle(region, n, seed=31)
    S, _ = unpack(orc.causal_matrix(region, c), n)
    i, j = np.triu_indices(n, 1)
    if region == W.MINK2_DIAMOND:
        r = (c[0][i] < c[0][j]) & (c[1][i] < c[1][j])
    elif region == W.MINK4_DIAMOND:
        dt = c[0][j] - c[0][i]
        d = [c[k][j] - c[k][i] for k in (1, 2, 3)]
        s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        r = (dt > 0) & (dt * dt > s)
    elif region == W.MINK3_DIAMOND:
        dt = c[0][j] - c[0][i]
        dx, dy = c[1][j] - c[1][i], c[2][j] - c[2][i]
        r = (dt > 0) & (dt * dt > dx * dx + dy * dy)
    else:
        cd = c[1][i] * c[1][j] + c[2][i] * c[2][j]
        dot = ((c[3][i] * c[3][j] + c[4][i] * c[4][j]) + c[5][i] * c[5][j]) + c[6][i] * c[6][j]
        r = (c[0][i] < c[0][j]) & (cd < dot)
    assert np.array_equal(S[i, j], r)


@pytest.mark.parametrize("region", [W.MINK2_DIAMOND, W.MINK4_DIAMOND, W.DS4_SLAB,
                                    W.MINK3_DIAMOND, W.DS2_SLAB])
def test_sampled_rows_equal_full_matrix(orc, region):
    n = 1100
    c = orc.sprinkle(region, n, seed=61)
    full = orc.causal_matrix(region, c)
    rows = [0, 1, 63, 64, 65, 500, 1098, 1099]
    assert np.array_equal(orc.causal_rows(region, c, rows), full[rows])
