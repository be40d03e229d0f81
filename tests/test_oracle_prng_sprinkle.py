"""Pins for the oracle's generator and sprinklings (CPU only).

Generator: the published SplitMix64 test vector, and the jump-ahead used for
counter-based draws against the sequential generator.
Sprinklings (App. A, "Causal Set Sprinklings"): support, time order, and
Kolmogorov-Smirnov / moment tests of the marginals each region fixes.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector(orc):
    with open(os.path.join(GOLDEN, "splitmix64_state0.txt")) as f:
        want = [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
    assert orc.splitmix64_sequence(0, len(want)) == want


@pytest.mark.parametrize("seed,stream,c", [(0, 0, 0), (1, 0, 5), (7, 3, 17), (2**63 + 5, 2, 40)])
def test_counter_draw_equals_sequential_generator(orc, seed, stream, c):
    key_seed = orc.splitmix64_sequence(seed, 1)[0]
    key_stream = orc.splitmix64_sequence(key_seed, stream + 1)[-1]
    want = orc.splitmix64_sequence(key_stream, c + 1)[-1]
    assert orc.draw(seed, stream, c) == want


def test_mink2_support_order_and_marginals(orc):
    n = 20000
    c = orc.sprinkle(W.MINK2_DIAMOND, n, seed=11)
    u, v = c
    assert np.all((u >= 0) & (u < 1) & (v >= 0) & (v < 1))
    key = np.round(u * 2**53).astype(np.uint64) + np.round(v * 2**53).astype(np.uint64)
    assert np.all(np.diff(key.astype(np.float64)) >= 0)  # time order by u+v
    assert np.all(u * 2**53 == np.floor(u * 2**53))       # 53-bit grid
    for x in (u, v):
        assert stats.kstest(x, "uniform").pvalue > 1e-4
    assert abs(np.corrcoef(u, v)[0, 1]) < 5 / math.sqrt(n)


def test_mink4_support_order_and_marginals(orc):
    n = 20000
    t, x, y, z = orc.sprinkle(W.MINK4_DIAMOND, n, seed=12)
    r = np.sqrt(x * x + y * y + z * z)
    rmax = np.minimum(t, 1 - t)
    assert np.all(r < rmax)
    assert np.all(np.diff(t) >= 0)
    # Time marginal of the height-1 diamond: density ∝ min(t,1-t)^3,
    # CDF 8t^4 on [0,1/2] and 1 - 8(1-t)^4 on [1/2,1].
    cdf = lambda s: np.where(s < 0.5, 8 * s**4, 1 - 8 * (1 - s) ** 4)
    assert stats.kstest(t, cdf).pvalue > 1e-4
    # Uniform in each spatial ball: (r/rmax)^3 ~ U(0,1); direction isotropic.
    assert stats.kstest((r / rmax) ** 3, "uniform").pvalue > 1e-4
    for w in (x, y, z):
        assert abs(np.mean(w / r)) < 5 / math.sqrt(3 * n)


def test_mink3_support_order_and_marginals(orc):
    n = 20000
    t, x, y = orc.sprinkle(W.MINK3_DIAMOND, n, seed=14)
    r = np.sqrt(x * x + y * y)
    rmax = np.minimum(t, 1 - t)
    assert np.all(r < rmax)
    assert np.all(np.diff(t) >= 0)
    # 2+1 diamond of height 1: time density ∝ min(t,1-t)^2, CDF 4t^3 / 1 - 4(1-t)^3.
    cdf = lambda s: np.where(s < 0.5, 4 * s**3, 1 - 4 * (1 - s) ** 3)
    assert stats.kstest(t, cdf).pvalue > 1e-4
    # Uniform in each disc: (r/rmax)^2 ~ U(0,1); the angle is uniform.
    assert stats.kstest((r / rmax) ** 2, "uniform").pvalue > 1e-4
    assert stats.kstest((np.arctan2(y, x) + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-4


def test_ds4_support_order_and_marginals(orc):
    n = 20000
    eta0 = W.DS_ETA0
    c = orc.sprinkle(W.DS4_SLAB, n, seed=13, eta0=eta0)
    x, ce, se, n0, n1, n2, n3 = c
    X = math.tan(eta0)
    assert np.all(np.abs(x) <= X * (1 + 1e-15))
    assert np.all(np.diff(x) >= 0)
    eta = np.arctan(x)
    assert np.allclose(ce, np.cos(eta), rtol=0, atol=1e-15)
    assert np.allclose(se, np.sin(eta), rtol=0, atol=1e-15)
    # Conformal-time marginal ∝ sec^4(eta) on [-eta0, eta0]:
    # CDF = (tan + tan^3/3 + Y) / 2Y, Y = X + X^3/3.
    Y = X + X**3 / 3
    cdf = lambda e: (np.tan(e) + np.tan(e) ** 3 / 3 + Y) / (2 * Y)
    assert stats.kstest(eta, cdf).pvalue > 1e-4
    nv = np.stack([n0, n1, n2, n3])
    assert np.allclose(np.sum(nv * nv, axis=0), 1.0, atol=1e-15)
    # Uniform on S^3 ⊂ R^4: E[n_k] = 0, E[n_k^2] = 1/4, E[n_k^4] = 3/(4*6) = 1/8.
    for k in range(4):
        assert abs(np.mean(nv[k])) < 5 * math.sqrt(0.25 / n)
        assert abs(np.mean(nv[k] ** 2) - 0.25) < 5 * math.sqrt((1 / 8 - 1 / 16) / n)
        assert abs(np.mean(nv[k] ** 4) - 0.125) < 0.01


def test_sprinkle_deterministic(orc):
    for region in (W.MINK2_DIAMOND, W.MINK4_DIAMOND, W.DS4_SLAB, W.MINK3_DIAMOND, W.DS2_SLAB):
        a = orc.sprinkle(region, 500, seed=99)
        b = orc.sprinkle(region, 500, seed=99)
        assert np.array_equal(a, b)
        assert not np.array_equal(a, orc.sprinkle(region, 500, seed=100))


def test_mink3_prefix_property(orc):
    a = orc.sprinkle(W.MINK3_DIAMOND, 300, seed=5)
    b = orc.sprinkle(W.MINK3_DIAMOND, 600, seed=5)
    # the first 300 accepted candidates are a subset of the first 600
    sa = set(map(tuple, a.T))
    assert sa <= set(map(tuple, b.T))


def test_mink4_prefix_property(orc):
    """The first n accepted candidates are kept: a smaller sprinkle is the
    subset of a larger one with the same seed (as a set of points)."""
    a = orc.sprinkle(W.MINK4_DIAMOND, 300, seed=5)
    b = orc.sprinkle(W.MINK4_DIAMOND, 600, seed=5)
    sa = {tuple(p) for p in a.T}
    sb = {tuple(p) for p in b.T}
    assert sa <= sb
