"""Pins for the oracle's 1+1 de Sitter slab (CPU only).

The slab of the thesis's action benchmark (Sec. 4.3): metric sec^2(eta)(-d eta^2 +
d theta^2), eta in [-eta0, eta0], theta on the circle, so the volume element is
sec^2(eta) d eta d theta and a pair is related when the angular separation, measured
the short way round, is below the conformal-time separation.  Pinned by:
  * the sampler: x = tan(eta) is uniform on [-tan eta0, tan eta0] (the sec^2 density
    is d tan(eta)/d eta) and theta uniform on [0, 2 pi) -- Kolmogorov-Smirnov tests;
  * the relation probability: theta_i - theta_j is uniform on the circle, so the short
    angular separation is uniform on [0, pi] and P(i ~ j) = E|eta_i - eta_j| / pi,
    with the expectation over the sec^2 density evaluated by quadrature;
  * symmetries of the cylinder: a rotation or a reflection of theta leaves every
    relation unchanged; the relation is a partial order (transitive, irreflexive);
  * hand-built pairs across theta = 0, related only when the separation is measured
    the short way round.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W

ETA0 = W.DS2_ETA0


def unpack(bits, n):
    b = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")
    return b[:, :n].astype(bool)


def test_sampler_marginals(orc):
    n = 20000
    x, eta, th = orc.sprinkle(W.DS2_SLAB, n, seed=31, eta0=ETA0)
    X = math.tan(ETA0)
    assert np.all(np.diff(x) >= 0)                      # labelled in time order
    assert np.all(np.diff(eta) >= 0)
    assert x.min() >= -X and x.max() < X
    assert np.all(np.abs(eta) <= ETA0)
    assert th.min() >= 0.0 and th.max() <= 2 * math.pi
    # tan(eta) uniform <=> eta has density sec^2(eta) / (2 tan eta0)
    assert stats.kstest((x + X) / (2 * X), "uniform").pvalue > 1e-3
    assert stats.kstest(th / (2 * math.pi), "uniform").pvalue > 1e-3
    # the conformal-time marginal itself, against its CDF (tan eta + tan eta0) / (2 tan eta0)
    assert stats.kstest(eta, lambda e: (np.tan(e) + X) / (2 * X)).pvalue > 1e-3


def _relation_probability(eta0):
    X = math.tan(eta0)
    rho = lambda e: 1.0 / (math.cos(e) ** 2 * 2 * X)
    # E|a - b| = 2 * int_{a > b} (a - b) rho(a) rho(b)
    val, _ = integrate.dblquad(lambda b, a: (a - b) * rho(a) * rho(b), -eta0, eta0,
                               lambda a: -eta0, lambda a: a, epsabs=1e-12, epsrel=1e-12)
    return 2 * val / math.pi


def test_relation_probability(orc):
    p = _relation_probability(ETA0)
    n, fr = 3000, []
    for seed in range(40, 45):
        c = orc.sprinkle(W.DS2_SLAB, n, seed, eta0=ETA0)
        _, _, _, rel = orc.degrees(orc.causal_matrix(W.DS2_SLAB, c), n)
        fr.append(rel / (n * (n - 1) / 2))
    # a non-cyclic separation would give about 0.94 of this; the sampling sd of one
    # fraction is about 1 % here
    assert abs(np.mean(fr) / p - 1) < 0.02, (np.mean(fr), p)


def test_cylinder_symmetries_and_order(orc):
    n = 900
    c = orc.sprinkle(W.DS2_SLAB, n, seed=33, eta0=ETA0)
    S = unpack(orc.causal_matrix(W.DS2_SLAB, c), n)
    assert np.array_equal(S, S.T) and not S.diagonal().any()
    C = np.triu(S, 1)
    two = (C.astype(np.int64) @ C.astype(np.int64)) > 0
    assert not (two & ~C).any()                          # transitive
    # rotations by multiples of pi/2 and the reflection theta -> 2 pi - theta keep
    # every short-way separation (exactly: these maps are exact or error-free here
    # up to pairs within a few ulps of the light cone, which do not occur)
    for shift in (0.5 * math.pi, math.pi, 1.5 * math.pi):
        r = c.copy()
        r[2] = np.mod(c[2] + shift, 2 * math.pi)
        assert np.array_equal(unpack(orc.causal_matrix(W.DS2_SLAB, r), n), S), shift
    r = c.copy()
    r[2] = 2 * math.pi - c[2]
    assert np.array_equal(unpack(orc.causal_matrix(W.DS2_SLAB, r), n), S)


def _pair(orc, a, b):
    """Relation of two hand-placed points (eta, theta), given in time order."""
    c = np.array([[math.tan(a[0]), math.tan(b[0])], [a[0], b[0]], [a[1], b[1]]])
    return bool(unpack(orc.causal_matrix(W.DS2_SLAB, c), 2)[0, 1])


def test_short_way_round(orc):
    tp = 2 * math.pi
    assert _pair(orc, (-0.125, 0.0625), (0.125, tp - 0.0625))      # 0.125 < 0.25
    assert not _pair(orc, (-0.125, 0.0625), (0.125, tp - 0.25))    # 0.3125 > 0.25
    assert _pair(orc, (-0.25, 1.0), (0.25, 1.25))                  # 0.25 < 0.5
    assert not _pair(orc, (-0.25, 1.0), (0.25, 1.5))               # null: strict
    assert not _pair(orc, (0.0, 1.0), (0.0, 1.0))                  # equal time
