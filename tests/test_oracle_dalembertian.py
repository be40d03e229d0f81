"""Pins for the oracle's discrete d'Alembertian B^(d+1) phi (Sec. 4.1, eqs. b2d_local and
b3d_local, b4d_local), CPU only:
  * brute force: every labelled 2D order on n <= 5 elements, exact rationals, with the
    order intervals found by enumerating each Alexandroff set;
  * a chain, where L_m(j) = {j - m}, gives the finite-difference stencil of the bracket;
  * an antichain, where every L_m is empty, gives -(K / ell^2) phi;
  * summed over the set with phi = 1 it gives -(1 / ell^2) times the local action
    (sum_j |L_m(j)| = N_{m-1}), whose coefficients are pinned separately;
  * linearity in phi.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import brute

K = {2: 2.0, 3: (math.pi / (3 * math.sqrt(2))) ** (2 / 3) / math.gamma(5 / 3),
     4: 4.0 / math.sqrt(6.0)}
C = {2: (2.0, -4.0, 2.0), 3: (1.0, -27 / 8, 9 / 4), 4: (1.0, -9.0, 16.0, -8.0)}


def _matrix(orc, region, pts):
    c = np.ascontiguousarray(np.array(pts, dtype=np.float64).T)
    return orc.causal_matrix(region, c), c.shape[1]


def test_brute_force_all_2d_orders(orc):
    rng = np.random.default_rng(3)
    ell = 0.5
    for n in (3, 4, 5):
        for u, v in brute.all_2d_orders(n):
            rel = brute.order_from_dominance(u, v)
            pts = [((u[k] + 1) / 8.0, (v[k] + 1) / 8.0) for k in range(n)]
            order = sorted(range(n), key=lambda k: (u[k] + v[k], k))
            pts = [pts[k] for k in order]
            inv = {k: r for r, k in enumerate(order)}
            rel = {(inv[a], inv[b]) for (a, b) in rel}
            bits, _ = _matrix(orc, W.MINK2_DIAMOND, pts)
            phi = rng.integers(-8, 9, n) / 4.0
            got, _, _ = orc.dalembertian(bits, n, 2, ell, phi)
            want = brute.dalembertian_2d_exact(n, rel, list(phi), Fraction(ell) ** 2)
            assert [float(w) for w in want] == list(got), (u, v)


@pytest.mark.parametrize("dim,region", [(2, W.MINK2_DIAMOND), (3, W.MINK3_DIAMOND),
                                        (4, W.MINK4_DIAMOND)])
def test_chain_stencil_and_antichain(orc, dim, region):
    n, ell = 12, 0.25
    phi = np.random.default_rng(4).normal(size=n)
    if dim == 2:
        chain = [((k + 1) / 16.0, (k + 1) / 16.0) for k in range(n)]
        anti = [((k + 1) / 16.0, (n - k) / 16.0) for k in range(n)]
    elif dim == 3:
        chain = [((k + 1) / 16.0, 0.0, 0.0) for k in range(n)]
        anti = [(0.5, (k - 6) / 64.0, 0.0) for k in range(n)]
    else:
        chain = [((k + 1) / 16.0, 0.0, 0.0, 0.0) for k in range(n)]
        anti = [(0.5, (k - 6) / 64.0, 0.0, 0.0) for k in range(n)]
    bits, _ = _matrix(orc, region, chain)
    got, terms, _ = orc.dalembertian(bits, n, dim, ell, phi)
    for j in range(n):
        br = -phi[j] + sum(c * phi[j - m - 1] for m, c in enumerate(C[dim]) if j - m - 1 >= 0)
        assert got[j] == pytest.approx(K[dim] / ell ** 2 * br, rel=1e-13, abs=1e-12)
        assert terms[j] == 1 + min(j, len(C[dim]))
    bits, _ = _matrix(orc, region, anti)
    got, terms, _ = orc.dalembertian(bits, n, dim, ell, phi)
    assert np.allclose(got, -K[dim] / ell ** 2 * phi, rtol=1e-14, atol=0)
    assert np.all(terms == 1)


@pytest.mark.parametrize("dim,region,n", [(2, W.MINK2_DIAMOND, 600), (3, W.MINK3_DIAMOND, 1000),
                                          (4, W.MINK4_DIAMOND, 1500)])
def test_sum_of_constant_field_is_minus_the_action(orc, dim, region, n):
    ell = 0.3
    c = orc.sprinkle(region, n, seed=5)
    bits = orc.causal_matrix(region, c)
    got, _, _ = orc.dalembertian(bits, n, dim, ell, np.ones(n))
    s_local = orc.action(orc.histogram_naive(bits, n), n, dim, 0.0)[0]
    assert -ell ** 2 * math.fsum(got) == pytest.approx(s_local, rel=1e-12, abs=1e-9)


def test_linearity(orc):
    n, ell = 800, 0.1
    c = orc.sprinkle(W.MINK2_DIAMOND, n, seed=6)
    bits = orc.causal_matrix(W.MINK2_DIAMOND, c)
    rng = np.random.default_rng(7)
    a, b = rng.normal(size=n), rng.normal(size=n)
    ba, _, ma = orc.dalembertian(bits, n, 2, ell, a)
    bb, _, mb = orc.dalembertian(bits, n, 2, ell, b)
    bab, terms, mab = orc.dalembertian(bits, n, 2, ell, 3 * a + b)
    bound = 4 * (terms + 2) * 2.0 ** -53 * 2 / ell ** 2 * (3 * ma + mb + mab)
    assert np.all(np.abs(bab - (3 * ba + bb)) <= bound)


def test_selected_elements_match_the_full_sums(orc):
    """The per-element entry point (used at sizes where the full sums are too slow) gives
    the full call's values for the elements it is asked for, in their order."""
    n = 900
    c = orc.sprinkle(W.MINK4_DIAMOND, n, 71)
    bits = orc.causal_matrix(W.MINK4_DIAMOND, c)
    phi = np.random.default_rng(72).normal(size=n)
    full = orc.dalembertian(bits, n, 4, 0.05, phi)
    js = np.array([n - 1, 0, 450, 451, 17, n - 1])
    part = orc.dalembertian_cols(bits, n, 4, 0.05, phi, js)
    for a, b in zip(full, part):
        assert np.array_equal(a[js], b)
