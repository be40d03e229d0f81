"""Pins for the oracle's Benincasa-Dowker actions (CPU only).

Local actions S^(1+1), S^(2+1), S^(3+1) and smeared actions S_eps with f_2, f_3, f_4
(Sec. 4.2).  Pinned by exact rational evaluation of the printed formulas (Python
fractions), closed forms for chains and antichains, the eps -> 1 reduction, and the
2+1 prefactor against scipy's gamma function.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import brute

C3 = (math.pi / (3 * math.sqrt(2))) ** (2.0 / 3.0) / __import__("scipy.special").special.gamma(5 / 3)


@pytest.mark.parametrize("dim", [2, 3, 4])
@pytest.mark.parametrize("eps", [0.05, 0.1, 0.2, 2.0**-6, 0.5])
def test_smear_weight_matches_printed_formula(orc, dim, eps):
    e = Fraction(eps)  # the exact value of the double
    for m in list(range(0, 12)) + [50, 333, 1000]:
        exact = brute.smear_exact(dim, m, e)
        got = orc.smear_weight(dim, m, eps)
        assert got == float(exact) or abs(got - float(exact)) <= 1e-15 * abs(float(exact)), (m, got)


@pytest.mark.parametrize("dim", [2, 3, 4])
def test_eps_one_reduces_to_local(orc, dim):
    rng = np.random.default_rng(5)
    for n in (2, 3, 4, 5, 40):
        h = rng.integers(0, 1000, size=n - 1).astype(np.uint64)
        loc, _ = orc.action(h, n, dim, 0.0)
        sm, _ = orc.action(h, n, dim, 1.0)
        assert sm == loc
        pref = 2.0 if dim == 2 else C3 if dim == 3 else 4 / math.sqrt(6)
        assert loc == pytest.approx(pref * float(brute.local_integer(h, n, dim)), rel=1e-15)


def test_chain_and_antichain_actions(orc):
    for n in (5, 17, 200):
        chain = np.array([n - 1 - m for m in range(n - 1)], dtype=np.uint64)
        anti = np.zeros(n - 1, dtype=np.uint64)
        assert orc.action(chain, n, 2)[0] == 2 * n
        assert orc.action(anti, n, 2)[0] == 2 * n
        assert orc.action(anti, n, 4)[0] == pytest.approx(4 / math.sqrt(6) * n, rel=1e-16)
        # 2+1: chain bracket N - (N-1) + (27/8)(N-2) - (9/4)(N-3), antichain N
        assert orc.action(anti, n, 3)[0] == pytest.approx(C3 * n, rel=1e-15)
        br = 1 + Fraction(27, 8) * (n - 2) - Fraction(9, 4) * (n - 3)
        assert orc.action(chain, n, 3)[0] == pytest.approx(C3 * float(br), rel=1e-15)


def test_2p1_prefactor(orc):
    """(pi / (3 sqrt 2))^(2/3) / Gamma(5/3), against scipy's gamma."""
    assert orc.lib().or_c3_double() == pytest.approx(C3, rel=2e-16)


@pytest.mark.parametrize("dim", [2, 3, 4])
@pytest.mark.parametrize("eps", [0.05, 0.1, 0.2])
def test_smeared_action_exact_rational(orc, dim, eps):
    """2D: S = 2 eps * bracket is rational, so the double must be the correctly
    rounded exact value (to 1 ulp).  4D: bracket exact, prefactor 4 sqrt(eps/6)."""
    region = {2: W.MINK2_DIAMOND, 3: W.MINK3_DIAMOND, 4: W.MINK4_DIAMOND}[dim]
    n = 300
    c = orc.sprinkle(region, n, seed=51)
    h = orc.histogram_naive(orc.causal_matrix(region, c), n)
    s, kappa = orc.action(h, n, dim, eps)
    e = Fraction(eps)
    br = brute.smeared_bracket_exact(h, n, dim, e)
    if dim == 2:
        exact = float(2 * e * br)
        assert abs(s - exact) <= math.ulp(exact)
    else:
        pref = 4 * math.sqrt(eps / 6) if dim == 4 else C3 * eps ** (2.0 / 3.0)
        assert s == pytest.approx(pref * float(br), rel=4e-16 if dim == 4 else 1e-15)
    assert kappa >= 1.0


def test_action_rejects_bad_arguments(orc):
    h = np.zeros(3, dtype=np.uint64)
    for args in [(h, 4, 5, 0.0), (h, 4, 2, -0.1), (h, 4, 4, 1.5), (h, 1, 2, 0.0)]:
        with pytest.raises(ValueError):
            orc.action(*args)
