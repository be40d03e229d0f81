"""The mean number of isolated elements of the 1+1 de Sitter slab (App. A, "Isolated
Elements in de Sitter Spacetime"), as a pin of the oracle's slab sprinkle and relation.

The appendix takes the slab eta in [0, eta0] with density sec^2(eta) / tan(eta0) on it.
An element at eta is isolated when no other element falls in its past or future light
cone inside the slab, of volume (in units of the de Sitter radius squared)
  V(eta) = 2 [(eta0 - eta) tan(eta0) + ln sec^2(eta) - ln sec(eta0)]
(the appendix's exponent of P(0)), against the slab's volume 2 pi tan(eta0).  With a fixed
number M of elements, uniform by volume, the other M - 1 avoid both cones with probability
(1 - V / (2 pi tan eta0))^(M - 1), so
  E[N_0 | M] = M int_0^eta0 sec^2(eta) / tan(eta0) (1 - V(eta) / (2 pi tan eta0))^(M-1) d eta,
the appendix's N int rho P(0) d eta for a fixed-size sprinkle, by quadrature.

The oracle sprinkles the symmetric slab [-eta0, eta0]; its elements with eta >= 0 are a
uniform sprinkle of the appendix's slab (their number M is binomial), and with labels in
time order they are the last n - m elements, whose induced order is the causal set of
[0, eta0].  Over many seeds the isolated elements of that sub-order are counted and
compared with sum_s E[N_0 | M_s].  On the wide slab (eta0 = 1.4) a sprinkle uniform in
eta instead of tan(eta) would miss it by many standard errors (checked below).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W


def cone_fraction(eta, eta0):
    v = 2 * ((eta0 - eta) * math.tan(eta0) + 2 * math.log(1 / math.cos(eta))
             - math.log(1 / math.cos(eta0)))
    return v / (2 * math.pi * math.tan(eta0))


def expected_isolated(m, eta0, density=None):
    """E[N_0 | M = m] on [0, eta0]; density defaults to sec^2(eta) / tan(eta0)."""
    if m < 1:
        return 0.0
    rho = density or (lambda e: 1.0 / (math.cos(e) ** 2 * math.tan(eta0)))
    val, _ = integrate.quad(lambda e: rho(e) * (1 - cone_fraction(e, eta0)) ** (m - 1),
                            0.0, eta0, epsabs=1e-13, epsrel=1e-12)
    return m * val


def isolated_upper_half(orc, n, seed, eta0):
    """(M, isolated elements of the order induced on the elements with eta >= 0)."""
    c = orc.sprinkle(W.DS2_SLAB, n, seed, eta0=eta0)
    m = int(np.searchsorted(c[0], 0.0))      # first element with tan(eta) >= 0
    bits = orc.causal_matrix(W.DS2_SLAB, c)
    S = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)
    sub = S[m:, m:]
    return n - m, int((~sub.any(axis=1)).sum())


@pytest.mark.parametrize("eta0,n,seeds,power", [(W.DS2_ETA0, 64, 2500, False),
                                                (1.4, 48, 3000, True)])
def test_mean_isolated_elements(orc, eta0, n, seeds, power):
    """power: also require the uniform-in-eta alternative to be rejected (on [0, 1/2]
    sec^2 is nearly constant and the two densities give the same count)."""
    seeds = range(5000, 5000 + seeds)
    got, want, wrong = [], [], []
    cache, cache_wrong = {}, {}
    # sprinkle uniform in eta on [0, eta0] instead of in tan(eta): must be rejected
    uniform_eta = lambda e: 1.0 / eta0
    for s in seeds:
        m, k = isolated_upper_half(orc, n, s, eta0)
        if m not in cache:
            cache[m] = expected_isolated(m, eta0)
            cache_wrong[m] = expected_isolated(m, eta0, uniform_eta)
        got.append(k)
        want.append(cache[m])
        wrong.append(cache_wrong[m])
    got, want, wrong = map(np.asarray, (got, want, wrong))
    resid = got - want
    se = resid.std(ddof=1) / math.sqrt(len(resid))
    assert want.mean() > 0.3                     # enough isolated elements to test
    assert abs(resid.mean()) < 4 * se, (got.mean(), want.mean(), se)
    if power:
        assert abs((got - wrong).mean()) > 8 * se, (got.mean(), wrong.mean(), se)


def test_cone_volume_closed_form():
    """The appendix's cone volume against direct integration of the cone's width 2|d eta|
    times the volume density sec^2(eta') over the slab."""
    eta0 = 1.1
    for eta in (0.0, 0.3, 0.77, 1.05):
        past, _ = integrate.quad(lambda e: 2 * (eta - e) / math.cos(e) ** 2, 0.0, eta)
        fut, _ = integrate.quad(lambda e: 2 * (e - eta) / math.cos(e) ** 2, eta, eta0)
        assert (past + fut) / (2 * math.pi * math.tan(eta0)) == pytest.approx(
            cone_fraction(eta, eta0), rel=1e-10)
