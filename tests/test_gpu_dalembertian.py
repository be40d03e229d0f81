"""GPU parity of the discrete d'Alembertian B^(d+1) phi (Sec. 4.1, eqs. b2d_local and
b4d_local) against the oracle, element by element.

The device accumulates each element's sum with fp64 atomics in a varying order, so the
bound per element is that of any summation order: (terms + 2) * 2^-52 * (sum of the
absolute summands) times K / ell^2, plus a few ulps for the prefactor.  Summand counts
and absolute sums come from the oracle.  Both MFMA counters, 1+1 and 3+1, sizes spanning
tiles with ragged tails; and the identity -ell^2 sum_j B1(j) = S_local at N = 16384.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K = {2: 2.0, 4: 4.0 / math.sqrt(6.0)}


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_04463_amd as cs
    cs.lib()
    return cs


def check(cs, orc, region, dim, n, seed, counter, ell=0.05):
    coords = orc.sprinkle(region, n, seed)
    bits = orc.causal_matrix(region, coords)
    phi = np.random.default_rng(seed).normal(size=n)
    want, terms, mag = orc.dalembertian(bits, n, dim, ell, phi)
    dev = torch.device("cuda")
    b = torch.from_numpy(bits.view(np.int64)).to(dev)
    got = cs.cs_dalembertian(b, n, dim, ell, torch.from_numpy(phi).to(dev), counter=counter)
    got = got.cpu().numpy()
    scale = K[dim] / ell ** 2
    bound = scale * (terms + 2) * 2.0 ** -52 * mag + 8 * 2.0 ** -52 * np.abs(want)
    err = np.abs(got - want)
    assert np.all(err <= bound), (n, counter, int(np.argmax(err / bound)), float(np.max(err / bound)))


@pytest.mark.parametrize("counter", [1, 2], ids=["mfma", "mfma_fp4"])
@pytest.mark.parametrize("n", [2, 3, 130, 700, 4097, 6000])
def test_dalembertian_1p1(cs, orc, n, counter):
    check(cs, orc, W.MINK2_DIAMOND, 2, n, 11 + n, counter)


@pytest.mark.parametrize("counter", [1, 2], ids=["mfma", "mfma_fp4"])
@pytest.mark.parametrize("n", [257, 4100])
def test_dalembertian_3p1(cs, orc, n, counter):
    check(cs, orc, W.MINK4_DIAMOND, 4, n, 12 + n, counter)


@pytest.mark.parametrize("region,dim", [(W.MINK2_DIAMOND, 2), (W.MINK4_DIAMOND, 4)])
def test_constant_field_gives_the_action(cs, region, dim):
    n, ell = 16384, 0.01
    c = cs.cs_sprinkle(region, n, 77)
    b = cs.cs_causal_matrix(region, c)
    h = cs.cs_interval_histogram(b, n, cs.CS_COUNT_MFMA_FP4)
    s_local = cs.cs_action(h, n, dim, 0.0).item()
    out = cs.cs_dalembertian(b, n, dim, ell, torch.ones(n, dtype=torch.float64, device="cuda"))
    total = -ell ** 2 * math.fsum(out.cpu().numpy())
    assert total == pytest.approx(s_local, rel=1e-9, abs=1e-6)


def test_n131072_sampled_elements(cs, orc):
    """At the bench size (3+1 diamond, N = 131072, fp4 tiles), B phi of sampled elements
    against the oracle's sums for those elements, within the summation-order bound; the
    device matrix is built from the oracle's coordinates, the oracle uses its own matrix."""
    cfg = W.WORKLOADS["mink4_n131072"]
    n, seed, ell = cfg["n"], cfg["seed"], 0.01
    coords = orc.sprinkle(W.MINK4_DIAMOND, n, seed)
    b = cs.cs_causal_matrix(W.MINK4_DIAMOND, torch.from_numpy(coords).cuda())
    phi = np.random.default_rng(73).normal(size=n)
    got = cs.cs_dalembertian(b, n, 4, ell, torch.from_numpy(phi).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    del b
    bits = orc.causal_matrix(W.MINK4_DIAMOND, coords)
    rng = np.random.default_rng(74)
    js = np.unique(np.concatenate([[0, 1, n // 2, n - 2, n - 1], rng.integers(0, n, 11)]))
    want, terms, mag = orc.dalembertian_cols(bits, n, 4, ell, phi, js)
    bound = K[4] / ell ** 2 * (terms + 2) * 2.0 ** -52 * mag + 8 * 2.0 ** -52 * np.abs(want)
    err = np.abs(got[js] - want)
    assert np.all(err <= bound), (js[np.argmax(err / bound)], float(np.max(err / bound)))
    assert terms.max() > 1
