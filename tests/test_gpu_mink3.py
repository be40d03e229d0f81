"""GPU parity on the 2+1 Minkowski diamond (Sec. 4.2's 2+1 action, eqs. s3d_local and
f_3; App. A's 2+1 diamond, sampled by rejection like the 3+1 one).  The sprinkle uses exact
operations only, so the whole path is bit-exact from the seed: coordinates, matrix, N_n for
every counter; actions agree to 1e-12 (local, smeared, and eps = 1, which equals the
local action); the d'Alembertian B^(2+1) within the summation-order bound."""
import math

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


def host_u64(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("n", [2, 3, 257, 1000, 5003])
def test_mink3_sprinkle_and_matrix(cs, orc, n):
    want = orc.sprinkle(W.MINK3_DIAMOND, n, 31 + n)
    c = cs.cs_sprinkle(W.MINK3_DIAMOND, n, 31 + n)
    assert np.array_equal(c.cpu().numpy(), want)
    b = cs.cs_causal_matrix(W.MINK3_DIAMOND, c)
    assert np.array_equal(host_u64(b), orc.causal_matrix(W.MINK3_DIAMOND, want))


def test_mink3_n16384_whole_path(cs, orc):
    cfg = W.WORKLOADS["mink3_n16384"]
    n, seed = cfg["n"], cfg["seed"]
    eps_list = tuple(cfg["eps"]) + (1.0,)
    coords, bits, hist, acts = orc.pipeline(W.MINK3_DIAMOND, n, seed, eps_list=eps_list, fast=True)
    c = cs.cs_sprinkle(W.MINK3_DIAMOND, n, seed)
    assert np.array_equal(c.cpu().numpy(), coords)
    b = cs.cs_causal_matrix(W.MINK3_DIAMOND, c)
    assert np.array_equal(host_u64(b), bits)
    local = orc.action(hist, n, 3, 0.0)[0]
    for counter in (cs.CS_COUNT_MFMA, cs.CS_COUNT_BITSET, cs.CS_COUNT_MFMA_FP4):
        h = cs.cs_interval_histogram(b, n, counter)
        assert np.array_equal(host_u64(h), hist), counter
        got = cs.cs_action(h, n, 3, 0.0).item()
        assert abs(got - local) <= 1e-12 * abs(local)
        for eps, want in acts.items():
            got = cs.cs_action(h, n, 3, eps).item()
            assert abs(got - want) <= 1e-12 * abs(want), (counter, eps, got, want)
    assert acts[1.0] == pytest.approx(local, rel=1e-14)


def test_mink3_dalembertian(cs, orc):
    n, ell, dim = 3000, 0.05, 3
    coords = orc.sprinkle(W.MINK3_DIAMOND, n, 41)
    bits = orc.causal_matrix(W.MINK3_DIAMOND, coords)
    phi = np.random.default_rng(41).normal(size=n)
    want, terms, mag = orc.dalembertian(bits, n, dim, ell, phi)
    b = torch.from_numpy(bits.view(np.int64)).cuda()
    got = cs.cs_dalembertian(b, n, dim, ell, torch.from_numpy(phi).cuda()).cpu().numpy()
    k = (math.pi / (3 * math.sqrt(2))) ** (2 / 3) / math.gamma(5 / 3)
    bound = k / ell ** 2 * (terms + 2) * 2.0 ** -52 * mag + 8 * 2.0 ** -52 * np.abs(want)
    assert np.all(np.abs(got - want) <= bound)


def test_mink3_n131072(cs, orc):
    """The 2+1 bench leg's size: coordinates and the whole matrix bit-exact against the
    oracle's; N_n of the int8, fp4 and bitset counters bin by bin against the stored oracle
    abundances; actions against the oracle's actions of those abundances."""
    from test_gpu_fullsize import fullsize_parity
    fullsize_parity(cs, orc, "mink3_n131072",
                    (cs.CS_COUNT_MFMA_FP4, cs.CS_COUNT_MFMA, cs.CS_COUNT_BITSET))
