"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact for coordinates of the Minkowski sprinklings, the causal matrix and N_n;
|S_gpu - S_oracle| <= 1e-12 |S_oracle| for the actions.  Inputs flow from the oracle to
the GPU, never back: the matrix and counters are fed the oracle's coordinates and
matrices.  Sizes span several tiles and ragged tails of both counters (128- and
256-wide output tiles, 64-wide builder blocks, 512-bit row padding).
"""
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


def dev_u64(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def host_u64(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def ulps(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.max(np.abs(a - b) / np.spacing(np.maximum(np.abs(a), np.abs(b))))


REGIONS = [W.MINK2_DIAMOND, W.MINK4_DIAMOND, W.DS4_SLAB]


# 8192 is the largest set ordered by rank placement, 8193 the smallest ordered by the sort
# network and gather; 2047-2049 straddle the network's LDS chunk.
@pytest.mark.parametrize("region", [W.MINK2_DIAMOND, W.MINK4_DIAMOND, W.MINK3_DIAMOND])
@pytest.mark.parametrize("n", [2, 3, 100, 2047, 2048, 2049, 5000, 8192, 8193])
def test_sprinkle_minkowski_bit_exact(cs, orc, region, n):
    want = orc.sprinkle(region, n, seed=1000 + n)
    got = cs.cs_sprinkle(region, n, seed=1000 + n).cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", [2, 777, 4096])
def test_sprinkle_ds_within_ulps(cs, orc, n):
    want = orc.sprinkle(W.DS4_SLAB, n, seed=77 + n, eta0=W.DS_ETA0)
    got = cs.cs_sprinkle(W.DS4_SLAB, n, seed=77 + n, eta0=W.DS_ETA0).cpu().numpy()
    assert ulps(got[0], want[0]) <= 8       # tan(eta): sinh/asinh of two libms
    assert ulps(got[1:3], want[1:3]) <= 8   # cos, sin from it
    assert np.array_equal(got[3:], want[3:])  # S^3 direction: exact operations only


@pytest.mark.parametrize("region", REGIONS)
@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 130, 511, 513, 1024, 1537, 2111])
def test_causal_matrix_bit_exact(cs, orc, region, n):
    coords = orc.sprinkle(region, n, seed=500 + n)
    want = orc.causal_matrix(region, coords)
    got = host_u64(cs.cs_causal_matrix(region, torch.from_numpy(coords).cuda()))
    assert got.shape == want.shape
    assert np.array_equal(got, want)


ALL_REGIONS = [(W.MINK2_DIAMOND, 1.2), (W.MINK4_DIAMOND, 1.2), (W.DS4_SLAB, W.DS_ETA0),
               (W.DS2_SLAB, W.DS2_ETA0), (W.MINK3_DIAMOND, 1.2)]


@pytest.mark.parametrize("region,eta0", ALL_REGIONS, ids=["mink2", "mink4", "ds4", "ds2", "mink3"])
@pytest.mark.parametrize("n", [3073, 5000, 9999])
def test_causal_matrix_patches_bit_exact(cs, orc, region, eta0, n):
    """Sizes with 8 or more 1024-point patches (dealt over the XCDs) and a ragged last block,
    in every region (the diamonds' column points come through scalar loads)."""
    coords = orc.sprinkle(region, n, seed=700 + n, eta0=eta0)
    want = orc.causal_matrix(region, coords)
    got = host_u64(cs.cs_causal_matrix(region, torch.from_numpy(coords).cuda()))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("region", [W.MINK4_DIAMOND, W.MINK3_DIAMOND], ids=["mink4", "mink3"])
def test_causal_matrix_ties_and_null_pairs(cs, orc, region):
    """Time-ordered points with runs of equal times and exactly null (dyadic) separations,
    over several 64-point blocks: the device builder, which takes t_j >= t_i as given and
    tests dt * dt > |dx|^2 alone, matches the oracle's dt > 0 and dt * dt > |dx|^2."""
    rng = np.random.default_rng(11)
    n = 300
    planes = 4 if region == W.MINK4_DIAMOND else 3
    # times on a coarse dyadic grid (many ties), space offsets on a dyadic grid too, so
    # that dt^2 and |dx|^2 are exact and many pairs sit exactly on the light cone
    t = np.sort(rng.integers(0, 16, n)).astype(np.float64) / 16.0
    x = rng.integers(-8, 9, (planes - 1, n)).astype(np.float64) / 16.0
    t[1], x[:, 1] = t[0], x[:, 0]  # one coincident pair
    coords = np.ascontiguousarray(np.vstack([t[None, :], x]))
    want = orc.causal_matrix(region, coords)
    got = host_u64(cs.cs_causal_matrix(region, torch.from_numpy(coords).cuda()))
    assert np.array_equal(got, want)
    # the case is not vacuous: null pairs exist, and related and unrelated pairs both occur
    dt = t[None, :] - t[:, None]
    d2 = sum((x[p][None, :] - x[p][:, None]) ** 2 for p in range(planes - 1))
    iu = np.triu_indices(n, 1)
    assert (dt[iu] ** 2 == d2[iu]).sum() > 100 and (dt[iu] == 0).sum() > 100
    assert ((dt[iu] == 0) & (d2[iu] == 0)).sum() > 0
    assert 0 < int(np.bitwise_count(want).sum()) < n * (n - 1)


def test_causal_matrix_wider_stride(cs, orc):
    n = 300
    coords = orc.sprinkle(W.MINK4_DIAMOND, n, seed=3)
    want = orc.causal_matrix(W.MINK4_DIAMOND, coords, ld=24)
    got = host_u64(cs.cs_causal_matrix(W.MINK4_DIAMOND, torch.from_numpy(coords).cuda(),
                                       ld_words=24))
    assert np.array_equal(got, want)


COUNT_CASES = [(W.MINK2_DIAMOND, n) for n in (2, 3, 5, 64, 129, 255, 256, 257, 700, 1024, 3001)] + \
              [(W.MINK4_DIAMOND, n) for n in (2, 100, 511, 1500, 4095, 4097, 5000)] + \
              [(W.DS4_SLAB, n) for n in (3, 600, 2500, 4100)]


@pytest.mark.parametrize("counter", [0, 1, 2, 3], ids=["bitset", "mfma", "mfma_fp4", "bitset_dense"])
@pytest.mark.parametrize("region,n", COUNT_CASES)
def test_interval_histogram_bit_exact(cs, orc, counter, region, n):
    coords = orc.sprinkle(region, n, seed=900 + n)
    bits = orc.causal_matrix(region, coords)
    want = orc.histogram_naive(bits, n) if n <= 1500 else orc.histogram_fast(bits, n)[0]
    got = host_u64(cs.cs_interval_histogram(dev_u64(bits), n, counter))
    assert np.array_equal(got, want)


def test_action_every_bin_filled(cs, orc):
    """Counts in every bin up to n - 2, so the smeared sums run into the bins where the
    weights (1 - eps)^m have underflowed (the kernel stops its walk there)."""
    rng = np.random.default_rng(10)
    n = 131072
    hist = rng.integers(0, 10**9, size=n - 1, dtype=np.uint64)
    for dim in (2, 3, 4):
        for eps in (2.0**-6, 0.05, 0.5, 0.9, 1.0):
            want, _ = orc.action(hist, n, dim, eps)
            got = cs.cs_action(dev_u64(hist), n, dim, eps).item()
            assert abs(got - want) <= 1e-12 * abs(want), (dim, eps, got, want)


@pytest.mark.parametrize("counter", [0, 1, 2, 3], ids=["bitset", "mfma", "mfma_fp4", "bitset_dense"])
@pytest.mark.parametrize("n", [2, 65, 300, 4500])
def test_chain_and_antichain_counts(cs, orc, counter, n):
    k = np.arange(1, n + 1, dtype=np.float64) / (n + 1)
    chain = orc.causal_matrix(W.MINK2_DIAMOND, np.stack([k, k]))
    got = host_u64(cs.cs_interval_histogram(dev_u64(chain), n, counter))
    assert np.array_equal(got, np.arange(n - 1, 0, -1, dtype=np.uint64))  # N_m = n-1-m
    anti = np.zeros((n, orc.ld_words(n)), dtype=np.uint64)
    got = host_u64(cs.cs_interval_histogram(dev_u64(anti), n, counter))
    assert not got.any()


def test_counters_deterministic(cs, orc):
    n = 3000
    bits = dev_u64(orc.causal_matrix(W.MINK4_DIAMOND, orc.sprinkle(W.MINK4_DIAMOND, n, seed=8)))
    a = host_u64(cs.cs_interval_histogram(bits, n, 1)).copy()
    b = host_u64(cs.cs_interval_histogram(bits, n, 1)).copy()
    c = host_u64(cs.cs_interval_histogram(bits, n, 0)).copy()
    d = host_u64(cs.cs_interval_histogram(bits, n, 2)).copy()
    e = host_u64(cs.cs_interval_histogram(bits, n, 3)).copy()
    assert np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d)
    assert np.array_equal(a, e)


@pytest.mark.parametrize("dim", [2, 4])
@pytest.mark.parametrize("eps", [0.0, 0.05, 0.1, 0.2, 2.0**-6, 1.0])
def test_action_within_1e12(cs, orc, dim, eps):
    region = W.MINK2_DIAMOND if dim == 2 else W.MINK4_DIAMOND
    for n, seed in ((2, 1), (4, 2), (700, 3), (3000, 4)):
        bits = orc.causal_matrix(region, orc.sprinkle(region, n, seed=seed))
        hist = orc.histogram_fast(bits, n)[0]
        want, kappa = orc.action(hist, n, dim, eps)
        got = cs.cs_action(dev_u64(hist), n, dim, eps).item()
        assert abs(got - want) <= 1e-12 * abs(want), (n, got, want, kappa)


def test_action_synthetic_histograms(cs, orc):
    rng = np.random.default_rng(9)
    for n in (5, 1000, 20000, 131072):
        hist = np.zeros(n - 1, dtype=np.uint64)
        hist[: min(n - 1, 4000)] = rng.integers(0, 10**9, size=min(n - 1, 4000), dtype=np.uint64)
        for dim in (2, 4):
            for eps in (0.0, 0.05, 0.1, 0.2, 0.7):
                want, _ = orc.action(hist, n, dim, eps)
                got = cs.cs_action(dev_u64(hist), n, dim, eps).item()
                assert abs(got - want) <= 1e-12 * abs(want), (n, dim, eps, got, want)


@pytest.mark.parametrize("counter", [0, 1, 2, 3], ids=["bitset", "mfma", "mfma_fp4", "bitset_dense"])
def test_pipeline_mink2_n1024(cs, orc, counter):
    """Whole path from the seed on the GPU against the whole path on the CPU."""
    cfg = W.WORKLOADS["mink2_n1024"]
    n, seed = cfg["n"], cfg["seed"]
    coords, bits, hist, acts = orc.pipeline(W.MINK2_DIAMOND, n, seed, eps_list=cfg["eps"])
    c = cs.cs_sprinkle(W.MINK2_DIAMOND, n, seed)
    b = cs.cs_causal_matrix(W.MINK2_DIAMOND, c)
    h = cs.cs_interval_histogram(b, n, counter)
    assert np.array_equal(host_u64(b), bits)
    assert np.array_equal(host_u64(h), hist)
    for eps, want in acts.items():
        got = cs.cs_action(h, n, 2, eps).item()
        assert abs(got - want) <= 1e-12 * abs(want)


def test_measured_mfma_peaks_are_plausible(cs):
    int8 = cs.cs_measure_mfma_peak(cs.CS_COUNT_MFMA)
    fp4 = cs.cs_measure_mfma_peak(cs.CS_COUNT_MFMA_FP4)
    assert 1000 < int8 < 5100      # TOP/s; published dense int8 peak 5000
    assert 2000 < fp4 < 10300      # published dense fp4 peak 10100
