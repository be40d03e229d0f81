"""GPU test of cs_interval_histogram_noalloc, the allocation-free variant of the
interval-abundance call (its scratch is the library's static device array).

Two calls in a row on the same device -- the second on a smaller matrix, so the array
holds the first call's counters when the second starts -- are checked bin by bin against
cs_interval_histogram with a caller workspace, and against the oracle's counts of the
same matrix built from the oracle's own coordinates."""
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
    return t.cpu().numpy().view(np.uint64).copy()


@pytest.mark.parametrize("counter", [1, 2, 0, 3], ids=["int8", "fp4", "bitset", "bitset_dense"])
def test_noalloc_matches_workspace_call(cs, orc, counter):
    cases = [(W.MINK4_DIAMOND, 5000, 31), (W.MINK2_DIAMOND, 1300, 32)]  # larger, then smaller
    for region, n, seed in cases:
        print(f"noalloc counter={counter} region={region} n={n} seed={seed}", flush=True)
        coords = orc.sprinkle(region, n, seed)
        want = orc.histogram_fast(orc.causal_matrix(region, coords), n)[0]
        b = cs.cs_causal_matrix(region, torch.from_numpy(coords).cuda())
        ref = host_u64(cs.cs_interval_histogram(b, n, counter))
        out = torch.full((n - 1,), -1, dtype=torch.int64, device="cuda")
        got = host_u64(cs.cs_interval_histogram_noalloc(b, n, out, counter))
        assert np.array_equal(got, ref), (region, n)
        assert np.array_equal(got, want), (region, n)
        # a second call on the same matrix reuses the scratch left by the first
        got2 = host_u64(cs.cs_interval_histogram_noalloc(b, n, out, counter))
        assert np.array_equal(got2, want), (region, n)
