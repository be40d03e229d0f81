"""The Python binding rejects mismatched tensors before any pointer crosses the ABI.

The library trusts the sizes it is handed (n, ld_words, buffer lengths), so a tensor
shorter than n implies would become an out-of-bounds device access.  Each case below
passes host tensors of the wrong shape or dtype and expects CausalError from the
binding's own checks, which run before the device check: no GPU is needed.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1805_04463_amd as cs
    from paper_1805_04463_amd import binding
    import os
    if not os.path.exists(binding.LIB_PATH):
        from paper_1805_04463_amd import build
        build.build()
    cs.lib()
    return cs


def words(rows, ld):
    return torch.zeros((rows, ld), dtype=torch.int64)


def raises(fn, match):
    from paper_1805_04463_amd import CausalError
    with pytest.raises(CausalError, match=match):
        fn()


def test_causal_matrix_checks_coords_and_out(cs):
    n = 1000
    ld = cs.cs_ld_words(n)
    raises(lambda: cs.cs_causal_matrix(1, torch.zeros((3, n), dtype=torch.float64)), "shape")
    raises(lambda: cs.cs_causal_matrix(1, torch.zeros((4, n), dtype=torch.float32)), "dtype")
    raises(lambda: cs.cs_causal_matrix(1, torch.zeros((4, n), dtype=torch.float64), n=n + 1),
           "shape")
    raises(lambda: cs.cs_causal_matrix(1, torch.zeros((4, n), dtype=torch.float64),
                                       out=words(n - 1, ld)), "shape")
    raises(lambda: cs.cs_causal_matrix(1, torch.zeros((4, n), dtype=torch.float64),
                                       ld_words=ld - 8), "ld_words")
    raises(lambda: cs.cs_causal_matrix(9, torch.zeros((4, n), dtype=torch.float64)), "region")
    # a well-formed host call gets as far as the device check
    raises(lambda: cs.cs_causal_matrix(1, torch.zeros((4, n), dtype=torch.float64),
                                       out=words(n, ld)), "device")


def test_histogram_checks_bits_out_and_workspace(cs):
    n = 1000
    ld = cs.cs_ld_words(n)
    raises(lambda: cs.cs_interval_histogram(words(n - 1, ld), n), "rows")
    raises(lambda: cs.cs_interval_histogram(words(n, ld - 8), n), "words per row")
    raises(lambda: cs.cs_interval_histogram(torch.zeros(n * ld, dtype=torch.int64), n), "2-D")
    raises(lambda: cs.cs_interval_histogram(words(n, ld).to(torch.float64), n), "dtype")
    raises(lambda: cs.cs_interval_histogram(words(n, ld), n,
                                            out=torch.zeros(n, dtype=torch.int64)), "elements")
    raises(lambda: cs.cs_interval_histogram(words(n, ld), n,
                                            out=torch.zeros(n - 1, dtype=torch.int32)), "dtype")
    raises(lambda: cs.cs_interval_histogram(words(n, ld), 1), "n = 1")
    raises(lambda: cs.cs_interval_histogram(words(n, ld), n, out=torch.zeros(n - 1, dtype=torch.int64),
                                            workspace=torch.zeros(16, dtype=torch.float32)),
           "dtype")


def test_action_checks_hist_and_out(cs):
    raises(lambda: cs.cs_action(torch.zeros(98, dtype=torch.int64), 100, 2), "at least 99")
    raises(lambda: cs.cs_action(torch.zeros(99, dtype=torch.float64), 100, 2), "dtype")
    raises(lambda: cs.cs_action(torch.zeros(99, dtype=torch.int64), 100, 2,
                                out=torch.zeros(0, dtype=torch.float64)), "at least 1")


def test_dalembertian_checks_phi_and_out(cs):
    n = 600
    b = words(n, cs.cs_ld_words(n))
    raises(lambda: cs.cs_dalembertian(b, n, 2, 0.1, torch.zeros(n - 1, dtype=torch.float64)),
           "phi")
    raises(lambda: cs.cs_dalembertian(b, n, 2, 0.1, torch.zeros(n, dtype=torch.float32)), "dtype")
    raises(lambda: cs.cs_dalembertian(b, n, 2, 0.1, torch.zeros(n, dtype=torch.float64),
                                      out=torch.zeros(n + 1, dtype=torch.float64)), "out")


def test_degrees_and_chains_check_bits(cs):
    n = 600
    raises(lambda: cs.cs_degrees(words(n - 5, cs.cs_ld_words(n)), n), "rows")
    b = words(n, cs.cs_ld_words(n))
    raises(lambda: cs.cs_longest_chain(b, n, [0, 1], [5]), "same length")
    raises(lambda: cs.cs_longest_chain(b, n, np.zeros((2, 2)), np.ones((2, 2))), "1-D")


def test_batch_buffers_checked_against_the_plan(cs):
    from paper_1805_04463_amd import BatchPlan
    plan = BatchPlan.__new__(BatchPlan)       # sizes only; no device plan is made
    plan.count, plan.hist_len, plan.eps, plan.handle = 3, 100, np.zeros(2), None
    seeds = torch.zeros(3, dtype=torch.int64)
    hist = torch.zeros(100, dtype=torch.int64)
    acts = torch.zeros(6, dtype=torch.float64)
    ws = torch.zeros(64, dtype=torch.uint8)
    raises(lambda: plan._buffers(torch.zeros(2, dtype=torch.int64), hist, acts, ws), "seeds")
    raises(lambda: plan._buffers(seeds, hist[:99], acts, ws), "hist")
    raises(lambda: plan._buffers(seeds, hist, acts[:5], ws), "actions")
    raises(lambda: plan._buffers(seeds, hist, acts.float(), ws), "dtype")
    raises(lambda: plan._buffers(seeds, hist, acts, ws), "device")
