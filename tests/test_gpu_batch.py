"""GPU parity of the ensemble path: per-instance N_n bit-exact and actions within 1e-12
of the oracle's pipeline on each instance; every counter with every tile configuration
the autotuner can choose, the HIP-graph replay, the tuner's cache, and the 256-instance
workload (sampled instances)."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [2, 3, 64, 100, 513, 1024, 2048, 3000, 4095, 4096, 5000, 8192]
EPS = (0.0, 0.1, 0.2)


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_04463_amd as cs
    cs.lib()
    return cs


def run_batch(cs, sizes, seeds, counter, tune_cache=None):
    plan = cs.BatchPlan(sizes, counter=counter, eps=EPS, tune_cache=tune_cache)
    dev = torch.device("cuda")
    s = torch.from_numpy(np.asarray(seeds, dtype=np.uint64).view(np.int64)).to(dev)
    hist = torch.empty(plan.hist_len, dtype=torch.int64, device=dev)
    acts = torch.empty(len(sizes) * len(EPS), dtype=torch.float64, device=dev)
    ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=dev)
    plan.run(s, hist, acts, ws)
    torch.cuda.synchronize()
    return plan, hist.cpu().numpy().view(np.uint64).copy(), acts.cpu().numpy().copy()


def check_instances(orc, plan, hist, acts, sizes, seeds, which):
    for k in which:
        n = int(sizes[k])
        _, _, h, a = orc.pipeline(W.MINK2_DIAMOND, n, int(seeds[k]), eps_list=EPS[1:], fast=True)
        off = plan.offsets[k]
        assert np.array_equal(hist[off:off + n - 1], h), (k, n)
        for e, eps in enumerate(EPS):
            got, want = acts[k * len(EPS) + e], a[eps]
            assert abs(got - want) <= 1e-12 * abs(want), (k, n, eps, got, want)


@pytest.mark.parametrize("counter", [0, 1, 2], ids=["bitset", "mfma", "mfma_fp4"])
def test_batch_mixed_sizes(cs, orc, counter):
    seeds = [1000 + 17 * k for k in range(len(SIZES))]
    plan, hist, acts = run_batch(cs, SIZES, seeds, counter)
    check_instances(orc, plan, hist, acts, SIZES, seeds, range(len(SIZES)))


# Every tile configuration the autotuner can choose: (mode, per_cu, pair_max).
MFMA_CHOICES = [(2, 2, 0), (2, 1, 0), (4, 1, 0)]
BITSET_CHOICES = [(0, 2, -1), (0, 2, 1152), (0, 2, 2304), (0, 1, 2304)]
BUCKETS = [(2, 1023), (1024, 2047), (2048, 4095), (4096, 8192)]
NAMES = {0: "bitset", 1: "mfma", 2: "mfma_fp4"}


def forced_cache(path, counter, choice):
    """A tuner cache whose entries give `choice` to every size bucket of `counter`."""
    mode, per_cu, pair_max = choice
    entries = [{"counter": NAMES[counter], "n_lo": lo, "n_hi": hi, "mode": mode,
                "tile": 256 if mode == 4 else 128, "per_cu": per_cu, "pair_max": pair_max,
                "ms": 1.0} for lo, hi in BUCKETS]
    path.write_text("{\n  \"format\": \"causal-batch-tune-2\",\n  \"entries\": [\n"
                    + ",\n".join("    " + json.dumps(e) for e in entries) + "\n  ]\n}\n")
    return str(path)


@pytest.mark.parametrize("counter,choice",
                         [(c, m) for c in (1, 2) for m in MFMA_CHOICES]
                         + [(0, m) for m in BITSET_CHOICES])
def test_batch_every_tuner_choice(cs, orc, tmp_path, counter, choice):
    cache = forced_cache(tmp_path / "tune.json", counter, choice)
    sizes = [2, 130, 700, 1024, 2500, 4100, 8000, 8192]
    seeds = [77, 78, 79, 80, 81, 82, 83, 84]
    plan, hist, acts = run_batch(cs, sizes, seeds, counter, tune_cache=cache)
    check_instances(orc, plan, hist, acts, sizes, seeds, range(len(sizes)))


# Seeds whose 8192-point diamonds hold two points with equal top 32 bits of the 54-bit time
# key (u + v) * 2^53: the ensemble sprinkle sorts on those bits and orders such ties by the
# whole key afterwards.  (Found by scanning the oracle's sprinklings; checked below.)
TIED_SEEDS = (5057, 5363)


def _tied_top_bits(coords):
    key = (np.round(coords[0] * 2.0**53).astype(np.uint64)
           + np.round(coords[1] * 2.0**53).astype(np.uint64))
    top = (key >> np.uint64(22)).astype(np.int64)
    return bool(np.any(np.diff(top) == 0))


def test_batch_coords_and_matrices_bit_exact(cs, orc):
    """Every instance's time-ordered coordinates and packed matrix, read from the workspace
    after a run, equal the oracle's bit for bit (the histogram alone would not see two
    spacelike points swapped): mixed sizes, the two builder item shapes (above and on the
    diagonal), and instances whose time keys tie in their top bits."""
    sizes = [8192, 3000, 2, 8192, 513, 64, 4097, 65]
    seeds = [TIED_SEEDS[0], 11, 12, TIED_SEEDS[1], 13, 14, 15, 16]
    plan = cs.BatchPlan(sizes, counter=2, eps=EPS)
    dev = torch.device("cuda")
    s = torch.from_numpy(np.asarray(seeds, dtype=np.uint64).view(np.int64)).to(dev)
    hist = torch.empty(plan.hist_len, dtype=torch.int64, device=dev)
    acts = torch.empty(len(sizes) * len(EPS), dtype=torch.float64, device=dev)
    ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=dev)
    plan.run(s, hist, acts, ws)
    torch.cuda.synchronize()
    host = ws.cpu().numpy()
    for k, (n, seed) in enumerate(zip(sizes, seeds)):
        want_c = orc.sprinkle(W.MINK2_DIAMOND, n, seed)
        if seed in TIED_SEEDS:
            assert _tied_top_bits(want_c), seed
        co = plan.coords_offsets[k]
        got_c = host[co:co + 16 * n].view(np.float64).reshape(2, n)
        assert np.array_equal(got_c.view(np.uint64), want_c.view(np.uint64)), (k, n)
        ld = cs.cs_ld_words(n)
        bo = plan.bits_offsets[k]
        got_b = host[bo:bo + 8 * n * ld].view(np.uint64).reshape(n, ld)
        want_b = orc.causal_matrix(W.MINK2_DIAMOND, want_c, ld=ld)
        assert np.array_equal(got_b, want_b), (k, n)


@pytest.mark.parametrize("counter", [1, 2], ids=["mfma", "mfma_fp4"])
def test_batch_graph_replays(cs, orc, counter):
    sizes = [300, 1500, 4200, 6000, 999]
    seeds = [5, 6, 7, 8, 9]
    dev = torch.device("cuda")
    plan = cs.BatchPlan(sizes, counter=counter, eps=EPS)
    s = torch.from_numpy(np.asarray(seeds, dtype=np.uint64).view(np.int64)).to(dev)
    hist = torch.empty(plan.hist_len, dtype=torch.int64, device=dev)
    acts = torch.empty(len(sizes) * len(EPS), dtype=torch.float64, device=dev)
    ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=dev)
    plan.run(s, hist, acts, ws)
    torch.cuda.synchronize()
    h0, a0 = hist.clone(), acts.clone()
    g = plan.graph(s, hist, acts, ws)
    for rep in range(4):
        hist.fill_(-1)
        acts.fill_(float("nan"))
        x = torch.randn(1024, device=dev).sum()  # eager work between replays
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(hist, h0), rep
        assert torch.equal(acts, a0), rep
        del x
    check_instances(orc, plan, h0.cpu().numpy().view(np.uint64), a0.cpu().numpy(), sizes, seeds,
                    range(len(sizes)))


@pytest.mark.parametrize("counter", [1, 2], ids=["mfma", "mfma_fp4"])
def test_batch_workload_256(cs, orc, counter):
    cfg = W.WORKLOADS["batch_mink2_256"]
    sizes, seeds = W.batch_instances(cfg["seed"], cfg["count"], cfg["nmin"], cfg["nmax"])
    plan, hist, acts = run_batch(cs, sizes, seeds, counter)
    rng = np.random.default_rng(0)
    which = sorted(set(rng.choice(len(sizes), 6, replace=False).tolist()
                       + [int(np.argmax(sizes)), int(np.argmin(sizes))]))
    check_instances(orc, plan, hist, acts, sizes, seeds, which)
    # every instance: ordering fraction 1/2 within 6 standard deviations (sd ~ 1/sqrt(n)/3)
    for k, n in enumerate(sizes):
        off = plan.offsets[k]
        R = int(hist[off:off + n - 1].sum())
        assert abs(R / (n * (n - 1) / 2) - 0.5) < 6 * 0.6 / np.sqrt(n), (k, n, R)


def test_batch_workload_256_counters_agree(cs):
    """All 256 instances: the bitset, int8 and fp4 counters give the same histograms, so
    the same actions (three independent ways of counting every pair)."""
    cfg = W.WORKLOADS["batch_mink2_256"]
    sizes, seeds = W.batch_instances(cfg["seed"], cfg["count"], cfg["nmin"], cfg["nmax"])
    runs = [run_batch(cs, sizes, seeds, c) for c in (0, 1, 2)]
    (_, h0, a0), (_, h1, a1), (_, h2, a2) = runs
    assert np.array_equal(h0, h1) and np.array_equal(h0, h2)
    assert np.array_equal(a0, a1) and np.array_equal(a0, a2)
    assert int(h0.sum()) > 0


def test_autotune_writes_cache(cs, orc, tmp_path):
    """Every (counter, bucket) gets an entry naming one of its candidates; tuning one
    counter and bucket again keeps the other entries; a plan reads the cache."""
    path = tmp_path / "tune.json"
    cs.cs_autotune(str(path))
    torch.cuda.synchronize()
    d = json.loads(path.read_text())
    got = {(e["counter"], e["n_lo"]): e for e in d["entries"]}
    for c, choices in ((0, BITSET_CHOICES), (1, MFMA_CHOICES), (2, MFMA_CHOICES)):
        for lo, hi in BUCKETS:
            e = got[(NAMES[c], lo)]
            assert (e["mode"], e["per_cu"], e["pair_max"]) in choices
            assert e["n_hi"] == hi and e["ms"] > 0
    before = path.read_text()
    cs.cs_autotune(str(path), n_bucket=3000, counter=cs.CS_COUNT_MFMA_FP4)
    torch.cuda.synchronize()
    d2 = json.loads(path.read_text())
    assert len(d2["entries"]) == len(d["entries"])
    same = [e for e in d2["entries"] if not (e["counter"] == "mfma_fp4" and e["n_lo"] == 2048)]
    assert all(e in d["entries"] for e in same), before
    sizes, seeds = [700, 3000, 6000], [1, 2, 3]
    for c in (0, 1, 2):
        plan, hist, acts = run_batch(cs, sizes, seeds, c, tune_cache=str(path))
        check_instances(orc, plan, hist, acts, sizes, seeds, range(len(sizes)))

