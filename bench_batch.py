"""Ensemble leg of bench.py: 256 independent 1+1 diamonds, N uniform in [512, 8192].

One HIP-graph launch of the batch pipeline (sprinkle, matrix, counts, actions for
every instance), with each of the three counters, against the same 256 instances as
separate per-instance calls of the single-instance entry points (int8 counter, and
again with the fp4 counter).  All are timed with HIP events on one stream.
"""
from __future__ import annotations

import os
import tempfile
import time

import numpy as np

import workloads as W


def run_batch(cs, torch, dev, stream, reps: int = 5):
    cfg = W.WORKLOADS["batch_mink2_256"]
    sizes, seeds = W.batch_instances(cfg["seed"], cfg["count"], cfg["nmin"], cfg["nmax"])
    eps = (0.0,) + tuple(cfg["eps"])
    count = len(sizes)

    tune = os.path.join(tempfile.gettempdir(), "cs_tune_gfx950.json")
    if os.path.exists(tune):
        os.remove(tune)
    t0 = time.perf_counter()
    cs.cs_autotune(tune, stream=stream)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    import json
    tuned = {}
    for e in json.load(open(tune))["entries"]:
        tuned.setdefault(e["counter"], []).append(
            {"n": [e["n_lo"], e["n_hi"]], "tile": e["tile"], "per_cu": e["per_cu"],
             **({"pair_max": e["pair_max"]} if e["counter"] == "bitset" else {}),
             "probe_ms": e["ms"], "probe": [e["probe_instances"], e["probe_n"]]})

    def ev():
        return torch.cuda.Event(enable_timing=True)

    out = {"instances": count, "n_range": [int(sizes.min()), int(sizes.max())],
           "autotune": {"seconds": tune_s, "choices": tuned}}
    results = {}
    # The fp4 counter also with 256x256 tiles (one workgroup per CU) for the instances of
    # 4096 points or more, the tuner's other candidate there, to show what its choice is
    # worth; a cache file of the tuner's format gives that configuration.
    alt = os.path.join(tempfile.gettempdir(), "cs_tune_fp4_tiles256.json")
    ent = [{"counter": "mfma_fp4", "n_lo": lo, "n_hi": hi, "mode": 4 if lo >= 4096 else 2,
            "tile": 256 if lo >= 4096 else 128, "per_cu": 1 if lo >= 4096 else 2,
            "pair_max": 0, "ms": 0.0}
           for lo, hi in ((2, 1023), (1024, 2047), (2048, 4095), (4096, 8192))]
    with open(alt, "w") as f:
        f.write('{\n  "format": "causal-batch-tune-2",\n  "entries": [\n'
                + ",\n".join("    " + json.dumps(e) for e in ent) + "\n  ]\n}\n")
    # each counter with the tuned tiles
    for name, counter, cache in (("mfma", cs.CS_COUNT_MFMA, tune),
                                 ("mfma_fp4", cs.CS_COUNT_MFMA_FP4, tune),
                                 ("bitset", cs.CS_COUNT_BITSET, tune),
                                 ("mfma_fp4_tiles256_from4096", cs.CS_COUNT_MFMA_FP4, alt)):
        plan = cs.BatchPlan(sizes, counter=counter, eps=eps, tune_cache=cache)
        s = torch.from_numpy(seeds.view(np.int64)).to(dev)
        hist = torch.empty(plan.hist_len, dtype=torch.int64, device=dev)
        acts = torch.empty(count * len(eps), dtype=torch.float64, device=dev)
        ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=dev)
        g = plan.graph(s, hist, acts, ws)
        for _ in range(2):
            g.launch(stream)
        times = []
        for _ in range(reps):
            a, b = ev(), ev()
            a.record(stream)
            g.launch(stream)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        results[name] = (hist.cpu().numpy().view(np.uint64).copy(), plan.offsets)
        out[f"graph_{name}_ms"] = min(times)
        out[f"graph_{name}_ensembles_per_s"] = count / (min(times) * 1e-3)
        out[f"graph_{name}_relations_per_s"] = float(
            results[name][0].sum()) / (min(times) * 1e-3)
        del g, plan

    # Per-instance baseline: the single-instance entry points, one instance at a time.
    nmax = int(sizes.max())
    ld = cs.cs_ld_words(nmax)
    L = cs.lib()
    coords = torch.empty(2 * nmax, dtype=torch.float64, device=dev)
    bits = torch.empty(nmax * ld, dtype=torch.int64, device=dev)
    hist1 = torch.empty(nmax, dtype=torch.int64, device=dev)
    acts1 = torch.empty(len(eps), dtype=torch.float64, device=dev)
    sp_ws = torch.empty(L.cs_sprinkle_workspace_bytes(0, nmax), dtype=torch.uint8, device=dev)
    h_ws = torch.empty(max(L.cs_histogram_workspace_bytes(nmax, c) for c in (1, 2)),
                       dtype=torch.uint8, device=dev)
    B = cs.binding
    last = {}

    def one_pass(counter, keep=False):
        for k in range(count):
            n = int(sizes[k])
            ldk = cs.cs_ld_words(n)
            B._check(L.cs_sprinkle(0, 1.2, int(seeds[k]), n, B._ptr(coords), B._ptr(sp_ws),
                                   sp_ws.numel(), B._stream(stream)), "sprinkle")
            B._check(L.cs_causal_matrix(0, B._ptr(coords), n, B._ptr(bits), ldk, B._stream(stream)),
                     "matrix")
            B._check(L.cs_interval_histogram(B._ptr(bits), n, ldk, counter, B._ptr(hist1), B._ptr(h_ws),
                                             h_ws.numel(), B._stream(stream)), "hist")
            for e, x in enumerate(eps):
                B._check(L.cs_action(B._ptr(hist1), n, 2, float(x),
                                     ctypes_ptr(acts1, e), B._stream(stream)), "action")
            if keep and k < 4:
                torch.cuda.synchronize()
                last[k] = hist1[:n - 1].cpu().numpy().view(np.uint64).copy()

    def timed_pass(counter):
        a, b = ev(), ev()
        a.record(stream)
        one_pass(counter)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    one_pass(cs.CS_COUNT_MFMA, keep=True)
    torch.cuda.synchronize()
    seq_ms = timed_pass(cs.CS_COUNT_MFMA)
    out["per_instance_ms"] = seq_ms
    out["per_instance_ensembles_per_s"] = count / (seq_ms * 1e-3)
    out["graph_vs_per_instance"] = seq_ms / out["graph_mfma_ms"]
    one_pass(cs.CS_COUNT_MFMA_FP4)
    seq4_ms = timed_pass(cs.CS_COUNT_MFMA_FP4)
    out["per_instance_fp4_ms"] = seq4_ms
    out["graph_fp4_vs_per_instance_fp4"] = seq4_ms / out["graph_mfma_fp4_ms"]
    hm, offs = results["mfma"]
    hb, _ = results["bitset"]
    out["mfma_equals_bitset"] = bool(np.array_equal(hm, hb))
    out["mfma_fp4_equals_bitset"] = bool(np.array_equal(results["mfma_fp4"][0], hb))
    out["per_instance_equals_graph"] = all(
        np.array_equal(last[k], hm[offs[k]:offs[k] + int(sizes[k]) - 1]) for k in last)
    return out


def ctypes_ptr(t, index):
    import ctypes
    return ctypes.c_void_p(t.data_ptr() + index * t.element_size())
