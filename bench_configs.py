"""Per-configuration leg of bench.py: the three smaller workloads of the benchmark set, each
the whole path (sprinkle, matrix, counter, local and smeared actions) on device buffers
allocated beforehand, timed by the thesis's protocol (Sec. 4.4: three warm-up runs, then
the minimum of the next five).

  mink2_n1024   1+1 diamond, N = 1024: latency-bound, reported in microseconds end to end
                (host clock around one synchronised pass), eagerly and as one HIP-graph
                replay of the same pass
  mink4_n16384  3+1 diamond, N = 16384
  ds4_n65536    3+1 de Sitter slab, N = 65536
For the two larger ones: the step time, and the fp4 and int8 counters' kernel times (HIP
events on the launch stream) with their fraction of the dense MFMA peak on the useful
work 2 N(N-1)(N-2)/6.

Beside each, the CPU oracle on the host cores (no GPU result enters it):
  mink2_n1024   the whole path with the definitional tier of the count
  mink4_n16384  the definitional tier over a sample of elements j (all pairs i ≺ j)
  ds4_n65536    the optimised tier over the whole matrix, run once (not repeated)
and the GPU/oracle ratio of related-pair counts per second.
"""
from __future__ import annotations

import time

import numpy as np

import workloads as W

PEAK_INT8_OPS = 5.0e15
PEAK_FP4_OPS = 10.1e15
FP4, INT8 = 2, 1


def _timed(fn, sync, warm=3, runs=5):
    """Thesis protocol: `warm` untimed runs, then the minimum of `runs` timed ones
    (host clock, each run bracketed by a synchronisation)."""
    for _ in range(warm):
        fn()
    sync()
    t = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        sync()
        t.append(time.perf_counter() - t0)
    return min(t), float(np.median(t))


def _counter_ms(cs, torch, stream, bits, n, counter, hist, ws, warm=3, runs=5):
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(runs)]
    for _ in range(warm):
        cs.cs_interval_histogram(bits, n, counter, out=hist, workspace=ws, stream=stream)
    for a, b in ev:
        a.record(stream)
        cs.cs_interval_histogram(bits, n, counter, out=hist, workspace=ws, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    return min(a.elapsed_time(b) for a, b in ev)


def run_config(cs, torch, dev, stream, name, cpu=True, cpu_seconds=8.0):
    cfg = W.WORKLOADS[name]
    region, n, seed, eps_list = cfg["region"], cfg["n"], cfg["seed"], tuple(cfg["eps"])
    dim = W.REGION_DIM[region]
    eta0 = cfg.get("eta0", W.DS_ETA0)
    L = cs.lib()
    ld = cs.cs_ld_words(n)
    coords = torch.empty((cs.cs_coord_planes(region), n), dtype=torch.float64, device=dev)
    bits = torch.empty((n, ld), dtype=torch.int64, device=dev)
    hist = torch.empty(n - 1, dtype=torch.int64, device=dev)
    acts = torch.empty(1 + len(eps_list), dtype=torch.float64, device=dev)
    sp_ws = torch.empty(L.cs_sprinkle_workspace_bytes(region, n), dtype=torch.uint8, device=dev)
    h_ws = torch.empty(max(L.cs_histogram_workspace_bytes(n, c) for c in (FP4, INT8)),
                       dtype=torch.uint8, device=dev)

    def step(counter=FP4, st=None):
        st = stream if st is None else st
        cs.binding._check(L.cs_sprinkle(region, eta0, seed, n, cs.binding._ptr(coords),
                                        cs.binding._ptr(sp_ws), sp_ws.numel(),
                                        cs.binding._stream(st)), "sprinkle")
        cs.cs_causal_matrix(region, coords, n, ld, out=bits, stream=st)
        cs.cs_interval_histogram(bits, n, counter, out=hist, workspace=h_ws, stream=st)
        cs.cs_action(hist, n, dim, 0.0, out=acts[0:1], stream=st)
        for k, e in enumerate(eps_list):
            cs.cs_action(hist, n, dim, e, out=acts[k + 1:k + 2], stream=st)

    t_min, t_med = _timed(step, torch.cuda.synchronize)
    h = hist.cpu().numpy().view(np.uint64).copy()
    R = int(h.sum())
    a = acts.cpu().tolist()
    graph = None
    if n <= 4096:
        # The same pass captured once in a HIP graph (every call only enqueues kernels on
        # the given stream and allocates nothing), replayed: launch gaps removed.  Each
        # replay is checked against the eager pass, with eager work between replays.
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                step(st=side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        ok = True
        for _ in range(3):
            hist.fill_(-1)
            acts.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            ok &= bool(np.array_equal(hist.cpu().numpy().view(np.uint64), h))
            ok &= acts.cpu().tolist() == a
        g_min, g_med = _timed(g.replay, torch.cuda.synchronize)
        graph = {"latency_us": g_min * 1e6, "latency_us_median": g_med * 1e6,
                 "replays_identical_to_eager": ok}
    out = {"region": W.REGION_NAMES[region], "n": n, "seed": seed, "relations": R,
           "counter": "mfma_fp4",
           "actions": {"local": a[0], **{f"eps={e}": v for e, v in zip(eps_list, a[1:])}},
           "protocol": "3 warm-up passes, minimum of the next 5 (host clock, synchronised)"}
    if n <= 4096:
        out["latency_us"] = t_min * 1e6
        out["latency_us_median"] = t_med * 1e6
        out["graph"] = graph
    else:
        out["ms_per_step"] = t_min * 1e3
        out["counts_per_s"] = R / t_min
    useful = 2 * (n * (n - 1) * (n - 2) // 6)
    for cname, c, peak in (("mfma_fp4", FP4, PEAK_FP4_OPS), ("mfma", INT8, PEAK_INT8_OPS)):
        ms = _counter_ms(cs, torch, stream, bits, n, c, hist, h_ws)
        same = bool(np.array_equal(hist.cpu().numpy().view(np.uint64), h))
        out[cname] = {"count_kernel_ms": ms, "frac_peak": useful / (ms * 1e-3) / peak,
                      "peak_TOPs": peak / 1e12, "identical_histogram": same}
    gpu_rate = R / t_min
    if not cpu:
        return out

    import oracle
    oracle.build(force=False)
    cores = oracle.max_threads()
    if name == "mink2_n1024":
        # the whole path on the CPU, definitional tier, best of three
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, _, oh, oa = oracle.pipeline(region, n, seed, eps_list=eps_list)
            ts.append(time.perf_counter() - t0)
        tc = min(ts)
        out["oracle"] = {"kind": "oracle", "tier": "definitional (whole path)", "cores": cores,
                         "seconds": tc, "counts_per_s": R / tc,
                         "gpu_over_cpu": tc / t_min,
                         "identical_histogram": bool(np.array_equal(oh, h))}
    elif name == "mink4_n16384":
        c_np = oracle.sprinkle(region, n, seed, eta0)
        b_np = oracle.causal_matrix(region, c_np)
        ind, _, _, _ = oracle.degrees(b_np, n)
        # elements j spread over the set; a pilot sizes the sample to about cpu_seconds
        pilot = np.linspace(1, n - 1, 4 * cores).astype(np.int64)
        tp = time.perf_counter()
        oracle.histogram_naive_elems(b_np, n, pilot)
        tpil = max(time.perf_counter() - tp, 1e-3)
        m = int(np.clip(len(pilot) * cpu_seconds / tpil, len(pilot), n - 1))
        js = np.linspace(1, n - 1, m).astype(np.int64)
        t0 = time.perf_counter()
        oracle.histogram_naive_elems(b_np, n, js)
        tc = time.perf_counter() - t0
        pairs = int(ind[js].sum())
        out["oracle"] = {"kind": "oracle", "tier": "definitional", "cores": cores,
                         "sample": f"{m} evenly spaced elements j, all {pairs} pairs i ≺ j",
                         "seconds": tc, "counts_per_s": pairs / tc,
                         "gpu_over_cpu": gpu_rate / (pairs / tc)}
    else:
        c_np = oracle.sprinkle(region, n, seed, eta0)
        b_np = oracle.causal_matrix(region, c_np)
        t0 = time.perf_counter()
        oh, pairs = oracle.histogram_fast(b_np, n)
        tc = time.perf_counter() - t0
        # the GPU's coordinates come from the device sprinkle (transcendentals may differ
        # by an ulp from the host's), so the histograms are reported, not required, equal
        out["oracle"] = {"kind": "oracle", "tier": "optimised (whole matrix, run once)",
                         "cores": cores, "seconds": tc, "counts_per_s": pairs / tc,
                         "gpu_over_cpu": gpu_rate / (pairs / tc),
                         "identical_histogram": bool(np.array_equal(oh, h))}
    return out


def run_configs(cs, torch, dev, stream, cpu=True):
    return {name: run_config(cs, torch, dev, stream, name, cpu=cpu)
            for name in ("mink2_n1024", "mink4_n16384", "ds4_n65536")}


if __name__ == "__main__":
    import argparse
    import json
    import os
    import sys

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    ap = argparse.ArgumentParser(description="one configuration of the benchmark set")
    ap.add_argument("workload", choices=["mink2_n1024", "mink4_n16384", "ds4_n65536"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    args = ap.parse_args()
    import torch

    import paper_1805_04463_amd as cs
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print(json.dumps(run_config(cs, torch, dev, torch.cuda.current_stream(), args.workload,
                                cpu=not args.no_cpu)))
