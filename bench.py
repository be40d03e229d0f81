#!/usr/bin/env python3
"""Benchmark of the causal-set interval-abundance path on one MI355X.

A step is one pass of the whole path over one synthetic causal set:
sprinkle (N points, time order) -> causal matrix -> interval histogram (fp4 MFMA counter
by default, --counter mfma for int8) -> actions (local and smeared for each eps).  Default workload: the 3+1 Minkowski
diamond of height 1 with N = 131072, eps in {0.05, 0.1, 0.2}.

Printed JSON line (rank 0 only):
  value        related-pair interval counts per second of whole steps, R / t_step
  roofline     the step's counter kernel: useful ops 2 * N(N-1)(N-2)/6 per launch over
               its mean duration from HIP events on the launch stream, against the
               MI355X dense peak of its operand type (fp4 10.1, int8 5.0 POP/s)
  mfma, bitset the other counters on the same matrix (R / t, fraction of their peak)
  batch        256 1+1 diamonds of N in [512, 8192]: ensembles/s in one graph launch
               against 256 per-instance launch sequences
  configs      the 1+1 N=1024 (latency), 3+1 N=16384 and de Sitter N=65536 workloads:
               whole path and counter kernels, with the oracle timed beside each
  cpu_baseline the CPU oracle's optimised tier timed on a row sample of the same matrix
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_INT8_OPS = 5.0e15   # MI355X dense int8 MFMA
PEAK_FP4_OPS = 10.1e15   # MI355X dense fp4 MFMA
PEAK_VALU_BITPAIRS = 256 * 4 * 16 * 2.4e9 * 16  # 2 VALU ops per 32 bit-pairs (AND, BCNT)
COUNTERS = {"bitset": 0, "mfma": 1, "mfma_fp4": 2, "bitset_dense": 3}
PEAKS = {"mfma": (PEAK_INT8_OPS, "int8"), "mfma_fp4": (PEAK_FP4_OPS, "fp4")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mink4_n131072", choices=sorted(
        k for k in W.WORKLOADS if not k.startswith("batch")))
    ap.add_argument("--counter", default="mfma_fp4", choices=["mfma", "mfma_fp4"],
                    help="interval counter used in the timed step (default: the fastest; all "
                         "counters give identical, exact histograms)")
    ap.add_argument("--no-bitset", action="store_true",
                    help="skip the side legs (the other two counters)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-field", action="store_true",
                    help="skip the discrete d'Alembertian leg on the step's matrix")
    ap.add_argument("--no-ds2", action="store_true",
                    help="skip the 1+1 de Sitter action series (the thesis's benchmark)")
    ap.add_argument("--no-chains", action="store_true",
                    help="skip the longest-chain and degree legs")
    ap.add_argument("--no-mink3", action="store_true",
                    help="skip the 2+1 diamond leg (whole path at the same N, fp4 counter)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the smaller configurations (1+1 N=1024, 3+1 N=16384, de Sitter "
                         "N=65536)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU work for the oracle sample")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB, a kernel of "
                         "known traffic for scaling HBM counters (FETCH_SIZE, WRITE_SIZE)")
    return ap.parse_args()


def events_ms(pairs):
    return [a.elapsed_time(b) for a, b in pairs]


def measured_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, or None when the
    kernel source has changed since the counters were taken (hash mismatch)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(os.path.join(ROOT, kernel_source), "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec["hbm_bytes_per_launch"]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every box here has one MI355X and the path is "
              "not sharded across GPUs; run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_1805_04463_amd as cs

    cfg = W.WORKLOADS[args.workload]
    region, n, seed, eps_list = cfg["region"], cfg["n"], cfg["seed"], tuple(cfg["eps"])
    dim = W.REGION_DIM[region]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # Preallocated device buffers: the timed region allocates nothing.
    planes = cs.cs_coord_planes(region)
    ld = cs.cs_ld_words(n)
    L = cs.lib()
    coords = torch.empty((planes, n), dtype=torch.float64, device=dev)
    bits = torch.empty((n, ld), dtype=torch.int64, device=dev)
    hist = torch.empty(n - 1, dtype=torch.int64, device=dev)
    acts = torch.empty(1 + len(eps_list), dtype=torch.float64, device=dev)
    sp_ws = torch.empty(L.cs_sprinkle_workspace_bytes(region, n), dtype=torch.uint8, device=dev)
    hist_ws = {c: torch.empty(L.cs_histogram_workspace_bytes(n, c), dtype=torch.uint8, device=dev)
               for c in COUNTERS.values()}
    main = COUNTERS[args.counter]
    eta0 = cfg.get("eta0", W.DS_ETA0)

    if args.copy_calibration_mb > 0:
        nb = args.copy_calibration_mb << 20
        src = torch.ones(nb // 8, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(counter, ev=None):
        sp_coords = coords
        cs.binding._check(L.cs_sprinkle(region, eta0, seed, n, cs.binding._ptr(sp_coords),
                                        cs.binding._ptr(sp_ws), sp_ws.numel(),
                                        cs.binding._stream(stream)), "sprinkle")
        cs.cs_causal_matrix(region, coords, n, ld, out=bits, stream=stream)
        if ev is not None:
            ev[0].record(stream)
        cs.cs_interval_histogram(bits, n, counter, out=hist, workspace=hist_ws[counter],
                                 stream=stream)
        if ev is not None:
            ev[1].record(stream)
        cs.cs_action(hist, n, dim, 0.0, out=acts[0:1], stream=stream)
        for k, e in enumerate(eps_list):
            cs.cs_action(hist, n, dim, e, out=acts[k + 1:k + 2], stream=stream)

    for _ in range(args.warmup):
        step(main)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(main, evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    count_ms = events_ms(evs)
    h = hist.cpu().numpy().view(np.uint64)
    R = int(h.sum())
    useful_macs = n * (n - 1) * (n - 2) // 6
    achieved = 2 * useful_macs / (np.mean(count_ms) * 1e-3)
    actions = acts.cpu().tolist()
    peak, kind = PEAKS[args.counter]
    measured_peak = cs.cs_measure_mfma_peak(COUNTERS[args.counter], stream=stream) * 1e12
    kernel = "k_count_mfma<4, %s, 0>" % ("true" if kind == "fp4" else "false")

    out = {
        "metric": "related-pair interval counts/sec (4D, N=131072), MFMA vs bitset; ensembles/sec",
        "value": R / (ms_step * 1e-3),
        "unit": "related-pair counts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("int8 MFMA with int32 accumulation" if kind == "int8" else
                  "fp4 (e2m1 0/1) MFMA with f32 accumulation") +
                 " (exact integer counts); fp64 coordinates and action",
        "data": "synthetic sprinkling (seeded counter-based SplitMix64), no dataset",
        "config": {"workload": args.workload, "region": W.REGION_NAMES[region], "n": n,
                   "seed": seed, "eps": list(eps_list), "counter": args.counter},
        "relations": R,
        "count_kernel_ms": {"mean": float(np.mean(count_ms)), "min": float(np.min(count_ms))},
        "counts_per_s_kernel": R / (np.mean(count_ms) * 1e-3),
        "actions": {"local": actions[0], **{f"eps={e}": a for e, a in zip(eps_list, actions[1:])}},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(
                         "paper_1805_04463_amd/csrc/count.hip",
                         f"traffic_count_{args.counter}_{args.workload}.json"),
                     "kernel": kernel,
                     "measured_peak": measured_peak / 1e12,
                     "frac_of_measured_peak": achieved / measured_peak,
                     "work_per_launch": f"2*N(N-1)(N-2)/6 = {2 * useful_macs:.4e} {kind} ops"},
    }

    if not args.no_bitset:
        wbits = None
        for name, c in COUNTERS.items():
            if name == args.counter:
                continue
            bev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(2)]
            for k in range(2):
                bev[k][0].record(stream)
                cs.cs_interval_histogram(bits, n, c, out=hist, workspace=hist_ws[c], stream=stream)
                bev[k][1].record(stream)
            torch.cuda.synchronize()
            hb = hist.cpu().numpy().view(np.uint64)
            bms = min(events_ms(bev))
            leg = {"count_kernel_ms": bms, "counts_per_s_kernel": R / (bms * 1e-3),
                   "identical_histogram": bool(np.array_equal(hb, h)),
                   "time_vs_main_counter": bms / float(np.min(count_ms))}
            if name.startswith("bitset"):
                # The related-pair work W_bits = sum over i ≺ j of (j - i - 1) bit-pairs, from
                # the degree vectors: sum_j j indeg(j) - sum_i i outdeg(i) - R.  It is the
                # bitset counters' roofline work; the dense triangle's N(N-1)(N-2)/6
                # bit-pairs is what CS_COUNT_BITSET_DENSE evaluates.
                if wbits is None:
                    ind, outd = cs.cs_degrees(bits, n, stream=stream)
                    idx = np.arange(n, dtype=np.float64)
                    wbits = float(idx @ ind.cpu().numpy().astype(np.float64)
                                  - idx @ outd.cpu().numpy().astype(np.float64)) - R
                rate = wbits / (bms * 1e-3)
                leg["roofline"] = {"bound": "alu", "achieved": rate / 1e12,
                                   "peak": PEAK_VALU_BITPAIRS / 1e12, "unit": "T bit-pairs/s",
                                   "frac": rate / PEAK_VALU_BITPAIRS,
                                   "work_per_launch": f"W_bits = sum over related pairs of "
                                                      f"(j - i - 1) = {wbits:.4e} bit-pairs"}
                leg["dense_triangle_bitpairs_per_s"] = useful_macs / (bms * 1e-3)
                leg["frac_valu_peak_dense_triangle"] = (useful_macs / (bms * 1e-3)
                                                        / PEAK_VALU_BITPAIRS)
            else:
                p, kd = PEAKS[name]
                leg["achieved_TOPs"] = 2 * useful_macs / (bms * 1e-3) / 1e12
                leg["frac_peak"] = 2 * useful_macs / (bms * 1e-3) / p
                leg["peak_TOPs"] = p / 1e12
            out[name] = leg

    if not args.no_batch and hasattr(L, "cs_batch_run"):
        from bench_batch import run_batch  # noqa: E402  (batch leg lives beside this file)
        out["batch"] = run_batch(cs, torch, dev, stream)

    if not args.no_field:
        # Discrete d'Alembertian on the step's matrix: the same MFMA tiles with the
        # per-column epilogue.  phi = 1 makes -ell^2 sum_j B1(j) equal the local action.
        phi = torch.ones(n, dtype=torch.float64, device=dev)
        bphi = torch.empty(n, dtype=torch.float64, device=dev)
        f_ws = torch.empty(max(L.cs_dalembertian_workspace_bytes(n, main), 1), dtype=torch.uint8,
                           device=dev)
        ell = 0.01
        fev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(3)]
        for k in range(3):
            fev[k][0].record(stream)
            cs.cs_dalembertian(bits, n, dim, ell, phi, counter=main, out=bphi, workspace=f_ws,
                               stream=stream)
            fev[k][1].record(stream)
        torch.cuda.synchronize()
        fms = min(events_ms(fev[1:]))
        ident = -ell ** 2 * math.fsum(bphi.cpu().numpy())
        out["dalembertian"] = {"kernel_ms": fms, "frac_peak": 2 * useful_macs / (fms * 1e-3)
                               / PEAKS[args.counter][0],
                               "minus_ell2_sum_B1": ident, "local_action": actions[0],
                               "identity_rel_err": abs(ident - actions[0]) / abs(actions[0])}

    if not args.no_chains:
        from bench_chain import run_chains  # noqa: E402  (lives beside this file)
        out["chains"] = run_chains(cs, torch, dev, stream, bits, n)

    if not args.no_mink3:
        # The 2+1 diamond at the same N: the whole path (sprinkle, matrix, fp4 counter, the
        # local and three smeared S^(2+1)) on the step's buffers, which it overwrites.
        r3 = W.MINK3_DIAMOND
        c3 = coords[:cs.cs_coord_planes(r3)]
        ws3 = torch.empty(L.cs_sprinkle_workspace_bytes(r3, n), dtype=torch.uint8, device=dev)
        fp4 = COUNTERS["mfma_fp4"]
        ev3 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(3)]
        whole = []
        for k in range(4):
            torch.cuda.synchronize()
            tk = time.perf_counter()
            cs.binding._check(L.cs_sprinkle(r3, eta0, seed, n, cs.binding._ptr(c3),
                                            cs.binding._ptr(ws3), ws3.numel(),
                                            cs.binding._stream(stream)), "sprinkle")
            cs.cs_causal_matrix(r3, c3, n, ld, out=bits, stream=stream)
            if k:
                ev3[k - 1][0].record(stream)
            cs.cs_interval_histogram(bits, n, fp4, out=hist, workspace=hist_ws[fp4], stream=stream)
            if k:
                ev3[k - 1][1].record(stream)
            cs.cs_action(hist, n, 3, 0.0, out=acts[0:1], stream=stream)
            for j, e in enumerate(eps_list):
                cs.cs_action(hist, n, 3, e, out=acts[j + 1:j + 2], stream=stream)
            torch.cuda.synchronize()
            if k:
                whole.append((time.perf_counter() - tk) * 1e3)
        k3 = min(events_ms(ev3))
        R3 = int(hist.cpu().numpy().view(np.uint64).sum())
        a3 = acts.cpu().tolist()
        out["mink3"] = {"n": n, "seed": seed, "relations": R3, "ms_per_step": min(whole),
                        "counts_per_s": R3 / (min(whole) * 1e-3),
                        "count_kernel_ms": k3,
                        "frac_peak": 2 * useful_macs / (k3 * 1e-3) / PEAKS["mfma_fp4"][0],
                        "actions": {"local": a3[0],
                                    **{f"eps={e}": a for e, a in zip(eps_list, a3[1:])}}}

    if not args.no_configs:
        from bench_configs import run_configs  # noqa: E402  (lives beside this file)
        out["configs"] = run_configs(cs, torch, dev, stream, cpu=not args.no_cpu_baseline)

    if not args.no_ds2:
        from bench_ds2 import run_ds2  # noqa: E402  (lives beside this file)
        out["ds2"] = run_ds2(cs, torch, dev, stream, main)

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        # The oracle sprinkles and links on its own; nothing is taken from the GPU.
        tm = time.perf_counter()
        c_np = oracle.sprinkle(region, n, seed, eta0)
        b_np = oracle.causal_matrix(region, c_np)
        t_link = time.perf_counter() - tm
        del c_np
        # Rows spread evenly over the set; a pilot of 8 rows per thread sizes the sample
        # so that the timed part takes about --cpu-seconds.
        npilot = 8 * oracle.max_threads()
        pilot = np.linspace(0, n - 2, npilot).astype(np.int64)
        tp = time.perf_counter()
        oracle.histogram_fast_rows(b_np, n, pilot)
        tpil = time.perf_counter() - tp
        nrows = int(np.clip(npilot * args.cpu_seconds / max(tpil, 1e-3), npilot, n - 1))
        rows = np.linspace(0, n - 2, nrows).astype(np.int64)
        tc = time.perf_counter()
        _, pairs = oracle.histogram_fast_rows(b_np, n, rows)
        tcpu = time.perf_counter() - tc
        model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                      if ln.startswith("model name")), "unknown")
        out["cpu_baseline"] = {"value": pairs / tcpu, "unit": "related-pair counts/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "cpu_model": model,
                               "gpu_over_cpu": out["value"] / (pairs / tcpu),
                               "sample": f"optimised-tier oracle (word AND + popcount) over "
                                         f"{nrows} evenly spaced rows of the same N={n} matrix: "
                                         f"{pairs} related pairs in {tcpu:.1f} s "
                                         f"(oracle sprinkle + matrix took {t_link:.1f} s)"}
        # The step's fp64 action sums against the oracle's quad-precision ones, both from
        # the step's (device) abundances: the error of the double-double sum, stated.
        errs = {}
        for e, a in zip((0.0,) + eps_list, actions):
            want, kappa = oracle.action(np.ascontiguousarray(h), n, dim, e)
            errs["local" if e == 0.0 else f"eps={e}"] = {
                "rel_err": abs(a - want) / abs(want), "kappa": kappa}
        out["cpu_baseline"]["action_vs_oracle"] = errs
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
