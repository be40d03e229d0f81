"""The thesis's action benchmark on the 1+1 de Sitter slab (Sec. 4.3): smeared
Benincasa-Dowker action with eps = 2^-6 on the slab eta in [-1/2, 1/2], ten seeds per
size, against the Einstein-Hilbert value 4 pi tan(eta0) that the mean approaches as N
grows.  Each graph is the whole path (sprinkle, matrix, counter, action) on device
buffers allocated beforehand, timed with HIP events on the launch stream."""
from __future__ import annotations

import math

import numpy as np

import workloads as W


def run_ds2(cs, torch, dev, stream, counter, sizes=(1 << 14, 1 << 15, 1 << 16, 1 << 17)):
    L = cs.lib()
    eps, eta0 = W.DS2_EPS, W.DS2_ETA0
    series = []
    for n in sizes:
        ld = cs.cs_ld_words(n)
        coords = torch.empty((3, n), dtype=torch.float64, device=dev)
        bits = torch.empty((n, ld), dtype=torch.int64, device=dev)
        hist = torch.empty(n - 1, dtype=torch.int64, device=dev)
        act = torch.empty(len(W.DS2_SEEDS), dtype=torch.float64, device=dev)
        sp_ws = torch.empty(L.cs_sprinkle_workspace_bytes(W.DS2_SLAB, n), dtype=torch.uint8,
                            device=dev)
        h_ws = torch.empty(L.cs_histogram_workspace_bytes(n, counter), dtype=torch.uint8,
                           device=dev)

        def graph(k, seed):
            cs.binding._check(L.cs_sprinkle(W.DS2_SLAB, eta0, seed, n, cs.binding._ptr(coords),
                                            cs.binding._ptr(sp_ws), sp_ws.numel(),
                                            cs.binding._stream(stream)), "sprinkle")
            cs.cs_causal_matrix(W.DS2_SLAB, coords, n, ld, out=bits, stream=stream)
            cs.cs_interval_histogram(bits, n, counter, out=hist, workspace=h_ws, stream=stream)
            cs.cs_action(hist, n, 2, eps, out=act[k:k + 1], stream=stream)

        graph(0, W.DS2_SEEDS[0])  # warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k, seed in enumerate(W.DS2_SEEDS):
            graph(k, seed)
        e1.record(stream)
        torch.cuda.synchronize()
        v = act.cpu().numpy()
        series.append({"n": n, "ms_per_graph": e0.elapsed_time(e1) / len(W.DS2_SEEDS),
                       "mean": float(v.mean()), "sd": float(v.std(ddof=1)),
                       "sem": float(v.std(ddof=1) / math.sqrt(len(v)))})
        del coords, bits, hist, sp_ws, h_ws
    return {"region": "ds2_slab", "eta0": eta0, "eps": eps, "seeds": list(W.DS2_SEEDS),
            "target_4pi_tan_eta0": 4 * math.pi * math.tan(eta0), "series": series}
