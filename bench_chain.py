"""Longest-chain and degree legs of bench.py (Sec. 2.5.2 algorithm "Maximal Chain Length";
Sec. 3.2 degree vectors).

  whole order   heights of every element of the step's matrix (pair (-1, N)): the layer
                partition by longest chain from below, and the height of the order;
  degrees       in- and out-degree of every element (one pass over the matrix), beside
                a measured read ceiling: torch's sum over the same matrix;
  profile       every (minimal, maximal) pair of a 16384-element 1+1 diamond, the
                candidates of the chain representation (Sec. 2.2), in one call.

Algorithmic bytes: the whole-order rounds must read every row k up to its own word at
least once, sum_k 8 (floor(k/64) + 1) bytes; the degrees read every row's ceil(N/64) words.
"""
from __future__ import annotations

import numpy as np

import workloads as W

HBM_PEAK = 8.0e12  # bytes/s


def _time(torch, stream, fn, reps=3):
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        res = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best, res


def run_chains(cs, torch, dev, stream, bits, n: int, profile_n: int = 16384, seed: int = 46):
    L = cs.lib()
    ws = torch.empty(L.cs_longest_chain_workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    ms, (length, height) = _time(torch, stream, lambda: cs.cs_longest_chain(
        bits, n, [-1], [n], heights=True, workspace=ws, stream=stream))
    rounds = int(length.item()) - 1
    words = np.arange(n, dtype=np.int64) // 64 + 1
    chain_bytes = 8.0 * float(words.sum())
    out = {"whole_order": {
        "ms": ms, "height": rounds, "rounds": rounds,
        "algorithmic_bytes": chain_bytes, "achieved_GBs": chain_bytes / (ms * 1e-3) / 1e9,
        "frac_hbm_peak": chain_bytes / (ms * 1e-3) / HBM_PEAK,
        "us_per_round": 1e3 * ms / max(rounds, 1)}}

    dms, (ind, outd) = _time(torch, stream, lambda: cs.cs_degrees(bits, n, stream=stream))
    deg_bytes = 8.0 * n * ((n + 63) // 64)
    minimal = int((ind == 0).sum().item())
    # A measured read ceiling: torch's own reduction over the same resident matrix.
    with torch.cuda.stream(stream):
        rms, _ = _time(torch, stream, lambda: bits.sum(), reps=5)
    read_GBs = bits.numel() * 8 / (rms * 1e-3) / 1e9
    out["degrees"] = {"ms": dms, "algorithmic_bytes": deg_bytes,
                      "achieved_GBs": deg_bytes / (dms * 1e-3) / 1e9,
                      "frac_hbm_peak": deg_bytes / (dms * 1e-3) / HBM_PEAK,
                      "measured_read_GBs": read_GBs,
                      "frac_of_measured_read": deg_bytes / (dms * 1e-3) / 1e9 / read_GBs,
                      "minimal_elements": minimal,
                      "minimal_have_height_1": bool(
                          torch.equal(height[0] == 1, ind == 0))}

    c = cs.cs_sprinkle(W.MINK2_DIAMOND, profile_n, seed, stream=stream)
    b2 = cs.cs_causal_matrix(W.MINK2_DIAMOND, c, stream=stream)
    i2, o2 = cs.cs_degrees(b2, profile_n, stream=stream)
    P = np.flatnonzero(i2.cpu().numpy() == 0)
    F = np.flatnonzero(o2.cpu().numpy() == 0)
    lo = np.repeat(P, len(F))
    hi = np.tile(F, len(P))
    keep = lo < hi
    lo, hi = lo[keep], hi[keep]
    ws2 = torch.empty(L.cs_longest_chain_workspace_bytes(profile_n, len(lo)), dtype=torch.uint8,
                      device=dev)
    pms, (plen, _) = _time(torch, stream, lambda: cs.cs_longest_chain(
        b2, profile_n, lo, hi, workspace=ws2, stream=stream))
    out["profile_mink2"] = {"n": profile_n, "seed": seed, "pairs": int(len(lo)),
                            "minimal": int(len(P)), "maximal": int(len(F)), "ms": pms,
                            "pairs_per_s": len(lo) / (pms * 1e-3),
                            "longest": int(plen.max().item())}
    return out
