#!/usr/bin/env python3
"""Turn two rocprofv3 --pmc runs of bench.py (FETCH_SIZE, then WRITE_SIZE) into the HBM
traffic summary that bench.py reports as roofline.traffic.

Both runs are made with `--copy-calibration-mb M`, so each also holds one device copy of
M MiB (`__amd_rocclr_copyBuffer`) whose true traffic is known: M MiB read and M MiB
written.  The counters of the kernel under study are scaled by (true / counted) of
that copy.  The summary records the SHA-256 of the kernel's source file, and bench.py
reports the traffic only while the source is unchanged.

Usage:
  python bench_traffic.py FETCH.csv WRITE.csv --kernel k_count_mfma --source \
      paper_1805_04463_amd/csrc/count.hip --copy-mib 1024 --name count_mfma_mink4_n131072 \
      --command "<the rocprofv3 command lines>" --algorithmic-bytes B
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.abspath(__file__))


def per_kernel(path: str):
    out = {}
    for r in csv.DictReader(open(path)):
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--source", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--name", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--algorithmic-bytes", type=float, required=True)
    a = ap.parse_args()

    f, w = per_kernel(a.fetch_csv), per_kernel(a.write_csv)
    copy_kib = a.copy_mib * 1024.0
    cf = max(v[0] for k, v in f.items() if "copyBuffer" in k)
    cw = max(v[0] for k, v in w.items() if "copyBuffer" in k)
    fetch_scale, write_scale = copy_kib / cf, copy_kib / cw
    kf = [v for k, vs in f.items() if a.kernel in k for v in vs]
    kw = [v for k, vs in w.items() if a.kernel in k for v in vs]
    fetch_kib, write_kib = max(kf), max(kw)   # the full-size launch
    hbm = fetch_kib * 1024 * fetch_scale + write_kib * 1024 * write_scale
    sha = hashlib.sha256(open(os.path.join(ROOT, a.source), "rb").read()).hexdigest()
    rec = {"kernel": a.kernel, "source": a.source, "source_sha256": sha,
           "fetch_kib_counted": fetch_kib, "write_kib_counted": write_kib,
           "copy_calibration_mib": a.copy_mib, "copy_fetch_kib_counted": cf,
           "copy_write_kib_counted": cw, "fetch_scale": fetch_scale, "write_scale": write_scale,
           "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": a.algorithmic_bytes,
           "hbm_over_algorithmic": hbm / a.algorithmic_bytes, "command": a.command}
    base = os.path.join(ROOT, "profiles", f"traffic_{a.name}")
    json.dump(rec, open(base + ".json", "w"), indent=1)
    md = [f"# HBM traffic: `{a.kernel}` ({a.name})", "", "Commands:", "", "```", a.command, "```",
          "", f"Calibration: one device copy of {a.copy_mib} MiB counted FETCH_SIZE {cf:.1f} KiB "
          f"and WRITE_SIZE {cw:.1f} KiB; scale factors {fetch_scale:.3f} (fetch), "
          f"{write_scale:.3f} (write).", "",
          "| quantity | value |", "|---|---:|",
          f"| FETCH_SIZE counted (KiB) | {fetch_kib:.1f} |",
          f"| WRITE_SIZE counted (KiB) | {write_kib:.1f} |",
          f"| HBM bytes per launch (scaled) | {hbm:.4e} |",
          f"| algorithmic bytes per launch | {a.algorithmic_bytes:.4e} |",
          f"| ratio | {hbm / a.algorithmic_bytes:.3f} |", "",
          f"Source measured: `{a.source}` sha256 `{sha}`."]
    open(base + ".md", "w").write("\n".join(md) + "\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
