#!/usr/bin/env python3
"""Benchmark of the gfx950 pms path on one GPU.

Workload: lower-star filtration of the Freudenthal triangulation of a 64^3
FP32 Gaussian random field (length scale 4 cells), H0-H2.  One step is the
whole device path on the grid already resident in HBM:

  filtration build (keys, sort, boundary matrix)  ->  pms reduction
  (Phase 0, rounds of Phase I / Phase II with clearing and compression)
  ->  low*, the persistence pairs and the essential simplices.

Prints one JSON line.  ``value`` is simplices reduced per second over the
whole step.  ``roofline`` prices the step's dominant kernel (largest summed
event time) with its algorithmic bytes per launch against the MI355X HBM
peak.  ``cpu_baseline`` times the CPU oracle (filtration build + standard
reduction) on the same grid.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "simplices reduced/s + % HBM peak; batched pms+grad vs plain pms, pairs bit-exact"


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(grid_np, m_gpu):
    """The oracle as it stands, single-threaded, on the full grid."""
    import oracle
    t0 = time.perf_counter()
    f = oracle.build_lowerstar(grid_np)
    low = oracle.reduce_standard(f.col_ptr, f.rows)
    t = time.perf_counter() - t0
    assert f.m == m_gpu
    return {"value": f.m / t, "unit": "simplices/s", "cores": 1, "kind": "oracle",
            "sample": "full 64^3 workload: oracle lower-star build + standard reduction, one thread",
            "seconds": round(t, 3), "cpu": _cpu_model(), "host_threads": os.cpu_count(),
            "n_pairs": int((low >= 0).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without the per-kernel events")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1708_04710_amd import api, synth

    dev = torch.device("cuda:0")
    grid_np = synth.gaussian_field(seed=5, n=64, sigma=4.0)
    grid = torch.as_tensor(grid_np, device=dev)
    f = api.build_lowerstar(grid)

    state = {}

    def step():
        api.build_lowerstar(grid, out=f)
        res = api.reduce_filtration(f)
        state["res"] = res
        return res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if not args.no_profile:
        api.profile_enable(True, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = api.profile_read(dev) if not args.no_profile else {}
    if not args.no_profile:
        api.profile_enable(False, dev)
    ms = (t1 - t0) * 1000.0 / args.steps
    res = state["res"]
    m = f.m

    # light self-check (no oracle on the GPU leg): a 3-ball has one essential class
    assert res.essential.numel() == 1

    roof = None
    kernels = {}
    if prof:
        for name, (tot_ms, n, by) in prof.items():
            kernels[name] = {"ms_total": round(tot_ms, 4), "launches": n,
                             "avg_us": round(1000.0 * tot_ms / n, 3),
                             "alg_bytes_per_launch": by / n}
        dom = max(prof, key=lambda k: prof[k][0])
        tot_ms, n, by = prof[dom]
        avg_s = tot_ms / n / 1000.0
        ach = (by / n) / avg_s / 1e9 if avg_s > 0 else 0.0
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None,
                "avg_launch_us": round(avg_s * 1e6, 3), "alg_bytes_per_launch": by / n}

    out = {
        "metric": METRIC,
        "value": m / (ms / 1000.0),
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "lowerstar_freudenthal_64^3_gaussian_field", "grid": [64, 64, 64],
                   "field": "white noise * Gaussian(sigma=4 cells, periodic), standardised, fp32, seed 5",
                   "m": m, "nnz": f.nnz, "homology": "H0-H2", "step": "build + reduce + pairs",
                   "rounds": res.rounds, "additions": res.additions, "n_pairs": int(res.pair_birth.numel()),
                   "n_essential": int(res.essential.numel())},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(grid_np, m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
