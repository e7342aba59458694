#!/usr/bin/env python3
"""Benchmark of the gfx950 pms path on one GPU.

Workload: lower-star filtration of the Freudenthal triangulation of a 64^3
FP32 Gaussian random field (length scale 4 cells), H0-H2.  One step is the
whole device path on the grid already resident in HBM:

  filtration build (keys, sort, boundary matrix)  ->  pms reduction
  (Phase 0, rounds of Phase I / Phase II with clearing and compression)
  ->  low*, the persistence pairs and the essential simplices
  ->  values of the pairs and the backward pass of the total H1 persistence
      to the grid values (through the critical vertices).

The same run also times the batched Vietoris-Rips workloads against one call
per cloud on the same GPU ("batched" field): 512 clouds of 32..256 points
(reduction only) and 64 FP32 clouds of 128 points (reduction + backward of
the sum of squared H1 persistences), each checked on the host for its size;
and ("vr_dim3") the 400-point torus taken to dimension 3 (3.8e6 simplices).

Before the warm-up steps, the chaining kernels' launch shapes and the
graph-mode round count are autotuned on each workload's own filtration
(``paper_1708_04710_amd.autotune``; outside every timed region), or read
from ``--tune-cache`` when it holds the workload's size class.

Prints one JSON line.  ``value`` is simplices reduced per second over the
whole step.  ``roofline`` prices the step's dominant kernel (largest summed
event time) with its algorithmic bytes per launch against the MI355X HBM
peak; the per-kernel times come from a second pass of the same K steps
with a HIP event pair around every launch (the events slow the step, so
``value`` and ``ms_per_step`` come from the first pass, without them).
``phases`` splits the step (build, reduction alone, the rest) and prices
the whole step's bytes against the peak.  ``multiscale`` gives the paper's
per-iteration measures (Sec. 4) from one more reduction with diagnostics:
relative l1-error of low (eq. "rel_error"), proportion of unreduced
columns and precision of the essential estimate, per round.  ``cpu_baseline`` times the
CPU oracle (filtration build + standard reduction) on the same grid.
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


def _host_threads():
    """Threads for the per-cloud oracle baselines: the host cores this
    process may run on (the GPU machine's share is 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _progress(msg):
    """A finished phase of the run, on stderr (the JSON line is stdout's only line)."""
    print(f"bench: {msg} ({time.strftime('%H:%M:%S')})", file=sys.stderr, flush=True)


def cpu_baseline(grid_np, m_gpu, batches=True):
    """The oracle as it stands on the host cores.  The headline value: the
    full 64^3 grid, oracle build + standard reduction (Alg. "Standard
    reduction"), one thread; beside it the same build + the twist reduction
    (Alg. "Standard reduction with a twist"), one thread, and the two
    batches cloud by cloud (build + twist per cloud) over a thread pool of
    host cores (the oracle is C behind ctypes, which drops the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    from paper_1708_04710_amd import synth
    t0 = time.perf_counter()
    f = oracle.build_lowerstar(grid_np)
    tb = time.perf_counter() - t0
    low, st = oracle.reduce_standard(f.col_ptr, f.rows, with_stats=True)
    t = time.perf_counter() - t0
    assert f.m == m_gpu
    t1 = time.perf_counter()
    lowt, stt = oracle.reduce_twist(f.col_ptr, f.rows, f.dim, with_stats=True)
    tt = tb + time.perf_counter() - t1
    assert np.array_equal(low, lowt)
    out = {"value": f.m / t, "unit": "simplices/s", "cores": 1, "kind": "oracle",
           "sample": "full 64^3 workload: oracle lower-star build + standard reduction, one thread",
           "seconds": round(t, 3), "cpu": _cpu_model(), "host_threads": os.cpu_count(),
           "n_pairs": int((low >= 0).sum()), "standard_additions": st["additions"],
           "twist": {"value": f.m / tt, "unit": "simplices/s", "cores": 1, "seconds": round(tt, 3),
                     "sample": "full 64^3 workload: oracle lower-star build + twist reduction, one thread",
                     "twist_additions": stt["additions"]}}
    if not batches:
        return out
    nt = _host_threads()
    oracle._load()

    def pool(jobs, fn):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nt) as ex:
            ms = list(ex.map(fn, jobs))
        return sum(ms), time.perf_counter() - t0

    def vr_i32(job):
        p, thr = job
        g = oracle.build_vr_i32(p, thr, 2)
        oracle.reduce_twist(g.col_ptr, g.rows, g.dim)
        return g.m

    def vr_f32(x):
        g = oracle.build_vr_f32(x, -1.0, 2)
        oracle.reduce_twist(g.col_ptr, g.rows, g.dim)
        return g.m

    m3, t3 = pool(synth.vr_batch(), vr_i32)
    m4, t4 = pool(list(synth.circle_batch()), vr_f32)
    out["batches"] = {
        "vr512": {"value": m3 / t3, "unit": "simplices/s", "cores": nt, "seconds": round(t3, 3),
                  "sample": "all 512 clouds: oracle build + twist reduction per cloud, thread pool"},
        "circles64": {"value": m4 / t4, "unit": "simplices/s", "cores": nt, "seconds": round(t4, 3),
                      "sample": "all 64 circles: oracle build + twist reduction per cloud (no gradient), "
                                "thread pool"}}
    return out


def _source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1708_04710_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprof PMC runs
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None when
    the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != _source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _timed(fn, torch, reps=3):
    """Best of `reps` timed calls after one warm-up (both sides of every
    batched-vs-plain comparison are timed alike)."""
    fn()  # warm-up (allocations, first launches)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return min(ts)


def _tune(tune, f, count=1):
    """Autotune (or read from the cache) the shapes for filtration f; returns
    the reduce keywords and the record (None: the built-in shapes)."""
    if tune is False:
        return {}, None
    from paper_1708_04710_amd import autotune
    rec = autotune.autotune(f, count=count, cache=tune, reps=3)
    return ({"graph_rounds": rec["graph_rounds"], "variant": rec["variant"]},
            {k: rec[k] for k in ("tuning", "graph_rounds", "variant", "ms", "cached")})


def grad_error_fp64(x, bv, dv, dims, torch):
    """Norm-wise relative error, per cloud, of the FP32 gradient of
    sum over H1 pairs of (death - birth)^2 (already in x.grad) against the
    FP64 gradient on the same pairing: each pair's birth and death values are
    the squared lengths of their critical edges, recomputed here from the
    coordinates in float64 on the host."""
    f, res = bv.grad_fn.f, bv.grad_fn.result
    crit = f.to_torch()["crit"].cpu().long()
    h1 = (dims == 1).cpu()
    pb = res.pair_birth.cpu().long()[h1]
    pd = res.pair_death.cpu().long()[h1]
    X = x.detach().cpu().double().reshape(-1, x.shape[-1])
    eb, ed = crit[pb], crit[pd]
    vb = X[eb[:, 0]] - X[eb[:, 1]]
    vd = X[ed[:, 0]] - X[ed[:, 1]]
    pers = (vd * vd).sum(1) - (vb * vb).sum(1)
    w = (4.0 * pers)[:, None]
    g = torch.zeros_like(X)
    g.index_add_(0, ed[:, 0], w * vd)
    g.index_add_(0, ed[:, 1], -w * vd)
    g.index_add_(0, eb[:, 0], -w * vb)
    g.index_add_(0, eb[:, 1], w * vb)
    g = g.reshape(x.shape)
    g32 = x.grad.detach().cpu().double()
    errs = ((g32 - g).flatten(1).norm(dim=1) / g.flatten(1).norm(dim=1)).numpy()
    return {"clouds": int(x.shape[0]), "max_rel_err": float(errs.max()), "median_rel_err": float(
        sorted(errs)[len(errs) // 2]), "tolerance": 1e-5,
        "reference": "FP64 gradient on the same pairing (critical edges' squared lengths in float64)"}


def batched_vs_plain(api, autograd, synth, torch, dev, tune):
    """Batched pms (+ backward) vs one plain pms call per cloud, same GPU.
    Each side runs with the shapes tuned for it (the plain side's tuned on its
    largest cloud)."""
    out = {}
    # 512 integer clouds, own 30th-percentile thresholds (reduction only)
    inst = synth.vr_batch()
    clouds = [torch.as_tensor(p, device=dev) for p, _ in inst]
    thrs = [t for _, t in inst]
    meta = {}
    wb, wp = api.Filtration(dev), api.Filtration(dev)  # reused device workspaces
    f, off = api.build_vr(clouds, thrs, 2, out=wb)
    kw_b, rec_b = _tune(tune, f, len(clouds))
    big = max(range(len(clouds)), key=lambda b: off[b + 1] - off[b])
    f1, _ = api.build_vr([clouds[big]], [thrs[big]], 2, out=wp)
    kw_p, rec_p = _tune(tune, f1)

    def batch3():
        f, off = api.build_vr(clouds, thrs, 2, out=wb)
        r = api.reduce_filtration(f, **kw_b)
        meta["m"], meta["rounds"], meta["adds"] = f.m, r.rounds, r.additions

    def plain3():
        for c, t in zip(clouds, thrs):
            f, _ = api.build_vr([c], [t], 2, out=wp)
            api.reduce_filtration(f, **kw_p)

    _tune(tune, f, len(clouds))
    tb = _timed(batch3, torch)
    _tune(tune, f1)
    tp = _timed(plain3, torch)
    out["vr512"] = {"clouds": len(clouds), "m": meta["m"], "rounds": meta["rounds"], "additions": meta["adds"],
                    "batched_s": round(tb, 5), "plain_s": round(tp, 5), "speedup": round(tp / tb, 3),
                    "batched_simplices_per_s": meta["m"] / tb, "tuning_batched": rec_b, "tuning_plain": rec_p}
    # 64 FP32 circles x 128 points, full 2-skeleton: batched reduce + backward vs plain reduce
    x = torch.as_tensor(synth.circle_batch(), device=dev)
    f, _ = api.build_vr(list(x.unbind(0)), None, 2, out=wb)
    kw_b, rec_b = _tune(tune, f, x.shape[0])
    f1, _ = api.build_vr([x[0]], None, 2, out=wp)
    kw_p, rec_p = _tune(tune, f1)

    def batch4():
        pts = x.clone().requires_grad_(True)
        bv, dv, dims, cloud = autograd.persistence_vr(pts, workspace=wb, **kw_b)
        torch.where(dims == 1, (dv - bv) ** 2, torch.zeros_like(dv)).sum().backward()
        meta["m4"] = int(bv.grad_fn.f.m)

    def plain4():
        for c in range(x.shape[0]):
            f, _ = api.build_vr([x[c]], None, 2, out=wp)
            api.reduce_filtration(f, **kw_p)

    _tune(tune, f, x.shape[0])
    tb = _timed(batch4, torch)
    # the gradient of the last batched step against the FP64 gradient
    pts = x.clone().requires_grad_(True)
    bv, dv, dims, cloud = autograd.persistence_vr(pts, workspace=wb, **kw_b)
    torch.where(dims == 1, (dv - bv) ** 2, torch.zeros_like(dv)).sum().backward()
    grad = grad_error_fp64(pts, bv, dv, dims, torch)
    _tune(tune, f1)
    tp = _timed(plain4, torch)
    out["circles64"] = {"clouds": int(x.shape[0]), "m": meta["m4"], "batched_with_backward_s": round(tb, 5),
                        "plain_reduce_only_s": round(tp, 5), "speedup": round(tp / tb, 3),
                        "batched_simplices_per_s": meta["m4"] / tb, "grad": grad, "tuning_batched": rec_b,
                        "tuning_plain": rec_p}
    return out


def vr_dim3(api, synth, torch, dev, tune):
    """Vietoris-Rips to dimension 3 (H0-H2 plus the tetrahedra): the 400-point
    torus at its 20th-percentile threshold, build + reduce on the device."""
    pts, thr = synth.vr_torus()
    cl = [torch.as_tensor(pts, device=dev)]
    w = api.Filtration(dev)
    f, _ = api.build_vr(cl, [thr], 3, out=w)
    kw, rec = _tune(tune, f)
    meta = {}

    def run():
        f, _ = api.build_vr(cl, [thr], 3, out=w)
        r = api.reduce_filtration(f, **kw)
        meta["m"], meta["rounds"], meta["adds"], meta["r"] = f.m, r.rounds, r.additions, r

    t = _timed(run, torch)
    dims = w.to_torch()["dim"]
    ess = meta["r"].essential
    return {"workload": "vr_torus400_p20_dim3", "m": meta["m"],
            "simplices_by_dim": torch.bincount(dims.long(), minlength=4).tolist(),
            "rounds": meta["rounds"], "additions": meta["adds"], "n_pairs": int(meta["r"].pair_birth.numel()),
            "essential_by_dim": torch.bincount(dims[ess].long(), minlength=4).tolist(),
            "build_reduce_s": round(t, 5), "simplices_per_s": meta["m"] / t, "tuning": rec}


def workload_only(args, api, autograd, synth, torch, dev):
    """``--workload circles64`` or ``vr512``: that batch alone, K timed steps
    after W warm-up steps (the kernels of the batched workloads, for
    profiling them without the 64^3 step around)."""
    tune = False if args.no_autotune else args.tune_cache
    w = api.Filtration(dev)
    if args.workload == "circles64":
        x = torch.as_tensor(synth.circle_batch(), device=dev)
        f, _ = api.build_vr(list(x.unbind(0)), None, 2, out=w)
        kw, rec = _tune(tune, f, x.shape[0])
        desc = "64 FP32 circles x 128 points, full 2-skeleton: build + reduce + backward of the sum of squared H1 persistences"

        def step():
            pts = x.clone().requires_grad_(True)
            bv, dv, dims, cloud = autograd.persistence_vr(pts, workspace=w, **kw)
            torch.where(dims == 1, (dv - bv) ** 2, torch.zeros_like(dv)).sum().backward()
    else:
        inst = synth.vr_batch()
        clouds = [torch.as_tensor(p, device=dev) for p, _ in inst]
        thrs = [t for _, t in inst]
        f, _ = api.build_vr(clouds, thrs, 2, out=w)
        kw, rec = _tune(tune, f, len(clouds))
        desc = "512 integer clouds of 32..256 points, own 30th-percentile thresholds: build + reduce"

        def step():
            fb, off = api.build_vr(clouds, thrs, 2, out=w)
            api.reduce_batched(fb, off, **kw)

    m = f.m
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    out = {"metric": "simplices/s", "value": m / (ms / 1000.0), "unit": "simplices/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
           "config": {"workload": args.workload, "m": m, "step": desc, "tuning": rec}}
    print(json.dumps(out), flush=True)


# the bench run autotunes and stores the shapes in <C>; the profiled runs
# read them from there (no candidate timings in the traces)
PROFILE_CMDS = [
    "python3 bench.py --steps 10 --warmup 2 --tune-cache <C>",
    "rocprofv3 --kernel-trace --stats --output-format csv -d <T> -o ls64 -- python3 bench.py --steps 3 "
    "--warmup 1 --no-cpu-baseline --no-batched --no-dim3 --no-multiscale --calibrate-copy --tune-cache <C>",
    "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <F> -o f -- python3 bench.py --steps 1 --warmup 0 "
    "--no-cpu-baseline --no-batched --no-dim3 --no-profile --no-multiscale --calibrate-copy --tune-cache <C>",
    "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <W> -o w -- python3 bench.py --steps 1 --warmup 0 "
    "--no-cpu-baseline --no-batched --no-dim3 --no-profile --no-multiscale --calibrate-copy --tune-cache <C>",
]
COPY_BYTES = 256 << 20


def _slot(kernel_name):
    """Profiler slot of a rocprof kernel name (pms::k_xor(...) -> k_xor)."""
    if "pms::" not in kernel_name:
        return None
    name = kernel_name.split("pms::", 1)[1].split("(", 1)[0].split("<", 1)[0]
    return {"k_vr_dist": "k_vr_edges", "k_vr_count": "k_vr_tri", "k_vr_emit": "k_vr_tri",
            "k_keep_count": "k_compact", "k_scan_max4": "k_scan", "k_scan_sum": "k_scan", "k_scan_sum2": "k_scan",
            "k_fin_count": "k_finalize", "k_fin_scatter": "k_finalize", "k_gather": "k_finalize",
            "k_backward_lowerstar": "k_backward", "k_backward_vr": "k_backward",
            "k_fill_i32": "k_fill", "k_fill_u64": "k_fill", "k_iota": "k_fill", "k_part_init": "k_fill",
            "k_stats_fold": "k_fill", "k_scan_i64": "k_build_scan", "k_tile_sums": "k_build_scan",
            "k_tile_apply": "k_build_scan", "k_rs_count": "k_sort", "k_rs_offsets": "k_sort",
            "k_rs_scatter": "k_sort", "k_setup": "k_fill", "k_round_end": "k_fill"}.get(name, name)


def rocprof_summary(tdir, fdir, wdir, out_md, bench_json=None):
    """Summarise the three rocprofv3 runs (PROFILE_CMDS) into a text summary
    and profiles/traffic.json (HBM bytes per launch, scaled by the copy);
    with the JSON line of the first (unprofiled) bench run, also each
    kernel's algorithmic bytes per launch (the library's byte model and
    the unit cost of the additions), its launch time from HIP events and the
    fraction of the HBM peak they make."""
    import csv
    import glob
    from collections import defaultdict

    def one(pattern):
        hits = glob.glob(os.path.join(pattern))
        if not hits:
            raise SystemExit(f"no file matches {pattern}")
        return hits[0]

    stats = list(csv.DictReader(open(one(os.path.join(tdir, "*kernel_stats.csv")))))
    trace = list(csv.DictReader(open(one(os.path.join(tdir, "*kernel_trace.csv")))))
    fetch = list(csv.DictReader(open(one(os.path.join(fdir, "*counter_collection.csv")))))
    write = list(csv.DictReader(open(one(os.path.join(wdir, "*counter_collection.csv")))))
    def copies(rows):  # the calibration copies: the copy dispatches with the largest grid
        cp = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        g = max(int(r["Grid_Size"]) for r in cp)
        return [r for r in cp if int(r["Grid_Size"]) == g]

    copy_rows, copy_w = copies(fetch), copies(write)
    f_kib = sum(float(r["Counter_Value"]) for r in copy_rows) / len(copy_rows)
    w_kib = sum(float(r["Counter_Value"]) for r in copy_w) / len(copy_w)
    f_scale, w_scale = (COPY_BYTES / 1024) / f_kib, (COPY_BYTES / 1024) / w_kib
    acc = defaultdict(lambda: [0.0, 0, 0.0, 0])
    for rows, col, scale in ((fetch, 0, f_scale), (write, 2, w_scale)):
        for r in rows:
            sl = _slot(r["Kernel_Name"])
            if sl is None:
                continue
            acc[sl][col] += float(r["Counter_Value"]) * 1024 * scale
            acc[sl][col + 1] += 1
    durs = defaultdict(list)
    for r in trace:
        sl = _slot(r["Kernel_Name"])
        if sl:
            durs[sl].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
    kernels = {}
    for sl, (fb, fn, wb, wn) in acc.items():
        if fn and wn:
            kernels[sl] = {"fetch_bytes_per_launch": fb / fn, "write_bytes_per_launch": wb / wn,
                           "bytes_per_launch": fb / fn + wb / wn}
    tj = {"source_hash": _source_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
          "copy_bytes": COPY_BYTES, "kernels": kernels}
    with open(os.path.join(os.path.dirname(os.path.abspath(out_md)), "traffic.json"), "w") as fh:
        json.dump(tj, fh, indent=1, sort_keys=True)
    lines = ["# rocprofv3 summary: 64^3 lower-star step (build + pms reduce + pairs + backward)", "",
             "Commands (run from the repository root; <T>, <F>, <W> are output folders, <C> the tuning cache the first writes):", ""]
    lines += [f"    {c}" for c in PROFILE_CMDS]
    lines += ["", "Summarised with: python3 bench.py --rocprof-summary <T> <F> <W> <this file> <the first command's "
              "JSON line>",
              "", "## Kernel time (kernel trace: 1 warm-up step, then 3 steps timed without and 3 with per-kernel events)", "",
              "| kernel (rocprof name, shortened) | calls | total ms | avg us |", "|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:16]:
        lines.append(f"| {r['Name'][:70]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} |")
    lines += ["", "## HBM traffic (PMC FETCH_SIZE / WRITE_SIZE per dispatch; one step, run unprofiled)", "",
              f"Copy calibration: a {COPY_BYTES >> 20} MiB device copy reads FETCH_SIZE = {f_kib:.0f} KiB and "
              f"WRITE_SIZE = {w_kib:.0f} KiB (expected {COPY_BYTES >> 10} KiB each): scales "
              f"fetch x{f_scale:.3f}, write x{w_scale:.3f}.", "",
              "| slot | launches | avg us (trace) | fetch MB/launch | write MB/launch |", "|---|---|---|---|---|"]
    for sl, k in sorted(kernels.items(), key=lambda kv: -sum(durs.get(kv[0], [0]))):
        d = durs.get(sl, [])
        avg = sum(d) / len(d) if d else float("nan")
        lines.append(f"| {sl} | {len(d)} | {avg:.1f} | {k['fetch_bytes_per_launch'] / 1e6:.3f} | "
                     f"{k['write_bytes_per_launch'] / 1e6:.3f} |")
    if bench_json:
        b = json.loads(open(bench_json).read().strip().splitlines()[-1])
        steps = b["steps"]
        lines += ["", "## Algorithmic bytes per kernel (the first command's run: HIP events around each launch)", "",
                  f"Step: {b['ms_per_step']} ms ({b['value']:.4g} {b['unit']}).  alg = the library's byte model "
                  "(every array a launch must read or write once); add = 4 (len t + len s + len t+s) summed over "
                  "the launch's column additions; GB/s and frac = alg bytes / average launch time against "
                  f"{HBM_PEAK_GBS:.0f} GB/s; counted/alg = (FETCH_SIZE + WRITE_SIZE) per launch / alg.", "",
                  "| kernel | launches/step | avg us | alg MB/launch | add MB/launch | GB/s | frac | counted/alg |",
                  "|---|---|---|---|---|---|---|---|"]
        for name, k in sorted(b["kernels"].items(), key=lambda kv: -kv[1]["ms_total"]):
            avg = k["avg_us"]
            alg = k.get("alg_bytes_per_launch", 0.0)
            add = k.get("addition_bytes_per_launch")
            gbs = alg / (avg * 1e-6) / 1e9 if avg > 0 else 0.0
            cnt = kernels.get(name, {}).get("bytes_per_launch")
            ratio = f"{cnt / alg:.2f}" if cnt and alg > 0 else "-"
            lines.append(f"| {name} | {k['launches'] / steps:.1f} | {avg:.1f} | {alg / 1e6:.3f} | "
                         f"{(add / 1e6) if add else 0.0:.3f} | {gbs:.1f} | {gbs / HBM_PEAK_GBS:.4f} | {ratio} |")
        if b.get("roofline_s8d"):
            lines += ["", "Sec. 8(d) roofline of the step: " + json.dumps(b["roofline_s8d"])]
    lines += ["", f"Source hash of the kernels measured: {tj['source_hash']}", ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    print(out_md)


def batch_summary(tdir, workload, bench_json, out_md):
    """Kernel-time summary of a batched workload's rocprofv3 kernel trace
    (the commands in BATCH_PROFILE_CMDS), with the unprofiled run's line."""
    import csv
    import glob
    hits = glob.glob(os.path.join(tdir, "*kernel_stats.csv"))
    if not hits:
        raise SystemExit(f"no kernel_stats.csv under {tdir}")
    stats = list(csv.DictReader(open(hits[0])))
    b = json.loads(open(bench_json).read().strip().splitlines()[-1])
    title = {"circles64": "64 FP32 circles x 128 points, batched (build + reduce + backward)",
             "vr512": "512 integer Vietoris-Rips clouds, batched (build + reduce)"}[workload]
    lines = [f"# rocprofv3 summary: {title}", "",
             "Commands (run from the repository root; <C> is the tuning cache the first writes, <T> the output "
             "folder):", ""]
    lines += [f"    {c.replace('<W>', workload)}" for c in BATCH_PROFILE_CMDS]
    lines += ["", f"Summarised with: python3 bench.py --batch-summary <T> {workload} <the first command's JSON line> "
              "<this file>", "",
              f"The first command's line: {b['ms_per_step']} ms per step, m = {b['config']['m']}, "
              f"{b['value']:.3g} simplices/s.", "",
              "## Kernel time (kernel trace: 1 warm-up step + 3 steps)", "",
              "| kernel (rocprof name, shortened) | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:16]:
        lines.append(f"| {r['Name'][:60]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    lines += [""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    print(out_md)


BATCH_PROFILE_CMDS = [
    "python3 bench.py --workload <W> --steps 5 --warmup 2 --tune-cache <C>",
    "rocprofv3 --kernel-trace --stats --output-format csv -d <T> -o b -- python3 bench.py --workload <W> "
    "--steps 3 --warmup 1 --tune-cache <C>",
]


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--batch-summary":
        batch_summary(*sys.argv[2:6])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--rocprof-summary":
        t, f, w, out = sys.argv[2:6]
        rocprof_summary(t, f, w, out, sys.argv[6] if len(sys.argv) > 6 else None)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without the per-kernel events")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of autotuned shapes by size class (read, and written on a miss)")
    ap.add_argument("--no-autotune", action="store_true", help="run with the library's built-in shapes")
    ap.add_argument("--no-multiscale", action="store_true", help="skip the reduction with per-round diagnostics")
    ap.add_argument("--no-dim3", action="store_true", help="skip the Vietoris-Rips dimension-3 workload")
    ap.add_argument("--workload", default="lowerstar64", choices=("lowerstar64", "circles64", "vr512"),
                    help="lowerstar64 (default): the full bench line; circles64 / vr512: that batch alone")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device copy (known bytes) to scale rocprof's FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1708_04710_amd import api, autograd, synth

    dev = torch.device("cuda:0")
    if args.workload != "lowerstar64":
        workload_only(args, api, autograd, synth, torch, dev)
        return
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    grid_np = synth.gaussian_field(seed=5, n=64, sigma=4.0)
    grid = torch.as_tensor(grid_np, device=dev)
    f = api.build_lowerstar(grid)
    tune = False if args.no_autotune else args.tune_cache
    rkw, tune_rec = _tune(tune, f)
    _progress("64^3 built and tuned")

    state = {}

    def step():
        x = grid.clone().requires_grad_(True)
        bv, dv, dims = autograd.persistence_lowerstar(x, workspace=f, **rkw)
        # total H1 persistence; a masked sum (boolean indexing would make the
        # host wait for the device to learn the mask's size)
        loss = torch.where(dims == 1, dv - bv, torch.zeros_like(dv)).sum()
        loss.backward()
        state["x"] = x
        state["fn"] = (bv, dv, dims)
        return loss

    for _ in range(args.warmup):
        step()
    # the timed region: K steps, no per-kernel events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    # the same K steps again with a HIP event pair around every kernel launch
    # (per-kernel times for the roofline; the events slow the step down)
    prof, prof_ms = {}, None
    if not args.no_profile:
        api.profile_enable(True, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        prof_ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        prof = api.profile_read(dev, addition_bytes=True)
        api.profile_enable(False, dev)
    bv, dv, dims = state["fn"]
    res = bv.grad_fn.result if hasattr(bv.grad_fn, "result") else None
    m = f.m
    g = state["x"].grad
    # light self-checks (no oracle on the GPU leg): the gradient of a total
    # persistence is a signed count of deaths minus births per vertex
    assert g is not None and torch.equal(g, g.round())
    n_pairs = int(bv.numel())

    # phases of the step, timed apart (outside the timed region): build, and
    # the reduction alone on the built filtration (the survey's t_reduce)
    def _med(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        ts.sort()
        return ts[len(ts) // 2] * 1000.0

    build_ms = _med(lambda: api.build_lowerstar(grid, out=f))
    reduce_ms = _med(lambda: api.reduce_filtration(f, **rkw))
    phases = {"profiled_ms_per_step": round(prof_ms, 4) if prof_ms else None,
              "build_ms": round(build_ms, 3), "reduce_ms": round(reduce_ms, 3),
              "pairs_gather_backward_ms": round(max(ms - build_ms - reduce_ms, 0.0), 3),
              "reduce_only_simplices_per_s": m / (reduce_ms / 1000.0)}

    # the paper's per-iteration measures (Sec. 4) on this filtration: one more
    # reduction with diagnostics, outside every timed region; once with the
    # bench's schedule (pivot chaining), once with the paper's own (Alg.
    # "Parallel multi-scale reduction" as printed: Phase II adds known pivots
    # only, one addition per column per round)
    def multiscale_block(kw, keep_rows):
        dres = api.reduce_filtration(f, diagnostics=True, **kw)
        ms_rows = api.multiscale(dres.round_stats, m, int(dres.essential.numel()))

        def first_round(pred):
            return next((r["round"] for r in ms_rows if pred(r)), None)

        def fmt(r):
            return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}

        keep = ms_rows if keep_rows is None else [r for r in ms_rows if r["round"] in keep_rows or r is ms_rows[-1]]
        return {
            "rounds": dres.rounds, "additions": dres.additions,
            "rounds_to_rel_l1_error": {f"1e-{k}": first_round(lambda r, k=k: r["rel_error"] <= 10.0 ** -k)
                                       for k in (1, 2, 3, 4)} | {"0": first_round(lambda r: r["rel_error"] == 0.0)},
            "rounds_to_unreduced": {str(p): first_round(lambda r, p=p: r["unreduced"] <= p)
                                    for p in (0.9, 0.5, 0.1, 0.05, 0.01)},
            "rounds_to_ess_precision": {str(p): first_round(lambda r, p=p: r["ess_precision"] >= p)
                                        for p in (0.1, 0.5, 0.9, 0.95, 1.0)},
            "per_round": [fmt(r) for r in keep],
        }

    multiscale = multiscale_paper = multiscale_priority = None
    _progress("timed steps done")
    if not args.no_multiscale:
        multiscale = multiscale_block(rkw, None)
        paper_kw = dict(variant=1, chain=False)
        multiscale_paper = multiscale_block(paper_kw, {0, 1, 2, 3, 5, 10, 20, 50, 100, 200, 500, 1000, 2000})
        multiscale_paper["schedule"] = ("Phase II adds known pivots only, one addition per column per round "
                                        "(no chaining): variant=1, chain=False")
        # Sec. 3.4: fewer processors than colliding columns -- at most a
        # budget of columns add per round, chosen by priority (0 column
        # order, 1 largest sets N first, 2 known negative first), on the
        # paper's schedule over a 24^3 grid of the same field recipe
        f24 = api.build_lowerstar(torch.as_tensor(synth.gaussian_field(n=24), device=dev))
        m24 = int(f24.m)
        multiscale_priority = {"grid": "24^3 lower-star, Gaussian field (seed 5, sigma 4)", "m": m24,
                               "schedule": "variant=1, chain=False, round_budget=2048"}
        for prio, name in ((0, "column_order"), (1, "largest_N_first"), (2, "known_negative_first")):
            dres = api.reduce_filtration(f24, diagnostics=True, variant=1, chain=False, round_budget=2048,
                                         priority=prio)
            rows = api.multiscale(dres.round_stats, m24, int(dres.essential.numel()))
            first = lambda pred: next((r["round"] for r in rows if pred(r)), None)
            multiscale_priority[name] = {
                "rounds": dres.rounds, "additions": dres.additions,
                "rounds_to_rel_l1_error": {f"1e-{k}": first(lambda r, k=k: r["rel_error"] <= 10.0 ** -k)
                                           for k in (1, 2, 3, 4)},
                "rounds_to_unreduced": {str(q): first(lambda r, q=q: r["unreduced"] <= q) for q in (0.5, 0.1, 0.01)}}

    # how each dominant-kernel candidate's bytes are counted (the library counts them in-kernel)
    OWN_BYTES_MODEL = {
        "k_chain": "the bytes the kernel's own design must move: each chained column read and written once, "
                   "one 32-byte record per chained step (plus a long pivot's column)",
        "k_chain_solve": "the bytes the kernel's own design must move: each chained column read and written once, "
                         "one 32-byte record per pivot that joins or leaves the added set (plus a long pivot's "
                         "column)"}
    ADD_BYTES_MODEL = {
        "k_chain_solve": "4 (len c + the added pivots' lengths + len out) per chained column: its additions "
                         "as one multi-way sum (each input read once, the result written once)"}
    roof = roof_s8d = None
    kernels = {}
    if prof:
        for name, (tot_ms, n, by, ab) in prof.items():
            kernels[name] = {"ms_total": round(tot_ms, 4), "launches": n,
                             "avg_us": round(1000.0 * tot_ms / n, 3),
                             "alg_bytes_per_launch": by / n}
            if ab > 0:
                kernels[name]["addition_bytes_per_launch"] = ab / n
        dom = max(prof, key=lambda k: prof[k][0])
        tot_ms, n, by, ab = prof[dom]
        avg_s = tot_ms / n / 1000.0
        ach = (by / n) / avg_s / 1e9 if avg_s > 0 else 0.0
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": measured_traffic(dom),
                "avg_launch_us": round(avg_s * 1e6, 3), "alg_bytes_per_launch": by / n,
                "bytes_model": OWN_BYTES_MODEL.get(dom, "the bytes the kernel's own design must move")}
        # the same kernel priced by the unit cost of a column addition: each
        # addition t <- t + s reads t and s and writes t + s, 4 bytes an entry
        ach2 = (ab / n) / avg_s / 1e9 if avg_s > 0 else 0.0
        roof_s8d = {"kernel": dom, "bound": "hbm", "achieved": round(ach2, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach2 / HBM_PEAK_GBS, 5), "traffic": measured_traffic(dom),
                    "avg_launch_us": round(avg_s * 1e6, 3), "alg_bytes_per_launch": ab / n,
                    "bytes_model": ADD_BYTES_MODEL.get(dom, "4 (len t + len s + len t+s) per column addition")}
        # the whole step's HBM traffic (rocprof FETCH+WRITE per kernel launch,
        # when the counters match these kernels) and algorithmic bytes
        alg = sum(v[2] for v in prof.values()) / args.steps
        meas, missing = 0.0, []
        for name, (_, nl, _, _) in prof.items():
            b = measured_traffic(name)
            if b is None:
                missing.append(name)
            else:
                meas += b * nl / args.steps
        phases["step_algorithmic_bytes"] = alg
        phases["step_algorithmic_frac_of_hbm_peak"] = round(alg / (ms / 1000.0) / (HBM_PEAK_GBS * 1e9), 5)
        if not missing:
            phases["step_measured_hbm_bytes"] = meas
            phases["step_measured_frac_of_hbm_peak"] = round(meas / (ms / 1000.0) / (HBM_PEAK_GBS * 1e9), 5)
        else:
            phases["step_measured_hbm_bytes"] = None  # kernels changed since the counters were taken
    # the reduction's bytes by the unit costs of the method: the CSC read
    # once (4 nnz + 8 m), 40 bytes per active column per round (low read and
    # written, leftmost table update and read, compaction, header), every
    # column addition at 4 (len t + len s + len t+s), and the finalisation
    # (4 m + 8 per pair + 4 per essential simplex), over the reduction's time
    if res is not None:
        s8d = (4.0 * f.nnz + 8.0 * m + 40.0 * res.active_sum + res.addition_bytes + 4.0 * m
               + 8.0 * n_pairs + 4.0 * int(res.essential.numel()))
        phases["reduce_unit_cost_bytes"] = s8d
        phases["reduce_unit_cost_parts"] = {"load": 4.0 * f.nnz + 8.0 * m, "rounds": 40.0 * res.active_sum,
                                            "additions": float(res.addition_bytes),
                                            "finalize": 4.0 * m + 8.0 * n_pairs + 4.0 * int(res.essential.numel())}
        phases["reduce_unit_cost_frac_of_hbm_peak"] = round(s8d / (reduce_ms / 1000.0) / (HBM_PEAK_GBS * 1e9), 5)

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
                   "m": m, "nnz": f.nnz, "homology": "H0-H2",
                   "step": "build + reduce + pairs + gather + backward of total H1 persistence",
                   "rounds": res.rounds if res else None, "additions": res.additions if res else None,
                   "n_pairs": n_pairs, "n_essential": int(res.essential.numel()) if res else None,
                   "tuning": tune_rec},
        "roofline": roof,
        "roofline_s8d": roof_s8d,
        "phases": phases,
        "multiscale": multiscale,
        "multiscale_paper": multiscale_paper,
        "multiscale_priority": multiscale_priority,
        "kernels": kernels,
        "cpu_baseline": None,
    }
    _progress("multiscale and profile done")
    if not args.no_batched:
        out["batched"] = batched_vs_plain(api, autograd, synth, torch, dev, tune)
        _progress("batched workloads done")
    if not args.no_dim3:
        out["vr_dim3"] = vr_dim3(api, synth, torch, dev, tune)
        _progress("dimension-3 workload done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(grid_np, m, batches=not args.no_batched)
        _progress("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
