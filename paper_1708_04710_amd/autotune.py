"""Autotuner of the chaining kernels' launch shapes and of the graph-mode
round count.

Pivot chaining (a column keeps adding the known pivot of its low within a
round, an addition to Phase II of Sec. 3.1) runs in a lane kernel and a
wavefront kernel whose grids and hand-over thresholds are a per-context
``pms_tuning``.  Every setting gives the same pairs (the lows of a reduced
matrix are unique, Sec. 2.3); only the speed changes, and the best setting
depends on the matrix: how many columns chain per round, and how long the
chains are.

The search is coordinate-wise: from the built-in setting each parameter in
turn is swept over a short list of values with the others held, and the
fastest value is kept; ``passes`` repeats the sweep (stopping early when a
pass changes nothing).  The timing is native (``pms_autotune``: one untimed
reduction, then the median of ``reps`` timed ones, of the caller's own
matrix).  Results are cached, in memory or in a JSON file, under a key of
device architecture, library version and the matrix's size class (bit
lengths of its column count, nonzero count and instance count), so one
search serves later matrices of that class.
"""
from __future__ import annotations

import json
import os
import tempfile

import torch

from . import _binding as B
from . import api

# values swept per parameter (the built-in value of each is among them)
GRID = {
    "lane_blocks": (1024, 2048, 4096),
    "chain_blocks": (256, 512, 1024),
    "lane_steps": (32, 128, 512),
    "lane_steps_few": (0, 8, 32),
    "lane_refill": (16, 32, 48),
    "lane_flush": (8, 16, 32),
    "wide_blocks": (1024, 2048, 4096),
    "lane_cap": (24, 32, 39),
    # most handed-over columns a round solves by sweeps (0: walk every chain)
    "solve": (0, 512, 4096),
    "graph_rounds": (0, 8),
    # Phase II source: 0 the leftmost column per low, 1 pivots only (Alg. 2);
    # both reach the same low*, so the faster one is kept
    "variant": (0, 1),
}
_OPTION_KEYS = ("graph_rounds", "variant")  # reduce options, not pms_tuning fields


def size_class(m: int, nnz: int, count: int = 1) -> str:
    """Bit lengths of the column count, the nonzero count and count - 1."""
    bl = lambda x: max(int(x), 0).bit_length()
    return f"m{bl(m)}.z{bl(nnz)}.b{bl(max(int(count), 1) - 1)}"


def cache_key(arch: str, version: str, m: int, nnz: int, count: int = 1) -> str:
    return f"{arch}/{version}/{size_class(m, nnz, count)}"


def coordinate_search(measure, start: dict, grid: dict, passes: int = 1):
    """Coordinate-wise minimisation of ``measure``.

    measure(list of candidate dicts) -> list of scores (lower is better);
    each call's candidates differ in one parameter only, the current best
    value listed first so that ties keep it.  Returns (best candidate, its
    score, number of candidates scored)."""
    if passes < 1:
        raise ValueError("passes must be >= 1")
    missing = set(grid) - set(start)
    if missing:
        raise KeyError(f"start lacks {sorted(missing)}")
    best = dict(start)
    best_score = None
    scored = 0
    for _ in range(passes):
        changed = False
        for p, values in grid.items():
            vals = list(dict.fromkeys([best[p], *values]))
            cands = [{**best, p: v} for v in vals]
            scores = list(measure(cands))
            if len(scores) != len(cands):
                raise ValueError("measure returned a score count that does not match the candidates")
            scored += len(cands)
            i = min(range(len(scores)), key=scores.__getitem__)
            changed = changed or vals[i] != best[p]
            best, best_score = cands[i], scores[i]
        if not changed:
            break
    return best, best_score, scored


class TuneCache:
    """A dict of tuning records, mirrored to a JSON file when ``path`` is given
    (written whole to a temporary file and renamed into place)."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as fh:
                data = json.load(fh)
            if not isinstance(data, dict):
                raise ValueError(f"{path}: not a JSON object")
            self.data = data

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, rec: dict):
        self.data[key] = rec
        if self.path:
            d = os.path.dirname(os.path.abspath(self.path))
            os.makedirs(d, exist_ok=True)
            fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune", suffix=".json")
            with os.fdopen(fd, "w") as fh:
                json.dump(self.data, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


_memory = TuneCache()


def autotune(f: "api.Filtration", *, count: int = 1, cache: TuneCache | str | None = None, reps: int = 3,
             grid: dict | None = None, passes: int = 1, **kw) -> dict:
    """Tune the context of ``f``'s device for matrices like ``f``.

    count: instances in ``f`` (a batch from ``build_vr``), part of the size
    class; cache: a TuneCache, a JSON path, or None for the process-wide
    in-memory cache; kw: the other reduce options (their ``graph_rounds``
    is the starting round count).  On a cache hit the stored setting is
    applied without timing.  Returns the record: ``tuning`` (now set on the
    context), ``graph_rounds`` and ``variant`` (pass them to the reductions), ``ms``,
    ``scored`` (candidates timed), ``key`` and ``cached``."""
    cache = _memory if cache is None else (TuneCache(cache) if isinstance(cache, str) else cache)
    v = f.view
    arch = torch.cuda.get_device_properties(f.device).gcnArchName
    key = cache_key(arch, B.load().pms_version().decode(), int(v.m), int(v.nnz), count)
    rec = cache.get(key)
    if rec is not None:
        api.set_tuning(rec["tuning"], device=f.device)
        return {"variant": 0, **rec, "key": key, "cached": True}
    grid = dict(GRID if grid is None else grid)
    start = {**api.default_tuning(), "graph_rounds": int(kw.pop("graph_rounds", 0)),
             "variant": int(kw.pop("variant", 0))}

    def measure(cands):
        ms, _, _ = api.time_candidates(f, cands, reps=reps, **kw)
        return ms

    best, ms, scored = coordinate_search(measure, start, grid, passes)
    tuning = {k: x for k, x in best.items() if k not in _OPTION_KEYS}
    api.set_tuning(tuning, device=f.device)
    rec = {"tuning": tuning, "graph_rounds": int(best["graph_rounds"]), "variant": int(best["variant"]), "ms": ms,
           "scored": scored}
    cache.put(key, rec)
    return {**rec, "key": key, "cached": False}
