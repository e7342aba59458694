"""Python front end of the gfx950 pms library.

PyTorch supplies device memory and the stream; each function only checks
shapes, allocates outputs and calls the C ABI.  All work runs in the
library's HIP kernels on ``torch.cuda.current_stream()``.
"""
from __future__ import annotations

import atexit
import ctypes
from dataclasses import dataclass

import torch

from . import _binding as B

_ctxs: dict = {}


def _ctx(device: torch.device):
    """The library context bound to ``device`` and its current stream."""
    lib = B.load()
    dev = device.index if device.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    c = _ctxs.get(key)
    if c is None:
        h = ctypes.c_void_p()
        st = lib.pms_create(ctypes.byref(h), dev, ctypes.c_void_p(stream))
        if st != B.PMS_OK:
            raise B.PmsError(st, "pms_create failed")
        c = h
        _ctxs[key] = c
    return c


@atexit.register
def _destroy_all():
    if B._lib is None:
        return
    for c in list(_ctxs.values()):
        B._lib.pms_destroy(c)
    _ctxs.clear()


def selftest(device=None):
    """Run the library's check of its wave-level primitives on ``device``."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    ctx = _ctx(dev)
    B.check(ctx, B.load().pms_selftest(ctx))


def profile_enable(enable: bool = True, device=None):
    """Start (and zero) or stop the library's per-kernel event timing on the
    context of ``device`` and its current stream."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    ctx = _ctx(dev)
    B.check(ctx, B.load().pms_profile_enable(ctx, int(bool(enable))))


def profile_read(device=None, addition_bytes=False) -> dict:
    """{kernel name: (total ms, launches, algorithmic bytes)} since
    profile_enable; with ``addition_bytes`` a fourth entry: the bytes of the
    kernel's column additions at 4 (len t + len s + len t+s) each (0 for the
    kernels that add no columns)."""
    lib = B.load()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    ctx = _ctx(dev)
    out = {}
    for k in range(lib.pms_profile_kernels()):
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        B.check(ctx, lib.pms_profile_read(ctx, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        if n.value:
            rec = (ms.value, n.value, by.value)
            if addition_bytes:
                ab = ctypes.c_double()
                B.check(ctx, lib.pms_profile_read_addition_bytes(ctx, k, ctypes.byref(ab)))
                rec = rec + (ab.value,)
            out[lib.pms_profile_kernel_name(k).decode()] = rec
    return out


def default_options() -> dict:
    o = B.load().pms_default_options()
    return {f: getattr(o, f) for f, _ in B.PmsOptions._fields_}


@dataclass
class ReduceResult:
    low_star: torch.Tensor    # int32 [m], -1 = no low*
    pair_birth: torch.Tensor  # int32 [n_pairs], low*(j), ascending in j
    pair_death: torch.Tensor  # int32 [n_pairs], j
    essential: torch.Tensor   # int32 [n_essential], ascending
    rounds: int
    phase0_pivots: int
    additions: int
    xor_entries: int
    active_sum: int = 0      # sum over rounds of the round's active columns
    addition_bytes: int = 0  # sum over additions of 4 (len t + len s + len t+s)
    # batched reductions only (reduce_batched): per-instance starts in the
    # pair / essential lists ([count+1] int64) and the instance of each pair
    inst_pair_off: torch.Tensor | None = None
    inst_ess_off: torch.Tensor | None = None
    pair_inst: torch.Tensor | None = None
    # diagnostics=True only: one dict per recorded round (round_stats) and
    # the essential estimate of the last one (bool [m], essential_estimate)
    round_stats: list | None = None
    essential_estimate: torch.Tensor | None = None


class Filtration:
    """A filtration built on the device (library-owned memory, freed with the
    object).  ``view`` holds its device pointers; ``to_torch`` copies it."""

    def __init__(self, device: torch.device):
        self.device = device
        self.handle = ctypes.c_void_p()
        self.view = B.PmsFiltrationView()

    def _refresh(self):
        B.check(None, B.load().pms_filtration_view_get(self.handle, ctypes.byref(self.view)))

    @property
    def m(self) -> int:
        return int(self.view.m)

    @property
    def nnz(self) -> int:
        return int(self.view.nnz)

    @property
    def value_dtype(self):
        return torch.float32 if self.view.value_f32 else torch.int64

    def to_torch(self) -> dict:
        m, nnz, dev = self.m, self.nnz, self.device
        out = {"col_ptr": torch.empty(m + 1, dtype=torch.int64, device=dev),
               "rows": torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
               "dim": torch.empty(max(m, 1), dtype=torch.int8, device=dev),
               "value": torch.empty(max(m, 1), dtype=self.value_dtype, device=dev),
               "crit": torch.empty(max(2 * m, 1), dtype=torch.int32, device=dev),
               "verts": torch.empty(max(4 * m, 1), dtype=torch.int32, device=dev)}
        ctx = _ctx(dev)
        B.check(ctx, B.load().pms_filtration_copy_out(ctx, self.handle, *[out[k].data_ptr() for k in
                                                                          ("col_ptr", "rows", "dim", "value",
                                                                           "crit", "verts")]))
        out["rows"] = out["rows"][:nnz]
        out["dim"] = out["dim"][:m]
        out["value"] = out["value"][:m]
        out["crit"] = out["crit"][:2 * m].view(m, 2)
        out["verts"] = out["verts"][:4 * m].view(m, 4)
        return out

    def left_beta(self):
        """(left, beta) as device int32 tensors (Defs. "left", "beta"; 2^31 - 1
        and -1 for none) when the builder produced them, else None."""
        if not self.view.left:
            return None
        m, dev = self.m, self.device
        left = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        beta = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        ctx = _ctx(dev)
        B.check(ctx, B.load().pms_filtration_copy_left_beta(ctx, self.handle, left.data_ptr(), beta.data_ptr()))
        return left[:m], beta[:m]

    def __del__(self):
        try:
            lib = B._lib
        except AttributeError:  # interpreter shutdown: the module is gone
            return
        if self.handle and lib is not None:
            lib.pms_filtration_free(self.handle)
            self.handle = ctypes.c_void_p()


def build_lowerstar(grid: torch.Tensor, out: Filtration | None = None) -> Filtration:
    """Lower-star filtration of the Freudenthal triangulation of a 3-D FP32
    grid of shape (nz, ny, nx) (``pms_build_lowerstar``)."""
    if not grid.is_cuda or grid.dtype != torch.float32 or grid.dim() != 3:
        raise ValueError("grid must be a 3-D float32 device tensor (nz, ny, nx)")
    grid = grid.contiguous()
    nz, ny, nx = grid.shape
    f = out if out is not None else Filtration(grid.device)
    ctx = _ctx(grid.device)
    B.check(ctx, B.load().pms_build_lowerstar(ctx, grid.data_ptr(), nx, ny, nz, ctypes.byref(f.handle)))
    f._refresh()
    return f


def build_vr(clouds, thresholds=None, maxdim: int = 2, out: Filtration | None = None):
    """Vietoris-Rips filtrations of one or more point clouds, concatenated
    block-diagonally (``pms_build_vr_i32`` / ``pms_build_vr_f32``).

    clouds: a device tensor [n, D] or a list of them, all int32 or all
    float32.  thresholds: None (keep every simplex) or one squared-distance
    threshold per cloud (< 0 = none).  Returns (filtration, col_off) where
    cloud b owns the columns col_off[b]:col_off[b+1] (a host list)."""
    if isinstance(clouds, torch.Tensor):
        clouds = [clouds]
    clouds = list(clouds)
    if not clouds:
        raise ValueError("no clouds")
    dtype = clouds[0].dtype
    if dtype not in (torch.int32, torch.float32) or any(c.dtype != dtype for c in clouds):
        raise TypeError("clouds must all be int32 or all float32")
    if any(not c.is_cuda or c.dim() != 2 for c in clouds):
        raise ValueError("clouds must be 2-D device tensors [n, D]")
    dev = clouds[0].device
    nb = len(clouds)
    n = (ctypes.c_int32 * nb)(*[int(c.shape[0]) for c in clouds])
    D = (ctypes.c_int32 * nb)(*[int(c.shape[1]) for c in clouds])
    offs, o = [], 0
    for c in clouds:
        offs.append(o)
        o += c.numel()
    pt_off = (ctypes.c_int64 * nb)(*offs)
    flat = torch.cat([c.reshape(-1) for c in clouds]) if o else torch.zeros(1, dtype=dtype, device=dev)
    f32 = dtype == torch.float32
    if thresholds is None:
        thresholds = [-1] * nb
    thr = (ctypes.c_float * nb)(*[float(t) for t in thresholds]) if f32 else \
        (ctypes.c_int64 * nb)(*[int(t) for t in thresholds])
    col_off = (ctypes.c_int64 * (nb + 1))()
    f = out if out is not None else Filtration(dev)
    ctx = _ctx(dev)
    fn = B.load().pms_build_vr_f32 if f32 else B.load().pms_build_vr_i32
    st = fn(ctx, flat.data_ptr(), nb, n, D, pt_off, thr, maxdim, ctypes.byref(f.handle), col_off)
    _binding_check(ctx, st)
    f._refresh()
    return f, [int(x) for x in col_off]


def _binding_check(ctx, st):
    B.check(ctx, st)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _options(variant=0, compression=True, max_rounds=0, chain=True, tail_active=1024, validate=True,
             arena_entries=0, graph_rounds=0, diagnostics=False, debug_invariants=False, c8=False, sweep=0,
             priority=0, round_budget=0):
    return B.PmsOptions(variant, int(bool(compression)), max_rounds, int(bool(chain)), tail_active,
                        int(bool(validate)), graph_rounds, int(bool(diagnostics)), arena_entries,
                        int(bool(debug_invariants)), int(bool(c8)), int(sweep), int(priority), int(round_budget), 0)


def _outputs(dev, m, outputs):
    """Output tensors and the pms_result pointing at them."""
    low_star = torch.empty(m, dtype=torch.int32, device=dev)
    cap_p = m // 2 + 1 if outputs else 0
    cap_e = m if outputs else 0
    t = dict(low_star=low_star, birth=torch.empty(cap_p, dtype=torch.int32, device=dev),
             death=torch.empty(cap_p, dtype=torch.int32, device=dev),
             ess=torch.empty(cap_e, dtype=torch.int32, device=dev))
    res = B.PmsResult()
    res.low_star = low_star.data_ptr() if m else None
    if outputs:
        res.pair_birth = t["birth"].data_ptr()
        res.pair_death = t["death"].data_ptr()
        res.cap_pairs = cap_p
        res.essential = t["ess"].data_ptr() if cap_e else None
        res.cap_essential = cap_e
    return res, t


def _result(res, t, **extra) -> ReduceResult:
    return ReduceResult(low_star=t["low_star"], pair_birth=t["birth"][:res.n_pairs],
                        pair_death=t["death"][:res.n_pairs], essential=t["ess"][:res.n_essential],
                        rounds=res.rounds, phase0_pivots=res.phase0_pivots, additions=res.additions,
                        xor_entries=res.xor_entries, active_sum=res.active_sum,
                        addition_bytes=res.addition_bytes, **extra)


def _reduce_ptrs(dev, m, col_ptr_p, rows_p, dim_p, *, outputs=True, inst_col_off=None, noalloc=False,
                 left_p=None, beta_p=None, **kw) -> ReduceResult:
    lib = B.load()
    ctx = _ctx(dev)
    bnd = B.PmsBoundary(m, col_ptr_p, rows_p, dim_p, left_p, beta_p)
    opt = _options(**kw)
    res, t = _outputs(dev, m, outputs)
    extra = {}
    if noalloc:
        if inst_col_off is not None:
            raise ValueError("the allocation-free entry point reduces one matrix")
        st = lib.pms_reduce_noalloc(ctx, ctypes.byref(bnd), ctypes.byref(opt), ctypes.byref(res))
    elif inst_col_off is None:
        st = lib.pms_reduce(ctx, ctypes.byref(bnd), ctypes.byref(opt), ctypes.byref(res))
    else:
        nb = inst_col_off.numel() - 1
        poff = torch.empty(nb + 1, dtype=torch.int64, device=dev)
        eoff = torch.empty(nb + 1, dtype=torch.int64, device=dev)
        pinst = torch.empty(max(res.cap_pairs, 1), dtype=torch.int32, device=dev)
        st = lib.pms_reduce_batched(ctx, nb, inst_col_off.data_ptr(), ctypes.byref(bnd), ctypes.byref(opt),
                                    ctypes.byref(res), poff.data_ptr(), eoff.data_ptr(),
                                    pinst.data_ptr() if outputs else None)
        extra = dict(inst_pair_off=poff, inst_ess_off=eoff, pair_inst=pinst[:res.n_pairs] if outputs else None)
    B.check(ctx, st)
    if kw.get("diagnostics"):
        extra.update(round_stats=round_stats(dev), essential_estimate=essential_estimate(m, dev))
    return _result(res, t, **extra)


def round_stats(device=None) -> list:
    """The per-round records of the last reduction with ``diagnostics=True``
    on the context of ``device`` (``pms_round_stats_read``), also after one
    stopped by ``max_rounds``: dicts with round, active, new_pivots,
    additions, xor_entries, low_l1 (sum of low + 1), ess_estimate (|E|) and
    c8_cleared (columns cleared by Lemma "Clearing by local compression")."""
    dev = _dev(device)
    ctx = _ctx(dev)
    lib = B.load()
    n = ctypes.c_int32(0)
    B.check(ctx, lib.pms_round_stats_read(ctx, 0, None, ctypes.byref(n)))
    arr = (B.PmsRoundStats * max(n.value, 1))()
    B.check(ctx, lib.pms_round_stats_read(ctx, n.value, arr, ctypes.byref(n)))
    return [{f: getattr(arr[i], f) for f, _ in B.PmsRoundStats._fields_} for i in range(n.value)]


def essential_estimate(m: int, device=None) -> torch.Tensor:
    """E of the last recorded round as a bool mask [m] (``pms_essential_estimate``)."""
    dev = _dev(device)
    ctx = _ctx(dev)
    words = torch.zeros(max((m + 31) // 32, 1), dtype=torch.int32, device=dev)
    B.check(ctx, B.load().pms_essential_estimate(ctx, m, words.data_ptr() if m else None))
    bits = torch.arange(32, device=dev, dtype=torch.int32)
    mask = ((words[:, None] >> bits[None, :]) & 1).reshape(-1)[:m]
    return mask.to(torch.bool)


def multiscale(stats: list, m: int, n_essential: int | None = None) -> list:
    """The paper's per-iteration measures from ``round_stats`` of a
    converged reduction: relative l1-error of low (eq. "rel_error", using
    ||low*||_1 = the last entry's low_l1), proportion of unreduced columns,
    and the precision |Ess| / |E| of the essential estimate."""
    if not stats:
        return []
    final = stats[-1]["low_l1"]
    ess = stats[-1]["ess_estimate"] if n_essential is None else n_essential
    out = []
    for s in stats:
        out.append({"round": s["round"],
                    "rel_error": (s["low_l1"] - final) / final if final else 0.0,
                    "unreduced": s["active"] / m if m else 0.0,
                    "ess_precision": ess / s["ess_estimate"] if s["ess_estimate"] else 1.0,
                    "additions": s["additions"], "c8_cleared": s["c8_cleared"]})
    return out


# ------------------------------------------------------------------ tuning
TUNING_FIELDS = tuple(f for f, _ in B.PmsTuning._fields_)


def default_tuning() -> dict:
    """The library's built-in launch shapes of the chaining kernels."""
    t = B.load().pms_default_tuning()
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def _tuning_struct(tuning: dict | None) -> B.PmsTuning:
    """A pms_tuning from ``tuning`` (fields it lacks take the built-in values)."""
    unknown = set(tuning or {}) - set(TUNING_FIELDS)
    if unknown:
        raise KeyError(f"unknown tuning fields {sorted(unknown)}")
    t = B.load().pms_default_tuning()
    for k, v in (tuning or {}).items():
        setattr(t, k, int(v))
    return t


def _dev(device):
    return torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)


def set_tuning(tuning: dict | None = None, device=None):
    """Set the chaining kernels' shapes for the context of ``device`` and its
    current stream (``pms_set_tuning``); ``None`` restores the built-in ones."""
    dev = _dev(device)
    ctx = _ctx(dev)
    t = _tuning_struct(tuning)
    B.check(ctx, B.load().pms_set_tuning(ctx, ctypes.byref(t)))


def get_tuning(device=None) -> dict:
    dev = _dev(device)
    ctx = _ctx(dev)
    t = B.PmsTuning()
    B.check(ctx, B.load().pms_get_tuning(ctx, ctypes.byref(t)))
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def time_candidates(f: "Filtration", candidates, reps: int = 3, **kw):
    """Time reductions of filtration ``f`` under each candidate
    (``pms_autotune``).  A candidate is a dict of tuning fields plus, optionally,
    ``graph_rounds`` and the Phase II ``variant`` (both give the same low*);
    ``kw`` are the other reduce options, common to all.
    Returns (median ms per candidate, index of the fastest, ReduceResult of
    one more run with it); the context keeps the fastest tuning."""
    n = len(candidates)
    if n < 1:
        raise ValueError("no candidates")
    kw = dict(kw)
    outputs = kw.pop("outputs", True)
    graph_rounds = kw.pop("graph_rounds", 0)
    variant = kw.pop("variant", 0)
    lib = B.load()
    ctx = _ctx(f.device)
    v = f.view
    m = int(v.m)
    bnd = B.PmsBoundary(m, v.col_ptr, v.rows, v.dim, v.left, v.beta)
    opts = (B.PmsOptions * n)()
    tunes = (B.PmsTuning * n)()
    for i, c in enumerate(candidates):
        c = dict(c)
        opts[i] = _options(graph_rounds=int(c.pop("graph_rounds", graph_rounds)),
                           variant=int(c.pop("variant", variant)), **kw)
        tunes[i] = _tuning_struct(c)
    res, t = _outputs(f.device, m, outputs)
    ms = (ctypes.c_double * n)()
    best = ctypes.c_int32(-1)
    st = lib.pms_autotune(ctx, ctypes.byref(bnd), n, opts, tunes, int(reps), ctypes.byref(res), ms,
                          ctypes.byref(best))
    B.check(ctx, st)
    return [ms[i] for i in range(n)], best.value, _result(res, t)


def reduce(col_ptr: torch.Tensor, rows: torch.Tensor, dim: torch.Tensor | None = None, **kw) -> ReduceResult:
    """Reduce the boundary matrix given as CSC device tensors (``pms_reduce``).

    col_ptr: int64 [m+1]; rows: int32 [nnz] ascending per column; dim: int8 [m]
    or None.  All on the same device.  Keyword options as in ``pms_options``:
    variant, compression, max_rounds, chain, tail_active, validate,
    graph_rounds, arena_entries, diagnostics, debug_invariants, c8, sweep,
    priority, round_budget; ``outputs=False``
    skips the pair / essential lists; ``noalloc=True`` calls the
    allocation-free entry point (``pms_reduce_noalloc``; the output tensors
    are still allocated here, by the caller of the library)."""
    if not col_ptr.is_cuda or not rows.is_cuda or (dim is not None and not dim.is_cuda):
        raise ValueError("col_ptr, rows and dim must be device tensors")
    if col_ptr.dtype != torch.int64 or rows.dtype != torch.int32 or (dim is not None and dim.dtype != torch.int8):
        raise TypeError("expected col_ptr int64, rows int32, dim int8")
    col_ptr = col_ptr.contiguous()
    rows = rows.contiguous()
    dim = dim.contiguous() if dim is not None else None
    m = col_ptr.numel() - 1
    if m < 0:
        raise ValueError("col_ptr must have m+1 >= 1 entries")
    if dim is not None and dim.numel() != m:
        raise ValueError("dim must have m entries")
    if rows.numel() == 0:
        rows = torch.zeros(1, dtype=torch.int32, device=col_ptr.device)  # a valid pointer
    return _reduce_ptrs(col_ptr.device, m, col_ptr.data_ptr(), rows.data_ptr(),
                        dim.data_ptr() if dim is not None and m else None, **kw)


def reduce_filtration(f: Filtration, **kw) -> ReduceResult:
    """Reduce a device-built filtration in place of its library-owned arrays.
    The input check (``validate``) is off unless asked for: the builders'
    matrices are those of compatible filtrations by construction."""
    kw.setdefault("validate", False)
    v = f.view
    return _reduce_ptrs(f.device, int(v.m), v.col_ptr, v.rows, v.dim, left_p=v.left, beta_p=v.beta, **kw)


def reduce_batched(f: Filtration, col_off, **kw) -> ReduceResult:
    """Reduce a batch built by ``build_vr`` (``pms_reduce_batched``): same as
    ``reduce_filtration``, plus the per-instance pair / essential offsets and
    the instance of every pair.  ``col_off``: the instances' column offsets
    (count + 1 entries, host list or int64 tensor)."""
    kw.setdefault("validate", False)
    off = torch.as_tensor(col_off, dtype=torch.int64).to(f.device)
    v = f.view
    return _reduce_ptrs(f.device, int(v.m), v.col_ptr, v.rows, v.dim, inst_col_off=off, left_p=v.left,
                        beta_p=v.beta, **kw)
