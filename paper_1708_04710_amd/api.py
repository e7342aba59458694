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


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def reduce(col_ptr: torch.Tensor, rows: torch.Tensor, dim: torch.Tensor | None = None, *,
           variant: int = 0, compression: bool = True, max_rounds: int = 0, chain: bool = True,
           tail_active: int = 1024, validate: bool = True, outputs: bool = True,
           arena_entries: int = 0) -> ReduceResult:
    """Reduce the boundary matrix given as CSC device tensors (``pms_reduce``).

    col_ptr: int64 [m+1]; rows: int32 [nnz] ascending per column; dim: int8 [m]
    or None.  All on the same CUDA (HIP) device."""
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
    dev = col_ptr.device
    lib = B.load()
    ctx = _ctx(dev)
    low_star = torch.empty(m, dtype=torch.int32, device=dev)
    cap_p = m // 2 + 1 if outputs else 0
    cap_e = m if outputs else 0
    birth = torch.empty(cap_p, dtype=torch.int32, device=dev)
    death = torch.empty(cap_p, dtype=torch.int32, device=dev)
    ess = torch.empty(cap_e, dtype=torch.int32, device=dev)
    bnd = B.PmsBoundary(m, col_ptr.data_ptr() if m >= 0 else None, rows.data_ptr() if rows.numel() else None,
                        dim.data_ptr() if dim is not None and m else None)
    if bnd.rows is None and m > 0:
        # an all-empty matrix still needs a valid pointer
        rows = torch.zeros(1, dtype=torch.int32, device=dev)
        bnd.rows = rows.data_ptr()
    opt = B.PmsOptions(variant, int(bool(compression)), max_rounds, int(bool(chain)), tail_active,
                       int(bool(validate)), arena_entries)
    res = B.PmsResult()
    res.low_star = low_star.data_ptr() if m else None
    if outputs:
        res.pair_birth = birth.data_ptr()
        res.pair_death = death.data_ptr()
        res.cap_pairs = cap_p
        res.essential = ess.data_ptr() if cap_e else None
        res.cap_essential = cap_e
    st = lib.pms_reduce(ctx, ctypes.byref(bnd), ctypes.byref(opt), ctypes.byref(res))
    B.check(ctx, st)
    return ReduceResult(low_star=low_star, pair_birth=birth[:res.n_pairs], pair_death=death[:res.n_pairs],
                        essential=ess[:res.n_essential], rounds=res.rounds, phase0_pivots=res.phase0_pivots,
                        additions=res.additions, xor_entries=res.xor_entries)
