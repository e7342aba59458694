"""Differentiable persistence: autograd Functions over the gfx950 path.

Forward: build the filtration on the device, reduce it (pms), gather the
birth and death values of every pair.  Backward: with the pairing fixed,
dL/d(birth, death) flows to the critical vertex (lower-star) or critical
edge (Vietoris-Rips) of each paired simplex and from there to the input
(``pms_backward_lowerstar`` / ``pms_backward_vr_f32``).  Gradients are FP32.
"""
from __future__ import annotations

import ctypes

import torch

from . import _binding as B
from . import api


def gather(f: api.Filtration, simplex: torch.Tensor):
    """(values, dims) of the given simplices (``pms_gather``)."""
    simplex = simplex.to(torch.int32).contiguous()
    n = simplex.numel()
    vals = torch.empty(n, dtype=f.value_dtype, device=f.device)
    dims = torch.empty(n, dtype=torch.int8, device=f.device)
    ctx = api._ctx(f.device)
    B.check(ctx, B.load().pms_gather(ctx, f.handle, n, simplex.data_ptr() if n else None,
                                     vals.data_ptr() if n else None, dims.data_ptr() if n else None))
    return vals, dims


class PersistenceLowerStar(torch.autograd.Function):
    """grid (nz, ny, nx) float32 -> (birth values, death values, pair dims)."""

    @staticmethod
    def forward(ctx, grid, reduce_kw=None, workspace=None):
        f = api.build_lowerstar(grid.detach(), out=workspace)
        res = api.reduce_filtration(f, **(reduce_kw or {}))
        idx = torch.cat([res.pair_birth, res.pair_death])
        vals, dims = gather(f, idx)
        n = res.pair_birth.numel()
        ctx.f, ctx.idx, ctx.shape = f, idx, grid.shape
        ctx.result = res
        pair_dims = dims[:n].to(torch.int64)
        ctx.mark_non_differentiable(pair_dims)
        return vals[:n], vals[n:], pair_dims

    @staticmethod
    def backward(ctx, g_birth, g_death, _g_dims):
        n = ctx.idx.numel() // 2
        zeros = torch.zeros(n, dtype=torch.float32, device=ctx.idx.device)
        g = torch.cat([g_birth if g_birth is not None else zeros,
                       g_death if g_death is not None else zeros]).to(torch.float32).contiguous()
        out = torch.zeros(ctx.shape, dtype=torch.float32, device=ctx.idx.device)
        c = api._ctx(ctx.f.device)
        B.check(c, B.load().pms_backward_lowerstar(c, ctx.f.handle, ctx.idx.numel(), ctx.idx.data_ptr(),
                                                   g.data_ptr(), out.data_ptr(), out.numel()))
        return out, None, None


class PersistenceVR(torch.autograd.Function):
    """points (B, n, D) float32 -> (birth values, death values, pair dims,
    cloud of each pair).  Full Vietoris-Rips complex to ``maxdim`` (no
    threshold unless ``thresholds`` is given, one squared distance per cloud)."""

    @staticmethod
    def forward(ctx, points, maxdim=2, thresholds=None, reduce_kw=None, workspace=None):
        if points.dim() != 3 or points.dtype != torch.float32:
            raise ValueError("points must be a float32 tensor (B, n, D)")
        pts = points.detach().contiguous()
        nb, n, D = pts.shape
        f, off = api.build_vr(list(pts.unbind(0)), thresholds, maxdim, out=workspace)
        res = api.reduce_batched(f, off, **(reduce_kw or {}))
        idx = torch.cat([res.pair_birth, res.pair_death])
        vals, dims = gather(f, idx)
        m = res.pair_birth.numel()
        cloud = res.pair_inst.to(torch.int64)
        ctx.f, ctx.idx, ctx.pts, ctx.D = f, idx, pts, D
        ctx.result = res
        pair_dims = dims[:m].to(torch.int64)
        ctx.mark_non_differentiable(pair_dims, cloud)
        return vals[:m], vals[m:], pair_dims, cloud

    @staticmethod
    def backward(ctx, g_birth, g_death, _g_dims, _g_cloud):
        m = ctx.idx.numel() // 2
        zeros = torch.zeros(m, dtype=torch.float32, device=ctx.idx.device)
        g = torch.cat([g_birth if g_birth is not None else zeros,
                       g_death if g_death is not None else zeros]).to(torch.float32).contiguous()
        out = torch.zeros_like(ctx.pts)
        npts = ctx.pts.shape[0] * ctx.pts.shape[1]
        c = api._ctx(ctx.f.device)
        B.check(c, B.load().pms_backward_vr_f32(c, ctx.f.handle, ctx.idx.numel(), ctx.idx.data_ptr(),
                                                g.data_ptr(), ctx.pts.data_ptr(), ctx.D, npts, out.data_ptr()))
        return out, None, None, None, None


def persistence_lowerstar(grid: torch.Tensor, workspace: api.Filtration | None = None, **reduce_kw):
    """Pairs of the lower-star filtration of ``grid`` with differentiable
    values.  ``workspace``: a Filtration whose device buffers are reused
    (it holds this call's filtration until the next call that reuses it, so
    run the backward of one call before the next forward)."""
    return PersistenceLowerStar.apply(grid, reduce_kw or None, workspace)


def persistence_vr(points: torch.Tensor, maxdim: int = 2, thresholds=None,
                   workspace: api.Filtration | None = None, **reduce_kw):
    """Pairs of the Vietoris-Rips filtrations of a batch of FP32 clouds with
    differentiable values (``workspace`` as in ``persistence_lowerstar``)."""
    return PersistenceVR.apply(points, maxdim, thresholds, reduce_kw or None, workspace)
