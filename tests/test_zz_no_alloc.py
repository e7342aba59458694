"""The allocation-free entry point (``pms_reduce_noalloc``) through the C ABI:
its low*, pairs and essential simplices equal those of ``pms_reduce`` on the
same matrix, on two calls in a row (the second on a smaller matrix, so the
region holds the first call's state when the second starts), with and
without the device invariant checks; a matrix beyond the region and the
options that would allocate are refused with their statuses."""
import numpy as np
import pytest
import torch

from paper_1708_04710_amd import _binding, api, synth

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert torch.equal(a.low_star, b.low_star)
    assert torch.equal(a.pair_birth, b.pair_birth) and torch.equal(a.pair_death, b.pair_death)
    assert torch.equal(a.essential, b.essential)
    assert a.rounds == b.rounds and a.additions == b.additions


def _lowerstar(gpu, n, seed):
    g = synth.gaussian_field(seed=seed, n=n)
    return api.build_lowerstar(torch.as_tensor(g, device=gpu))


@pytest.mark.parametrize("kw", [dict(), dict(variant=1, debug_invariants=True)])
def test_noalloc_matches_reduce_two_calls(gpu, kw):
    big = _lowerstar(gpu, 32, 21)    # 792 051 columns: near the region's limit
    small = _lowerstar(gpu, 9, 22)
    for f in (big, small):
        v = f.view
        got = api._reduce_ptrs(f.device, int(v.m), v.col_ptr, v.rows, v.dim, noalloc=True, **kw)
        want = api.reduce_filtration(f, **kw)
        _same(got, want)


def test_noalloc_vr_torus_then_small_cloud(gpu):
    pts, thr = synth.vr_torus()
    f, _ = api.build_vr([torch.as_tensor(pts, device=gpu)], [thr], 2)
    v = f.view
    _same(api._reduce_ptrs(gpu, int(v.m), v.col_ptr, v.rows, v.dim, noalloc=True), api.reduce_filtration(f))
    f2, _ = api.build_vr([torch.as_tensor(synth.vr_grid_cloud()[:20], device=gpu)], [-1], 2)
    v2 = f2.view
    _same(api._reduce_ptrs(gpu, int(v2.m), v2.col_ptr, v2.rows, v2.dim, noalloc=True), api.reduce_filtration(f2))


def test_noalloc_refuses_too_large_and_allocating_options(gpu):
    m = 2_000_000  # empty columns: ~180 MB of per-column state alone
    cp = torch.zeros(m + 1, dtype=torch.int64, device=gpu)
    rows = torch.zeros(1, dtype=torch.int32, device=gpu)
    with pytest.raises(_binding.PmsError) as e:
        api.reduce(cp, rows, None, noalloc=True)
    assert e.value.status == _binding.PMS_ERR_TOO_LARGE
    f = _lowerstar(gpu, 5, 23)
    v = f.view
    for bad in (dict(graph_rounds=2), dict(diagnostics=True), dict(arena_entries=1 << 20)):
        with pytest.raises(_binding.PmsError) as e:
            api._reduce_ptrs(gpu, int(v.m), v.col_ptr, v.rows, v.dim, noalloc=True, **bad)
        assert e.value.status == _binding.PMS_ERR_INVALID_ARG
    # the region still works after the refusals
    _same(api._reduce_ptrs(gpu, int(v.m), v.col_ptr, v.rows, v.dim, noalloc=True), api.reduce_filtration(f))
