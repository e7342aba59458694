"""The device-built filtrations are byte-identical to the oracle's: same
compatible order (value, dimension, lexicographic vertex tuple), same
boundary matrix, same values; and reducing them gives the oracle's pairs."""
import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import _binding, api, synth

pytestmark = pytest.mark.gpu


def _compare_lowerstar(g, dev):
    f = api.build_lowerstar(torch.as_tensor(g, device=dev))
    ref = oracle.build_lowerstar(g)
    got = {k: v.cpu().numpy() for k, v in f.to_torch().items()}
    assert f.m == ref.m and f.nnz == ref.nnz
    assert np.array_equal(got["col_ptr"], ref.col_ptr)
    assert np.array_equal(got["rows"], ref.rows)
    assert np.array_equal(got["dim"], ref.dim)
    assert np.array_equal(got["value"].view(np.uint32), ref.value.astype(np.float32).view(np.uint32))
    assert np.array_equal(got["verts"], ref.verts)
    # critical vertex: the argmax of the vertex values by (value, id)
    flat = g.reshape(-1)
    vv = np.where(ref.verts >= 0, flat[np.maximum(ref.verts, 0)], -np.inf)
    best = vv.max(axis=1, keepdims=True)
    crit = np.where(vv == best, ref.verts, -1).max(axis=1)
    assert np.array_equal(got["crit"][:, 0], crit)
    return f, ref


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 5), (2, 2, 2), (1, 3, 4), (5, 6, 7), (13, 9, 11), (3, 1, 7)])
def test_lowerstar_builder_matches_oracle(gpu, shape):
    _compare_lowerstar(synth.random_grid(21, shape), gpu)


def test_lowerstar_builder_ties_and_zero_signs(gpu):
    g = synth.random_grid(22, (7, 8, 9), ties=True)
    g[0, 0, :3] = np.array([0.0, -0.0, 0.0], np.float32)  # -0 and +0 are one value
    _compare_lowerstar(g, gpu)


def test_lowerstar_builder_gaussian_64_and_reduce(gpu):
    g = synth.gaussian_field()
    f, ref = _compare_lowerstar(g, gpu)
    res = api.reduce_filtration(f)
    low_ref = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
    assert np.array_equal(res.low_star.cpu().numpy(), low_ref)
    b, d = oracle.pairs(low_ref)
    assert np.array_equal(res.pair_birth.cpu().numpy(), b) and np.array_equal(res.pair_death.cpu().numpy(), d)


def test_lowerstar_builder_rebuild_in_place(gpu):
    f = api.build_lowerstar(torch.as_tensor(synth.random_grid(23, (6, 6, 6)), device=gpu))
    g2 = synth.random_grid(24, (4, 5, 3))
    api.build_lowerstar(torch.as_tensor(g2, device=gpu), out=f)
    ref = oracle.build_lowerstar(g2)
    got = f.to_torch()
    assert np.array_equal(got["rows"].cpu().numpy(), ref.rows)


def test_lowerstar_builder_rejects_nan(gpu):
    g = synth.random_grid(25, (3, 3, 3))
    g[1, 1, 1] = np.nan
    with pytest.raises(_binding.PmsError) as e:
        api.build_lowerstar(torch.as_tensor(g, device=gpu))
    assert e.value.status == _binding.PMS_ERR_INVALID_ARG
