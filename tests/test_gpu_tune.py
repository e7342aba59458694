"""Tuning of the chaining kernels (pms_set_tuning, pms_autotune) through the
C ABI: every setting, extreme ones included, gives the oracle's low*, pairs
and essential simplices; invalid settings are rejected and leave the
context's setting as it was; the autotuner keeps the fastest candidate and a
cache hit applies the stored setting without timing."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import _binding, api, autotune, synth

pytestmark = pytest.mark.gpu

SETTINGS = [
    dict(),                                    # built-in
    dict(lane_steps=0, lane_steps_few=0),      # every chain moves to the wavefront kernel at its first pivot
    dict(lane_many=0, lane_steps=1 << 30),     # lanes keep every chain they can hold
    dict(lane_blocks=1, chain_blocks=1, wide_blocks=1),  # two lane waves, one wide, four wavefront waves
    dict(lane_refill=1, lane_flush=1),
    dict(lane_refill=64, lane_flush=64),
    dict(lane_blocks=65535, chain_blocks=4096, lane_steps=3, lane_steps_few=1),
    dict(lane_cap=4),                          # most columns go through the wide pass
    dict(lane_cap=0, wide_blocks=2, lane_refill=1),  # every column does
    dict(solve=0),                             # handed-over chains walked by wavefronts, not solved by sweeps
    dict(solve=0, lane_steps=0, lane_steps_few=0),
    dict(lane_steps=0, lane_steps_few=0, chain_blocks=1),  # one workgroup solves every chain
    dict(solve=1 << 30, lane_steps=1, lane_steps_few=1),   # sweeps at any queue length
    dict(solve=1),                             # sweeps only in rounds that hand on one column
]


@pytest.fixture
def builtin_after(gpu):
    yield
    api.set_tuning(None, device=gpu)


def _lowerstar(gpu):
    g = synth.gaussian_field(seed=51, n=28)
    f = api.build_lowerstar(torch.as_tensor(g, device=gpu))
    ref = oracle.build_lowerstar(g)
    return f, oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)


def _circles(gpu):
    x = synth.circle_batch(seed=52, clouds=4, n=48)
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in x], [-1.0] * len(x), 2)
    want = []
    for b, c in enumerate(x):
        ref = oracle.build_vr_f32(c, -1.0, 2)
        low = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
        want.append(np.where(low >= 0, low + off[b], -1))
    return f, np.concatenate(want).astype(np.int32)


def _check(res, low_ref):
    low = res.low_star.cpu().numpy()
    bad = np.nonzero(low != low_ref)[0]
    assert bad.size == 0, f"{bad.size} columns differ, first {bad[:5]}"
    b, d = oracle.pairs(low_ref)
    assert np.array_equal(res.pair_birth.cpu().numpy(), b)
    assert np.array_equal(res.pair_death.cpu().numpy(), d)
    assert np.array_equal(res.essential.cpu().numpy(), oracle.essential(low_ref))


@pytest.mark.parametrize("work", ["lowerstar28", "circles4x48"])
def test_every_setting_gives_the_oracle_pairs(gpu, builtin_after, work):
    f, low_ref = (_lowerstar if work == "lowerstar28" else _circles)(gpu)
    for s in SETTINGS:
        api.set_tuning(s, device=gpu)
        assert api.get_tuning(device=gpu) == {**api.default_tuning(), **s}
        for kw in (dict(), dict(graph_rounds=4)):
            res = api.reduce_filtration(f, **kw)
            _check(res, low_ref)


def test_wide_pass_takes_the_long_columns(gpu, builtin_after):
    """With the first lane pass's buffer cut to 6 entries (and the long step
    cap in force at any queue length), the working
    columns of full 2-skeletons of 64-point circles outgrow it: the wide pass
    takes them (it moves bytes) and the pairs stay the oracle's, also with the
    wide pass on one block, with a late refill, and with every chain handed to
    wavefronts at once."""
    api.set_tuning(dict(lane_cap=6, lane_many=0), device=gpu)
    x = synth.circle_batch(seed=53, clouds=2, n=64)
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in x], [-1.0] * len(x), 2)
    want = []
    for b, c in enumerate(x):
        ref = oracle.build_vr_f32(c, -1.0, 2)
        low = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
        want.append(np.where(low >= 0, low + off[b], -1))
    low_ref = np.concatenate(want).astype(np.int32)
    api.profile_enable(True, gpu)
    res = api.reduce_filtration(f)
    prof = api.profile_read(gpu)
    api.profile_enable(False, gpu)
    assert prof["k_chain_wide"][2] > 0
    _check(res, low_ref)
    for s in (dict(lane_cap=6, lane_many=0, wide_blocks=1), dict(lane_cap=6, lane_many=0, wide_blocks=3, lane_refill=64),
              dict(lane_cap=6, lane_steps=0, lane_steps_few=0)):
        api.set_tuning(s, device=gpu)
        _check(api.reduce_filtration(f), low_ref)


def test_invalid_settings_are_rejected_and_change_nothing(gpu, builtin_after):
    keep = dict(lane_blocks=777, lane_refill=5)
    api.set_tuning(keep, device=gpu)
    want = {**api.default_tuning(), **keep}
    for bad in (dict(lane_refill=0), dict(lane_refill=65), dict(lane_flush=0), dict(lane_flush=65),
                dict(lane_blocks=0), dict(lane_blocks=65536), dict(chain_blocks=0), dict(chain_blocks=65536),
                dict(lane_steps=-1), dict(lane_steps_few=(1 << 30) + 1), dict(lane_many=-1),
                dict(wide_blocks=0), dict(wide_blocks=65536), dict(lane_cap=-1), dict(lane_cap=40),
                dict(solve=-1), dict(solve=(1 << 30) + 1)):
        with pytest.raises(_binding.PmsError) as e:
            api.set_tuning(bad, device=gpu)
        assert e.value.status == _binding.PMS_ERR_INVALID_ARG, bad
        assert api.get_tuning(device=gpu) == want
    with pytest.raises(KeyError):
        api.set_tuning(dict(lane_width=3), device=gpu)


def test_time_candidates_keeps_the_fastest(gpu, builtin_after):
    f, low_ref = _lowerstar(gpu)
    cands = [dict(), dict(lane_blocks=768, graph_rounds=4), dict(lane_steps=32, chain_blocks=256)]
    ms, best, res = api.time_candidates(f, cands, reps=3)
    assert len(ms) == 3 and all(x > 0 for x in ms)
    assert best == int(np.argmin(ms))
    win = {k: v for k, v in cands[best].items() if k != "graph_rounds"}
    assert api.get_tuning(device=gpu) == {**api.default_tuning(), **win}
    _check(res, low_ref)


def test_time_candidates_rejects_a_bad_candidate_before_running(gpu, builtin_after):
    f, _ = _lowerstar(gpu)
    api.set_tuning(dict(chain_blocks=300), device=gpu)
    with pytest.raises(_binding.PmsError) as e:
        api.time_candidates(f, [dict(), dict(lane_refill=0)], reps=1)
    assert e.value.status == _binding.PMS_ERR_INVALID_ARG
    assert "candidate 1" in str(e.value)
    assert api.get_tuning(device=gpu)["chain_blocks"] == 300


def test_autotune_search_and_cache(gpu, builtin_after, tmp_path):
    f, low_ref = _circles(gpu)
    path = tmp_path / "tune.json"
    grid = {"lane_blocks": (1024, 2048), "lane_steps_few": (8, 0), "graph_rounds": (0, 4)}
    rec = autotune.autotune(f, count=4, cache=str(path), reps=1, grid=grid)
    assert not rec["cached"] and rec["scored"] == 6
    assert rec["tuning"]["lane_blocks"] in (1024, 2048) and rec["graph_rounds"] in (0, 4)
    assert api.get_tuning(device=gpu) == rec["tuning"]
    stored = json.load(open(path))
    assert stored[rec["key"]]["tuning"] == rec["tuning"]
    assert rec["key"].endswith(autotune.size_class(f.m, f.nnz, 4))
    api.set_tuning(None, device=gpu)
    again = autotune.autotune(f, count=4, cache=str(path), reps=1, grid=grid)
    assert again["cached"] and again["tuning"] == rec["tuning"]
    assert api.get_tuning(device=gpu) == rec["tuning"]
    _check(api.reduce_filtration(f, graph_rounds=again["graph_rounds"]), low_ref)


def test_autotune_picks_the_phase2_variant(gpu, builtin_after):
    """The Phase II source (leftmost column per low, or pivots only as in
    Alg. 2) is a tuned option like graph_rounds: both reach the oracle's
    low*, and the record names the faster one without putting it among the
    kernel shapes."""
    f, low_ref = _lowerstar(gpu)
    ms, best, res = api.time_candidates(f, [dict(variant=0), dict(variant=1, lane_steps=32)], reps=1)
    assert len(ms) == 2 and best in (0, 1)
    _check(res, low_ref)
    assert api.get_tuning(device=gpu)["lane_steps"] == (32 if best == 1 else api.default_tuning()["lane_steps"])
    rec = autotune.autotune(f, cache=autotune.TuneCache(), reps=1, grid={"variant": (0, 1)})
    assert rec["variant"] in (0, 1) and "variant" not in rec["tuning"]
    _check(api.reduce_filtration(f, variant=rec["variant"]), low_ref)
    _check(api.reduce_filtration(f, variant=1 - rec["variant"]), low_ref)
