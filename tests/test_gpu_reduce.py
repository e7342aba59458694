"""Parity of the HIP pms reduction (through the C ABI) with the CPU oracle.

low*, the pairs and the essential simplices must match bit for bit: the
arithmetic is F2 and low* is unique for a filtration (Sec. 2.3)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import _binding, api, synth
from tests import brute

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _dev(cp, rows, dim, device):
    return (torch.as_tensor(np.asarray(cp, np.int64), device=device),
            torch.as_tensor(np.asarray(rows, np.int32), device=device),
            None if dim is None else torch.as_tensor(np.asarray(dim, np.int8), device=device))


def _check(res, ref):
    low = res.low_star.cpu().numpy()
    bad = np.nonzero(low != ref)[0]
    assert bad.size == 0, f"{bad.size} columns differ, first {bad[:5]}: got {low[bad[:5]]} want {ref[bad[:5]]}"
    b, d = oracle.pairs(ref)
    assert np.array_equal(res.pair_birth.cpu().numpy(), b)
    assert np.array_equal(res.pair_death.cpu().numpy(), d)
    assert np.array_equal(res.essential.cpu().numpy(), oracle.essential(ref))


def _reduce(cp, rows, dim, device, **kw):
    c, r, d = _dev(cp, rows, dim, device)
    return api.reduce(c, r, d, **kw)


def test_wave_primitives_selftest(gpu):
    api.selftest(gpu)


def test_hand_examples(gpu):
    for ex in json.load(open(GOLDEN))["examples"]:
        for variant in (0, 1):
            res = _reduce(ex["col_ptr"], ex["rows"], ex["dim"], gpu, variant=variant)
            _check(res, np.array(ex["low_star"], np.int32))


@pytest.mark.parametrize("facets", [
    [(0, 1), (1, 2), (0, 2)],
    [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)],
    [tuple(sorted((i % 7, (i + 1) % 7, (i + 3) % 7))) for i in range(7)] +
    [tuple(sorted((i % 7, (i + 2) % 7, (i + 3) % 7))) for i in range(7)],
    [(1, 2, 3), (1, 3, 4), (1, 4, 5), (1, 5, 6), (1, 2, 6), (2, 3, 5), (2, 4, 5), (2, 4, 6), (3, 4, 6), (3, 5, 6)],
], ids=["circle", "tetra_boundary", "torus7", "rp2"])
def test_small_complexes(gpu, facets):
    cp, rows, dim, _, _ = brute.complex_from_facets(facets)
    ref = oracle.reduce_standard(cp, rows)
    for kw in ({}, {"variant": 1}, {"compression": False}, {"chain": False}):
        _check(_reduce(cp, rows, dim, gpu, **kw), ref)


def test_fuzz_random_filtrations(gpu):
    rng = np.random.default_rng(2024)
    opts = [dict(), dict(variant=1), dict(compression=False), dict(chain=False), dict(tail_active=0),
            dict(variant=1, compression=False, chain=False)]
    for t in range(300):
        cp, rows, dim, _, _ = brute.random_filtration(rng, n_vertices=int(rng.integers(2, 9)),
                                                      n_facets=int(rng.integers(1, 9)),
                                                      max_dim=int(rng.integers(1, 4)))
        ref = oracle.reduce_standard(cp, rows)
        kw = opts[t % len(opts)]
        _check(_reduce(cp, rows, dim if t % 7 else None, gpu, **kw), ref)


@pytest.mark.parametrize("kw", [dict(), dict(variant=1), dict(compression=False), dict(chain=False),
                                dict(variant=1, chain=False, compression=False)],
                         ids=["default", "pivot_gated", "no_compression", "no_chain", "paper_plain"])
def test_vr_grid50_full(gpu, kw):
    f = oracle.build_vr_i32(synth.vr_grid_cloud(), -1, 2)
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    res = _reduce(f.col_ptr, f.rows, f.dim, gpu, **kw)
    _check(res, ref)
    assert res.rounds >= 1


def test_vr_torus400(gpu):
    pts, thr = synth.vr_torus()
    f = oracle.build_vr_i32(pts, thr, 2)
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu), ref)


def test_vr_f32_circle_cloud(gpu):
    x = synth.circle_batch()[0]
    f = oracle.build_vr_f32(x, -1.0, 2)
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu), ref)


@pytest.mark.parametrize("shape,ties", [((8, 8, 8), False), ((13, 17, 11), False), ((9, 10, 12), True),
                                        ((1, 30, 40), False), ((24, 24, 24), False)])
def test_lowerstar_grids(gpu, shape, ties):
    g = synth.random_grid(7, shape, ties=ties)
    f = oracle.build_lowerstar(g)
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    for kw in ({}, {"variant": 1}, {"chain": False}):
        _check(_reduce(f.col_ptr, f.rows, f.dim, gpu, **kw), ref)


def test_lowerstar_gaussian_64(gpu):
    """The full 64^3 Gaussian-field workload."""
    f = oracle.build_lowerstar(synth.gaussian_field())
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    res = _reduce(f.col_ptr, f.rows, f.dim, gpu)
    _check(res, ref)
    assert res.essential.numel() == 1


# ---------------------------------------------------------------- edges
def test_empty_and_trivial(gpu):
    res = _reduce([0], np.zeros(0, np.int32), np.zeros(0, np.int8), gpu)
    assert res.low_star.numel() == 0 and res.pair_birth.numel() == 0 and res.essential.numel() == 0
    res = _reduce([0, 0], np.zeros(0, np.int32), [0], gpu)  # one vertex
    _check(res, np.array([-1], np.int32))
    res = _reduce([0, 0, 0, 0], np.zeros(0, np.int32), [0, 0, 0], gpu)  # vertices only
    _check(res, np.array([-1, -1, -1], np.int32))


def test_rejects_incompatible(gpu):
    with pytest.raises(_binding.PmsError) as e:
        _reduce([0, 0, 0, 2], [1, 0], [0, 0, 1], gpu)  # unsorted rows
    assert e.value.status == _binding.PMS_ERR_NOT_COMPATIBLE
    with pytest.raises(_binding.PmsError) as e:
        _reduce([0, 1], [0], [1], gpu)  # row >= column
    assert e.value.status == _binding.PMS_ERR_NOT_COMPATIBLE
    with pytest.raises(_binding.PmsError) as e:
        _reduce([0, 0, 1], [0], [0, 2], gpu)  # facet of the wrong dimension
    assert e.value.status == _binding.PMS_ERR_NOT_COMPATIBLE


def test_max_rounds_not_converged(gpu):
    f = oracle.build_vr_i32(synth.vr_grid_cloud(), -1, 2)
    with pytest.raises(_binding.PmsError) as e:
        _reduce(f.col_ptr, f.rows, f.dim, gpu, max_rounds=1, chain=False)
    assert e.value.status == _binding.PMS_ERR_NOT_CONVERGED


def test_arena_regrowth(gpu):
    """A 1024-entry arena forces several regrowths; the result is unchanged."""
    f = oracle.build_vr_i32(synth.vr_grid_cloud(), -1, 2)
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu, arena_entries=1024), ref)
    # the next call on the same context starts from a normal arena again
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu), ref)


def test_pipelined_rounds_match_rounds_read_one_by_one(gpu):
    """By default a round is queued before the previous round's counters reach
    the host (its grid bounded by the count that round started with; a round
    queued after convergence does nothing).  The low*, round count and
    additions equal those of rounds the host reads one by one (a round cap far
    above the rounds needed turns the pipelining off), also with the twist
    sweep, and with an arena small enough to grow while a round is queued."""
    big = 1 << 24
    cases = [oracle.build_vr_i32(synth.vr_grid_cloud(), -1, 2),
             oracle.build_lowerstar(synth.random_grid(81, (9, 10, 11)))]
    for f in cases:
        ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
        for kw in (dict(), dict(sweep=True), dict(chain=False)):
            a = _reduce(f.col_ptr, f.rows, f.dim, gpu, arena_entries=big, **kw)
            b = _reduce(f.col_ptr, f.rows, f.dim, gpu, arena_entries=big, max_rounds=1 << 20, **kw)
            _check(a, ref)
            _check(b, ref)
            assert (a.rounds, a.additions) == (b.rounds, b.additions), kw
        _check(_reduce(f.col_ptr, f.rows, f.dim, gpu, arena_entries=1024), ref)


# ---------------------------------------------------------------- graph mode
@pytest.mark.parametrize("k", [1, 2, 5])
def test_graph_rounds_parity(gpu, k):
    """Rounds replayed as a captured HIP graph give the oracle's low* and the
    same number of rounds as one round at a time (graph_rounds rounds per
    host synchronisation; the rounds after convergence do nothing)."""
    f = oracle.build_vr_i32(synth.vr_grid_cloud(), -1, 2)
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    # same arena for both (an arena overflow redoes a round's dropped additions
    # one round later, so the round count depends on the arena's size)
    big = 1 << 24
    eager = _reduce(f.col_ptr, f.rows, f.dim, gpu, chain=False, arena_entries=big)
    res = _reduce(f.col_ptr, f.rows, f.dim, gpu, chain=False, graph_rounds=k, arena_entries=big)
    _check(res, ref)
    assert res.rounds == eager.rounds
    assert res.additions == eager.additions
    # the default path (chaining) and a replay longer than the whole reduction
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu, graph_rounds=64), ref)


def test_graph_rounds_fuzz_and_lowerstar(gpu):
    rng = np.random.default_rng(77)
    for t in range(40):
        cp, rows, dim, _, _ = brute.random_filtration(rng, n_vertices=int(rng.integers(2, 9)),
                                                      n_facets=int(rng.integers(1, 9)),
                                                      max_dim=int(rng.integers(1, 4)))
        ref = oracle.reduce_standard(cp, rows)
        _check(_reduce(cp, rows, dim, gpu, graph_rounds=1 + t % 4), ref)
    g = synth.random_grid(81, (9, 10, 11))
    f = oracle.build_lowerstar(g)
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu, graph_rounds=4), oracle.reduce_twist(f.col_ptr, f.rows, f.dim))


def test_graph_rounds_arena_regrowth(gpu):
    """An arena overflow inside a replay: the arena grows, the graph is
    captured again and the result is unchanged."""
    f = oracle.build_vr_i32(synth.vr_grid_cloud(), -1, 2)
    ref = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu, arena_entries=1024, graph_rounds=4), ref)
    _check(_reduce(f.col_ptr, f.rows, f.dim, gpu), ref)


def _long_pivot_matrix(seed):
    """A boundary matrix (no dimensions) whose chains need pivot columns far
    longer than an LDS buffer: rows 0..7999 are empty columns; ten pivots
    P_a hold 600..2000 random rows below 6000 plus the row 7990 - a as their
    low; short pivots Q_r = {r-3, r-2, r-1, r} own the rows r in [6003, 7000);
    sixty targets hold all ten lows of the P_a, a few rows in [6003, 7000) and
    a few rows below 6000.  A target's first addition (P_0) leaves it with
    P_1's low: its chain then merges the long P_a one after another, grows
    past the LDS buffer, and walks down the short pivots from global memory."""
    rng = np.random.default_rng(seed)
    B = 8000
    cols = [[] for _ in range(B)]
    for a in range(10):
        k = int(rng.integers(600, 2001))
        cols.append(sorted(rng.choice(6000, k - 1, replace=False).tolist()) + [7990 - a])
    for r in range(6003, 7000):
        cols.append([r - 3, r - 2, r - 1, r])
    for _ in range(60):
        extra = set(rng.choice(np.arange(6003, 7000), 4, replace=False).tolist())
        extra |= set(rng.choice(6000, 5, replace=False).tolist())
        cols.append(sorted(extra) + [7990 - a for a in range(9, -1, -1)])
    cp = np.zeros(len(cols) + 1, np.int64)
    cp[1:] = np.cumsum([len(c) for c in cols])
    rows = np.concatenate([np.asarray(c, np.int32) for c in cols if c])
    return cp, rows


@pytest.mark.parametrize("solve", [0, 1 << 30])
def test_long_pivots_global_paths(gpu, capfd, monkeypatch, solve):
    """With the sweep kernel off, the wavefront chain kernel's paths for
    columns and pivots too long for LDS (a long pivot merged in global memory,
    and the working column flushed to the arena) give the oracle's low*; the
    kernel's trace counters show that the global-memory merge ran.  With it
    on, the same chains (long pivots read from their columns) are solved by
    sweeps or handed on, with the same low*."""
    monkeypatch.setenv("PMS_TRACE", "1")
    api.set_tuning(dict(solve=solve), device=gpu)
    try:
        for seed in (1, 2):
            cp, rows = _long_pivot_matrix(seed)
            ref = oracle.reduce_standard(cp, rows)
            for kw in (dict(), dict(compression=False), dict(variant=1)):
                res = _reduce(cp, rows, None, gpu, validate=False, tail_active=1 << 30, **kw)
                _check(res, ref)
    finally:
        api.set_tuning(None, device=gpu)
    err = capfd.readouterr().err
    if solve == 0:
        glob = [int(x) for x in __import__("re").findall(r"global (\d+)", err)]
        assert glob and sum(glob) > 0, err[-2000:]
    else:
        solved = [int(x) for x in __import__("re").findall(r"solve: columns (\d+)", err)]
        assert solved and sum(solved) > 0, err[-2000:]
