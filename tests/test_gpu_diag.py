"""Multi-scale diagnostics (pms_round_stats_read, pms_essential_estimate)
through the C ABI, pinned by the paper's definitions rather than by the
schedule: after Phase 0 they follow from beta alone (Def. "beta"); the
essential estimate contains Ess at every stop (Lemma "Essential
estimation") and equals it at convergence; ||low^l||_1 never increases and
ends at ||low*||_1 (eq. "rel_error"); the unreduced columns end at zero.
Round-by-round values beyond these depend on the schedule and are checked
only through these properties."""
import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import _binding, api, synth
from tests import brute

pytestmark = pytest.mark.gpu


def _dev(cp, rows, dim, device):
    return (torch.as_tensor(np.asarray(cp, np.int64), device=device),
            torch.as_tensor(np.asarray(rows, np.int32), device=device),
            None if dim is None else torch.as_tensor(np.asarray(dim, np.int8), device=device))


def _phase0(cp, rows, m):
    """low^0, ||low^0||_1, active and E after Phase 0 from the definitions
    (compression: rows of columns with beta defined are deleted)."""
    _, beta = oracle.left_beta(cp, rows)
    known_neg = beta >= 0
    low0 = np.full(m, -1, np.int64)
    for j in range(m):
        col = rows[cp[j]:cp[j + 1]]
        keep = col[~known_neg[col]] if col.size else col
        low0[j] = keep[-1] if keep.size else -1
    ess = ~known_neg
    ess[low0[low0 >= 0]] = False
    return int((low0 + 1).sum()), int((low0 >= 0).sum()), ess


def _check_run(res, stats, est, cp, rows, low_ref, first_exact=True):
    m = low_ref.size
    assert [s["round"] for s in stats] == list(range(len(stats)))
    assert len(stats) == res.rounds + 1
    l1 = [s["low_l1"] for s in stats]
    ne = [s["ess_estimate"] for s in stats]
    act = [s["active"] for s in stats]
    assert all(a >= b for a, b in zip(l1, l1[1:])), l1
    assert all(a >= b for a, b in zip(ne, ne[1:])), ne
    assert all(a >= b for a, b in zip(act, act[1:])), act
    assert l1[-1] == int((low_ref.astype(np.int64) + 1).sum())
    assert act[-1] == 0
    ess_ref = np.zeros(m, bool)
    ess_ref[oracle.essential(low_ref)] = True
    assert np.array_equal(est.cpu().numpy(), ess_ref)
    assert ne[-1] == int(ess_ref.sum())
    assert sum(s["additions"] for s in stats) == res.additions
    if first_exact:
        l0, a0, e0 = _phase0(np.asarray(cp), np.asarray(rows), m)
        assert (stats[0]["low_l1"], stats[0]["active"], stats[0]["ess_estimate"]) == (l0, a0, int(e0.sum()))


@pytest.mark.parametrize("kw", [dict(), dict(variant=1, chain=False, tail_active=0), dict(graph_rounds=4)])
def test_diagnostics_random_filtrations(gpu, kw):
    rng = np.random.default_rng(77)
    for t in range(60):
        cp, rows, dim, _, _ = brute.random_filtration(rng, n_vertices=int(rng.integers(3, 9)),
                                                      n_facets=int(rng.integers(1, 9)), max_dim=int(rng.integers(1, 4)))
        low_ref = oracle.reduce_standard(cp, rows)
        c, r, d = _dev(cp, rows, dim, gpu)
        res = api.reduce(c, r, d, diagnostics=True, **kw)
        assert np.array_equal(res.low_star.cpu().numpy(), low_ref)
        _check_run(res, res.round_stats, res.essential_estimate, cp, rows, low_ref)


def test_diagnostics_lowerstar_and_vr_batch(gpu):
    g = synth.gaussian_field(seed=61, n=20)
    f = api.build_lowerstar(torch.as_tensor(g, device=gpu))
    ref = oracle.build_lowerstar(g)
    low_ref = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
    res = api.reduce_filtration(f, diagnostics=True)
    plain = api.reduce_filtration(f)
    assert torch.equal(res.low_star, plain.low_star)
    _check_run(res, res.round_stats, res.essential_estimate, ref.col_ptr, ref.rows, low_ref)
    ms = api.multiscale(res.round_stats, f.m)
    assert ms[-1]["rel_error"] == 0.0 and ms[0]["rel_error"] > 0.0 and ms[-1]["ess_precision"] == 1.0

    x = synth.circle_batch(seed=62, clouds=3, n=40)
    fb, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in x], [-1.0] * len(x), 2)
    want = []
    for b, cl in enumerate(x):
        rb = oracle.build_vr_f32(cl, -1.0, 2)
        lb = oracle.reduce_twist(rb.col_ptr, rb.rows, rb.dim)
        want.append(np.where(lb >= 0, lb + off[b], -1))
    low_b = np.concatenate(want).astype(np.int32)
    res = api.reduce_batched(fb, off, diagnostics=True)
    v = fb.to_torch()
    _check_run(res, res.round_stats, res.essential_estimate, v["col_ptr"].cpu().numpy(), v["rows"].cpu().numpy(),
               low_b)


def test_early_stop_estimate_contains_essential(gpu):
    """Stopped after l rounds (max_rounds), the estimate of the last completed
    round contains Ess and the pairs known so far are the oracle's."""
    g = synth.gaussian_field(seed=63, n=14)
    f = api.build_lowerstar(torch.as_tensor(g, device=gpu))
    ref = oracle.build_lowerstar(g)
    low_ref = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
    ess_ref = np.zeros(f.m, bool)
    ess_ref[oracle.essential(low_ref)] = True
    full = api.reduce_filtration(f, diagnostics=True, chain=False)
    assert full.rounds >= 3
    for stop in range(1, full.rounds):
        with pytest.raises(_binding.PmsError) as e:
            api.reduce_filtration(f, diagnostics=True, chain=False, max_rounds=stop)
        assert e.value.status == _binding.PMS_ERR_NOT_CONVERGED
        stats = api.round_stats(gpu)
        assert len(stats) == stop + 1 and stats[-1]["round"] == stop
        est = api.essential_estimate(f.m, gpu).cpu().numpy()
        assert np.all(est[ess_ref]), stop            # Ess is a subset of E^l
        assert stats[-1]["low_l1"] >= full.round_stats[-1]["low_l1"]


def test_diagnostics_errors(gpu):
    c, r, d = _dev([0, 0, 0, 2], [0, 1], [0, 0, 1], gpu)
    api.reduce(c, r, d)  # without diagnostics: no estimate to read
    with pytest.raises(_binding.PmsError):
        api.essential_estimate(3, gpu)
    res = api.reduce(c, r, d, diagnostics=True)
    assert res.essential_estimate.tolist() == [True, False, False]
    with pytest.raises(_binding.PmsError):
        api.essential_estimate(4, gpu)  # not the last reduction's m
    opt = _binding.load().pms_default_options()
    opt.diagnostics = 2
    ctx = api._ctx(gpu)
    bnd = _binding.PmsBoundary(3, c.data_ptr(), r.data_ptr(), d.data_ptr())
    out = torch.empty(3, dtype=torch.int32, device=gpu)
    rs = _binding.PmsResult()
    rs.low_star = out.data_ptr()
    assert _binding.load().pms_reduce(ctx, bnd, opt, rs) == _binding.PMS_ERR_INVALID_ARG
