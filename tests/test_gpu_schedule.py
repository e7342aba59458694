"""Options that change which columns work when leave low* unchanged
(low* is a property of the complex, Sec. 2.3):

* ``c8``: clearing by local compression every round (Sec. 3.2, Lemma
  "Clearing by local compression" and its Corollary, the case L_j = {0}),
  per complex of a batch;
* ``sweep=1``: the twist order (Alg. "Standard reduction with a twist"): one
  dimension at a time, from the top down;
* ``priority`` 0 / 1 / 2 with ``round_budget``: at most that many columns
  add per round (Sec. 3.4, fewer processors than colliding columns), chosen
  in column order, from the largest sets N first, or known negative first.

Each is compared with the oracle on random small filtrations (invariant
checks on), on a lower-star grid and on every instance of the circle batch;
c8 and the budget are also checked to act (columns cleared; additions per
round within the budget)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import _binding, api, synth
from tests import brute
from tests.test_gpu_full_batches import _check_every_instance
from tests.test_gpu_invariants import _check

pytestmark = pytest.mark.gpu

OPTS = [dict(c8=True), dict(sweep=1), dict(c8=True, sweep=1), dict(round_budget=1),
        dict(round_budget=3, priority=1), dict(round_budget=2, priority=2),
        dict(round_budget=5, priority=1, chain=False, compression=False),
        dict(c8=True, sweep=1, round_budget=4, priority=2, variant=1),
        dict(c8=True, variant=1, tail_active=0), dict(sweep=1, chain=False, round_budget=1, priority=1)]


@pytest.mark.parametrize("chunk", range(2))
def test_fuzz_schedules_with_invariants(gpu, chunk):
    rng = np.random.default_rng(9100 + chunk)
    for t in range(1000):
        cp, rows, dim, _, _ = brute.random_filtration(rng, n_vertices=int(rng.integers(2, 10)),
                                                      n_facets=int(rng.integers(1, 10)),
                                                      max_dim=int(rng.integers(1, 4)))
        ref = oracle.reduce_standard(cp, rows)
        kw = OPTS[t % len(OPTS)]
        c = torch.as_tensor(cp, device=gpu)
        r = torch.as_tensor(rows if rows.size else np.zeros(1, np.int32), device=gpu)
        d = torch.as_tensor(dim, device=gpu)
        _check(api.reduce(c, r, d, debug_invariants=True, **kw), ref)


@pytest.mark.parametrize("kw", [dict(c8=True), dict(sweep=1), dict(sweep=1, variant=1),
                                dict(c8=True, sweep=1, chain=False),
                                dict(round_budget=5000, priority=1), dict(round_budget=5000, priority=2)])
def test_lowerstar24_schedules(gpu, kw):
    g = synth.gaussian_field(seed=21, n=24)
    f = api.build_lowerstar(torch.as_tensor(g, device=gpu))
    res = api.reduce_filtration(f, debug_invariants=True, **kw)
    ref_f = oracle.build_lowerstar(g)
    _check(res, oracle.reduce_twist(ref_f.col_ptr, ref_f.rows, ref_f.dim))


@pytest.mark.parametrize("kw", [dict(c8=True), dict(sweep=1), dict(c8=True, sweep=1)])
def test_circles64_every_cloud_schedules(gpu, kw):
    x = synth.circle_batch()
    _check_every_instance(list(x), [-1.0] * len(x), gpu, **kw)


def test_c8_clears_positive_triangles(gpu):
    """On full VR 2-skeletons (b1 = 0) every edge is paired eventually; the
    triangles still unreduced then have L_j = {0} and are cleared."""
    x = synth.circle_batch()[:8]
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in x], [-1.0] * len(x), 2)
    base = api.reduce_batched(f, off, diagnostics=True)
    res = api.reduce_batched(f, off, c8=True, diagnostics=True)
    stats = api.round_stats(gpu)
    cleared = sum(s["c8_cleared"] for s in stats)
    assert cleared > 0
    assert torch.equal(res.low_star, base.low_star)
    assert res.additions < base.additions


@pytest.mark.parametrize("priority", [0, 1, 2])
def test_round_budget_caps_additions(gpu, priority):
    """Without chaining a column adds at most once per round, so a round's
    additions are at most the budget; low* is unchanged and more rounds run."""
    x = synth.circle_batch()[:1, :40]  # 40 points: 9880 triangles
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in x], [-1.0], 2)
    base = api.reduce_batched(f, off, chain=False)
    budget = 200
    res = api.reduce_batched(f, off, chain=False, round_budget=budget, priority=priority, diagnostics=True)
    stats = api.round_stats(gpu)
    assert max(s["additions"] for s in stats) <= budget
    assert torch.equal(res.low_star, base.low_star)
    assert res.rounds > base.rounds


def test_schedule_options_rejected(gpu):
    cp, rows, dim, _, _ = brute.random_filtration(np.random.default_rng(5), n_vertices=5, n_facets=4, max_dim=2)
    c = torch.as_tensor(cp, device=gpu)
    r = torch.as_tensor(rows, device=gpu)
    for kw in (dict(c8=True), dict(sweep=1)):  # need dim
        with pytest.raises(_binding.PmsError) as e:
            api.reduce(c, r, None, **kw)
        assert e.value.status == _binding.PMS_ERR_INVALID_ARG
    d = torch.as_tensor(dim, device=gpu)
    for kw in (dict(sweep=2), dict(priority=3), dict(round_budget=-1)):
        with pytest.raises(_binding.PmsError) as e:
            api.reduce(c, r, d, **kw)
        assert e.value.status == _binding.PMS_ERR_INVALID_ARG
