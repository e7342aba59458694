"""The reduction with ``debug_invariants`` on: every property the theory
guarantees (lows never rise, Sec. 3.1; beta_j <= low(j) and beta_j defined
=> column j never zero, Thm. "Properties of beta_j" P.5 / P.3; pivots frozen;
one writer per column per kernel; Ess a subset of every E^l, Lemma
"Essential estimation"; low* the last low) is checked on the device after
Phase 0, after every writing kernel and after every round, while the result
is compared with the oracle.

* 10^4 random small filtrations through the C ABI, in four chunks, with
  the options rotating over every variant, compression, chaining and tail
  setting, half of them without dimensions;
* the full-size workloads: the 64^3 lower-star grid (both Phase II
  variants), the 64 x 128 circle batch and the 512-cloud batch, plus the
  paper's own schedule (pivot-gated, no chaining) on a 24^3 grid.

The detectors themselves are checked by ``pms_selftest`` on fabricated
states that each break one property (``test_gpu_reduce``'s self-test)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import api, synth
from tests import brute

pytestmark = pytest.mark.gpu

OPTS = [dict(), dict(variant=1), dict(compression=False), dict(chain=False), dict(tail_active=0),
        dict(variant=1, compression=False, chain=False), dict(variant=1, tail_active=1 << 30),
        dict(chain=False, compression=False)]


def _check(res, ref):
    low = res.low_star.cpu().numpy()
    assert np.array_equal(low, ref)
    b, d = oracle.pairs(ref)
    assert np.array_equal(res.pair_birth.cpu().numpy(), b)
    assert np.array_equal(res.pair_death.cpu().numpy(), d)
    assert np.array_equal(res.essential.cpu().numpy(), oracle.essential(ref))


@pytest.mark.parametrize("chunk", range(4))
def test_fuzz_10k_with_invariants(gpu, chunk):
    rng = np.random.default_rng(9000 + chunk)
    for t in range(2500):
        cp, rows, dim, _, _ = brute.random_filtration(rng, n_vertices=int(rng.integers(2, 10)),
                                                      n_facets=int(rng.integers(1, 10)),
                                                      max_dim=int(rng.integers(1, 4)))
        ref = oracle.reduce_standard(cp, rows)
        kw = OPTS[t % len(OPTS)]
        c = torch.as_tensor(cp, device=gpu)
        r = torch.as_tensor(rows if rows.size else np.zeros(1, np.int32), device=gpu)
        d = torch.as_tensor(dim, device=gpu) if t % 2 else None
        _check(api.reduce(c, r, d, debug_invariants=True, **kw), ref)


@pytest.mark.parametrize("variant", [0, 1])
def test_invariants_lowerstar64(gpu, variant):
    g = synth.gaussian_field()
    f = api.build_lowerstar(torch.as_tensor(g, device=gpu))
    res = api.reduce_filtration(f, variant=variant, debug_invariants=True)
    ref_f = oracle.build_lowerstar(g)
    _check(res, oracle.reduce_twist(ref_f.col_ptr, ref_f.rows, ref_f.dim))


def test_invariants_paper_schedule(gpu):
    """Alg. "Parallel multi-scale reduction" as printed: pivot-gated Phase II,
    one addition per column per round (hundreds of rounds)."""
    g = synth.gaussian_field(seed=15, n=24)
    f = api.build_lowerstar(torch.as_tensor(g, device=gpu))
    res = api.reduce_filtration(f, variant=1, chain=False, tail_active=0, debug_invariants=True)
    ref_f = oracle.build_lowerstar(g)
    _check(res, oracle.reduce_twist(ref_f.col_ptr, ref_f.rows, ref_f.dim))
    assert res.rounds > 20


def test_invariants_batches(gpu):
    x = synth.circle_batch()
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in x], [-1.0] * len(x), 2)
    api.reduce_batched(f, off, debug_invariants=True)
    api.reduce_batched(f, off, variant=1, debug_invariants=True)
    inst = synth.vr_batch()
    f, off = api.build_vr([torch.as_tensor(p, device=gpu) for p, _ in inst], [t for _, t in inst], 2)
    api.reduce_batched(f, off, debug_invariants=True)
