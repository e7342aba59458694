"""The workgroup kernel that solves a round's long chains by sweeps
(k_chain_solve) against the oracle on boundary matrices built to drive each
of its paths: more membership changes in one sweep than it applies at once
(the rest wait a sweep), more long pivots in one sweep than the workgroup
spreads (the rest go through one thread each), and a column touching more
rows than its LDS list holds (handed to the wavefront kernel).  Every chain
adds known pivots only, so the pivots it adds are the standard reduction's
(Alg. "Standard reduction") and low* must equal the oracle's.  The trace
counters show that each path ran."""
import re

import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import api

pytestmark = pytest.mark.gpu


def _csc(cols):
    cp = np.zeros(len(cols) + 1, np.int64)
    cp[1:] = np.cumsum([len(c) for c in cols])
    rows = np.concatenate([np.asarray(c, np.int32) for c in cols if len(c)])
    return cp, rows


def _many_changes():
    """3000 one-entry pivots {r} and two columns holding every row 0..2999:
    their chains add all 3000 pivots, which join the set in the first sweep."""
    n = 3000
    cols = [[] for _ in range(n)] + [[r] for r in range(n)]
    cols += [list(range(n)), list(range(n))]
    return _csc(cols)


def _many_long_pivots(seed):
    """100 pivots with eight entries below their lows 900..999, and targets
    holding every one of those lows plus a few low rows."""
    rng = np.random.default_rng(seed)
    cols = [[] for _ in range(1000)]
    for a in range(100):
        cols.append(sorted(rng.choice(900, 8, replace=False).tolist()) + [900 + a])
    for _ in range(3):
        extra = sorted(rng.choice(900, 5, replace=False).tolist())
        cols.append(extra + list(range(900, 1000)))
    return _csc(cols)


def _list_overflow(seed):
    """20 pivots with 800 entries each among 9900 rows: a target holding all
    their lows touches about 8000 distinct rows, more than the list holds."""
    rng = np.random.default_rng(seed)
    base = 9900
    cols = [[] for _ in range(base + 20)]
    for a in range(20):
        cols.append(sorted(rng.choice(base, 800, replace=False).tolist()) + [base + a])
    cols.append([3, 7] + [base + a for a in range(20)])
    return _csc(cols)


def _reduce(cp, rows, gpu, **kw):
    c = torch.as_tensor(cp, device=gpu)
    r = torch.as_tensor(rows, device=gpu)
    return api.reduce(c, r, None, validate=False, **kw)


def _check(res, ref):
    low = res.low_star.cpu().numpy()
    bad = np.nonzero(low != ref)[0]
    assert bad.size == 0, f"{bad.size} columns differ, first {bad[:5]}"
    b, d = oracle.pairs(ref)
    assert np.array_equal(res.pair_birth.cpu().numpy(), b)
    assert np.array_equal(res.pair_death.cpu().numpy(), d)
    assert np.array_equal(res.essential.cpu().numpy(), oracle.essential(ref))


def _counts(err, name):
    return [int(x) for x in re.findall(name + r" (\d+)", err)]


@pytest.fixture
def sweeps_always(gpu, monkeypatch):
    monkeypatch.setenv("PMS_TRACE", "1")
    api.set_tuning(dict(solve=1 << 30), device=gpu)
    yield
    api.set_tuning(None, device=gpu)


def test_more_changes_than_a_sweep_applies(gpu, capfd, sweeps_always):
    cp, rows = _many_changes()
    ref = oracle.reduce_standard(cp, rows)
    for kw in (dict(), dict(variant=1), dict(compression=False)):
        res = _reduce(cp, rows, gpu, **kw)
        _check(res, ref)
    err = capfd.readouterr().err
    assert sum(_counts(err, "deferred changes")) > 0, err[-2000:]
    assert sum(_counts(err, "solve: columns")) > 0


@pytest.mark.parametrize("seed", [1, 2])
def test_more_long_pivots_than_the_workgroup_spreads(gpu, capfd, sweeps_always, seed):
    cp, rows = _many_long_pivots(seed)
    ref = oracle.reduce_standard(cp, rows)
    for kw in (dict(), dict(variant=1)):
        _check(_reduce(cp, rows, gpu, **kw), ref)
    err = capfd.readouterr().err
    assert max(_counts(err, "long pivots")) > 64, err[-2000:]


@pytest.mark.parametrize("seed", [1, 2])
def test_list_overflow_hands_the_column_on(gpu, capfd, sweeps_always, seed):
    cp, rows = _list_overflow(seed)
    ref = oracle.reduce_standard(cp, rows)
    for kw in (dict(), dict(compression=False)):
        _check(_reduce(cp, rows, gpu, **kw), ref)
    err = capfd.readouterr().err
    assert sum(_counts(err, "to k_chain")) > 0, err[-2000:]
