"""Pins of the oracle's FP64 Vietoris-Rips builder (``oracle.build_vr_f64``),
the reference pipeline of the FP32 gradient checks (no GPU).

Each pin reaches its facts by another road than the builder:

* dyadic coordinates (multiples of 2^-10) make every FP64 squared distance
  exact, so values, order and boundary are compared with exact rational
  arithmetic and with the integer builder on the same points scaled by 2^10
  (a filtration whose order cannot change under a common scale);
* on general coordinates each value is within the forward error bound of a
  sum of D squares, gamma_D = D u / (1 - D u) with u = 2^-53, of the exact
  rational squared diameter, and the order is the (value, dim, lex) order;
* the loss sum over H1 pairs of (death - birth)^2 built from the oracle's
  values agrees with the analytic FP64 gradient (through the critical edge
  of each paired simplex, computed from the vertex tuples only) by central
  differences where the pairing stays put: the loss is a quartic polynomial
  of the coordinates there, so the difference quotient is exact up to
  rounding."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1708_04710_amd import synth

U = 2.0 ** -53


def _exact_sqd(x, a, b):
    return sum((Fraction(float(x[a, k])) - Fraction(float(x[b, k]))) ** 2 for k in range(x.shape[1]))


def _simplex(f, j):
    return tuple(int(v) for v in f.verts[j] if v >= 0)


def _check_boundary(f):
    index = {_simplex(f, j): j for j in range(f.m)}
    for j in range(f.m):
        s = _simplex(f, j)
        want = sorted(index[t] for t in itertools.combinations(s, len(s) - 1)) if len(s) > 1 else []
        assert f.rows[f.col_ptr[j]:f.col_ptr[j + 1]].tolist() == want


def _brute_cliques(n, ok, maxdim):
    out = [(a,) for a in range(n)]
    for k in range(2, maxdim + 2):
        out += [t for t in itertools.combinations(range(n), k)
                if all(ok(p, q) for p, q in itertools.combinations(t, 2))]
    return out


@pytest.mark.parametrize("maxdim", [2, 3])
def test_vr_f64_dyadic_exact(maxdim):
    """Coordinates k / 1024 with |k| <= 2048: differences, squares and their
    sums are exact in FP64.  Values equal the exact squared diameters; the
    simplices are the cliques of the threshold graph in (value, dim, lex)
    order; ties (frequent on this coarse grid) fall to the lexicographic
    vertex tuple; the result is the integer builder's filtration of the
    points times 1024, values scaled by 2^20."""
    rng = np.random.default_rng(11)
    n, D = 11, 3
    k = rng.integers(-2048, 2049, size=(n, D))
    x = k.astype(np.float64) / 1024.0
    sq = {(a, b): _exact_sqd(x, a, b) for a in range(n) for b in range(n)}
    vals = sorted(sq[a, b] for a in range(n) for b in range(a + 1, n))
    thr = vals[int(0.6 * len(vals))]
    f = oracle.build_vr_f64(x, float(thr), maxdim)
    cl = _brute_cliques(n, lambda p, q: sq[p, q] <= thr, maxdim)

    def value(s):
        return max((sq[p, q] for p, q in itertools.combinations(s, 2)), default=Fraction(0))

    want = sorted(cl, key=lambda s: (value(s), len(s) - 1, s))
    assert [_simplex(f, j) for j in range(f.m)] == want
    assert all(Fraction(float(f.value[j])) == value(want[j]) for j in range(f.m))
    assert np.array_equal(f.dim, np.array([len(s) - 1 for s in want], np.int8))
    _check_boundary(f)
    # the integer builder on the scaled points: same order, values x 2^20
    fi = oracle.build_vr_i32(k.astype(np.int32), int(thr * (1 << 20)), maxdim)
    assert np.array_equal(fi.col_ptr, f.col_ptr) and np.array_equal(fi.rows, f.rows)
    assert np.array_equal(fi.verts, f.verts) and np.array_equal(fi.dim, f.dim)
    assert np.array_equal(fi.value, (f.value * (1 << 20)).astype(np.int64))


def test_vr_f64_rounding_bound_and_order():
    """Gaussian coordinates in R^4: each value within gamma_4 of the exact
    rational squared diameter, the full 2-skeleton's counts, and the order
    strictly increasing in (value, dim, lex)."""
    rng = np.random.default_rng(12)
    n, D = 10, 4
    x = rng.normal(size=(n, D))
    f = oracle.build_vr_f64(x, -1.0, 2)
    assert np.bincount(f.dim).tolist() == [n, math.comb(n, 2), math.comb(n, 3)]
    g = D * U / (1 - D * U)
    for j in range(f.m):
        s = _simplex(f, j)
        exact = max((_exact_sqd(x, p, q) for p, q in itertools.combinations(s, 2)), default=Fraction(0))
        assert abs(Fraction(float(f.value[j])) - exact) <= Fraction(g) * exact
    keys = [(float(f.value[j]), int(f.dim[j]), _simplex(f, j)) for j in range(f.m)]
    assert all(keys[j] < keys[j + 1] for j in range(f.m - 1))
    _check_boundary(f)


def test_vr_f64_threshold_keeps_ties():
    """A threshold equal to an attained squared distance keeps the simplices
    at that value (<=), and a threshold just below it drops them."""
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    f = oracle.build_vr_f64(x, 1.0, 2)
    assert np.bincount(f.dim, minlength=3).tolist() == [4, 4, 0]
    f = oracle.build_vr_f64(x, 2.0, 2)
    assert np.bincount(f.dim, minlength=3).tolist() == [4, 6, 4]
    f = oracle.build_vr_f64(x, np.nextafter(1.0, 0.0), 2)
    assert np.bincount(f.dim, minlength=3).tolist() == [4, 0, 0]


def _crit_edge_vertices(f, j):
    """The two vertices of simplex j's edge of largest squared length, the
    latest such edge in (value, lex) order: the edge whose value is j's."""
    s = _simplex(f, j)
    if len(s) == 2:
        return s
    index = {_simplex(f, t): t for t in range(f.m) if f.dim[t] == 1}
    return max(((p, q) for p, q in itertools.combinations(s, 2)), key=lambda e: index[e])


def _loss_and_signature(x):
    f = oracle.build_vr_f64(x, -1.0, 2)
    low = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    b, d = oracle.pairs(low)
    h1 = f.dim[b] == 1
    pers = f.value[d[h1]] - f.value[b[h1]]
    sig = sorted((_simplex(f, bi), _crit_edge_vertices(f, di)) for bi, di in zip(b[h1], d[h1]))
    return float((pers * pers).sum()), sig, f, b[h1], d[h1]


def test_vr_f64_loss_gradient_by_central_differences():
    """d/dx of sum over H1 pairs of (death - birth)^2, analytic (through the
    critical edges, from vertex tuples only) against central differences of
    the loss built from the oracle's values, h = 1e-6, to 1e-7 of the
    largest gradient entry, on every coordinate where the H1 signature is the
    same at x - h, x and x + h."""
    x = synth.circle_batch(seed=13, clouds=1, n=16)[0].astype(np.float64)
    loss0, sig0, f, hb, hd = _loss_and_signature(x)
    assert len(sig0) > 0 and loss0 > 0
    grad = np.zeros_like(x)
    for bi, di in zip(hb, hd):
        ba, bb = _crit_edge_vertices(f, bi)
        da, db = _crit_edge_vertices(f, di)
        pd = x[da] - x[db]
        pb = x[ba] - x[bb]
        pers = pd @ pd - pb @ pb
        grad[da] += 2 * pers * 2 * pd
        grad[db] -= 2 * pers * 2 * pd
        grad[ba] -= 2 * pers * 2 * pb
        grad[bb] += 2 * pers * 2 * pb
    scale = np.abs(grad).max()
    assert scale > 0
    h = 1e-6
    checked = 0
    for k in range(x.size):
        xp, xm = x.copy().reshape(-1), x.copy().reshape(-1)
        xp[k] += h
        xm[k] -= h
        lp, sp, *_ = _loss_and_signature(xp.reshape(x.shape))
        lm, sm, *_ = _loss_and_signature(xm.reshape(x.shape))
        if sp != sig0 or sm != sig0:
            continue
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad.reshape(-1)[k]) <= 1e-7 * scale, (k, fd, grad.reshape(-1)[k])
        checked += 1
    assert checked >= x.size // 2, checked
