"""Pins of the CPU oracle against facts fixed by the paper and by the
mathematics (no GPU).  Each test would fail on a plausible slip in the
oracle: a dropped cancellation, an off-by-one low, a wrong facet, a
transposed order key, a wrong tie-break."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1708_04710_amd import synth
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _hand():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _hand(), ids=lambda e: e["name"])
def test_hand_examples(ex):
    cp = np.array(ex["col_ptr"], np.int64)
    rows = np.array(ex["rows"], np.int32)
    dim = np.array(ex["dim"], np.int8)
    for low in (oracle.reduce_standard(cp, rows), oracle.reduce_twist(cp, rows, dim)):
        assert low.tolist() == ex["low_star"]
        b, d = oracle.pairs(low)
        assert [[int(x), int(y)] for x, y in zip(b, d)] == ex["pairs"]
        assert oracle.essential(low).tolist() == ex["essential"]
    left, beta = oracle.left_beta(cp, rows)
    assert left.tolist() == ex["left"]
    assert beta.tolist() == ex["beta"]
    assert brute.rank_formula_low_star(cp, rows).tolist() == ex["low_star"]


# Known F2 Betti numbers of small triangulations (Sec. 2.1: b_p = rank H_p).
CIRCLE = [(0, 1), (1, 2), (0, 2)]
TETRA_BOUNDARY = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
TORUS7 = [tuple(sorted(((i) % 7, (i + 1) % 7, (i + 3) % 7))) for i in range(7)] + \
         [tuple(sorted(((i) % 7, (i + 2) % 7, (i + 3) % 7))) for i in range(7)]
RP2_6 = [(1, 2, 3), (1, 3, 4), (1, 4, 5), (1, 5, 6), (1, 2, 6), (2, 3, 5), (2, 4, 5), (2, 4, 6), (3, 4, 6),
         (3, 5, 6)]


@pytest.mark.parametrize("facets,betti", [
    (CIRCLE, [1, 1]), (TETRA_BOUNDARY, [1, 0, 1]), (TORUS7, [1, 2, 1]), (RP2_6, [1, 1, 1])],
    ids=["circle", "tetrahedron_boundary", "torus7", "rp2_6"])
def test_known_betti(facets, betti):
    cp, rows, dim, simp, _ = brute.complex_from_facets(facets)
    # the rank formula b_p = #K_p - rank d_p - rank d_{p+1} agrees with the textbook values
    assert brute.betti_by_rank(cp, rows, dim) == betti
    for low in (oracle.reduce_standard(cp, rows), oracle.reduce_twist(cp, rows, dim)):
        ess = oracle.essential(low)
        got = [int((dim[ess] == p).sum()) for p in range(len(betti))]
        assert got == betti


def test_rank_formula_random_small():
    """Alg. 1 = Alg. T = the pairing lemma on random compatible filtrations."""
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(120):
        cp, rows, dim, simp, val = brute.random_filtration(rng, n_vertices=int(rng.integers(3, 7)),
                                                           n_facets=int(rng.integers(1, 6)))
        if len(dim) > 48:
            continue
        ref = brute.rank_formula_low_star(cp, rows)
        assert np.array_equal(oracle.reduce_standard(cp, rows), ref)
        assert np.array_equal(oracle.reduce_twist(cp, rows, dim), ref)
        checked += 1
    assert checked > 80


def test_beta_bounds_random():
    """Thm. 'Properties of beta_j': P.5 beta_j <= low*(j) <= low(j), P.3 beta_j>0 => negative."""
    rng = np.random.default_rng(12)
    for _ in range(60):
        cp, rows, dim, _, _ = brute.random_filtration(rng, n_vertices=6, n_facets=5)
        low0 = np.array([rows[cp[j + 1] - 1] if cp[j + 1] > cp[j] else -1 for j in range(len(dim))])
        ls = oracle.reduce_standard(cp, rows)
        _, beta = oracle.left_beta(cp, rows)
        assert (beta <= ls).all() and (ls <= low0).all()
        assert (ls[beta >= 0] >= 0).all()


def test_euler_characteristic_and_order_independence():
    """sum (-1)^p #K_p = sum (-1)^p #Ess_p, and the (birth value, death value)
    multiset of pairs with death > birth does not depend on how ties in value
    are broken (low* is a property of the filtration, Sec. 2.3)."""
    rng = np.random.default_rng(13)
    for trial in range(30):
        facets = [tuple(sorted(rng.choice(7, size=int(rng.integers(2, 5)), replace=False).tolist()))
                  for _ in range(6)]
        values = rng.integers(0, 3, size=len(facets)).tolist()
        cp, rows, dim, simp, val = brute.complex_from_facets(facets, values)
        ls = oracle.reduce_standard(cp, rows)
        ess = oracle.essential(ls)
        chi_k = sum((-1) ** int(p) for p in dim)
        chi_e = sum((-1) ** int(dim[i]) for i in ess)
        assert chi_k == chi_e
        b, d = oracle.pairs(ls)
        ref = sorted((val[x], val[y], int(dim[x])) for x, y in zip(b, d) if val[y] > val[x])
        ref_ess = sorted((val[i], int(dim[i])) for i in ess)
        # random compatible re-ordering inside each value: (value, dim, random)
        perm_key = {s: rng.random() for s in simp}
        order = sorted(simp, key=lambda s: (val[simp.index(s)], len(s), perm_key[s]))
        index = {s: i for i, s in enumerate(order)}
        cp2, rows2 = [0], []
        for s in order:
            if len(s) > 1:
                rows2.extend(sorted(index[t] for t in itertools.combinations(s, len(s) - 1)))
            cp2.append(len(rows2))
        vv = [val[simp.index(s)] for s in order]
        dd = np.array([len(s) - 1 for s in order])
        ls2 = oracle.reduce_standard(np.array(cp2, np.int64), np.array(rows2, np.int32))
        b2, d2 = oracle.pairs(ls2)
        got = sorted((vv[x], vv[y], int(dd[x])) for x, y in zip(b2, d2) if vv[y] > vv[x])
        got_ess = sorted((vv[i], int(dd[i])) for i in oracle.essential(ls2))
        assert got == ref and got_ess == ref_ess


def test_rejects_incompatible():
    cp = np.array([0, 0, 0, 2], np.int64)
    with pytest.raises(oracle.OracleError):
        oracle.reduce_standard(cp, np.array([1, 0], np.int32))  # unsorted
    with pytest.raises(oracle.OracleError):
        oracle.reduce_standard(np.array([0, 1], np.int64), np.array([0], np.int32))  # row >= column
    with pytest.raises(oracle.OracleError):
        oracle.reduce_twist(np.array([0, 0, 1], np.int64), np.array([0], np.int32),
                            np.array([0, 2], np.int8))  # facet of wrong dimension


# ---------------------------------------------------------------- builders
def _check_boundary_by_definition(f):
    """Column j lists exactly the filtration indices of the codimension-1
    faces of simplex j (eq. 'def:boundary_matrix')."""
    index = {}
    for j in range(f.m):
        index[tuple(int(v) for v in f.verts[j] if v >= 0)] = j
    for j in range(f.m):
        s = tuple(int(v) for v in f.verts[j] if v >= 0)
        want = sorted(index[t] for t in itertools.combinations(s, len(s) - 1)) if len(s) > 1 else []
        assert f.rows[f.col_ptr[j]:f.col_ptr[j + 1]].tolist() == want


def _check_order(f):
    """(value, dim, lex) non-decreasing and strictly increasing overall."""
    keys = [(float(f.value[j]), int(f.dim[j]), tuple(int(v) for v in f.verts[j])) for j in range(f.m)]
    assert all(keys[j] < keys[j + 1] for j in range(len(keys) - 1))


def test_vr_int_counts_values_order():
    pts = synth.vr_grid_cloud(seed=7, n=14, side=64)
    thr = synth.percentile_threshold_sqd(pts, 0.5)
    f = oracle.build_vr_i32(pts, thr, 2)
    x = pts.astype(np.int64)
    sq = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    n = len(pts)
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if sq[a, b] <= thr]
    tris = [t for t in itertools.combinations(range(n), 3)
            if all(sq[p, q] <= thr for p, q in itertools.combinations(t, 2))]
    assert np.bincount(f.dim, minlength=3).tolist() == [n, len(edges), len(tris)]
    for j in range(f.m):
        s = [int(v) for v in f.verts[j] if v >= 0]
        want = max((sq[p, q] for p, q in itertools.combinations(s, 2)), default=0)
        assert f.value[j] == want
    _check_order(f)
    _check_boundary_by_definition(f)


def test_vr_full_closed_form_counts():
    pts = synth.vr_grid_cloud()
    f = oracle.build_vr_i32(pts, -1, 2)
    assert np.bincount(f.dim).tolist() == [50, math.comb(50, 2), math.comb(50, 3)]
    assert f.nnz == 2 * math.comb(50, 2) + 3 * math.comb(50, 3)


def test_vr_dim3_counts_values_order():
    """Tetrahedra (maxdim 3): every 4-clique of the threshold graph, its value
    the largest squared distance among its vertices, compatible order, and
    each column the four triangle faces (eq. 'def:boundary_matrix')."""
    pts = synth.vr_grid_cloud(seed=8, n=12, side=64)
    thr = synth.percentile_threshold_sqd(pts, 0.6)
    f = oracle.build_vr_i32(pts, thr, 3)
    x = pts.astype(np.int64)
    sq = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    n = len(pts)
    cliques = [[t for t in itertools.combinations(range(n), k)
                if all(sq[p, q] <= thr for p, q in itertools.combinations(t, 2))] for k in (2, 3, 4)]
    assert len(cliques[2]) > 0
    assert np.bincount(f.dim, minlength=4).tolist() == [n] + [len(c) for c in cliques]
    for j in range(f.m):
        s = [int(v) for v in f.verts[j] if v >= 0]
        assert f.value[j] == max((sq[p, q] for p, q in itertools.combinations(s, 2)), default=0)
    _check_order(f)
    _check_boundary_by_definition(f)


def test_vr_dim3_full_skeleton_homology():
    """The full complex on n points to dimension 3 is the 3-skeleton of the
    (n-1)-simplex: reduced homology only in degree 3, of rank C(n-1, 4), so
    the essential simplices are one vertex and C(n-1, 4) tetrahedra."""
    n = 9
    f = oracle.build_vr_i32(synth.vr_grid_cloud(seed=9, n=n), -1, 3)
    assert np.bincount(f.dim).tolist() == [n, math.comb(n, 2), math.comb(n, 3), math.comb(n, 4)]
    assert f.nnz == 2 * math.comb(n, 2) + 3 * math.comb(n, 3) + 4 * math.comb(n, 4)
    low = oracle.reduce_standard(f.col_ptr, f.rows)
    ess = oracle.essential(low)
    assert np.bincount(f.dim[ess], minlength=4).tolist() == [1, 0, 0, math.comb(n - 1, 4)]


def test_vr_octahedron_sphere():
    """The six points +-e_i: at squared scale 2 the complex is the octahedral
    2-sphere (no 4-clique avoids an antipodal pair), and at 4 the antipodal
    edges and the tetrahedra fill it, so the one H2 class with non-zero
    persistence is born at 2 and dies at 4."""
    pts = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.int32)
    f = oracle.build_vr_i32(pts, -1, 3)
    assert np.bincount(f.dim).tolist() == [6, 15, 20, 15]
    low = oracle.reduce_standard(f.col_ptr, f.rows)
    pairs = [(int(f.dim[low[j]]), int(f.value[low[j]]), int(f.value[j])) for j in range(f.m) if low[j] >= 0]
    assert sorted(p for p in pairs if p[1] != p[2]) == [(0, 0, 2)] * 5 + [(2, 2, 4)]
    assert [int(f.dim[i]) for i in oracle.essential(low)] == [0] + [3] * 5


@pytest.mark.parametrize("maxdim", [2, 3])
def test_vr_f32_values_stepwise(maxdim):
    x = synth.circle_batch(seed=9, clouds=1, n=12)[0]
    f = oracle.build_vr_f32(x, -1.0, maxdim)
    assert np.bincount(f.dim).tolist() == [12] + [math.comb(12, k) for k in range(2, maxdim + 2)]
    for j in range(f.m):
        s = [int(v) for v in f.verts[j] if v >= 0]
        best = np.float32(0)
        for p, q in itertools.combinations(s, 2):
            d0 = np.float32(x[p, 0] - x[q, 0])
            d1 = np.float32(x[p, 1] - x[q, 1])
            v = np.float32(np.float32(d0 * d0) + np.float32(d1 * d1))
            best = max(best, v)
        assert f.value[j] == best
    _check_order(f)


def _freudenthal_brute(nx, ny, nz):
    """Every vertex subset (size <= 4) of the grid that is a chain whose steps
    are non-zero 0/1 vectors with disjoint supports."""
    pts = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    vid = {p: p[0] + nx * (p[1] + ny * p[2]) for p in pts}
    out = set()
    for k in range(1, 5):
        for combo in itertools.combinations(pts, k):
            c = sorted(combo)
            # sort by coordinate sum: a chain must be increasing in every coordinate
            c = sorted(combo, key=lambda p: sum(p))
            ok = True
            used = [0, 0, 0]
            for a, b in zip(c, c[1:]):
                d = [b[t] - a[t] for t in range(3)]
                if any(v not in (0, 1) for v in d) or sum(d) == 0:
                    ok = False
                    break
                for t in range(3):
                    if d[t]:
                        if used[t]:
                            ok = False
                        used[t] = 1
            if ok:
                out.add(tuple(sorted(vid[p] for p in combo)))
    return out


@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 3, 3), (1, 3, 4), (3, 3, 3)])
def test_freudenthal_brute_force(shape):
    nz, ny, nx = shape
    g = synth.random_grid(1, shape)
    f = oracle.build_lowerstar(g)
    got = {tuple(int(v) for v in f.verts[j] if v >= 0) for j in range(f.m)}
    assert got == _freudenthal_brute(nx, ny, nz)
    flat = g.reshape(-1)
    for j in range(f.m):
        s = [int(v) for v in f.verts[j] if v >= 0]
        assert f.value[j] == flat[s].max()
    _check_order(f)
    _check_boundary_by_definition(f)


def test_freudenthal_closed_form_counts():
    n = 7
    f = oracle.build_lowerstar(synth.random_grid(2, (n, n, n)))
    V, E, T = n ** 3, 3 * n * n * (n - 1) + 3 * n * (n - 1) ** 2 + (n - 1) ** 3, 6 * (n - 1) ** 3
    F = 1 - V + E + T  # Euler characteristic of a 3-ball
    assert np.bincount(f.dim).tolist() == [V, E, F, T]


@pytest.mark.parametrize("kind", ["vr", "lowerstar", "lowerstar_ties"])
def test_h0_union_find(kind):
    if kind == "vr":
        pts = synth.vr_grid_cloud(seed=3, n=30, side=256)
        f = oracle.build_vr_i32(pts, synth.percentile_threshold_sqd(pts, 0.3), 2)
    else:
        f = oracle.build_lowerstar(synth.random_grid(4, (6, 7, 5), ties=kind.endswith("ties")))
    ls = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    b, d = oracle.pairs(ls)
    h0 = [(int(x), int(y)) for x, y in zip(b, d) if f.dim[x] == 0]
    assert h0 == brute.union_find_h0(f.dim, f.verts, f.m)


def test_lowerstar_ball_betti():
    f = oracle.build_lowerstar(synth.random_grid(5, (5, 6, 7)))
    ls = oracle.reduce_standard(f.col_ptr, f.rows)
    ess = oracle.essential(ls)
    assert ess.size == 1 and f.dim[ess[0]] == 0  # a 3-ball: b = (1, 0, 0, 0)
    assert np.array_equal(ls, oracle.reduce_twist(f.col_ptr, f.rows, f.dim))
