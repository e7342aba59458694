"""Independent checks used to pin the oracle (test code only).

None of these routines performs the column reduction that the oracle and
the GPU path perform; each one reaches the same facts by another road:

* ``rank_formula_low_star`` -- the pairing lemma: low*(j) = i iff
  r(i,j) - r(i+1,j) - r(i,j-1) + r(i+1,j-1) = 1, where r(i,j) is the F2 rank
  of the lower-left submatrix d[i:, :j+1].  Ranks of lower-left submatrices
  are unchanged by left-to-right column additions, and in a reduced matrix
  r(i,j) counts the columns k <= j with low*(k) >= i.
* ``betti_by_rank`` -- b_p = #K_p - rank d_p - rank d_{p+1} (Sec. 2.1).
* ``union_find_h0`` -- zero-dimensional pairs by Kruskal's union-find with the
  elder rule, in filtration order.
* ``complex_from_facets`` / ``random_filtration`` -- small complexes in a
  compatible order.
"""
from __future__ import annotations

import itertools

import numpy as np


def csc_to_bitcols(col_ptr, rows):
    m = len(col_ptr) - 1
    cols = []
    for j in range(m):
        v = 0
        for r in rows[col_ptr[j]:col_ptr[j + 1]]:
            v |= 1 << int(r)
        cols.append(v)
    return cols


def _rank_insert(basis: dict, v: int) -> bool:
    """Insert v into an F2 basis keyed by leading bit; True if independent."""
    while v:
        h = v.bit_length() - 1
        if h in basis:
            v ^= basis[h]
        else:
            basis[h] = v
            return True
    return False


def rank_formula_low_star(col_ptr, rows) -> np.ndarray:
    cols = csc_to_bitcols(col_ptr, rows)
    m = len(cols)
    # r[i][j+1] = rank of rows >= i, columns <= j
    r = np.zeros((m + 2, m + 1), dtype=np.int64)
    for i in range(m + 1):
        mask = ~((1 << i) - 1)
        basis = {}
        rank = 0
        for j in range(m):
            if _rank_insert(basis, cols[j] & mask):
                rank += 1
            r[i, j + 1] = rank
    low = np.full(m, -1, np.int32)
    for j in range(m):
        for i in range(m):
            x = r[i, j + 1] - r[i + 1, j + 1] - r[i, j] + r[i + 1, j]
            if x == 1:
                assert low[j] == -1
                low[j] = i
    return low


def f2_rank(vectors) -> int:
    basis = {}
    return sum(1 for v in vectors if _rank_insert(basis, v))


def betti_by_rank(col_ptr, rows, dim) -> list:
    cols = csc_to_bitcols(col_ptr, rows)
    dim = np.asarray(dim)
    top = int(dim.max()) if len(dim) else 0
    rank = [0] * (top + 2)
    for p in range(1, top + 1):
        rank[p] = f2_rank([cols[j] for j in range(len(cols)) if dim[j] == p])
    return [int((dim == p).sum()) - rank[p] - rank[p + 1] for p in range(top + 1)]


def complex_from_facets(facets, values=None):
    """All faces of the given simplices, ordered by (value, dim, lex) where the
    value of a face is the min over the facets containing it (default 0).
    Returns (col_ptr int64, rows int32, dim int8, simplices list, value list)."""
    val = {}
    for k, f in enumerate(facets):
        f = tuple(sorted(f))
        fv = 0 if values is None else values[k]
        for r in range(1, len(f) + 1):
            for s in itertools.combinations(f, r):
                val[s] = min(val.get(s, fv), fv)
    # make values monotone: a face never after a coface
    simp = sorted(val, key=lambda s: (len(s), s))
    for s in sorted(simp, key=lambda s: -len(s)):
        for t in itertools.combinations(s, len(s) - 1):
            if t:
                val[t] = min(val[t], val[s])
    order = sorted(simp, key=lambda s: (val[s], len(s) - 1, s))
    index = {s: i for i, s in enumerate(order)}
    col_ptr = [0]
    rows = []
    for s in order:
        if len(s) > 1:
            rows.extend(sorted(index[t] for t in itertools.combinations(s, len(s) - 1)))
        col_ptr.append(len(rows))
    dim = [len(s) - 1 for s in order]
    return (np.array(col_ptr, np.int64), np.array(rows, np.int32), np.array(dim, np.int8), order,
            [val[s] for s in order])


def random_filtration(rng, n_vertices=6, n_facets=6, max_dim=3, n_values=4):
    facets = []
    for _ in range(n_facets):
        k = int(rng.integers(1, max_dim + 2))
        k = min(k, n_vertices)
        facets.append(tuple(sorted(rng.choice(n_vertices, size=k, replace=False).tolist())))
    values = rng.integers(0, n_values, size=len(facets)).tolist()
    return complex_from_facets(facets, values)


def union_find_h0(dim, verts, m):
    """Pairs (birth vertex index, death edge index) of H0 by Kruskal with the
    elder rule; verts[j] lists the vertex ids of simplex j."""
    vindex = {}
    for j in range(m):
        if dim[j] == 0:
            vindex[int(verts[j][0])] = j
    parent = {v: v for v in vindex}
    oldest = {v: vindex[v] for v in vindex}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    pairs = []
    for j in range(m):
        if dim[j] != 1:
            continue
        a, b = find(int(verts[j][0])), find(int(verts[j][1]))
        if a == b:
            continue
        young, old = (a, b) if oldest[a] > oldest[b] else (b, a)
        pairs.append((oldest[young], j))
        parent[young] = old
    return sorted(pairs, key=lambda p: p[1])
