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
    # left and beta (Defs. "left", "beta") from the builder: the oracle's on small
    # grids; on large ones the definitions evaluated with numpy scatters
    lb = f.left_beta()
    assert lb is not None
    left, beta = (t.cpu().numpy() for t in lb)
    if ref.m <= 200_000:
        want_left, want_beta = oracle.left_beta(ref.col_ptr, ref.rows)
    else:
        colidx = np.repeat(np.arange(ref.m), np.diff(ref.col_ptr))
        want_left = np.full(ref.m, ref.m, np.int64)
        np.minimum.at(want_left, ref.rows, colidx)
        want_left[want_left == ref.m] = -1
        hit = want_left[ref.rows] == colidx
        want_beta = np.full(ref.m, -1, np.int64)
        np.maximum.at(want_beta, colidx[hit], ref.rows[hit])
    assert np.array_equal(np.where(left == 0x7FFFFFFF, -1, left), want_left)
    assert np.array_equal(beta, want_beta)
    return f, ref


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 5), (2, 2, 2), (1, 3, 4), (5, 6, 7), (13, 9, 11), (3, 1, 7)])
def test_lowerstar_builder_matches_oracle(gpu, shape):
    _compare_lowerstar(synth.random_grid(21, shape), gpu)


def test_lowerstar_builder_ties_and_zero_signs(gpu):
    g = synth.random_grid(22, (7, 8, 9), ties=True)
    g[0, 0, :3] = np.array([0.0, -0.0, 0.0], np.float32)  # -0 and +0 are one value
    _compare_lowerstar(g, gpu)


@pytest.mark.parametrize("levels", [1, 2])
def test_lowerstar_builder_few_values_many_tiles(gpu, levels):
    """A constant grid and a two-valued one over 94 sort tiles (193 K keys):
    the order keys then differ only in their dimension, anchor and shape bits,
    so most sort passes move long runs of equal digits; the filtration must
    still be the oracle's."""
    rng = np.random.default_rng(31 + levels)
    g = rng.integers(0, levels, (23, 19, 17)).astype(np.float32)
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


# ---------------------------------------------------------------- Vietoris-Rips
def _vr_ref(cloud, thr, maxdim):
    if cloud.dtype == np.float32:
        return oracle.build_vr_f32(cloud, float(thr), maxdim)
    return oracle.build_vr_i32(cloud, int(thr), maxdim)


def _check_vr_segment(got, off, b, pbase, ref):
    lo, hi = off[b], off[b + 1]
    assert hi - lo == ref.m
    cp = got["col_ptr"][lo:hi + 1]
    assert np.array_equal(cp - cp[0], ref.col_ptr)
    rows = got["rows"][cp[0]:cp[-1]]
    assert np.array_equal(rows - lo, ref.rows)
    assert np.array_equal(got["dim"][lo:hi], ref.dim)
    gv = got["value"][lo:hi]
    if ref.value.dtype == np.float32:
        assert np.array_equal(gv.view(np.uint32), ref.value.view(np.uint32))
    else:
        assert np.array_equal(gv, ref.value)
    verts = got["verts"][lo:hi]
    assert np.array_equal(np.where(verts >= 0, verts - pbase, -1), ref.verts)
    # critical edge: the edge of the simplex latest in the filtration (edges:
    # themselves; triangles: their last facet)
    crit = got["crit"][lo:hi]
    want = np.full((ref.m, 2), -1, np.int64)
    e = ref.dim == 1
    want[e] = ref.verts[e][:, :2]
    t = np.nonzero(ref.dim == 2)[0]
    if t.size:
        last = ref.rows[ref.col_ptr[t + 1] - 1]
        want[t] = ref.verts[last][:, :2]
    q = np.nonzero(ref.dim == 3)[0]
    if q.size:  # tetrahedra: the latest of their six edges
        n = int(ref.verts.max()) + 1
        eid = np.full((n, n), -1, np.int64)
        ei = np.nonzero(e)[0]
        eid[ref.verts[ei, 0], ref.verts[ei, 1]] = ei
        V = ref.verts[q]
        best = np.stack([eid[V[:, u], V[:, w]] for u in range(4) for w in range(u + 1, 4)], 1).max(1)
        want[q] = ref.verts[best][:, :2]
    assert np.array_equal(np.where(crit >= 0, crit - pbase, -1), want)


def _compare_vr(clouds, thrs, maxdim, dev):
    f, off = api.build_vr([torch.as_tensor(c, device=dev) for c in clouds], thrs, maxdim)
    got = {k: v.cpu().numpy() for k, v in f.to_torch().items()}
    refs = [_vr_ref(c, t, maxdim) for c, t in zip(clouds, thrs)]
    pbase = 0
    for b, (c, ref) in enumerate(zip(clouds, refs)):
        _check_vr_segment(got, off, b, pbase, ref)
        pbase += len(c)
    return f, off, refs


def test_vr_builder_grid50_full(gpu):
    _compare_vr([synth.vr_grid_cloud()], [-1], 2, gpu)


def test_vr_builder_torus400_threshold(gpu):
    pts, thr = synth.vr_torus()
    _compare_vr([pts], [thr], 2, gpu)


def test_vr_builder_f32_circle(gpu):
    _compare_vr([synth.circle_batch(clouds=1)[0]], [-1.0], 2, gpu)


@pytest.mark.parametrize("maxdim", [0, 1, 2, 3])
def test_vr_builder_batch_mixed(gpu, maxdim):
    inst = synth.vr_batch(seed=31, count=6, n_range=(3, 40))
    clouds = [p for p, _ in inst] + [np.zeros((0, 3), np.int32), np.array([[5, 5, 5]], np.int32),
                                     np.array([[0, 0], [3, 4]], np.int32)]
    thrs = [t for _, t in inst] + [-1, -1, 24]
    _compare_vr(clouds, thrs, maxdim, gpu)


def test_vr_builder_ties(gpu):
    # many equal distances: the (value, dim, lex) tie-break decides the order
    g = np.array([[x, y] for x in range(5) for y in range(4)], np.int32)
    _compare_vr([g, g[:7]], [4, -1], 2, gpu)


def test_vr_builder_dim3_small(gpu):
    """Tetrahedra: a thresholded integer cloud, a full FP32 cloud, ties."""
    pts, _ = synth.vr_torus(seed=12, n=60)
    _compare_vr([pts], [synth.percentile_threshold_sqd(pts, 0.3)], 3, gpu)
    _compare_vr([synth.circle_batch(seed=13, clouds=1, n=14)[0]], [-1.0], 3, gpu)
    g = np.array([[x, y] for x in range(4) for y in range(4)], np.int32)
    _compare_vr([g, g[:9]], [5, -1], 3, gpu)


def test_vr_dim3_reduce_and_octahedron(gpu):
    """Dimension-3 batches reduce to the oracle's low* cloud by cloud; the
    octahedron's one persistent H2 class is born at 2 and dies at 4."""
    octa = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.int32)
    inst = synth.vr_batch(seed=33, count=5, n_range=(4, 30))
    clouds = [octa] + [p for p, _ in inst]
    thrs = [-1] + [t for _, t in inst]
    f, off, refs = _compare_vr(clouds, thrs, 3, gpu)
    res = api.reduce_filtration(f)
    low = res.low_star.cpu().numpy()
    for b, ref in enumerate(refs):
        want = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
        seg = low[off[b]:off[b + 1]]
        assert np.array_equal(np.where(seg >= 0, seg - off[b], -1), want), b
    v = f.to_torch()
    val, dm = v["value"].cpu().numpy(), v["dim"].cpu().numpy()
    pb, pd = res.pair_birth.cpu().numpy(), res.pair_death.cpu().numpy()
    octa_pairs = (pd < off[1]) & (dm[pb] == 2) & (val[pb] != val[pd])
    assert [(int(val[i]), int(val[j])) for i, j in zip(pb[octa_pairs], pd[octa_pairs])] == [(2, 4)]


def test_vr_torus400_dim3_full(gpu):
    """The 400-point torus at its 20th-percentile threshold taken to dimension
    3 (3.8e6 simplices, 3.5e6 tetrahedra): the built matrix and the reduced
    low* equal the oracle's element by element."""
    pts, thr = synth.vr_torus()
    f, off, refs = _compare_vr([pts], [thr], 3, gpu)
    assert int(np.sum(refs[0].dim == 3)) > 3_000_000
    res = api.reduce_filtration(f)
    want = oracle.reduce_twist(refs[0].col_ptr, refs[0].rows, refs[0].dim)
    assert np.array_equal(res.low_star.cpu().numpy(), want)
    b, d = oracle.pairs(want)
    assert np.array_equal(res.pair_birth.cpu().numpy(), b) and np.array_equal(res.pair_death.cpu().numpy(), d)
    assert np.array_equal(res.essential.cpu().numpy(), oracle.essential(want))


def test_vr_builder_rejects_maxdim4(gpu):
    with pytest.raises(_binding.PmsError):
        api.build_vr([torch.zeros((5, 2), dtype=torch.int32, device=gpu)], [-1], 4)


def test_vr_batch_reduce_f32_circles(gpu):
    x = synth.circle_batch(seed=41, clouds=5, n=36)
    f, off, refs = _compare_vr(list(x), [-1.0] * 5, 2, gpu)
    res = api.reduce_filtration(f)
    low = res.low_star.cpu().numpy()
    for b, ref in enumerate(refs):
        want = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
        seg = low[off[b]:off[b + 1]]
        assert np.array_equal(np.where(seg >= 0, seg - off[b], -1), want)


def test_vr_batch512_sampled(gpu):
    """The 512-cloud batch at full size: build and reduce on the device in one
    go, then check a sample of clouds (the largest, the smallest and a few
    others) against the oracle one by one."""
    inst = synth.vr_batch()
    clouds = [p for p, _ in inst]
    thrs = [t for _, t in inst]
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in clouds], thrs, 2)
    res = api.reduce_filtration(f)
    low = res.low_star.cpu().numpy()
    sizes = np.diff(off)
    rng = np.random.default_rng(0)
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes))} | set(rng.choice(len(clouds), 4, replace=False).tolist()))
    for b in pick:
        ref = oracle.build_vr_i32(clouds[b], thrs[b], 2)
        assert off[b + 1] - off[b] == ref.m
        want = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
        seg = low[off[b]:off[b + 1]]
        assert np.array_equal(np.where(seg >= 0, seg - off[b], -1), want), b


@pytest.mark.parametrize("maxdim", [2, 3])
def test_vr_builder_largest_clouds(gpu, maxdim):
    """The largest clouds accepted (511 integer points, 1023 FP32 points), two
    per batch: the lex field at its widest (n^3, or n^4 to dimension 3), the
    integer key a full 64 bits (sorted by key, then by cloud) and the FP32 key
    with its cloud bit exactly 64 (one pass); built and reduced as the oracle."""
    rng = np.random.default_rng(5)
    ints = [rng.integers(0, 1 << 16, (511, 3)).astype(np.int32) for _ in range(2)]
    flts = [rng.normal(0.0, 1.0, (1023, 2)).astype(np.float32) for _ in range(2)]
    thr_i = [synth.percentile_threshold_sqd(p, 0.01) for p in ints]
    thr_f = []
    for x in flts:
        d = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
        thr_f.append(float(np.quantile(d[np.triu_indices(len(x), 1)], 0.005)))
    for clouds, thrs in ((ints, thr_i), (flts, thr_f)):
        f, off, refs = _compare_vr(clouds, thrs, maxdim, gpu)
        low = api.reduce_filtration(f).low_star.cpu().numpy()
        for b, ref in enumerate(refs):
            want = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
            seg = low[off[b]:off[b + 1]]
            assert np.array_equal(np.where(seg >= 0, seg - off[b], -1), want), b


def test_vr_builder_rejects_large_cloud(gpu):
    with pytest.raises(_binding.PmsError):
        api.build_vr([torch.zeros((600, 2), dtype=torch.int32, device=gpu)], [-1], 2)


def test_reduce_batched_instance_offsets(gpu):
    """pms_reduce_batched: each instance's pairs and essential simplices are
    the contiguous slices its offsets name, equal to the oracle's for that
    cloud alone; pair_inst names the instance of every pair."""
    inst = synth.vr_batch(seed=33, count=7, n_range=(3, 36))
    clouds = [np.zeros((0, 3), np.int32)] + [p for p, _ in inst] + [np.array([[1, 2, 3]], np.int32)]
    thrs = [-1] + [t for _, t in inst] + [-1]
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in clouds], thrs, 2)
    res = api.reduce_batched(f, off)
    poff = res.inst_pair_off.cpu().numpy()
    eoff = res.inst_ess_off.cpu().numpy()
    pb, pd = res.pair_birth.cpu().numpy(), res.pair_death.cpu().numpy()
    ess = res.essential.cpu().numpy()
    pinst = res.pair_inst.cpu().numpy()
    assert poff[0] == 0 and poff[-1] == len(pd) and eoff[0] == 0 and eoff[-1] == len(ess)
    for b, (c, t) in enumerate(zip(clouds, thrs)):
        ref = oracle.build_vr_i32(c, t, 2)
        low = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
        rb, rd = oracle.pairs(low)
        re = oracle.essential(low)
        sl = slice(poff[b], poff[b + 1])
        assert np.array_equal(pb[sl] - off[b], rb) and np.array_equal(pd[sl] - off[b], rd), b
        assert np.array_equal(ess[eoff[b]:eoff[b + 1]] - off[b], re), b
        assert np.all(pinst[sl] == b)


def test_reduce_batched_rejects_bad_offsets(gpu):
    f, off = api.build_vr([torch.as_tensor(synth.vr_grid_cloud()[:20], device=gpu)], [-1], 2)
    for bad in ([0, off[1] - 1], [1, off[1]]):
        with pytest.raises(_binding.PmsError) as e:
            api.reduce_batched(f, bad)
        assert e.value.status == _binding.PMS_ERR_INVALID_ARG


def test_vr_circles64_batch_sampled(gpu):
    """The 64-cloud x 128-point FP32 batch (full 2-skeleton) at full size:
    built and reduced on the device in one go; three clouds' pairs and
    essential simplices checked against the oracle run on each alone."""
    x = synth.circle_batch()
    f, off = api.build_vr([torch.as_tensor(c, device=gpu) for c in x], [-1.0] * len(x), 2)
    res = api.reduce_batched(f, off)
    poff = res.inst_pair_off.cpu().numpy()
    eoff = res.inst_ess_off.cpu().numpy()
    pb, pd = res.pair_birth.cpu().numpy(), res.pair_death.cpu().numpy()
    ess = res.essential.cpu().numpy()
    for b in (0, 29, len(x) - 1):
        ref = oracle.build_vr_f32(x[b], -1.0, 2)
        assert off[b + 1] - off[b] == ref.m
        low = oracle.reduce_twist(ref.col_ptr, ref.rows, ref.dim)
        rb, rd = oracle.pairs(low)
        sl = slice(poff[b], poff[b + 1])
        assert np.array_equal(pb[sl] - off[b], rb) and np.array_equal(pd[sl] - off[b], rd), b
        assert np.array_equal(ess[eoff[b]:eoff[b + 1]] - off[b], oracle.essential(low)), b
