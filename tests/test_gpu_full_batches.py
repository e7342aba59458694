"""Every instance of the two batched workloads at full size, through the
batched entry point (``pms_reduce_batched``), against the oracle run on each
cloud alone:

* 512 integer clouds (n ~ U{32..256}, D ~ U{2..8}, cube / noisy sphere /
  noisy circle, own 30th-percentile threshold): every cloud's filtration
  (byte for byte), low*, pairs, essential simplices, per-instance offsets and
  pair instances;
* 64 FP32 noisy circles x 128 points, full 2-skeleton: the same per cloud,
  and the FP32 gradient of sum over H1 pairs of (death - birth)^2 of every
  cloud against the FP64 gradient on the oracle's pairing (norm-wise
  relative error <= 1e-5; the maximum and median are printed).

The oracle is plain C behind ctypes, which releases the GIL, so the clouds
are checked by a thread pool of host cores."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_1708_04710_amd import api, synth
from tests.test_gpu_build import _check_vr_segment
from tests.test_gpu_grad import TOL, _gpu_vr_grad, _vr_loss_grad64

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, os.cpu_count() or 1))


def _oracle_cloud(args):
    cloud, thr = args
    f = oracle.build_vr_f32(cloud, float(thr), 2) if cloud.dtype == np.float32 else \
        oracle.build_vr_i32(cloud, int(thr), 2)
    low = oracle.reduce_twist(f.col_ptr, f.rows, f.dim)
    return f, low


def _refs(clouds, thrs):
    oracle._load()
    with ThreadPoolExecutor(WORKERS) as ex:
        return list(ex.map(_oracle_cloud, zip(clouds, thrs)))


def _check_every_instance(clouds, thrs, dev, **kw):
    f, off = api.build_vr([torch.as_tensor(c, device=dev) for c in clouds], thrs, 2)
    got_f = {k: v.cpu().numpy() for k, v in f.to_torch().items()}
    refs = _refs(clouds, thrs)
    pbase = 0
    for b, (c, (rf, _)) in enumerate(zip(clouds, refs)):
        _check_vr_segment(got_f, off, b, pbase, rf)
        pbase += len(c)
    for variant in (0, 1):
        res = api.reduce_batched(f, off, variant=variant, **kw)
        low = res.low_star.cpu().numpy()
        poff = res.inst_pair_off.cpu().numpy()
        eoff = res.inst_ess_off.cpu().numpy()
        pb, pd = res.pair_birth.cpu().numpy(), res.pair_death.cpu().numpy()
        ess = res.essential.cpu().numpy()
        pinst = res.pair_inst.cpu().numpy()
        assert poff[0] == 0 and poff[-1] == len(pd) and eoff[0] == 0 and eoff[-1] == len(ess)
        for b, (_, want) in enumerate(refs):
            seg = low[off[b]:off[b + 1]]
            assert np.array_equal(np.where(seg >= 0, seg - off[b], -1), want), (variant, b)
            rb, rd = oracle.pairs(want)
            sl = slice(poff[b], poff[b + 1])
            assert np.array_equal(pb[sl] - off[b], rb) and np.array_equal(pd[sl] - off[b], rd), (variant, b)
            assert np.array_equal(ess[eoff[b]:eoff[b + 1]] - off[b], oracle.essential(want)), (variant, b)
            assert np.all(pinst[sl] == b), (variant, b)
    return refs


def test_vr_batch512_every_cloud(gpu):
    inst = synth.vr_batch()
    _check_every_instance([p for p, _ in inst], [t for _, t in inst], gpu)


def test_vr_circles64_every_cloud(gpu):
    x = synth.circle_batch()
    _check_every_instance(list(x), [-1.0] * len(x), gpu)


def test_vr_circles64_grad_every_cloud(gpu):
    """FP32 gradients of the 64-cloud batch in one pass; each cloud against
    the FP64 gradient on the oracle's pairing."""
    x = synth.circle_batch()
    got = _gpu_vr_grad(x, gpu)
    oracle._load()
    with ThreadPoolExecutor(WORKERS) as ex:
        refs = list(ex.map(lambda c: _vr_loss_grad64(x[c])[1], range(len(x))))
    errs = np.array([np.linalg.norm(got[c] - refs[c]) / np.linalg.norm(refs[c]) for c in range(len(x))])
    print(f"\nFP32 vs FP64 gradient, 64 clouds: max rel. err {errs.max():.3e}, median {np.median(errs):.3e}")
    assert errs.max() <= TOL, (int(errs.argmax()), float(errs.max()))
