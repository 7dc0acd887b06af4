"""GPU parity of the multi-instance batched launch (pfsp_multi_*): every
instance's rows must equal the oracle on that instance, bit for bit, across
graph replays, launch shapes and the autotuner's choice."""
import numpy as np
import pytest

import oracle
from paper_2012_09511_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = binding.Context(0)
    yield c
    c.close()


def _batch(insts, per, seed, stride):
    perms, d1s, d2s, seg = [], [], [], [0]
    for k, (n, m, p) in enumerate(insts):
        cnt = per[k]
        perm, d1, d2 = inputs.random_pool(n, cnt, seed + k)
        pad = np.zeros((cnt, stride), dtype=np.uint8)
        pad[:, :n] = perm
        perms.append(pad)
        d1s.append(d1)
        d2s.append(d2)
        seg.append(seg[-1] + cnt)
    return np.concatenate(perms), np.concatenate(d1s), np.concatenate(d2s), np.array(seg)


def _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, kind):
    lb, pr, dr = lb.cpu().numpy(), pr.cpu().numpy(), dr.cpu().numpy()
    stride = perm.shape[1]
    for k, (n, m, p) in enumerate(insts):
        a, b = seg[k], seg[k + 1]
        if a == b:
            continue
        olb, opr, odr = oracle.bound_children(p, perm[a:b, :n], d1[a:b], d2[a:b], kind, ub[k],
                                              threads=8)
        np.testing.assert_array_equal(lb[a:b, :, :n], olb)
        np.testing.assert_array_equal(pr[a:b, :, :n], opr)
        np.testing.assert_array_equal(dr[a:b], odr)
        assert (lb[a:b, :, n:] == binding.INT32_MAX).all() and (pr[a:b, :, n:] == 1).all()


def _dev(ctx, *a):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(x)).to(ctx.device) for x in a]


@pytest.mark.parametrize("kind", [binding.LB1, binding.LB2_FULL])
def test_mixed_instances(ctx, kind):
    """(n, m) round-robin over {20, 50, 100} x {5, 10, 20}, every fourth instance
    job-correlated; includes an empty segment."""
    insts = inputs.mixed_instances(9, 1234)
    per = [40, 7, 0, 25, 3, 30, 2, 12, 5]
    per = [x if insts[i][0] < 100 else min(x, 3) for i, x in enumerate(per)]
    stride = max(n for n, _, _ in insts)
    perm, d1, d2, seg = _batch(insts, per, 55, stride)
    ub = np.array([1400 + 300 * i for i in range(len(insts))], dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    dev = _dev(ctx, perm, d1, d2)
    out = mt.outputs(len(perm), stride)
    for rep in range(2):     # capture, then a replay
        lb, pr, dr = mt.bound(*dev, seg, ub, kind, out=out)
        _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, kind)
    mt.set_shape(tile=16, waves_small=2, waves_large=1, blocks_per_cu=1)
    lb, pr, dr = mt.bound(*dev, seg, ub, kind, out=out)
    _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, kind)
    mt.close()


def test_autotune_keeps_results(ctx):
    insts = [(20, 20, inputs.instance(20, 20, 7)), (20, 5, inputs.instance(20, 5, 8)),
             (50, 10, inputs.instance(50, 10, 9))]
    per = [300, 200, 20]
    perm, d1, d2, seg = _batch(insts, per, 77, 50)
    ub = np.array([2400, 1500, 3200], dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    dev = _dev(ctx, perm, d1, d2)
    rep = mt.autotune(*dev, seg, ub, binding.LB2_FULL, reps=1)
    assert rep["best"]["ms"] > 0 and rep["candidates"] > 10
    lb, pr, dr = mt.bound(*dev, seg, ub, binding.LB2_FULL)
    _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, binding.LB2_FULL)
    mt.close()


def test_class_with_fewer_machines_than_batch(ctx):
    """The n <= 64 class holds only an m = 10 instance while the batch's largest
    m is 20: the costs rows must be read with the batch's stride."""
    insts = [(20, 20, inputs.instance(20, 20, 17)), (50, 10, inputs.instance(50, 10, 19))]
    perm, d1, d2, seg = _batch(insts, [64, 30], 91, 50)
    ub = np.array([2400, 3200], dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    lb, pr, dr = mt.bound(*_dev(ctx, perm, d1, d2), seg, ub, binding.LB2_FULL)
    _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, binding.LB2_FULL)
    mt.close()


def test_wide_classes(ctx):
    """Instances of every class in one batch: n <= 20 (quick), 20 < n <= 64 and
    64 < n <= 128 with 16-bit X (wide), n <= 64 with times past the 16-bit
    limit (scan kernel) and n > 128 (generic); root and leaf-parent rows."""
    rng = np.random.default_rng(4242)
    shapes = [(12, 6, 99), (25, 5, 99), (50, 20, 99), (64, 3, 99), (65, 11, 99),
              (100, 20, 273), (128, 4, 99), (40, 10, 900), (130, 3, 99)]
    insts = [(n, m, rng.integers(1, hi + 1, size=(n, m)).astype(np.int32)) for n, m, hi in shapes]
    per = [50, 40, 12, 30, 10, 4, 6, 20, 3]
    stride = max(n for n, _, _ in insts)
    perm, d1, d2, seg = _batch(insts, per, 303, stride)
    for k, (n, m, p) in enumerate(insts):   # first row: the root; second: one job left
        a = seg[k]
        d1[a], d2[a] = 0, 0
        d1[a + 1], d2[a + 1] = n - 1, 0
    ub = np.array([3000 + 500 * k for k in range(len(insts))], dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    dev = _dev(ctx, perm, d1, d2)
    for rep in range(2):
        lb, pr, dr = mt.bound(*dev, seg, ub, binding.LB2_FULL)
        _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, binding.LB2_FULL)
    mt.set_shape(tile=8, waves_small=3, waves_large=2, blocks_per_cu=1)
    lb, pr, dr = mt.bound(*dev, seg, ub, binding.LB2_FULL)
    _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, binding.LB2_FULL)
    mt.close()


def test_invalid_rows_and_instance_blocks(ctx):
    """Segments long enough for blocks of one instance (the costs pass stages
    that instance's times) beside blocks that straddle two, with rows that are
    not valid nodes (d1 + d2 = n, a repeated job, a job id out of range): those
    come back fully pruned and raise the context's error, the others equal the
    oracle."""
    import torch
    insts = [(20, 20, inputs.instance(20, 20, 27)), (50, 10, inputs.instance(50, 10, 28)),
             (100, 5, inputs.instance(100, 5, 29)), (7, 3, inputs.instance(7, 3, 30)),
             (40, 4, inputs.instance(40, 4, 31))]
    per = [300, 261, 140, 5, 97]
    stride = 100
    perm, d1, d2, seg = _batch(insts, per, 131, stride)
    bad = []
    for k, (n, m, p) in enumerate(insts):
        a = seg[k]
        d1[a + 1], d2[a + 1] = n - 2, 2
        perm[a + 2, 1] = perm[a + 2, 0]
        perm[a + 3, n - 1] = 200
        bad += [a + 1, a + 2, a + 3]
    good = np.setdiff1d(np.arange(seg[-1]), bad)
    ub = np.array([2400, 3200, 6000, 900, 2300], dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    lb, pr, dr = mt.bound(*_dev(ctx, perm, d1, d2), seg, ub, binding.LB2_FULL)
    torch.cuda.synchronize()
    with pytest.raises(binding.PfspError):
        ctx.check()
    lb, pr, dr = lb.cpu().numpy(), pr.cpu().numpy(), dr.cpu().numpy()
    assert (lb[bad] == binding.INT32_MAX).all() and (pr[bad] == 1).all() and (dr[bad] == 0).all()
    for k, (n, m, p) in enumerate(insts):
        rows = good[(good >= seg[k]) & (good < seg[k + 1])]
        olb, opr, odr = oracle.bound_children(p, perm[rows, :n], d1[rows], d2[rows],
                                              binding.LB2_FULL, ub[k], threads=8)
        np.testing.assert_array_equal(lb[rows, :, :n], olb)
        np.testing.assert_array_equal(pr[rows, :, :n], opr)
        np.testing.assert_array_equal(dr[rows], odr)
    mt.close()
    ctx.check()   # the condition was cleared


def test_costs_pass_at_its_limits(ctx):
    """The multi-instance costs pass at the sizes its register and row-mask
    layouts end at: a 128-job instance, a 32-machine one (32 registers per
    cost vector) and a two-machine one in one batch, with root rows and
    rows of one job left."""
    rng = np.random.default_rng(977)
    shapes = [(128, 4), (40, 32), (33, 25), (8, 2)]
    insts = [(n, m, rng.integers(1, 100, size=(n, m)).astype(np.int32)) for n, m in shapes]
    per = [24, 6, 60, 30]
    stride = 128
    perm, d1, d2, seg = _batch(insts, per, 515, stride)
    for k, (n, m, p) in enumerate(insts):
        a = seg[k]
        d1[a], d2[a] = 0, 0
        d1[a + 1], d2[a + 1] = 0, n - 1
    ub = np.array([9000, 8000, 4000, 600], dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    lb, pr, dr = mt.bound(*_dev(ctx, perm, d1, d2), seg, ub, binding.LB2_FULL)
    _check(insts, perm, d1, d2, seg, ub, lb, pr, dr, binding.LB2_FULL)
    mt.close()


def test_full_size_batch_sampled(ctx):
    """The multi-instance benchmark batch at full size (64 instances, 16,384
    parents each, incumbent open) in the default and an autotuned launch
    shape; 4 sampled rows per instance against the oracle, and at every row
    exactly 2(n - d) finite children."""
    import torch
    insts = inputs.mixed_instances(64, 4000)
    stride = max(n for n, _, _ in insts)
    per = 16384
    perm, d1, d2, seg = [], [], [], [0]
    for k, (n, m, p) in enumerate(insts):
        pk, a, b = inputs.random_pool(n, per, 5000 + k)
        pad = np.zeros((per, stride), dtype=np.uint8)
        pad[:, :n] = pk
        perm.append(pad)
        d1.append(a)
        d2.append(b)
        seg.append(seg[-1] + per)
    perm, d1, d2, seg = np.concatenate(perm), np.concatenate(d1), np.concatenate(d2), np.array(seg)
    ub = np.full(64, binding.INT32_MAX, dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    dev = _dev(ctx, perm, d1, d2)
    rng = np.random.default_rng(64)
    for shape in (None, dict(tile=64, waves_small=12, waves_large=0, blocks_per_cu=2)):
        if shape:
            mt.set_shape(**shape)
        lb, pr, dr = mt.bound(*dev, seg, ub, binding.LB2_FULL)
        torch.cuda.synchronize()
        lb, pr, dr = lb.cpu().numpy(), pr.cpu().numpy(), dr.cpu().numpy()
        for k, (n, m, p) in enumerate(insts):
            rows = seg[k] + np.sort(rng.choice(per, 4, replace=False))
            olb, opr, odr = oracle.bound_children(p, perm[rows, :n], d1[rows], d2[rows],
                                                  binding.LB2_FULL, binding.INT32_MAX, threads=8)
            np.testing.assert_array_equal(lb[rows, :, :n], olb)
            np.testing.assert_array_equal(pr[rows, :, :n], opr)
            np.testing.assert_array_equal(dr[rows], odr)
        r = np.repeat(np.array([n for n, _, _ in insts]), per) - d1.astype(np.int64) - d2
        np.testing.assert_array_equal((lb < binding.INT32_MAX).sum(axis=(1, 2)), 2 * r)
    mt.close()
