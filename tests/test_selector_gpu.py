"""GPU checks of the learned pair selector against oracle/selector.py.

Floating-point results (features, scores, loss, gradients, Adam updates) are
compared within a tolerance derived from fp32 accumulation over at most 190
terms of magnitude <= ~10 (relative 1e-4 of the largest magnitude); integer
decisions are compared exactly where they are unique, and by validity where
fp32 rounding could reorder near-ties.
"""
import numpy as np
import pytest

import oracle
from oracle import selector as S
from paper_2012_09511_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = binding.Context(0)
    yield c
    c.close()


def _t(ctx, a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(ctx.device) if dtype is None else t.to(ctx.device, dtype)


def _params(seed):
    ps = inputs.selector_params(seed, scale=2.0)
    rng = np.random.default_rng(seed)
    ps[1] = (rng.normal(size=64) * 0.1).astype(np.float32)
    ps[3] = (rng.normal(size=64) * 0.1).astype(np.float32)
    ps[5] = (rng.normal(size=190) * 0.1).astype(np.float32)
    return ps


def _close(got, ref, rel=1e-4):
    scale = max(1.0, float(np.abs(ref).max()))
    np.testing.assert_allclose(got, ref, rtol=0, atol=rel * scale)


@pytest.mark.parametrize("n,m", [(20, 20), (12, 7), (50, 20)])
def test_features(ctx, n, m):
    p = inputs.instance(n, m, 70 + m)
    perm, d1, d2 = inputs.random_pool(n, 300, 71)
    ctx.load_instance(p)
    f = ctx.selector_features(*[_t(ctx, a) for a in (perm, d1, d2)]).cpu().numpy()
    _close(f, S.features(p, perm, d1, d2), rel=1e-6)


def test_forward_and_select(ctx):
    n, m = 20, 13
    p = inputs.instance(n, m, 80)
    ctx.load_instance(p)
    params = _params(81)
    ctx.selector_set(params)
    np.testing.assert_array_equal(ctx.selector_get(),
                                  np.concatenate([q.reshape(-1) for q in params]))
    rng = np.random.default_rng(82)
    x = rng.random((500, 64)).astype(np.float32)
    sc = ctx.selector_forward(_t(ctx, x)).cpu().numpy()
    p64 = [q.astype(np.float64) for q in params]
    ref, _ = S.forward(p64, x.astype(np.float64))
    valid = S.valid_pairs(m)
    assert np.isneginf(sc[:, ~valid]).all()
    # per score, against the sum of absolute terms: the bf16 hi/lo split of the
    # activations loses at most 2^-16 of each, fp32 sums of 128 products at most
    # 128 * 2^-24, three layers
    tol = 1e-4 * S.forward_magnitude(p64, x.astype(np.float64))
    assert (np.abs(sc[:, valid] - ref[:, valid]) <= tol[:, valid]).all()
    for k in (1, 16, 32):
        mk = ctx.selector_select(_t(ctx, sc), k).cpu().numpy().view(np.uint32)
        P = m * (m - 1) // 2
        bits = np.array([[(mk[i, b >> 5] >> (b & 31)) & 1 for b in range(P)]
                         for i in range(len(x))], dtype=bool)
        # exact against the oracle's top-k of the same (GPU) scores
        ref_mask = S.topk_mask(sc, valid, k)
        inst = np.zeros((len(x), P), dtype=bool)
        for u in range(m):
            for v in range(u + 1, m):
                inst[:, oracle.pair_index(m, u, v)] = ref_mask[:, S.pair20(u, v)]
        np.testing.assert_array_equal(bits, inst)


def test_targets_from_logged_argmax(ctx):
    n, m = 15, 9
    p = inputs.instance(n, m, 90)
    perm, d1, d2 = inputs.random_pool(n, 200, 91)
    ctx.load_instance(p)
    dev = [_t(ctx, a) for a in (perm, d1, d2)]
    _, _, _, ap = ctx.bound_children(*dev, kind=binding.LB2_FULL, want_argpair=True)
    tg = ctx.selector_targets(*dev, ap).cpu().numpy()
    _, _, _, oap = oracle.bound_children(p, perm, d1, d2, oracle.LB2_FULL, with_argpair=True)
    _close(tg, S.pair_histogram(oap, d1, d2, m), rel=1e-6)


def test_train_step_gradients_and_adam(ctx):
    n, m = 20, 20
    p = inputs.instance(n, m, 100)
    ctx.load_instance(p)
    params = _params(101)
    rng = np.random.default_rng(102)
    B = 257
    x = rng.random((B, 64)).astype(np.float32)
    valid = S.valid_pairs(m)
    t = (rng.random((B, 190)) * valid).astype(np.float32)
    t[::7] = 0
    t /= np.maximum(t.sum(axis=1, keepdims=True), 1e-30)
    t = t.astype(np.float32)
    ctx.selector_set(params)
    loss, g = ctx.selector_train_step(_t(ctx, x), _t(ctx, t), 0.0, want_grad=True)
    p64 = [q.astype(np.float64) for q in params]
    rl, rg = S.loss_and_grads(p64, x.astype(np.float64), t.astype(np.float64), valid)
    assert abs(loss - rl) <= 1e-4 * max(1.0, abs(rl))
    flat = np.concatenate([q.reshape(-1) for q in rg])
    _close(g.cpu().numpy(), flat, rel=1e-4)
    # one Adam step of size 1e-3 against the reference update
    ctx.selector_set(params)
    ctx.selector_train_step(_t(ctx, x), _t(ctx, t), 1e-3)
    new = ctx.selector_get()
    ref = S.adam_step(p64, rg, {}, lr=1e-3)
    _close(new, np.concatenate([q.reshape(-1) for q in ref]), rel=1e-5)


def test_training_lowers_the_loss(ctx):
    n, m = 20, 20
    p = inputs.instance(n, m, 110)
    perm, d1, d2 = inputs.random_pool(n, 4096, 111)
    ctx.load_instance(p)
    dev = [_t(ctx, a) for a in (perm, d1, d2)]
    _, _, _, ap = ctx.bound_children(*dev, kind=binding.LB2_FULL, want_argpair=True)
    tg = ctx.selector_targets(*dev, ap)
    x = ctx.selector_features(*dev)
    ctx.selector_set(inputs.selector_params(112))
    first, _ = ctx.selector_train_step(x, tg, 3e-3)
    for _ in range(60):
        last, _ = ctx.selector_train_step(x, tg, 3e-3)
    assert last < 0.8 * first


@pytest.mark.parametrize("n,ub", [(20, 1900), (50, 4170)])
@pytest.mark.parametrize("topk", [1, 16, 190])
def test_learned_bound_equals_subset_bound(ctx, topk, n, ub):
    """LB2_LEARNED = subset LB2 over the pairs the selector picks (checked
    against the oracle with the same mask) and never above full LB2; at
    n = 50 through the packed wide kernel (four parents per wave for
    k <= 16, two for k = 32)."""
    import torch
    m = 20
    p = inputs.instance(n, m, 120)
    perm, d1, d2 = inputs.random_pool(n, 300 if n <= 20 else 150, 121)
    ctx.load_instance(p)
    ctx.selector_set(_params(122))
    dev = [_t(ctx, a) for a in (perm, d1, d2)]
    k = min(topk, 32)
    ctx.set_option("learned_topk", k)
    lb, pr, dr, _ = ctx.bound_children(*dev, kind=binding.LB2_LEARNED, ub=ub)
    torch.cuda.synchronize()
    mask = ctx.selector_infer(*dev, k).cpu().numpy().view(np.uint32)
    olb, opr, odr = oracle.bound_children(p, perm, d1, d2, oracle.LB2_SUBSET, ub,
                                          pair_mask=mask, threads=8)
    np.testing.assert_array_equal(lb.cpu().numpy(), olb)
    np.testing.assert_array_equal(pr.cpu().numpy(), opr)
    np.testing.assert_array_equal(dr.cpu().numpy(), odr)
    assert 0 < opr.mean() < 1   # the incumbent prunes some children, not all
    full, _, _ = oracle.bound_children(p, perm, d1, d2, oracle.LB2_FULL, ub, threads=8)
    assert (olb <= full).all()
    ctx.set_option("learned_topk", 16)


def _bits_layout(mask_words, m):
    """uint32 words over instance pairs -> bool [B, 190] over layout pairs."""
    out = np.zeros((mask_words.shape[0], 190), dtype=bool)
    for u in range(m):
        for v in range(u + 1, m):
            pi = u * (2 * m - u - 1) // 2 + (v - u - 1)
            out[:, S.pair20(u, v)] = (mask_words[:, pi >> 5] >> (pi & 31)) & 1
    return out


@pytest.mark.parametrize("n,m", [(20, 20), (50, 20), (12, 7)])
@pytest.mark.parametrize("k", [1, 16, 32])
def test_float_inference_masks(ctx, n, m, k):
    """The learned bound's float form (features from the costs, bf16 MFMA
    layers, ranking keys, top-k) selects exactly the oracle's top-k by key of
    the scores that pfsp_selector_forward computes with the same arithmetic
    from the library's features; those scores are within the error bound of
    the oracle's (test_forward_and_select), the features within 1e-6."""
    import torch
    p = inputs.instance(n, m, 140 + n + m)
    perm, d1, d2 = _quant_pool(n, 141)
    ctx.load_instance(p)
    params = _params(142)
    ctx.selector_set(params)
    dev = [_t(ctx, a) for a in (perm, d1, d2)]
    got = ctx.selector_infer(*dev, k).cpu().numpy().view(np.uint32)
    feat = ctx.selector_features(*dev)
    sc = ctx.selector_forward(feat).cpu().numpy()
    torch.cuda.synchronize()
    _close(feat.cpu().numpy(), S.features(p, perm, d1, d2), rel=1e-6)
    valid = S.valid_pairs(m)
    assert np.isneginf(sc[:, ~valid]).all()
    want = S.topk_keys_mask(S.score_keys(np.where(valid, sc, 0.0)), valid, k)
    np.testing.assert_array_equal(_bits_layout(got, m), want)
    p64 = [q.astype(np.float64) for q in params]
    x = S.features(p, perm, d1, d2)
    ref, _ = S.forward(p64, x)
    tol = 1e-4 * S.forward_magnitude(p64, x)
    assert (np.abs(sc[:, valid] - ref[:, valid]) <= tol[:, valid]).all()


# ---------------------------------------------------------------- integer model
def _qblob(seed, ties=False):
    """A random integer-model blob (layout of pfsp_selector_set_quant); with
    ties, the output layer gives many pairs the same score."""
    rng = np.random.default_rng(seed)
    W3 = rng.integers(-127, 128, (190, 64))
    b3 = rng.integers(-5000, 5000, 190)
    if ties:
        W3[:, 8:] = 0
        W3[:, :8] = rng.integers(-1, 2, (1, 8))     # one row for every pair
        b3 = rng.integers(0, 3, 190) * 1000
    head = [int(np.array([20.0 + seed], dtype=np.float32).view(np.int32)[0]),
            int(rng.integers(300, 1024)), int(rng.integers(10, 16)),
            int(rng.integers(300, 1024)), int(rng.integers(10, 16))]
    parts = [rng.integers(-127, 128, (64, 64)), rng.integers(-5000, 5000, 64),
             rng.integers(-127, 128, (64, 64)), rng.integers(-5000, 5000, 64), W3, b3]
    return np.concatenate([np.array(head)] + [a.reshape(-1) for a in parts]).astype(np.int32)


def _words(layout_mask, m):
    """bool [B, 190] over layout pairs -> uint32 words over instance pair indices."""
    P = m * (m - 1) // 2
    out = np.zeros((layout_mask.shape[0], (P + 31) // 32), dtype=np.uint32)
    for u in range(m):
        for v in range(u + 1, m):
            pi = u * (2 * m - u - 1) // 2 + (v - u - 1)
            out[:, pi >> 5] |= layout_mask[:, S.pair20(u, v)].astype(np.uint32) << (pi & 31)
    return out


def _quant_pool(n, seed):
    parts = [inputs.random_pool(n, 250, seed), inputs.random_pool(n, 6, seed + 1, depth=0),
             inputs.random_pool(n, 9, seed + 2, depth=n - 1)]
    return tuple(np.concatenate([q[i] for q in parts]) for i in range(3))


@pytest.mark.parametrize("m", [20, 13, 2])
@pytest.mark.parametrize("k", [1, 16, 17, 32, 33, 64])
@pytest.mark.parametrize("ties", [False, True])
def test_integer_selector_masks(ctx, m, k, ties):
    """The fused int8-MFMA inference selects exactly the oracle's pairs: random
    blobs (with and without tied scores), every k, fewer pairs than k (m = 2),
    pools of 265 rows (a partial last wave), root and leaf-parent rows."""
    n = 20
    p = inputs.instance(n, m, 400 + m)
    perm, d1, d2 = _quant_pool(n, 410 + m)
    ctx.load_instance(p)
    blob = _qblob(420 + m + k, ties)
    ctx.selector_set_quant(blob)
    try:
        got = ctx.selector_infer(*[_t(ctx, a) for a in (perm, d1, d2)], k)
        got = got.cpu().numpy().view(np.uint32)
        exp = _words(S.quant_masks(blob, p, perm, d1, d2, k), m)
        np.testing.assert_array_equal(got, exp)
    finally:
        ctx.selector_set_quant(None)


@pytest.mark.parametrize("k", [16, 32, 64])
def test_learned_bound_integer_model(ctx, k):
    """LB2_LEARNED with the quantized trained selector (calibrated by the
    library's own quantizer) equals subset LB2 over the oracle's pairs."""
    import torch
    from paper_2012_09511_amd import selector_quant
    n, m = 20, 20
    p = inputs.instance(n, m, 430)
    perm, d1, d2 = _quant_pool(n, 431)
    ctx.load_instance(p)
    import os
    flat = np.load(os.path.join(os.path.dirname(inputs.__file__), "data", "selector_n20m20.npy"),
                   allow_pickle=False)
    ctx.selector_set(flat)
    blob = selector_quant.quantize(flat, selector_quant.calibration_features(ctx, n, 2048))
    ctx.selector_set_quant(blob)
    ctx.set_option("learned_topk", k)
    try:
        dev = [_t(ctx, a) for a in (perm, d1, d2)]
        lb, pr, dr, _ = ctx.bound_children(*dev, kind=binding.LB2_LEARNED, ub=1900)
        torch.cuda.synchronize()
        mask = _words(S.quant_masks(blob, p, perm, d1, d2, k), m)
        olb, opr, odr = oracle.bound_children(p, perm, d1, d2, oracle.LB2_SUBSET, 1900,
                                              pair_mask=mask, threads=8)
        np.testing.assert_array_equal(lb.cpu().numpy(), olb)
        np.testing.assert_array_equal(pr.cpu().numpy(), opr)
        np.testing.assert_array_equal(dr.cpu().numpy(), odr)
    finally:
        ctx.set_option("learned_topk", 16)
        ctx.selector_set_quant(None)


def test_integer_selector_rejects_bad_blobs(ctx):
    ctx.load_instance(inputs.instance(10, 5, 3))
    good = _qblob(3)
    for idx, val in ((1, 0), (1, 1024), (2, 0), (2, 31), (10, 128), (5 + 4096, 1 << 19)):
        bad = good.copy()
        bad[idx] = val
        with pytest.raises(binding.PfspError):
            ctx.selector_set_quant(bad)
    with pytest.raises(binding.PfspError):
        ctx.selector_set_quant(good[:-1])
    # more than 32 pairs needs the integer model
    import torch
    perm, d1, d2 = inputs.random_pool(10, 4, 5)
    dev = [_t(ctx, a) for a in (perm, d1, d2)]
    ctx.selector_set(_params(9))
    ctx.selector_set_quant(None)
    with pytest.raises(binding.PfspError):
        ctx.selector_infer(*dev, 33)
    ctx.selector_set_quant(good)
    ctx.selector_infer(*dev, 64)
    torch.cuda.synchronize()
    ctx.selector_set_quant(None)


def _trained_blob(ctx, n):
    import os
    from paper_2012_09511_amd import selector_quant
    flat = np.load(os.path.join(os.path.dirname(inputs.__file__), "data", "selector_n20m20.npy"),
                   allow_pickle=False)
    ctx.selector_set(flat)
    return selector_quant.quantize(flat, selector_quant.calibration_features(ctx, n, 2048))


def test_trained_selector_gains(ctx):
    """What training gains, with 16 of the 190 pairs per parent on 4,096 random
    nodes of a 20 x 20 instance: the trained selector's bound equals full LB2
    on more children, and prunes more at an incumbent in the middle of the
    bounds, than 16 pairs drawn at random or picked by an untrained network
    (LB1 alone is the floor).  Values go to stdout."""
    import torch
    n, m, k = 20, 20, 16
    p = inputs.instance(n, m, 650)
    perm, d1, d2 = inputs.random_pool(n, 4096, 651)
    ctx.load_instance(p)
    dev = [_t(ctx, a) for a in (perm, d1, d2)]

    def bound(kind, mask=None):
        tm = None if mask is None else _t(ctx, mask)
        lb, _, _, _ = ctx.bound_children(*dev, kind=kind, ub=binding.INT32_MAX, pair_mask=tm)
        torch.cuda.synchronize()
        return lb.cpu().numpy()

    full = bound(binding.LB2_FULL)
    lb1 = bound(binding.LB1)
    fin = full < binding.INT32_MAX
    ub = int(np.percentile(full[fin], 40))
    ctx.set_option("learned_topk", k)
    try:
        ctx.selector_set_quant(_trained_blob(ctx, n))
        trained = bound(binding.LB2_LEARNED)
        ctx.selector_set_quant(None)
        ctx.selector_set(_params(652))            # an untrained network
        untrained = bound(binding.LB2_LEARNED)
    finally:
        ctx.set_option("learned_topk", 16)
    rng = np.random.default_rng(653)
    P = m * (m - 1) // 2
    sel = np.argsort(rng.random((len(perm), P)), axis=1)[:, :k]
    mask = np.zeros((len(perm), (P + 31) // 32), dtype=np.uint32)
    for w in range(mask.shape[1]):
        bits = np.where((sel >> 5) == w, np.left_shift(np.uint64(1), (sel & 31).astype(np.uint64)), 0)
        mask[:, w] = np.bitwise_or.reduce(bits, axis=1).astype(np.uint32)
    rand = bound(binding.LB2_SUBSET, mask)
    stats = {}
    for name, x in (("trained", trained), ("untrained", untrained), ("random", rand),
                    ("lb1", lb1)):
        assert (x[fin] <= full[fin]).all() and (x[fin] >= lb1[fin]).all()
        stats[name] = (float((x[fin] == full[fin]).mean()), int((x[fin] >= ub).sum()))
    stats["full"] = (1.0, int((full[fin] >= ub).sum()))
    print("recall of full LB2, prunes at ub =", ub, stats)
    for other in ("untrained", "random", "lb1"):
        assert stats["trained"][0] > stats[other][0] + 0.05
        assert stats["trained"][1] > stats[other][1]


def test_learned_search_same_optimum(ctx):
    """Learned-pair LB2 (the trained selector's int8 form, 32 pairs) proves the
    same optimum as full LB2 on a 20 x 20 instance from NEH + 1."""
    p = inputs.instance(20, 20, 601)
    ctx.load_instance(p)
    ctx.selector_set_quant(_trained_blob(ctx, 20))
    ctx.set_option("learned_topk", 32)
    try:
        ub0, _ = ctx.neh()
        full = ctx.search(ub0 + 1, 0, binding.LB2_FULL)
        learned = ctx.search(ub0 + 1, 0, binding.LB2_LEARNED)
    finally:
        ctx.set_option("learned_topk", 16)
        ctx.selector_set_quant(None)
    assert full["proven"] and learned["proven"]
    assert full["best"] == learned["best"] <= ub0
    assert learned["nodes"] >= full["nodes"]       # a subset never prunes more
    for r in (full, learned):                      # the schedules, re-evaluated
        assert sorted(r["perm"].tolist()) == list(range(20))
        assert oracle.makespan(p, r["perm"]) == r["best"]


@pytest.mark.parametrize("k", [16, 32])
def test_learned_exact_bound(ctx, k):
    """Exact mode (option learned_exact): a parent that keeps a child under the
    selected pairs is bounded again with all pairs, so every prune flag is full
    LB2's, and so are the bounds and the MinMin choice of every parent that
    keeps a child.  A parent the subset prunes entirely keeps the subset's
    bounds (all at least the incumbent)."""
    import torch
    n, m = 20, 20
    p = inputs.instance(n, m, 430)
    perm, d1, d2 = _quant_pool(n, 432)
    flb, _, _ = oracle.bound_children(p, perm, d1, d2, oracle.LB2_FULL, threads=8)
    ub = int(np.percentile(flb[flb < binding.INT32_MAX], 30))   # some parents keep children
    ctx.load_instance(p)
    blob = _trained_blob(ctx, n)
    ctx.selector_set_quant(blob)
    ctx.set_option("learned_topk", k)
    ctx.set_option("learned_exact", 1)
    try:
        dev = [_t(ctx, a) for a in (perm, d1, d2)]
        lb, pr, dr, _ = ctx.bound_children(*dev, kind=binding.LB2_LEARNED, ub=ub)
        torch.cuda.synchronize()
    finally:
        ctx.set_option("learned_exact", 0)
        ctx.set_option("learned_topk", 16)
        ctx.selector_set_quant(None)
    lb, pr, dr = lb.cpu().numpy(), pr.cpu().numpy(), dr.cpu().numpy()
    flb, fpr, fdr = oracle.bound_children(p, perm, d1, d2, oracle.LB2_FULL, ub, threads=8)
    mask = _words(S.quant_masks(blob, p, perm, d1, d2, k), m)
    slb, spr, sdr = oracle.bound_children(p, perm, d1, d2, oracle.LB2_SUBSET, ub,
                                          pair_mask=mask, threads=8)
    np.testing.assert_array_equal(pr, fpr)
    r = n - d1.astype(int) - d2.astype(int)
    reopened = (spr == 0).any(axis=(1, 2)) & (r >= 2)
    assert 0 < reopened.mean() < 1
    np.testing.assert_array_equal(lb[reopened], flb[reopened])
    np.testing.assert_array_equal(dr[reopened], fdr[reopened])
    np.testing.assert_array_equal(lb[~reopened], slb[~reopened])
    np.testing.assert_array_equal(dr[~reopened], sdr[~reopened])


@pytest.mark.parametrize("seed", [1, 2])
def test_learned_exact_search_same_tree(ctx, seed):
    """With the incumbent at the optimum, exact mode decomposes exactly the
    critical tree of full LB2 (the oracle's count), and the pure learned bound
    at least as many nodes.  20 x 10 instances of the search workload."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "search_20x10.json")) as f:
        g = {c["seed"]: c for c in json.load(f)["cases"]}[seed]
    p = inputs.instance(20, 10, seed)
    ctx.load_instance(p)
    ctx.selector_set_quant(_trained_blob(ctx, 20))
    ctx.set_option("learned_topk", 16)
    try:
        ctx.set_option("learned_exact", 1)
        exact = ctx.search(g["opt"], 0, binding.LB2_LEARNED)
        ctx.set_option("learned_exact", 0)
        pure = ctx.search(g["opt"], 0, binding.LB2_LEARNED)
        ctx.set_option("learned_exact", 1)
        found = ctx.search(g["neh"] + 1, 0, binding.LB2_LEARNED)
    finally:
        ctx.set_option("learned_exact", 0)
        ctx.selector_set_quant(None)
    assert exact["proven"] and not exact["found"]
    assert exact["nodes"] == g["critical_nodes_lb2"]
    assert exact["children"] == g["critical_children_lb2"]
    assert pure["proven"] and pure["nodes"] >= exact["nodes"]
    assert found["proven"] and found["best"] == g["opt"]
    assert oracle.makespan(p, found["perm"]) == g["opt"]
