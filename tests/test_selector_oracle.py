"""Pins of the selector reference (oracle/selector.py): bf16 rounding against
torch's conversion, gradients against finite differences and against torch
autograd, Adam against torch.optim, and closed forms of the features."""
import numpy as np
import pytest
import torch

import oracle
from oracle import selector as S
from paper_2012_09511_amd import inputs


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000).astype(np.float32),
                        np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, -1 - 2**-8, 0.0, -0.0,
                                  3.0e38, 1e-40], dtype=np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(S.bf16_round(x), ref)
    assert S.bf16_round(np.float32(1 + 2**-8)) == 1.0          # tie to even
    assert S.bf16_round(np.float32(1 + 3 * 2**-8)) == 1 + 2**-6  # tie to even, up


def _problem(seed, B=6):
    rng = np.random.default_rng(seed)
    params = [p.astype(np.float64) for p in inputs.selector_params(seed, scale=2.0)]
    params[1] = rng.normal(size=64) * 0.1
    params[3] = rng.normal(size=64) * 0.1
    params[5] = rng.normal(size=190) * 0.1
    x = rng.random((B, 64))
    valid = S.valid_pairs(12)
    t = rng.random((B, 190)) * valid
    t[1] = 0                                   # a row without target is ignored
    t /= np.maximum(t.sum(axis=1, keepdims=True), 1e-300)
    return params, x, t, valid


def test_gradients_match_finite_differences():
    params, x, t, valid = _problem(1)
    loss, grads = S.loss_and_grads(params, x, t, valid, round_weights=False)
    rng = np.random.default_rng(2)
    h = 1e-6
    for pi in range(6):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in params[pi].shape)
            pp = [p.copy() for p in params]
            pp[pi][idx] += h
            lp, _ = S.loss_and_grads(pp, x, t, valid, round_weights=False)
            pp[pi][idx] -= 2 * h
            lm, _ = S.loss_and_grads(pp, x, t, valid, round_weights=False)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[pi][idx]) <= 1e-3 * max(1e-3, abs(fd))


def test_gradients_match_torch_autograd():
    params, x, t, valid = _problem(3)
    loss, grads = S.loss_and_grads(params, x, t, valid)
    tp = [torch.tensor(S.bf16_round(p.astype(np.float32)).astype(np.float64)
                       if p.ndim == 2 else p, requires_grad=True) for p in params]
    X = torch.tensor(x)
    h1 = torch.relu(X @ tp[0].T + tp[1])
    h2 = torch.relu(h1 @ tp[2].T + tp[3])
    s = h2 @ tp[4].T + tp[5]
    s = s.masked_fill(~torch.tensor(valid), float("-inf"))
    T = torch.tensor(t)
    rows = T.sum(dim=1) > 0
    logp = torch.log_softmax(s, dim=1).masked_fill(~torch.tensor(valid), 0.0)
    L = -(T * logp).sum(dim=1)[rows].mean()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    for g, p in zip(grads, tp):
        np.testing.assert_allclose(g, p.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_adam_matches_torch():
    params, x, t, valid = _problem(4)
    _, grads = S.loss_and_grads(params, x, t, valid)
    state = {}
    new = S.adam_step(params, grads, state, lr=1e-2)
    tp = [torch.tensor(p, requires_grad=True) for p in params]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for p, g in zip(tp, grads):
        p.grad = torch.tensor(g)
    opt.step()
    for a, b in zip(new, tp):
        np.testing.assert_allclose(a, b.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_topk_and_histogram():
    rng = np.random.default_rng(5)
    valid = S.valid_pairs(7)
    sc = np.round(rng.normal(size=(4, 190)), 1)      # many ties
    mk = S.topk_mask(sc, valid, 5)
    assert (mk.sum(axis=1) == 5).all() and not (mk & ~valid).any()
    for i in range(4):
        chosen = sc[i][mk[i]]
        rest = sc[i][valid & ~mk[i]]
        assert chosen.min() >= rest.max()
    # histogram of logged argmax pairs: one per node that has a child needing a
    # pair (LB2 > LB1), zero otherwise
    n, m = 9, 6
    p = inputs.instance(n, m, 3)
    perm, d1, d2 = inputs.random_pool(n, 20, 4)
    l1, _, _ = oracle.bound_children(p, perm, d1, d2, oracle.LB1)
    l2, _, _, ap = oracle.bound_children(p, perm, d1, d2, oracle.LB2_FULL, with_argpair=True)
    h = S.pair_histogram(ap, d1, d2, m)
    needs = ((l2 > l1) & (l1 < 2**31 - 1)).reshape(len(perm), -1).any(axis=1)
    assert needs.any() and not needs.all()
    np.testing.assert_allclose(h.sum(axis=1), needs.astype(float))
    assert ((ap >= 0) == ((l2 > l1) & (l1 < 2**31 - 1))).all()
    assert not (h[:, ~S.valid_pairs(m)] > 0).any()


def test_root_features_closed_form():
    n, m = 15, 8
    p = inputs.instance(n, m, 9)
    f = S.features(p, np.arange(n)[None, :].astype(np.uint8), [0], [0])[0]
    T = p.sum(axis=0)
    np.testing.assert_allclose(f[40:48], T / T.max())
    assert f[63] == 1.0 and f[62] == 1.0 and f[60] == 0 and f[:8].sum() == 0
