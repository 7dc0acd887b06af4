"""Reference of the learned machine-pair selector (test infrastructure only).

The paper allows LB2 variants that evaluate between m and m(m-1)/2 machine
pairs (Section 2.4); any subset S of pairs gives a valid bound
max(LB1, max over S of the pair values).  The selector picks S per node: a
small MLP maps 64 features of a parent node to one score per pair of a
20-machine layout, and the k best-scoring pairs that exist on the instance
form S.  It is trained on the pairs that attain the full LB2 of the children
of logged nodes.

Everything here is float64 numpy, with the weights rounded to bfloat16 (round
to nearest even) before use, as the kernels do.  Pinned in
tests/test_selector_oracle.py against torch (bf16 conversion, autograd, Adam),
finite differences and closed forms of the features.  The integer model at the
end (int8 codes, exact int64 sums) is pinned there by hand-computed codes and
layers, invariances (hidden-unit permutation, score scaling) and brute force.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, M_MAX = 64, 64, 20
N_OUT = M_MAX * (M_MAX - 1) // 2   # 190


def bf16_round(w) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returns float32."""
    a = np.ascontiguousarray(w, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    out = np.where(nan, a, out)
    return out.astype(np.float32)


def pair20(u: int, v: int) -> int:
    """Index of machine pair u < v in the 20-machine lexicographic layout."""
    return u * (2 * M_MAX - u - 1) // 2 + (v - u - 1)


def valid_pairs(m: int) -> np.ndarray:
    """bool[190]: pairs of the 20-machine layout that exist on an m-machine instance."""
    ok = np.zeros(N_OUT, dtype=bool)
    for u in range(min(m, M_MAX)):
        for v in range(u + 1, min(m, M_MAX)):
            ok[pair20(u, v)] = True
    return ok


def features(p, perm, d1, d2):
    """64 features per node: front, back and remaining work per machine (first
    20 machines, zero-padded) and the node's LB1, all divided by the largest
    machine load of the instance; then d1/n, d2/n and the unscheduled share."""
    import oracle
    p = np.asarray(p)
    n, m = p.shape
    norm = float(p.sum(axis=0).max())
    out = np.zeros((len(perm), N_IN), dtype=np.float64)
    for i in range(len(perm)):
        a, b = int(d1[i]), int(d2[i])
        C1 = oracle.front(p, perm[i][:a])
        C2 = oracle.back(p, perm[i][n - b:])
        R = p[perm[i][a:n - b]].sum(axis=0).astype(np.int64)
        k = min(m, M_MAX)
        out[i, 0:k] = C1[:k] / norm
        out[i, 20:20 + k] = C2[:k] / norm
        out[i, 40:40 + k] = R[:k] / norm
        out[i, 60] = a / n
        out[i, 61] = b / n
        out[i, 62] = (n - a - b) / n
        out[i, 63] = oracle.lb1_parts(C1, R, C2) / norm
    return out


def _weights(params, round_weights):
    W1, _, W2, _, W3, _ = params
    if round_weights:
        return [bf16_round(W).astype(np.float64) for W in (W1, W2, W3)]
    return [np.asarray(W, dtype=np.float64) for W in (W1, W2, W3)]


def forward(params, x, round_weights=True):
    """Scores [B, 190] and the activations (h1, h2) with bf16-rounded weights."""
    W1, b1, W2, b2, W3, b3 = params
    W1q, W2q, W3q = _weights(params, round_weights)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1q.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2q.T + b2
    h2 = np.maximum(z2, 0)
    s = h2 @ W3q.T + b3
    return s, (h1, h2)


def forward_magnitude(params, x):
    """[B, 190] bound on the sum of absolute terms behind each score: the
    forward pass with |W| (bf16-rounded), |b| and |x|, ReLU left out.  A float
    evaluation whose every sum has relative error e is within about
    3 e times this bound of the exact score."""
    W1, b1, W2, b2, W3, b3 = params
    W1q, W2q, W3q = _weights(params, True)
    x = np.abs(np.asarray(x, dtype=np.float64))
    h1 = x @ np.abs(W1q).T + np.abs(b1)
    h2 = h1 @ np.abs(W2q).T + np.abs(b2)
    return h2 @ np.abs(W3q).T + np.abs(b3)


def score_keys(scores) -> np.ndarray:
    """int64 [B, 190] ranking keys of the float form: each score rounded to
    float32 and mapped to an order-preserving integer (non-negative: its bits;
    negative: bits xor 0x7fffffff, as a signed 32-bit value) whose low 8 bits
    are replaced by 255 - layout index, so that scores agreeing in their
    leading 24 bits rank by the lower index."""
    s = np.ascontiguousarray(np.asarray(scores, dtype=np.float64).astype(np.float32))
    u = s.view(np.uint32).astype(np.int64)
    ordv = np.where(u >= 2**31, (u ^ 0x7FFFFFFF) - 2**32, u)
    return (ordv & ~0xFF) | (255 - np.arange(N_OUT, dtype=np.int64))


def topk_keys_mask(keys, valid, k):
    """bool [B, 190]: the k largest keys among valid pairs."""
    out = np.zeros(keys.shape, dtype=bool)
    idx = np.flatnonzero(valid)
    for i in range(keys.shape[0]):
        order = idx[np.argsort(-keys[i, idx], kind="stable")]
        out[i, order[:k]] = True
    return out


def masked_log_softmax(s, valid):
    s = np.where(valid, s, -np.inf)
    mx = s.max(axis=1, keepdims=True)
    z = s - mx
    lse = np.log(np.exp(z).sum(axis=1, keepdims=True))
    return np.where(valid, z - lse, 0.0)


def loss_and_grads(params, x, target, valid, round_weights=True):
    """Mean soft-target cross-entropy over rows with a non-empty target, and its
    gradients with respect to the fp32 master parameters (the bf16 rounding is
    passed through unchanged)."""
    W1, b1, W2, b2, W3, b3 = params
    W1q, W2q, W3q = _weights(params, round_weights)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    rows = t.sum(axis=1) > 0
    B = max(int(rows.sum()), 1)
    s, (h1, h2) = forward(params, x, round_weights)
    ls = masked_log_softmax(s, valid)
    loss = -(t * ls).sum(axis=1)
    loss = float(loss[rows].sum() / B)
    prob = np.where(valid, np.exp(ls), 0.0)
    ds = (prob - t) * rows[:, None] / B
    gW3 = ds.T @ h2
    gb3 = ds.sum(axis=0)
    dh2 = (ds @ W3q) * (h2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2q) * (h1 > 0)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the fp32 master parameters (float64 arithmetic)."""
    t = state.get("t", 0) + 1
    state["t"] = t
    ms = state.setdefault("m", [np.zeros_like(p, dtype=np.float64) for p in params])
    vs = state.setdefault("v", [np.zeros_like(p, dtype=np.float64) for p in params])
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        ms[i] = beta1 * ms[i] + (1 - beta1) * g
        vs[i] = beta2 * vs[i] + (1 - beta2) * g * g
        mh = ms[i] / (1 - beta1 ** t)
        vh = vs[i] / (1 - beta2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out


def topk_mask(scores, valid, k):
    """bool [B, 190]: the k highest scores among valid pairs, ties to the lower index."""
    out = np.zeros(scores.shape, dtype=bool)
    for i in range(scores.shape[0]):
        idx = [j for j in range(N_OUT) if valid[j]]
        idx.sort(key=lambda j: (-scores[i, j], j))
        out[i, idx[:k]] = True
    return out


def pair_histogram(argpair, d1, d2, m):
    """Soft targets [B, 190]: among a node's children whose full LB2 exceeds
    LB1, the share whose LB2 is attained first (lowest index) by each pair;
    argpair holds instance pair indices [B, 2, n] (-1: LB1 suffices, or no
    child).  A node none of whose children needs a pair gets a zero row."""
    B, _, n = argpair.shape
    to20 = np.zeros(m * (m - 1) // 2, dtype=np.int64)
    for u in range(m):
        for v in range(u + 1, m):
            to20[u * (2 * m - u - 1) // 2 + (v - u - 1)] = pair20(u, v)
    out = np.zeros((B, N_OUT), dtype=np.float64)
    for i in range(B):
        r = n - int(d1[i]) - int(d2[i])
        vals = argpair[i, :, :r].reshape(-1)
        vals = vals[vals >= 0]
        if len(vals):
            np.add.at(out[i], to20[vals], 1.0)
            out[i] /= len(vals)
    return out


# ---------------------------------------------------------------- integer model
# The deployed form of the selector: int8 weights and activations, int32
# sums, so that every score is an exact integer.  A blob of int32 holds
#   [0] the feature scale sx (float32 bits), [1..4] M1, S1, M2, S2,
#   W1[64][64], b1[64], W2[64][64], b2[64], W3[190][64], b3[190].
Q_HEAD = 5
Q_LEN = Q_HEAD + N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_OUT * N_HID + N_OUT


def quant_unpack(blob):
    """(sx float32, M1, S1, M2, S2, W1, b1, W2, b2, W3, b3) with int64 arrays."""
    b = np.asarray(blob, dtype=np.int64).reshape(-1)
    assert b.size == Q_LEN
    sx = np.array([b[0]], dtype=np.int64).astype(np.uint32).view(np.float32)[0]
    o = Q_HEAD
    out = []
    for shape in ((N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_OUT, N_HID), (N_OUT,)):
        size = int(np.prod(shape))
        out.append(b[o:o + size].reshape(shape))
        o += size
    return (sx, int(b[1]), int(b[2]), int(b[3]), int(b[4]), *out)


def quant_code(c, q) -> int:
    """clamp(rint(float32(c) * q), 0, 127), the product in float32 (ties to even)."""
    v = np.float32(c) * np.float32(q)
    return int(min(max(np.rint(v), np.float32(0)), np.float32(127)))


def quant_features(p, perm, d1, d2, sx):
    """int64 [B, 64] feature codes of the integer model: each feature of
    features() has an integer numerator c (C1, C2, R, LB1 over the largest
    machine load norm; d1, d2 and the unscheduled count over n) and its code is
    quant_code(c, sx / norm) or quant_code(c, sx / n), both quotients in
    float32."""
    import oracle
    p = np.asarray(p)
    n, m = p.shape
    norm = np.float32(int(p.sum(axis=0).max()))
    qs = np.float32(np.float32(sx) / norm)
    qd = np.float32(np.float32(sx) / np.float32(n))
    out = np.zeros((len(perm), N_IN), dtype=np.int64)
    for i in range(len(perm)):
        a, b = int(d1[i]), int(d2[i])
        C1 = oracle.front(p, perm[i][:a])
        C2 = oracle.back(p, perm[i][n - b:])
        R = p[perm[i][a:n - b]].sum(axis=0).astype(np.int64)
        for k in range(min(m, M_MAX)):
            out[i, k] = quant_code(int(C1[k]), qs)
            out[i, 20 + k] = quant_code(int(C2[k]), qs)
            out[i, 40 + k] = quant_code(int(R[k]), qs)
        out[i, 60] = quant_code(a, qd)
        out[i, 61] = quant_code(b, qd)
        out[i, 62] = quant_code(n - a - b, qd)
        out[i, 63] = quant_code(int(oracle.lb1_parts(C1, R, C2)), qs)
    return out


def requant(a, M, S):
    """min(127, (max(a, 0) * M + 2^(S-1)) >> S): ReLU, then the fixed-point
    multiply by M / 2^S rounded half up, saturated to int8."""
    a = np.maximum(np.asarray(a, dtype=np.int64), 0)
    return np.minimum((a * M + (1 << (S - 1))) >> S, 127)


def quant_forward(blob, xq):
    """int64 scores [B, 190] of the integer model on feature codes xq [B, 64]."""
    _, M1, S1, M2, S2, W1, b1, W2, b2, W3, b3 = quant_unpack(blob)
    x = np.asarray(xq, dtype=np.int64)
    h1 = requant(x @ W1.T + b1, M1, S1)
    h2 = requant(h1 @ W2.T + b2, M2, S2)
    return h2 @ W3.T + b3


def quant_masks(blob, p, perm, d1, d2, k):
    """bool [B, 190]: the learned bound's pairs under the integer model."""
    sx = quant_unpack(blob)[0]
    s = quant_forward(blob, quant_features(p, perm, d1, d2, sx))
    return topk_mask(s, valid_pairs(np.asarray(p).shape[1]), k)
