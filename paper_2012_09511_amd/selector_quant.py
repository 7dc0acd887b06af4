"""Post-training quantization of the learned pair selector to its integer form.

The float model (weights rounded to bfloat16, float32 activations) is mapped
to int8 weights and activations with int32 sums, the form the bound kernels
run (blob layout of pfsp_selector_set_quant):
  * weights: one symmetric scale per layer, 127 / max |W|;
  * features: scale sx = 127 / (the `pct` percentile of the calibration
    features), codes clamp(rint(x * sx), 0, 127);
  * hidden layers: the code scale of h is 127 / (its `pct` percentile on the
    calibration rows), reached from the int32 sums by the fixed-point multiply
    M / 2^S (M in [512, 1023] when the range allows);
  * biases in the units of each layer's sums.
Calibration features come from pfsp_selector_features on representative
nodes.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 64, 64, 190
Q_LEN = 5 + N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_OUT * N_HID + N_OUT
B_LIM = (1 << 19) - 1


def _wq(W):
    amax = float(np.abs(W).max())
    s = 127.0 / amax if amax > 0 else 1.0
    return np.clip(np.rint(W * s), -127, 127).astype(np.int64), s


def _fixed_point(mult):
    """(M, S) with M / 2^S close to mult, M <= 1023, 1 <= S <= 30."""
    S = int(np.floor(np.log2(1023.0 / mult))) if mult > 0 else 30
    S = min(max(S, 1), 30)
    M = int(np.clip(np.rint(mult * 2.0 ** S), 1, 1023))
    return M, S


def _requant(a, M, S):
    return np.minimum((np.maximum(a, 0) * M + (1 << (S - 1))) >> S, 127)


def quantize(params, X, pct=99.9):
    """int32 blob of the integer model from the float parameters
    [W1, b1, W2, b2, W3, b3] and calibration features X [N, 64] (float)."""
    if not isinstance(params, (list, tuple)):      # flat layout of pfsp_selector_set
        flat = np.asarray(params, dtype=np.float64).reshape(-1)
        sizes = [N_HID * N_IN, N_HID, N_HID * N_HID, N_HID, N_OUT * N_HID, N_OUT]
        shapes = [(N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_OUT, N_HID), (N_OUT,)]
        offs = np.cumsum([0] + sizes)
        params = [flat[offs[i]:offs[i + 1]].reshape(shapes[i]) for i in range(6)]
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    X = np.asarray(X, dtype=np.float64)
    xr = float(np.percentile(X, pct)) if X.size else 1.0
    sx = np.float32(127.0 / max(xr, 1e-6))
    xq = np.clip(np.rint(X * float(sx)), 0, 127).astype(np.int64)
    scale_in = float(sx)
    head = [int(np.array([sx], dtype=np.float32).view(np.int32)[0])]
    layers = []
    h = xq
    for W, b in ((W1, b1), (W2, b2)):
        Wq, sw = _wq(W)
        acc_scale = sw * scale_in                       # real value = sum / acc_scale
        bq = np.clip(np.rint(b * acc_scale), -B_LIM, B_LIM).astype(np.int64)
        a = h @ Wq.T + bq
        real = np.maximum(a, 0) / acc_scale
        hr = float(np.percentile(real, pct)) if real.size else 1.0
        s_out = 127.0 / max(hr, 1e-6)
        M, S = _fixed_point(s_out / acc_scale)
        head += [M, S]
        layers += [Wq, bq]
        h = _requant(a, M, S)
        scale_in = acc_scale * M / 2.0 ** S             # code = real * scale_in
    W3q, sw3 = _wq(W3)
    b3q = np.clip(np.rint(b3 * sw3 * scale_in), -B_LIM, B_LIM).astype(np.int64)
    layers += [W3q, b3q]
    blob = np.concatenate([np.array(head, dtype=np.int64)] + [a.reshape(-1) for a in layers])
    assert blob.size == Q_LEN
    return blob.astype(np.int32)


def calibration_features(ctx, n, count=8192, seed=77):
    """Selector features of `count` random nodes (uniform depth and split) of
    the loaded instance, as a host array [count, 64]."""
    import torch

    from . import inputs
    perm, d1, d2 = inputs.random_pool(n, count, seed)
    dev = [torch.from_numpy(a).to(ctx.device) for a in (perm, d1, d2)]
    x = ctx.selector_features(*dev)
    torch.cuda.synchronize()
    return x.cpu().numpy()
