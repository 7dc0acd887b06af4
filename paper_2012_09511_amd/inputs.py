"""Seeded synthetic inputs for the flow-shop bounding path.

This module only draws random numbers and arranges them into the shapes the
library and its checks consume. It holds none of the method's arithmetic: no
makespans, bounds or orderings are computed here.

Instances follow the structure of Taillard's benchmark classes used in the
paper's experiments (Section 5): integer processing times drawn uniformly
from [1, 99] for n jobs on m machines.  A job-correlated variant draws a
per-job base time a_j in [1, 99] and adds a uniform [0, 20] term per machine.

Pools are bidirectional partial schedules (Section 2.3): a permutation of
the n jobs whose first d1 entries form the prefix sigma1, whose last d2 entries
form the suffix sigma2, and whose middle holds the unscheduled jobs.
"""
from __future__ import annotations

import numpy as np

PMIN, PMAX = 1, 99


def instance(n: int, m: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """Processing times p[j, k] (int32, shape (n, m)), row j = job, column k = machine."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(PMIN, PMAX + 1, size=(n, m), dtype=np.int32)
    if kind == "correlated":
        a = rng.integers(PMIN, PMAX + 1, size=(n, 1), dtype=np.int32)
        return (a + rng.integers(0, 21, size=(n, m), dtype=np.int32)).astype(np.int32)
    raise ValueError(f"unknown instance kind {kind!r}")


def random_pool(n: int, count: int, seed: int, depth: int | None = None,
                max_depth: int | None = None):
    """A pool of `count` random bidirectional partial schedules.

    Total depth d = d1 + d2 is uniform on {0, ..., max_depth} (default n - 2)
    unless `depth` fixes it; d1 is uniform on {0, ..., d}; d2 = d - d1; the
    permutation is uniform.  Returns (perm uint8 [count, n], d1 uint8 [count],
    d2 uint8 [count]).
    """
    if not 2 <= n <= 255:
        raise ValueError("n must be in [2, 255]")
    rng = np.random.default_rng(seed)
    hi = n - 2 if max_depth is None else max_depth
    if depth is None:
        d = rng.integers(0, hi + 1, size=count)
    else:
        d = np.full(count, depth, dtype=np.int64)
    if count and (d.max() > n - 1):
        raise ValueError("depth must leave at least one unscheduled job")
    d1 = (rng.random(count) * (d + 1)).astype(np.int64)
    d1 = np.minimum(d1, d)
    d2 = d - d1
    perm = rng.permuted(np.tile(np.arange(n, dtype=np.uint8), (count, 1)), axis=1)
    return (np.ascontiguousarray(perm, dtype=np.uint8), d1.astype(np.uint8),
            d2.astype(np.uint8))


def mixed_instances(count: int, seed: int, ns=(20, 50, 100), ms=(5, 10, 20),
                    correlated_every: int = 4):
    """A list of (n, m, p) instances, (n, m) taken round-robin over ns x ms.

    Every `correlated_every`-th instance (index i with i % correlated_every ==
    correlated_every - 1) uses job-correlated times, i.e. 25 % of them by default.
    """
    shapes = [(n, m) for n in ns for m in ms]
    out = []
    for i in range(count):
        n, m = shapes[i % len(shapes)]
        kind = "correlated" if i % correlated_every == correlated_every - 1 else "uniform"
        out.append((n, m, instance(n, m, seed + i, kind)))
    return out


def selector_params(seed: int, n_in: int = 64, n_hidden: int = 64, n_out: int = 190,
                    scale: float = 1.0):
    """Random initial parameters of the pair-selector MLP (fp32 master copies).

    Layer l has weight W_l [out, in] and bias b_l [out]; weights are drawn from
    U(-s, s) with s = scale / sqrt(in).
    """
    rng = np.random.default_rng(seed)
    dims = [(n_hidden, n_in), (n_hidden, n_hidden), (n_out, n_hidden)]
    params = []
    for (o, i) in dims:
        s = scale / np.sqrt(i)
        params.append(rng.uniform(-s, s, size=(o, i)).astype(np.float32))
        params.append(np.zeros(o, dtype=np.float32))
    return params
