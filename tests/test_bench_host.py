"""Host logic of bench.py: the algorithmic operation count behind the
roofline fraction, checked against its definition on hand-sized cases."""
import numpy as np

import bench


def _ops(n, m, pairs):
    d1 = np.array([a for a, _ in pairs], dtype=np.uint8)
    d2 = np.array([b for _, b in pairs], dtype=np.uint8)
    return bench.alg_ops_lb2(n, m, d1, d2)


def test_alg_ops_by_jobs_left():
    n, m = 20, 20
    P = m * (m - 1) // 2
    assert _ops(n, m, [(19, 0)]) == 8 * m                    # one job left: LB1 only
    assert _ops(n, m, [(10, 8)]) == 12 * m                   # two left: two completions
    assert _ops(n, m, [(10, 7)]) == 11 * 3 * P + 8 * 3 * m   # three left: the scans
    assert _ops(n, m, [(0, 0)]) == 11 * n * P + 8 * n * m    # the root
    assert _ops(n, m, [(19, 0), (10, 8), (0, 0)]) == (8 * m + 12 * m + 11 * n * P + 8 * n * m)


def test_alg_ops_never_exceed_a_full_scan():
    # at any depth the count stays below one pass over all n positions per
    # pair and direction with the children's work, so a fraction of the peak
    # computed from it cannot pass 1 for a kernel that scans everything
    n, m = 20, 20
    P = m * (m - 1) // 2
    for d in range(n):
        for a in range(d + 1):
            ops = _ops(n, m, [(a, d - a)])
            assert 0 < ops <= 11 * n * P + 8 * n * m
