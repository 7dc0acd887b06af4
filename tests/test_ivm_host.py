"""Host checks of the IVM search's work-unit arithmetic and decoding
(pfsp_factoradic, pfsp_ivm_decode: no device needed).

Pinned against the textbook factorial number system (Section 2.6): digit L of
an n-digit position lies in [0, n - L) with weight (n - 1 - L)!, so the
lexicographic rank of a permutation is its Lehmer code read in this system,
and sums, differences and halvings agree with Python's integers."""
import itertools
import math

import numpy as np
import pytest

from paper_2012_09511_amd import binding


def to_int(d, top=0):
    n = len(d)
    return top * math.factorial(n) + sum(int(d[L]) * math.factorial(n - 1 - L) for L in range(n))


def from_int(v, n):
    top, v = divmod(v, math.factorial(n))
    d = []
    for L in range(n):
        w = math.factorial(n - 1 - L)
        d.append(v // w)
        v %= w
    return np.array(d, dtype=np.uint8), top


def test_lexicographic_rank_is_the_factoradic_value():
    """n = 5: V runs 00000, 00010, 00100, ..., 43210 over the 120 schedules in
    lexicographic order (the Lehmer code of each permutation)."""
    for rank, perm in enumerate(itertools.permutations(range(5))):
        rest = list(range(5))
        code = []
        for j in perm:
            code.append(rest.index(j))
            rest.remove(j)
        assert to_int(code) == rank
    assert to_int([0, 0, 0, 1, 0]) == 1 and to_int([4, 3, 2, 1, 0]) == 119


@pytest.mark.parametrize("n", [1, 2, 4, 5, 10, 20, 33, 64])
def test_factoradic_ops_match_integers(n):
    import random
    rng = random.Random(n)
    N = math.factorial(n)
    for _ in range(200):
        x, y = sorted((rng.randrange(N + 1), rng.randrange(N + 1)))
        a, at = from_int(x, n)
        b, bt = from_int(y, n)
        d, dt = binding.factoradic(1, a, at, b, bt)               # b - a
        assert to_int(d, dt) == y - x
        h, ht = binding.factoradic(2, b, bt)                      # b // 2
        assert to_int(h, ht) == y // 2
        mid, mt = binding.factoradic(3, a, at, b, bt)             # a + (b - a) // 2
        assert to_int(mid, mt) == x + (y - x) // 2
        if x + y <= N:
            s, st = binding.factoradic(0, a, at, b, bt)
            assert to_int(s, st) == x + y


def test_work_unit_example_n4():
    """Splitting [0, 4!) and its halves gives the midpoints of the integer
    interval; e.g. the right half of [16, 24) starts at 20 = 3100 in factoradic
    (the work units of Section 2.6, Figure 6)."""
    lo, _ = from_int(16, 4)
    hi, ht = from_int(24, 4)
    assert ht == 1 and not hi.any()                               # 4! itself
    mid, mt = binding.factoradic(3, lo, 0, hi, ht)
    assert (to_int(mid, mt), mid.tolist()) == (20, [3, 1, 0, 0])
    assert from_int(9, 4)[0].tolist() == [1, 1, 1, 0] and from_int(15, 4)[0].tolist() == [2, 1, 1, 0]


def test_ivm_decode_example_n5():
    """The n = 5 example of Section 2.5 (jobs numbered from 0 here): jobs 2, 1
    and 3 chosen at levels 0, 1, 2, the first scheduled at the front and the
    other two at the back, designate the node 2 / 0 4 / 3 1."""
    n = 5
    M = np.zeros((n, n), dtype=np.uint8)
    M[0, :5] = [0, 1, 2, 3, 4]
    M[1, :4] = [0, 1, 3, 4]          # row 0 without job 2
    M[2, :3] = [0, 3, 4]             # row 1 without job 1
    V = np.array([2, 1, 1], dtype=np.uint8)
    D = np.array([0, 1, 1], dtype=np.uint8)
    perm, d1, d2 = binding.ivm_decode(M, V, D, 2)
    assert (perm.tolist(), d1, d2) == ([2, 0, 4, 3, 1], 1, 2)
    with pytest.raises(binding.PfspError):
        binding.ivm_decode(M, np.array([2, 4, 1], dtype=np.uint8), D, 2)   # V[1] >= n - 1
