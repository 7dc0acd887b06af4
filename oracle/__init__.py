"""ctypes wrapper of the plain C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

LB1, LB2_FULL, LB2_SUBSET = 1, 2, 3
INT32_MAX = 2**31 - 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP only for the batch loop)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror", "-fopenmp",
               "-shared", "-fPIC", os.path.join(HERE, "oracle.c"), "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.or_makespan.restype = i64
        L.or_makespan.argtypes = [i32, vp, vp, i32]
        L.or_front.argtypes = [i32, vp, vp, i32, vp]
        L.or_back.argtypes = [i32, vp, vp, i32, vp]
        L.or_lb1_parts.restype = i64
        L.or_lb1_parts.argtypes = [i32, vp, vp, vp]
        for f in (L.or_pair_value, L.or_pair_value_bruteforce):
            f.restype = i64
            f.argtypes = [i32, vp, vp, i32, i32, i32, i64, i64, i64, i64]
        L.or_johnson_lag_order.argtypes = [i32, vp, vp, i32, i32, i32]
        L.or_node_bound.restype = i64
        L.or_node_bound.argtypes = [i32, i32, vp, vp, i32, i32, i32, vp, vp]
        L.or_best_completion.restype = i64
        L.or_best_completion.argtypes = [i32, i32, vp, vp, i32, i32, vp]
        L.or_minmin.restype = i32
        L.or_minmin.argtypes = [i32, vp, vp]
        L.or_bound_children.restype = i32
        L.or_bound_children.argtypes = [i32, i32, vp, i32, vp, vp, vp, i32, i64, vp, i32,
                                        vp, vp, vp, vp, i32]
        L.or_search.restype = i32
        L.or_search.argtypes = [i32, i32, vp, i64, i32, i64, vp, vp, vp, vp, vp, vp]
        L.or_search_ex.restype = i32
        L.or_search_ex.argtypes = [i32, i32, vp, i64, i32, vp, i64, i32, i32, vp, vp, vp, vp, vp,
                                   vp]
        L.or_bruteforce.restype = i64
        L.or_bruteforce.argtypes = [i32, i32, vp, vp]
        L.or_neh.restype = i64
        L.or_neh.argtypes = [i32, i32, vp, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ci32(p):
    return np.ascontiguousarray(p, dtype=np.int32)


def _cu8(x):
    return np.ascontiguousarray(x, dtype=np.uint8)


def makespan(p, seq) -> int:
    p = _ci32(p)
    s = _cu8(seq)
    return int(lib().or_makespan(p.shape[1], _p(p), _p(s), len(s)))


def front(p, seq) -> np.ndarray:
    p = _ci32(p)
    s = _cu8(seq)
    out = np.zeros(p.shape[1], dtype=np.int64)
    lib().or_front(p.shape[1], _p(p), _p(s), len(s), _p(out))
    return out


def back(p, seq) -> np.ndarray:
    p = _ci32(p)
    s = _cu8(seq)
    out = np.zeros(p.shape[1], dtype=np.int64)
    lib().or_back(p.shape[1], _p(p), _p(s), len(s), _p(out))
    return out


def lb1_parts(C1, R, C2) -> int:
    a, b, c = (np.ascontiguousarray(x, dtype=np.int64) for x in (C1, R, C2))
    return int(lib().or_lb1_parts(len(a), _p(a), _p(b), _p(c)))


def pair_value(p, jobs, u, v, hu, hv, tu, tv, brute=False) -> int:
    p = _ci32(p)
    j = _cu8(jobs)
    f = lib().or_pair_value_bruteforce if brute else lib().or_pair_value
    return int(f(p.shape[1], _p(p), _p(j), len(j), u, v, hu, hv, tu, tv))


def johnson_lag_order(p, jobs, u, v) -> np.ndarray:
    p = _ci32(p)
    j = _cu8(jobs).copy()
    lib().or_johnson_lag_order(p.shape[1], _p(p), _p(j), len(j), u, v)
    return j


def node_bound(p, perm, d1, d2, kind=LB1, pair_mask=None, with_argpair=False):
    p = _ci32(p)
    perm = _cu8(perm)
    n, m = p.shape
    mask = None if pair_mask is None else np.ascontiguousarray(pair_mask, dtype=np.uint32)
    ap = np.full(1, -1, dtype=np.int32)
    x = int(lib().or_node_bound(n, m, _p(p), _p(perm), d1, d2, kind,
                                None if mask is None else _p(mask), _p(ap)))
    return (x, int(ap[0])) if with_argpair else x


def best_completion(p, perm, d1, d2):
    p = _ci32(p)
    perm = _cu8(perm)
    n, m = p.shape
    out = np.zeros(n, dtype=np.uint8)
    c = int(lib().or_best_completion(n, m, _p(p), _p(perm), d1, d2, _p(out)))
    return c, out


def minmin(lbf, lbb) -> int:
    a = np.ascontiguousarray(lbf, dtype=np.int64)
    b = np.ascontiguousarray(lbb, dtype=np.int64)
    return int(lib().or_minmin(len(a), _p(a), _p(b)))


def bound_children(p, perm, d1, d2, kind=LB1, ub=INT32_MAX, pair_mask=None,
                   with_argpair=False, threads=1):
    """Returns (lb int32 [N,2,n], prune uint8 [N,2,n], dir uint8 [N][, argpair int32 [N,2,n]])."""
    p = _ci32(p)
    n, m = p.shape
    perm = _cu8(perm).reshape(-1, n)
    N = perm.shape[0]
    d1 = _cu8(d1)
    d2 = _cu8(d2)
    lb = np.empty((N, 2, n), dtype=np.int32)
    pr = np.empty((N, 2, n), dtype=np.uint8)
    dr = np.empty(N, dtype=np.uint8)
    ap = np.empty((N, 2, n), dtype=np.int32) if with_argpair else None
    if pair_mask is not None:
        mask = np.ascontiguousarray(pair_mask, dtype=np.uint32).reshape(N, -1)
        words = mask.shape[1]
    else:
        mask, words = None, 0
    rc = lib().or_bound_children(n, m, _p(p), N, _p(perm), _p(d1), _p(d2), kind, int(ub),
                                 None if mask is None else _p(mask), words, _p(lb), _p(pr),
                                 _p(dr), None if ap is None else _p(ap), int(threads))
    if rc != 0:
        raise ValueError(f"or_bound_children failed with {rc}")
    return (lb, pr, dr, ap) if with_argpair else (lb, pr, dr)


def search(p, ub0=INT32_MAX, kind=LB1, budget=0, pair_mask=None, threads=1, lb1_r=0):
    """Depth-first B&B; returns dict(best, perm, nodes, children, found, proven).
    kind LB2_SUBSET bounds every node over the pairs of pair_mask (uint32 words);
    threads > 1 runs the OpenMP-task search (no budget).  lb1_r > 0: nodes with
    at most lb1_r unscheduled jobs bound their children with LB1 instead of
    kind (the bound chosen by depth; Section 2.4 ranks LB1 the cheaper)."""
    p = _ci32(p)
    n, m = p.shape
    best = np.zeros(1, dtype=np.int64)
    perm = np.zeros(n, dtype=np.uint8)
    nodes = np.zeros(1, dtype=np.int64)
    ch = np.zeros(1, dtype=np.int64)
    found = np.zeros(1, dtype=np.int32)
    proven = np.zeros(1, dtype=np.int32)
    mask = None if pair_mask is None else np.ascontiguousarray(pair_mask, dtype=np.uint32)
    rc = lib().or_search_ex(n, m, _p(p), int(ub0), kind, None if mask is None else _p(mask),
                            int(budget), int(threads), int(lb1_r), _p(best), _p(perm),
                            _p(nodes), _p(ch),
                            _p(found), _p(proven))
    if rc != 0:
        raise ValueError(f"or_search failed with {rc}")
    return dict(best=int(best[0]), perm=perm, nodes=int(nodes[0]), children=int(ch[0]),
                found=bool(found[0]), proven=bool(proven[0]))


def bruteforce(p):
    p = _ci32(p)
    n, m = p.shape
    out = np.zeros(n, dtype=np.uint8)
    c = int(lib().or_bruteforce(n, m, _p(p), _p(out)))
    return c, out


def neh(p):
    p = _ci32(p)
    n, m = p.shape
    out = np.zeros(n, dtype=np.uint8)
    c = int(lib().or_neh(n, m, _p(p), _p(out)))
    return c, out


def pair_index(m: int, u: int, v: int) -> int:
    """Lexicographic index of machine pair u < v among the m(m-1)/2 pairs."""
    return u * (2 * m - u - 1) // 2 + (v - u - 1)
