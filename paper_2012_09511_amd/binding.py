"""Thin ctypes binding of libpfsp.so (include/pfsp.h).

Only argument marshalling happens here: torch tensors provide device memory
and the stream; every step of the bounding path runs in the library's HIP
kernels.  Importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpfsp.so")

PFSP_OK, PFSP_BUDGET = 0, 1
PFSP_EINVAL, PFSP_ENOINST, PFSP_ERANGE, PFSP_ENOMEM, PFSP_EDEVICE = -1, -2, -3, -4, -5
LB1, LB2_FULL, LB2_SUBSET, LB2_LEARNED = 1, 2, 3, 4
INT32_MAX = 2**31 - 1

# every symbol declared in include/pfsp.h
EXPORTS = ["pfsp_create", "pfsp_destroy", "pfsp_last_error", "pfsp_load_instance",
           "pfsp_pair_count", "pfsp_bound_children", "pfsp_check", "pfsp_search", "pfsp_neh",
           "pfsp_set_option", "pfsp_get_option", "pfsp_kernel_time", "pfsp_selector_set",
           "pfsp_selector_get", "pfsp_selector_features", "pfsp_selector_forward",
           "pfsp_selector_select", "pfsp_selector_targets", "pfsp_selector_train_step",
           "pfsp_search_log", "pfsp_multi_create", "pfsp_multi_destroy", "pfsp_multi_bound",
           "pfsp_multi_set_shape", "pfsp_multi_autotune", "pfsp_autotune",
           "pfsp_selector_set_quant", "pfsp_selector_infer", "pfsp_bound_children_noalloc",
           "pfsp_pair_mask", "pfsp_search_set_pairs", "pfsp_search_dump", "pfsp_search_resume",
           "pfsp_search_ivm", "pfsp_search_ivm_dump", "pfsp_search_ivm_resume",
           "pfsp_factoradic", "pfsp_ivm_decode"]
PAIRS_ADJACENT, PAIRS_LAST = 1, 2
SELECTOR_PARAMS = 20670
SELECTOR_QPARAMS = 20675


class PfspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pfsp error {code}: {msg}")
        self.code = code


class Pool(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n", ctypes.c_int32),
                ("perm", ctypes.c_void_p), ("d1", ctypes.c_void_p), ("d2", ctypes.c_void_p),
                ("pair_mask", ctypes.c_void_p), ("mask_words", ctypes.c_int32),
                ("dir_out", ctypes.c_void_p), ("argpair_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("best_cmax", ctypes.c_int32), ("found", ctypes.c_int32),
                ("proven", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("nodes_decomposed", ctypes.c_int64), ("children_bounded", ctypes.c_int64),
                ("max_pool", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("best_perm", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2012_09511_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.pfsp_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
        L.pfsp_create.restype = ctypes.c_int
        L.pfsp_destroy.argtypes = [vp]
        L.pfsp_destroy.restype = None
        L.pfsp_last_error.argtypes = [vp]
        L.pfsp_last_error.restype = ctypes.c_char_p
        L.pfsp_load_instance.argtypes = [vp, i32, i32, vp]
        L.pfsp_pair_count.argtypes = [vp]
        L.pfsp_bound_children.argtypes = [vp, ctypes.POINTER(Pool), ctypes.c_int, i32, vp, vp]
        L.pfsp_bound_children_noalloc.argtypes = [vp, ctypes.POINTER(Pool), ctypes.c_int, i32,
                                                  vp, vp]
        L.pfsp_check.argtypes = [vp]
        L.pfsp_pair_mask.argtypes = [vp, ctypes.c_int, vp, i32]
        L.pfsp_search_set_pairs.argtypes = [vp, vp, i32]
        L.pfsp_search_dump.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
        L.pfsp_search_ivm.argtypes = [vp, i32, i64, ctypes.c_int, i32, ctypes.POINTER(Result),
                                      ctypes.POINTER(i64)]
        L.pfsp_search_ivm_dump.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
        L.pfsp_search_ivm_resume.argtypes = [vp, vp, i64, i64, ctypes.POINTER(Result),
                                             ctypes.POINTER(i64)]
        L.pfsp_factoradic.argtypes = [ctypes.c_int, i32, vp, i32, vp, i32, vp,
                                      ctypes.POINTER(i32)]
        L.pfsp_ivm_decode.argtypes = [i32, vp, vp, vp, i32, vp, ctypes.POINTER(i32),
                                      ctypes.POINTER(i32)]
        L.pfsp_search_resume.argtypes = [vp, vp, i64, i64, ctypes.POINTER(Result)]
        L.pfsp_search.argtypes = [vp, i32, i64, ctypes.c_int, ctypes.POINTER(Result)]
        L.pfsp_neh.argtypes = [vp, vp, vp]
        L.pfsp_set_option.argtypes = [vp, ctypes.c_char_p, i64]
        L.pfsp_get_option.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i64)]
        L.pfsp_kernel_time.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(i64), ctypes.c_int]
        L.pfsp_search_log.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.pfsp_autotune.argtypes = [vp, ctypes.POINTER(Pool), ctypes.c_int, i32, vp, vp, i32,
                                    ctypes.c_char_p, i32]
        L.pfsp_multi_create.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(vp)]
        L.pfsp_multi_destroy.argtypes = [vp]
        L.pfsp_multi_destroy.restype = None
        L.pfsp_multi_bound.argtypes = [vp, ctypes.c_int, vp, vp, vp, i32, vp, vp, vp, vp, vp]
        L.pfsp_multi_set_shape.argtypes = [vp, i32, i32, i32, i32]
        L.pfsp_multi_autotune.argtypes = [vp, ctypes.c_int, vp, vp, vp, i32, vp, vp, vp, vp, vp,
                                          i32, ctypes.c_char_p, i32]
        L.pfsp_selector_set.argtypes = [vp, vp, i64]
        L.pfsp_selector_get.argtypes = [vp, vp, i64]
        L.pfsp_selector_features.argtypes = [vp, ctypes.POINTER(Pool), vp]
        L.pfsp_selector_forward.argtypes = [vp, vp, i32, vp]
        L.pfsp_selector_select.argtypes = [vp, vp, i32, i32, vp]
        L.pfsp_selector_targets.argtypes = [vp, ctypes.POINTER(Pool), vp, vp]
        L.pfsp_selector_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float,
                                               ctypes.POINTER(ctypes.c_float), vp]
        L.pfsp_selector_set_quant.argtypes = [vp, vp, i64]
        L.pfsp_selector_infer.argtypes = [vp, ctypes.POINTER(Pool), i32, vp]
        for name in EXPORTS:
            if name not in ("pfsp_destroy", "pfsp_last_error", "pfsp_multi_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def factoradic(op, a, atop=0, b=None, btop=0):
    """pfsp_factoradic on digit vectors: (digits, top)."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    n = len(a)
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(n, dtype=np.uint8)
    top = ctypes.c_int32()
    rc = lib().pfsp_factoradic(int(op), n, a.ctypes.data_as(ctypes.c_void_p), int(atop),
                               None if bb is None else bb.ctypes.data_as(ctypes.c_void_p),
                               int(btop), out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(top))
    if rc != 0:
        raise PfspError(rc, "pfsp_factoradic failed")
    return out, top.value


def ivm_decode(M, V, D, level):
    """pfsp_ivm_decode: (perm, d1, d2) of the node an IVM designates."""
    M = np.ascontiguousarray(M, dtype=np.uint8)
    n = M.shape[0]
    V = np.ascontiguousarray(V, dtype=np.uint8)
    D = np.ascontiguousarray(D, dtype=np.uint8)
    out = np.zeros(n, dtype=np.uint8)
    d1, d2 = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().pfsp_ivm_decode(n, M.ctypes.data_as(ctypes.c_void_p),
                               V.ctypes.data_as(ctypes.c_void_p), D.ctypes.data_as(ctypes.c_void_p),
                               int(level), out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(d1),
                               ctypes.byref(d2))
    if rc != 0:
        raise PfspError(rc, "pfsp_ivm_decode failed")
    return out, d1.value, d2.value


class Context:
    """One library context on one device, launching on the current torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib().pfsp_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise PfspError(rc, "pfsp_create failed")
        self.h = h
        self.n = self.m = None

    def close(self):
        if self.h:
            lib().pfsp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise PfspError(rc, lib().pfsp_last_error(self.h).decode())
        return rc

    def load_instance(self, p):
        p = np.ascontiguousarray(p, dtype=np.int32)
        n, m = p.shape
        self._check(lib().pfsp_load_instance(self.h, n, m, p.ctypes.data_as(ctypes.c_void_p)))
        self.n, self.m = n, m
        self.P = self._check(lib().pfsp_pair_count(self.h))
        self.mask_words = max(1, (self.P + 31) // 32)

    def bound_children(self, perm, d1, d2, kind=LB1, ub=INT32_MAX, pair_mask=None,
                       out_lb=None, out_prune=None, dir_out=None, argpair_out=None,
                       want_dir=True, want_argpair=False):
        """Device tensors in, device tensors out: (lb [N,2,n] int32, prune [N,2,n] uint8,
        dir [N] uint8 or None, argpair [N,2,n] int16 or None)."""
        torch = self.torch
        N = perm.shape[0]
        n = self.n
        if out_lb is None:
            out_lb = torch.empty((N, 2, n), dtype=torch.int32, device=self.device)
        if out_prune is None:
            out_prune = torch.empty((N, 2, n), dtype=torch.uint8, device=self.device)
        if dir_out is None and want_dir:
            dir_out = torch.empty(N, dtype=torch.uint8, device=self.device)
        if argpair_out is None and want_argpair:
            argpair_out = torch.empty((N, 2, n), dtype=torch.int16, device=self.device)
        for t, dt in ((perm, torch.uint8), (d1, torch.uint8), (d2, torch.uint8)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError("perm/d1/d2 must be contiguous uint8 device tensors")
        pool = Pool(N, perm.shape[1] if perm.dim() == 2 else n, _ptr(perm), _ptr(d1), _ptr(d2),
                    _ptr(pair_mask), 0 if pair_mask is None else pair_mask.shape[-1],
                    _ptr(dir_out), _ptr(argpair_out))
        self._check(lib().pfsp_bound_children(self.h, ctypes.byref(pool), kind, int(ub),
                                              _ptr(out_lb), _ptr(out_prune)))
        return out_lb, out_prune, dir_out, argpair_out

    def pair_mask(self, variant) -> np.ndarray:
        """Host bit mask (uint32 words) of a fixed pair variant on the loaded instance."""
        words = (self.m * (self.m - 1) // 2 + 31) // 32
        out = np.zeros(max(words, 1), dtype=np.uint32)
        self._check(lib().pfsp_pair_mask(self.h, int(variant),
                                         out.ctypes.data_as(ctypes.c_void_p), len(out)))
        return out

    def search_set_pairs(self, mask):
        """Pair set of PFSP_LB2_SUBSET searches (host uint32 words)."""
        mask = np.ascontiguousarray(mask, dtype=np.uint32)
        self._check(lib().pfsp_search_set_pairs(self.h, mask.ctypes.data_as(ctypes.c_void_p),
                                                len(mask)))

    def bound_children_noalloc(self, perm, d1, d2, out_lb, out_prune, kind=LB1, ub=INT32_MAX,
                               pair_mask=None, dir_out=None):
        """pfsp_bound_children_noalloc on caller-allocated device outputs."""
        N = perm.shape[0]
        pool = Pool(N, perm.shape[1] if perm.dim() == 2 else self.n, _ptr(perm), _ptr(d1),
                    _ptr(d2), _ptr(pair_mask), 0 if pair_mask is None else pair_mask.shape[-1],
                    _ptr(dir_out), None)
        self._check(lib().pfsp_bound_children_noalloc(self.h, ctypes.byref(pool), kind, int(ub),
                                                      _ptr(out_lb), _ptr(out_prune)))
        return out_lb, out_prune, dir_out

    def autotune(self, perm, d1, d2, kind=LB2_FULL, ub=INT32_MAX, reps=3, pair_mask=None):
        """Times LB2 block shapes on this pool and keeps the fastest; returns the report."""
        import json
        torch = self.torch
        N = perm.shape[0]
        lb = torch.empty((N, 2, self.n), dtype=torch.int32, device=self.device)
        pr = torch.empty((N, 2, self.n), dtype=torch.uint8, device=self.device)
        pool = Pool(N, self.n, _ptr(perm), _ptr(d1), _ptr(d2), _ptr(pair_mask),
                    0 if pair_mask is None else pair_mask.shape[-1], None, None)
        buf = ctypes.create_string_buffer(4096)
        self._check(lib().pfsp_autotune(self.h, ctypes.byref(pool), kind, int(ub), _ptr(lb),
                                        _ptr(pr), reps, buf, 4096))
        return json.loads(buf.value.decode())

    def check(self):
        return self._check(lib().pfsp_check(self.h))

    @staticmethod
    def _result(res, perm, rc):
        return dict(best=res.best_cmax, found=bool(res.found), proven=bool(res.proven),
                    steps=res.steps, nodes=res.nodes_decomposed,
                    children=res.children_bounded, max_pool=res.max_pool,
                    seconds=res.seconds, perm=perm.astype(np.uint8), budget_hit=rc == 1)

    def search(self, ub0=INT32_MAX, budget=0, kind=LB1):
        perm = np.zeros(self.n, dtype=np.int32)
        res = Result()
        res.best_perm = perm.ctypes.data_as(ctypes.c_void_p)
        rc = self._check(lib().pfsp_search(self.h, int(ub0), int(budget), kind,
                                           ctypes.byref(res)))
        return self._result(res, perm, rc)

    def search_ivm(self, ub0=INT32_MAX, budget=0, kind=LB1, explorers=4096):
        """IVM explorers with factoradic work units and work stealing."""
        perm = np.zeros(self.n, dtype=np.int32)
        res = Result()
        res.best_perm = perm.ctypes.data_as(ctypes.c_void_p)
        steals = ctypes.c_int64()
        rc = self._check(lib().pfsp_search_ivm(self.h, int(ub0), int(budget), kind,
                                               int(explorers), ctypes.byref(res),
                                               ctypes.byref(steals)))
        out = self._result(res, perm, rc)
        out["steals"] = steals.value
        return out

    def search_ivm_dump(self) -> bytes:
        """Checkpoint of the last IVM search that stopped on its budget."""
        size = ctypes.c_int64()
        self._check(lib().pfsp_search_ivm_dump(self.h, None, 0, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        self._check(lib().pfsp_search_ivm_dump(self.h, buf, size.value, ctypes.byref(size)))
        return buf.raw[:size.value]

    def search_ivm_resume(self, ckpt: bytes, budget=0):
        perm = np.zeros(self.n, dtype=np.int32)
        res = Result()
        res.best_perm = perm.ctypes.data_as(ctypes.c_void_p)
        steals = ctypes.c_int64()
        rc = self._check(lib().pfsp_search_ivm_resume(self.h, ckpt, len(ckpt), int(budget),
                                                      ctypes.byref(res), ctypes.byref(steals)))
        out = self._result(res, perm, rc)
        out["steals"] = steals.value
        return out

    def search_dump(self) -> bytes:
        """Checkpoint of the last search that stopped on its budget."""
        size = ctypes.c_int64()
        self._check(lib().pfsp_search_dump(self.h, None, 0, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        self._check(lib().pfsp_search_dump(self.h, buf, size.value, ctypes.byref(size)))
        return buf.raw[:size.value]

    def search_resume(self, ckpt: bytes, budget=0):
        perm = np.zeros(self.n, dtype=np.int32)
        res = Result()
        res.best_perm = perm.ctypes.data_as(ctypes.c_void_p)
        rc = self._check(lib().pfsp_search_resume(self.h, ckpt, len(ckpt), int(budget),
                                                  ctypes.byref(res)))
        return self._result(res, perm, rc)

    def search_log(self, max_records):
        """Nodes logged by the last search: (perm [k, n] u8, d1 [k], d2 [k]) on the host."""
        perm = np.zeros((max_records, self.n), dtype=np.uint8)
        d1 = np.zeros(max_records, dtype=np.uint8)
        d2 = np.zeros(max_records, dtype=np.uint8)
        k = ctypes.c_int64()
        self._check(lib().pfsp_search_log(self.h, perm.ctypes.data_as(ctypes.c_void_p),
                                          d1.ctypes.data_as(ctypes.c_void_p),
                                          d2.ctypes.data_as(ctypes.c_void_p), max_records,
                                          ctypes.byref(k)))
        return perm[:k.value], d1[:k.value], d2[:k.value]

    def neh(self):
        perm = np.zeros(self.n, dtype=np.int32)
        c = np.zeros(1, dtype=np.int32)
        self._check(lib().pfsp_neh(self.h, perm.ctypes.data_as(ctypes.c_void_p),
                                   c.ctypes.data_as(ctypes.c_void_p)))
        return int(c[0]), perm.astype(np.uint8)

    def set_option(self, key: str, value: int):
        self._check(lib().pfsp_set_option(self.h, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = ctypes.c_int64()
        self._check(lib().pfsp_get_option(self.h, key.encode(), ctypes.byref(v)))
        return v.value

    def kernel_time(self, kernel: str, reset: bool = False):
        """(total ms, launches) of a kernel since the last reset (option "timing")."""
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        self._check(lib().pfsp_kernel_time(self.h, kernel.encode(), ctypes.byref(ms),
                                           ctypes.byref(k), int(reset)))
        return ms.value, k.value

    # ---------------------------------------------------------------- selector
    def _pool(self, perm, d1, d2):
        return Pool(perm.shape[0], self.n, _ptr(perm), _ptr(d1), _ptr(d2), None, 0, None, None)

    def selector_set(self, params):
        """params: list [W1, b1, W2, b2, W3, b3] (float32) or a flat array of 20670."""
        flat = np.concatenate([np.asarray(p, dtype=np.float32).reshape(-1) for p in params]) \
            if isinstance(params, (list, tuple)) else np.asarray(params, dtype=np.float32)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(lib().pfsp_selector_set(self.h, flat.ctypes.data_as(ctypes.c_void_p),
                                            flat.size))

    def selector_get(self):
        out = np.empty(SELECTOR_PARAMS, dtype=np.float32)
        self._check(lib().pfsp_selector_get(self.h, out.ctypes.data_as(ctypes.c_void_p),
                                            out.size))
        return out

    def selector_set_quant(self, blob):
        """blob: int32 array of 20675 (the integer model), or None for the float model."""
        if blob is None:
            self._check(lib().pfsp_selector_set_quant(self.h, None, 0))
            return
        flat = np.ascontiguousarray(np.asarray(blob, dtype=np.int32).reshape(-1))
        self._check(lib().pfsp_selector_set_quant(self.h, flat.ctypes.data_as(ctypes.c_void_p),
                                                  flat.size))

    def selector_infer(self, perm, d1, d2, k):
        """Pair masks [N][ceil(P/32)] (int32 view of the uint32 words) of the learned bound."""
        torch = self.torch
        out = torch.empty((perm.shape[0], self.mask_words), dtype=torch.int32,
                          device=self.device)
        pool = self._pool(perm, d1, d2)
        self._check(lib().pfsp_selector_infer(self.h, ctypes.byref(pool), int(k), _ptr(out)))
        return out

    def selector_features(self, perm, d1, d2):
        torch = self.torch
        out = torch.empty((perm.shape[0], 64), dtype=torch.float32, device=self.device)
        pool = self._pool(perm, d1, d2)
        self._check(lib().pfsp_selector_features(self.h, ctypes.byref(pool), _ptr(out)))
        return out

    def selector_forward(self, x):
        torch = self.torch
        out = torch.empty((x.shape[0], 190), dtype=torch.float32, device=self.device)
        self._check(lib().pfsp_selector_forward(self.h, _ptr(x), x.shape[0], _ptr(out)))
        return out

    def selector_select(self, scores, k):
        torch = self.torch
        out = torch.empty((scores.shape[0], self.mask_words), dtype=torch.int32,
                          device=self.device)
        self._check(lib().pfsp_selector_select(self.h, _ptr(scores), scores.shape[0], int(k),
                                               _ptr(out)))
        return out

    def selector_targets(self, perm, d1, d2, argpair):
        torch = self.torch
        out = torch.empty((perm.shape[0], 190), dtype=torch.float32, device=self.device)
        pool = self._pool(perm, d1, d2)
        self._check(lib().pfsp_selector_targets(self.h, ctypes.byref(pool), _ptr(argpair),
                                                _ptr(out)))
        return out

    def selector_train_step(self, x, target, lr, want_grad=False):
        torch = self.torch
        loss = ctypes.c_float()
        g = torch.empty(SELECTOR_PARAMS, dtype=torch.float32, device=self.device) \
            if want_grad else None
        self._check(lib().pfsp_selector_train_step(self.h, _ptr(x), _ptr(target), x.shape[0],
                                                   float(lr), ctypes.byref(loss), _ptr(g)))
        return loss.value, g


class Multi:
    """Several instances bounded together (pfsp_multi_*); owned by a Context."""

    def __init__(self, ctx: Context, instances):
        """instances: list of int32 arrays p[n, m]."""
        self.ctx = ctx
        ps = [np.ascontiguousarray(p, dtype=np.int32) for p in instances]
        self.shapes = [p.shape for p in ps]
        ns = np.array([s[0] for s in self.shapes], dtype=np.int32)
        ms = np.array([s[1] for s in self.shapes], dtype=np.int32)
        ptrs = (ctypes.c_void_p * len(ps))(*[p.ctypes.data for p in ps])
        h = ctypes.c_void_p()
        ctx._check(lib().pfsp_multi_create(ctx.h, len(ps), ns.ctypes.data_as(ctypes.c_void_p),
                                           ms.ctypes.data_as(ctypes.c_void_p), ptrs,
                                           ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().pfsp_multi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _args(self, perm, d1, d2, seg, ub, out):
        seg = np.ascontiguousarray(seg, dtype=np.int64)
        ub = np.ascontiguousarray(ub, dtype=np.int32)
        lb, pr, dr = out
        return (_ptr(perm), _ptr(d1), _ptr(d2), perm.shape[1],
                seg.ctypes.data_as(ctypes.c_void_p), ub.ctypes.data_as(ctypes.c_void_p),
                _ptr(lb), _ptr(pr), _ptr(dr)), (seg, ub)

    def outputs(self, N, stride):
        torch = self.ctx.torch
        dev = self.ctx.device
        return (torch.empty((N, 2, stride), dtype=torch.int32, device=dev),
                torch.empty((N, 2, stride), dtype=torch.uint8, device=dev),
                torch.empty(N, dtype=torch.uint8, device=dev))

    def bound(self, perm, d1, d2, seg, ub, kind=LB2_FULL, out=None):
        if out is None:
            out = self.outputs(perm.shape[0], perm.shape[1])
        args, keep = self._args(perm, d1, d2, seg, ub, out)
        self.ctx._check(lib().pfsp_multi_bound(self.h, kind, *args))
        return out

    def set_shape(self, tile=256, waves_small=0, waves_large=0, blocks_per_cu=0):
        self.ctx._check(lib().pfsp_multi_set_shape(self.h, tile, waves_small, waves_large,
                                                   blocks_per_cu))

    def autotune(self, perm, d1, d2, seg, ub, kind=LB2_FULL, out=None, reps=3):
        import json
        if out is None:
            out = self.outputs(perm.shape[0], perm.shape[1])
        args, keep = self._args(perm, d1, d2, seg, ub, out)
        buf = ctypes.create_string_buffer(4096)
        self.ctx._check(lib().pfsp_multi_autotune(self.h, kind, *args, reps, buf, 4096))
        return json.loads(buf.value.decode())
