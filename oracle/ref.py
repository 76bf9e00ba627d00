"""ctypes binding of the C oracle (oracle/pcba_ref.h).

TEST INFRASTRUCTURE ONLY: see the header of pcba_ref.h.  Takes numpy arrays;
imports nothing from the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

MAX_DIM = 8
RUNNING, OPTIMAL, INFEASIBLE, MEMORY_LIMIT, MAX_ITER = -1, 0, 1, 2, 3
OUTCOME_NAMES = {OPTIMAL: "optimal", INFEASIBLE: "infeasible",
                 MEMORY_LIMIT: "memory_limit", MAX_ITER: "max_iter", RUNNING: "running"}


class RefResult(C.Structure):
    _fields_ = [("outcome", C.c_int), ("has_x", C.c_int),
                ("p_up", C.c_double), ("p_lo", C.c_double),
                ("x_lo", C.c_double * MAX_DIM), ("x_hi", C.c_double * MAX_DIM),
                ("x_depth", C.c_int * MAX_DIM), ("x_index", C.c_uint * MAX_DIM),
                ("rounds", C.c_int), ("steps", C.c_int),
                ("list_len", C.c_longlong), ("peak_len", C.c_longlong),
                ("depth", C.c_int * MAX_DIM), ("next_dir", C.c_int)]


_lib = None


def lib():
    """The oracle library built from oracle/pcba_ref.c (rebuilt if stale)."""
    global _lib
    if _lib is None:
        path = _build.LIB
        src = os.path.join(os.path.dirname(path), "pcba_ref.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        _lib = load(path)
    return _lib


def load(path):
    """Loads an oracle build at `path` (the tests also load mutated builds)."""
    if True:
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
        L.pcba_ref_to_bernstein.argtypes = [C.c_int, ip, dp, dp, dp, dp]
        L.pcba_ref_to_bernstein.restype = C.c_int
        L.pcba_ref_split.argtypes = [C.c_int, ip, C.c_int, dp, dp, dp]
        L.pcba_ref_split.restype = C.c_int
        L.pcba_ref_split_at.argtypes = [C.c_int, ip, C.c_int, C.c_double, dp, dp, dp]
        L.pcba_ref_split_at.restype = C.c_int
        L.pcba_ref_set_split.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.pcba_ref_set_split.restype = C.c_int
        L.pcba_ref_split_round.argtypes = [C.c_int, ip, dp, dp]
        L.pcba_ref_split_round.restype = C.c_int
        L.pcba_ref_set_fused.argtypes = [C.c_void_p, C.c_int]
        L.pcba_ref_set_fused.restype = C.c_int
        L.pcba_ref_create.argtypes = [C.c_int, dp, dp, ip, dp, C.c_int, C.c_void_p, C.c_void_p,
                                      C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                      C.c_double, C.c_longlong, C.c_int]
        L.pcba_ref_create.restype = C.c_void_p
        L.pcba_ref_step.argtypes = [C.c_void_p]
        L.pcba_ref_step.restype = C.c_int
        L.pcba_ref_solve.argtypes = [C.c_void_p]
        L.pcba_ref_solve.restype = C.c_int
        L.pcba_ref_result_get.argtypes = [C.c_void_p, C.POINTER(RefResult)]
        L.pcba_ref_result_get.restype = None
        L.pcba_ref_patch_words.argtypes = [C.c_void_p]
        L.pcba_ref_patch_words.restype = C.c_longlong
        L.pcba_ref_kind_degree.argtypes = [C.c_void_p, C.c_int, ip]
        L.pcba_ref_kind_degree.restype = None
        L.pcba_ref_list.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.pcba_ref_list.restype = None
        L.pcba_ref_derive.argtypes = [C.c_void_p, ip, up, dp]
        L.pcba_ref_derive.restype = C.c_int
        L.pcba_ref_destroy.argtypes = [C.c_void_p]
        L.pcba_ref_destroy.restype = None
    return L


def to_bernstein(mono: np.ndarray, lo, hi, L=None) -> np.ndarray:
    """Bernstein coefficients of a monomial tensor over the box [lo, hi]."""
    mono = np.ascontiguousarray(mono, dtype=np.float64)
    deg = np.array([s - 1 for s in mono.shape], dtype=np.int32)
    out = np.empty_like(mono)
    rc = (L or lib()).pcba_ref_to_bernstein(mono.ndim, deg, np.ascontiguousarray(lo, dtype=np.float64),
                                     np.ascontiguousarray(hi, dtype=np.float64), mono.ravel(),
                                     out.reshape(-1))
    if rc != 0:
        raise ValueError("pcba_ref_to_bernstein rejected its arguments")
    return out


def split(patch: np.ndarray, r: int, L=None):
    """Left and right child patches of a midpoint split along axis r."""
    patch = np.ascontiguousarray(patch, dtype=np.float64)
    deg = np.array([s - 1 for s in patch.shape], dtype=np.int32)
    left = np.empty_like(patch)
    right = np.empty_like(patch)
    rc = (L or lib()).pcba_ref_split(patch.ndim, deg, r, patch.reshape(-1), left.reshape(-1),
                              right.reshape(-1))
    if rc != 0:
        raise ValueError("pcba_ref_split rejected its arguments")
    return left, right


def split_at(patch: np.ndarray, r: int, lam: float, L=None):
    """Children of a split along axis r at parameter lam (left: [a, a + lam (b-a)])."""
    patch = np.ascontiguousarray(patch, dtype=np.float64)
    deg = np.array([s - 1 for s in patch.shape], dtype=np.int32)
    left = np.empty_like(patch)
    right = np.empty_like(patch)
    rc = (L or lib()).pcba_ref_split_at(patch.ndim, deg, r, float(lam), patch.reshape(-1), left.reshape(-1),
                                        right.reshape(-1))
    if rc != 0:
        raise ValueError("pcba_ref_split_at rejected its arguments")
    return left, right


def split_round(patch: np.ndarray, L=None) -> np.ndarray:
    """The 2^l children of a patch bisected along every axis, axis 0 first;
    child c (axis 0's bit most significant) at out[c]."""
    patch = np.ascontiguousarray(patch, dtype=np.float64)
    deg = np.array([s - 1 for s in patch.shape], dtype=np.int32)
    out = np.empty((1 << patch.ndim,) + patch.shape)
    rc = (L or lib()).pcba_ref_split_round(patch.ndim, deg, patch.reshape(-1), out.reshape(-1))
    if rc != 0:
        raise ValueError("pcba_ref_split_round rejected its arguments")
    return out


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


class RefSolver:
    """One problem instance in the oracle.  `inst` is an instances.Instance-like
    object (l, lo, hi, cost_deg, cost_flat, ineq_deg, ineq_flat, eq_deg, eq_flat,
    eps, delta, eps_eq, max_boxes, max_iters)."""

    def __init__(self, inst, L=None, fused=False, rule=0, lam=0.5, **override):
        L = L or lib()
        self.L = L
        g = lambda k: override.get(k, getattr(inst, k))
        self.l = int(inst.l)
        self._keep = [np.ascontiguousarray(inst.ineq_deg, dtype=np.int32).ravel(),
                      np.ascontiguousarray(inst.ineq_flat, dtype=np.float64),
                      np.ascontiguousarray(inst.eq_deg, dtype=np.int32).ravel(),
                      np.ascontiguousarray(inst.eq_flat, dtype=np.float64)]
        h = L.pcba_ref_create(self.l, np.ascontiguousarray(inst.lo, dtype=np.float64),
                              np.ascontiguousarray(inst.hi, dtype=np.float64),
                              np.ascontiguousarray(inst.cost_deg, dtype=np.int32),
                              np.ascontiguousarray(inst.cost_flat, dtype=np.float64),
                              int(inst.n_ineq), _ptr(self._keep[0]), _ptr(self._keep[1]),
                              int(inst.n_eq), _ptr(self._keep[2]), _ptr(self._keep[3]),
                              float(g("eps")), float(g("delta")), float(g("eps_eq")),
                              int(g("max_boxes")), int(g("max_iters")))
        if not h:
            raise ValueError("pcba_ref_create rejected the problem")
        self.h = h
        self.words = int(L.pcba_ref_patch_words(h))
        if (rule != 0 or lam != 0.5) and L.pcba_ref_set_split(h, int(rule), float(lam)) != 0:
            raise ValueError("pcba_ref_set_split rejected the rule or parameter")
        if fused and L.pcba_ref_set_fused(h, 1) != 0:
            raise ValueError("pcba_ref_set_fused failed")

    def close(self):
        if getattr(self, "h", None):
            self.L.pcba_ref_destroy(self.h)
            self.h = None

    __del__ = close

    def step(self) -> int:
        return self.L.pcba_ref_step(self.h)

    def solve(self) -> int:
        return self.L.pcba_ref_solve(self.h)

    def result(self) -> dict:
        r = RefResult()
        self.L.pcba_ref_result_get(self.h, C.byref(r))
        l = self.l
        return dict(outcome=r.outcome, has_x=bool(r.has_x), p_up=r.p_up, p_lo=r.p_lo,
                    x_lo=np.array(r.x_lo[:l]), x_hi=np.array(r.x_hi[:l]),
                    x_depth=np.array(r.x_depth[:l]), x_index=np.array(r.x_index[:l], dtype=np.uint32),
                    rounds=r.rounds, steps=r.steps, list_len=r.list_len, peak_len=r.peak_len,
                    depth=np.array(r.depth[:l]), next_dir=r.next_dir)

    def kind_degree(self, kind: int) -> np.ndarray:
        d = np.zeros(self.l, dtype=np.int32)
        self.L.pcba_ref_kind_degree(self.h, kind, d)
        return d

    def list(self):
        n = self.result()["list_len"]
        ids = np.empty((n, self.l), dtype=np.uint32)
        pat = np.empty((n, self.words), dtype=np.float64)
        self.L.pcba_ref_list(self.h, ids.ctypes.data, pat.ctypes.data)
        return ids, pat

    def derive(self, depth, index) -> np.ndarray:
        out = np.empty(self.words, dtype=np.float64)
        rc = self.L.pcba_ref_derive(self.h, np.ascontiguousarray(depth, dtype=np.int32),
                                   np.ascontiguousarray(index, dtype=np.uint32), out)
        if rc != 0:
            raise ValueError("pcba_ref_derive rejected the box id")
        return out
