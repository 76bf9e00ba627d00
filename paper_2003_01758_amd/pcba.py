"""Python binding of the PCBA HIP library (include/pcba.h).

Argument marshalling only: every step of the solver runs in libpcba.so.  The
library must have been built (paper_2003_01758_amd/build.py); importing this
module without it raises, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcba.so")

MAX_DIM = 8
FP64_PLAIN, FP32 = 0, 1
SPLIT_VALU, SPLIT_MFMA = 0, 1
RUNNING, OPTIMAL, INFEASIBLE, MEMORY_LIMIT, MAX_ITER, TIMEOUT = -1, 0, 1, 2, 3, 4
OUTCOME_NAMES = {RUNNING: "running", OPTIMAL: "optimal", INFEASIBLE: "infeasible",
                 MEMORY_LIMIT: "memory_limit", MAX_ITER: "max_iter", TIMEOUT: "timeout"}
E_ARG, E_NOMEM, E_DEVICE, E_STATE = -1, -2, -3, -4
MAX_TRACE = 512
STATIC_SCRATCH_BYTES = 64 << 20   # PCBA_STATIC_SCRATCH_BYTES
KERNELS = ("sub_fp64", "sub_fp32", "rederive_fp32", "cut", "plan")


class Options(C.Structure):
    _fields_ = [("eps", C.c_double), ("delta", C.c_double), ("eps_eq", C.c_double),
                ("max_boxes", C.c_int64), ("max_iters", C.c_int32), ("precision", C.c_int32),
                ("rederive_every", C.c_int32), ("stale_filter", C.c_int32),
                ("retire_satisfied", C.c_int32), ("fused_round", C.c_int32),
                ("time_limit_s", C.c_double), ("tile_coefs", C.c_int32), ("wg_per_cu", C.c_int32),
                ("direction_rule", C.c_int32), ("split_engine", C.c_int32),
                ("subdiv_lambda", C.c_double), ("persistent_steps", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("outcome", C.c_int32), ("has_x", C.c_int32),
                ("p_up", C.c_double), ("p_lo", C.c_double),
                ("x_lo", C.c_double * MAX_DIM), ("x_hi", C.c_double * MAX_DIM),
                ("x_depth", C.c_int32 * MAX_DIM), ("x_index", C.c_uint32 * MAX_DIM),
                ("rounds", C.c_int32), ("steps", C.c_int32),
                ("list_len", C.c_int64), ("peak_len", C.c_int64),
                ("depth", C.c_int32 * MAX_DIM), ("next_dir", C.c_int32),
                ("certified", C.c_int32),
                ("p_cert", C.c_double), ("cert_err", C.c_double), ("err_max", C.c_double),
                ("seconds", C.c_double), ("capacity", C.c_int64)]


class PcbaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pcba error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2003_01758_amd/build.py "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.pcba_set_cut_split.argtypes = [C.c_int64, C.c_int32]
        L.pcba_set_cut_split.restype = C.c_int32
        L.pcba_default_options.argtypes = [C.POINTER(Options)]
        L.pcba_default_options.restype = None
        L.pcba_create_problem.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, i32, vp, vp,
                                          C.POINTER(Options), C.POINTER(vp)]
        L.pcba_create_problem.restype = C.c_int
        for name in ("pcba_solve",):
            getattr(L, name).argtypes = [vp, vp]
            getattr(L, name).restype = C.c_int
        L.pcba_step.argtypes = [vp, i32, vp]
        L.pcba_step.restype = C.c_int
        L.pcba_solve_batch.argtypes = [C.POINTER(vp), i32, vp]
        L.pcba_solve_batch.restype = C.c_int
        L.pcba_result.argtypes = [vp, C.POINTER(Result)]
        L.pcba_result.restype = C.c_int
        L.pcba_result_batch.argtypes = [C.POINTER(vp), i32, vp]
        L.pcba_result_batch.restype = C.c_int
        L.pcba_list_size.argtypes = [vp, C.POINTER(i64)]
        L.pcba_list_size.restype = C.c_int
        L.pcba_read_list.argtypes = [vp, vp, vp, i64]
        L.pcba_read_list.restype = C.c_int
        L.pcba_read_errors.argtypes = [vp, vp, i64]
        L.pcba_read_errors.restype = C.c_int
        L.pcba_read_list_noalloc.argtypes = [vp, vp, vp, i64, vp]
        L.pcba_read_list_noalloc.restype = C.c_int
        L.pcba_rtd_constraints.argtypes = [vp, vp, vp, i32, vp, dp, vp]
        L.pcba_rtd_constraints.restype = C.c_int
        L.pcba_read_root.argtypes = [vp, vp]
        L.pcba_read_root.restype = C.c_int
        L.pcba_patch_words.argtypes = [vp]
        L.pcba_patch_words.restype = i64
        L.pcba_item_bytes.argtypes = [vp]
        L.pcba_item_bytes.restype = i64
        L.pcba_footprint_bytes.argtypes = [vp, i64]
        L.pcba_footprint_bytes.restype = i64
        L.pcba_destroy_problem.argtypes = [vp]
        L.pcba_destroy_problem.restype = None
        L.pcba_engine_create.argtypes = [i64, i64, vp, C.POINTER(vp)]
        L.pcba_engine_create.restype = C.c_int
        L.pcba_engine_submit.argtypes = [vp, vp, C.POINTER(i32)]
        L.pcba_engine_submit.restype = C.c_int
        L.pcba_engine_run.argtypes = [vp, i32, C.POINTER(i32)]
        L.pcba_engine_run.restype = C.c_int
        L.pcba_engine_poll.argtypes = [vp, C.POINTER(vp), i32, C.POINTER(i32)]
        L.pcba_engine_poll.restype = C.c_int
        L.pcba_engine_used_bytes.argtypes = [vp]
        L.pcba_engine_used_bytes.restype = i64
        L.pcba_engine_destroy.argtypes = [vp]
        L.pcba_engine_destroy.restype = None
        L.pcba_reset_batch.argtypes = [C.POINTER(vp), i32, vp]
        L.pcba_reset_batch.restype = C.c_int
        L.pcba_reset.argtypes = [vp, vp]
        L.pcba_reset.restype = C.c_int
        L.pcba_read_trace.argtypes = [vp, vp, vp, vp, vp, i32]
        L.pcba_read_trace.restype = C.c_int
        L.pcba_read_trace_patches.argtypes = [vp, vp, vp, i32]
        L.pcba_read_trace_patches.restype = C.c_int
        L.pcba_release_cached_memory.argtypes = []
        L.pcba_release_cached_memory.restype = None
        L.pcba_profile_enable.argtypes = [i32]
        L.pcba_profile_enable.restype = None
        L.pcba_profile_reset.argtypes = []
        L.pcba_profile_reset.restype = None
        L.pcba_profile_read.argtypes = [vp, vp]
        L.pcba_profile_read.restype = None
        L.pcba_last_error.argtypes = []
        L.pcba_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise PcbaError(rc, lib().pcba_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):   # torch.cuda.Stream
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def default_options(**kw) -> Options:
    o = Options()
    lib().pcba_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FP64_PLAIN, "fp32": FP32}[v]
        if k == "split_engine" and isinstance(v, str):
            v = {"valu": SPLIT_VALU, "mfma": SPLIT_MFMA}[v]
        setattr(o, k, v)
    return o


def set_cut_split(children: int = 32768, part: int = 4096) -> None:
    """pcba_set_cut_split: children per step above which a problem's cut runs
    across workgroups of `part` children (children 0: never)."""
    _check(lib().pcba_set_cut_split(int(children), int(part)))


def rtd_constraints(w, pts, eps_q: float) -> np.ndarray:
    """pcba_rtd_constraints: w of shape (xdeg0+1, xdeg1+1, qdeg0+1, qdeg1+1),
    pts (n, 2); returns (n, qdeg0+1, qdeg1+1) coefficients of w(x_i, q) + eps_q."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    xdeg = np.array([w.shape[0] - 1, w.shape[1] - 1], dtype=np.int32)
    qdeg = np.array([w.shape[2] - 1, w.shape[3] - 1], dtype=np.int32)
    out = np.empty((len(pts), w.shape[2], w.shape[3]))
    _check(lib().pcba_rtd_constraints(xdeg.ctypes.data, qdeg.ctypes.data, w.ctypes.data, len(pts),
                                      pts.ctypes.data, float(eps_q), out.ctypes.data))
    return out


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


class Problem:
    """Problem (P) on the device.  `inst` is an instances.Instance-like object;
    keyword options override its tolerances (eps, delta, eps_eq, max_boxes,
    max_iters) and set precision ('fp64'|'fp32'), rederive_every, stale_filter,
    retire_satisfied, fused_round, time_limit_s, tile_coefs, wg_per_cu,
    direction_rule, split_engine ('valu'|'mfma'), subdiv_lambda, persistent_steps."""

    def __init__(self, inst, **kw):
        L = lib()
        opts = dict(eps=inst.eps, delta=inst.delta, eps_eq=inst.eps_eq,
                    max_boxes=int(inst.max_boxes), max_iters=int(inst.max_iters))
        opts.update(kw)
        self.options = default_options(**opts)
        self.l = int(inst.l)
        keep = [_arr(inst.lo, np.float64), _arr(inst.hi, np.float64),
                _arr(inst.cost_deg, np.int32), _arr(inst.cost_flat, np.float64),
                _arr(inst.ineq_deg, np.int32).ravel(), _arr(inst.ineq_flat, np.float64),
                _arr(inst.eq_deg, np.int32).ravel(), _arr(inst.eq_flat, np.float64)]
        ptr = [None if a.size == 0 else a.ctypes.data for a in keep]
        h = C.c_void_p()
        _check(L.pcba_create_problem(self.l, ptr[0], ptr[1], ptr[2], ptr[3], int(inst.n_ineq),
                                     ptr[4], ptr[5], int(inst.n_eq), ptr[6], ptr[7],
                                     C.byref(self.options), C.byref(h)))
        self.h = h
        self.n_polys = 1 + int(inst.n_ineq) + int(inst.n_eq)
        self.words = int(L.pcba_patch_words(h))

    def close(self):
        if getattr(self, "h", None):
            lib().pcba_destroy_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, stream=None):
        _check(lib().pcba_solve(self.h, _stream_ptr(stream)))
        return self.result()

    def step(self, n: int = 1, stream=None):
        _check(lib().pcba_step(self.h, int(n), _stream_ptr(stream)))
        return self.result()

    def result(self) -> dict:
        r = Result()
        _check(lib().pcba_result(self.h, C.byref(r)))
        l = self.l
        return dict(outcome=r.outcome, has_x=bool(r.has_x), p_up=r.p_up, p_lo=r.p_lo,
                    x_lo=np.array(r.x_lo[:l]), x_hi=np.array(r.x_hi[:l]),
                    x_depth=np.array(r.x_depth[:l]), x_index=np.array(r.x_index[:l], dtype=np.uint32),
                    rounds=r.rounds, steps=r.steps, list_len=r.list_len, peak_len=r.peak_len,
                    depth=np.array(r.depth[:l]), next_dir=r.next_dir, certified=bool(r.certified),
                    p_cert=r.p_cert, cert_err=r.cert_err, err_max=r.err_max, seconds=r.seconds,
                    capacity=r.capacity)

    def list(self):
        n = C.c_int64()
        _check(lib().pcba_list_size(self.h, C.byref(n)))
        n = n.value
        ids = np.empty((n, self.l), dtype=np.uint32)
        pat = np.empty((n, self.words), dtype=np.float64)
        if n:
            _check(lib().pcba_read_list(self.h, ids.ctypes.data, pat.ctypes.data, n))
        return ids, pat

    def list_noalloc(self, stream=None):
        """list() through pcba_read_list_noalloc: no device allocation, staging
        in the library's static per-device array."""
        n = C.c_int64()
        _check(lib().pcba_list_size(self.h, C.byref(n)))
        n = n.value
        ids = np.empty((n, self.l), dtype=np.uint32)
        pat = np.empty((n, self.words), dtype=np.float64)
        _check(lib().pcba_read_list_noalloc(self.h, ids.ctypes.data, pat.ctypes.data, n, _stream_ptr(stream)))
        return ids, pat

    def errors(self) -> np.ndarray:
        n = C.c_int64()
        _check(lib().pcba_list_size(self.h, C.byref(n)))
        n = n.value
        err = np.empty((n, self.n_polys), dtype=np.float64)
        if n:
            _check(lib().pcba_read_errors(self.h, err.ctypes.data, n))
        return err

    def reset(self, stream=None):
        _check(lib().pcba_reset(self.h, _stream_ptr(stream)))

    def trace(self):
        """Per-step records of the last solve: k_in, k_kept, p_up, p_lo."""
        cap = MAX_TRACE
        k_in = np.zeros(cap, dtype=np.int32)
        k_kept = np.zeros(cap, dtype=np.int32)
        p_up = np.zeros(cap)
        p_lo = np.zeros(cap)
        n = lib().pcba_read_trace(self.h, k_in.ctypes.data, k_kept.ctypes.data, p_up.ctypes.data,
                                  p_lo.ctypes.data, cap)
        if n < 0:
            _check(n)
        return dict(k_in=k_in[:n], k_kept=k_kept[:n], p_up=p_up[:n], p_lo=p_lo[:n])

    def trace_patches(self):
        """Per-step inequality patches carried by the parents (a_in) and by the
        kept children (a_kept) in the last solve."""
        cap = MAX_TRACE
        a_in = np.zeros(cap, dtype=np.int64)
        a_kept = np.zeros(cap, dtype=np.int64)
        n = lib().pcba_read_trace_patches(self.h, a_in.ctypes.data, a_kept.ctypes.data, cap)
        if n < 0:
            _check(n)
        return dict(a_in=a_in[:n], a_kept=a_kept[:n])

    def root(self) -> np.ndarray:
        out = np.empty(self.words, dtype=np.float64)
        _check(lib().pcba_read_root(self.h, out.ctypes.data))
        return out

    def item_bytes(self) -> int:
        return int(lib().pcba_item_bytes(self.h))

    def footprint(self, boxes: int) -> int:
        return int(lib().pcba_footprint_bytes(self.h, int(boxes)))


def release_cached_memory():
    """Returns the fully free chunks of the library's device arena."""
    lib().pcba_release_cached_memory()


def profile_enable(on: bool = True):
    lib().pcba_profile_enable(1 if on else 0)


def profile_reset():
    lib().pcba_profile_reset()


def profile_read() -> dict:
    """Per kernel: (total milliseconds, launches) from HIP events around each launch."""
    ms = np.zeros(len(KERNELS))
    n = np.zeros(len(KERNELS), dtype=np.int64)
    lib().pcba_profile_read(ms.ctypes.data, n.ctypes.data)
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}


RESULT_DTYPE = np.dtype(Result)


class Batch:
    """A fixed sequence of problems whose handle array is built once, for
    repeated batch calls (reset_batch, solve_batch and results accept it in
    place of a list)."""

    def __init__(self, problems):
        self.problems = list(problems)
        self.handles = (C.c_void_p * len(self.problems))(*[p.h for p in self.problems])

    def __len__(self):
        return len(self.problems)

    def __iter__(self):
        return iter(self.problems)


def _handles(problems):
    if isinstance(problems, Batch):
        return problems.handles
    return (C.c_void_p * len(problems))(*[p.h for p in problems])


def reset_batch(problems, stream=None):
    _check(lib().pcba_reset_batch(_handles(problems), len(problems), _stream_ptr(stream)))


def results(problems) -> np.ndarray:
    """The results of the problems' last solves in one call, as a structured
    array with the fields of pcba_result_t (record b belongs to problem b)."""
    out = np.zeros(len(problems), dtype=RESULT_DTYPE)
    _check(lib().pcba_result_batch(_handles(problems), len(problems), out.ctypes.data))
    return out


def solve_batch(problems, stream=None, as_array=False):
    """Solves the problems together.  Returns one dict per problem (as
    Problem.result), or with as_array the structured array of `results`."""
    _check(lib().pcba_solve_batch(_handles(problems), len(problems), _stream_ptr(stream)))
    if as_array:
        return results(problems)
    return [p.result() for p in problems]


class Engine:
    """Continuous batching: admit problems while their footprints fit the
    budget, advance all admitted problems together, harvest finished ones."""

    def __init__(self, budget_bytes: int = 0, reserve_boxes: int = 0, stream=None):
        h = C.c_void_p()
        _check(lib().pcba_engine_create(int(budget_bytes), int(reserve_boxes), _stream_ptr(stream),
                                        C.byref(h)))
        self.h = h
        self._by_handle = {}

    def close(self):
        if getattr(self, "h", None):
            lib().pcba_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, prob: Problem) -> bool:
        adm = C.c_int32()
        _check(lib().pcba_engine_submit(self.h, prob.h, C.byref(adm)))
        if adm.value:
            self._by_handle[prob.h.value] = prob
        return bool(adm.value)

    def run(self, n_steps: int) -> int:
        act = C.c_int32()
        _check(lib().pcba_engine_run(self.h, int(n_steps), C.byref(act)))
        return act.value

    def poll(self, cap: int = 256):
        arr = (C.c_void_p * cap)()
        n = C.c_int32()
        _check(lib().pcba_engine_poll(self.h, arr, cap, C.byref(n)))
        return [self._by_handle.pop(arr[i]) for i in range(n.value)]

    def used_bytes(self) -> int:
        return int(lib().pcba_engine_used_bytes(self.h))
