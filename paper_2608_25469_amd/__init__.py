"""Python binding of the gfx950 TRSM library (``libhsma.so``).

Argument marshalling only: every step of every solve runs in the library's
HIP kernels.  Tensors are torch tensors on the GPU; PyTorch provides device
memory and streams.  The library must have been built
(``python -m paper_2608_25469_amd.build``); importing works without it, but
every call then raises ``HsmaError`` -- there is no CPU fallback.

Layout: matrices are column-major, as in BLAS.  A column-major m x n matrix
with leading dimension ld is the transpose of a row-major (n, ld) tensor,
sliced to m rows: ``storage[:, :m].t()`` (strides (1, ld)).  Use
:func:`colmajor` / :func:`to_colmajor` to make them.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsma.so")

R64F, C64F, R32F, C32F = 0, 1, 2, 3
NON_UNIT, UNIT = 0, 1

STATUS = {
    0: "SUCCESS", 1: "INVALID_VALUE", 2: "INVALID_SIZE", 3: "INVALID_POINTER",
    4: "ALLOC_FAILED", 5: "HIP_ERROR", 6: "NOT_SUPPORTED", 7: "TOO_LARGE",
    8: "QUEUE_CLOSED", 9: "PENDING", 10: "TIMEOUT", 11: "NOT_FOUND",
    12: "WORKSPACE_TOO_SMALL",
}


class HsmaError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}" if what else STATUS.get(status, str(status)))


class TrsmOptions(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("path", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("want_backward_error", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2),
                ("refine_tol", ctypes.c_double)]


class TrsmReport(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5),
                ("backward_error", ctypes.c_double)]


PREC_FP64, PREC_MIXED = 0, 1


class Problem(ctypes.Structure):
    _fields_ = [("diag", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("alpha_re", ctypes.c_double), ("alpha_im", ctypes.c_double),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64)]


class PhaseStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("flops", ctypes.c_double)]


class QueueConfig(ctypes.Structure):
    _fields_ = [("backend", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("poll_us", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("sim_flops_per_ns", ctypes.c_double),
                ("sim_fixed_ns", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("prob", Problem), ("input", ctypes.c_int32),
                ("release_on_completion", ctypes.c_int32), ("key", ctypes.c_uint64),
                ("t_arrival_ns", ctypes.c_double)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("path", ctypes.c_int32),
                ("t_arrival_ns", ctypes.c_double), ("t_admit_ns", ctypes.c_double),
                ("t_done_ns", ctypes.c_double), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64)]


class LatencySummary(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("p50_ns", ctypes.c_double),
                ("p99_ns", ctypes.c_double), ("max_ns", ctypes.c_double),
                ("mean_ns", ctypes.c_double)]


LATENCY_CLASSES = 3
LATENCY_CLASS_NAMES = ["m<=64", "64<m<=512", "m>512"]


class QueueStatistics(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("pending", ctypes.c_int64), ("inflight", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_uint64), ("bytes_peak", ctypes.c_uint64),
                ("p50_ns", ctypes.c_double), ("p99_ns", ctypes.c_double),
                ("max_ns", ctypes.c_double), ("mean_ns", ctypes.c_double),
                ("solves_per_s", ctypes.c_double), ("rounds", ctypes.c_int64),
                ("launch_ms", ctypes.c_double),
                ("t_first_submit_ns", ctypes.c_double), ("t_last_done_ns", ctypes.c_double),
                ("all", LatencySummary), ("by_class", LatencySummary * LATENCY_CLASSES)]


BACKEND_HIP, BACKEND_SIMULATED = 0, 1
INPUT_DEVICE, INPUT_SYNTHETIC = 0, 1


PHASE_DIAG_INV, PHASE_UPDATE, PHASE_LEAF, PHASE_SMALL, PHASE_OTHER, PHASE_FACTOR, PHASE_TINY = range(7)
PHASE_COUNT = 7
PHASE_NAMES = ["diag_inv", "update", "leaf_solve", "small", "other", "factor", "tiny"]

_lib = None


def lib():
    """The loaded library (raises HsmaError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HsmaError(6, f"{LIB_PATH} not built; run python -m paper_2608_25469_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32
        L.hsma_trsm.argtypes = [i32, i64, i64, vp, vp, i64, vp, i64, i32, vp]
        L.hsma_trsm.restype = i32
        L.hsma_trsm_ex.argtypes = [i32, i64, i64, vp, vp, i64, vp, i64, i32,
                                   ctypes.POINTER(TrsmOptions), ctypes.POINTER(TrsmReport), vp]
        L.hsma_trsm_ex.restype = i32
        L.hsma_trsm_general.argtypes = [i32, i32, i32, i32, i64, i64, vp, vp, i64, vp, i64, i32, vp]
        L.hsma_trsm_general.restype = i32
        L.hsma_potrf.argtypes = [i64, vp, i64, i32, vp]
        L.hsma_potrf.restype = i32
        L.hsma_potrs.argtypes = [i64, i64, vp, i64, vp, i64, i32, vp]
        L.hsma_potrs.restype = i32
        L.hsma_trsm_noalloc.argtypes = [i32, i64, i64, vp, vp, i64, vp, i64, i32, vp]
        L.hsma_trsm_noalloc.restype = i32
        L.hsma_noalloc_scratch_bytes.argtypes = []
        L.hsma_noalloc_scratch_bytes.restype = ctypes.c_uint64
        L.hsma_status_string.argtypes = [i32]
        L.hsma_status_string.restype = ctypes.c_char_p
        L.hsma_last_hip_error.argtypes = []
        L.hsma_last_hip_error.restype = ctypes.c_int
        L.hsma_version.argtypes = []
        L.hsma_version.restype = ctypes.c_char_p
        L.hsma_lookup_block_size.argtypes = [i32, i64, i64]
        L.hsma_lookup_block_size.restype = i32
        L.hsma_trsm_batched.argtypes = [ctypes.POINTER(Problem), i64, ctypes.POINTER(i64), vp]
        L.hsma_trsm_batched.restype = i32
        L.hsma_batch_plan_create.argtypes = [ctypes.POINTER(Problem), i64, ctypes.POINTER(i64),
                                             ctypes.POINTER(vp)]
        L.hsma_batch_plan_create.restype = i32
        L.hsma_batch_plan_execute.argtypes = [vp, vp]
        L.hsma_batch_plan_execute.restype = i32
        L.hsma_batch_plan_destroy.argtypes = [vp]
        L.hsma_batch_plan_destroy.restype = i32
        L.hsma_workspace_release.argtypes = []
        L.hsma_workspace_release.restype = i32
        L.hsma_graph_cache_clear.argtypes = []
        L.hsma_graph_cache_clear.restype = i32
        L.hsma_mfma_peak.argtypes = [i32, i64, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
        L.hsma_mfma_peak.restype = i32
        L.hsma_graph_stats.argtypes = [ctypes.POINTER(i64)] * 3
        L.hsma_graph_stats.restype = i32
        L.hsma_profile_begin.argtypes = []
        L.hsma_profile_begin.restype = i32
        L.hsma_profile_end.argtypes = [ctypes.POINTER(PhaseStat), ctypes.c_int]
        L.hsma_profile_end.restype = i32
        u64 = ctypes.c_uint64
        L.hsma_generate_inputs.argtypes = [i32, i64, i64, u64, vp, vp, vp]
        L.hsma_generate_inputs.restype = i32
        L.hsma_request_footprint.argtypes = [ctypes.POINTER(Request), ctypes.POINTER(u64)]
        L.hsma_request_footprint.restype = i32
        L.hsma_clock_ns.argtypes = []
        L.hsma_clock_ns.restype = ctypes.c_double
        L.hsma_queue_create.argtypes = [ctypes.POINTER(QueueConfig), ctypes.POINTER(vp)]
        L.hsma_queue_create.restype = i32
        L.hsma_queue_submit.argtypes = [vp, ctypes.POINTER(Request), i64, ctypes.POINTER(u64)]
        L.hsma_queue_submit.restype = i32
        L.hsma_queue_poll.argtypes = [vp, u64, ctypes.POINTER(RequestInfo)]
        L.hsma_queue_poll.restype = i32
        L.hsma_queue_wait.argtypes = [vp, u64, i64, ctypes.POINTER(RequestInfo)]
        L.hsma_queue_wait.restype = i32
        L.hsma_queue_release.argtypes = [vp, u64]
        L.hsma_queue_release.restype = i32
        L.hsma_queue_stats.argtypes = [vp, ctypes.POINTER(QueueStatistics)]
        L.hsma_queue_stats.restype = i32
        L.hsma_queue_stats_reset.argtypes = [vp, ctypes.c_double]
        L.hsma_queue_stats_reset.restype = i32
        L.hsma_queue_destroy.argtypes = [vp]
        L.hsma_queue_destroy.restype = i32
        _lib = L
    return _lib


def _check(st: int, what: str) -> None:
    if st != 0:
        extra = ""
        if st == 5:
            extra = f" (hipError {lib().hsma_last_hip_error()})"
        raise HsmaError(st, what + extra)


# ---------------------------------------------------------------------------
# Layout helpers
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def colmajor(m: int, n: int, dtype, ld: Optional[int] = None, device="cuda", fill=None):
    """A column-major m x n tensor with leading dimension ``ld`` (>= m)."""
    torch = _torch()
    ld = max(1, m) if ld is None else ld
    if ld < max(1, m):
        raise ValueError("ld < m")
    store = torch.empty((max(n, 1), ld), dtype=dtype, device=device)
    if fill is not None:
        store.fill_(fill)
    return store[:n, :m].t()


def to_colmajor(a: np.ndarray, device="cuda", ld: Optional[int] = None):
    """Copy a 2-D numpy array (any layout) to a column-major device tensor."""
    torch = _torch()
    m, n = a.shape
    dt = {np.dtype(np.float64): torch.float64, np.dtype(np.complex128): torch.complex128,
          np.dtype(np.float32): torch.float32, np.dtype(np.complex64): torch.complex64}[a.dtype]
    out = colmajor(m, n, dt, ld=ld, device=device)
    if m and n:
        out.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return out


def from_colmajor(t) -> np.ndarray:
    """Device column-major tensor -> numpy array in Fortran order."""
    return np.asfortranarray(t.detach().cpu().numpy())


def leading_dim(t) -> int:
    m, n = t.shape
    s0, s1 = t.stride()
    if s0 != 1 and m > 1:
        raise ValueError("matrix must be column-major (stride(0) == 1)")
    if n <= 1:
        return max(1, m) if s1 < m else s1
    return s1


_DTYPE_CODES = None


def _dtype_code(t) -> int:
    global _DTYPE_CODES
    if _DTYPE_CODES is None:
        torch = _torch()
        _DTYPE_CODES = {torch.float64: R64F, torch.complex128: C64F, torch.float32: R32F,
                        torch.complex64: C32F}
    code = _DTYPE_CODES.get(t.dtype)
    if code is None:
        raise TypeError("tensors must be float64, complex128, float32 or complex64")
    return code


# Host scalars of nonzero real Python numbers, shared between calls: the
# library copies alpha before it returns, so a buffer is only ever read.
# (Zeros are not cached: -0.0 and 0.0 are one dictionary key.)
_ALPHA_BUFS: dict = {}


def _alpha_buf(alpha, code):
    """Host scalar of the data type: double[2] for FP64, float[2] for FP32."""
    plain = type(alpha) in (float, int) and alpha != 0
    if plain:
        buf = _ALPHA_BUFS.get((alpha, type(alpha), code))
        if buf is not None:
            return buf
    a = complex(alpha)
    if code in (R64F, R32F) and a.imag != 0:
        raise ValueError("complex alpha for a real problem")
    if code in (R32F, C32F):
        buf = (ctypes.c_float * 2)(a.real, a.imag)
    else:
        buf = (ctypes.c_double * 2)(a.real, a.imag)
    if plain:
        if len(_ALPHA_BUFS) >= 256:
            _ALPHA_BUFS.clear()
        _ALPHA_BUFS[(alpha, type(alpha), code)] = buf
    return buf


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        # torch's current stream on the current device, without building a
        # Stream object per call
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return raw(torch.cuda.current_device())
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# Solves
# ---------------------------------------------------------------------------

def trsm(L, B, alpha=1.0, unit: bool = False, block_size: int = 0, path: int = 0,
         stream=None, report: bool = False, mixed: bool = False, refine_steps: int = 0,
         backward_error: bool = False, refine_tol: float = 0.0, graph: bool = False):
    """B <- alpha * inv(tril(L)) * B in place (left, lower, no transpose).

    L: m x m, B: m x n, both column-major device tensors of the same dtype
    (float64 or complex128).  ``block_size`` forces the blocked path's I_B,
    ``path`` forces 1 = small kernel or 2 = blocked.  ``mixed`` runs the
    trailing updates on the FP32 matrix cores; ``refine_steps`` (0..4, or -1
    for "until the backward error is <= refine_tol") adds FP64-residual
    refinement; ``backward_error`` reports the result's normwise backward
    error; ``graph`` replays the blocked schedule as a cached HIP graph.  Asynchronous on ``stream`` (default: torch's current stream)
    unless a backward error is needed.  Returns B (and the library's report
    if ``report``).
    """
    code = _dtype_code(B)
    if L.dtype != B.dtype:
        raise TypeError("L and B must have the same dtype")
    m, n = B.shape
    if L.shape[0] != m or L.shape[1] < m:
        raise ValueError("L must be m x m")
    if m and n and (not L.is_cuda or not B.is_cuda):
        raise ValueError("tensors must be on the GPU")
    if not (block_size or path or report or mixed or refine_steps or backward_error
            or refine_tol or graph):
        # A plain solve: the options-free entry point, nothing built per call.
        st = lib().hsma_trsm(UNIT if unit else NON_UNIT, m, n, _alpha_buf(alpha, code),
                             L.data_ptr(), leading_dim(L), B.data_ptr(), leading_dim(B), code,
                             _stream_handle(stream))
        _check(st, "hsma_trsm")
        return B
    opts = TrsmOptions(block_size, path, PREC_MIXED if mixed else PREC_FP64, refine_steps,
                       1 if backward_error else 0, 1 if graph else 0, (ctypes.c_int32 * 2)(),
                       refine_tol)
    rep = TrsmReport()
    st = lib().hsma_trsm_ex(UNIT if unit else NON_UNIT, m, n, _alpha_buf(alpha, code),
                            ctypes.c_void_p(L.data_ptr()), leading_dim(L),
                            ctypes.c_void_p(B.data_ptr()), leading_dim(B), code,
                            ctypes.byref(opts), ctypes.byref(rep),
                            ctypes.c_void_p(_stream_handle(stream)))
    _check(st, "hsma_trsm_ex")
    if report:
        return B, {"path": rep.path, "block_size": rep.block_size,
                   "refine_steps": rep.refine_steps, "backward_error": rep.backward_error}
    return B


SIDE = {"L": 0, "R": 1}
UPLO = {"L": 0, "U": 1}
OP = {"N": 0, "T": 1, "C": 2}


def trsm_general(A, B, alpha=1.0, side: str = "L", uplo: str = "L", trans: str = "N",
                 unit: bool = False, stream=None):
    """B <- X with op(A) X = alpha B (side "L") or X op(A) = alpha B (side
    "R"), in place.  ``uplo`` names the stored triangle of A ("L" or "U"),
    ``trans`` is "N", "T" or "C" (conjugate transpose).  A is k x k with k = m
    (left) or n (right); both column-major device tensors of one dtype."""
    code = _dtype_code(B)
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    m, n = B.shape
    k = m if side.upper() == "L" else n
    if A.shape[0] != k or A.shape[1] < k:
        raise ValueError(f"A must be {k} x {k}")
    if m and n and (not A.is_cuda or not B.is_cuda):
        raise ValueError("tensors must be on the GPU")
    st = lib().hsma_trsm_general(SIDE[side.upper()], UPLO[uplo.upper()], OP[trans.upper()],
                                 UNIT if unit else NON_UNIT, m, n, _alpha_buf(alpha, code),
                                 ctypes.c_void_p(A.data_ptr()), leading_dim(A),
                                 ctypes.c_void_p(B.data_ptr()), leading_dim(B), code,
                                 ctypes.c_void_p(_stream_handle(stream)))
    _check(st, "hsma_trsm_general")
    return B


def potrf(A, stream=None):
    """A = L L^H in place on the lower triangle of the square column-major
    device tensor A (float64 or complex128)."""
    code = _dtype_code(A)
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    _check(lib().hsma_potrf(n, ctypes.c_void_p(A.data_ptr()), leading_dim(A), code,
                            ctypes.c_void_p(_stream_handle(stream))), "hsma_potrf")
    return A


def potrs(L, B, stream=None):
    """B <- X with L L^H X = B (L from potrf)."""
    code = _dtype_code(B)
    n, nrhs = B.shape
    if L.dtype != B.dtype or L.shape[0] != n:
        raise ValueError("L must be n x n of B's dtype")
    _check(lib().hsma_potrs(n, nrhs, ctypes.c_void_p(L.data_ptr()), leading_dim(L),
                            ctypes.c_void_p(B.data_ptr()), leading_dim(B), code,
                            ctypes.c_void_p(_stream_handle(stream))), "hsma_potrs")
    return B


def problem_struct(L, B, alpha=1.0, unit: bool = False) -> Problem:
    """Descriptor of one solve for the batched entry points (device tensors)."""
    code = _dtype_code(B)
    m, n = B.shape
    a = complex(alpha)
    if code == R64F and a.imag != 0:
        raise ValueError("complex alpha for a real problem")
    return Problem(UNIT if unit else NON_UNIT, code, m, n, a.real, a.imag,
                   ctypes.c_void_p(L.data_ptr()), leading_dim(L),
                   ctypes.c_void_p(B.data_ptr()), leading_dim(B))


def _problem_array(problems):
    arr = (Problem * max(1, len(problems)))()
    for i, p in enumerate(problems):
        arr[i] = p if isinstance(p, Problem) else problem_struct(*p)
    return arr


def trsm_batched(problems, stream=None) -> None:
    """Solve every problem in place.  ``problems``: Problem structs or tuples
    (L, B, alpha[, unit]) of device tensors.  Raises HsmaError (with
    ``.first_bad``) if a descriptor is invalid; nothing is enqueued then."""
    arr = _problem_array(problems)
    bad = ctypes.c_int64(-1)
    st = lib().hsma_trsm_batched(arr, len(problems), ctypes.byref(bad),
                                 ctypes.c_void_p(_stream_handle(stream)))
    if st != 0:
        err = HsmaError(st, f"hsma_trsm_batched (first bad problem {bad.value})")
        err.first_bad = bad.value
        raise err


class BatchPlan:
    """A batch prepared once (descriptors resident on the device) and run
    many times: ``plan.execute(stream)``."""

    def __init__(self, problems):
        arr = _problem_array(problems)
        bad = ctypes.c_int64(-1)
        h = ctypes.c_void_p()
        st = lib().hsma_batch_plan_create(arr, len(problems), ctypes.byref(bad), ctypes.byref(h))
        if st != 0:
            err = HsmaError(st, f"hsma_batch_plan_create (first bad problem {bad.value})")
            err.first_bad = bad.value
            raise err
        self._h = h

    def execute(self, stream=None) -> None:
        _check(lib().hsma_batch_plan_execute(self._h, ctypes.c_void_p(_stream_handle(stream))),
               "hsma_batch_plan_execute")

    def close(self) -> None:
        if self._h:
            _check(lib().hsma_batch_plan_destroy(self._h), "hsma_batch_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_batch(Ls, Bs, device="cuda", align_bytes: int = 256):
    """Copy lists of numpy L and B matrices into two device pools, each
    matrix column-major at its own 256-byte aligned offset (as if separately
    allocated).  Returns (pool_L, pool_B, views_L, views_B)."""
    torch = _torch()
    cx = np.iscomplexobj(Bs[0])
    dt = torch.complex128 if cx else torch.float64
    es = 16 if cx else 8
    al = max(1, align_bytes // es)

    def layout(mats):
        offs, pos = [], 0
        for a in mats:
            offs.append(pos)
            pos += a.shape[0] * a.shape[1]
            pos = (pos + al - 1) // al * al
        return offs, pos

    def fill(mats):
        offs, total = layout(mats)
        host = np.zeros(max(total, 1), dtype=np.complex128 if cx else np.float64)
        for a, o in zip(mats, offs):
            host[o:o + a.size] = np.asfortranarray(a).ravel(order="F")
        pool = torch.from_numpy(host).to(device)
        views = [pool[o:o + a.shape[0] * a.shape[1]].view(a.shape[1], a.shape[0]).t()
                 for a, o in zip(mats, offs)]
        return pool, views

    pl, vl = fill(Ls)
    pb, vb = fill(Bs)
    return pl, pb, vl, vb


def profile_begin() -> None:
    _check(lib().hsma_profile_begin(), "hsma_profile_begin")


def profile_end() -> dict:
    """Per-phase kernel time since profile_begin (waits for the events)."""
    stats = (PhaseStat * PHASE_COUNT)()
    _check(lib().hsma_profile_end(stats, PHASE_COUNT), "hsma_profile_end")
    return {PHASE_NAMES[i]: {"launches": stats[i].launches, "ms": stats[i].ms,
                             "flops": stats[i].flops} for i in range(PHASE_COUNT)}


def graph_cache_clear() -> None:
    _check(lib().hsma_graph_cache_clear(), "hsma_graph_cache_clear")


def mfma_peak(fp32: bool = False, iters: int = 10000):
    """(sustained matrix-core TFLOP/s, shader clock GHz during the run) of
    this GPU for FP64 or FP32 MFMA."""
    t, g = ctypes.c_double(), ctypes.c_double()
    _check(lib().hsma_mfma_peak(1 if fp32 else 0, iters, ctypes.byref(t), ctypes.byref(g)),
           "hsma_mfma_peak")
    return t.value, g.value


def graph_stats() -> dict:
    """Graph-cache counters: instantiations, in-place updates, replays."""
    c, u, r = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().hsma_graph_stats(ctypes.byref(c), ctypes.byref(u), ctypes.byref(r)), "hsma_graph_stats")
    return {"captures": c.value, "updates": u.value, "replays": r.value}


def workspace_release() -> None:
    """Return the library's idle cached workspace blocks to the device."""
    _check(lib().hsma_workspace_release(), "hsma_workspace_release")


def lookup_block_size(complex_: bool, m: int, n: int) -> int:
    return lib().hsma_lookup_block_size(C64F if complex_ else R64F, m, n)


def version() -> str:
    return lib().hsma_version().decode()


# ---------------------------------------------------------------------------
# Synthetic inputs and the serving queue
# ---------------------------------------------------------------------------

def generate_inputs(m: int, n: int, key: int, complex_: bool = False, stream=None):
    """L (m x m) and B (m x n), column-major with ld = m, drawn on the GPU from
    Philox4x32-10 under ``key`` (the library's synthetic workload)."""
    torch = _torch()
    dt = torch.complex128 if complex_ else torch.float64
    L = colmajor(m, m, dt)
    B = colmajor(m, n, dt)
    st = lib().hsma_generate_inputs(C64F if complex_ else R64F, m, n, key & (2**64 - 1),
                                    ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                    ctypes.c_void_p(_stream_handle(stream)))
    _check(st, "hsma_generate_inputs")
    return L, B


def matrix_from_pointer(ptr: int, rows: int, cols: int, ld: int, complex_: bool = False) -> np.ndarray:
    """Host copy (numpy, column-major) of a device matrix known only by its
    address, such as a kept synthetic result of the queue."""
    hip = ctypes.CDLL("libamdhip64.so.7")   # the runtime the library and torch share
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    buf = np.empty((cols, ld), dtype=np.complex128 if complex_ else np.float64)
    if buf.size:
        st = hip.hipMemcpy(buf.ctypes.data, ptr, buf.nbytes, 2)   # device to host
        if st != 0:
            raise HsmaError(5, f"hipMemcpy failed ({st})")
    return np.asfortranarray(buf[:, :rows].T)


def clock_ns() -> float:
    """The queue's monotonic clock (ns)."""
    return lib().hsma_clock_ns()


def request(m: int, n: int, alpha=1.0, unit: bool = False, complex_: bool = False,
            key: Optional[int] = None, L=None, B=None, release_on_completion: bool = True,
            t_arrival_ns: float = 0.0, forget: bool = False) -> Request:
    """A queue request: synthetic (``key`` given; the server allocates and
    fills L and B) or on caller tensors ``L``, ``B``.  ``forget`` makes it
    fire-and-forget (release_on_completion = 2): its record is dropped when it
    finishes, so poll/wait then report NOT_FOUND; it still counts in the
    statistics."""
    code = C64F if complex_ else R64F
    a = complex(alpha)
    if code == R64F and a.imag != 0:
        raise ValueError("complex alpha for a real problem")
    if key is not None:
        prob = Problem(UNIT if unit else NON_UNIT, code, m, n, a.real, a.imag, None, max(1, m),
                       None, max(1, m))
        return Request(prob, INPUT_SYNTHETIC, 2 if forget else (1 if release_on_completion else 0),
                       key & (2**64 - 1), t_arrival_ns)
    prob = problem_struct(L, B, alpha, unit)
    return Request(prob, INPUT_DEVICE, 2 if forget else 0, 0, t_arrival_ns)


def request_footprint(req: Request) -> int:
    """Bytes of HBM budget the queue reserves for ``req``."""
    b = ctypes.c_uint64()
    _check(lib().hsma_request_footprint(ctypes.byref(req), ctypes.byref(b)), "hsma_request_footprint")
    return int(b.value)


class Queue:
    """Continuous-batching request queue (``hsma_queue_*``).

    ``Queue(simulated=True, ...)`` runs the same scheduler with modelled
    device time and no GPU work (for policy tests)."""

    def __init__(self, simulated: bool = False, n_streams: int = 0, max_inflight: int = 0,
                 poll_us: int = 0, hbm_budget_bytes: int = 0, sim_flops_per_ns: float = 0.0,
                 sim_fixed_ns: float = 0.0):
        cfg = QueueConfig(BACKEND_SIMULATED if simulated else BACKEND_HIP, n_streams,
                          max_inflight, poll_us, hbm_budget_bytes, sim_flops_per_ns, sim_fixed_ns)
        h = ctypes.c_void_p()
        _check(lib().hsma_queue_create(ctypes.byref(cfg), ctypes.byref(h)), "hsma_queue_create")
        self._h = h
        self._keep = {}   # caller tensors of device-input requests, kept alive

    def submit(self, reqs, tensors=None):
        """Submit Request structs (one or a list); returns the tickets.  Pass
        the tensors a device-input request uses in ``tensors`` to keep them
        alive until it is released."""
        single = isinstance(reqs, Request)
        reqs = [reqs] if single else list(reqs)
        arr = (Request * max(1, len(reqs)))(*reqs)
        tk = (ctypes.c_uint64 * max(1, len(reqs)))()
        _check(lib().hsma_queue_submit(self._h, arr, len(reqs), tk), "hsma_queue_submit")
        out = [int(tk[i]) for i in range(len(reqs))]
        if tensors is not None:
            for t, ts in zip(out, [tensors] if single else tensors):
                self._keep[t] = ts
        return out[0] if single else out

    @staticmethod
    def _info(info: RequestInfo) -> dict:
        return {"status": info.status, "path": info.path, "t_arrival_ns": info.t_arrival_ns,
                "t_admit_ns": info.t_admit_ns, "t_done_ns": info.t_done_ns,
                "A": info.A, "B": info.B, "lda": info.lda, "ldb": info.ldb}

    def poll(self, ticket: int):
        """(status code, info dict)."""
        info = RequestInfo()
        st = lib().hsma_queue_poll(self._h, ticket, ctypes.byref(info))
        return st, self._info(info)

    def wait(self, ticket: int, timeout_s: Optional[float] = None) -> dict:
        info = RequestInfo()
        t = -1 if timeout_s is None else int(timeout_s * 1e9)
        st = lib().hsma_queue_wait(self._h, ticket, t, ctypes.byref(info))
        _check(st, f"hsma_queue_wait({ticket})")
        return self._info(info)

    def release(self, ticket: int) -> None:
        _check(lib().hsma_queue_release(self._h, ticket), f"hsma_queue_release({ticket})")
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        s = QueueStatistics()
        _check(lib().hsma_queue_stats(self._h, ctypes.byref(s)), "hsma_queue_stats")

        def summ(x):
            return {f[0]: getattr(x, f[0]) for f in LatencySummary._fields_}
        out = {f[0]: getattr(s, f[0]) for f in QueueStatistics._fields_
               if f[0] not in ("all", "by_class")}
        out["all"] = summ(s.all)
        out["by_class"] = {LATENCY_CLASS_NAMES[c]: summ(s.by_class[c]) for c in range(LATENCY_CLASSES)}
        return out

    def stats_reset(self, t_from_ns: float) -> None:
        """New latency window: only arrivals at or after ``t_from_ns`` count."""
        _check(lib().hsma_queue_stats_reset(self._h, t_from_ns), "hsma_queue_stats_reset")

    def close(self) -> None:
        if self._h:
            _check(lib().hsma_queue_destroy(self._h), "hsma_queue_destroy")
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
