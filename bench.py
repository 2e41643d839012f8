#!/usr/bin/env python3
"""Throughput benchmark of the gfx950 TRSM library.

Default (no --workload): the batched configuration -- 10 000 independent
double-complex solves, m, n ~ U{8..64}, alpha = (1, 0.5), seed 1, one step =
the whole batch with descriptors resident in HBM (hsma_batch_plan_execute).
`value` is solves/s; the roofline is that of the grouped small-solve kernel
(HBM-bound).  The same JSON line carries the other parts of the headline
metric, each measured in this run: DTRSM m = n = 16384 and ZTRSM
m = n = 8192 (GFLOP/s, % of FP64 peak, roofline of the trailing-update
kernel, rocBLAS on the same GPU), graph replay against eager launches on a
mid-size blocked solve, the mixed-precision mode against FP64 at equal
backward error (kappa ~1e3 and ~1e6), and the serving run (p50/p99 latency,
solves/s) -- under "headline".

Single workloads (--workload):
  large_real     DTRSM m = n = 16384, alpha = -1, seed 2 (one step = one solve)
  large_complex  ZTRSM m = n = 8192, alpha = (-1, 0), seed 2
  batched        the default configuration alone
  single         DTRSM m = n = 32, alpha = 1, seed 0
  mixed          DTRSM m = 8192, n = 4096: mixed precision vs FP64 at equal
                 backward error, kappa(L) ~ 1e3 .. 1e6, seed 3
  serving        open-loop Poisson arrivals (--rate per s, --duration s) of
                 requests with m, n log-uniform in [8, 4096] x [1, 512], 30 %
                 complex, alpha ~ U(-2, 2), inputs drawn on the device from
                 Philox keys, 32 GiB budget, 60 s; reports p50/p99 latency
                 from scheduled arrival to completion (overall and per size
                 class) and solves/s

Prints one JSON line: metric/value, the roofline of the dominant kernel
measured with HIP events on its launch stream, rocBLAS on the same GPU and
inputs, and the CPU oracle timed on a bounded sample of the same work.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Hardware queues per process (HIP reads this once, at start-up, so it is set
# before torch is imported).  The serving queue runs a small-solve stream and
# eight blocked-class streams; with HIP's default of 4 queues these share
# in-order hardware queues, so a round's small solves wait behind other
# streams' blocked chains (20 s runs at 20 000 requests/s: p50 22.1 ms, small
# requests 17.0 ms with 4 queues; 16.3 ms and 10.3 ms with 12).  The
# benchmark process runs with 12 (HSMA_BENCH_HW_QUEUES overrides).
os.environ["GPU_MAX_HW_QUEUES"] = os.environ.get("HSMA_BENCH_HW_QUEUES", "12")
HW_QUEUES = int(os.environ["GPU_MAX_HW_QUEUES"])

import workloads as W  # noqa: E402

METRIC = "DTRSM/ZTRSM GFLOP/s and %FP64 peak; batched solves/s; served p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3     # MI355X dense FP32 (vector and matrix)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="default",
                    choices=["default", "large_real", "large_complex", "large_real_fp32",
                             "large_complex_fp32", "batched", "single", "mixed", "serving", "variants",
                             "cholesky", "tiny"])
    ap.add_argument("--ib", type=int, default=0, help="force I_B (0 = tuning table)")
    ap.add_argument("--m", type=int, default=0, help="override m (and n) for sweeps")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--count", type=int, default=0, help="batched: number of problems")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rocblas", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled parity check")
    ap.add_argument("--rate", type=float, default=20000.0, help="serving: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--streams", type=int, default=0, help="serving: queue streams (0 = default)")
    ap.add_argument("--budget-gib", type=float, default=0.0,
                    help="serving: HBM admission budget in GiB (0 = the library's 32 GiB)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="fill a 1 GiB tensor and copy it first (reference kernels of known size for counter runs)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# rocBLAS on the same GPU (comparison only; called through its public C API)
# ---------------------------------------------------------------------------
class RocBlas:
    SIDE_LEFT, FILL_LOWER, OP_NONE, DIAG_NON_UNIT, DIAG_UNIT = 141, 122, 111, 131, 132

    def __init__(self, stream_handle):
        self.lib = ctypes.CDLL("librocblas.so")
        self.h = ctypes.c_void_p()
        st = self.lib.rocblas_create_handle(ctypes.byref(self.h))
        if st != 0:
            raise RuntimeError(f"rocblas_create_handle: {st}")
        self.lib.rocblas_set_stream(self.h, ctypes.c_void_p(stream_handle))
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        for f in (self.lib.rocblas_dtrsm, self.lib.rocblas_ztrsm, self.lib.rocblas_strsm,
                  self.lib.rocblas_ctrsm):
            f.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp, i32, vp, i32]
            f.restype = i32

    def trsm_batched(self, cx, m, n, alpha, A_ptrs, lda, B_ptrs, ldb, count):
        """rocblas_ztrsm_batched or rocblas_dtrsm_batched (left, lower, no
        transpose, non-unit) on device arrays of device pointers."""
        f = self.lib.rocblas_ztrsm_batched if cx else self.lib.rocblas_dtrsm_batched
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        f.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp, i32, vp, i32, i32]
        f.restype = i32
        a = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
        st = f(self.h, self.SIDE_LEFT, self.FILL_LOWER, self.OP_NONE, self.DIAG_NON_UNIT, m, n, a,
               ctypes.c_void_p(A_ptrs), lda, ctypes.c_void_p(B_ptrs), ldb, count)
        if st != 0:
            raise RuntimeError(f"rocblas_{'z' if cx else 'd'}trsm_batched: {st}")

    SIDE = {"L": 141, "R": 142}
    UPLO = {"U": 121, "L": 122}
    OP = {"N": 111, "T": 112, "C": 113}

    def trsm_general(self, A, B, alpha, side, uplo, trans, unit=False):
        import torch
        import paper_2608_25469_amd as hs
        m, n = B.shape
        cx = B.dtype == torch.complex128
        a = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
        f = self.lib.rocblas_ztrsm if cx else self.lib.rocblas_dtrsm
        st = f(self.h, self.SIDE[side], self.UPLO[uplo], self.OP[trans],
               self.DIAG_UNIT if unit else self.DIAG_NON_UNIT, m, n, a,
               ctypes.c_void_p(A.data_ptr()), hs.leading_dim(A),
               ctypes.c_void_p(B.data_ptr()), hs.leading_dim(B))
        if st != 0:
            raise RuntimeError(f"rocblas trsm: {st}")

    def trsm(self, L, B, alpha, unit=False):
        import torch
        import paper_2608_25469_amd as hs
        m, n = B.shape
        single = B.dtype in (torch.float32, torch.complex64)
        cx = B.dtype in (torch.complex128, torch.complex64)
        st = ctypes.c_float if single else ctypes.c_double
        a = (st * 2)(complex(alpha).real, complex(alpha).imag)
        if single:
            f = self.lib.rocblas_ctrsm if cx else self.lib.rocblas_strsm
        else:
            f = self.lib.rocblas_ztrsm if cx else self.lib.rocblas_dtrsm
        st = f(self.h, self.SIDE_LEFT, self.FILL_LOWER, self.OP_NONE,
               self.DIAG_UNIT if unit else self.DIAG_NON_UNIT, m, n, a,
               ctypes.c_void_p(L.data_ptr()), hs.leading_dim(L),
               ctypes.c_void_p(B.data_ptr()), hs.leading_dim(B))
        if st != 0:
            raise RuntimeError(f"rocblas trsm: {st}")


def measured_traffic(name, sources, ok=True):
    """HBM bytes per launch of a kernel from a committed rocprofv3
    FETCH_SIZE/WRITE_SIZE measurement (profiles/<name>.json), if it was taken
    on the current kernel sources; otherwise None."""
    import hashlib
    if not ok:
        return None
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", name + ".json")))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for src in sources:
        try:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        except OSError:
            return None
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    return rec.get("hbm_bytes_per_launch")


GEMM_SOURCES = ["paper_2608_25469_amd/csrc/gemm.hip"]
SMALL_SOURCES = ["paper_2608_25469_amd/csrc/small_kernels.h", "paper_2608_25469_amd/csrc/dpp_fma.h",
                 "paper_2608_25469_amd/csrc/strip.hip", "paper_2608_25469_amd/csrc/batched.cpp",
                 "paper_2608_25469_amd/csrc/strip_pack.h"]


def time_gpu(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / steps


def cpu_oracle_columns(L, B, alpha, target_s, complex_):
    """Oracle on a growing column sample until it takes about target_s."""
    import oracle
    n = B.shape[1]
    rng = np.random.default_rng(123)
    k = 2
    while True:
        cols = rng.choice(n, size=min(k, n), replace=False)
        Bs = np.asfortranarray(B[:, cols])
        t1 = time.perf_counter()
        oracle.solve(L, Bs, alpha)
        dt = time.perf_counter() - t1
        if dt * 4 > target_s or k >= n:
            break
        k = min(n, max(k * 2, int(k * target_s / max(dt, 1e-3) / 1.2)))
    gf = W.flops(L.shape[0], len(cols), complex_) / dt / 1e9
    return {"value": round(gf, 3), "unit": "GFLOP/s", "cores": min(oracle.num_threads(), len(cols)),
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"{len(cols)} of {n} columns of the same solve (columns are independent)"}


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def run_single_problem(args, torch, hs, cfg):
    m, n, cx, alpha, seed = cfg["m"], cfg["n"], cfg["complex_"], cfg["alpha"], cfg["seed"]
    f32 = bool(cfg.get("fp32"))
    t0 = time.time()
    L, B = W.problem(seed, m, n, cx)
    if f32:
        # the FP32 problem; the oracle solves it exactly promoted to FP64
        L = np.asfortranarray(L.astype(np.complex64 if cx else np.float32))
        B = np.asfortranarray(B.astype(np.complex64 if cx else np.float32))
    log(f"inputs m={m} n={n} complex={cx} fp32={f32} generated in {time.time() - t0:.1f}s")
    Ld = hs.to_colmajor(L)
    Bd = hs.to_colmajor(B)
    torch.cuda.synchronize()

    _, rep = hs.trsm(Ld, Bd, alpha, block_size=args.ib, report=True)
    torch.cuda.synchronize()
    parity = None
    if not args.no_check:
        import oracle
        cols = np.unique(np.linspace(0, n - 1, num=min(n, 8)).astype(int))
        Xs = np.asfortranarray(Bd[:, cols.tolist()].cpu().numpy())
        Bs = np.asfortranarray(B[:, cols])
        Lo = L
        if f32:
            wide = np.complex128 if cx else np.float64
            Xs, Bs = np.asfortranarray(Xs.astype(wide)), np.asfortranarray(Bs.astype(wide))
            Lo = np.asfortranarray(L.astype(wide))
        ref = oracle.solve(Lo, Bs, alpha)
        rel = oracle.rel_err_fro(Xs, ref)
        eta = oracle.backward_error(Lo, Xs, Bs, alpha)
        bound = 10 * m * 2.0 ** (-24 if f32 else -53)
        parity = {"sampled_columns": int(len(cols)), "rel_err_fro": rel, "backward_error": eta,
                  "bound": bound, "ok": bool(eta <= bound and (f32 or rel <= 1e-12))}
        log(f"parity on {len(cols)} columns: rel={rel:.2e} eta={eta:.2e}")

    for _ in range(args.warmup):
        hs.trsm(Ld, Bd, alpha, block_size=args.ib)
    torch.cuda.synchronize()
    if rep["path"] != 2:
        # A lone small solve is bound by call and launch latency: time it
        # without the phase profiler's events, then profile a second pass of
        # the same length for the kernel's own duration.
        ts = time.perf_counter()
        for _ in range(args.steps):
            hs.trsm(Ld, Bd, alpha, block_size=args.ib)
        torch.cuda.synchronize()
        te = time.perf_counter()
        hs.profile_begin()
        for _ in range(args.steps):
            hs.trsm(Ld, Bd, alpha, block_size=args.ib)
        torch.cuda.synchronize()
        prof = hs.profile_end()
    else:
        hs.profile_begin()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(args.steps):
            hs.trsm(Ld, Bd, alpha, block_size=args.ib)
        torch.cuda.synchronize()
        te = time.perf_counter()
        prof = hs.profile_end()
    ms = (te - ts) * 1e3 / args.steps
    fl = W.flops(m, n, cx)

    phases = {}
    busy = sum(v["ms"] for v in prof.values())
    for k, v in prof.items():
        phases[k] = {"launches_per_step": v["launches"] // args.steps, "ms_per_step": v["ms"] / args.steps,
                     "share": v["ms"] / busy if busy else None}
    if rep["path"] == 2:
        up = prof["update"]
        avg = up["ms"] / up["launches"]
        ach = (up["flops"] / up["launches"]) / (avg * 1e-3) / 1e12
        peak = FP32_PEAK_TFLOPS if f32 else FP64_PEAK_TFLOPS
        roof = {"bound": "mfma", "kernel": "hsma_gemm32 (trailing-update role)" if f32 else
                "hsma_gemm (trailing-update role)", "achieved": round(ach, 3),
                "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                "traffic": measured_traffic("gemm_update_dtrsm16384_traffic", GEMM_SOURCES,
                                            (m, n, cx, args.ib, f32) == (16384, 16384, False, 0, False)),
                "avg_launch_ms": avg, "launches_per_step": up["launches"] // args.steps,
                "flops_per_launch": up["flops"] / up["launches"],
                "per_unit": "2 flops per real multiply-add of C -= A B (complex: its real expansion)"}
    else:
        sm = prof["small"]
        avg = sm["ms"] / max(1, sm["launches"])
        byts = W.algorithmic_bytes(m, n, cx)
        ach = byts / (avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "hsma_strip_solve", "achieved": round(ach, 3),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 6),
                "traffic": None, "avg_launch_ms": avg,
                "per_unit": "bytes: lower triangle of L once, B read and written once"}

    rocblas = None
    if not args.no_rocblas:
        try:
            rb = RocBlas(torch.cuda.current_stream().cuda_stream)
            Bd2 = hs.to_colmajor(B)
            rms = time_gpu(lambda: rb.trsm(Ld, Bd2, alpha), max(2, args.steps), 1, torch)
            rocblas = {"ms_per_step": round(rms, 4), "gflops": round(fl / (rms * 1e-3) / 1e9, 2),
                       "speedup_ours": round(rms / ms, 3)}
            del Bd2
        except Exception as e:  # rocBLAS missing or failing is reported, not fatal
            rocblas = {"error": str(e)}

    cpu = None
    if not args.no_cpu_baseline:
        if f32:
            wide = np.complex128 if cx else np.float64
            cpu = cpu_oracle_columns(np.asfortranarray(L.astype(wide)), np.asfortranarray(B.astype(wide)),
                                     alpha, args.cpu_seconds, cx)
        else:
            cpu = cpu_oracle_columns(L, B, alpha, args.cpu_seconds, cx)

    value = fl / (ms * 1e-3) / 1e9
    out_peak = FP32_PEAK_TFLOPS if f32 else FP64_PEAK_TFLOPS
    return {
        "value": round(value, 2), "unit": "GFLOP/s", "ms_per_step": round(ms, 4),
        "dtype": ("c64" if cx else "f32") if f32 else ("c128" if cx else "f64"),
        "pct_fp64_peak": round(100 * value / (FP64_PEAK_TFLOPS * 1e3), 2),
        "pct_of_own_peak": round(100 * value / (out_peak * 1e3), 2),
        "extra_config": {"m": m, "n": n, "complex": cx, "path": rep["path"],
                         "block_size": rep["block_size"], "flops_per_step": fl},
        "phases": phases, "parity": parity, "roofline": roof, "rocblas": rocblas, "cpu_baseline": cpu,
    }


# Worker processes of the problem-parallel CPU baseline (the host share of
# one GPU).
CPU_WORKERS = 16


def _cpu_batch_worker(job):
    """One process of the batched CPU baseline: the oracle on one thread,
    solving problems rank, rank + P, ... of the seeded batch for about
    `seconds`.  Returns (solves, flops, seconds)."""
    rank, nproc, bcfg, seconds = job
    import oracle
    oracle.set_num_threads(1)
    b = W.batched(**bcfg)
    count = len(b.shapes)
    t1 = time.perf_counter()
    done, fl, i = 0, 0.0, rank % count
    while time.perf_counter() - t1 < seconds:
        oracle.solve(b.L[i], b.B[i], b.alpha)
        fl += W.flops(*b.shapes[i], b.complex_)
        done += 1
        i += nproc
        if i >= count:
            i = rank % count
    return done, fl, time.perf_counter() - t1


def run_batched(args, torch, hs, cfg):
    count = args.count or cfg["count"]
    t0 = time.time()
    b = W.batched(seed=cfg["seed"], count=count, lo=cfg["lo"], hi=cfg["hi"],
                  complex_=cfg["complex_"], alpha=cfg["alpha"])
    pl, pb, vl, vb = hs.pack_batch(b.L, b.B)
    pb0 = pb.clone()
    torch.cuda.synchronize()
    log(f"batch of {count} generated and packed in {time.time() - t0:.1f}s")
    probs = [hs.problem_struct(L, B, b.alpha) for L, B in zip(vl, vb)]
    plan = hs.BatchPlan(probs)
    plan.execute()
    torch.cuda.synchronize()
    parity = None
    if not args.no_check:
        import oracle
        worst_rel = worst_eta = 0.0
        idx = list(range(0, count, max(1, count // 200)))
        for i in idx:
            X = hs.from_colmajor(vb[i])
            ref = oracle.solve(b.L[i], b.B[i], b.alpha)
            worst_rel = max(worst_rel, oracle.rel_err_fro(X, ref))
            worst_eta = max(worst_eta, oracle.backward_error(b.L[i], X, b.B[i], b.alpha) /
                            (10 * b.shapes[i][0] * 2.0 ** -53))
        parity = {"sampled_problems": len(idx), "worst_rel_err_fro": worst_rel,
                  "worst_backward_error_over_bound": worst_eta,
                  "ok": bool(worst_rel <= 1e-12 and worst_eta <= 1.0)}
        log(f"parity on {len(idx)} problems: rel<={worst_rel:.2e} eta/bound<={worst_eta:.2e}")

    # Timed: K executions of the whole batch (descriptors resident).
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        plan.execute()
    torch.cuda.synchronize()
    hs.profile_begin()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.execute()
    ev1.record(stream)
    torch.cuda.synchronize()
    te = time.perf_counter()
    prof = hs.profile_end()
    ms = (te - ts) * 1e3 / args.steps
    ev_ms = ev0.elapsed_time(ev1) / args.steps
    fl = b.total_flops()
    byts = b.total_bytes()
    # The dominant kernel is the strip kernel.  Problems with m, n <= 16 ride
    # in its launch when the batch has other small problems (else they run in
    # the fused kernel's own launch, and are left out of its bytes).
    cx = bool(cfg["complex_"])
    es = 16 if cx else 8
    tiny = [(m_, n_) for m_, n_ in b.shapes if m_ <= 16 and n_ <= 16]
    tiny_launched = prof["tiny"]["launches"] > 0
    byts_small = byts - (sum(W.algorithmic_bytes(m_, n_, cx) for m_, n_ in tiny) if tiny_launched else 0)
    sm = prof["small"]
    launches = max(1, sm["launches"] // args.steps)
    avg_launch_ms = sm["ms"] / max(1, sm["launches"])
    bytes_per_launch = byts_small / launches
    ach = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    traffic = measured_traffic("strip_solve_batched10000_traffic", SMALL_SOURCES,
                               count == cfg["count"] and dict(cfg) == dict(W.BATCHED))
    roof = {"bound": "hbm", "kernel": "hsma_strip_solve (grouped: four 16-column strips per wavefront)",
            "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_ms": avg_launch_ms, "launches_per_step": launches,
            "bytes_per_launch": bytes_per_launch, "bytes_per_step": byts,
            "very_small_problems": len(tiny), "very_small_in_strip_launch": not tiny_launched,
            "fused_launch_ms_per_step": prof["tiny"]["ms"] / args.steps,
            "step_ms_events": ev_ms,
            "step_rate_gbs": round(byts / (ev_ms * 1e-3) / 1e9, 2),
            "per_unit": f"per problem: {es} (m(m+1)/2 + 2mn) bytes (lower triangle of L once, B read and "
                        "written once); a launch serves one (dtype, diag) group, so bytes per "
                        "launch = bytes of the group's problems (one group here: every problem is "
                        f"{'complex' if cx else 'real'} with a non-unit diagonal, the ones with "
                        "m, n <= 16 included as one-strip items)" if not tiny_launched else
                        f"per problem: {es} (m(m+1)/2 + 2mn) bytes; the problems with m, n <= 16 ran "
                        "in the fused kernel's own launch and are not counted"}

    # One-shot API (host descriptors uploaded each call) for reference.
    oneshot_ms = time_gpu(lambda: hs.trsm_batched(probs), max(2, args.steps), 1, torch)

    rocblas = None
    if not args.no_rocblas:
        try:
            rb = RocBlas(torch.cuda.current_stream().cuda_stream)
            pb.copy_(pb0)

            def rb_loop():
                for L, B in zip(vl, vb):
                    rb.trsm(L, B, b.alpha)
            rms = time_gpu(rb_loop, 2, 1, torch)
            rocblas = {"kind": f"rocblas_{'z' if cx else 'd'}trsm called once per problem",
                       "ms_per_step": round(rms, 3),
                       "solves_per_s": round(count / (rms * 1e-3), 1), "speedup_ours": round(rms / ms, 2)}
            # rocBLAS's batched call on each uniform (m, n) group of the batch
            groups = {}
            for i, (m_, n_) in enumerate(b.shapes):
                groups.setdefault((m_, n_), []).append(i)
            ptrs = []
            for (m_, n_), idx in groups.items():
                pa = torch.tensor([vl[i].data_ptr() for i in idx], dtype=torch.int64, device="cuda")
                pbp = torch.tensor([vb[i].data_ptr() for i in idx], dtype=torch.int64, device="cuda")
                ptrs.append((m_, n_, pa, pbp, len(idx)))
            pb.copy_(pb0)

            def rb_groups():
                for m_, n_, pa, pbp, cnt in ptrs:
                    rb.trsm_batched(cx, m_, n_, b.alpha, pa.data_ptr(), m_, pbp.data_ptr(), m_, cnt)
            gms = time_gpu(rb_groups, 3, 1, torch)
            rocblas_batched = {"kind": f"rocblas_{'z' if cx else 'd'}trsm_batched once per uniform (m, n) group",
                               "groups": len(ptrs), "ms_per_step": round(gms, 3),
                               "solves_per_s": round(count / (gms * 1e-3), 1),
                               "speedup_ours": round(gms / ms, 2)}
            rocblas = {"per_problem_loop": rocblas, "batched_per_shape": rocblas_batched}
        except Exception as e:
            rocblas = {"error": str(e)}

    cpu = None
    if not args.no_cpu_baseline:
        # The oracle in parallel over problems: worker processes, each the
        # oracle on one thread, over their share of the same seeded batch
        # (regenerated in the worker) for about cpu_seconds.
        import multiprocessing as mp
        nproc = min(CPU_WORKERS, os.cpu_count() or 1)
        bcfg = dict(seed=cfg["seed"], count=count, lo=cfg["lo"], hi=cfg["hi"],
                    complex_=cfg["complex_"], alpha=cfg["alpha"])
        with mp.get_context("spawn").Pool(nproc) as pool:
            res = pool.map(_cpu_batch_worker, [(r, nproc, bcfg, args.cpu_seconds) for r in range(nproc)])
        done = sum(r[0] for r in res)
        fl_done = sum(r[1] for r in res)
        dt = max(r[2] for r in res)
        passes = done / count
        cpu = {"value": round(fl_done / dt / 1e9, 3), "unit": "GFLOP/s", "cores": nproc,
               "kind": "oracle", "solves_per_s": round(done / dt, 1), "seconds": round(dt, 2),
               "sample": (f"{passes:.1f} passes over all {count} problems" if passes >= 1 else
                          f"{done} of {count} problems") +
                         f", {nproc} processes, each the oracle on one thread over every "
                         f"{nproc}th problem"}
    plan.close()
    gflops = fl / (ms * 1e-3) / 1e9
    return {
        "value": round(count / (ms * 1e-3), 1), "unit": "solves/s", "ms_per_step": round(ms, 4),
        "dtype": "c128" if cx else "f64", "gflops": round(gflops, 2),
        "pct_fp64_peak": round(100 * gflops / (FP64_PEAK_TFLOPS * 1e3), 3),
        "solves_per_s": round(count / (ms * 1e-3), 1),
        "extra_config": {"count": count, "flops_per_step": fl, "bytes_per_step": byts,
                         "oneshot_ms_per_call": round(oneshot_ms, 4)},
        "parity": parity, "roofline": roof, "rocblas": rocblas, "cpu_baseline": cpu,
    }


def run_variants(args, torch, hs, k=8192, reps=3):
    """The general BLAS TRSM (hsma_trsm_general) on DTRSM m = n = k in every
    real form (side x stored triangle x op(A)), against rocBLAS's same form,
    with the share of time spent in the re-indexing copies and an oracle check
    on sampled columns (left side) or rows (right side)."""
    import oracle
    rows = []
    L, B = W.problem(2, k, k, False)
    Ld = hs.to_colmajor(L)
    Ud = hs.to_colmajor(np.asfortranarray(L.T))
    B0 = hs.to_colmajor(B)
    Bd = hs.colmajor(k, k, torch.float64)
    fl = W.flops(k, k, False)
    try:
        rb = RocBlas(torch.cuda.current_stream().cuda_stream)
    except Exception as e:  # reported, not fatal
        rb = None
        log(f"rocBLAS unavailable: {e}")
    for side in "LR":
        for uplo in "LU":
            for trans in "NT":
                A = Ld if uplo == "L" else Ud
                Ah = L if uplo == "L" else np.asfortranarray(L.T)

                def ours():
                    hs.trsm_general(A, Bd, -1.0, side=side, uplo=uplo, trans=trans)
                Bd.copy_(B0)
                ours()
                torch.cuda.synchronize()
                idx = np.unique(np.linspace(0, k - 1, num=4).astype(int)).tolist()
                if side == "L":
                    Xs = np.asfortranarray(Bd[:, idx].cpu().numpy())
                    Bs = np.asfortranarray(B[:, idx])
                else:
                    Xs = np.asfortranarray(Bd[idx, :].cpu().numpy())
                    Bs = np.asfortranarray(B[idx, :])
                ref = oracle.solve_general(Ah, Bs, -1.0, side, uplo, trans)
                rel = oracle.rel_err_fro(Xs, ref)
                ts = []
                hs.profile_begin()
                for _ in range(reps):
                    Bd.copy_(B0)
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    ours()
                    torch.cuda.synchronize()
                    ts.append((time.perf_counter() - t) * 1e3)
                prof = hs.profile_end()
                busy = sum(v["ms"] for v in prof.values())
                ms = min(ts)
                row = {"side": side, "uplo": uplo, "trans": trans, "ms": round(ms, 3),
                       "gflops": round(fl / (ms * 1e-3) / 1e9, 1),
                       "copy_share": round(prof["other"]["ms"] / busy, 4) if busy else None,
                       "sampled": f"{len(idx)} {'columns' if side == 'L' else 'rows'}",
                       "rel_err_fro_vs_oracle": rel, "parity_ok": bool(rel <= 1e-12)}
                if rb is not None:
                    rts = []
                    for _ in range(reps):
                        Bd.copy_(B0)
                        torch.cuda.synchronize()
                        t = time.perf_counter()
                        rb.trsm_general(A, Bd, -1.0, side, uplo, trans)
                        torch.cuda.synchronize()
                        rts.append((time.perf_counter() - t) * 1e3)
                    row["rocblas_ms"] = round(min(rts), 3)
                    row["speedup_over_rocblas"] = round(min(rts) / ms, 3)
                rows.append(row)
                log(f"variant {side}{uplo}{trans} k={k}: {ms:.2f} ms ({row['gflops']} GF/s), "
                    f"rocBLAS {row.get('rocblas_ms')} ms, copies {row['copy_share']}, rel {rel:.1e}")
    del Ld, Ud, B0, Bd
    return {"workload": f"DTRSM m=n={k}, alpha=-1, seed 2, every real (side, uplo, trans)",
            "flops_per_solve": fl, "rows": rows}


def hermitian_pd(n, cx, seed):
    """A = (R + R^H)/2 + n I, R with entries U(-1, 1) (complex: real and
    imaginary parts): Hermitian, eigenvalues within n +- 2 sqrt(n), so
    positive definite and well conditioned; O(n^2) to draw."""
    rng = np.random.default_rng(seed)
    R = rng.uniform(-1.0, 1.0, size=(n, n))
    if cx:
        R = R + 1j * rng.uniform(-1.0, 1.0, size=(n, n))
    A = (R + R.conj().T) * 0.5
    A[np.diag_indices(n)] += n
    return np.asfortranarray(A)


def run_cholesky(args, torch, hs, sizes=((16384, False), (8192, True)), reps=3):
    """Cholesky factorization on the library's TRSM (hsma_potrf) against
    rocSOLVER's potrf on the same GPU; flops n^3/3 (complex 4 n^3/3).  The
    factor is checked by its reconstruction residual on sampled columns."""
    rows = []
    for n, cx in sizes:
        A = hermitian_pd(n, cx, 5)
        Ad0 = hs.to_colmajor(A)
        Ad = hs.colmajor(n, n, Ad0.dtype)
        fl = (4.0 if cx else 1.0) * n ** 3 / 3.0
        Ad.copy_(Ad0)
        hs.potrf(Ad)
        torch.cuda.synchronize()
        cols = np.unique(np.linspace(0, n - 1, num=8).astype(int))
        Lh = np.tril(Ad.cpu().numpy())          # (n, n) host copy (logical order), lower part
        res = 0.0
        for j in cols:
            col = Lh @ np.conj(Lh[j, :])          # (L L^H)[:, j]
            res = max(res, np.max(np.abs(col - A[:, j])) / np.max(np.abs(A)))
        del Lh
        ts = []
        hs.profile_begin()
        for _ in range(reps):
            Ad.copy_(Ad0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            hs.potrf(Ad)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        prof = hs.profile_end()
        busy = sum(v["ms"] for v in prof.values())
        ms = min(ts)
        trsm_ms = sum(prof[k]["ms"] for k in ("diag_inv", "update", "leaf_solve", "small", "other")) / reps
        row = {"workload": f"{'ZPOTRF' if cx else 'DPOTRF'} n={n}, A = (R + R^H)/2 + n I, seed 5",
               "ms": round(ms, 3), "gflops": round(fl / (ms * 1e-3) / 1e9, 1),
               "trsm_share": round(trsm_ms * reps / busy, 4) if busy else None,
               "factor_share": round(prof["factor"]["ms"] / busy, 4) if busy else None,
               "reconstruction_residual_sampled": res, "parity_ok": bool(res <= 10 * n * 2.0 ** -53)}
        try:
            lib = ctypes.CDLL("librocsolver.so")
            rb = RocBlas(torch.cuda.current_stream().cuda_stream)
            f = lib.rocsolver_zpotrf if cx else lib.rocsolver_dpotrf
            f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                          ctypes.c_int32, ctypes.c_void_p]
            f.restype = ctypes.c_int32
            info = torch.zeros(1, dtype=torch.int32, device="cuda")
            rts = []
            for _ in range(reps):
                Ad.copy_(Ad0)
                torch.cuda.synchronize()
                t = time.perf_counter()
                st = f(rb.h, 122, n, ctypes.c_void_p(Ad.data_ptr()), hs.leading_dim(Ad),
                       ctypes.c_void_p(info.data_ptr()))
                torch.cuda.synchronize()
                rts.append((time.perf_counter() - t) * 1e3)
                if st != 0:
                    raise RuntimeError(f"rocsolver potrf: {st}")
            row["rocsolver_ms"] = round(min(rts), 3)
            row["speedup_over_rocsolver"] = round(min(rts) / ms, 3)
        except Exception as e:  # reported, not fatal
            row["rocsolver"] = {"error": repr(e)}
        rows.append(row)
        log(f"potrf n={n} complex={cx}: {ms:.2f} ms ({row['gflops']} GF/s), rocSOLVER {row.get('rocsolver_ms')} ms, "
            f"TRSM share {row['trsm_share']}, residual {res:.1e}")
        del Ad, Ad0
        torch.cuda.empty_cache()
    return {"rows": rows, "flop_convention": "n^3/3 (complex 4 n^3/3)"}


def run_tiny(args, torch, hs, count=100000, reps=10):
    """Very small solves, fused four per wavefront: `count` complex problems
    with m, n ~ U{1..16}, alpha = (1, 0.5), seed 6, as one resident plan;
    solves/s and algorithmic HBM bytes/s; every 50th problem against the
    oracle."""
    import oracle
    b = W.batched(seed=6, count=count, lo=1, hi=16, complex_=True, alpha=complex(1.0, 0.5))
    pl, pb, vl, vb = hs.pack_batch(b.L, b.B)
    pb0 = pb.clone()
    plan = hs.BatchPlan([hs.problem_struct(L, B, b.alpha) for L, B in zip(vl, vb)])
    plan.execute()
    torch.cuda.synchronize()
    worst = 0.0
    for i in range(0, count, 50):
        X = hs.from_colmajor(vb[i])
        worst = max(worst, oracle.rel_err_fro(X, oracle.solve(b.L[i], b.B[i], b.alpha)))
    pb.copy_(pb0)
    ms = time_gpu(plan.execute, reps, 2, torch)
    plan.close()
    byts = b.total_bytes()
    return {"workload": f"{count} complex solves, m, n ~ U{{1..16}}, alpha=(1,0.5), seed 6",
            "ms_per_batch": round(ms, 4), "solves_per_s": round(count / (ms * 1e-3), 1),
            "algorithmic_gbs": round(byts / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "parity": {"sampled_problems": len(range(0, count, 50)), "worst_rel_err_fro": worst,
                       "ok": bool(worst <= 1e-12)}}


def run_graph(args, torch, hs, sizes=(256, 512, 1024), reps=32):
    """The blocked schedule replayed as a per-shape HIP graph (arguments of
    each call moved into the instantiated graph) vs launched eagerly, on
    mid-size DTRSMs where launch overhead matters: `reps` back-to-back solves
    over 8 different (L, B) pairs, so nearly every call changes the pointers.
    The first call of each mode is untimed (it captures); results compared
    bit for bit."""
    return [run_graph_one(torch, hs, m, m, reps) for m in sizes]


def run_graph_one(torch, hs, m, n, reps, nbuf=8):
    pairs = [W.problem(2 + k, m, n, False) for k in range(nbuf)]
    Ls = [hs.to_colmajor(L) for L, _ in pairs]
    B0 = [hs.to_colmajor(B) for _, B in pairs]
    Bs = [b.clone() for b in B0]
    out = {}
    hs.graph_cache_clear()
    for mode in ("eager", "graph"):
        g = mode == "graph"
        for b, b0 in zip(Bs, B0):
            b.copy_(b0)
        for k in range(nbuf):          # first pass: captures, results kept
            hs.trsm(Ls[k], Bs[k], -1.0, graph=g)
        torch.cuda.synchronize()
        out[mode + "_first"] = [b.clone() for b in Bs]
        stats0 = hs.graph_stats()
        t = time.perf_counter()
        for r in range(reps):
            k = r % nbuf
            hs.trsm(Ls[k], Bs[k], -1.0, graph=g)   # re-solves in place: same work each time
        torch.cuda.synchronize()
        out[mode + "_ms"] = (time.perf_counter() - t) * 1e3 / reps
        if g:
            st = hs.graph_stats()
            out["timed_captures"] = st["captures"] - stats0["captures"]
            out["timed_updates"] = st["updates"] - stats0["updates"]
    same = all(bool(torch.equal(a, b)) for a, b in zip(out.pop("eager_first"), out.pop("graph_first")))
    hs.graph_cache_clear()
    return {"workload": f"DTRSM m=n={m}, blocked path, {nbuf} (L, B) pairs in turn",
            "eager_ms": round(out["eager_ms"], 4), "graph_ms": round(out["graph_ms"], 4),
            "speedup": round(out["eager_ms"] / out["graph_ms"], 3), "bitwise_equal": same,
            "captures_in_timed_loop": out["timed_captures"], "updates_in_timed_loop": out["timed_updates"]}


def run_mixed(args, torch, hs, cfg, kappas=(1e3, 1e4, 1e5, 1e6)):
    """Mixed precision vs plain FP64 at equal backward error (<= 1e-13) on
    m = 8192, n = 4096, for kappa_inf(L) of about 1e3, 1e4, 1e5, 1e6."""
    import oracle
    m, n = (args.m or cfg["m"]), (args.n or cfg["n"])
    kappas = list(kappas)
    rows = []
    fl = W.flops(m, n, False)

    def timed(fn, Bd, Bpristine, reps):
        ts = []
        out = None
        for _ in range(reps):
            Bd.copy_(Bpristine)
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        return min(ts), sum(ts) / len(ts), out

    for kappa in kappas:
        L, B = W.mixed_problem(m, n, kappa, seed=cfg["seed"])
        Ld, Bd, Bp = hs.to_colmajor(L), hs.to_colmajor(B), hs.to_colmajor(B)
        torch.cuda.synchronize()
        # plain FP64 solve time, then its backward error (separate call)
        reps = max(2, args.steps)
        hs.trsm(Ld, Bd, 1.0)
        t64, a64, _ = timed(lambda: hs.trsm(Ld, Bd, 1.0), Bd, Bp, reps)
        Bd.copy_(Bp)
        _, r64 = hs.trsm(Ld, Bd, 1.0, backward_error=True, report=True)
        cols64 = np.unique(np.linspace(0, n - 1, num=8).astype(int))
        X64 = np.asfortranarray(Bd[:, cols64.tolist()].cpu().numpy())
        eta64_or = oracle.backward_error(L, X64, np.asfortranarray(B[:, cols64]), 1.0)
        tol = max(1e-13, r64["backward_error"])
        # mixed: FP32 updates, refine until the backward error reaches tol
        hs.trsm(Ld, Bd, 1.0, mixed=True)
        tmx, amx, (_, rmx) = timed(lambda: hs.trsm(Ld, Bd, 1.0, mixed=True, refine_steps=-1,
                                                   refine_tol=tol, report=True), Bd, Bp, reps)
        # and the mixed solve alone (no refinement), for the kernel-level ratio
        t32, _, _ = timed(lambda: hs.trsm(Ld, Bd, 1.0, mixed=True), Bd, Bp, reps)
        # one fixed refinement step without the certifying residual (its
        # backward error is checked by the oracle on sampled columns below)
        t1s, _, _ = timed(lambda: hs.trsm(Ld, Bd, 1.0, mixed=True, refine_steps=1), Bd, Bp, reps)
        cols1 = np.unique(np.linspace(0, n - 1, num=8).astype(int))
        X1 = np.asfortranarray(Bd[:, cols1.tolist()].cpu().numpy())
        eta1 = oracle.backward_error(L, X1, np.asfortranarray(B[:, cols1]), 1.0)
        Bd.copy_(Bp)
        hs.trsm(Ld, Bd, 1.0, mixed=True, refine_steps=-1, refine_tol=tol)
        torch.cuda.synchronize()
        cols = np.unique(np.linspace(0, n - 1, num=8).astype(int))
        X = np.asfortranarray(Bd[:, cols.tolist()].cpu().numpy())
        ref = oracle.solve(L, np.asfortranarray(B[:, cols]), 1.0)
        eta_or = oracle.backward_error(L, X, np.asfortranarray(B[:, cols]), 1.0)
        rows.append({"kappa_target": kappa, "scale": W.mixed_scale(m, kappa),
                     "fp64_ms": round(t64, 3), "fp64_eta": r64["backward_error"],
                     "fp64_eta_oracle_sampled": eta64_or,
                     "mixed_ms": round(tmx, 3), "mixed_eta": rmx["backward_error"],
                     "mixed_refine_steps": rmx["refine_steps"], "target_eta": tol,
                     "mixed_solve_only_ms": round(t32, 3),
                     "mixed_one_step_ms": round(t1s, 3), "mixed_one_step_eta_sampled": eta1,
                     "speedup_one_step_over_fp64": round(t64 / t1s, 3),
                     "speedup_mixed_over_fp64": round(t64 / tmx, 3),
                     "oracle_eta_sampled": eta_or, "forward_err_vs_oracle": oracle.rel_err_fro(X, ref)})
        log(f"kappa {kappa:.0e}: fp64 {t64:.2f} ms eta {r64['backward_error']:.2e} | mixed {tmx:.2f} ms "
            f"({rmx['refine_steps']} steps) eta {rmx['backward_error']:.2e} | solve-only {t32:.2f} ms")
        del Ld, Bd, Bp
    first = rows[0]
    value = fl / (first["mixed_ms"] * 1e-3) / 1e9
    return {
        "value": round(value, 2), "unit": "GFLOP/s", "ms_per_step": first["mixed_ms"], "dtype": "f64",
        "pct_fp64_peak": round(100 * value / (FP64_PEAK_TFLOPS * 1e3), 2),
        "extra_config": {"m": m, "n": n, "flops_per_solve": fl,
                         "value_is": "effective GFLOP/s of the mixed mode with refinement at kappa 1e3"},
        "mixed": rows,
    }


def run_serving(args, torch, hs):
    """Open-loop serving run through the library's request queue.

    Requests are fire-and-forget (their records are dropped when they finish)
    except a small sample kept for the oracle check; latencies come from the
    queue's own statistics, windowed to arrivals after the warm-up."""
    import bisect
    rate, duration = args.rate, args.duration
    warm_s = min(5.0, duration / 4)
    seed = 4
    stream = W.serving_stream(seed=seed, rate=rate, duration=duration)
    N = len(stream)
    # Requests to verify against the oracle: spread over the run, cheap on the CPU.
    sample = set()
    budget_flops = 3e9
    for i in range(0, N, max(1, N // 400)):
        r = stream[i]
        f = W.flops(r.m, r.n, r.complex_)
        if f <= budget_flops / 40:
            sample.add(i)
            budget_flops -= f
        if budget_flops <= 0 or len(sample) >= 40:
            break
    arr = (hs.Request * N)()
    t_sched = np.array([r.t_arrival for r in stream])
    for i, r in enumerate(stream):
        keep = i in sample
        arr[i] = hs.request(r.m, r.n, r.alpha, complex_=r.complex_, key=W.serving_key(seed, r.rid),
                            release_on_completion=not keep, forget=not keep)
    total_flops = sum(W.flops(r.m, r.n, r.complex_) for r in stream)
    log(f"serving: {N} requests over {duration:.0f} s at {rate:.0f}/s, "
        f"{total_flops / duration / 1e12:.2f} TFLOP/s offered")
    L = hs.lib()
    budget = int(args.budget_gib * 2**30) if args.budget_gib > 0 else 0
    q = hs.Queue(n_streams=args.streams, hbm_budget_bytes=budget)
    # Warm-up (first launches of every kernel family, memory pool growth).
    wk = [hs.request(m, n, 1.0, complex_=cx, key=W.serving_key(99, k))
          for k, (m, n, cx) in enumerate([(m, n, cx) for m in (8, 40, 64, 100, 300, 1000, 3000)
                                          for n in (1, 64, 500) for cx in (False, True)])]
    for t in q.submit(wk):
        q.wait(t, 120)
    rsz = ctypes.sizeof(hs.Request)
    tickets = (ctypes.c_uint64 * N)()
    t0 = hs.clock_ns() + 2e6
    for i in range(N):
        arr[i].t_arrival_ns = t0 + t_sched[i] * 1e9
    sched_ns = t0 + t_sched * 1e9
    q.stats_reset(t0 + warm_s * 1e9)
    base_completed = q.stats()["completed"]
    submitted = 0
    last_log = time.time()
    while submitted < N:
        now = hs.clock_ns()
        hi = bisect.bisect_right(sched_ns, now, lo=submitted)
        if hi > submitted:
            st = L.hsma_queue_submit(q._h, ctypes.cast(ctypes.addressof(arr) + submitted * rsz,
                                                       ctypes.POINTER(hs.Request)),
                                     hi - submitted,
                                     ctypes.cast(ctypes.addressof(tickets) + submitted * 8,
                                                 ctypes.POINTER(ctypes.c_uint64)))
            if st != 0:
                raise hs.HsmaError(st, "hsma_queue_submit")
            submitted = hi
        else:
            time.sleep(min(2e-4, max(0.0, (sched_ns[submitted] - now) * 1e-9)))
        if time.time() - last_log > 2.0:
            s = q.stats()
            log(f"  t={(now - t0) * 1e-9:5.1f}s submitted {submitted} completed {s['completed'] - base_completed} "
                f"pending {s['pending']} inflight {s['inflight']} rounds {s['rounds']} "
                f"launch {s['launch_ms']:.0f} ms budget {s['bytes_in_use'] / 2**30:.1f} GiB "
                f"p50 {s['p50_ns'] * 1e-6:.1f} ms p99 {s['p99_ns'] * 1e-6:.1f} ms")
            last_log = time.time()
    t_end_submit = hs.clock_ns()
    deadline = time.time() + max(60.0, 4 * duration)
    while True:
        s = q.stats()
        if s["completed"] + s["failed"] - base_completed >= N or time.time() > deadline:
            break
        if time.time() - last_log > 2.0:
            log(f"  draining: completed {s['completed'] - base_completed} pending {s['pending']} "
                f"inflight {s['inflight']} rounds {s['rounds']} launch {s['launch_ms']:.0f} ms "
                f"budget {s['bytes_in_use'] / 2**30:.1f} GiB")
            last_log = time.time()
        time.sleep(0.01)
    s = q.stats()
    completed = s["completed"] - base_completed
    failed = s["failed"]
    span = (s["t_last_done_ns"] - t0) * 1e-9 if completed else float("nan")
    backlog_s = (s["t_last_done_ns"] - t_end_submit) * 1e-9 if completed else float("nan")
    # parity on the kept sample
    parity = None
    info = hs.RequestInfo()
    if sample and not args.no_check:
        import oracle
        worst = 0.0
        checked = 0
        for i in sorted(sample):
            r = stream[i]
            st = L.hsma_queue_poll(q._h, tickets[i], ctypes.byref(info))
            if st != 0:
                continue
            X = hs.matrix_from_pointer(info.B, r.m, r.n, r.m, r.complex_)
            Lh, Bh = W.synthetic_inputs(r.m, r.n, W.serving_key(seed, r.rid), r.complex_)
            worst = max(worst, oracle.rel_err_fro(X, oracle.solve(Lh, Bh, r.alpha)))
            checked += 1
            hs.lib().hsma_queue_release(q._h, tickets[i])
        parity = {"sampled_requests": checked, "worst_rel_err_fro": worst,
                  "ok": bool(checked == len(sample) and worst <= 1e-12)}
        log(f"parity on {checked} served requests: rel <= {worst:.2e}")
    q.close()

    def ms(x):
        return round(x * 1e-6, 3) if x else None

    def summ(d):
        return {"count": d["count"], "p50_ms": ms(d["p50_ns"]), "p99_ms": ms(d["p99_ns"]),
                "max_ms": ms(d["max_ns"]), "mean_ms": ms(d["mean_ns"])}
    solves_per_s = completed / span if completed else 0.0
    saturated = bool(backlog_s > 0.5)
    lat = summ(s["all"])
    return {
        "value": round(solves_per_s, 1), "unit": "solves/s",
        "ms_per_step": round(span * 1e3, 2), "dtype": "f64+c128",
        "pct_fp64_peak": round(100 * total_flops / span / (FP64_PEAK_TFLOPS * 1e12), 3),
        "solves_per_s": round(solves_per_s, 1),
        "serving": {"p50_ms": lat["p50_ms"], "p99_ms": lat["p99_ms"], "max_ms": lat["max_ms"],
                    "mean_ms": lat["mean_ms"], "by_size_class": {k: summ(v) for k, v in s["by_class"].items()},
                    "latency_from": "scheduled arrival to completion event",
                    "latency_window": f"arrivals after the first {warm_s:.0f} s ({lat['count']} requests)",
                    "percentile_resolution": "histogram of 64 log bins per doubling (within 0.6 %)",
                    "offered_per_s": rate, "duration_s": duration, "requests": N, "completed": completed,
                    "failed": failed, "rejected": s["rejected"], "peak_budget_bytes": s["bytes_peak"],
                    "budget_bytes": budget or 32 << 30, "saturated": saturated,
                    "drain_after_last_arrival_s": round(backlog_s, 3),
                    "gpu_max_hw_queues": HW_QUEUES,
                    "admission_rounds": s["rounds"], "scheduler_launch_ms": round(s["launch_ms"], 1),
                    "served_tflops": round(total_flops / span / 1e12, 3)},
        "extra_config": {"rate_per_s": rate, "duration_s": duration, "seed": seed,
                         "m_range": [8, 4096], "n_range": [1, 512], "p_complex": 0.3,
                         "budget_bytes": budget or 32 << 30,
                         "inputs": "generated on the device (Philox4x32-10 keyed by seed and request id)"},
        "parity": parity,
    }


def run_baselines(args, torch, hs):
    """Reference rates next to the results: the matrix-core peaks this GPU
    sustains (beside the datasheet's), a plain device copy's bandwidth, and
    the oracle on the host for the single, large and mixed workloads, on all
    threads and on one (bounded samples of the same work)."""
    import oracle
    p64, g64 = hs.mfma_peak(False)
    p32, g32 = hs.mfma_peak(True)
    out = {"fp64_mfma_tflops_measured": round(p64, 2), "fp64_probe_shader_ghz": round(g64, 3),
           "fp64_datasheet_tflops": FP64_PEAK_TFLOPS,
           "fp32_mfma_tflops_measured": round(p32, 2), "fp32_probe_shader_ghz": round(g32, 3),
           "fp32_datasheet_tflops": FP32_PEAK_TFLOPS}
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    cms = time_gpu(lambda: dst.copy_(src), 10, 2, torch)
    out["device_copy_gbs"] = round(2 * src.numel() * 8 / (cms * 1e-3) / 1e9, 1)
    out["hbm_datasheet_gbs"] = HBM_PEAK_GBS
    del src, dst
    torch.cuda.empty_cache()
    threads = oracle.num_threads()
    cpu = {}
    try:
        # single small solve: 10 calls, mean of the last 9 (the paper's method) and median
        L, B = W.problem(0, 32, 32, False)
        for t in (threads, 1):
            oracle.set_num_threads(t)
            ts = []
            for _ in range(10):
                t0 = time.perf_counter()
                oracle.solve(L, B, 1.0)
                ts.append((time.perf_counter() - t0) * 1e6)
            cpu[f"single_32_threads{t}"] = {"us_mean_last9": round(float(np.mean(ts[1:])), 2),
                                            "us_median": round(float(np.median(ts)), 2)}
        for key, cfg in (("large_real_16384", W.LARGE_REAL), ("large_complex_8192", W.LARGE_COMPLEX)):
            L, B = W.problem(cfg["seed"], cfg["m"], cfg["n"], cfg["complex_"])
            for t in (threads, 1):
                oracle.set_num_threads(t)
                cpu[f"{key}_threads{t}"] = cpu_oracle_columns(L, B, cfg["alpha"], 4.0, cfg["complex_"])
            del L, B
        L, B = W.mixed_problem(W.MIXED["m"], W.MIXED["n"], 1e3, seed=W.MIXED["seed"])
        for t in (threads, 1):
            oracle.set_num_threads(t)
            cpu[f"mixed_8192x4096_threads{t}"] = cpu_oracle_columns(L, B, 1.0, 4.0, False)
        del L, B
    finally:
        oracle.set_num_threads(threads)
    out["oracle_cpu"] = cpu
    out["host_threads"] = threads
    return out


def run_headline(args, torch, hs, names):
    """The rest of the headline metric in the same run: the large DTRSM and
    ZTRSM solves, a lone small solve, graph replay, mixed precision and the
    serving run (each failure is reported, not fatal)."""
    import copy
    out = {}
    sub = copy.copy(args)
    sub.no_cpu_baseline = True
    sub.steps, sub.warmup = 3, 1
    try:
        out["baselines"] = run_baselines(sub, torch, hs)
    except Exception as e:  # reported, not fatal
        out["baselines"] = {"error": repr(e)}
    for key in ("large_real", "large_complex", "large_real_fp32", "large_complex_fp32"):
        cfg = dict({"large_real": W.LARGE_REAL, "large_complex": W.LARGE_COMPLEX,
                    "large_real_fp32": dict(W.LARGE_REAL, fp32=True),
                    "large_complex_fp32": dict(W.LARGE_COMPLEX, fp32=True)}[key])
        sub.workload = key
        try:
            r = run_single_problem(sub, torch, hs, cfg)
            out[key] = {"workload": names[key], "gflops": r["value"], "pct_fp64_peak": r["pct_fp64_peak"],
                        "pct_of_own_peak": r["pct_of_own_peak"], "dtype": r["dtype"],
                        "ms_per_solve": r["ms_per_step"], "roofline": r.get("roofline"),
                        "rocblas": r.get("rocblas"), "parity": r.get("parity"),
                        "phases": r.get("phases")}
        except Exception as e:  # reported in the line
            out[key] = {"error": repr(e)}
        torch.cuda.empty_cache()
        hs.workspace_release()
    try:
        # A lone small solve: call latency against rocBLAS's.
        one = copy.copy(sub)
        one.workload, one.steps, one.warmup = "single", 200, 20
        r = run_single_problem(one, torch, hs, dict(W.SINGLE_SMALL))
        out["single"] = {"workload": names["single"], "ms_per_call": r["ms_per_step"],
                         "kernel_ms": r["phases"]["small"]["ms_per_step"],
                         "rocblas": r.get("rocblas"), "parity": r.get("parity")}
    except Exception as e:
        out["single"] = {"error": repr(e)}
    try:
        out["variants"] = run_variants(sub, torch, hs)
    except Exception as e:
        out["variants"] = {"error": repr(e)}
    torch.cuda.empty_cache()
    hs.workspace_release()
    try:
        out["very_small_batched"] = run_tiny(sub, torch, hs)
    except Exception as e:
        out["very_small_batched"] = {"error": repr(e)}
    try:
        # The batched shapes as real problems (the strip kernel's real form).
        rs = copy.copy(sub)
        rs.workload, rs.steps, rs.warmup, rs.count = "batched_real", 20, 5, 0
        r = run_batched(rs, torch, hs, dict(W.BATCHED_REAL))
        out["batched_real"] = {"workload": names["batched_real"], "solves_per_s": r["value"],
                               "ms_per_batch": r["ms_per_step"], "dtype": r["dtype"],
                               "avg_launch_ms": r["roofline"]["avg_launch_ms"],
                               "hbm_frac": r["roofline"]["frac"], "parity": r["parity"],
                               "rocblas": r["rocblas"]}
    except Exception as e:
        out["batched_real"] = {"error": repr(e)}
    torch.cuda.empty_cache()
    try:
        out["cholesky"] = run_cholesky(sub, torch, hs)
    except Exception as e:
        out["cholesky"] = {"error": repr(e)}
    torch.cuda.empty_cache()
    hs.workspace_release()
    try:
        out["graph"] = run_graph(sub, torch, hs)
    except Exception as e:
        out["graph"] = {"error": repr(e)}
    try:
        sub.workload = "mixed"
        r = run_mixed(sub, torch, hs, dict(W.MIXED), kappas=(1e3, 1e6))
        out["mixed"] = {"workload": "DTRSM m=8192, n=4096, kappa_inf ~1e3 and ~1e6, seed 3",
                        "rows": r["mixed"]}
    except Exception as e:
        out["mixed"] = {"error": repr(e)}
    torch.cuda.empty_cache()
    hs.workspace_release()
    try:
        sub.workload = "serving"
        r = run_serving(sub, torch, hs)
        out["serving"] = dict(r["serving"], solves_per_s=r["solves_per_s"], parity=r.get("parity"),
                              workload=f"Poisson {sub.rate:.0f} req/s for {sub.duration:.0f} s, "
                                       "m log-U[8,4096], n log-U[1,512], 30% complex, seed 4")
    except Exception as e:
        out["serving"] = {"error": repr(e)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); "
              "multi-GPU sharding (columns of B, L broadcast once) is not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2608_25469_amd as hs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    hs.lib()

    if args.calibrate_copy:
        # Plain kernels of known traffic, the references that rocprofv3's
        # FETCH_SIZE / WRITE_SIZE are scaled by: a fill (1 GiB written) and
        # an elementwise dst = src + 1 (1 GiB read, 1 GiB written; ordinary
        # vector loads, unlike the runtime's copy blit, whose FETCH_SIZE
        # reads half of what it moves).
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    names = {"large_real": "DTRSM left-lower, m=n=16384, FP64, alpha=-1, seed 2",
             "large_complex": "ZTRSM left-lower, m=n=8192, complex FP64, alpha=(-1,0), seed 2",
             "large_real_fp32": "STRSM left-lower, m=n=16384, FP32, alpha=-1, seed 2 (the DTRSM draw rounded)",
             "large_complex_fp32": "CTRSM left-lower, m=n=8192, complex FP32, alpha=(-1,0), seed 2",
             "batched": "ZTRSM batched: 10000 solves, m,n ~ U{8..64}, alpha=(1,0.5), seed 1",
             "batched_real": "DTRSM batched: 10000 solves, m,n ~ U{8..64}, alpha=0.5, seed 1",
             "single": "DTRSM left-lower, m=n=32, FP64, alpha=1, seed 0"}
    headline = None
    if args.workload == "default":
        res = run_batched(args, torch, hs, dict(W.BATCHED))
        workload = names["batched"]
        headline = run_headline(args, torch, hs, names)
    elif args.workload == "mixed":
        res = run_mixed(args, torch, hs, dict(W.MIXED))
        workload = "DTRSM mixed precision vs FP64, m=8192, n=4096, kappa_inf ~1e3..1e6, seed 3"
    elif args.workload == "serving":
        res = run_serving(args, torch, hs)
        workload = (f"TRSM serving: Poisson {args.rate:.0f} req/s for {args.duration:.0f} s, m log-U[8,4096], "
                    f"n log-U[1,512], 70% real / 30% complex, seed 4")
    elif args.workload == "tiny":
        r = run_tiny(args, torch, hs, count=args.count or 100000)
        res = {"value": r["solves_per_s"], "unit": "solves/s", "ms_per_step": r["ms_per_batch"],
               "dtype": "c128", "pct_fp64_peak": None, "extra_config": {}, "very_small_batched": r}
        workload = r["workload"]
    elif args.workload == "cholesky":
        r = run_cholesky(args, torch, hs)
        first = r["rows"][0]
        res = {"value": first["gflops"], "unit": "GFLOP/s", "ms_per_step": first["ms"], "dtype": "f64",
               "pct_fp64_peak": round(100 * first["gflops"] / (FP64_PEAK_TFLOPS * 1e3), 2),
               "extra_config": {}, "cholesky": r}
        workload = first["workload"]
    elif args.workload == "variants":
        r = run_variants(args, torch, hs, k=args.m or 8192)
        first = r["rows"][0]
        res = {"value": first["gflops"], "unit": "GFLOP/s", "ms_per_step": first["ms"], "dtype": "f64",
               "pct_fp64_peak": round(100 * first["gflops"] / (FP64_PEAK_TFLOPS * 1e3), 2),
               "extra_config": {"m": args.m or 8192}, "variants": r}
        workload = r["workload"]
    elif args.workload == "batched":
        res = run_batched(args, torch, hs, dict(W.BATCHED))
        workload = names["batched"] if not args.count else f"ZTRSM batched: {args.count} solves"
    else:
        cfg = dict({"large_real": W.LARGE_REAL, "large_complex": W.LARGE_COMPLEX,
                    "large_real_fp32": dict(W.LARGE_REAL, fp32=True),
                    "large_complex_fp32": dict(W.LARGE_COMPLEX, fp32=True),
                    "single": W.SINGLE_SMALL}[args.workload])
        if args.m:
            cfg["m"], cfg["n"] = args.m, args.n or args.m
        res = run_single_problem(args, torch, hs, cfg)
        workload = names[args.workload] if not args.m else \
            f"{'ZTRSM' if cfg['complex_'] else 'DTRSM'} left-lower m={cfg['m']} n={cfg['n']}"

    out = {
        "metric": METRIC, "value": res["value"], "unit": res["unit"], "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": res["dtype"], "data": "synthetic",
        "pct_fp64_peak": res["pct_fp64_peak"],
        "config": dict({"workload": workload, "parallelism": "single GPU",
                        "flop_convention": "real m^2 n; complex 4 m^2 n + 2 m n"}, **res["extra_config"]),
    }
    for k in ("solves_per_s", "gflops", "phases", "parity", "roofline", "rocblas", "cpu_baseline",
              "mixed", "serving", "variants", "cholesky", "very_small_batched"):
        if k in res:
            out[k] = res[k]
    if headline is not None:
        out["headline"] = headline
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
