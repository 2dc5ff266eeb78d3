"""Benchmark: Ax = b solve GFLOP/s at n = 16384, mixed precision + FP64
iterative refinement vs FP64, at normwise backward error <= 1e-14.

One step = one whole solve from A (FP64) and b resident in HBM to x (FP64)
meeting the backward-error bar: FP32 conversion of A, FP32 LU with partial
pivoting (MFMA trailing updates), and FP64 refinement (FP64 residual, FP32
triangular solves, FP64 update) until eta <= 1e-14.  The FP64 direct solve
(getrf + getrs) of the same system is timed beside it with events, with A
restored from a pristine copy between repetitions outside the timed events.

GFLOP/s counts the nominal FP64 work 2/3 n^3 + 2 n^2 nrhs for both paths.
The JSON line carries the roofline of the dominant kernel (the MFMA trailing
update: algorithmic 2 m n k flops per launch over its average launch time,
from events around each launch on its own stream during the timed steps) and
the CPU oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 16384]

Other workloads (one JSON line each; the default above is the headline):
  --workload chol      Cholesky potrf + potrs and the FP32 + FP64-refinement SPD solve, n = 16384
  --workload adjoint   differentiable solve, batch 64 x n = 2048 (forward + backward), FP64 and FP32+IR
  --workload vbatched  2000 SPD systems, n ~ U{32..1024}, nrhs 4, one persistent launch
  --workload kernels   per-kernel-class times and rates of FP64 and FP32 getrf + getrs at n = 16384
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Ax=b solve GFLOP/s at n=16384: mixed+IR vs FP64, at backward err ≤1e-14"
PEAK_TF = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "fp16": 2500.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(n_sample: int):
    """The oracle (plain C GEPP + substitutions, OpenMP) on a bounded sample."""
    import oracle
    import synth
    oracle.build()
    A, X, B = synth.uniform_system(n_sample, 1, synth.SEED_SMALL_LU)
    t = time.perf_counter()
    LU, ipiv, info = oracle.getrf(A)
    x = oracle.getrs(LU, ipiv, B[:, 0])
    dt = time.perf_counter() - t
    fl = 2.0 / 3.0 * n_sample ** 3 + 2.0 * n_sample ** 2
    return {"value": round(fl / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "getrf+getrs n=%d nrhs=1 uniform[-1,1], one run, %.1f s (a bounded sample: the "
                      "plain method at the metric's n = 16384 takes about 8 times as long)" % (n_sample, dt),
            "cpu_model": cpu_model(), "eta": oracle.eta_inf(A, x, B[:, 0])}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _events_time(fn, reps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    import numpy as np
    return float(np.median(ts)), float(min(ts)), float(max(ts))


def _line(d):
    print(json.dumps(d), flush=True)


def bench_chol(args):
    """Cholesky at n = 16384: A = M M^T / n + I with M ~ U[-1,1] (generated on the device from a seeded
    generator), potrf GFLOP/s (1/3 n^3), potrs time, and the FP32 Cholesky + FP64 refinement solve."""
    import numpy as np
    import torch
    import oracle
    import paper_1511_07174_amd as cds
    from paper_1511_07174_amd.cds import decode_results
    dev = torch.device("cuda", 0)
    n = args.n
    g = torch.Generator(device=dev).manual_seed(6)
    M = torch.rand(n, n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    A = cds.colmajor(M @ M.T / n + torch.eye(n, dtype=torch.float64, device=dev))
    del M
    b = torch.rand(n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    h = cds.handle()
    L = torch.empty_like(A)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    tc, _, _ = _events_time(lambda: L.copy_(A), 3, 1)
    t, tmin, tmax = _events_time(lambda: (L.copy_(A), h.potrf_(L, info)), args.steps, args.warmup)
    t -= tc
    x = torch.empty_like(b)
    ts, _, _ = _events_time(lambda: (x.copy_(b), h.potrs_(L, x)), args.steps, args.warmup)
    X = torch.zeros_like(b)
    Llo = torch.empty(n * n, dtype=torch.float32, device=dev)
    res = torch.zeros(cds.cds.IR_RESULT_BYTES, dtype=torch.uint8, device=dev)
    prm = cds.default_params(tol=1e-14, success_tol=1e-14, host_check=1)
    tm, _, _ = _events_time(lambda: h.posv_mixed(A, b, X, Llo, res, precision="fp32", params=prm), args.steps,
                            args.warmup)
    r = decode_results(res)[0]
    # per-class times of one FP64 potrf (events around every launch)
    from paper_1511_07174_amd.cds import OPT_KERNEL_TIMING
    h.set_option(OPT_KERNEL_TIMING, 1)
    h.kernel_timing_reset()
    L.copy_(A)
    torch.cuda.synchronize()
    h.potrf_(L, info)
    torch.cuda.synchronize()
    cls = {}
    for kc, name in (("update", "syrk"), ("panel", "potf2"), ("trsm", "trsm")):
        cnt, ms, fl, by = h.kernel_timing(kc)
        cls[name] = {"launches": cnt, "ms": round(ms, 3), "TFLOPs": round(fl / max(ms, 1e-9) / 1e9, 2)}
    h.set_option(OPT_KERNEL_TIMING, 0)
    oracle.build()
    Ah = np.asfortranarray(A.cpu().numpy())
    bh = b.cpu().numpy()
    eta64 = oracle.eta_inf(Ah, x.cpu().numpy(), bh)
    eta_mixed = oracle.eta_inf(Ah, X.cpu().numpy(), bh)
    _line({"metric": "Cholesky potrf GFLOP/s (1/3 n^3) and SPD solve times", "workload": "chol", "n": n,
           "info": int(info.item()), "potrf_ms": round(t * 1e3, 3), "potrf_gflops": round(n ** 3 / 3 / t / 1e9, 1),
           "potrf_frac_of_f64_peak": round(n ** 3 / 3 / t / 78.6e12, 4), "potrs_ms": round(ts * 1e3, 3),
           "potrs_GBps": round(8.0 * n * n / ts / 1e9, 1), "fp64_eta": eta64,
           "posv_fp32_ir_ms": round(tm * 1e3, 3), "posv_ir_iters": r.iters, "posv_eta": eta_mixed,
           "posv_converged": bool(r.converged), "classes": cls, "data": "synthetic, device generator seed 6"})


def bench_krylov(args):
    """Krylov solvers at n = 16384 (FP64): CG on A = M M^T / n + I, BiCG, BiCGSTAB and GMRES(30) on
    A = I + R / (2 sqrt(n)), R ~ U[-1, 1]; b ~ U[-1, 1]; tol 1e-10.  Time to solution, iterations, and the
    HBM rate of the products with A (8 n^2 bytes each), against the 8 TB/s peak."""
    import numpy as np
    import torch
    import paper_1511_07174_amd as cds
    from paper_1511_07174_amd.cds import OPT_KERNEL_TIMING
    dev = torch.device("cuda", 0)
    n = args.n
    g = torch.Generator(device=dev).manual_seed(50)
    M = torch.rand(n, n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    S = cds.colmajor(M @ M.T / n + torch.eye(n, dtype=torch.float64, device=dev))
    G = cds.colmajor(torch.eye(n, dtype=torch.float64, device=dev) + M / (2.0 * n ** 0.5))
    del M
    b = torch.rand(n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    h = cds.handle()
    out = {}
    for method in ("cg", "bicg", "bicgstab", "gmres"):
        A = S if method == "cg" else G
        prm = cds.cds.krylov_params(tol=1e-10, max_iter=500, restart=30, check_every=10)
        x = torch.zeros_like(b)
        res = torch.zeros(cds.cds.KRYLOV_RESULT_BYTES, dtype=torch.uint8, device=dev)

        def run():
            x.zero_()
            h.krylov(method, A, b, x, res, prm)
        t, tmin, tmax = _events_time(run, args.steps, args.warmup)
        r = cds.cds.decode_krylov(res)
        h.set_option(OPT_KERNEL_TIMING, 1)
        h.kernel_timing_reset()
        run()
        torch.cuda.synchronize()
        cnt, ms, fl, by = h.kernel_timing("krylov_gemv")
        h.set_option(OPT_KERNEL_TIMING, 0)
        true = float(torch.linalg.vector_norm(b - A @ x) / torch.linalg.vector_norm(b))
        avg = ms / max(cnt, 1)
        out[method] = {"ms": round(t * 1e3, 3), "iters": r.iters, "converged": r.converged, "relres": r.relres,
                       "true_relres": true, "products": cnt, "product_avg_us": round(avg * 1e3, 1),
                       "product_GBps": round(8.0 * n * n / (avg * 1e-3) / 1e9, 1),
                       "product_frac_of_hbm": round(8.0 * n * n / (avg * 1e-3) / 8e12, 4)}
        log("%s: %.2f ms, %d iterations, product %.1f us (%.0f GB/s)" % (method, t * 1e3, r.iters, avg * 1e3,
                                                                       8.0 * n * n / (avg * 1e-3) / 1e9))
    _line({"metric": "Krylov solve time and product bandwidth", "workload": "krylov", "n": n, "tol": 1e-10,
           "methods": out, "data": "synthetic, device generator seed 50"})


def bench_householder(args):
    """Mixed precision + FP64 refinement on A = H1 diag(sigma) H2 (4 + 4 Householder reflectors, sigma
    geometric from 1 to 1/kappa), x_true ~ U[-1, 1], b = A x_true: n in {8192, 16384, 32768} x kappa in
    {1e2, 1e4, 1e6} x factorization in {FP32, BF16, FP16}.  Per case: time to solution, refinement steps,
    eta (double-double residual on the host), forward error against the closed-form solution, fallback.
    Where classical refinement stops without reaching eta <= 1e-14, GMRES-based refinement is run too."""
    import numpy as np
    import torch
    import oracle
    import synth
    import paper_1511_07174_amd as cds
    from paper_1511_07174_amd.cds import decode_results
    dev = torch.device("cuda", 0)
    oracle.build()
    sizes = [int(v) for v in args.sizes.split(",")]
    for n in sizes:
        for kappa in (1e2, 1e4, 1e6):
            seed = synth.householder_seed(n, kappa)
            rg = synth.rng(seed)
            vl = [rg.standard_normal(n) for _ in range(4)]
            vr = [rg.standard_normal(n) for _ in range(4)]
            sigma = float(kappa) ** (-np.arange(n, dtype=np.float64) / max(1, n - 1))
            # the construction of synth.householder_system, on the device
            A = torch.eye(n, dtype=torch.float64, device=dev)
            for v in vr:
                vt = torch.from_numpy(v).to(dev)
                w = A @ vt
                A -= torch.outer(w, (2.0 / float(v @ v)) * vt)
            A *= torch.from_numpy(sigma).to(dev)[:, None]
            for v in reversed(vl):
                vt = torch.from_numpy(v).to(dev)
                w = vt @ A
                A -= torch.outer((2.0 / float(v @ v)) * vt, w)
            A = cds.colmajor(A)
            xt = torch.from_numpy(rg.uniform(-1.0, 1.0, n)).to(dev)
            b = A @ xt
            bh = b.cpu().numpy()
            xs = oracle.householder_solve(vl, vr, sigma, bh)
            Ah = np.asfortranarray(A.cpu().numpy()) if n <= 16384 else None
            for prec in ("fp32", "bf16", "fp16"):
                prm = cds.default_params(tol=1e-14, success_tol=1e-14, host_check=1)
                X = torch.zeros_like(b)
                LUlo = torch.empty(n * n, dtype=torch.float32, device=dev)
                ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
                res = torch.zeros(cds.cds.IR_RESULT_BYTES, dtype=torch.uint8, device=dev)
                h = cds.handle()
                t, _, _ = _events_time(lambda: h.gesv_mixed(A, b, X, LUlo, ipiv, res, precision=prec, params=prm),
                                       1, 1)
                r = decode_results(res)[0]
                x = X.cpu().numpy()
                line = {"metric": "mixed-precision solve on a Householder matrix", "workload": "householder",
                        "n": n, "kappa": kappa, "precision": prec, "seed": seed, "ms": round(t * 1e3, 3),
                        "gflops": round((2.0 / 3.0 * n ** 3 + 2.0 * n * n) / t / 1e9, 1),
                        "ir_iters": r.iters, "stop_reason": r.stop_reason, "converged": bool(r.converged),
                        "eta_gpu": r.eta, "fell_back": bool(r.fell_back),
                        "fwd_err": float(np.max(np.abs(x - xs)) / np.max(np.abs(x)))}
                if Ah is not None:
                    line["eta_oracle"] = oracle.eta_inf(Ah, x, bh)
                if not r.converged:
                    res2 = torch.zeros(cds.cds.IR_RESULT_BYTES, dtype=torch.uint8, device=dev)
                    X2 = torch.zeros_like(b)
                    t2, _, _ = _events_time(lambda: h.gesv_gmres_ir(A, b, X2, LUlo, ipiv, res2, precision=prec,
                                                                     params=prm), 1, 1)
                    r2 = decode_results(res2)[0]
                    x2 = X2.cpu().numpy()
                    inner = int(res2.cpu()[36:40].view(torch.int32).item())
                    line["gmres_ir"] = {"ms": round(t2 * 1e3, 3), "corrections": r2.iters, "gmres_iters": inner,
                                        "converged": bool(r2.converged), "eta_gpu": r2.eta,
                                        "fwd_err": float(np.max(np.abs(x2 - xs)) / np.max(np.abs(x2)))}
                    if Ah is not None:
                        line["gmres_ir"]["eta_oracle"] = oracle.eta_inf(Ah, x2, bh)
                _line(line)
                del LUlo
            del A, Ah
            torch.cuda.empty_cache()


def bench_adjoint(args):
    """Batched differentiable solve: 64 systems of n = 2048, A, b, w ~ U[-1,1]; loss = sum(w x); forward
    (batched getrf + getrs, or FP32 + FP64 refinement) and backward (A^-T w, -bbar x^T) timed apart."""
    import torch
    import paper_1511_07174_amd as cds
    dev = torch.device("cuda", 0)
    batch, n = 64, 2048
    g = torch.Generator(device=dev).manual_seed(20)
    A0 = torch.rand(batch, n, n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    b0 = torch.rand(batch, n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    w = torch.rand(batch, n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    out = {"metric": "batched differentiable solve, forward and backward ms", "workload": "adjoint",
           "batch": batch, "n": n, "data": "synthetic, device generator seed 20"}
    for prec in ("fp64", "fp32"):
        A = A0.clone().requires_grad_(True)
        b = b0.clone().requires_grad_(True)
        state = {}

        def fwd():
            state["x"] = cds.solve_ad(A, b, prec)

        def bwd():
            A.grad = None
            b.grad = None
            (state["x"] * w).sum().backward()
        tf, _, _ = _events_time(fwd, args.steps, args.warmup)
        fwd()
        torch.cuda.synchronize()
        tb, _, _ = _events_time(lambda: (fwd(), bwd()), args.steps, args.warmup)
        tb -= tf
        out[prec] = {"forward_ms": round(tf * 1e3, 3), "backward_ms": round(tb * 1e3, 3),
                     "forward_gflops": round(batch * 2.0 / 3.0 * n ** 3 / tf / 1e9, 1),
                     "backward_GBps": round(batch * (8.0 * n * n * 2) / tb / 1e9, 1)}
        del A, b
    _line(out)


def bench_vbatched(args):
    """2000 SPD systems, n ~ U{32..1024}, A_i = M M^T / n + I, B_i ~ U[-1,1] n x 4: FP32 Cholesky +
    FP64 refinement to eta <= 1e-14 in one persistent launch, largest systems first.  The descriptors (sizes, pointers,
    leading dimensions) are built once; the timed step is the replay of a graph holding the counter
    reset and the persistent launch.  systems/s and the per-system latency (device timestamps,
    100 MHz) p50 / p99."""
    import numpy as np
    import torch
    import paper_1511_07174_amd as cds
    from paper_1511_07174_amd.cds import IR_RESULT_BYTES, decode_results
    dev = torch.device("cuda", 0)
    count = 2000
    rng = np.random.default_rng(30)
    sizes = rng.integers(32, 1025, size=count)
    g = torch.Generator(device=dev).manual_seed(30)
    systems = []
    for ni in sizes:
        ni = int(ni)
        M = torch.rand(ni, ni, generator=g, dtype=torch.float64, device=dev) * 2 - 1
        A = cds.colmajor(M @ M.T / ni + torch.eye(ni, dtype=torch.float64, device=dev))
        B = cds.colmajor(torch.rand(ni, 4, generator=g, dtype=torch.float64, device=dev) * 2 - 1)
        systems.append((A, B))
    order = torch.as_tensor(np.argsort(-sizes, kind="stable"), dtype=torch.int32, device=dev)
    ns = torch.tensor([a.shape[0] for a, _ in systems], dtype=torch.int32, device=dev)
    Ap = torch.tensor([a.data_ptr() for a, _ in systems], dtype=torch.int64, device=dev)
    lda = torch.tensor([a.stride(1) for a, _ in systems], dtype=torch.int64, device=dev)
    Bp = torch.tensor([b.data_ptr() for _, b in systems], dtype=torch.int64, device=dev)
    ldb = torch.tensor([b.stride(1) for _, b in systems], dtype=torch.int64, device=dev)
    Xs = [cds.colmajor(torch.zeros_like(b)) for _, b in systems]
    Xp = torch.tensor([x.data_ptr() for x in Xs], dtype=torch.int64, device=dev)
    ldx = torch.tensor([x.stride(1) for x in Xs], dtype=torch.int64, device=dev)
    res = torch.zeros(count * IR_RESULT_BYTES, dtype=torch.uint8, device=dev)
    t0 = torch.zeros(count, dtype=torch.int64, device=dev)
    t1 = torch.zeros(count, dtype=torch.int64, device=dev)
    h = cds.handle()
    nmax = int(sizes.max())
    prm = cds.default_params(tol=1e-14, success_tol=1e-14)

    def call():
        h.posv_mixed_vbatched(count, nmax, ns, Ap, lda, Bp, ldb, Xp, ldx, 4, res, order=order, t_start=t0,
                              t_end=t1, params=prm, device=dev)
    te, _, _ = _events_time(call, args.steps, args.warmup)        # eager (also sizes the workspace)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    t, tmin, tmax = _events_time(graph.replay, args.steps, args.warmup)
    lat = (t1.cpu().numpy() - t0.cpu().numpy()) * 10e-9
    R = decode_results(res)
    conv = sum(1 for r in R if r.converged)
    flops = float(np.sum(sizes.astype(np.float64) ** 3 / 3.0))
    _line({"metric": "batched uneven SPD systems/s", "workload": "vbatched", "systems": count,
           "value": round(count / t, 1), "unit": "systems/s", "ms": round(t * 1e3, 3),
           "ms_min": round(tmin * 1e3, 3), "ms_max": round(tmax * 1e3, 3), "eager_launch_ms": round(te * 1e3, 3),
           "latency_p50_us": round(float(np.percentile(lat, 50)) * 1e6, 1),
           "latency_p99_us": round(float(np.percentile(lat, 99)) * 1e6, 1),
           "factor_gflops": round(flops / t / 1e9, 1), "converged": conv,
           "max_iters": max(r.iters for r in R), "max_eta": max(r.eta for r in R), "tol": prm.tol,
           "data": "synthetic, sizes numpy seed 30, matrices device generator seed 30; timed: graph replay"})


def bench_kernels(args):
    """Per-kernel-class times of getrf + getrs at n = 16384 (FP64 and FP32), from events around every
    launch on the stream it runs on, with each class's algorithmic rate."""
    import torch
    import paper_1511_07174_amd as cds
    from paper_1511_07174_amd.cds import OPT_KERNEL_TIMING
    dev = torch.device("cuda", 0)
    n = args.n
    g = torch.Generator(device=dev).manual_seed(3)
    A = cds.colmajor(torch.rand(n, n, generator=g, dtype=torch.float64, device=dev) * 2 - 1)
    b = torch.rand(n, generator=g, dtype=torch.float64, device=dev) * 2 - 1
    h = cds.handle()
    out = {"metric": "kernel classes of getrf + getrs", "workload": "kernels", "n": n}
    for dt, src in (("fp64", A), ("fp32", A.float())):
        LU = src.clone()
        ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        x = b.to(src.dtype)
        tc, _, _ = _events_time(lambda: LU.copy_(src), 3, 1)
        t, _, _ = _events_time(lambda: (LU.copy_(src), h.getrf_(LU, ipiv, info)), args.steps, args.warmup)
        t -= tc
        ts, _, _ = _events_time(lambda: h.getrs_(LU, ipiv, x.clone()), args.steps, args.warmup)
        h.set_option(OPT_KERNEL_TIMING, 1)
        h.kernel_timing_reset()
        LU.copy_(src)
        torch.cuda.synchronize()
        h.getrf_(LU, ipiv, info)
        h.getrs_(LU, ipiv, x.clone())
        torch.cuda.synchronize()
        cls = {}
        for kc in ("update", "panel", "laswp", "trsm", "trsv"):
            cnt, ms, fl, by = h.kernel_timing(kc)
            cls[kc] = {"launches": cnt, "ms": round(ms, 3), "TFLOPs": round(fl / max(ms, 1e-9) / 1e9, 2),
                       "GBps": round(by / max(ms, 1e-9) / 1e6, 1)}
        h.set_option(OPT_KERNEL_TIMING, 0)
        out[dt] = {"getrf_ms": round(t * 1e3, 3), "getrf_tflops": round(2.0 / 3.0 * n ** 3 / t / 1e12, 2),
                   "getrs_ms": round(ts * 1e3, 3), "info": int(info.item()), "classes": cls}
    _line(out)


def bench_copy(args):
    """A plain 1 GiB device-to-device copy (reads 1 GiB, writes 1 GiB): the HBM reference for the
    rooflines, and the kernel whose FETCH_SIZE / WRITE_SIZE counters calibrate the traffic figures."""
    import torch
    dev = torch.device("cuda", 0)
    x = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    y = torch.empty_like(x)
    t, tmin, _ = _events_time(lambda: y.copy_(x), args.steps, args.warmup)
    nbytes = 2.0 * x.numel() * 4
    _line({"metric": "device copy GB/s (read + write)", "workload": "copy", "bytes": nbytes,
           "ms": round(t * 1e3, 3), "GBps": round(nbytes / t / 1e9, 1), "GBps_best": round(nbytes / tmin / 1e9, 1)})


def traffic_for(kernel_key):
    """HBM bytes per launch of a kernel from the committed counter summary (profiles/traffic.json),
    or None when the kernel's source changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "traffic.json")
    try:
        with open(path) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    e = tab.get(kernel_key)
    if not e:
        return None
    with open(os.path.join(here, e["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != e["source_sha256"]:
            return None
    return e["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--cpu-n", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--workload", default="lu",
                    choices=["lu", "chol", "adjoint", "vbatched", "kernels", "copy", "krylov", "householder"])
    ap.add_argument("--sizes", default="8192,16384,32768", help="householder workload: matrix sizes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the factorization of one "
              "matrix runs on a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload != "lu":
        {"chol": bench_chol, "adjoint": bench_adjoint, "vbatched": bench_vbatched,
         "kernels": bench_kernels, "copy": bench_copy, "krylov": bench_krylov,
         "householder": bench_householder}[args.workload](args)
        return

    import numpy as np
    import torch
    import synth
    import paper_1511_07174_amd as cds
    from paper_1511_07174_amd.cds import OPT_KERNEL_TIMING, decode_results

    dev = torch.device("cuda", 0)
    n, nrhs = args.n, 1
    seed = synth.SEED_LU.get(n, 3)
    log("generating the n=%d system (uniform[-1,1], seed %d)" % (n, seed))
    A_h, X_h, B_h = synth.uniform_system(n, nrhs, seed)
    A = torch.from_numpy(A_h).to(dev)          # column-major (Fortran order keeps strides (1, n))
    A = cds.colmajor(A) if A.stride(0) != 1 else A
    b = torch.from_numpy(np.ascontiguousarray(B_h[:, 0])).to(dev)
    del A_h
    h = cds.handle()
    nominal = 2.0 / 3.0 * n ** 3 + 2.0 * n * n * nrhs

    # ---------------------------------------------------------------- mixed precision + IR (the value)
    X = torch.zeros(n, dtype=torch.float64, device=dev)
    LUlo = torch.empty(n * n, dtype=torch.float32, device=dev)
    ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
    res = torch.zeros(cds.cds.IR_RESULT_BYTES, dtype=torch.uint8, device=dev)
    prm = cds.default_params(tol=1e-14, success_tol=1e-14, host_check=1)

    def mixed_step():
        h.gesv_mixed(A, b, X, LUlo, ipiv, res, precision=args.precision, params=prm)

    for _ in range(args.warmup):
        mixed_step()
    torch.cuda.synchronize()
    # the timed region: the K steps alone, no per-kernel events
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mixed_step()
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    r = decode_results(res)[0]
    # the same K steps again with HIP events around every launch on the stream it runs on (the
    # library's kernel timer), for the roofline of the trailing update and the panel time
    h.set_option(OPT_KERNEL_TIMING, 1)
    h.kernel_timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mixed_step()
    torch.cuda.synchronize()
    t_instr = (time.perf_counter() - t0) / args.steps
    upd = h.kernel_timing("update")
    pan = h.kernel_timing("panel")
    h.set_option(OPT_KERNEL_TIMING, 0)
    log("mixed %s+IR: %.2f ms/step, iters %d, eta %.2e, converged %s" % (args.precision, t_mixed * 1e3, r.iters,
                                                                       r.eta, r.converged))

    # ---------------------------------------------------------------- FP64 getrf + getrs (comparison)
    fp64 = None
    if not args.no_fp64:
        LU = torch.empty_like(A)
        ip = torch.zeros(n, dtype=torch.int32, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        xb = torch.empty_like(b)
        e0, em, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        times, tf = [], []
        for it in range(args.warmup + min(args.steps, 3)):
            LU.copy_(A)
            xb.copy_(b)
            e0.record()
            h.getrf_(LU, ip, info)
            em.record()
            h.getrs_(LU, ip, xb)
            e1.record()
            torch.cuda.synchronize()
            if it >= args.warmup:
                times.append(e0.elapsed_time(e1) * 1e-3)
                tf.append(e0.elapsed_time(em) * 1e-3)
        t64 = float(np.median(times))
        tgetrf = float(np.median(tf))
        import oracle
        oracle.build()
        eta64 = oracle.eta_inf(np.asfortranarray(A.cpu().numpy()), xb.cpu().numpy(), B_h[:, 0])
        fp64 = {"ms": round(t64 * 1e3, 3), "gflops": round(nominal / t64 / 1e9, 1), "eta": eta64,
                "valid": bool(eta64 <= 1e-14), "info": int(info.item()), "getrf_ms": round(tgetrf * 1e3, 3),
                "getrf_frac_of_f64_peak": round(2.0 / 3.0 * n ** 3 / tgetrf / 78.6e12, 4)}
        log("fp64 getrf+getrs: %.2f ms, eta %.2e" % (t64 * 1e3, eta64))

    # independent check of the mixed solution's backward error (double-double residual on the host)
    import oracle
    eta_host = oracle.eta_inf(np.asfortranarray(A.cpu().numpy()), X.cpu().numpy(), B_h[:, 0])
    valid = bool(r.converged) and eta_host <= 1e-14

    cpu = None
    if not args.no_cpu:
        log("cpu oracle baseline on n=%d" % args.cpu_n)
        cpu = cpu_baseline(args.cpu_n)

    cnt, ms, fl, by = upd
    upd_avg_ms = ms / cnt if cnt else float("nan")
    achieved = (fl / cnt) / (upd_avg_ms * 1e-3) / 1e12 if cnt else None
    peak = PEAK_TF["f32" if args.precision == "fp32" else args.precision]
    out = {
        "metric": METRIC,
        "value": round(nominal / t_mixed / 1e9, 1) if valid else 0.0,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 3),
        "ms_per_step_instrumented": round(t_instr * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32" else args.precision + "+f32+f64",
        "data": "synthetic",
        "config": {"workload": "dense Ax=b, n=%d, nrhs=1, A uniform[-1,1] i.i.d. (seed %d), b = A x_true; "
                               "%s LU with partial pivoting + FP64 iterative refinement to eta<=1e-14, "
                               "vs FP64 getrf+getrs" % (n, seed, args.precision.upper()),
                   "n": n, "nrhs": nrhs, "precision": args.precision},
        "valid": valid,
        "eta": eta_host,
        "ir_iters": r.iters,
        "fp64": fp64,
        "speedup_vs_fp64": round(fp64["ms"] / (t_mixed * 1e3), 3) if fp64 else None,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2) if achieved else None, "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4) if achieved else None,
                     "traffic": traffic_for("update_%s_n%d" % (args.precision, n)),
                     "kernel": "trailing update (%s MFMA), %d launches/step, avg %.1f us" %
                               (args.precision, cnt // max(1, args.steps), upd_avg_ms * 1e3)},
        "panel": {"launches_per_step": pan[0] // max(1, args.steps),
                  "ms_per_step": round(pan[1] / max(1, args.steps), 3)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
