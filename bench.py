#!/usr/bin/env python3
"""Benchmark of the multilevel QR path on one MI355X.

Headline: CAQR FP64 GFLOP/s on an 8192 x 8192 N(0,1) matrix (seed 2), panel
width 64, leaf rows 256, arity-4 tree per panel (one 256-row leaf per
workgroup, then the device-wide levels), flops counted as LAPACK's 4 n^3 / 3.  One step = one factorization
(every panel: leaf QR, reduction tree, trailing update).  A is restored from a
pristine device copy before each step, outside the event-timed factorization.

Also reported: the live rooflines of the panel kernel and of the trailing
update (from HIP events the library records around each launch on the stream
it runs on), the dominant one as `roofline`; the oracle's CPU rate on the
headline workload; and secondary lines (TSQR, batched, least squares, mixed
precision, served stream).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector and MFMA)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E


def update_flops(rows: int, cols: int, b: int, leaves: int) -> float:
    """Algorithmic flops of one Q^T update launch of a panel (rows x b reflectors,
    `leaves` leaves) on `cols` columns: per leaf W = Y^T C and C -= Y W (4 rows b
    per column) plus T^T W (b^2 per column); per tree node V^T C2, T^T W and V W
    on b x b triangles (3 b^2 per column)."""
    return cols * (4.0 * rows * b + leaves * b * b + 3.0 * (leaves - 1) * b * b)


UPDATE_SOURCES = ("update.hip", "staging.hpp", "kernels.hpp", "device_common.hpp")
PANEL_SOURCES = ("panel_body.hpp", "panel_a4.hip", "kernels.hpp", "device_common.hpp")
TRAFFIC_PROFILES = {
    "update": (os.path.join(ROOT, "profiles", "caqr_8192_update_traffic.md"), UPDATE_SOURCES),
    "panel": (os.path.join(ROOT, "profiles", "caqr_8192_panel_traffic.md"), PANEL_SOURCES),
}


def traffic_per_call(which):
    """Measured HBM bytes per call of a kernel (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, scaled by the same counters on a plain copy), from the
    committed profile summary; None when the kernel's sources changed since it
    was taken (their hash is recorded with the figure)."""
    import hashlib
    import re

    path, sources = TRAFFIC_PROFILES[which]
    try:
        text = open(path).read()
    except OSError:
        return None
    m_b = re.search(r"traffic_bytes_per_call: (\d+)", text)
    m_h = re.search(r"sources_sha256: ([0-9a-f]+)", text)
    if not (m_b and m_h):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1303_5837_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m_b.group(1)) if h.hexdigest() == m_h.group(1) else None


def sources_sha256(which):
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_PROFILES[which][1]:
        with open(os.path.join(ROOT, "paper_1303_5837_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def panel_flops(rows, b, h=256):
    """Flops of one panel factorization (leaf QRs and stacked eliminations)."""
    L = -(-rows // h)
    total = 0.0
    for i in range(L):
        hi = max(min(h, rows - i * h), b)
        total += 2.0 * hi * b * b - 2.0 * b ** 3 / 3.0
    return total + (L - 1) * 2.0 * b ** 3 / 3.0


def executed_flops(m: int, n: int, nb: int, h: int = 256) -> float:
    """Flops the CAQR factorization executes (the LAPACK count 4n^3/3 of a square
    matrix omits the tree's redundant work): per panel s (rows m_s, width b,
    L = ceil(m_s / h) leaves) the leaf QRs (2 h_i b^2 - 2b^3/3 each, h_i the
    leaf's rows, at least b), L - 1 stacked eliminations (2b^3/3 each) and the
    update of the n_t columns right of it (update_flops); T formation is not
    counted."""
    total = 0.0
    for c0 in range(0, n, nb):
        ms, b = m - c0, min(nb, n - c0)
        L = -(-ms // h)
        for i in range(L):
            hi = max(min(h, ms - i * h), b)
            total += 2.0 * hi * b * b - 2.0 * b ** 3 / 3.0
        total += (L - 1) * 2.0 * b ** 3 / 3.0
        nt = n - c0 - b
        if nt > 0:
            total += update_flops(ms, nt, b, L)
    return total


def panel_bytes(rows: int, b: int) -> float:
    """Algorithmic HBM bytes of one panel factorization: read A, write Y/R."""
    return 16.0 * rows * b


def batched_line(dtype_name: str):
    """The uneven 2000-problem batch in one element type (float: the double draws
    rounded), tuned first; median of 10 timed tsqr_factor_batched calls."""
    import numpy as np
    import torch

    from paper_1303_5837_amd import caqr, inputs

    dtype = {"f64": torch.float64, "f32": torch.float32}[dtype_name]
    ms, ns = inputs.batched_tsqr_sizes()
    seed = inputs.SEEDS["batched_tsqr"]
    P = [inputs.gaussian_device(int(m), int(n), seed * 100003 + i).to(dtype) for i, (m, n) in enumerate(zip(ms, ns))]
    P = [a.t().contiguous().t() for a in P]
    W = [torch.empty_like(a.t()).t() for a in P]
    t_tune = time.perf_counter()
    caqr.tune_batched(dtype=dtype)
    t_tune = time.perf_counter() - t_tune
    times = []
    for it in range(3 + 10):
        for w, a in zip(W, P):
            w.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        Bt = caqr.tsqr_batched(W)
        e1.record()
        torch.cuda.synchronize()
        if it >= 3:
            times.append(e0.elapsed_time(e1))
        Bt.close()
    t = float(np.median(times))
    es = 8 if dtype == torch.float64 else 4
    alg = float(sum(2.0 * es * int(m) * int(n) for m, n in zip(ms, ns)))  # read A, write R and Y
    flops = float(sum(2.0 * int(m) * int(n) ** 2 - 2.0 * int(n) ** 3 / 3 for m, n in zip(ms, ns)))
    plans = {}
    for m, n in zip(ms, ns):
        k = "h%d/lpw%d/k%d" % caqr.batch_plan_for(int(m), int(n), dtype=dtype)
        plans[k] = plans.get(k, 0) + 1
    del P, W
    torch.cuda.empty_cache()
    return {
        "dtype": dtype_name,
        "median_ms": round(t, 4), "p10_ms": round(float(np.percentile(times, 10)), 4),
        "p90_ms": round(float(np.percentile(times, 90)), 4),
        "matrices_per_s": round(len(ms) / (t * 1e-3), 1), "gflops": round(flops / (t * 1e-3) / 1e9, 1),
        "algorithmic_GBps": round(alg / (t * 1e-3) / 1e9, 1),
        "pct_hbm_peak": round(100 * alg / (t * 1e-3) / 1e9 / PEAK_HBM_GBS, 2),
        "bytes": alg, "tune_s": round(t_tune, 2), "plans": plans,
        "timed": "one tsqr_factor_batched call incl. planning and table upload (HIP events)"}


def batched_ls_line(reps=5, eta_sample=8):
    """Batched least squares over the uneven batch's shapes (2000 problems, m
    log-uniform in [256, 65536], n in {8, 16, 32, 64}, one right-hand side):
    median of `reps` ls_solve_batched calls (synchronous; planning, factorization,
    Q^T b and back substitution), against the same problems solved one
    ls_solve call at a time (once)."""
    import numpy as np
    import torch

    from paper_1303_5837_amd import caqr, inputs

    ms, ns = inputs.batched_tsqr_sizes()
    seed = inputs.SEEDS["batched_tsqr"]
    P = [inputs.gaussian_device(int(m), int(n), seed * 100003 + i) for i, (m, n) in enumerate(zip(ms, ns))]
    Q = [inputs.gaussian_device(int(m), 1, seed * 100003 + 500000 + i) for i, m in enumerate(ms)]
    WA = [torch.empty_like(a.t()).t() for a in P]
    WB = [torch.empty_like(b.t()).t() for b in Q]

    def restore():
        for w, a in zip(WA, P):
            w.copy_(a)
        for w, b in zip(WB, Q):
            w.copy_(b)
        torch.cuda.synchronize()

    caqr.tune_batched()
    times = []
    for it in range(1 + reps):
        restore()
        t0 = time.perf_counter()
        _, info = caqr.ls_solve_batched(WA, WB)
        t = time.perf_counter() - t0
        if it >= 1:
            times.append(t)
    ok = sum(1 for st in info if st[0] == 0)

    def eta(A, x, b):
        v = torch.ones(A.shape[1], 1, dtype=torch.float64, device=A.device)
        for _ in range(30):
            v = A.t() @ (A @ v)
            v = v / torch.linalg.norm(v)
        na = float(torch.linalg.norm(A @ v))
        r = b - A @ x
        return float(torch.linalg.norm(A.t() @ r)) / (na * (na * float(torch.linalg.norm(x)) + float(torch.linalg.norm(b))))

    etas = [eta(P[i], WB[i][: P[i].shape[1]], Q[i]) for i in range(0, len(P), len(P) // eta_sample)]
    restore()
    t0 = time.perf_counter()
    for a, b in zip(WA, WB):
        caqr.ls_solve(a, b)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t = float(np.median(times))
    flops = float(sum(2.0 * int(m) * int(n) ** 2 - 2.0 * int(n) ** 3 / 3 for m, n in zip(ms, ns)))
    del P, Q, WA, WB
    torch.cuda.empty_cache()
    return {"problems": len(ms), "median_ms": round(t * 1e3, 3), "solves_per_s": round(len(ms) / t, 1),
            "qr_gflops": round(flops / t / 1e9, 1), "status_ok": ok,
            "eta_sample_max": max(etas), "plain_ms": round(t_plain * 1e3, 2),
            "plain_solves_per_s": round(len(ms) / t_plain, 1), "speedup_vs_plain": round(t_plain / t, 2),
            "timed": "one ls_solve_batched call (host wall clock; it waits for the device) vs one ls_solve per problem"}


def served_lines(rates=(200, 500, 1000, 2000), duration=2.0, workers=8, pool=512, budget=64 << 30,
                 eta_sample=8, plain=True):
    """Served least-squares stream: Poisson arrivals at each rate for `duration`
    seconds over a cached pool of problems (m log-uniform in [1024, 262144], n
    in [16, 512], kappa in [1e2, 1e6]); latency = completion - scheduled
    arrival.  The same stream through one worker is the plain (one solve at a
    time) reference.  A rate is skipped for a configuration once a lower rate
    left it overloaded (p99 above 5 s)."""
    import threading

    import numpy as np
    import torch

    from paper_1303_5837_amd import caqr, inputs

    seed = inputs.SEEDS["served_ls"]
    ms, ns, ks = inputs.served_ls_requests(pool)
    t_pool = time.perf_counter()
    P = [(inputs.conditioned_device(int(m), int(n), float(k), seed * 1000003 + i),
          inputs.gaussian_device(int(m), 1, seed * 1000003 + 500000 + i)) for i, (m, n, k) in enumerate(zip(ms, ns, ks))]
    torch.cuda.synchronize()
    t_pool = time.perf_counter() - t_pool
    flops = np.array([2.0 * m * n * n - 2.0 * n ** 3 / 3 for m, n in zip(ms, ns)])

    def eta(A, x, b):
        v = torch.ones(A.shape[1], 1, dtype=torch.float64, device=A.device)
        for _ in range(30):  # power iteration for ||A||_2
            v = A.t() @ (A @ v)
            v = v / torch.linalg.norm(v)
        na = float(torch.linalg.norm(A @ v))
        r = b - A @ x
        return float(torch.linalg.norm(A.t() @ r)) / (na * (na * float(torch.linalg.norm(x)) + float(torch.linalg.norm(b))))

    out = {"pool": pool, "pool_build_s": round(t_pool, 1), "duration_s": duration, "budget_bytes": budget,
           "request_gflop_mean": round(float(flops.mean()) / 1e9, 3)}
    for label, w in (("served", workers), ("plain", 1)) if plain else (("served", workers),):
        S = caqr.Server(workers=w, budget_bytes=budget)
        for i in range(2 * w):  # first use of every worker's handle
            A, B = P[i % pool]
            X = torch.empty((1, A.shape[1]), dtype=torch.float64, device="cuda").t()
            S.wait(S.submit(A, B, X))
        per = {}
        overloaded = False
        for rate in rates:
            if overloaded:
                per[str(rate)] = "skipped (overloaded at a lower rate)"
                continue
            arr = inputs.poisson_arrivals(float(rate), duration, seed * 7919 + rate)
            pick = np.random.default_rng(seed * 31 + rate).integers(0, pool, len(arr))
            tickets = [None] * len(arr)
            ends = np.zeros(len(arr), dtype=np.int64)
            status = np.zeros(len(arr), dtype=np.int64)
            keep = {}
            ready = threading.Semaphore(0)

            def waiter():
                for j in range(len(arr)):
                    ready.acquire()
                    st, _, _, _, end = S.wait(tickets[j])
                    ends[j], status[j] = end, st

            th = threading.Thread(target=waiter)
            th.start()
            t0 = time.monotonic_ns()
            for j, (ta, pi) in enumerate(zip(arr, pick)):
                target = t0 + int(ta * 1e9)
                while True:
                    dt = (target - time.monotonic_ns()) / 1e9
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 0.002))
                A, B = P[pi]
                X = torch.empty((1, A.shape[1]), dtype=torch.float64, device="cuda").t()
                tickets[j] = S.submit(A, B, X)
                if j < eta_sample:
                    keep[j] = X
                ready.release()
            th.join()
            lat = (ends - (t0 + (arr * 1e9).astype(np.int64))) / 1e6
            span = (ends.max() - t0) / 1e9
            etas = [eta(P[pick[j]][0], keep[j], P[pick[j]][1]) for j in keep]
            per[str(rate)] = {
                "requests": int(len(arr)), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "max_ms": round(float(lat.max()), 3),
                "solves_per_s": round(len(arr) / span, 1),
                "sustained_gflops": round(float(flops[pick].sum()) / span / 1e9, 1),
                "status_ok": int((status == 0).sum()),
                "eta_sample_max": float(max(etas)) if etas else None,
                "eta_sample_le_1e-12": float(np.mean([e <= 1e-12 for e in etas])) if etas else None}
            overloaded = per[str(rate)]["p99_ms"] > 5000.0
        S.close()
        out[label] = {"workers": w, "rates": per}
    del P
    torch.cuda.empty_cache()
    return out


def inner_block_line(dev, n, reps=3):
    """The per-level block size variant (leaves and eliminations factored in
    inner blocks of 16 or 32 columns) against none, on the headline square and
    the tall TSQR: median times of `reps` runs after one warm-up."""
    import numpy as np
    import torch

    from paper_1303_5837_amd import caqr, inputs

    out = {}
    for key, m2, n2, fn in [("caqr_%dx%d" % (n, n), n, n, lambda A, ib: caqr.caqr(A, nb=64, inner_block=ib)),
                            ("tsqr_1Mx64", 1 << 20, 64, lambda A, ib: caqr.tsqr(A, inner_block=ib))]:
        seed = inputs.SEEDS["caqr_8192sq"] if m2 == n else inputs.SEEDS["tsqr_1Mx64"]
        B0 = caqr.fortran(inputs.gaussian(m2, n2, seed), device=dev)
        B = torch.empty_like(B0.t()).t()
        row = {}
        for ib in (0, 16, 32):
            times = []
            for it in range(1 + reps):
                B.copy_(B0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                G = fn(B, ib)
                e1.record()
                torch.cuda.synchronize()
                if it >= 1:
                    times.append(e0.elapsed_time(e1))
                G.close()
            row["inner_block_%d_ms" % ib] = round(float(np.median(times)), 3)
        out[key] = row
        del B0, B
        torch.cuda.empty_cache()
    return out


def mixed_ls_line(m=65536, n=1024, kappas=(1e2, 1e4, 1e6), reps=5):
    """Mixed-precision least squares on A = U diag(s) V^T (U, V orthonormal
    factors of seeded Gaussian draws, s geometric from 1 to 1/kappa, ||A||_2 =
    1), b ~ N(0,1): ls_solve with FP32-MFMA trailing updates and FP64
    refinement to eta <= 1e-12, against the plain FP64 ls_solve of the same
    problem; median of `reps` calls each (synchronous calls, host clock; A
    and b restored outside the timed calls).  Both solves get b stored right
    after A ([A | b] in one buffer), so both factor [A | b] and get Q^T b from
    the trailing updates.  eta of both results from its definition with
    ||A||_2 = 1."""
    import numpy as np
    import torch

    from paper_1303_5837_amd import caqr, inputs

    seed = inputs.SEEDS["mixed_ls"]
    rngs = inputs.substreams(seed, 3)
    U = torch.as_tensor(np.linalg.qr(rngs[0].standard_normal((m, n)))[0], device="cuda")
    V = torch.as_tensor(np.linalg.qr(rngs[1].standard_normal((n, n)))[0], device="cuda")
    b0 = caqr.fortran(rngs[2].standard_normal((m, 1)))
    out = {"m": m, "n": n, "construction": "A = U diag(s) V^T, s geometric 1 .. 1/kappa; b ~ N(0,1)"}
    for kappa in kappas:
        s = torch.as_tensor(inputs.geometric_singular_values(n, kappa), device="cuda")
        A0 = torch.empty((n, m), dtype=torch.float64, device="cuda").t()
        A0.copy_((U * s) @ V.t())
        M = torch.empty((n + 1, m), dtype=torch.float64, device="cuda").t()  # [A | b], column-major
        A, B = M[:, :n], M[:, n:]

        def eta(X):
            r = b0 - A0 @ X
            return float(torch.linalg.norm(A0.t() @ r)) / (float(torch.linalg.norm(X)) + float(torch.linalg.norm(b0)))

        row = {}
        for label, prec in (("plain_f64", caqr.LS_F64), ("mixed_f32", caqr.LS_MIXED_F32)):
            ts, info = [], None
            for it in range(2 + reps):
                A.copy_(A0)
                B.copy_(b0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                X, info = caqr.ls_solve(A, B, precision=prec)
                t1 = time.perf_counter()
                if it >= 2:
                    ts.append((t1 - t0) * 1e3)
            row[label] = {"median_ms": round(float(np.median(ts)), 3), "status": int(info.status),
                          "eta": eta(X.clone()), "iters": int(info.iters), "fallback": int(info.fallback),
                          "eta_bound": float(info.eta)}
        row["speedup_mixed_vs_plain"] = round(row["plain_f64"]["median_ms"] / row["mixed_f32"]["median_ms"], 3)
        out["kappa_%.0e" % kappa] = row
        del A0, A, B, M
    del U, V
    torch.cuda.empty_cache()
    return out


TSQR_LINES = {"tsqr_1Mx64": (1 << 20, 64), "tsqr_4096x32": (4096, 32)}


def tsqr_line(key):
    """One tall-skinny TSQR (default tree) timed by HIP events: median, p10 and
    p90 of 20 calls (50 for 4096 x 32) after 5 warm-ups; algorithmic bytes 16mn
    (read A, write Y/R)."""
    import numpy as np
    import torch

    from paper_1303_5837_amd import caqr, inputs

    m2, n2 = TSQR_LINES[key]
    B0 = caqr.fortran(inputs.gaussian(m2, n2, inputs.SEEDS[key]))
    B = torch.empty_like(B0.t()).t()
    times = []
    reps = 20 if m2 > 4096 else 50
    arity = 2 if key == "tsqr_4096x32" else 0  # 4096 x 32: its binary tree over 16 leaves
    for it in range(5 + reps):
        B.copy_(B0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        G = caqr.tsqr(B, arity=arity)
        e1.record()
        torch.cuda.synchronize()
        if it >= 5:
            times.append(e0.elapsed_time(e1))
        G.close()
    t = float(np.median(times))
    gbs = panel_bytes(m2, n2) / (t * 1e-3) / 1e9
    del B0, B
    return {"median_us": round(t * 1e3, 2), "p10_us": round(float(np.percentile(times, 10)) * 1e3, 2),
            "p90_us": round(float(np.percentile(times, 90)) * 1e3, 2),
            "gflops": round((2.0 * m2 * n2 * n2 - 2.0 * n2 ** 3 / 3) / (t * 1e-3) / 1e9, 1),
            "algorithmic_GBps": round(gbs, 1), "pct_hbm_peak": round(100 * gbs / PEAK_HBM_GBS, 2)}


def served_line_child(workers, hw_queues=16, which="served"):
    """The served stream in a child process started with GPU_MAX_HW_QUEUES =
    2 x workers (the HIP runtime reads it once, at initialization): each worker
    drives two streams, and with the default four hardware queues the workers'
    streams would share queues and run one after the other."""
    import subprocess

    env = dict(os.environ, GPU_MAX_HW_QUEUES=str(max(hw_queues, 2 * workers)))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--only", which, "--served-workers",
                        str(workers)], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": f"served child exited {r.returncode}", "stderr_tail": r.stderr[-2000:]}
    line = json.loads(r.stdout.strip().splitlines()[-1])[which]
    line["hw_queues"] = int(env["GPU_MAX_HW_QUEUES"])
    return line


def measured_peaks(dev):
    """Achievable rates on this device, as context for the spec peaks: HBM from a
    plain 512 MiB device-to-device copy (bytes read + written / time) and FP64
    matrix throughput from the vendor BLAS (torch.matmul on float64, 8192^3)."""
    import numpy as np
    import torch

    def timed(fn, reps):
        ts = []
        for it in range(reps + 2):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if it >= 2:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    src = torch.empty(64 << 20, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src), 10)
    hbm = 2.0 * src.numel() * 8 / (t * 1e-3) / 1e9
    del src, dst
    a = torch.randn(8192, 8192, dtype=torch.float64, device=dev)
    b = torch.randn(8192, 8192, dtype=torch.float64, device=dev)
    t = timed(lambda: torch.matmul(a, b), 5)
    dg = 2.0 * 8192 ** 3 / (t * 1e-3) / 1e12
    del a, b
    torch.cuda.empty_cache()
    return {"hbm_copy_GBps": round(hbm, 1), "hbm_spec_GBps": PEAK_HBM_GBS,
            "dgemm_8192_TFLOPs": round(dg, 2), "fp64_spec_TFLOPs": PEAK_FP64_TFLOPS,
            "how": "512 MiB device copy (read + write bytes); torch.matmul float64 8192^3 (vendor BLAS)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--only", choices=["batched_tsqr", "batched_tsqr_f32", "batched_ls", "served", "served_long",
                                       "tsqr_1Mx64", "tsqr_4096x32", "mixed_ls"],
                    help="run one secondary workload alone and print its line (for profiling)")
    ap.add_argument("--served-workers", type=int, default=8, help="worker threads of the served stream's server")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(row blocks sharded over GPUs with one all-gather of R factors per panel is a design, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1303_5837_amd import caqr, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.only:
        fn = {"batched_tsqr": lambda: batched_line("f64"), "batched_tsqr_f32": lambda: batched_line("f32"),
              "batched_ls": batched_ls_line, "served": lambda: served_lines(workers=args.served_workers),
              "served_long": lambda: served_lines(rates=(1000, 2000), duration=10.0, workers=args.served_workers,
                                                  plain=False),
              "tsqr_1Mx64": lambda: tsqr_line("tsqr_1Mx64"), "tsqr_4096x32": lambda: tsqr_line("tsqr_4096x32"),
              "mixed_ls": mixed_ls_line}[args.only]
        print(json.dumps({args.only: fn()}))
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    nb = 64
    A0 = caqr.fortran(inputs.gaussian(n, n, inputs.SEEDS["caqr_8192sq"]), device=dev)
    A = torch.empty_like(A0.t()).t()
    h = caqr.handle(0)

    def one_step():
        A.copy_(A0)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        F = caqr.caqr(A, nb=nb)
        ev1.record()
        return F, ev0, ev1

    for _ in range(args.warmup):
        F, _, _ = one_step()
        F.close()
    torch.cuda.synchronize()

    # events bracket the wide trailing-update calls (a leaf launch plus one
    # launch per tree level, on the second stream), the kernel whose roofline
    # the line reports; the panel factorizations (on the critical chain, where
    # the events' own cost would lengthen the step) are timed in the
    # diagnostic step below
    h.set_trace_kinds(["update_t_levels"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    events = []
    for _ in range(args.steps):
        F, e0, e1 = one_step()
        events.append((e0, e1))
        F.close()  # waits for the device before freeing the factors' buffers
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    trace = h.take_trace()
    h.set_trace(False)
    step_ms = [a.elapsed_time(b) for a, b in events]
    ms = float(np.mean(step_ms))
    lapack_flops = 4.0 * n ** 3 / 3.0
    gflops = lapack_flops / (ms * 1e-3) / 1e9

    # diagnostics outside the timed steps: the step without any event, and one
    # step with every launch bracketed (the panel chain's parts)
    untraced = []
    for _ in range(2):
        F, e0, e1 = one_step()
        F.close()
        untraced.append(e0.elapsed_time(e1))
    h.set_trace(True)
    F, e0, e1 = one_step()
    F.close()
    full_ms = e0.elapsed_time(e1)
    full = h.take_trace()
    h.set_trace(False)
    chain = {}
    for e in full:
        chain[e["kind"]] = chain.get(e["kind"], 0.0) + e["ms"]

    upd = [e for e in trace if e["kind"] == "update_t_levels"]
    upd_alg_bytes = sum(16.0 * e["rows"] * e["cols"] for e in upd) / max(1, len(upd))
    upd_ms = sum(e["ms"] for e in upd)
    upd_flops = sum(update_flops(e["rows"], e["cols"], e["width"], e["leaves"]) for e in upd)
    upd_achieved = upd_flops / (upd_ms * 1e-3) / 1e12 if upd_ms > 0 else 0.0
    pan = [e for e in full if e["kind"] == "panel"]  # the diagnostic step (every launch bracketed)
    pan_bytes = sum(panel_bytes(e["rows"], e["width"]) for e in pan)
    pan_ms = sum(e["ms"] for e in pan)
    pan_gbs = pan_bytes / (pan_ms * 1e-3) / 1e9 if pan_ms > 0 else 0.0
    pan_tflops = sum(panel_flops(e["rows"], e["width"]) for e in pan) / (pan_ms * 1e-3) / 1e12 if pan_ms > 0 else 0.0
    roof_update = {
        "kernel": "trailing update call Q_s^T C of the columns beyond the next panel: leaf_res_kernel "
                  "(each leaf's Y and T resident in LDS, one workgroup per CU over 128-column tiles) + one "
                  "node_res_kernel per tree level (each node's V and T resident in LDS; the root one also "
                  "applies D)",
        "bound": "mfma",
        "achieved": round(upd_achieved, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(upd_achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": traffic_per_call("update"),
        "traffic_unit": "HBM bytes per update call (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "traffic_algorithmic": round(upd_alg_bytes),
        "launches_per_step": len(upd) // max(1, args.steps),
        "avg_launch_ms": round(upd_ms / max(1, len(upd)), 5),
        "share_of_step": round(upd_ms / max(1e-9, sum(step_ms)), 4),
    }
    roof_panel = {
        "kernel": "panel factorization tsqr_panel_kernel (256-row leaves, one per workgroup, and the arity-4 "
                  "tree climbed with tickets): one launch per panel",
        "bound": "hbm",
        "achieved": round(pan_gbs, 3),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(pan_gbs / PEAK_HBM_GBS, 5),
        "traffic": traffic_per_call("panel"),
        "traffic_unit": "HBM bytes per panel launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "traffic_algorithmic": round(pan_bytes / max(1, len(pan))),
        "algorithmic_bytes": "16 m_s b per panel (read the panel, write its Y and R)",
        "fp64_tflops": round(pan_tflops, 4),
        "launches_per_step": len(pan),
        "avg_launch_ms": round(pan_ms / max(1, len(pan)), 5),
        "share_of_step": round(pan_ms / max(1e-9, full_ms), 4),
        "timed": "one diagnostic step with every launch bracketed, after the timed steps",
        "bound_note": "latency: 64 sequential Householder steps per leaf and per tree level",
    }
    panel_dominant = pan_ms >= upd_ms / max(1, args.steps)

    out = {
        "metric": "CAQR FP64 GFLOP/s (% peak); batched LS solves/s + p99 latency vs plain",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"caqr_fp64_{n}x{n}_nb{nb}", "m": n, "n": n, "nb": nb, "leaf_rows": 256,
                   "tree": "arity 4 per panel: 256-row leaf per workgroup (leaves_per_wg 1), device-wide levels "
                           "by tickets", "seed": inputs.SEEDS["caqr_8192sq"],
                   "flop_count": "LAPACK 4n^3/3"},
        "pct_fp64_peak": round(100.0 * gflops / (PEAK_FP64_TFLOPS * 1e3), 2),
        "gflops_executed": round(executed_flops(n, n, nb) / (ms * 1e-3) / 1e9, 2),
        "executed_flop_count": "leaf QRs + stacked eliminations + trailing updates with their tree nodes",
        "step_ms": [round(x, 4) for x in step_ms],
        "step_ms_p10_p50_p90": [round(float(np.percentile(step_ms, q)), 4) for q in (10, 50, 90)],
        "wall_ms_timed_region": round(wall_ms, 2),
        "ms_per_step_untraced": round(float(np.mean(untraced)), 4),
        "panel_chain_ms_per_step": {k: round(v, 3) for k, v in sorted(chain.items())},
        "panel_chain_note": "one step with every launch bracketed: panel = panel kernels, form_t = T "
                            "formation, update_t = the next panel's single-launch update (these three are the "
                            "chain), update_t_levels = the wide updates beside it",
        "roofline": roof_panel if panel_dominant else roof_update,
        "roofline_other": roof_update if panel_dominant else roof_panel,
    }
    del F
    A0 = A = None
    torch.cuda.empty_cache()

    if not args.no_secondary:
        out["peaks_measured"] = measured_peaks(dev)
        sec = {}
        for key in ("tsqr_1Mx64", "tsqr_4096x32"):
            sec[key] = tsqr_line(key)
        sec["inner_block"] = inner_block_line(dev, n)
        # uneven batch (2000 problems, m log-uniform in [256, 65536], n in {8,16,32,64}),
        # plans from the autotuner; one step = one tsqr_factor_batched call
        sec["batched_tsqr_2000_uneven"] = batched_line("f64")
        sec["batched_tsqr_2000_uneven_f32"] = batched_line("f32")
        sec["batched_ls_2000_uneven"] = batched_ls_line()
        sec["mixed_ls_65536x1024"] = mixed_ls_line()
        sec["served_ls"] = served_line_child(args.served_workers)
        # the two highest rates again over 10 s of arrivals (served configuration only)
        sec["served_ls_10s"] = served_line_child(args.served_workers, which="served_long")
        out["secondary"] = sec

    if not args.no_cpu_baseline:
        import oracle

        ns = n  # the headline workload itself: about 15-30 s of CPU work on 16 cores
        S = inputs.gaussian(ns, ns, inputs.SEEDS["caqr_8192sq"])
        t0 = time.perf_counter()
        oracle.qr_r(S)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(4.0 * ns ** 3 / 3.0 / dt / 1e9, 3),
            "unit": "GFLOP/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"oracle Householder QR of a {ns}x{ns} N(0,1) matrix (seed 2), one run of {dt:.1f} s, "
                      f"LAPACK flop count 4n^3/3, OpenMP over trailing columns",
        }
        # labelled secondary CPU reference (not the baseline): the host LAPACK
        # QR (numpy.linalg.qr, R only) of the same matrix on all host cores
        t0 = time.perf_counter()
        np.linalg.qr(S, mode="r")
        dt = time.perf_counter() - t0
        out["cpu_reference_lapack"] = {"value": round(4.0 * ns ** 3 / 3.0 / dt / 1e9, 3), "unit": "GFLOP/s",
                                       "seconds": round(dt, 2), "kind": "host LAPACK dgeqrf via numpy.linalg.qr",
                                       "host_cpus": os.cpu_count()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
