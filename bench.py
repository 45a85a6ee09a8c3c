"""Benchmark: incremental maintenance of an A^16 view, n = 8192, FP32,
rank-1 updates (LINVIEW IncrExp) against dense re-evaluation on the GPU.

One step = one rank-1 update Delta A = u v^T fully applied to every stored
power (A, A^2, A^4, A^8, A^16).  Inputs (A and all update vectors) are
resident in HBM before the timed region.  Prints ONE JSON line on stdout;
progress goes to stderr.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "updates/s + HBM GB/s, incremental A^16 n=8192 rank-1 vs re-eval; p99 latency"
HBM_PEAK_GBPS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=8192)
    p.add_argument("--k", type=int, default=16)
    p.add_argument("--rank", type=int, default=1)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--latency-samples", type=int, default=200)
    p.add_argument("--timing-updates", type=int, default=100)
    p.add_argument("--reeval-reps", type=int, default=2)
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-reeval", action="store_true")
    p.add_argument("--quick", action="store_true", help="timed region only (for profilers)")
    p.add_argument("--no-secondary", action="store_true",
                   help="skip the rank-4, batched and serving workloads")
    p.add_argument("--serve-seconds", type=float, default=4.0)
    p.add_argument("--only", choices=["rank4", "batched", "serving", "sums", "general", "models", "ols", "glin", "ceiling",
                                      "fp64", "small", "serving32", "capacity", "serving_kernels"],
                   help="run one secondary workload alone and print its result (for profilers)")
    return p.parse_args()


def bench_rank4(torch, lv, synth, dev, steps=200, drift_every=100):
    """A^16 view, n = 16384, rank-4 updates: plain FP32 and FP32 with
    bfloat16 shadows (skinny products on the matrix cores), updates/s and the
    per-kind kernel time of one update.  Both views run the periodic drift
    check every `drift_every` updates with the mode's default bound (the
    timed updates include those checks); one check is also timed alone."""
    n, k, r = 16384, 16, 4
    A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=3).astype(np.float32)).to(dev)
    U, V = synth.update_factors(n, r, steps + 5, seed=0, config=3)
    Ud = torch.from_numpy(U.astype(np.float32)).to(dev)
    Vd = torch.from_numpy(V.astype(np.float32)).to(dev)
    out = {"workload": "A^16, n=16384, rank-4 updates"}
    for tag, mode in (("fp32", lv.LV_FP32), ("bf16shadow", lv.LV_FP32_BF16SHADOW)):
        view = lv.View(A, k, r_max=r, mode=mode)
        tiles = view.autotune(pipelined=True, trial_updates=12)
        view.update_batch(Ud[:5], Vd[:5])
        view.set_drift_check(drift_every)          # counts from here: 5 updates applied
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        view.update_batch(Ud[5:], Vd[5:])
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        st = view.stats()
        z = torch.from_numpy(synth.rng(0, 3, 77).choice([-1.0, 1.0], size=n)).to(dev)
        view.drift_check(z, tau=st["drift_tau"])
        torch.cuda.synchronize()
        a.record()
        view.drift_check(z, tau=st["drift_tau"])
        b.record()
        torch.cuda.synchronize()
        drift = {"every": drift_every, "tau": st["drift_tau"], "checks_in_timed_updates": int(st["drift_checks"]),
                 "reanchors": int(st["drift_reanchors"]), "last_residual": st["last_residual"],
                 "check_ms": a.elapsed_time(b),
                 "check_cost_per_update_ms": a.elapsed_time(b) / drift_every}
        view.set_timing(True)
        view.update(Ud[0], Vd[0])
        tm = view.timing()
        view.set_timing(False)
        view.close()
        out[tag] = {"ms_per_update": ms, "updates_per_s": 1000.0 / ms, "rank1_equiv_per_s": 4000.0 / ms,
                    "tile_rows": tiles,
                    "level_passes_ms": tm["fused_ms"], "tails_ms": tm["tail_ms"], "top_update_ms": tm["top_ms"],
                    "drift_check": drift}
    del A
    return out


def stream_ceiling(torch, lv, dev, power_bytes, reps=5):
    """Measured HBM ceiling for the level passes' access pattern: the
    library's streaming kernels (lv_stream_probe: 16-byte non-temporal loads
    and stores, whole 1 KiB row segments per wave) swept over work-groups
    per CU (1..32), 4 KiB chunks in flight per iteration (1..32) and
    pipelined / plain issue, on buffers of 2 GiB and of one stored power.
    Per kind and size the best median rate; RMW (read and write of one
    buffer in place) is the level passes' pattern."""
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    big = 2 << 30
    a = torch.zeros(big // 4, dtype=torch.float32, device=dev)
    b = torch.zeros(big // 4, dtype=torch.float32, device=dev)
    sink = torch.zeros(32 * cus * 256, dtype=torch.float32, device=dev)
    names = {lv.LV_STREAM_RMW: "rmw", lv.LV_STREAM_COPY: "copy", lv.LV_STREAM_READ: "read",
             lv.LV_STREAM_WRITE: "write"}
    out = {"kernel": "lv_stream_probe", "cus": cus}
    for nbytes, tag in ((big, "2GiB"), (power_bytes, "one_power")):
        nbytes -= nbytes % (4096 * 32)
        for kind, name in names.items():
            best = None
            for depth in (1, 2, 4, 8, 16, 32):
                for bpc in (1, 2, 4, 8, 16, 32):
                    for pipe in ((0,) if kind == lv.LV_STREAM_WRITE else (0, 1)):
                        if kind == lv.LV_STREAM_READ:
                            f = lambda: lv.lv_stream_probe(kind, sink, a, nbytes, bpc * cus, depth, pipe)
                        elif kind == lv.LV_STREAM_COPY:
                            f = lambda: lv.lv_stream_probe(kind, b, a, nbytes, bpc * cus, depth, pipe)
                        else:
                            f = lambda: lv.lv_stream_probe(kind, a, None, nbytes, bpc * cus, depth, pipe)
                        f()
                        evs = []
                        for _ in range(reps):
                            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                            e0.record()
                            f()
                            e1.record()
                            evs.append((e0, e1))
                        torch.cuda.synchronize()
                        ms = sorted(x.elapsed_time(y) for x, y in evs)[reps // 2]
                        moved = nbytes * (2 if kind in (lv.LV_STREAM_RMW, lv.LV_STREAM_COPY) else 1)
                        gbps = moved / (ms * 1e-3) / 1e9
                        if best is None or gbps > best["GBps"]:
                            best = {"GBps": gbps, "blocks_per_cu": bpc, "depth": depth, "pipelined": pipe,
                                    "bytes": nbytes}
            out[f"{name}_{tag}"] = best
    del a, b, sink
    torch.cuda.empty_cache()
    return out


def _time_ms(torch, fn, reps=3):
    """Best of `reps` event-timed runs of fn() on the current stream."""
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def bench_fp64(torch, lv, synth, dev, steps=100):
    """The headline view in the paper's precision (Sec. 7: double-precision
    matrices): A^16, n = 8192, FP64, rank-1 updates; updates/s, algorithmic
    HBM rate (one read and one write of each stored power, 80 n^2 bytes per
    update) and FP64 re-evaluation (the library's f64 matrix-core GEMM and
    torch.matmul)."""
    n, k = 8192, 16
    A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=2)).to(dev)
    U, V = synth.update_factors(n, 1, steps + 5, seed=0, config=2)
    Ud, Vd = torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev)
    view = lv.View(A, k)
    tiles = view.autotune(pipelined=True, trial_updates=12)
    view.update_batch(Ud[:5], Vd[:5])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    view.update_batch(Ud[5:], Vd[5:])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    n_pad = view.stats()["n_pad"]
    view.close()
    own = _time_ms(torch, lambda: lv.reeval(A, k, Ud[0], Vd[0]), reps=2)

    def vendor():
        X = torch.addmm(A, Ud[0], Vd[0].t())
        for _ in range(4):
            X = torch.matmul(X, X)
        return X
    tm = _time_ms(torch, vendor, reps=2)
    alg = 2 * 8 * 5 * n_pad * n_pad
    del A
    return {"workload": "A^16 matrix-power view, n=8192, FP64, rank-1 updates (IncrExp)",
            "ms_per_update": ms, "updates_per_s": 1000.0 / ms, "alg_bytes_per_update": alg,
            "alg_GBps": alg / (ms * 1e-3) / 1e9, "tile_rows": tiles,
            "reeval_own_f64_mfma_ms": own, "reeval_torch_matmul_ms": tm,
            "reeval_own_tflops": 2.0 * n ** 3 * 4 / (own * 1e-3) / 1e12,
            "speedup_incremental_vs_best_reeval": min(own, tm) / ms}


def bench_small_fp64(torch, lv, synth, dev, updates=100):
    """The small configuration: A^16, n = 256, FP64, 100 rank-1 updates;
    incremental updates on the GPU, GPU re-evaluation after each update, and
    the FP64 oracle's incremental update and re-evaluation on the host."""
    import oracle as O
    n, k = 256, 16
    A64 = synth.gaussian_matrix(n, seed=0, config=1)
    Us, Vs = synth.update_factors(n, 1, updates, seed=0, config=1)
    A = torch.from_numpy(A64).to(dev)
    Ud, Vd = torch.from_numpy(Us).to(dev), torch.from_numpy(Vs).to(dev)
    view = lv.View(A, k)
    view.update_batch(Ud[:5], Vd[:5])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    view.update_batch(Ud, Vd)
    b.record()
    torch.cuda.synchronize()
    gpu_incr = a.elapsed_time(b) / updates
    view.close()
    gpu_reeval = _time_ms(torch, lambda: lv.reeval(A, k, Ud[0], Vd[0]))
    P = O.reeval(A64, k)
    t0 = time.perf_counter()
    for t in range(updates):
        P = O.incr_update(P, Us[t], Vs[t])
    cpu_incr = (time.perf_counter() - t0) / updates * 1e3
    t0 = time.perf_counter()
    for _ in range(10):
        O.reeval(A64, k)
    cpu_reeval = (time.perf_counter() - t0) / 10 * 1e3
    return {"workload": "A^16, n=256, FP64, 100 rank-1 updates",
            "gpu_incremental_ms": gpu_incr, "gpu_reeval_ms": gpu_reeval,
            "oracle_incremental_ms": cpu_incr, "oracle_reeval_ms": cpu_reeval,
            "note": "fits in cache and is bound by launch latency; no roofline claim"}


def bench_sums(torch, lv, synth, dev, steps=200):
    """A^16 view with its sums of powers S_1..S_16 (LV_WITH_SUMS), n = 8192,
    FP32, rank-1 updates: updates/s and algorithmic HBM bytes per update
    (one read and one write of each stored power and of S_2 .. S_16: P_j Q_j
    rides on the powers' pass, S_j^T V_j on the update pass of S_j)."""
    n, k = 8192, 16
    A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=2).astype(np.float32)).to(dev)
    U, V = synth.update_factors(n, 1, steps + 5, seed=0, config=2)
    Ud = torch.from_numpy(U.astype(np.float32)).to(dev)
    Vd = torch.from_numpy(V.astype(np.float32)).to(dev)
    view = lv.View(A, k, sums=True)
    del A
    view.update_batch(Ud[:5], Vd[:5])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    view.update_batch(Ud[5:], Vd[5:])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    n_pad = view.stats()["n_pad"]
    view.close()
    alg = (40 + 32) * n_pad * n_pad
    return {"workload": "A^16 and sums of powers S_1..S_16, n=8192, FP32, rank-1 updates",
            "ms_per_update": ms, "updates_per_s": 1000.0 / ms, "alg_bytes_per_update": alg,
            "alg_GBps": alg / (ms * 1e-3) / 1e9}


def bench_general(torch, lv, synth, dev, steps=100, ps=(1, 16, 64)):
    """General form T_{i+1} = A T_i + B (hybrid deltas on the exponential
    model), n = 8192, k = 16, FP32, rank-1 updates, for several p: ms per
    update of the general-form view (powers, sums and T_1..T_16 current),
    against re-evaluation by the linear model on the GPU (A += U V^T, then
    16 steps T = A T + B with torch.matmul; it yields T_16 only)."""
    n, k = 8192, 16
    A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=2).astype(np.float32)).to(dev)
    U, V = synth.update_factors(n, 1, steps + 5, seed=0, config=2)
    Ud = torch.from_numpy(U.astype(np.float32)).to(dev)
    Vd = torch.from_numpy(V.astype(np.float32)).to(dev)
    out = {"workload": "general form T_{i+1} = A T_i + B, n=8192, k=16, FP32, rank-1 updates"}
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for p in ps:
        T0, B = (torch.from_numpy(x.astype(np.float32)).to(dev) for x in synth.general_operands(n, p, seed=0))
        view = lv.View(A, k, general=(T0, B))
        view.update_batch(Ud[:5], Vd[:5])
        torch.cuda.synchronize()
        a.record()
        view.update_batch(Ud[5:], Vd[5:])
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        view.close()
        del view
        torch.cuda.empty_cache()
        Ar = A.clone()
        reps = 20

        def reeval_lin(t):
            Ar.addmm_(Ud[t], Vd[t].t())
            T = T0
            for _ in range(k):
                T = torch.addmm(B, Ar, T)
            return T
        reeval_lin(0)
        torch.cuda.synchronize()
        a.record()
        for t in range(reps):
            reeval_lin(1 + t)
        b.record()
        torch.cuda.synchronize()
        lin_ms = a.elapsed_time(b) / reps
        del Ar
        out[f"p{p}"] = {"hybrid_exp_ms_per_update": ms, "updates_per_s": 1000.0 / ms,
                        "reeval_lin_torch_ms": lin_ms, "reeval_lin_over_hybrid": lin_ms / ms}
    # factored deltas (App. B) at p = 16 and at the regression experiment's p = 1000
    for p in (16, 1000):
        T0, B = (torch.from_numpy(x.astype(np.float32)).to(dev) for x in synth.general_operands(n, p, seed=0))
        view = lv.View(A, k, general=(T0, B), strategy=lv.LV_GENERAL_FACTORED)
        view.update_batch(Ud[:5], Vd[:5])
        torch.cuda.synchronize()
        a.record()
        view.update_batch(Ud[5:5 + steps // 2], Vd[5:5 + steps // 2])
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / (steps // 2)
        view.close()
        del view
        torch.cuda.empty_cache()
        Ar = A.clone()

        def reeval_lin(t):
            Ar.addmm_(Ud[t], Vd[t].t())
            T = T0
            for _ in range(k):
                T = torch.addmm(B, Ar, T)
            return T
        reeval_lin(0)
        torch.cuda.synchronize()
        a.record()
        for t in range(5):
            reeval_lin(1 + t)
        b.record()
        torch.cuda.synchronize()
        lin_ms = a.elapsed_time(b) / 5
        del Ar
        out[f"p{p}_factored"] = {"factored_exp_ms_per_update": ms, "updates_per_s": 1000.0 / ms,
                                 "reeval_lin_torch_ms": lin_ms, "reeval_lin_over_factored": lin_ms / ms}
    # skip-4 model with factored deltas (Table 1, App. B): powers and sums up
    # to P_4, S_4; T_1, T_2, T_4, then T_8, T_12, T_16 by steps of 4
    for p in (16, 1000):
        T0, B = (torch.from_numpy(x.astype(np.float32)).to(dev) for x in synth.general_operands(n, p, seed=0))
        view = lv.View(A, k, general=(T0, B), strategy=lv.LV_GENERAL_FACTORED, skip=4)
        view.update_batch(Ud[:5], Vd[:5])
        torch.cuda.synchronize()
        a.record()
        view.update_batch(Ud[5:5 + steps // 2], Vd[5:5 + steps // 2])
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / (steps // 2)
        view.close()
        del view
        torch.cuda.empty_cache()
        out[f"p{p}_factored_skip4"] = {"factored_skip4_ms_per_update": ms, "updates_per_s": 1000.0 / ms}
    del A
    return out


def _app_a_ops(model, n, k, s=None):
    """Operations of one rank-1 refresh of every stored matrix, App. A's
    closed forms (linear, exponential; skip-s: the exponential part up to s
    plus the k/s - 1 skip products)."""
    if model == "lin":
        return n * n * (k * k + k - 1) + 1.5 * n * k * (k - 1)
    if model == "exp":
        return n * n * (4 * k - 3) + n * (k - 1) * (2 * k + 5) / 3
    K = k // s
    return (n * n * (4 * s - 3) + n * (s - 1) * (2 * s + 5) / 3 + n * n * (k * k / s + k - 2 * s)
            + (2 * s + 1) * n * s * K * (K - 1) / 2)


def bench_models(torch, lv, synth, dev, ks=(4, 8, 16, 32, 64), n=8192, skip_s=4):
    """k sweep of the iterative models for A^k (the GPU analog of the k sweep
    of Sec. 7, Fig. mp3, with the models of Table 2), n = 8192, FP32,
    rank-1 updates: ms per update of IncrExp (the exponential view),
    IncrLin and IncrSkip-s (model views), ReevalExp (own MFMA squaring
    chain), with App. A's operation count of each incremental model."""
    A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=2).astype(np.float32)).to(dev)
    U, V = synth.update_factors(n, 1, 40, seed=0, config=2)
    Ud = torch.from_numpy(U.astype(np.float32)).to(dev)
    Vd = torch.from_numpy(V.astype(np.float32)).to(dev)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn(0)
        torch.cuda.synchronize()
        a.record()
        for t in range(reps):
            fn(1 + t)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {"workload": f"A^k, n={n}, FP32, rank-1 updates, k sweep", "skip_s": skip_s}
    ws = torch.empty(lv.lv_reeval_footprint(n, 1, lv.LV_FP32), dtype=torch.uint8, device=dev)
    res = torch.empty(n, n, dtype=torch.float32, device=dev)
    for k in ks:
        row = {}
        view = lv.View(A, k)
        row["incr_exp_ms"] = timed(lambda t: view.update(Ud[t], Vd[t]), 20)
        view.close()
        del view
        for name, model, s, reps in (("incr_lin_ms", lv.LV_MODEL_LIN, 0, 3 if k >= 32 else 8),
                                     ("incr_skip_ms", lv.LV_MODEL_SKIP, skip_s, 8)):
            if model == lv.LV_MODEL_SKIP and k < skip_s:
                continue
            ch = lv.Chain(A, k, model=model, s=s)
            row[name] = timed(lambda t: ch.update(Ud[t], Vd[t]), reps)
            ch.close()
            del ch
            torch.cuda.empty_cache()
        row["reeval_exp_ms"] = timed(lambda t: lv.lv_reeval(A, k, Ud[t], Vd[t], lv.LV_FP32, res, ws), 2)
        row["ops_app_a"] = {"lin": _app_a_ops("lin", n, k), "exp": _app_a_ops("exp", n, k),
                            "skip": _app_a_ops("skip", n, k, skip_s) if k >= skip_s else None}
        out[f"k{k}"] = row
        log(f"models k={k}: {row}")
    del A, ws, res
    return out


def bench_ols(torch, lv, synth, dev, m=16384, n=8192, p=16, steps=50):
    """Least squares under data changes (Sec. 5.1, Sherman-Morrison), X
    16384 x 8192, Y 16384 x 16, FP32: ms per row change and per dense
    rank-1 change of X, against re-evaluation (the view's own creation:
    X^T X, Newton-Schulz inverse, beta; and torch: X^T X, Cholesky solve)."""
    g = synth.rng(0, 2, 94)
    X = torch.from_numpy(g.standard_normal((m, n)).astype(np.float32)).to(dev)
    Y = torch.from_numpy(g.standard_normal((m, p)).astype(np.float32)).to(dev)
    rows = g.integers(0, m, size=steps + 5)
    dx = torch.from_numpy((g.standard_normal((steps + 5, n)) * 0.3).astype(np.float32)).to(dev)
    us = torch.from_numpy((g.standard_normal((steps + 5, m)) * 0.05).astype(np.float32)).to(dev)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ols = lv.Ols(X, Y)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    info = ols.info()

    def timed(fn, reps):
        fn(0)
        torch.cuda.synchronize()
        a.record()
        for t in range(reps):
            fn(1 + t)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps
    row_ms = timed(lambda t: ols.update_row(int(rows[t]), dx[t]), steps)
    dense_ms = timed(lambda t: ols.update(us[t], dx[t]), steps // 2)
    ols.close()
    del ols
    torch.cuda.empty_cache()

    def torch_reeval(t):
        Z = X.t() @ X
        L = torch.linalg.cholesky(Z)
        return torch.cholesky_solve(X.t() @ Y, L)
    torch_ms = timed(torch_reeval, 3)
    del X, Y
    alg = 3 * n * n * 4
    return {"workload": f"OLS X {m}x{n}, Y {m}x{p}, FP32", "row_update_ms": row_ms, "dense_update_ms": dense_ms,
            "row_updates_per_s": 1000.0 / row_ms, "row_update_alg_bytes": alg,
            "row_update_alg_GBps": alg / (row_ms * 1e-3) / 1e9, "reeval_own_create_s": create_s,
            "newton_schulz": info, "reeval_torch_cholesky_ms": torch_ms,
            "speedup_row_vs_torch_reeval": torch_ms / row_ms}


def bench_glin(torch, lv, synth, dev, ps=(1, 16, 64, 1000)):
    """The general form under the linear model with B = 0 (the p sweep of the
    paper's general-form experiment), n = 8192, k = 16, FP32, rank-1 updates:
    ms per update of re-evaluation, hybrid and incremental evaluation
    (every T_1 .. T_16 kept current by each)."""
    n, k = 8192, 16
    A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=2).astype(np.float32)).to(dev)
    U, V = synth.update_factors(n, 1, 40, seed=0, config=2)
    Ud = torch.from_numpy(U.astype(np.float32)).to(dev)
    Vd = torch.from_numpy(V.astype(np.float32)).to(dev)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"workload": "general form T_{i+1} = A T_i (B = 0), linear model, n=8192, k=16, FP32, rank-1 updates"}
    for p in ps:
        T0 = torch.from_numpy(synth.general_operands(n, p, seed=0)[0].astype(np.float32)).to(dev)
        B = torch.zeros_like(T0)
        row = {}
        for name, strat in (("reeval_lin_ms", lv.LV_GLIN_REEVAL), ("hybrid_lin_ms", lv.LV_GLIN_HYBRID),
                            ("incr_lin_ms", lv.LV_GLIN_INCR)):
            g = lv.GLin(A, k, T0, B, strategy=strat)
            g.update(Ud[0], Vd[0])
            torch.cuda.synchronize()
            reps = 10
            a.record()
            for t in range(reps):
                g.update(Ud[1 + t], Vd[1 + t])
            b.record()
            torch.cuda.synchronize()
            row[name] = a.elapsed_time(b) / reps
            g.close()
            del g
            torch.cuda.empty_cache()
        out[f"p{p}"] = row
        log(f"glin p={p}: {row}")
    del A
    return out


def bench_batched(torch, lv, synth, dev, rounds=30):
    """64 views, n in {512..4096}, k in {8, 16}, rank 1..8, FP32: one graph
    replay per round (every view applies one update)."""
    g = synth.rng(0, 4, 0)
    ns = g.choice([512, 1024, 2048, 4096], size=64)
    ks = g.choice([8, 16], size=64)
    rs = g.integers(1, 9, size=64)
    views = []
    bytes_round = 0
    for v in range(64):
        n, k, r = int(ns[v]), int(ks[v]), int(rs[v])
        A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=4, view=v).astype(np.float32)).to(dev)
        views.append(lv.View(A, k, r_max=r))
        bytes_round += 2 * 4 * (int(np.log2(k)) + 1) * views[-1].stats()["n_pad"] ** 2
    import tempfile
    t0 = time.perf_counter()
    batch = lv.Batch(views)
    tune_s = time.perf_counter() - t0
    tuning = dict(batch.tuning())
    # the tuner's choices persist through its JSON cache: a fresh process
    # cache loaded from the file serves a new batch of the same views
    cache = os.path.join(tempfile.mkdtemp(), "linview_tune.json")
    lv.lv_tune_cache_save(cache)
    lv.lv_tune_cache_clear()
    tuning["cache_entries"] = lv.lv_tune_cache_load(cache)
    batch.close()
    t0 = time.perf_counter()
    batch = lv.Batch(views)
    tuning["reload"] = dict(batch.tuning())
    tuning["create_s"], tuning["create_from_cache_s"] = tune_s, time.perf_counter() - t0
    tuning["tile_rows"] = sorted({t for x in views for t in x.tile_rows()})
    for v in range(64):
        n, r = int(ns[v]), int(rs[v])
        U, V = synth.update_factors(n, r, 1, seed=0, config=4, view=v)
        batch.stage(v, torch.from_numpy(U[0].astype(np.float32)).to(dev),
                    torch.from_numpy(V[0].astype(np.float32)).to(dev))
    batch.update()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(rounds):
        batch.update()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / rounds
    # Bound on overlapping successive rounds: a second batch of the same
    # shapes (other matrices) runs its rounds beside the first on a second
    # stream; the time per round of the pair is what overlapping rounds of one
    # batch could reach at best.
    views2 = []
    for v in range(64):
        n, k, r = int(ns[v]), int(ks[v]), int(rs[v])
        A = torch.from_numpy(synth.gaussian_matrix(n, seed=1, config=4, view=v).astype(np.float32)).to(dev)
        views2.append(lv.View(A, k, r_max=r))
    batch2 = lv.Batch(views2)
    for v in range(64):
        U, V = synth.update_factors(int(ns[v]), int(rs[v]), 1, seed=1, config=4, view=v)
        batch2.stage(v, torch.from_numpy(U[0].astype(np.float32)).to(dev),
                     torch.from_numpy(V[0].astype(np.float32)).to(dev))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    batch2.update()
    torch.cuda.synchronize()
    a.record(cur)
    s1.wait_stream(cur)
    s2.wait_stream(cur)
    for _ in range(rounds):
        batch.update(stream=s1)
        batch2.update(stream=s2)
    cur.wait_stream(s1)
    cur.wait_stream(s2)
    b.record(cur)
    torch.cuda.synchronize()
    pair_ms = a.elapsed_time(b) / rounds
    for x in (batch, batch2):
        x.close()
    for x in views + views2:
        x.close()
    return {"workload": "64 views, n in {512,1024,2048,4096}, k in {8,16}, rank 1..8, FP32",
            "round_ms": ms, "view_updates_per_s": 64 * 1000.0 / ms,
            "alg_bytes_per_round": bytes_round, "alg_GBps": bytes_round / (ms * 1e-3) / 1e9,
            "two_batches_side_by_side_ms_per_round": pair_ms / 2,
            "autotune": tuning}


def bench_serving(torch, lv, synth, dev, seconds=4.0, rate=20000.0, r_coalesce=32, shadow=True,
                  hold=(32, 0.2), drift_every=100, budget_bytes=None, evict=4):
    """32 views, n log-uniform in [2048, 16384], k = 16, FP32 (with bfloat16
    shadows by default); Poisson arrivals at `rate` requests/s over views with
    Zipf(1.1) popularity; per-view coalescing, continuous batching; rounds
    hold a view until it has hold[0] requests queued or its oldest has waited
    hold[1] s.  Every view runs the periodic drift check every
    `drift_every` of its coalesced updates (inside the served rounds).
    With budget_bytes the arena is that large and the admission queue is on:
    views are added hottest first, those that do not fit wait (their
    requests queue), and half-way through the run the `evict` coldest
    admitted views are removed, which admits waiting views."""
    mode = lv.LV_FP32_BF16SHADOW if shadow else lv.LV_FP32
    g = synth.rng(0, 5, 0)
    ns = np.exp(g.uniform(np.log(2048), np.log(16384), size=32)).astype(int)
    pop = np.arange(1, 33, dtype=np.float64) ** -1.1
    pop /= pop.sum()
    perm = g.permutation(32)
    probe = lv.Server(16 << 20, mode=mode, r_coalesce=r_coalesce)
    need = sum(probe.view_bytes(int(n), 16) for n in ns)
    probe.close()
    arena = (16 << 20) + need if budget_bytes is None else int(budget_bytes)
    srv = lv.Server(arena, mode=mode, r_coalesce=r_coalesce)
    srv.set_hold(*hold)
    if budget_bytes is not None:
        srv.set_admission_queue(True)
    # views by popularity rank: hottest first (the add order decides admission under a budget)
    rank_of = np.empty(32, dtype=int)
    rank_of[perm] = np.arange(32)          # view perm[j] has popularity rank j
    ids = [None] * 32
    for v in sorted(range(32), key=lambda x: rank_of[x]):
        A = torch.from_numpy(synth.gaussian_matrix(int(ns[v]), seed=0, config=5, view=v).astype(np.float32)).to(dev)
        ids[v] = srv.add_view(A, 16)
        if srv.view_handle(ids[v]):      # admitted (not waiting)
            srv.set_drift_check(ids[v], drift_every)
        del A
    torch.cuda.synchronize()
    st_start = srv.stats()
    removed = set()
    pool = []
    for v in range(32):
        U, V = synth.update_factors(int(ns[v]), 1, 8, seed=0, config=5, view=v)
        pool.append((U[:, :, 0].astype(np.float32), V[:, :, 0].astype(np.float32)))
    count = int(rate * seconds)
    gaps = g.exponential(1.0 / rate, size=count)
    targets = perm[g.choice(32, size=count, p=pop)]
    t0 = srv.now() + 0.05
    arrivals = t0 + np.cumsum(gaps)
    i = 0
    half = count // 2
    while i < count:
        now = srv.now()
        while i < count and arrivals[i] <= now:
            v = int(targets[i])
            if v not in removed:
                u, w = pool[v]
                srv.submit(ids[v], u[i % 8], w[i % 8], float(arrivals[i]))
            i += 1
            if budget_bytes is not None and i == half:
                # the coldest admitted views leave; their room admits waiting views
                admitted = [v for v in range(32) if srv.view_handle(ids[v])]
                for v in sorted(admitted, key=lambda x: -rank_of[x])[:evict]:
                    srv.remove_view(ids[v])
                    removed.add(v)
        srv.step()
    while srv.step() > 0:
        pass
    srv.drain()
    t_end = srv.now()
    st = srv.stats()
    vst = [srv.view_stats(ids[v]) for v in range(32) if v not in removed and srv.view_handle(ids[v])]
    srv.close()
    return {"workload": "32 views, n log-uniform [2048,16384], k=16, %s, Poisson %.0f req/s, Zipf(1.1), "
                        "hold %d requests / %.0f ms" % ("FP32 + BF16 shadows" if shadow else "FP32", rate, hold[0],
                                                        hold[1] * 1e3),
            "offered_per_s": rate, "completed": int(st["completed"]),
            "throughput_per_s": st["completed"] / (t_end - t0), "rounds": int(st["rounds"]),
            "mean_coalesced_rank": st["completed"] / max(st["coalesced_updates"], 1),
            "latency_p50_ms": st["latency_p50_s"] * 1e3, "latency_p99_ms": st["latency_p99_s"] * 1e3,
            "arena_GB": arena / 1e9, "views_need_GB": need / 1e9,
            "drift_check": {"every": drift_every, "checks": int(sum(x["drift_checks"] for x in vst)),
                            "reanchors": int(sum(x["drift_reanchors"] for x in vst)),
                            "max_last_residual": float(max(x["last_residual"] for x in vst))},
            **({} if budget_bytes is None else {
                "budget_GB": arena / 1e9, "views_admitted_at_start": int(st_start["views"]),
                "views_waiting_at_start": int(st_start["views_waiting"]), "views_removed_midway": len(removed),
                "views_admitted_later": int(st["admitted_late"]), "views_still_waiting": int(st["views_waiting"]),
                "requests_submitted": int(st["submitted"]),
                "requests_waiting_for_admission": int(st["submitted"] - st["completed"])})}


def bench_serving_capacity(torch, lv, synth, dev, rate=20000.0, r_cap=32, shadow=True, reps=6):
    """A bound for the serving workload from measured update times: every
    one of its 32 views (same orders, k = 16, same mode) applies rank-r_cap
    updates alone on the device; even if every request were coalesced into
    a full rank-r_cap update (the widest a k = 16 view takes: k r_max <= 512),
    serving `rate` requests/s needs sum_v (rate p_v / r_cap) T_v seconds of
    device time per second.  Above 1 the offered rate cannot be sustained by
    any coalescing within the cap; rate / need is the best the device can
    sustain."""
    mode = lv.LV_FP32_BF16SHADOW if shadow else lv.LV_FP32
    g = synth.rng(0, 5, 0)
    ns = np.exp(g.uniform(np.log(2048), np.log(16384), size=32)).astype(int)
    pop = np.arange(1, 33, dtype=np.float64) ** -1.1
    pop /= pop.sum()
    perm = g.permutation(32)
    share = np.empty(32)
    share[perm] = pop
    times = {}
    need = 0.0
    per_view = []
    for v in range(32):
        n = int(ns[v])
        A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=5, view=v).astype(np.float32)).to(dev)
        U, V = synth.update_factors(n, r_cap, reps + 2, seed=0, config=5, view=v)
        Ud, Vd = torch.from_numpy(U.astype(np.float32)).to(dev), torch.from_numpy(V.astype(np.float32)).to(dev)
        view = lv.View(A, 16, r_max=r_cap, mode=mode)
        del A
        view.update_batch(Ud[:2], Vd[:2])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        view.update_batch(Ud[2:], Vd[2:])
        b.record()
        torch.cuda.synchronize()
        view.close()
        t = a.elapsed_time(b) / reps * 1e-3
        times[n] = t
        need += rate * share[v] / r_cap * t
        per_view.append((float(share[v]), n, t))
    hottest = max(per_view)
    return {"workload": "32 serving views (n log-uniform [2048,16384], k=16, %s), rank-%d updates timed alone"
                        % ("FP32 + BF16 shadows" if shadow else "FP32", r_cap),
            "offered_per_s": rate,
            "device_s_per_s_at_full_coalescing": need,
            "max_sustainable_per_s": rate / need,
            "hottest_view": {"n": hottest[1], "share": hottest[0], "update_ms": hottest[2] * 1e3,
                             "max_rate_per_s": r_cap / hottest[2], "offered_per_s": rate * hottest[0]},
            "update_ms_by_n": {str(n): t * 1e3 for n, t in sorted(times.items())}}


def bench_serving_kernels(torch, lv, synth, dev, reps=2, r=32):
    """The kernels of one rank-r update of serving views (r = 32: the
    serving workload's coalescing width), for a kernel trace: the largest
    serving view (n = 15278) and a middle one (n = 7022) with bfloat16
    shadows, and the largest in plain FP32, each applying rank-r updates one
    at a time (as a serving round runs a view's levels)."""
    out = {}
    for n, mode, tag in ((15278, lv.LV_FP32_BF16SHADOW, "shadow"), (7022, lv.LV_FP32_BF16SHADOW, "shadow"),
                         (15278, lv.LV_FP32, "fp32")):
        A = torch.from_numpy(synth.gaussian_matrix(n, seed=0, config=5, view=1).astype(np.float32)).to(dev)
        U, V = synth.update_factors(n, r, reps + 2, seed=0, config=5, view=1)
        Ud, Vd = torch.from_numpy(U.astype(np.float32)).to(dev), torch.from_numpy(V.astype(np.float32)).to(dev)
        view = lv.View(A, 16, r_max=r, mode=mode)
        del A
        view.set_pipeline(False)
        view.update_batch(Ud[:2], Vd[:2])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        view.update_batch(Ud[2:], Vd[2:])
        b.record()
        torch.cuda.synchronize()
        view.close()
        out[f"n{n}_{tag}"] = {"rank": r, "ms_per_update": a.elapsed_time(b) / reps}
    return out


def counter_traffic(n, k, r):
    """HBM bytes per fused launch from the committed rocprofv3 counter
    summary, or None when the workload differs or the kernel source has
    changed since the counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "k_level_fused_n8192_k16_fp32_rank1_traffic.md")
    srcs = [os.path.join(ROOT, "paper_1403_6968_amd", "csrc", f) for f in ("lv_fused.hip", "lv_device.h")]
    if (n, k, r) != (8192, 16, 1) or not os.path.exists(prof) or not all(os.path.exists(f) for f in srcs):
        return None
    vals = {}
    for line in open(prof):
        if line.startswith("traffic_bytes_per_launch k_level_fused ="):
            vals["bytes"] = float(line.split("=")[1].split()[0])
        elif line.startswith("source_sha256_prefix ="):
            vals["sha"] = line.split("=")[1].strip()
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(f, "rb").read())
    sha = h.hexdigest()[:16]
    if vals.get("sha") != sha or "bytes" not in vals:
        return None
    return vals["bytes"]


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A32, Us, Vs, k, budget_s, one_thread_s=8.0):
    """The FP64 oracle (unchanged) timed on the host on a bounded sample of
    the same workload: as many of the first updates as fit in the budget
    with the BLAS pool at its default size, then with one thread."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    A = A32.astype(np.float64)
    t0 = time.perf_counter()
    P = O.reeval(A, k)
    t_setup = time.perf_counter() - t0
    log(f"cpu oracle: reeval (setup) {t_setup:.1f} s")

    def run(P, first, budget):
        done, t0 = 0, time.perf_counter()
        while first + done < len(Us):
            P = O.incr_update(P, Us[first + done].astype(np.float64), Vs[first + done].astype(np.float64))
            done += 1
            if time.perf_counter() - t0 >= budget:
                break
        return P, done, time.perf_counter() - t0

    P, done, el = run(P, 0, budget_s)
    one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            _, d1, e1 = run(P, done, one_thread_s)
        one = {"value": d1 / e1, "updates": d1, "seconds": e1}
        log(f"cpu oracle: 1 thread {d1 / e1:.3f} updates/s")
    return {
        "value": done / el, "unit": "updates/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{done} rank-1 updates of the same n={A.shape[0]} k={k} view in FP64 "
                  f"({el:.1f} s); oracle re-evaluation of all powers took {t_setup:.1f} s; then "
                  f"{one['updates'] if one else 0} more updates with one BLAS thread",
        "reeval_s": t_setup, "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
        "one_thread": one,
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(views would shard by whole views, or by row blocks of the stored powers)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1403_6968_amd import linview as lv

    lv.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.only:
        fn = {"rank4": lambda: bench_rank4(torch, lv, synth, dev),
              "batched": lambda: bench_batched(torch, lv, synth, dev),
              "serving": lambda: bench_serving(torch, lv, synth, dev, args.serve_seconds),
              "serving32": lambda: bench_serving(torch, lv, synth, dev, args.serve_seconds, budget_bytes=32e9),
              "capacity": lambda: bench_serving_capacity(torch, lv, synth, dev),
              "serving_kernels": lambda: bench_serving_kernels(torch, lv, synth, dev),
              "sums": lambda: bench_sums(torch, lv, synth, dev),
              "general": lambda: bench_general(torch, lv, synth, dev),
              "models": lambda: bench_models(torch, lv, synth, dev),
              "ols": lambda: bench_ols(torch, lv, synth, dev),
              "glin": lambda: bench_glin(torch, lv, synth, dev),
              "fp64": lambda: bench_fp64(torch, lv, synth, dev),
              "ceiling": lambda: stream_ceiling(torch, lv, dev, 4 * 8192 * 8192),
              "small": lambda: bench_small_fp64(torch, lv, synth, dev)}[args.only]
        print(json.dumps({"only": args.only, "result": fn()}), flush=True)
        return
    n, k, r = args.n, args.k, args.rank
    total = args.warmup + args.steps

    t0 = time.perf_counter()
    A64 = synth.gaussian_matrix(n, seed=args.seed, config=2)
    A32 = A64.astype(np.float32)
    del A64
    Us64, Vs64 = synth.update_factors(n, r, total + 2 * args.latency_samples + args.timing_updates,
                                      seed=args.seed, config=2)
    Us, Vs = Us64.astype(np.float32), Vs64.astype(np.float32)
    del Us64, Vs64
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s")

    Ad = torch.from_numpy(A32).to(dev)
    Ud = torch.from_numpy(Us).to(dev)
    Vd = torch.from_numpy(Vs).to(dev)
    stream = torch.cuda.current_stream(dev)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    view = lv.View(Ad, k, r_max=r)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    log(f"view created in {create_s:.2f} s (FP64 MFMA squarings)")
    # tile rows for pipelined batches, picked by timing zero updates (the
    # view's values are unchanged); every later call uses them
    tile_rows = view.autotune(pipelined=True, trial_updates=24)
    log(f"autotuned tile rows: {tile_rows}")

    # warmup
    view.update_batch(Ud[:args.warmup], Vd[:args.warmup])
    torch.cuda.synchronize()

    # timed region: exactly `steps` updates
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    view.update_batch(Ud[args.warmup:total], Vd[args.warmup:total])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    ups = 1000.0 / ms_per_step
    log(f"timed: {args.steps} updates in {ms:.1f} ms (wall {wall * 1e3:.1f} ms): {ups:.1f} updates/s")

    elem = 4
    n_pad = view.stats()["n_pad"]
    levels = view.stats()["levels"]
    alg_bytes_update = 2 * elem * levels * n_pad * n_pad
    result = {
        "metric": METRIC, "value": ups, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"A^{k} matrix-power view, n={n}, FP32, rank-{r} updates (IncrExp)",
                   "n": n, "k": k, "rank": r, "updates_timed": args.steps,
                   "batch": "one lv_view_update_batch call, levels pipelined over streams",
                   "tile_rows": tile_rows},
        "rank1_equiv_updates_per_s": ups * r,
        "hbm_GBps_algorithmic": alg_bytes_update * ups / 1e9,
        "create_s": create_s,
    }

    def latency(base):
        """p50 / p99 of single lv_view_update calls (event pairs on the stream)."""
        lat = []
        for t in range(args.latency_samples):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            view.update(Ud[base + t], Vd[base + t])
            b.record(stream)
            lat.append((a, b))
        torch.cuda.synchronize()
        lat_ms = np.array([a.elapsed_time(b) for a, b in lat])
        return {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                "samples": int(len(lat_ms))}

    if not args.quick:
        # per-update latency (single updates are sequential: each one's levels form a chain)
        base = total
        result["latency_ms"] = latency(base)
        log(f"latency p50 {result['latency_ms']['p50']:.3f} ms p99 {result['latency_ms']['p99']:.3f} ms")

        # dominant kernel: the fused level pass, timed with events by the library
        base += args.latency_samples
        view.set_timing(True)
        view.update_batch(Ud[base:base + args.timing_updates], Vd[base:base + args.timing_updates])
        tm = view.timing()
        view.set_timing(False)
        fused_ms = tm["fused_ms"] / max(tm["fused_launches"], 1)
        bytes_launch = 2 * elem * n_pad * n_pad
        achieved = bytes_launch / (fused_ms * 1e-3) / 1e9
        result["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                              "frac": achieved / HBM_PEAK_GBPS, "traffic": counter_traffic(n, k, r),
                              "kernel": "k_level_fused (levels 0..m-1)",
                              "avg_launch_ms": fused_ms, "bytes_per_launch": bytes_launch,
                              # every pass of the timed (pipelined) region: the algorithmic bytes of
                              # all m + 1 stored powers per update over the region's event time
                              "timed_region_all_passes": {
                                  "GBps": result["hbm_GBps_algorithmic"],
                                  "frac": result["hbm_GBps_algorithmic"] / HBM_PEAK_GBPS}}
        result["kernel_ms_per_update"] = {
            "fused": tm["fused_ms"] / args.timing_updates, "tail": tm["tail_ms"] / args.timing_updates,
            "top_update": tm["top_ms"] / args.timing_updates}
        top_ms = tm["top_ms"] / max(tm["top_launches"], 1)
        result["top_update_GBps"] = bytes_launch / (top_ms * 1e-3) / 1e9
        log(f"fused pass avg {fused_ms * 1e3:.1f} us -> {achieved:.0f} GB/s; "
            f"top update avg {top_ms * 1e3:.1f} us; per update {result['kernel_ms_per_update']}")

        # the same view with tiles tuned for single updates instead (the
        # tiles that suit pipelined batches lengthen each pass run alone)
        lat_tiles = view.autotune(pipelined=False, trial_updates=24)
        base += args.timing_updates
        result["latency_ms_single_update_tiles"] = dict(latency(base), tile_rows=lat_tiles)
        log(f"with tile rows {lat_tiles}: latency p50 {result['latency_ms_single_update_tiles']['p50']:.3f} ms "
            f"p99 {result['latency_ms_single_update_tiles']['p99']:.3f} ms")

    if True:
        # measured streaming ceiling: a plain device copy of one stored power's size
        # (also the reference kernel for scaling HBM traffic counters)
        src = torch.empty(n_pad * n_pad, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(10):
            dst.copy_(src)
        b.record(stream)
        torch.cuda.synchronize()
        copy_ms = a.elapsed_time(b) / 10
        result["copy_ref"] = {"bytes": 2 * 4 * n_pad * n_pad, "ms": copy_ms,
                              "GBps": 2 * 4 * n_pad * n_pad / (copy_ms * 1e-3) / 1e9}
        log(f"copy reference: {result['copy_ref']['GBps']:.0f} GB/s")
        del src, dst
    if not args.quick:
        # measured ceiling of the passes' access pattern (in-place read and write)
        ceil = stream_ceiling(torch, lv, dev, 4 * n_pad * n_pad)
        result["stream_ceiling"] = ceil
        rmw = max(ceil["rmw_one_power"]["GBps"], ceil["rmw_2GiB"]["GBps"])
        log(f"streaming ceiling (in-place read+write): {ceil['rmw_one_power']['GBps']:.0f} GB/s on one power, "
            f"{ceil['rmw_2GiB']['GBps']:.0f} GB/s on 2 GiB; copy {ceil['copy_2GiB']['GBps']:.0f}, "
            f"read {ceil['read_2GiB']['GBps']:.0f}, write {ceil['write_2GiB']['GBps']:.0f}")
        if "roofline" in result:
            result["roofline"]["frac_of_copy"] = result["roofline"]["achieved"] / result["copy_ref"]["GBps"]
            result["roofline"]["frac_of_stream_ceiling"] = result["roofline"]["achieved"] / rmw
            agg = result["roofline"]["timed_region_all_passes"]
            agg["frac_of_stream_ceiling"] = agg["GBps"] / rmw

    if not args.quick and not args.no_reeval:
        ws = torch.empty(lv.lv_reeval_footprint(n, r, lv.LV_FP32), dtype=torch.uint8, device=dev)
        out = torch.empty(n, n, dtype=torch.float32, device=dev)
        u0, v0 = Ud[0], Vd[0]

        def own():
            lv.lv_reeval(Ad, k, u0, v0, lv.LV_FP32, out, ws)

        def vendor():
            X = torch.addmm(Ad, u0, v0.t())
            for _ in range(int(np.log2(k))):
                X = torch.matmul(X, X)
            return X

        res = {}
        for name, fn in (("own_mfma_ms", own), ("torch_matmul_ms", vendor)):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(args.reeval_reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            res[name] = float(min(ts))
        best = min(res.values())
        res["flops"] = 2.0 * n ** 3 * int(np.log2(k))
        res["own_tflops"] = res["flops"] / (res["own_mfma_ms"] * 1e-3) / 1e12
        res["speedup_incremental_vs_best_reeval"] = best / ms_per_step
        result["reeval"] = res
        log(f"reeval: own {res['own_mfma_ms']:.1f} ms ({res['own_tflops']:.1f} TF/s), "
            f"torch {res['torch_matmul_ms']:.1f} ms; speedup {res['speedup_incremental_vs_best_reeval']:.1f}x")
        del ws, out

    view.close()
    del Ad, Ud, Vd
    torch.cuda.empty_cache()
    if not args.quick and not args.no_secondary:
        sec = {}
        for name, fn in (("fp64_n8192", lambda: bench_fp64(torch, lv, synth, dev)),
                         ("small_n256_fp64", lambda: bench_small_fp64(torch, lv, synth, dev)),
                         ("rank4_n16384", lambda: bench_rank4(torch, lv, synth, dev)),
                         ("sums_n8192", lambda: bench_sums(torch, lv, synth, dev)),
                         ("general_n8192", lambda: bench_general(torch, lv, synth, dev)),
                         ("models_k_sweep_n8192", lambda: bench_models(torch, lv, synth, dev)),
                         ("ols_16384x8192", lambda: bench_ols(torch, lv, synth, dev)),
                         ("general_linear_model_n8192", lambda: bench_glin(torch, lv, synth, dev)),
                         ("batched_64_views", lambda: bench_batched(torch, lv, synth, dev)),
                         ("serving_32_views", lambda: bench_serving(torch, lv, synth, dev, args.serve_seconds)),
                         ("serving_32_views_fp32",
                          lambda: bench_serving(torch, lv, synth, dev, args.serve_seconds, shadow=False)),
                         ("serving_32_views_5k",
                          lambda: bench_serving(torch, lv, synth, dev, args.serve_seconds, rate=5000.0)),
                         ("serving_32_views_32GB",
                          lambda: bench_serving(torch, lv, synth, dev, args.serve_seconds, budget_bytes=32e9)),
                         ("serving_capacity_bound", lambda: bench_serving_capacity(torch, lv, synth, dev))):
            sec[name] = fn()
            torch.cuda.empty_cache()
            log(f"{name}: {sec[name]}")
        result["secondary"] = sec
    if not args.quick and not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(A32, Us, Vs, k, args.cpu_seconds)
        log(f"cpu oracle: {result['cpu_baseline']['value']:.3f} updates/s on "
            f"{result['cpu_baseline']['cores']} threads")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
