#!/usr/bin/env python3
"""Benchmark of the chunked backward-Euler solver on one MI355X.

Workload: Van der Pol, n = 2, 512 series x 5000 uniform steps on t in [0, 10],
mu log-uniform in [1, 1000], y0 ~ U(-2, 2), FP64, the paper's tolerances
(tol_a 1e-8, tol_r 1e-6), forward integration.  One step of the benchmark is
one full solve of the workload (every chunk, every Newton iteration, inputs
resident in HBM).  The chunk length and the lane tiling come from the
autotuner (run during warm-up, untimed).

Printed as one JSON line: throughput in series*steps/s, the chunk = 1
sequential GPU solver (same library, one lane per series) on the same
inputs, the roofline of the dominant kernel, the standalone block-bidiagonal
solve against the HBM roofline, forward+adjoint throughput, and the CPU
oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "series·steps/s fwd+adjoint at tol 1e-8 vs chunk=1 sequential; % HBM peak"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
TIMING_TOL = (1e-8, 1e-6)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def vdp_flops_per_step_iter(chunk):
    """Algorithmic flops of one Newton iteration per series-step (Van der Pol):
    residual, Jacobian, block inverse and update (44) plus one composition of
    2x2 affine maps per reduction level (24 per level, ceil(log2 C) levels)."""
    levels = 0
    while (1 << levels) < chunk:
        levels += 1
    return 44 + 24 * levels


def csrc_hash():
    """Hash of the kernel sources; HBM traffic from profiler counters is reported
    only while the sources still match the ones the counters were taken from."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2310_08649_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from profiles/traffic.json (FETCH_SIZE and
    WRITE_SIZE scaled by a plain-copy calibration), or None if stale or absent."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != csrc_hash():
        return None
    return rec["bytes_per_dispatch"]


def time_launches(fn, reps, stream):
    """Average launch duration (ms) by HIP events on the launching stream."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in evs]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=0, help="0 = autotune")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline measurement")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(series would shard across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2310_08649_amd import autotune, tvi, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tvi.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w = workloads.vanderpol()  # 512 x 5000
    B, N = w["y0"].shape[0], w["times"].shape[0] - 1
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    y0, times, mu = d(w["y0"]), d(w["times"]), d(w["params"])
    y_out = torch.empty((B, N + 1, 2), dtype=torch.float64, device=dev)

    # ---- autotune chunk length and tiling (untimed)
    log("autotuning chunk / tiling")
    tuned = autotune.tune_forward("vanderpol", y0, times, mu, tol=TIMING_TOL, y_out=y_out, use_cache=False,
                                  chunks=(10, 50, 100, 200, 500) if args.chunk == 0 else (args.chunk,))
    best = tuned["best"]
    C, S, T = best["chunk"], best["lanes"], best["steps_per_lane"]
    log("chosen chunk=%d lanes=%d steps_per_lane=%d (%.3f ms)" % (C, S, T, best["ms"]))

    def step():
        return tvi.solve_forward("vanderpol", y0, times, mu, chunk=C, lanes=S, steps_per_lane=T, tol=TIMING_TOL,
                                 y_out=y_out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, status, iters, _ = step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    value = B * N / (ms_per_step * 1e-3)
    st = status.cpu().numpy()
    it = iters.cpu().numpy()
    durs = time_launches(step, args.steps, stream)
    kern_ms = float(np.mean(durs))

    flops = float(it.sum()) * C * vdp_flops_per_step_iter(C)
    achieved_tflops = flops / (kern_ms * 1e-3) / 1e12
    kname = "tvi::forward_kernel<tvi::VanDerPol, double, %d, %d>" % (S, T)
    roofline = {"kernel": kname, "bound": "alu",
                "achieved": achieved_tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tflops / PEAK_FP64_TFLOPS, "traffic": measured_traffic(kname),
                "avg_launch_ms": kern_ms,
                "note": "latency-bound: a chain of N/C chunk solves x Newton iterations per series"}

    out = {"metric": METRIC, "value": value, "unit": "series*steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "vanderpol n=2 B=512 N=5000 t=[0,10] mu=10^U(0,3) y0=U(-2,2) forward "
                                  "tol_a=1e-8 tol_r=1e-6", "chunk": C, "lanes": S, "steps_per_lane": T,
                      "series_failed": int((st != 0).sum()), "newton_iters_per_series": float(it.mean())},
           "roofline": roofline, "autotune": tuned["table"]}

    if not args.no_extras:
        # chunk = 1 sequential solver: one lane per series, one Newton solve per step
        log("chunk=1 sequential baseline")
        seq = lambda: tvi.solve_forward("vanderpol", y0, times, mu, chunk=1, lanes=1, steps_per_lane=1,
                                        tol=TIMING_TOL, y_out=y_out)
        seq()
        sd = time_launches(seq, max(3, args.steps // 4), stream)
        seq_ms = float(np.mean(sd))
        out["chunk1"] = {"value": B * N / (seq_ms * 1e-3), "ms_per_step": seq_ms,
                         "speedup_of_chunked": seq_ms / ms_per_step}

        # forward + adjoint (Frobenius loss, checkpoints + recomputation)
        log("forward + adjoint")
        g = torch.empty_like(y_out)

        def fwd_adj():
            y, st_, _, ck = tvi.solve_forward("vanderpol", y0, times, mu, chunk=C, lanes=S, steps_per_lane=T,
                                              tol=TIMING_TOL, y_out=y_out, checkpoints=True, iters=False)
            torch.div(y, torch.linalg.vector_norm(y), out=g)
            return tvi.solve_adjoint("vanderpol", times, mu, g, ckpt=ck, chunk=C, lanes=S, steps_per_lane=T,
                                     tol=TIMING_TOL)

        fwd_adj()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(3, args.steps // 2)
        for _ in range(reps):
            fwd_adj()
        torch.cuda.synchronize()
        fa_ms = (time.perf_counter() - t0) * 1e3 / reps
        out["fwd_adjoint"] = {"value": B * N / (fa_ms * 1e-3), "ms_per_step": fa_ms, "loss": "frobenius",
                              "states": "recomputed from chunk checkpoints"}

        # standalone block-bidiagonal solve on a working set far beyond the caches
        log("standalone PCR solve, n=2 fp64, 4 GiB per launch")
        nb, m, n = 1 << 20, 64, 2
        gen = torch.Generator(device=dev)
        gen.manual_seed(5)
        D = torch.eye(n, dtype=torch.float64, device=dev).expand(nb, m, n, n).contiguous()
        D.add_(torch.randn(D.shape, generator=gen, dtype=torch.float64, device=dev), alpha=0.2)
        r = torch.randn((nb, m, n), generator=gen, dtype=torch.float64, device=dev)
        x = torch.empty_like(r)
        pcr = lambda: tvi.pcr_solve(D, r, out=x)
        pcr()
        pd = time_launches(pcr, 10, stream)
        pcr_ms = float(np.mean(pd))
        bytes_alg = nb * m * (n * n + 2 * n) * 8
        gbs = bytes_alg / (pcr_ms * 1e-3) / 1e9
        pname = "tvi::pcr_kernel<2, double, 64, 1, false>(long, int, double const*, double const*, double*)"
        out["pcr_roofline"] = {"kernel": pname, "bound": "hbm", "achieved": gbs,
                               "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                               "traffic": measured_traffic(pname),
                               "bytes_per_launch": bytes_alg, "avg_launch_ms": pcr_ms,
                               "systems": nb, "block_rows": m, "n": n}
        del D, r, x

    if args.probe_copy:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
        del src, dst

    if not args.no_cpu:
        log("CPU oracle on the host cores")
        import oracle
        threads = oracle.default_threads()
        reps, t_cpu = 0, 0.0
        t0 = time.perf_counter()
        while t_cpu < 2.0 and reps < 50:
            oracle.forward("vanderpol", w["y0"], w["times"], w["params"], tol=TIMING_TOL, threads=threads)
            reps += 1
            t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": reps * B * N / t_cpu, "unit": "series*steps/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "the full workload (512 x 5000, forward) repeated %d times, "
                                         "sequential backward Euler with a dense Newton solve per step" % reps}

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
