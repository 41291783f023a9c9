#!/usr/bin/env python3
"""Benchmark of the chunked backward-Euler solver on one MI355X.

Headline workload: Van der Pol, n = 2, 512 series x 5000 uniform steps on
t in [0, 10], mu log-uniform in [1, 1000], y0 ~ U(-2, 2), FP64, the paper's
tolerances (tol_a 1e-8, tol_r 1e-6), forward integration.  One step of the
benchmark is one full solve of the workload (every chunk, every Newton
iteration, inputs resident in HBM).  The chunk length, the lane tiling and
the initial iterate come from the autotuner (run before timing, untimed).

Printed as one JSON line: throughput in series*steps/s, the roofline of the
dominant kernel, and, beside it, the chunk = 1 sequential GPU solver on the
same inputs, the same workload with float storage, forward + adjoint in one
captured graph, the small linear system, the standalone block-bidiagonal
solve against the HBM roofline, the headline kernel on a chip-filling
batch, the neural-ODE path (forward + adjoint, and a chip-filling forward
batch) against the matrix-core peak, the ragged Robertson batch as one captured
graph, the learned chunk predictor against its fallbacks, and the CPU oracle
timed on the host cores.
"""
import argparse
import json
import os
import sys
import time
import traceback

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "series·steps/s fwd+adjoint at tol 1e-8 vs chunk=1 sequential; % HBM peak"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
TIMING_TOL = (1e-8, 1e-6)
MLP_F_FLOPS = 2 * (64 * 8 + 64 * 64 + 8 * 64)      # h(y): three layers
MLP_J_FLOPS = 2 * (64 * 64 * 8 + 8 * 64 * 8) + 2 * 64 * 8  # W3 diag W2 diag W1


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def levels(chunk):
    L = 0
    while (1 << L) < chunk:
        L += 1
    return L


def vdp_flops_per_step_iter(chunk):
    """Algorithmic flops of one Newton iteration per series-step (Van der Pol):
    residual, Jacobian, block inverse and update (44) plus one composition of
    2x2 affine maps per reduction level (24 per level, ceil(log2 C) levels)."""
    return 44 + 24 * levels(chunk)


def csrc_hash():
    """Hash of the kernel sources with comments and blank space removed; HBM
    traffic from profiler counters is reported only while the code still
    matches the code the counters were taken from."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2310_08649_amd", "csrc", "*"))):
        with open(p) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        src = " ".join(src.split())
        h.update(os.path.basename(p).encode())
        h.update(src.encode())
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
    """Durations (ms) of `reps` calls of fn, by HIP events on the launching stream."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in evs]


def stats(ds):
    s = sorted(ds)
    return {"mean_ms": sum(s) / len(s), "median_ms": s[len(s) // 2], "min_ms": s[0]}


def extra(out, name, fn):
    """Run one side measurement; a failure is recorded, not fatal to the line."""
    log(name)
    t0 = time.perf_counter()
    try:
        out[name] = fn()
    except Exception as e:  # noqa: BLE001 - the headline must still be printed
        traceback.print_exc()
        out[name] = {"error": "%s: %s" % (type(e).__name__, e)}
    log("%s done in %.1f s" % (name, time.perf_counter() - t0))


# ---------------------------------------------------------------------------
# side measurements
# ---------------------------------------------------------------------------
def run_chunk1(ctx, steps):
    import numpy as np
    from paper_2310_08649_amd import tvi
    y0, times, mu, y_out, B, N = ctx["y0"], ctx["times"], ctx["mu"], ctx["y_out"], ctx["B"], ctx["N"]
    seq = lambda: tvi.solve_forward("vanderpol", y0, times, mu, chunk=1, lanes=1, steps_per_lane=1,
                                    tol=TIMING_TOL, y_out=y_out, iters=False)
    seq()
    d = time_launches(seq, max(3, steps // 3), ctx["stream"])
    ms = float(np.mean(d))
    return {"value": B * N / (ms * 1e-3), "unit": "series*steps/s", "ms_per_step": ms,
            "speedup_of_chunked": ms / ctx["ms_per_step"],
            "note": "same library, chunk 1: one lane per series, one Newton solve per step"}


def run_jacobian_reuse(ctx, steps):
    """The headline workload with chord steps allowed (jacobian_reuse: a correction
    reuses the previous factorization while the residual keeps falling by that
    factor), tuned over chunk, start and factor, against the full-Newton headline."""
    from paper_2310_08649_amd import autotune
    tuned = autotune.tune_forward("vanderpol", ctx["y0"], ctx["times"], ctx["mu"], tol=TIMING_TOL,
                                  chunks=(32, 50, 64, 100), inits=("zero", "extrap"), reuses=(0.1, 0.2, 0.3),
                                  reps=5, y_out=ctx["y_out"], use_cache=False)
    b = tuned["best"]
    fast = min((r for r in tuned["table"] if r["failed"] <= ctx["failed"]), key=lambda r: r["ms"], default=None)
    out = {"fewest_failed": b, "fewest_failed_value": ctx["B"] * ctx["N"] / (b["ms"] * 1e-3),
           "unit": "series*steps/s", "full_newton_ms": ctx["ms_per_step"], "full_newton_failed": ctx["failed"],
           "note": "not the headline: chord steps do less arithmetic per correction than the paper's Newton "
                   "iteration that the roofline counts"}
    if fast is not None:
        out["fastest_no_more_failures"] = fast
        out["fastest_value"] = ctx["B"] * ctx["N"] / (fast["ms"] * 1e-3)
        out["speedup_over_full_newton"] = ctx["ms_per_step"] / fast["ms"]
    return out


def run_vdp_fp32(ctx, steps):
    """The headline workload with float storage (residual, blocks and scans in double)."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import tvi
    f = lambda a: a.to(torch.float32)
    y0, times, mu = f(ctx["y0"]), f(ctx["times"]), f(ctx["mu"])
    y = torch.empty(ctx["y_out"].shape, dtype=torch.float32, device=ctx["dev"])
    res = {}
    for C, S, T in ((ctx["C"], ctx["S"], ctx["T"]), (1, 1, 1)):
        fn = lambda: tvi.solve_forward("vanderpol", y0, times, mu, chunk=C, lanes=S, steps_per_lane=T,
                                       tol=TIMING_TOL, y_out=y, iters=False)
        st = fn()[1]
        ms = float(np.mean(time_launches(fn, max(3, steps // 2), ctx["stream"])))
        res["chunk%d" % C] = {"value": ctx["B"] * ctx["N"] / (ms * 1e-3), "ms": ms,
                              "failed": int((st != 0).sum().item())}
    res["unit"] = "series*steps/s"
    return res


def run_linear(ctx, steps):
    """The linear stiff system, n = 4, 8 series x 200 steps, chunk 20, FP64 (a
    launch-latency-sized problem: one chunk per lane segment, 10 chunks)."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import tvi, workloads
    w = workloads.linear()
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=ctx["dev"])
    y0, times, A = d(w["y0"]), d(w["times"]), d(w["params"])
    B, N = w["y0"].shape[0], w["times"].shape[0] - 1
    y = torch.empty((B, N + 1, 4), dtype=torch.float64, device=ctx["dev"])
    res = {"unit": "series*steps/s"}
    for C in (20, 1):
        fn = lambda: tvi.solve_forward("linear", y0, times, A, chunk=C, tol=TIMING_TOL, y_out=y, iters=False)
        fn()
        ms = float(np.mean(time_launches(fn, 20, ctx["stream"])))
        res["chunk%d" % C] = {"value": B * N / (ms * 1e-3), "ms": ms}
    return res


def run_tiling_study(ctx, steps):
    """PCR against Thomas over the block size n: the linear stiff system (one Newton
    correction per chunk, so the launch is the block work itself), FP64, n = 2, 3, 4,
    for every tiling of chunks of 8 and 64 steps.  S lanes per series run
    ceil(log2 S) PCR levels and each lane runs T steps by the serial (Thomas)
    recurrence; S = 1 is Thomas alone, T = 1 is PCR alone.  Two sizes: 512 series x
    5000 steps (B*S lanes: a narrow tiling leaves most of the chip idle) and 65536
    series x 1000 steps (every tiling fills the chip, so the work per step decides)."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import tvi, workloads
    tilings = ((1, 1, 1), (8, 8, 1), (8, 4, 2), (8, 1, 8), (64, 64, 1), (64, 32, 2), (64, 16, 4), (64, 8, 8))
    res = {"unit": "ms per launch", "workload": "linear, A = -Q diag(10^U(-1,3)) Q^T per series, t=[0,1], FP64"}
    for B, N, reps in ((512, 5000, 10), (65536, 1000, 3)):
        size = {}
        for n in (2, 3, 4):
            w = workloads.linear(B=B, N=N, n=n, seed=110 + n)
            d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=ctx["dev"])
            y0, times, A = d(w["y0"]), d(w["times"]), d(w["params"])
            y = torch.empty((B, N + 1, n), dtype=torch.float64, device=ctx["dev"])
            row = {}
            for C, S, T in tilings:
                fn = lambda: tvi.solve_forward("linear", y0, times, A, chunk=C, lanes=S, steps_per_lane=T,
                                               tol=TIMING_TOL, y_out=y, iters=False)
                st = fn()[1]
                ms = float(np.median(time_launches(fn, reps, ctx["stream"])))
                row["C%d_S%d_T%d" % (C, S, T)] = {"ms": ms, "failed": int((st != 0).sum().item())}
            size["n%d" % n] = row
            del y, y0, times, A
        res["B%d_N%d" % (B, N)] = size
    return res


def run_saturated(ctx, steps):
    """The headline kernel on a batch that fills the chip: 65,536 Van der Pol
    series (mu = 10^U(0,3) as in the headline) x 1000 steps on [0, 2], FP64,
    forward, C = 50 with S = 64, T = 1 and the hybrid tilings; algorithmic
    FP64 flops per second against the vector peak (the same count as the
    headline roofline)."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import tvi, workloads
    w = workloads.vanderpol(B=65536, N=1000, t_end=2.0, seed=121)
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=ctx["dev"])
    y0, times, mu = d(w["y0"]), d(w["times"]), d(w["params"])
    B, N = w["y0"].shape[0], w["times"].shape[0] - 1
    y = torch.empty((B, N + 1, 2), dtype=torch.float64, device=ctx["dev"])
    res = {"workload": "vanderpol B=65536 N=1000 t=[0,2] mu=10^U(0,3) f64 forward", "unit": "series*steps/s"}
    for C, S, T in ((50, 64, 1), (50, 16, 4), (50, 8, 8)):
        fn = lambda: tvi.solve_forward("vanderpol", y0, times, mu, chunk=C, lanes=S, steps_per_lane=T,
                                       tol=TIMING_TOL, y_out=y)
        _, st, it, _ = fn()
        ms = float(np.median(time_launches(fn, 3, ctx["stream"])))
        flops = float(it.sum().item()) * C * vdp_flops_per_step_iter(C)
        tf = flops / (ms * 1e-3) / 1e12
        res["C%d_S%d_T%d" % (C, S, T)] = {"ms": ms, "value": B * N / (ms * 1e-3), "achieved_tflops": tf,
                                         "frac_fp64_peak": tf / PEAK_FP64_TFLOPS,
                                         "failed": int((st != 0).sum().item())}
    del y
    return res


def run_vdp_fwd_adjoint(ctx, steps):
    import torch
    from paper_2310_08649_amd import graph, workloads
    B, N = ctx["B"], ctx["N"]
    obs = torch.zeros((B, N + 1), dtype=torch.uint8)
    obs[:, torch.as_tensor(workloads.observed_steps(N, every=50))] = 1
    res = {"loss": "mean of |y|^2 at 100 sampled steps per series"}
    for recompute in (False, True):
        cs = graph.CapturedStep("vanderpol", ctx["y0"], ctx["times"], ctx["mu"], chunk=ctx["C"], lanes=ctx["S"],
                                steps_per_lane=ctx["T"], tol=TIMING_TOL, init=ctx["init"], loss="mean_square",
                                observed=obs.reshape(-1), recompute=recompute).capture()
        for _ in range(2):
            cs.replay()
        d = time_launches(cs.replay, max(5, steps), torch.cuda.current_stream())
        st = stats(d)
        res["recompute" if recompute else "stored"] = dict(
            value=B * N / (st["mean_ms"] * 1e-3), unit="series*steps/s", **st,
            failed=int(((cs.status_fwd != 0) | (cs.status_adj != 0)).sum().item()),
            states="recomputed from chunk checkpoints" if recompute else "read from the stored trajectory")
        del cs
    return res


def run_pcr(ctx, steps):
    import numpy as np
    import torch
    from paper_2310_08649_amd import tvi
    dev = ctx["dev"]
    res = []
    target = 4 << 30
    for dt, n in ((torch.float64, 2), (torch.float64, 3), (torch.float64, 4), (torch.float32, 2),
                  (torch.float32, 4)):
        m = 64
        es = torch.finfo(dt).bits // 8
        per_sys = m * (n * n + 2 * n) * es
        nb = target // per_sys
        gen = torch.Generator(device=dev)
        gen.manual_seed(5)
        D = torch.eye(n, dtype=dt, device=dev).expand(nb, m, n, n).contiguous()
        D.add_(torch.randn(D.shape, generator=gen, dtype=dt, device=dev), alpha=0.2 / n)
        r = torch.randn((nb, m, n), generator=gen, dtype=dt, device=dev)
        x = torch.empty_like(r)
        fn = lambda: tvi.pcr_solve(D, r, out=x)
        fn()
        d = time_launches(fn, 10, ctx["stream"])
        ms = float(np.mean(d))
        gbs = nb * per_sys / (ms * 1e-3) / 1e9
        res.append({"n": n, "dtype": "f64" if dt == torch.float64 else "f32", "systems": int(nb), "block_rows": m,
                    "bytes_per_launch": int(nb * per_sys), "avg_launch_ms": ms, "achieved": gbs,
                    "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS})
        del D, r, x
        torch.cuda.empty_cache()
    best = res[0]
    pname = "tvi::pcr_kernel<2, double, 64, 1, false>(long, int, double const*, double const*, double*)"
    return {"kernel": pname, "bound": "hbm", "achieved": best["achieved"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": best["frac"], "traffic": measured_traffic(pname), "bytes_per_launch": best["bytes_per_launch"],
            "avg_launch_ms": best["avg_launch_ms"], "systems": best["systems"], "block_rows": 64, "n": 2,
            "sweep": res}


def run_mlp(ctx, steps):
    """Neural ODE n = 8, 2 x 64 tanh, 64 series x 1e4 steps, chunk 100, FP32,
    forward + adjoint of the mean squared state at 100 sampled times."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import graph, tvi, workloads
    dev = ctx["dev"]
    w = workloads.mlp()
    B, N, C = w["y0"].shape[0], w["times"].shape[0] - 1, 100
    f = lambda a: torch.as_tensor(a, dtype=torch.float32, device=dev)
    y0, times, theta = f(w["y0"]), f(w["times"]), f(w["params"])
    obs = torch.zeros((B, N + 1), dtype=torch.uint8)
    obs[:, torch.as_tensor(workloads.observed_steps(N))] = 1
    cs = graph.CapturedStep("mlp", y0, times, theta, chunk=C, tol=TIMING_TOL, loss="mean_square",
                            observed=obs.reshape(-1), recompute=True).capture()
    cs.replay()
    d = time_launches(cs.replay, max(3, steps // 2), torch.cuda.current_stream())
    st = stats(d)
    corrections = int(cs.iters.sum().item())
    failed = int(((cs.status_fwd != 0) | (cs.status_adj != 0)).sum().item())
    # forward kernel alone, and its matrix-core work
    fwd = lambda: tvi.solve_forward("mlp", y0, times, theta, chunk=C, tol=TIMING_TOL, y_out=cs.y,
                                    checkpoints=False, iters=False)
    fwd()
    fms = float(np.mean(time_launches(fwd, 3, ctx["stream"])))
    attempts = B * (N // C)
    # every trip evaluates h on the attempt's steps; every correction also evaluates J
    flops = (corrections + attempts) * C * MLP_F_FLOPS + corrections * C * MLP_J_FLOPS
    tf = flops / (fms * 1e-3) / 1e12
    # the same step with the adjoint reading the stored trajectory
    cs2 = graph.CapturedStep("mlp", y0, times, theta, chunk=C, tol=TIMING_TOL, loss="mean_square",
                             observed=obs.reshape(-1), recompute=False).capture()
    cs2.replay()
    st2 = stats(time_launches(cs2.replay, max(3, steps // 2), torch.cuda.current_stream()))
    # a batch that fills the chip: 1024 series (four workgroups per CU), 1000 steps of the same
    # length (1e-4), forward
    wb = workloads.mlp(B=1024, N=1000, seed=131, t_end=0.1)
    yb0, tb, thb = f(wb["y0"]), f(wb["times"]), f(wb["params"])
    Bb, Nb = wb["y0"].shape[0], wb["times"].shape[0] - 1
    yb = torch.empty((Bb, Nb + 1, wb["n"]), dtype=torch.float32, device=dev)
    fb = lambda: tvi.solve_forward("mlp", yb0, tb, thb, chunk=C, tol=TIMING_TOL, y_out=yb, checkpoints=False)
    _, stb, itb, _ = fb()
    bms = float(np.median(time_launches(fb, 3, ctx["stream"])))
    corr_b = float(itb.sum().item())
    tfb = ((corr_b + Bb * (Nb // C)) * C * MLP_F_FLOPS + corr_b * C * MLP_J_FLOPS) / (bms * 1e-3) / 1e12
    saturated = {"workload": "mlp n=8 H=64 tanh B=1024 N=1000 t=[0,0.1] chunk=100 f32 forward",
                 "ms": bms, "value": Bb * Nb / (bms * 1e-3), "achieved_tflops": tfb,
                 "frac_bf16_peak": tfb / PEAK_BF16_TFLOPS, "failed": int((stb != 0).sum().item())}
    del yb
    return {"workload": "mlp n=8 H=64 tanh B=64 N=10000 t=[0,1] chunk=100 f32 (bf16-split MFMA) "
                        "fwd+adjoint, mean-square loss at 100 sampled times, states recomputed",
            "value": B * N / (st["mean_ms"] * 1e-3), "unit": "series*steps/s", **st,
            "stored_trajectory_value": B * N / (st2["mean_ms"] * 1e-3),
            "forward_ms": fms, "forward_value": B * N / (fms * 1e-3), "newton_corrections": corrections,
            "failed": failed, "chip_filling_forward": saturated,
            "roofline": {"kernel": "tvi::mlp_forward_kernel<float, false>", "bound": "mfma", "achieved": tf,
                         "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_BF16_TFLOPS,
                         "flops_counted": "h: %d per step per Newton trip, J: %d per step per correction "
                                          "(useful products, not the bf16 split)" % (MLP_F_FLOPS, MLP_J_FLOPS)}}


def run_forward_euler(ctx, steps):
    """The explicit scheme (Eq. forward-euler) solved in chunks by the same Newton
    and scan kernels: Van der Pol 512 x 5000 FP64 on [0, 10] with mu = 10^U(0,1)
    (steps stable for forward Euler), forward, chunk swept against chunk 1; and
    the neural ODE 64 x 1e4 FP32, chunk 100, forward + adjoint of the mean
    squared state at 100 sampled times as one captured graph."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import graph, tvi, workloads
    dev = ctx["dev"]
    res = {"unit": "series*steps/s"}
    w = workloads.vanderpol(mu_range=(1.0, 10.0), seed=120)
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    y0, times, mu = d(w["y0"]), d(w["times"]), d(w["params"])
    B, N = w["y0"].shape[0], w["times"].shape[0] - 1
    y = torch.empty((B, N + 1, 2), dtype=torch.float64, device=dev)
    vdp = {}
    for C in (1, 16, 32, 64, 128, 256):
        fn = lambda: tvi.solve_forward("vanderpol", y0, times, mu, chunk=C, tol=TIMING_TOL, y_out=y, iters=False,
                                       scheme="forward_euler", **({"lanes": 1, "steps_per_lane": 1} if C == 1 else {}))
        st = fn()[1]
        ms = float(np.median(time_launches(fn, max(3, steps // 2), ctx["stream"])))
        vdp["chunk%d" % C] = {"value": B * N / (ms * 1e-3), "ms": ms, "failed": int((st != 0).sum().item())}
    best = min((v["ms"], k) for k, v in vdp.items() if k != "chunk1" and v["failed"] == 0)
    vdp["speedup_of_best_over_chunk1"] = vdp["chunk1"]["ms"] / best[0]
    res["vanderpol_forward"] = vdp
    del y
    wm = workloads.mlp()
    f = lambda a: torch.as_tensor(a, dtype=torch.float32, device=dev)
    Bm, Nm = wm["y0"].shape[0], wm["times"].shape[0] - 1
    obs = torch.zeros((Bm, Nm + 1), dtype=torch.uint8)
    obs[:, torch.as_tensor(workloads.observed_steps(Nm))] = 1
    mlp = {}
    for C in (100, 1):
        cs = graph.CapturedStep("mlp", f(wm["y0"]), f(wm["times"]), f(wm["params"]), chunk=C, tol=TIMING_TOL,
                                loss="mean_square", observed=obs.reshape(-1), recompute=True,
                                scheme="forward_euler").capture()
        cs.replay()
        st = stats(time_launches(cs.replay, 3, torch.cuda.current_stream()))
        mlp["chunk%d" % C] = dict(value=Bm * Nm / (st["mean_ms"] * 1e-3), **st,
                                  failed=int(((cs.status_fwd != 0) | (cs.status_adj != 0)).sum().item()))
        del cs
    res["mlp_forward_adjoint"] = mlp
    return res


def run_paper_grid(ctx, steps):
    """The paper's chunk-efficiency study (Section 5.3, its parameter table) on
    its Chaboche (1 to 5 backstresses) and coupled-neuron (1 and 2 neurons) example
    problems, FP64: n_time = 2000, n_batch in {3, 10, 30, 50}, chunks
    {1, 3, 10, 30, 100, 300, 512} (512 is the longest chunk here; the paper's
    grid ends at 1000; 3-5 backstresses and 2 neurons run one step per lane,
    chunks up to 64), forward + adjoint of the Frobenius loss of the whole
    trajectory as one captured graph (states read from the stored trajectory).
    Each chunk runs with PCR across lanes (T = 1 up to 64 steps) and with the
    PCR->Thomas hybrid at T = 8; the speed-up is chunk 1 against the best."""
    import torch
    from paper_2310_08649_amd import graph, workloads
    dev = ctx["dev"]
    out = {"unit": "ms per forward+adjoint", "paper_best_speedup": {"chaboche": 190, "neuron": 94}}
    best_by_model = {}
    for kind, nu in (("chaboche", 1), ("chaboche", 2), ("chaboche", 3), ("chaboche", 4), ("chaboche", 5),
                     ("neuron", 1), ("neuron", 2)):
        big = (kind == "chaboche" and nu >= 3) or (kind == "neuron" and nu >= 2)  # one step per lane: C <= 64
        for nb in (3, 10, 30, 50):
            w = getattr(workloads, kind)(nu, nb)
            d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
            row = {}
            for C in ((1, 3, 10, 30, 64) if big else (1, 3, 10, 30, 100, 300, 512)):
                tilings = [(1, 1)] if C == 1 else [(0, 0)] + ([(-(-C // 8), 8)] if C >= 32 and not big else [])
                for S, T in tilings:
                    if S > 64:
                        continue
                    S2 = S if S in (0, 1) else max(4, 1 << (S - 1).bit_length())
                    cs = graph.CapturedStep(kind, d(w["y0"]), d(w["times"]), d(w["params"]), chunk=C, lanes=S2,
                                            steps_per_lane=T, tol=TIMING_TOL, loss="frobenius",
                                            recompute=False).capture()
                    cs.replay()
                    st = stats(time_launches(cs.replay, 3, torch.cuda.current_stream()))
                    failed = int(((cs.status_fwd != 0) | (cs.status_adj != 0)).sum().item())
                    key = "C%d" % C + ("" if T in (0, 1) else "_T%d" % T)
                    row[key] = {"ms": st["median_ms"], "failed": failed}
                    del cs
            ok = {k: v["ms"] for k, v in row.items() if v["failed"] == 0}
            bk = min(ok, key=ok.get)
            sp = row["C1"]["ms"] / ok[bk]
            row["best"] = {"config": bk, "ms": ok[bk], "speedup_over_chunk1": sp}
            out["%s_nu%d_B%d" % (kind, nu, nb)] = row
            best_by_model[kind] = max(best_by_model.get(kind, 0.0), sp)
    out["best_speedup"] = best_by_model
    return out


def run_forward_ad(ctx, steps):
    """The state Jacobian by forward-mode AD (one evaluation of the rate on dual
    numbers) against the hand-written one, FP64, same chunk and tiling: the
    headline Van der Pol forward; the linear system n = 4 (512 x 5000, C = 64);
    Robertson (2000 ragged series, C = 256, longest first, forward); the paper's
    Chaboche (2 backstresses) and neuron problems at n_batch = 50, C = 100,
    forward + adjoint.  The paper reports AD at 2-8x the analytic cost (Section 5.4)."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import graph, tvi, workloads
    dev = ctx["dev"]
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    res = {"unit": "ms per launch (forward) or per forward+adjoint graph"}

    def pair(fn_of_jac, reps):
        out = {}
        for jac in ("analytic", "forward_ad"):
            fn = fn_of_jac(jac)
            fn()
            out[jac] = float(np.median(time_launches(fn, reps, ctx["stream"])))
        out["ad_over_analytic"] = out["forward_ad"] / out["analytic"]
        return out

    res["vanderpol"] = pair(lambda jac: lambda: tvi.solve_forward(
        "vanderpol", ctx["y0"], ctx["times"], ctx["mu"], chunk=ctx["C"], lanes=ctx["S"], steps_per_lane=ctx["T"],
        tol=TIMING_TOL, init=ctx["init"], y_out=ctx["y_out"], iters=False, jacobian=jac), max(3, steps // 2))
    # inputs resident on the device before the timed launches
    w = workloads.linear(B=512, N=5000, n=4, seed=114)
    yl = torch.empty((512, 5001, 4), dtype=torch.float64, device=dev)
    la = (d(w["y0"]), d(w["times"]), d(w["params"]))
    res["linear_n4"] = pair(lambda jac: lambda: tvi.solve_forward(
        "linear", *la, chunk=64, tol=TIMING_TOL, y_out=yl, iters=False, jacobian=jac), 5)
    del yl, la
    w = workloads.robertson()
    off = torch.as_tensor(w["offsets"], device=dev)
    order = tvi.order_longest_first(off)
    yr = torch.empty((w["times"].shape[0], 3), dtype=torch.float64, device=dev)
    ra = (d(w["y0"]), d(w["times"]), d(w["params"]))
    res["robertson"] = pair(lambda jac: lambda: tvi.solve_forward(
        "robertson", *ra, offsets=off, chunk=256, lanes=64, steps_per_lane=4, tol=TIMING_TOL, y_out=yr,
        iters=False, order=order, jacobian=jac, n_max=int(w["steps"].max())), 3)
    del yr, ra
    for kind, nu in (("chaboche", 2), ("neuron", 1)):
        w = getattr(workloads, kind)(nu, 50)
        row = {}
        for jac in ("analytic", "forward_ad"):
            cs = graph.CapturedStep(kind, d(w["y0"]), d(w["times"]), d(w["params"]), chunk=100, tol=TIMING_TOL,
                                    loss="frobenius", recompute=False, jacobian=jac).capture()
            cs.replay()
            row[jac] = stats(time_launches(cs.replay, 5, torch.cuda.current_stream()))["median_ms"]
            del cs
        row["ad_over_analytic"] = row["forward_ad"] / row["analytic"]
        res["%s_nu%d" % (kind, nu)] = row
    return res


def run_robertson(ctx, steps):
    """2000 ragged Robertson series (100..20000 log-spaced steps), FP64,
    forward + adjoint (Frobenius loss) as one captured graph, with the
    adjoint's states recomputed from checkpoints or read from the stored
    trajectory; chunk, tiling and start autotuned for each pair."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import autotune, graph, tvi, workloads
    dev = ctx["dev"]
    w = workloads.robertson()
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    y0, times, sp = d(w["y0"]), d(w["times"]), d(w["params"])
    off = torch.as_tensor(w["offsets"], device=dev)
    total = int(w["steps"].sum())
    y_out = torch.empty((times.shape[0], 3), dtype=torch.float64, device=dev)
    order = tvi.order_longest_first(off)  # ragged series launch longest first
    tune = lambda adjoint: autotune.tune_forward("robertson", y0, times, sp, offsets=off, tol=TIMING_TOL,
                                                 y_out=y_out, use_cache=False, chunks=(16, 32, 64, 128, 256),
                                                 inits=("zero", "extrap"), adjoint=adjoint, order=order,
                                                 n_max=int(w["steps"].max()))["best"]
    res = {"workload": "robertson n=3 B=2000 ragged N_b=exp U(ln 100, ln 2e4) log-spaced t=[1e-5,1e4] f64 "
                       "fwd+adjoint (Frobenius loss), one captured graph, series launched longest first",
           "series_steps": total}
    for mode in ("recompute", "stored"):
        b = tune(mode)
        cs = graph.CapturedStep("robertson", y0, times, sp, offsets=off, chunk=b["chunk"], lanes=b["lanes"],
                                steps_per_lane=b["steps_per_lane"], tol=TIMING_TOL, init=b["init"],
                                loss="frobenius", recompute=mode == "recompute").capture()
        cs.replay()
        st = stats(time_launches(cs.replay, max(3, steps // 2), torch.cuda.current_stream()))
        res[mode] = dict(value=total / (st["mean_ms"] * 1e-3), unit="series*steps/s", **st, tuned=b,
                         failed=int(((cs.status_fwd != 0) | (cs.status_adj != 0)).sum().item()))
        del cs
    res["value"] = res["recompute"]["value"]
    res["unit"] = "series*steps/s"
    b = tune(None)
    nmax = int(w["steps"].max())
    fwd = lambda: tvi.solve_forward("robertson", y0, times, sp, offsets=off, chunk=b["chunk"], lanes=b["lanes"],
                                    steps_per_lane=b["steps_per_lane"], tol=TIMING_TOL, init=b["init"],
                                    y_out=y_out, iters=False, order=order, n_max=nmax)
    seq = lambda: tvi.solve_forward("robertson", y0, times, sp, offsets=off, chunk=1, lanes=1, steps_per_lane=1,
                                    tol=TIMING_TOL, y_out=y_out, iters=False, order=order, n_max=nmax)
    fms = float(np.mean(time_launches(fwd, 3, ctx["stream"])))
    seq()
    sms = float(np.mean(time_launches(seq, 3, ctx["stream"])))
    ctx["rob_tuned"] = b
    res.update(forward_value=total / (fms * 1e-3), forward_tuned=b, chunk1_forward_value=total / (sms * 1e-3),
               forward_speedup_over_chunk1=sms / fms)
    return res


def run_predictor(ctx, steps):
    """Learned chunk predictor on the neural ODE: trained on ~1e5 chunks the
    solver computed (500 series x 1e4 steps, chunk 50), evaluated on 256 new
    series x 1e4 steps against the extrapolated and the zero start."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import predictor as pred
    from paper_2310_08649_amd import tvi, workloads
    dev = ctx["dev"]
    C = 50
    f = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float32, device=dev)
    theta = f(workloads.mlp(B=1, seed=103)["params"])
    times = f(np.linspace(0.0, 1.0, 10001))
    tr_y0 = f(np.random.default_rng(105).standard_normal((500, 8)))
    ev_y0 = f(np.random.default_rng(107).standard_normal((256, 8)))
    t0 = time.perf_counter()
    y, st, _, _ = tvi.solve_forward("mlp", tr_y0, times, theta, chunk=C, tol=TIMING_TOL, init="extrap")
    x, inc, dts = pred.chunk_samples(y, times, C)
    ok = torch.isfinite(inc).all(dim=1) & torch.isfinite(x).all(dim=1)
    x, inc, dts = x[ok].contiguous(), inc[ok].contiguous(), dts[ok].contiguous()
    p = pred.corrections("mlp", x, inc, dts, theta, 8)
    d = pred.dims(8, C)
    net, hist = pred.fit_predictor(d, x, p, epochs=30, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = {"train_chunks": int(x.shape[0]), "train_seconds": t_train, "train_loss": [hist[0], hist[-1]]}
    y_ref = None
    for init in ("zero", "extrap", "predictor"):
        kw = dict(predictor=pred.solver_args(d, net, 8, base=1)) if init == "predictor" else {}
        fn = lambda: tvi.solve_forward("mlp", ev_y0, times, theta, chunk=C, tol=TIMING_TOL, init=init, **kw)
        yy, stt, it, _ = fn()
        ms = float(np.mean(time_launches(fn, 3, ctx["stream"])))
        if y_ref is None:
            y_ref = yy.clone()
        res[init] = {"newton_corrections": int(it.sum().item()), "ms": ms,
                     "failed": int((stt != 0).sum().item()),
                     "max_rel_diff_vs_zero_start": float(((yy - y_ref).abs().max() / y_ref.abs().max()).item())}
    # initial-iterate error against the converged chunks of the evaluation set
    xe, ie, de = pred.chunk_samples(y_ref, times, C)
    ext = pred.extrapolated("mlp", xe, de, theta, 8)
    res["initial_iterate_mse"] = {"zero": float((ie ** 2).mean().item()),
                                  "extrap": float(((ext - ie) ** 2).mean().item()),
                                  "predictor": float(((ext + pred.forward(d, net, xe) - ie) ** 2).mean().item())}
    out = {"mlp": res}
    try:
        out["robertson"] = _predictor_robertson(ctx)
    except Exception as e:  # noqa: BLE001
        traceback.print_exc()
        out["robertson"] = {"error": "%s: %s" % (type(e).__name__, e)}
    return out


def _predictor_robertson(ctx):
    """The same on the stiff kinetics: trained on ~1e5 chunks of 2000 other
    ragged series, evaluated on the benchmark's ragged batch at its tuned
    chunk and tiling."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import predictor as pred
    from paper_2310_08649_amd import tvi, workloads
    dev = ctx["dev"]
    b = ctx.get("rob_tuned") or {"chunk": 64, "lanes": 64, "steps_per_lane": 1}
    C, S, T = b["chunk"], b["lanes"], b["steps_per_lane"]
    d64 = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    tr = workloads.robertson(seed=106)
    off = torch.as_tensor(tr["offsets"], device=dev)
    y, st, _, _ = tvi.solve_forward("robertson", d64(tr["y0"]), d64(tr["times"]), d64(tr["params"]), offsets=off,
                                    chunk=C, lanes=S, steps_per_lane=T, tol=TIMING_TOL)
    x, ys, inc, dts, series = pred.chunk_samples_ragged(y, d64(tr["times"]), off, C)
    ok = torch.isfinite(inc).all(dim=1)
    d = pred.dims(3, C)
    # corrections to the zero start: on log-spaced grids the extrapolation overshoots
    net, hist = pred.fit_predictor(d, x[ok].contiguous(), inc[ok].float().contiguous(), epochs=20, seed=0)
    torch.cuda.synchronize()
    res = {"chunk": C, "lanes": S, "steps_per_lane": T, "base": "zero", "train_chunks": int(ok.sum().item()),
           "train_seconds": time.perf_counter() - t0, "train_loss": [hist[0], hist[-1]]}
    ev = workloads.robertson()
    eoff = torch.as_tensor(ev["offsets"], device=dev)
    args = (d64(ev["y0"]), d64(ev["times"]), d64(ev["params"]))
    y_ref = None
    for key in ("zero", "extrap", "predictor", "extrap_zero_reference"):
        init = key.split("_")[0]
        kw = dict(predictor=pred.solver_args(d, net, 3, base=0)) if init == "predictor" else {}
        if key.endswith("zero_reference"):
            kw["reference"] = "zero"  # Algorithm 1's n0: a better start may stop sooner
        fn = lambda: tvi.solve_forward("robertson", *args, offsets=eoff, chunk=C, lanes=S, steps_per_lane=T,
                                       tol=TIMING_TOL, init=init, n_max=int(ev["steps"].max()), **kw)
        yy, stt, it, _ = fn()
        ms = float(np.mean(time_launches(fn, 3, ctx["stream"])))
        if y_ref is None:
            y_ref = yy.clone()
        res[key] = {"newton_corrections": int(it.sum().item()), "newton_corrections_max": int(it.max().item()),
                    "ms": ms, "failed": int((stt != 0).sum().item())}
    xe, yse, ie, de, se = pred.chunk_samples_ragged(y_ref, args[1], eoff, C)
    pe = pred.corrections_at("robertson", yse, ie, de, args[2][se].contiguous())
    res["initial_iterate_mse"] = {"zero": float((ie ** 2).mean().item()),
                                  "extrap": float((pe.double() ** 2).mean().item()),
                                  "predictor": float(((ie - pred.forward(d, net, xe).double()) ** 2).mean().item())}
    return res


def run_cpu_baseline(w, target_s=10.0):
    import oracle
    B, N = w["y0"].shape[0], w["times"].shape[0] - 1
    threads = oracle.default_threads()
    reps, t = 0, 0.0
    t0 = time.perf_counter()
    while t < target_s and reps < 5000:
        oracle.forward("vanderpol", w["y0"], w["times"], w["params"], tol=TIMING_TOL, threads=threads)
        reps += 1
        t = time.perf_counter() - t0
    # one core on a slice of the series
    sl = slice(0, 64)
    reps1, t1 = 0, 0.0
    t0 = time.perf_counter()
    while t1 < target_s / 4 and reps1 < 500:
        oracle.forward("vanderpol", w["y0"][sl], w["times"], w["params"][sl], tol=TIMING_TOL, threads=1)
        reps1 += 1
        t1 = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": reps * B * N / t, "unit": "series*steps/s", "cores": threads, "kind": "oracle",
            "sample": "the full workload (512 x 5000, forward) solved %d times in %.1f s, sequential backward "
                      "Euler with a dense Newton solve per step" % (reps, t),
            "one_core_value": reps1 * 64 * N / t1, "cpu_model": cpu, "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=0, help="0 = autotune")
    ap.add_argument("--init", default="", help="initial iterate (zero | extrap); empty = autotune")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline measurement")
    ap.add_argument("--only", default="", help="comma-separated side measurements to run")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (series are independent and "
              "would shard across GPUs, each running the same kernels on its share)", file=sys.stderr)
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

    # ---- autotune chunk length, tiling and initial iterate (untimed)
    log("autotuning chunk / tiling / initial iterate")
    tuned = autotune.tune_forward("vanderpol", y0, times, mu, tol=TIMING_TOL, y_out=y_out, use_cache=False,
                                  chunks=(10, 16, 32, 50, 64, 100, 128, 200, 256, 500) if args.chunk == 0
                                  else (args.chunk,),
                                  inits=("zero", "extrap") if not args.init else (args.init,))
    best = tuned["best"]
    C, S, T, init = best["chunk"], best["lanes"], best["steps_per_lane"], best["init"]
    log("chosen chunk=%d lanes=%d steps_per_lane=%d init=%s (%.3f ms)" % (C, S, T, init, best["ms"]))

    def step():
        return tvi.solve_forward("vanderpol", y0, times, mu, chunk=C, lanes=S, steps_per_lane=T, tol=TIMING_TOL,
                                 y_out=y_out, init=init)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, status, iters, _ = step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    peak_mem = torch.cuda.max_memory_allocated()  # every device buffer is the caller's (torch)
    value = B * N / (ms_per_step * 1e-3)
    st = status.cpu().numpy()
    it = iters.cpu().numpy()
    durs = time_launches(step, args.steps, stream)
    kst = stats(durs)
    kern_ms = kst["mean_ms"]

    flops = float(it.sum()) * C * vdp_flops_per_step_iter(C)
    achieved_tflops = flops / (kern_ms * 1e-3) / 1e12
    kname = "tvi::forward_kernel<tvi::VanDerPol, double, %d, %d, %s, false, false, false>" % (
        S, T, "true" if init == "predictor" else "false")
    roofline = {"kernel": kname, "bound": "alu",
                "achieved": achieved_tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tflops / PEAK_FP64_TFLOPS, "traffic": measured_traffic(kname),
                "avg_launch_ms": kern_ms, "median_launch_ms": kst["median_ms"], "min_launch_ms": kst["min_ms"],
                "algorithmic_bytes_per_launch": B * (N + 1) * 2 * 8,
                "note": "latency-bound: each series is a chain of N/C chunk solves x Newton iterations; "
                        "the slowest series sets the launch time"}

    out = {"metric": METRIC, "value": value, "unit": "series*steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "vanderpol n=2 B=512 N=5000 t=[0,10] mu=10^U(0,3) y0=U(-2,2) forward "
                                  "tol_a=1e-8 tol_r=1e-6", "chunk": C, "lanes": S, "steps_per_lane": T,
                      "init": init, "series_failed": int((st != 0).sum()),
                      "newton_iters_per_series": float(it.mean()), "newton_iters_max": int(it.max())},
           "peak_device_memory_bytes": int(peak_mem),
           "roofline": roofline, "autotune": tuned["table"]}

    ctx = dict(dev=dev, stream=stream, y0=y0, times=times, mu=mu, y_out=y_out, B=B, N=N, C=C, S=S, T=T, init=init,
               ms_per_step=ms_per_step, failed=int((st != 0).sum()))
    if not args.no_extras:
        runs = [("chunk1", run_chunk1), ("jacobian_reuse", run_jacobian_reuse), ("fp32", run_vdp_fp32), ("fwd_adjoint", run_vdp_fwd_adjoint),
                ("linear", run_linear), ("tiling_study", run_tiling_study), ("saturated", run_saturated),
                ("pcr_roofline", run_pcr),
                ("mlp", run_mlp), ("robertson", run_robertson), ("predictor", run_predictor),
                ("forward_euler", run_forward_euler), ("paper_grid", run_paper_grid),
                ("forward_ad", run_forward_ad)]
        only = set(filter(None, args.only.split(",")))
        for name, fn in runs:
            if not only or name in only:
                extra(out, name, lambda fn=fn: fn(ctx, args.steps))

    if args.probe_copy:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
        del src, dst

    if not args.no_cpu:
        log("CPU oracle on the host cores")
        out["cpu_baseline"] = run_cpu_baseline(w)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
