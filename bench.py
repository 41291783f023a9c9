#!/usr/bin/env python3
"""Benchmark of the chunked backward-Euler solver and its adjoint on one MI355X.

Headline workload: the ragged stiff-kinetics batch.  2000 Robertson series
(n = 3; rate constants 0.04 s1, 3e7 s2, 1e4 s3 with s_i = 10^U(log 0.5, log 2)),
N_b = round(exp U(ln 100, ln 20000)) log-spaced steps on t in [1e-5, 1e4],
y0 = (1, 0, 0), FP64, the paper's tolerances (tol_a 1e-8, tol_r 1e-6).  One
step of the benchmark is one replay of a captured HIP graph holding the whole
training step: the chunked forward solve, the gradient of the Frobenius loss
L = sqrt(sum y^2) over every output (the timing loss of Section 5.2), and the
discrete adjoint (Appendix A) with dL/dp and dL/dy0, series launched longest
first.  Chunk length, lane tiling, initial iterate and the adjoint's state
source (stored trajectory or recomputation from checkpoints) come from the
autotuner, run before timing.  Inputs are resident in HBM.

The last stdout line is one compact JSON object: throughput in series*steps/s
(only steps of series whose forward and adjoint both succeeded), the same
graph at chunk = 1 (the sequential GPU baseline: one lane per series, one
Newton solve per step), the roofline of the dominant kernel (timed with HIP
events on its launch stream), and the CPU oracle timed on the host cores.
Further measurements (Van der Pol, the neural ODE, the standalone
block-bidiagonal solve, the tiling study, the paper's example problems, the
learned predictor) run only with --extras FILE and are written to FILE.
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
COPY_PROBE_BYTES = 1 << 28  # the plain device copy that calibrates the HBM byte counters
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


# Robertson (n = 3) per-step flop counts: an affine-map composition
# (F = Fa + Fb + Fa Fb, z = (I + Fa) zb + za) and the block factorization
# (inverse and z = -M r) are 2 n^3 + 2 n^2 = 72 each; the residual (rates 8,
# state 3, residual 9, squared norm 6) 26; the Jacobian and D = I - dt j 24;
# a replay (I + F) x + z 24; the parameter product (dh/dp)^T w and dt lam 12.
ROB_LEVEL, ROB_FACT, ROB_RES, ROB_JAC, ROB_REPLAY, ROB_VJP = 72, 72, 26, 24, 24, 12


def _lane_levels(S):
    """Map compositions per lane of the reduction across S lanes: log2(S) within a
    wave; across waves (S > 64) the value entering a wave is applied to each
    lane's composed map instead (ROB_REPLAY flops, no composition)."""
    return levels(min(S, 64)), (ROB_REPLAY if S > 64 else 0)


def rob_forward_flops_per_step(S, T):
    """Algorithmic flops per series-step of one Newton correction of the hybrid
    PCR/Thomas solve (Section 3.3): residual, Jacobian, factorization, the
    lane's serial compositions (T - 1 per T steps) and log2(S) reduction levels
    per lane (shared by its T steps), and the replay when T > 1."""
    lv, cross = _lane_levels(S)
    return (ROB_RES + ROB_JAC + ROB_FACT + (ROB_LEVEL * ((T - 1) + lv) + cross) / T
            + (ROB_REPLAY if T > 1 else 0))


def rob_adjoint_flops_per_step(S, T):
    """Per series-step of the adjoint (one transposed solve, no Newton loop):
    Jacobian, factorization, compositions and levels as above, the replay and
    the parameter product."""
    lv, cross = _lane_levels(S)
    return ROB_JAC + ROB_FACT + (ROB_LEVEL * ((T - 1) + lv) + cross) / T + ROB_REPLAY + ROB_VJP


def csrc_hash(files=None):
    """Hash of kernel sources (comments and blank space removed): all of csrc,
    or the listed basenames.  HBM traffic from profiler counters is reported
    only while the sources the kernel is built from still match."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    paths = sorted(glob.glob(os.path.join(ROOT, "paper_2310_08649_amd", "csrc", "*")))
    if files is not None:
        want = set(files)
        paths = [p for p in paths if os.path.basename(p) in want]
    for p in paths:
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
    if not rec or rec.get("source_hash") != csrc_hash(rec.get("sources")):
        return None
    return rec["bytes_per_dispatch"]


# Files each solver kernel is built from: its traffic record goes stale when one changes
# (the first key found in the kernel's name decides; no key: every source file).
WIDE_SOURCES = ["wide.hpp", "model_robertson_wide.hip", "model_vanderpol_wide.hip", "solver.hpp", "device.hpp",
                "models.hpp", "dual.hpp", "dispatch.hpp"]
KERNEL_SOURCES = {"wide::": WIDE_SOURCES,
                  "Robertson": ["model_robertson.hip", "solver.hpp", "device.hpp", "models.hpp", "dual.hpp",
                                "dispatch.hpp"],
                  "VanDerPol": ["model_vanderpol.hip", "solver.hpp", "device.hpp", "models.hpp", "dual.hpp",
                                "dispatch.hpp"],
                  "pcr_kernel": ["pcr.hip", "device.hpp", "solver.hpp", "models.hpp", "dual.hpp", "dispatch.hpp"]}


def _counter_rows(path):
    """(kernel name, dispatch id, counter value) from a rocprofv3 counter_collection.csv
    (the file itself, or the directory it was written under)."""
    import csv
    import glob
    if os.path.isdir(path):
        found = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
        if not found:
            raise FileNotFoundError("no counter_collection.csv under " + path)
        path = found[0]
    out = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            if name.startswith("void "):
                name = name[5:]
            out.append((name, r.get("Dispatch_Id", r.get("Correlation_Id")), float(r["Counter_Value"])))
    return out


def record_traffic(fetch_path, write_path, copy_bytes):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs of the same command
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  Each counter is scaled by what
    it reads for the plain device copy of copy_bytes bytes in the same run (the
    largest __amd_rocclr_copyBuffer dispatch): bytes = KiB * 1024 * scale."""
    def per_kernel(rows):
        acc = {}
        for name, disp, v in rows:
            acc.setdefault(name, {}).setdefault(disp, 0.0)
            acc[name][disp] += v  # counters summed over the dispatch's instances
        return {k: list(d.values()) for k, d in acc.items()}
    fetch, write = per_kernel(_counter_rows(fetch_path)), per_kernel(_counter_rows(write_path))
    copy = "__amd_rocclr_copyBuffer"
    f_scale = copy_bytes / (max(fetch[copy]) * 1024.0)
    w_scale = copy_bytes / (max(write[copy]) * 1024.0)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        table = {}
    # records of earlier runs stay while their kernel's sources still match
    table = {k: v for k, v in table.items() if v.get("source_hash") == csrc_hash(v.get("sources"))}
    for name in fetch:
        if name not in write or not name.startswith("tvi::"):
            continue
        srcs = next((v for k, v in KERNEL_SOURCES.items() if k in name), None)
        fv, wv = fetch[name], write[name]
        table[name] = {"bytes_per_dispatch": (sum(fv) / len(fv) * f_scale + sum(wv) / len(wv) * w_scale) * 1024.0,
                       "fetch_kib": sum(fv) / len(fv), "write_kib": sum(wv) / len(wv), "dispatches": len(fv),
                       "fetch_scale": f_scale, "write_scale": w_scale, "sources": srcs,
                       "source_hash": csrc_hash(srcs)}
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    return table


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
    """Run one side measurement; a failure is recorded, not fatal."""
    log(name)
    t0 = time.perf_counter()
    try:
        out[name] = fn()
    except Exception as e:  # noqa: BLE001 - the headline must still be printed
        traceback.print_exc()
        out[name] = {"error": "%s: %s" % (type(e).__name__, e)}
    log("%s done in %.1f s" % (name, time.perf_counter() - t0))


# ---------------------------------------------------------------------------
# headline: ragged Robertson, forward + loss gradient + adjoint, one graph
# ---------------------------------------------------------------------------
def rob_inputs(dev):
    import torch
    from paper_2310_08649_amd import workloads
    w = workloads.robertson()
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    return w, d(w["y0"]), d(w["times"]), d(w["params"]), torch.as_tensor(w["offsets"], device=dev)


def kernel_names(S, T, init, recompute):
    """Demangled names of the solver kernels a Robertson step launches."""
    if S > 64:  # chunks over S / 64 waves (wide.hpp)
        W = S // 64
        return ("tvi::wide::forward_kernel<tvi::Robertson, double, %d, %d>(tvi::SolveArgs<double>, double*)" % (W, T),
                "tvi::wide::adjoint_kernel<tvi::Robertson, double, %d, %d>(tvi::SolveArgs<double>, double const*)"
                % (W, T))
    pred = "true" if init == "predictor" else "false"
    fwd = "tvi::forward_kernel<tvi::Robertson, double, %d, %d, %s, false, false>(tvi::SolveArgs<double>)" % (
        S, T, pred)
    adj = "tvi::adjoint_kernel<tvi::Robertson, double, %d, %d, %s, %s, false, false>(tvi::SolveArgs<double>)" % (
        S, T, "true" if recompute else "false", pred if recompute else "false")
    return fwd, adj


def time_stages(cs, reps, stream):
    """HIP-event durations (ms) of the forward, loss and adjoint launches of a
    captured step, run eagerly on `stream` (the stream they are launched on)."""
    import torch
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
    for e in evs:
        e[0].record(stream)
        cs.launch_forward()
        e[1].record(stream)
        cs.launch_loss()
        e[2].record(stream)
        cs.launch_adjoint()
        e[3].record(stream)
    torch.cuda.synchronize()
    return {name: stats([e[i].elapsed_time(e[i + 1]) for e in evs])
            for i, name in enumerate(("forward", "loss", "adjoint"))}


def run_headline(args, dev, stream):
    import numpy as np
    import torch
    from paper_2310_08649_amd import autotune, graph, tvi
    w, y0, times, sp, off = rob_inputs(dev)
    B = w["y0"].shape[0]
    lens = np.asarray(w["steps"], dtype=np.int64)
    total = int(lens.sum())
    nmax = int(lens.max())
    order = tvi.order_longest_first(off)

    # ---- autotune (untimed): chunk, tiling, start, and where the adjoint takes its states
    if args.config:
        parts = args.config.split(",")
        C, S, T, init, mode = parts[:5]
        best = {"chunk": int(C), "lanes": int(S), "steps_per_lane": int(T), "init": init, "adjoint": mode,
                "max_newton_chunk": int(parts[5]) if len(parts) > 5 else 0}
        if len(parts) > 8:
            best["adjoint_tiling"] = tuple(int(v) for v in parts[6:9])
        table = None
        log("configuration given: %s" % args.config)
    else:
        log("autotuning chunk / tiling / start / adjoint state source")
        y_out = torch.empty((times.shape[0], 3), dtype=torch.float64, device=dev)
        cands = []
        for mode in ("stored", "recompute"):
            r = autotune.tune_forward("robertson", y0, times, sp, offsets=off, tol=TIMING_TOL, y_out=y_out,
                                      use_cache=False, chunks=(32, 64, 128, 256, 512, 1024, 2048),
                                      inits=("zero", "extrap"), caps=(0, 8),
                                      adjoint=mode, order=order, n_max=nmax)
            for row in r["table"]:
                cands.append(dict(row, adjoint=mode))
        del y_out
        best = min(cands, key=lambda r: (r["failed"], r["ms"]))
        table = cands
        log("chosen chunk=%d lanes=%d steps_per_lane=%d init=%s adjoint=%s cap=%d (%.3f ms)" % (
            best["chunk"], best["lanes"], best["steps_per_lane"], best["init"], best["adjoint"],
            best["max_newton_chunk"], best["ms"]))
    C, S, T, init, mode = best["chunk"], best["lanes"], best["steps_per_lane"], best["init"], best["adjoint"]
    cap = best.get("max_newton_chunk", 0)
    adj_table = None
    if mode == "stored" and "adjoint_tiling" not in best:
        # the stored-trajectory adjoint is a linear solve: its own chunk and tiling
        log("autotuning the adjoint's chunk / tiling")
        y_t, st_t, _, _ = tvi.solve_forward("robertson", y0, times, sp, offsets=off, chunk=C, lanes=S,
                                            steps_per_lane=T, tol=TIMING_TOL, init=init, max_newton_chunk=cap,
                                            order=order, n_max=nmax)
        ra = autotune.tune_adjoint("robertson", times, sp, y_t, y_t, offsets=off, tol=TIMING_TOL, order=order,
                                   n_max=nmax)
        ab = ra["best"]
        best["adjoint_tiling"] = (ab["chunk"], ab["lanes"], ab["steps_per_lane"])
        adj_table = ra["table"]
        del y_t, st_t
        log("adjoint: chunk=%d lanes=%d steps_per_lane=%d (%.3f ms)" % (ab["chunk"], ab["lanes"],
                                                                      ab["steps_per_lane"], ab["ms"]))
    aTil = best.get("adjoint_tiling", (C, S, T))

    def fusable(adj_lanes, recompute):
        # the stored-trajectory adjoint over several waves reads g = y / L from the
        # trajectory (no gradient array is formed: one streaming kernel less)
        return adj_lanes > 64 and not recompute

    def capture(chunk, lanes, spl, start, recompute, mnc=0, adj=None):
        al = adj[1] if adj is not None else lanes
        return graph.CapturedStep("robertson", y0, times, sp, offsets=off, chunk=chunk, lanes=lanes,
                                  steps_per_lane=spl, tol=TIMING_TOL, init=start, loss="frobenius", n_max=nmax,
                                  recompute=recompute, max_newton_chunk=mnc, adjoint_tiling=adj,
                                  fused=fusable(al, recompute)).capture()

    cs = capture(C, S, T, init, mode == "recompute", cap, aTil if mode == "stored" else None)
    for _ in range(args.warmup):
        cs.replay()
    torch.cuda.synchronize()
    log("timing %d graph replays" % args.steps)
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cs.replay()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    peak_mem = int(torch.cuda.max_memory_allocated())
    replay = stats(time_launches(cs.replay, args.steps, stream))

    st_f, st_a = cs.status_fwd.cpu().numpy(), cs.status_adj.cpu().numpy()
    it = cs.iters.cpu().numpy().astype(np.float64)
    ok = (st_f == 0) & (st_a == 0)
    good_steps = int(lens[ok].sum())
    value = good_steps / (ms_per_step * 1e-3)

    # ---- per-kernel durations with HIP events on the launch stream (eager launches of the same step)
    stages = time_stages(cs, args.steps, stream)
    fwd_name = kernel_names(S, T, init, mode == "recompute")[0]
    adj_name = kernel_names(aTil[1], aTil[2], init, mode == "recompute")[1]
    chunks_b = np.maximum(1, (lens + C - 1) // C)
    fwd_flops = float(np.sum(it * lens / chunks_b)) * rob_forward_flops_per_step(S, T)
    adj_flops = float(total) * rob_adjoint_flops_per_step(aTil[1], aTil[2])
    points = int(times.shape[0])
    fwd_bytes = points * (3 * 8 + 8)                      # write y, read t
    fused = fusable(aTil[1], mode == "recompute")
    # read y, g (g is y itself when fused), t; write dL/dp, dL/dy0
    adj_bytes = points * (3 * 8 + (0 if fused else 3 * 8) + 8) + B * 6 * 8
    if mode == "recompute":
        fwd_bytes += 3 * 8 * int(np.sum(chunks_b + 1))     # checkpoints
        adj_flops += fwd_flops                             # the adjoint re-solves every chunk
    # fused: L from the forward pass's per-series sums (read B doubles); else read y, write g
    loss_bytes = B * 8 if fused else points * 2 * 3 * 8
    kern = {
        "forward": {"kernel": fwd_name, "flops": fwd_flops, "bytes": fwd_bytes, **stages["forward"]},
        "adjoint": {"kernel": adj_name, "flops": adj_flops, "bytes": adj_bytes, **stages["adjoint"]},
    }
    dom_key = max(kern, key=lambda k: kern[k]["mean_ms"])
    dom = kern[dom_key]
    tf = dom["flops"] / (dom["mean_ms"] * 1e-3) / 1e12
    gbs = dom["bytes"] / (dom["mean_ms"] * 1e-3) / 1e9
    other = kern["adjoint" if dom_key == "forward" else "forward"]
    roofline = {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": measured_traffic(dom["kernel"]),
                "kernel": dom["kernel"], "avg_launch_ms": round(dom["mean_ms"], 4),
                "algorithmic_flops": dom["flops"], "algorithmic_bytes": dom["bytes"],
                "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                "other_kernel": {"kernel": other["kernel"], "avg_launch_ms": round(other["mean_ms"], 4),
                                 "tflops": round(other["flops"] / (other["mean_ms"] * 1e-3) / 1e12, 3),
                                 "hbm_gbs": round(other["bytes"] / (other["mean_ms"] * 1e-3) / 1e9, 1)},
                "loss_ms": round(stages["loss"]["mean_ms"], 4),
                "loss_hbm_gbs": round(loss_bytes / (stages["loss"]["mean_ms"] * 1e-3) / 1e9, 1)}
    head = {"value": value, "ms_per_step": ms_per_step, "replay": replay, "config": {
        "workload": "robertson n=3 B=2000 ragged N_b=round(exp U(ln 100, ln 2e4)) log-spaced t=[1e-5,1e4] "
                    "y0=(1,0,0) s_i=10^U(log 0.5, log 2) f64 tol=(1e-8,1e-6) fwd + Frobenius-loss gradient + "
                    "adjoint (dL/dp, dL/dy0) in one captured graph, longest first",
        "chunk": C, "lanes": S, "steps_per_lane": T, "init": init, "max_newton_chunk": cap, "adjoint_states": mode,
        "adjoint_tiling": list(aTil),
        "gradient": ("g = y / L read by the adjoint, L from the forward pass's per-series sums" if fused
                     else "g formed by the loss kernel"), "series": B,
        "series_steps": total, "series_failed": int((~ok).sum()), "series_steps_counted": good_steps,
        "newton_corrections": int(it.sum())}, "roofline": roofline, "peak_device_memory_bytes": peak_mem}
    del cs

    # ---- the other adjoint state source (at the same settings where they hold it: the
    # recomputing adjoint runs in one wave, so for chunks over several waves the best
    # one-wave tiling the autotuner found for it), and the chunk = 1 baseline
    other_mode = "recompute" if mode != "recompute" else "stored"
    aC, aS, aT, ainit, acap = C, S, T, init, cap
    if other_mode == "recompute" and S > 64:
        rc = [r for r in (table or []) if r["adjoint"] == "recompute"]
        if rc:
            rb = min(rc, key=lambda r: (r["failed"], r["ms"]))
            aC, aS, aT, ainit, acap = rb["chunk"], rb["lanes"], rb["steps_per_lane"], rb["init"], rb["max_newton_chunk"]
        else:
            aC, aS, aT = 512, 64, 8
    alt = capture(aC, aS, aT, ainit, other_mode == "recompute", acap)
    alt.replay()
    a_st = stats(time_launches(alt.replay, max(3, args.steps // 2), stream))
    a_ok = ((alt.status_fwd == 0) & (alt.status_adj == 0)).cpu().numpy()
    head["other_adjoint_states"] = {"adjoint_states": other_mode,
                                    "value": int(lens[a_ok].sum()) / (a_st["mean_ms"] * 1e-3),
                                    "ms_per_step": a_st["mean_ms"], "chunk": aC, "lanes": aS, "steps_per_lane": aT,
                                    "init": ainit}
    del alt
    log("chunk = 1 baseline")
    seq = capture(1, 1, 1, "zero", False)
    seq.replay()
    torch.cuda.synchronize()
    reps1 = max(3, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps1):
        seq.replay()
    torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t0) * 1e3 / reps1
    s_ok = ((seq.status_fwd == 0) & (seq.status_adj == 0)).cpu().numpy()
    head["chunk1"] = {"value": int(lens[s_ok].sum()) / (ms1 * 1e-3), "ms_per_step": ms1,
                      "series_failed": int((~s_ok).sum()), "speedup_of_chunked": ms1 / ms_per_step}
    del seq
    if table is not None:
        head["autotune_best"] = {k: best[k] for k in ("chunk", "lanes", "steps_per_lane", "init", "adjoint",
                                                       "max_newton_chunk", "failed", "ms")}
        head["autotune_candidates"] = len(table)
    head["_table"] = table
    head["_adjoint_table"] = adj_table
    return head, w


def subset_ragged(w, idx):
    """The ragged series idx of workload w as a workload of their own."""
    import numpy as np
    off = w["offsets"]
    pts = [np.arange(off[b], off[b + 1]) for b in idx]
    lens = np.array([len(p) for p in pts], dtype=np.int64)
    return {"y0": w["y0"][idx], "params": w["params"][idx], "times": w["times"][np.concatenate(pts)],
            "offsets": np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), "steps": lens - 1}


def run_cpu_baseline(w, target_s=10.0):
    """The oracle (sequential backward Euler with a dense Newton solve per step,
    then its discrete adjoint) on the headline workload: the whole batch solved
    repeatedly for about target_s seconds on every host thread, and one thread
    on every tenth series."""
    import numpy as np
    import oracle

    def once(ww, threads):
        y, st, _ = oracle.forward("robertson", ww["y0"], ww["times"], ww["params"], offsets=ww["offsets"],
                                  tol=TIMING_TOL, threads=threads)
        yy = np.where(np.isfinite(y), y, 0.0)
        g = yy / np.sqrt(np.sum(yy ** 2))
        _, _, sa = oracle.adjoint("robertson", yy, ww["times"], ww["params"], g, offsets=ww["offsets"],
                                  threads=threads)
        ok = (st == 0) & (sa == 0)
        return int(np.asarray(ww["steps"])[ok].sum())

    threads = oracle.default_threads()
    reps, steps, t = 0, 0, 0.0
    t0 = time.perf_counter()
    while t < target_s and reps < 1000:
        steps += once(w, threads)
        reps += 1
        t = time.perf_counter() - t0
    sub = subset_ragged(w, np.arange(0, w["y0"].shape[0], 10))
    reps1, steps1, t1 = 0, 0, 0.0
    t0 = time.perf_counter()
    while t1 < target_s / 2 and reps1 < 100:
        steps1 += once(sub, 1)
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
    return {"value": steps / t, "unit": "series*steps/s", "cores": threads, "kind": "oracle",
            "sample": "the whole headline batch (2000 ragged Robertson series, forward + Frobenius-loss "
                      "adjoint) solved %d times in %.1f s on %d threads" % (reps, t, threads),
            "one_core_value": steps1 / t1, "one_core_sample": "every tenth series, %d times in %.1f s" % (reps1, t1),
            "cpu_model": cpu, "nproc": os.cpu_count()}


# ---------------------------------------------------------------------------
# side measurements (--extras FILE)
# ---------------------------------------------------------------------------
def vdp_context(dev, stream, steps):
    """Van der Pol n = 2, 512 series x 5000 uniform steps on [0, 10],
    mu = 10^U(0, 3), y0 = U(-2, 2), FP64, forward, autotuned: the context the
    Van der Pol side measurements share."""
    import torch
    from paper_2310_08649_amd import autotune, tvi, workloads
    w = workloads.vanderpol()
    B, N = w["y0"].shape[0], w["times"].shape[0] - 1
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    y0, times, mu = d(w["y0"]), d(w["times"]), d(w["params"])
    y_out = torch.empty((B, N + 1, 2), dtype=torch.float64, device=dev)
    tuned = autotune.tune_forward("vanderpol", y0, times, mu, tol=TIMING_TOL, y_out=y_out, use_cache=False,
                                  chunks=(10, 16, 32, 50, 64, 100, 128, 200, 256, 500, 1024, 2048),
                                  inits=("zero", "extrap"), caps=(0, 5, 10), limits=(50, 200, 400))
    b = tuned["best"]
    C, S, T, init, cap, mn = (b["chunk"], b["lanes"], b["steps_per_lane"], b["init"], b["max_newton_chunk"],
                              b["max_newton"])
    fn = lambda: tvi.solve_forward("vanderpol", y0, times, mu, chunk=C, lanes=S, steps_per_lane=T, tol=TIMING_TOL,
                                   y_out=y_out, init=init, max_newton=mn, max_newton_chunk=cap)
    _, st, it, _ = fn()
    kst = stats(time_launches(fn, steps, stream))
    return dict(dev=dev, stream=stream, y0=y0, times=times, mu=mu, y_out=y_out, B=B, N=N, C=C, S=S, T=T, init=init,
                cap=cap, mn=mn,
                ms_per_step=kst["mean_ms"], failed=int((st != 0).sum().item()), iters=it, kst=kst)


def run_vanderpol(ctx, steps):
    """Van der Pol forward (the workload is forward only), its chunk = 1
    baseline and the FP64 roofline of its kernel."""
    import numpy as np
    from paper_2310_08649_amd import tvi
    B, N, C, S, T = ctx["B"], ctx["N"], ctx["C"], ctx["S"], ctx["T"]
    kms = ctx["kst"]["mean_ms"]
    flops = float(ctx["iters"].sum().item()) * C * vdp_flops_per_step_iter(C)
    seq = lambda: tvi.solve_forward("vanderpol", ctx["y0"], ctx["times"], ctx["mu"], chunk=1, lanes=1,
                                    steps_per_lane=1, tol=TIMING_TOL, y_out=ctx["y_out"], iters=False,
                                    max_newton=ctx["mn"])
    st1 = seq()[1]
    ms1 = float(np.mean(time_launches(seq, max(3, steps // 3), ctx["stream"])))
    return {"value": B * N / (kms * 1e-3), "unit": "series*steps/s", "ms": kms, "chunk": C, "lanes": S,
            "steps_per_lane": T, "init": ctx["init"], "max_newton": ctx["mn"], "max_newton_chunk": ctx["cap"],
            "failed": ctx["failed"],
            "achieved_tflops": flops / (kms * 1e-3) / 1e12,
            "frac_fp64_peak": flops / (kms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "chunk1": {"value": B * N / (ms1 * 1e-3), "ms": ms1, "speedup_of_chunked": ms1 / kms,
                       "failed": int((st1 != 0).sum().item())}}


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
                                       tol=TIMING_TOL, y_out=y, iters=False, max_newton=ctx["mn"],
                                       init=ctx["init"] if C > 1 else "zero", max_newton_chunk=ctx["cap"])
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
                                observed=obs.reshape(-1), recompute=recompute, max_newton=ctx["mn"],
                                max_newton_chunk=ctx["cap"]).capture()
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
                  (torch.float32, 3), (torch.float32, 4), (torch.float32, 8)):
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


def run_block_grid(ctx, steps):
    """The paper's chunk-efficiency study (Section 5.3, its parameter table) on
    the problems the block solver takes: the mass-damper-spring chain
    (n_unit 1, 2, 3, 5, 10; n = 2 n_unit), the coupled neurons with 3 to 10
    units (n = 12..40) and the forced neural ODE (n_unit 1, 5, ..., 25), FP64,
    n_time = 2000, chunks {1, 3, 10, 30, 100, 300, 1000}, each with Thomas's
    algorithm (T = chunk) and with PCR (T = 1), forward + Frobenius-loss
    gradient + adjoint as one captured graph (states read from the stored
    trajectory), at the batch sizes the table lists (largest and smallest)."""
    import torch
    from paper_2310_08649_amd import graph, workloads
    dev = ctx["dev"]
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    out = {"unit": "ms per forward+adjoint", "paper_best_speedup": {"mass_damper_spring": 106, "neuron": 94,
                                                                    "neural_ode": 97}}
    grid = [("mds", nu, (3, 100)) for nu in (1, 2, 3, 5, 10)] + \
           [("neuron", nu, (3, 50)) for nu in (3, 5, 10)] + \
           [("fnode", nu, (3, 100)) for nu in (1, 5, 10, 15, 20, 25)]
    best_by_model = {}
    for kind, nu, batches in grid:
        for nb in batches:
            w = getattr(workloads, kind)(nu, nb)
            row = {}
            for C in (1, 3, 10, 30, 100, 300, 1000):
                for name, T in (("thomas", C), ("pcr", 1)):
                    if C == 1 and name == "pcr":
                        continue
                    cs = graph.CapturedStep(kind, d(w["y0"]), d(w["times"]), d(w["params"]), chunk=C,
                                            steps_per_lane=T, tol=TIMING_TOL, loss="frobenius",
                                            recompute=False).capture()
                    cs.replay()
                    st = stats(time_launches(cs.replay, 3, torch.cuda.current_stream()))
                    failed = int(((cs.status_fwd != 0) | (cs.status_adj != 0)).sum().item())
                    row["C%d_%s" % (C, name)] = {"ms": st["median_ms"], "failed": failed}
                    del cs
            ok = {k: v["ms"] for k, v in row.items() if v["failed"] == 0}
            bk = min(ok, key=ok.get)
            sp = row["C1_thomas"]["ms"] / ok[bk]
            row["best"] = {"config": bk, "ms": ok[bk], "speedup_over_chunk1": sp}
            out["%s_nu%d_B%d" % (kind, nu, nb)] = row
            log("block grid %s nu=%d B=%d best %s %.3f ms (%.1fx over chunk 1)" % (kind, nu, nb, bk, ok[bk], sp))
            best_by_model[kind] = max(best_by_model.get(kind, 0.0), sp)
    out["best_speedup"] = best_by_model
    return out


def run_crossover(ctx, steps):
    """Thomas against PCR and the hybrids over the state size (Section 3: PCR
    pays log2 levels of n^3 block products, Thomas a serial chain of n^2
    products): the mass-damper-spring chain at n = 2, 4, 8, 12, 20, 40, 100
    series, 2000 steps, chunk 100 and 1000, forward + adjoint graph, every
    segment length T (T = chunk: Thomas; T = 1: PCR)."""
    import torch
    from paper_2310_08649_amd import graph, workloads
    dev = ctx["dev"]
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    out = {"unit": "ms per forward+adjoint", "series": 100, "n_time": 2000}
    for nu in (1, 2, 4, 6, 10, 20):
        w = workloads.mds(nu, 100)
        for C in (100, 1000):
            row = {}
            for T in sorted({C, 1, 4, 16, 64} - {t for t in (4, 16, 64) if t >= C}):
                cs = graph.CapturedStep("mds", d(w["y0"]), d(w["times"]), d(w["params"]), chunk=C, steps_per_lane=T,
                                        tol=TIMING_TOL, loss="frobenius", recompute=False).capture()
                cs.replay()
                st = stats(time_launches(cs.replay, 3, torch.cuda.current_stream()))
                failed = int(((cs.status_fwd != 0) | (cs.status_adj != 0)).sum().item())
                row["T%d" % T] = {"ms": st["median_ms"], "failed": failed}
                del cs
            best = min((k for k in row if row[k]["failed"] == 0), key=lambda k: row[k]["ms"])
            row["best"] = best
            out["n%d_C%d" % (2 * nu, C)] = row
            log("crossover n=%d C=%d best %s" % (2 * nu, C, best))
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
        tol=TIMING_TOL, init=ctx["init"], y_out=ctx["y_out"], iters=False, jacobian=jac, max_newton=ctx["mn"],
        max_newton_chunk=ctx["cap"]), max(3, steps // 2))
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
    """The same on the stiff kinetics, as the predictor workload specifies it:
    chunk 50, trained on 1e5 chunks drawn from 2000 other ragged series,
    evaluated on the benchmark's ragged batch (64 lanes, one step per lane)."""
    import numpy as np
    import torch
    from paper_2310_08649_amd import predictor as pred
    from paper_2310_08649_amd import tvi, workloads
    dev = ctx["dev"]
    C, S, T = 50, 64, 1
    d64 = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    tr = workloads.robertson(seed=106)
    off = torch.as_tensor(tr["offsets"], device=dev)
    y, st, _, _ = tvi.solve_forward("robertson", d64(tr["y0"]), d64(tr["times"]), d64(tr["params"]), offsets=off,
                                    chunk=C, lanes=S, steps_per_lane=T, tol=TIMING_TOL)
    x, ys, inc, dts, series = pred.chunk_samples_ragged(y, d64(tr["times"]), off, C)
    ok = torch.nonzero(torch.isfinite(inc).all(dim=1)).flatten()
    g = torch.Generator(device=dev)
    g.manual_seed(106)
    ok = ok[torch.randperm(ok.numel(), generator=g, device=dev)[:100000]]  # 1e5 training chunks
    d = pred.dims(3, C)
    # corrections to the zero start: on log-spaced grids the extrapolation overshoots
    net, hist = pred.fit_predictor(d, x[ok].contiguous(), inc[ok].float().contiguous(), epochs=20, seed=0)
    torch.cuda.synchronize()
    res = {"chunk": C, "lanes": S, "steps_per_lane": T, "base": "zero", "train_chunks": int(ok.numel()),
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




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--config", default="",
                    help="chunk,lanes,steps_per_lane,init,adjoint (stored | recompute)[,cap[,adjoint chunk,"
                         "lanes,steps_per_lane]]: skip the autotuner")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--extras", default="", help="also run the side measurements and write them to this JSON file")
    ap.add_argument("--only", default="", help="comma-separated side measurements to run (with --extras)")
    ap.add_argument("--extras-only", action="store_true",
                    help="with --extras: run only the side measurements (no headline; for profiling them)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH", "WRITE"),
                    help="no GPU work: write profiles/traffic.json from the counter_collection.csv of a "
                         "rocprofv3 --pmc FETCH_SIZE run and of a --pmc WRITE_SIZE run of this script "
                         "with --probe-copy")
    args = ap.parse_args()
    if args.record_traffic:
        table = record_traffic(args.record_traffic[0], args.record_traffic[1], COPY_PROBE_BYTES)
        print(json.dumps({k: round(v["bytes_per_dispatch"]) for k, v in table.items()}, indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (series are independent and "
              "would shard across GPUs, each running the same kernels on its share)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2310_08649_amd import tvi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tvi.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    if args.extras_only:
        if not args.extras:
            print("--extras-only needs --extras FILE", file=sys.stderr)
            sys.exit(2)
        head, w, table, out = None, None, None, {"extras": args.extras}
    else:
        head, w = run_headline(args, dev, stream)
        table = head.pop("_table")
        adj_table = head.pop("_adjoint_table")
        out = compose_line(args, head)

    if args.extras:
        ext = {"headline_autotune_table": table} if table is not None else {}
        if head is not None and adj_table is not None:
            ext["headline_adjoint_autotune_table"] = adj_table
        only = set(filter(None, args.only.split(",")))
        want = lambda name: not only or name in only
        ctx = {"dev": dev, "stream": stream}
        vdp_runs = [("vanderpol", run_vanderpol), ("fp32", run_vdp_fp32), ("fwd_adjoint", run_vdp_fwd_adjoint)]
        if any(want(n) for n in [r[0] for r in vdp_runs] + ["forward_ad"]):
            log("Van der Pol context (autotune)")
            ctx = vdp_context(dev, stream, args.steps)
        if head is not None:
            c = head["config"]
            ctx["rob_tuned"] = {"chunk": c["chunk"], "lanes": c["lanes"], "steps_per_lane": c["steps_per_lane"]}
        runs = vdp_runs + [("linear", run_linear), ("tiling_study", run_tiling_study),
                           ("saturated", run_saturated), ("pcr_roofline", run_pcr), ("mlp", run_mlp),
                           ("predictor", run_predictor), ("forward_euler", run_forward_euler),
                           ("paper_grid", run_paper_grid), ("forward_ad", run_forward_ad),
                           ("block_grid", run_block_grid), ("crossover", run_crossover)]
        for name, fn in runs:
            if want(name):
                extra(ext, name, lambda fn=fn: fn(ctx, args.steps))
        with open(args.extras, "w") as f:
            json.dump(ext, f, indent=1)
        log("side measurements written to %s" % args.extras)

    if args.probe_copy:
        src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
        del src, dst

    if not args.no_cpu and w is not None:
        log("CPU oracle on the host cores")
        out["cpu_baseline"] = run_cpu_baseline(w)

    print(json.dumps(out, separators=(",", ":")), flush=True)


def compose_line(args, head):
    """The benchmark's JSON line (printed last, compact) from the headline results."""
    out = {"metric": METRIC, "value": head["value"], "unit": "series*steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": head["config"],
           "speedup_vs_chunk1": head["chunk1"]["speedup_of_chunked"], "chunk1": head["chunk1"],
           "other_adjoint_states": head["other_adjoint_states"], "replay_event_ms": head["replay"],
           "roofline": head["roofline"], "peak_device_memory_bytes": head["peak_device_memory_bytes"]}
    if "autotune_best" in head:
        out["autotune_best"] = head["autotune_best"]
        out["autotune_candidates"] = head["autotune_candidates"]
    return out


if __name__ == "__main__":
    main()
