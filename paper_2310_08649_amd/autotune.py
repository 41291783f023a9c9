"""Autotuner for the chunk length and the lane tiling.

The best chunk length is problem- and device-specific (Section 5.3: too short
a chunk starves the device, too long a chunk costs more Newton iterations and
reduction levels).  For a problem signature the tuner times the forward solve
for each candidate (chunk C, lanes per series S, steps per lane T) with HIP
events on the current stream, keeps the fastest, and caches the choice in a
JSON file keyed by (model, n, dtype, batch, steps, device).
"""
from __future__ import annotations

import json
import os
import threading

import torch

from . import tvi

_CACHE_PATH = os.environ.get("TVI_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tvi_autotune.json"))
_lock = threading.Lock()


def tilings(chunk):
    """(S, T) candidates with S * T >= chunk and less than half of the lanes idle."""
    if chunk <= 1:
        return [(1, 1)]
    out = []
    for T in (1, 2, 4, 8):
        for S in (4, 8, 16, 32, 64):
            if S * T >= chunk and S * T < 2 * max(chunk, 4):
                out.append((S, T))
    if not out:
        out = [(64, 8)]
    return out


def _key(kind, y0, times, offsets, extra=""):
    dev = torch.cuda.get_device_name(y0.device)
    N = times.shape[0] - 1 if offsets is None else int(times.shape[0] - y0.shape[0])
    return "%s|n=%d|%s|B=%d|N=%d|%s|%s" % (kind, y0.shape[1], str(y0.dtype), y0.shape[0], N, dev, extra)


def _load_cache():
    try:
        with open(_CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache):
    try:
        os.makedirs(os.path.dirname(_CACHE_PATH), exist_ok=True)
        tmp = _CACHE_PATH + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, _CACHE_PATH)
    except OSError:
        pass


def _time(fn, reps):
    stream = torch.cuda.current_stream()
    fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    return ts[len(ts) // 2]


def tune_forward(kind, y0, times, params, offsets=None, tol=(1e-8, 1e-6), chunks=(10, 50, 100, 200, 500),
                 reps=3, y_out=None, use_cache=True, inits=("zero",), adjoint=None, reuses=(0.0,), **kw):
    """Returns {"best": {chunk, lanes, steps_per_lane, init, jacobian_reuse, failed, ms}, "table": [...]}.

    ``reuses``: Jacobian-reuse factors to try (0: full Newton); a factor that
    the tiling does not support is skipped.

    Candidates are ranked by the number of series that failed to converge,
    then by time: a faster configuration never wins by giving up on series.
    With ``adjoint="stored"`` or ``"recompute"`` each candidate is timed as a
    forward solve followed by the adjoint (Frobenius-loss gradient, states
    read from the trajectory or recomputed from checkpoints): the tiling that
    suits the forward pass alone need not suit the pair."""
    key = _key(kind, y0, times, offsets, "tol=%g,%g|chunks=%s|inits=%s|adjoint=%s|reuses=%s"
               % (tol[0], tol[1], ",".join(map(str, chunks)), ",".join(inits), adjoint, ",".join(map(str, reuses))))
    if use_cache:
        with _lock:
            hit = _load_cache().get(key)
        if hit:
            return hit
    table = []
    for C in chunks:
        for S, T in tilings(C):
            for init, reuse in [(i, r) for i in inits for r in reuses]:
                res = {}

                def fn():
                    y, st, _, ck = tvi.solve_forward(kind, y0, times, params, offsets=offsets, chunk=C, lanes=S,
                                                     steps_per_lane=T, tol=tol, y_out=y_out, init=init,
                                                     iters=False, checkpoints=adjoint == "recompute",
                                                     jacobian_reuse=reuse, **kw)
                    res["st"] = st
                    if adjoint:
                        g = y if "g" not in res else res["g"]
                        res["g"] = g
                        src = dict(ckpt=ck) if adjoint == "recompute" else dict(y=y)
                        tvi.solve_adjoint(kind, times, params, g, offsets=offsets, chunk=C, lanes=S,
                                          steps_per_lane=T, tol=tol, init=init, jacobian_reuse=reuse, **src, **kw)
                try:
                    ms = _time(fn, reps)
                except tvi.TviError:
                    if reuse > 0.0:
                        continue  # this tiling keeps too many matrices per lane for reuse
                    raise
                failed = int((res["st"] != 0).sum().item())
                table.append({"chunk": C, "lanes": S, "steps_per_lane": T, "init": init, "jacobian_reuse": reuse,
                              "failed": failed, "ms": ms})
    best = min(table, key=lambda r: (r["failed"], r["ms"]))
    res = {"best": best, "table": table}
    if use_cache:
        with _lock:
            cache = _load_cache()
            cache[key] = res
            _store_cache(cache)
    return res
