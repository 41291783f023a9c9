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


# models with chunks over 2 or 4 waves (128 or 256 lanes, 2, 4 or 8 steps per lane; double storage)
WIDE_KINDS = ("robertson", "vanderpol")


def tilings(chunk, wide=False):
    """(S, T) candidates with S * T >= chunk and less than half of the lanes
    idle; with ``wide`` also 128 and 256 lanes (chunks up to 2048)."""
    if chunk <= 1:
        return [(1, 1)]
    out = []
    for T in (1, 2, 4, 8):
        for S in (4, 8, 16, 32, 64) + ((128, 256) if wide and T >= 2 else ()):
            if S * T >= chunk and S * T < 2 * max(chunk, 4):
                out.append((S, T))
    if not out and chunk <= 8 * 64:
        out = [(64, 8)]
    return out  # empty: no tiling holds the chunk (over 512 steps without the wide kernels)


def source_hash():
    """Hash of the library's kernel sources (comments and blank space removed):
    a tuning made for other kernel code is not reused."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for p in sorted(glob.glob(os.path.join(here, "csrc", "*"))):
        with open(p) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(os.path.basename(p).encode())
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def _key(kind, y0, times, offsets, extra=""):
    """Problem signature: model, size, dtype, batch, steps, device, the ragged
    lengths (a hash of the offsets), the kernel sources and the caller's options."""
    import hashlib
    dev = torch.cuda.get_device_name(y0.device)
    N = times.shape[0] - 1 if offsets is None else int(times.shape[0] - y0.shape[0])
    lens = "uniform"
    if offsets is not None:
        lens = hashlib.sha256(offsets.detach().cpu().numpy().tobytes()).hexdigest()[:16]
    return "%s|n=%d|%s|B=%d|N=%d|%s|lens=%s|src=%s|%s" % (kind, y0.shape[1], str(y0.dtype), y0.shape[0], N, dev,
                                                        lens, source_hash(), extra)


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
                 reps=3, y_out=None, use_cache=True, inits=("zero",), adjoint=None, caps=(0,), limits=None, **kw):
    """Returns {"best": {chunk, lanes, steps_per_lane, init, max_newton, max_newton_chunk, failed, ms},
    "table": [...]}.

    Candidates are ranked by the number of series that failed to converge
    (forward, or forward or adjoint when the adjoint is timed), then by time:
    a faster configuration never wins by giving up on series.  With
    ``adjoint="stored"`` or ``"recompute"`` each candidate is timed as a
    forward solve followed by the adjoint (Frobenius-loss gradient, states
    read from the trajectory or recomputed from checkpoints): the tiling that
    suits the forward pass alone need not suit the pair.  Further keyword
    options (scheme, jacobian, order, max_newton, n_max, ...) are passed to
    both solves and are part of the cache key.  ``caps``: values of
    max_newton_chunk tried (corrections before a multi-step attempt is halved;
    0 = max_newton).  ``limits``: values of max_newton tried (the corrections a
    single step may take before its series is given up), or None for the one
    in ``kw`` (default 50)."""
    opts = ",".join("%s=%s" % (k, "tensor" if isinstance(v, torch.Tensor) else v) for k, v in sorted(kw.items()))
    kw_limit = kw.pop("max_newton", 50)
    lims = tuple(limits) if limits else (kw_limit,)
    key = _key(kind, y0, times, offsets, "tol=%g,%g|chunks=%s|inits=%s|adjoint=%s|caps=%s|limits=%s|%s"
               % (tol[0], tol[1], ",".join(map(str, chunks)), ",".join(inits), adjoint,
                  ",".join(map(str, caps)), ",".join(map(str, lims)), opts))
    if use_cache:
        with _lock:
            hit = _load_cache().get(key)
        if hit:
            return hit
    table = []
    wide = kind in WIDE_KINDS and y0.dtype == torch.float64 and not adjoint == "recompute"
    for C in chunks:
        for S, T, init, cap, lim in [(S, T, i, c, l) for S, T in tilings(C, wide) for i in inits for c in caps
                                     for l in lims]:
            res = {}

            def fn():
                y, st, _, ck = tvi.solve_forward(kind, y0, times, params, offsets=offsets, chunk=C, lanes=S,
                                                 steps_per_lane=T, tol=tol, y_out=y_out, init=init,
                                                 iters=False, checkpoints=adjoint == "recompute",
                                                 max_newton=lim, max_newton_chunk=cap, **kw)
                res["st"] = st
                if adjoint:
                    g = y if "g" not in res else res["g"]
                    res["g"] = g
                    src = dict(ckpt=ck) if adjoint == "recompute" else dict(y=y)
                    _, _, sa = tvi.solve_adjoint(kind, times, params, g, offsets=offsets, chunk=C, lanes=S,
                                                 steps_per_lane=T, tol=tol, init=init, max_newton=lim,
                                                 max_newton_chunk=cap, **src, **kw)
                    res["sa"] = sa
            ms = _time(fn, reps)
            bad = res["st"] != 0
            if adjoint:
                bad = bad | (res["sa"] != 0)
            table.append({"chunk": C, "lanes": S, "steps_per_lane": T, "init": init, "max_newton": lim,
                          "max_newton_chunk": cap, "failed": int(bad.sum().item()), "ms": ms})
    best = min(table, key=lambda r: (r["failed"], r["ms"]))
    res = {"best": best, "table": table}
    if use_cache:
        with _lock:
            cache = _load_cache()
            cache[key] = res
            _store_cache(cache)
    return res


def tune_adjoint(kind, times, params, y, g, offsets=None, tol=(1e-8, 1e-6), chunks=(256, 512, 1024, 2048), reps=3,
                 **kw):
    """The stored-trajectory adjoint's own chunk and lane tiling.

    The adjoint system is linear (Appendix A): one reduction per chunk, no
    Newton iteration, so its chunking changes only the rounding order, not
    the gradient, and it need not match the forward pass's.  Times the adjoint
    alone (trajectory ``y``, gradient ``g``) for every (C, S, T) candidate,
    ranks failed series first, then time.  Returns {"best": {chunk, lanes,
    steps_per_lane, failed, ms}, "table": [...]} (not cached)."""
    wide = kind in WIDE_KINDS and y.dtype == torch.float64
    table = []
    for C in chunks:
        for S, T in tilings(C, wide):
            res = {}

            def fn():
                _, _, sa = tvi.solve_adjoint(kind, times, params, g, y=y, offsets=offsets, chunk=C, lanes=S,
                                             steps_per_lane=T, tol=tol, **kw)
                res["sa"] = sa
            ms = _time(fn, reps)
            table.append({"chunk": C, "lanes": S, "steps_per_lane": T, "failed": int((res["sa"] != 0).sum().item()),
                          "ms": ms})
    best = min(table, key=lambda r: (r["failed"], r["ms"]))
    return {"best": best, "table": table}
