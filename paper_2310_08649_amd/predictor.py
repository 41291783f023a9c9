"""Learned chunk predictor: data from the solver's own trajectories, training
on the GPU by the library's kernels, and use as the Newton start.

The network maps the chunk-start features x = [y_s, t_s, log dt] to the
corrections p_j = dy_j - base_j, j = 1..C, of the converged chunk's
increments dy_j = y_{s+j} - y_s over a base start: the extrapolated
increments (t_{s+j} - t_s) h(y_s) (base 1; the last step's slope carried over
the chunk), or zero (base 0; the paper's start, better where extrapolation
over a chunk overshoots, as on log-spaced grids).  The solver starts Newton
from dy0_j = base_j + p_j.  The untrained network (zero last layer) is exactly
the base start, and the loss is the mean squared error of the initial iterate
itself, the quantity Newton's work depends on.  Targets are scaled to unit variance for training and the
scale is folded back into the last layer.

Training data are windows of trajectories that the chunked solver itself
computed; nothing else is needed.  The parameter vector is the network's
(W1, b1, W2, b2, W3, b3) followed by the input standardisation constants
(mean[n_in], std[n_in]) taken from the training set.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import tvi


class Predictor(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_out", ctypes.c_int32)]


def _lib():
    lib = tvi.load()
    if not hasattr(lib, "_pred_bound"):
        P, i32, i64, sz, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
        PP = ctypes.POINTER(Predictor)
        lib.tvi_predictor_param_count.argtypes = [PP]
        lib.tvi_predictor_param_count.restype = i64
        lib.tvi_predictor_workspace_bytes.argtypes = [PP, i64]
        lib.tvi_predictor_workspace_bytes.restype = sz
        lib.tvi_predictor_forward.argtypes = [PP, i64, P, P, P, P, sz, P]
        lib.tvi_predictor_forward.restype = i32
        lib.tvi_predictor_train_step.argtypes = [PP, i64, P, P, P, P, P, P, i64, f32, P, P, sz, P]
        lib.tvi_predictor_train_step.restype = i32
        lib.tvi_predictor_pack.argtypes = [PP, P, P, P]
        lib.tvi_predictor_pack.restype = i32
        lib._pred_bound = True
    return lib


def dims(n, chunk, hidden=128):
    return Predictor(n + 2, hidden, n * chunk)


def param_count(d):
    return int(_lib().tvi_predictor_param_count(ctypes.byref(d)))


def net_param_count(d):
    return param_count(d) - 2 * d.n_in


def init_params(d, seed=0, device="cuda"):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, last layer zero
    (the untrained network proposes the extrapolation start), identity standardisation."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((d.n_in, d.hidden), (d.hidden, d.hidden)):
        bnd = 1.0 / math.sqrt(fan_in)
        parts += [rng.uniform(-bnd, bnd, fan_out * fan_in), rng.uniform(-bnd, bnd, fan_out)]
    parts += [np.zeros(d.n_out * d.hidden), np.zeros(d.n_out)]
    parts += [np.zeros(d.n_in), np.ones(d.n_in)]
    return torch.as_tensor(np.concatenate(parts), dtype=torch.float32, device=device)


def chunk_samples(y, times, chunk, stride=None):
    """Training pairs from trajectories y [B, N+1, n] on a shared grid: features
    [y_s, t_s, log dt_s], increments [y_{s+j} - y_s]_j and offsets [t_{s+j} - t_s]_j."""
    y = torch.as_tensor(y)
    t = torch.as_tensor(times, dtype=y.dtype, device=y.device)
    B, Np1, n = y.shape
    starts = torch.arange(0, Np1 - 1 - chunk + 1, stride or chunk, device=y.device)
    ys = y[:, starts]                                              # [B, S, n]
    idx = starts[:, None] + torch.arange(1, chunk + 1, device=y.device)[None]
    dt = (t[idx] - t[starts][:, None])                             # [S, chunk]
    inc = y[:, idx] - ys[:, :, None]                               # [B, S, chunk, n]
    h = t[starts + 1] - t[starts]
    feat = torch.cat([ys, t[starts][None, :, None].expand(B, -1, 1),
                      torch.log(h)[None, :, None].expand(B, -1, 1)], dim=2)
    dts = dt[None].expand(B, -1, -1).reshape(-1, chunk)
    return (feat.reshape(-1, n + 2).float().contiguous(), inc.reshape(-1, chunk * n).float().contiguous(),
            dts.float().contiguous())


def chunk_samples_ragged(y, times, offsets, chunk):
    """Pairs from ragged series (y [points, n], times [points], point offsets
    [B+1]) at the nominal chunk starts s = 0, C, 2C, ... of every series that
    has C more steps: float features, and in y's precision the chunk-start
    states, increments [y_{s+j} - y_s]_j, offsets [t_{s+j} - t_s]_j, and the
    series index of each pair."""
    y = torch.as_tensor(y)
    t = torch.as_tensor(times, dtype=y.dtype, device=y.device)
    off = torch.as_tensor(offsets, device=y.device).long()
    p0 = off[:-1]
    steps = off[1:] - off[:-1] - 1
    nck = torch.div(steps, chunk, rounding_mode="floor")            # full chunks per series
    series = torch.repeat_interleave(torch.arange(nck.shape[0], device=y.device), nck)
    first = torch.cumsum(nck, 0) - nck
    c = torch.arange(series.shape[0], device=y.device) - first[series]
    start = p0[series] + c * chunk                                   # point index of y_s
    idx = start[:, None] + torch.arange(1, chunk + 1, device=y.device)[None]
    ys = y[start]
    inc = y[idx] - ys[:, None, :]
    dts = t[idx] - t[start][:, None]
    feat = torch.cat([ys, t[start][:, None], torch.log(t[start + 1] - t[start])[:, None]], dim=1)
    return feat.float().contiguous(), ys.contiguous(), inc.reshape(inc.shape[0], -1).contiguous(), \
        dts.contiguous(), series


def corrections_at(kind, ys, inc, dts, model_params):
    """Targets p_j = dy_j - (t_{s+j} - t_s) h(y_s) from the chunk-start states ys
    (in their own precision; model_params per pair or shared), as float."""
    f, _ = tvi.model_eval(kind, ys, model_params, jacobian=False)
    ext = (dts[:, :, None] * f[:, None, :]).reshape(ys.shape[0], -1)
    return (inc - ext).float().contiguous()


def extrapolated(kind, x, dts, model_params, n):
    """Increments of the extrapolation start, (t_{s+j} - t_s) h(y_s), for features x."""
    f, _ = tvi.model_eval(kind, x[:, :n].contiguous(), model_params, jacobian=False)
    return (dts[:, :, None] * f[:, None, :]).reshape(x.shape[0], -1).contiguous()


def corrections(kind, x, inc, dts, model_params, n):
    """Targets p_j = dy_j - (t_{s+j} - t_s) h(y_s)."""
    return (inc - extrapolated(kind, x, dts, model_params, n)).contiguous()


def fit_predictor(d, x, target, epochs, batch=256, lr=2e-3, seed=0):
    """Initialise, standardise inputs, train on unit-variance targets, fold the
    target scale into the last layer.  Returns (theta, per-epoch loss)."""
    theta = set_standardisation(init_params(d, seed=seed, device=x.device), d, x)
    sigma = float(target.std().item()) or 1.0
    hist = Trainer(d, theta, batch=batch, lr=lr).fit(x, (target / sigma).contiguous(), epochs=epochs, seed=seed)
    H, n_in, n_out = d.hidden, d.n_in, d.n_out
    o3 = H * n_in + H + H * H + H
    theta[o3:o3 + n_out * H + n_out] *= sigma
    return theta, hist


def set_standardisation(theta, d, x):
    mu = x.mean(dim=0)
    sd = x.std(dim=0)
    sd = torch.where(sd > 1e-12, sd, torch.ones_like(sd))
    P = net_param_count(d)
    theta[P:P + d.n_in] = mu
    theta[P + d.n_in:P + 2 * d.n_in] = sd
    return theta


def pack(d, theta):
    """The inference layout the solvers read (weights transposed), a new tensor."""
    out = torch.empty_like(theta)
    tvi._check(_lib().tvi_predictor_pack(ctypes.byref(d), tvi._ptr(theta), tvi._ptr(out), tvi._stream()),
               "tvi_predictor_pack")
    return out


def solver_args(d, theta, n, base=1):
    """The ``predictor=`` argument of ``tvi.solve_forward`` / ``solve_adjoint``
    for a network trained on corrections to the zero start (base 0) or to the
    extrapolated start (base 1)."""
    return (pack(d, theta), d.hidden, d.n_out // n, base)


def forward(d, theta, x):
    lib = _lib()
    M = x.shape[0]
    out = torch.empty((M, d.n_out), dtype=torch.float32, device=x.device)
    wsb = lib.tvi_predictor_workspace_bytes(ctypes.byref(d), M)
    ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=x.device)
    tvi._check(lib.tvi_predictor_forward(ctypes.byref(d), M, tvi._ptr(x.contiguous()), tvi._ptr(theta),
                                         tvi._ptr(out), tvi._ptr(ws), wsb, tvi._stream()), "tvi_predictor_forward")
    return out


class Trainer:
    """Adam on the mean squared error of the network's outputs, every step in the library's kernels."""

    def __init__(self, d, theta, batch, lr=1e-3):
        lib = _lib()
        self.d, self.theta, self.batch, self.lr = d, theta, batch, lr
        dev = theta.device
        P = net_param_count(d)
        self.grad = torch.zeros(P, dtype=torch.float32, device=dev)
        self.m = torch.zeros(P, dtype=torch.float32, device=dev)
        self.v = torch.zeros(P, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.wsb = lib.tvi_predictor_workspace_bytes(ctypes.byref(d), batch)
        self.ws = torch.empty(max(1, self.wsb), dtype=torch.uint8, device=dev)
        self.step_count = 0

    def step(self, x, target, lr=None):
        lib = _lib()
        assert x.shape[0] <= self.batch
        self.step_count += 1
        tvi._check(lib.tvi_predictor_train_step(
            ctypes.byref(self.d), x.shape[0], tvi._ptr(x), tvi._ptr(target), tvi._ptr(self.theta),
            tvi._ptr(self.grad), tvi._ptr(self.m), tvi._ptr(self.v), self.step_count,
            float(self.lr if lr is None else lr), tvi._ptr(self.loss), tvi._ptr(self.ws), self.wsb, tvi._stream()),
            "tvi_predictor_train_step")
        return self.loss

    def fit(self, x, target, epochs, seed=0):
        """Shuffled mini-batch epochs; returns the per-epoch mean loss (synchronises once per epoch)."""
        g = torch.Generator(device=x.device)
        g.manual_seed(seed)
        hist = []
        M = x.shape[0]
        for _ in range(epochs):
            perm = torch.randperm(M, generator=g, device=x.device)
            acc = torch.zeros(1, dtype=torch.float64, device=x.device)
            nb = 0
            for i in range(0, M - self.batch + 1, self.batch):
                sel = perm[i:i + self.batch]
                acc += self.step(x[sel].contiguous(), target[sel].contiguous()).double()
                nb += 1
            hist.append(float(acc.item()) / max(1, nb))
        return hist
