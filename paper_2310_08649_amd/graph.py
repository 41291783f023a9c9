"""One captured HIP graph for a whole training step of a batch of series:
chunked backward-Euler forward pass (with chunk-boundary checkpoints), the
loss gradient, and the adjoint, either with interior states recomputed from
the checkpoints or read from the stored trajectory.

Every buffer is allocated once, before capture, so a replay touches only
device memory the graph owns; the launches are the library's kernels on the
capture stream (no host synchronisation, no allocation, no memset inside).
Ragged series (point offsets) run in the same launches as uniform ones,
longest first.
"""
from __future__ import annotations

import ctypes

import torch

from . import tvi

LOSS = {"frobenius": 0, "mean_square": 1}


class CapturedStep:
    """forward -> loss gradient -> adjoint, captured once, replayed many times.

    Inputs (y0, times, params, offsets) are the graph's own copies: call
    ``set_inputs`` to change their values between replays.  ``adjoint_tiling``
    (chunk, lanes, steps_per_lane), with the stored trajectory only: the
    adjoint's own chunking (its system is linear, so the chunking changes only
    the rounding order); default the forward pass's.
    """

    def __init__(self, kind, y0, times, params, offsets=None, chunk=64, tol=(1e-8, 1e-6), lanes=0, steps_per_lane=0,
                 max_newton=50, init="zero", loss="frobenius", observed=None, n_max=None, recompute=True,
                 longest_first=True, scheme="backward_euler", jacobian="analytic", fused=False,
                 max_newton_chunk=0, adjoint_tiling=None):
        lib = tvi.load()
        self.kind = kind
        self.recompute = recompute
        dt = y0.dtype
        dev = y0.device
        self.y0 = y0.detach().clone().contiguous()
        self.times = times.detach().clone().contiguous()
        self.params = params.detach().clone().contiguous()
        self.offsets = None if offsets is None else offsets.detach().clone().contiguous()
        B, n = self.y0.shape
        if self.offsets is None:
            N = self.times.shape[0] - 1
            yshape = (B, N + 1, n)
        else:
            N = int(n_max if n_max is not None else (self.offsets[1:] - self.offsets[:-1]).max().item() - 1)
            yshape = (self.times.shape[0], n)
        self.B, self.n, self.N = B, n, N
        shared = self.params.dim() == 1
        self.model = tvi.Model(tvi.KINDS[kind], n, tvi._io_dtype(self.y0), 1 if shared else 0, 64)
        # ragged series launch longest first (computed once: the lengths are inputs)
        self.order = tvi.order_longest_first(self.offsets) if self.offsets is not None and longest_first else None
        self.opt = tvi.make_options(chunk, tol, max_newton, lanes, steps_per_lane, init, True, order=self.order,
                                    scheme=scheme, jacobian=jacobian, max_newton_chunk=max_newton_chunk)
        if adjoint_tiling is not None and recompute:
            raise tvi.TviError("an adjoint tiling of its own needs the stored trajectory")
        a_chunk, a_lanes, a_spl = adjoint_tiling if adjoint_tiling is not None else (chunk, lanes, steps_per_lane)
        self.opt_adj = tvi.make_options(a_chunk, tol, max_newton, a_lanes, a_spl, init, True, order=self.order,
                                        scheme=scheme, jacobian=jacobian, max_newton_chunk=max_newton_chunk)
        P = lib.tvi_param_count(ctypes.byref(self.model))
        K = (N + chunk - 1) // chunk + 1
        self.y = torch.empty(yshape, dtype=dt, device=dev)
        # checkpoints only where the adjoint recomputes from them
        self.ckpt = torch.empty((B, K, n), dtype=torch.float64, device=dev) if recompute else None
        self.status_fwd = torch.empty(B, dtype=torch.int32, device=dev)
        self.iters = torch.empty(B, dtype=torch.int32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float64, device=dev)
        self.loss_kind = LOSS[loss]
        # fused (Frobenius loss only): the loss kernel computes L alone and the adjoint
        # reads g = y / L from the trajectory (tvi_options.g_divisor), never forming g
        if fused and self.loss_kind != LOSS["frobenius"]:
            raise tvi.TviError("the fused gradient is the Frobenius loss's (g = y / L)")
        wide = kind in ("robertson", "vanderpol") and dt == torch.float64 and jacobian == "analytic"
        wide_fwd = wide and lanes > 64
        wide_adj = wide and not recompute and a_lanes > 64
        if fused and not (kind == "mlp" or tvi.is_block(kind, n) or wide_adj):
            raise tvi.TviError("the fused gradient is offered by the neural-ODE and block solvers and by the "
                               "stored-trajectory adjoint over several waves (lanes 128 or 256)")
        self.fused = fused
        self.g = None if fused else torch.empty_like(self.y)
        # fused with a forward pass over several waves: it also sums each series' squares,
        # so the loss needs no pass over the trajectory (tvi_loss_from_sums)
        self.sums = torch.empty(B, dtype=torch.float64, device=dev) if fused and wide_fwd else None
        self.observed = None if observed is None else observed.to(device=dev, dtype=torch.uint8).contiguous()
        self.n_observed = int(self.observed.sum().item()) if self.observed is not None else 0
        self.loss_ws = torch.empty(max(1, lib.tvi_loss_workspace_bytes()), dtype=torch.uint8, device=dev)
        self.dLdp = torch.empty((P,) if shared else (B, P), dtype=dt, device=dev)
        self.dLdy0 = torch.empty((B, n), dtype=dt, device=dev)
        self.status_adj = torch.empty(B, dtype=torch.int32, device=dev)
        # the block solver's forward scratch (larger state sizes)
        fwb = lib.tvi_forward_workspace_bytes(ctypes.byref(self.model), ctypes.byref(self.opt), B)
        self.fws = torch.empty(fwb, dtype=torch.uint8, device=dev) if fwb else None
        if fwb:
            self.opt.workspace = self.fws.data_ptr()
            self.opt.workspace_bytes = fwb
        wsb = lib.tvi_adjoint_workspace_bytes(ctypes.byref(self.model), ctypes.byref(self.opt_adj), B)
        self.ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)
        self.ws_bytes = wsb
        self.graph = None
        self.stream = torch.cuda.Stream(device=dev)

    def set_inputs(self, y0=None, times=None, params=None):
        for dst, src in ((self.y0, y0), (self.times, times), (self.params, params)):
            if src is not None:
                dst.copy_(src)

    def launch_forward(self):
        """The forward solve alone (current stream)."""
        lib = tvi.load()
        P = tvi._ptr
        self.opt.series_sumsq = self.sums.data_ptr() if self.sums is not None else None
        tvi._check(lib.tvi_solve_forward(ctypes.byref(self.model), ctypes.byref(self.opt), self.B, self.N,
                                         P(self.offsets), P(self.times), P(self.y0), P(self.params), P(self.y),
                                         P(self.ckpt), P(self.status_fwd), P(self.iters), tvi._stream()),
                   "tvi_solve_forward")
        self.opt.series_sumsq = None

    def launch_loss(self):
        """The loss value and its gradient g = dL/dy alone (current stream); fused over
        several waves, the loss alone from the forward pass's per-series sums."""
        lib = tvi.load()
        P = tvi._ptr
        if self.sums is not None:
            tvi._check(lib.tvi_loss_from_sums(P(self.sums), self.B, P(self.loss), tvi._stream()),
                       "tvi_loss_from_sums")
            return
        points = self.y.numel() // self.n
        tvi._check(lib.tvi_loss_grad(self.loss_kind, self.model.dtype, points, self.n, P(self.y), P(self.observed),
                                     self.n_observed, P(self.g), P(self.loss), P(self.loss_ws),
                                     self.loss_ws.numel(), tvi._stream()), "tvi_loss_grad")

    @property
    def grad_input(self):
        """What the adjoint reads as g (the trajectory itself when fused)."""
        return self.y if self.fused else self.g

    def launch_adjoint(self):
        """The adjoint alone (current stream)."""
        lib = tvi.load()
        P = tvi._ptr
        self.opt_adj.g_divisor = self.loss.data_ptr() if self.fused else None
        tvi._check(lib.tvi_solve_adjoint(ctypes.byref(self.model), ctypes.byref(self.opt_adj), self.B, self.N,
                                         P(self.offsets), P(self.times), P(self.params),
                                         None if self.recompute else P(self.y), P(self.ckpt),
                                         P(self.grad_input), P(self.dLdp), P(self.dLdy0), P(self.status_adj),
                                         P(self.ws), self.ws_bytes, tvi._stream()), "tvi_solve_adjoint")

    def _launch(self):
        self.launch_forward()
        self.launch_loss()
        self.launch_adjoint()

    def run_eager(self):
        """The same launches without a graph (on the current stream)."""
        self._launch()

    def capture(self):
        # one eager run first: kernel attributes and lazy module loading happen outside capture
        self._launch()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._launch()
        torch.cuda.synchronize()
        return self

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
