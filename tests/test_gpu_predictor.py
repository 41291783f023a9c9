"""Learned chunk predictor: forward, gradient and Adam step of the GPU kernels
against the float64 reference, and what the trained network gains over the
solver started without it."""
import numpy as np
import pytest

import oracle
from oracle import predictor as PR
from paper_2310_08649_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_08649_amd import predictor, tvi
    tvi.load()
    return predictor, tvi


def _case(pred, n_in=10, hidden=128, n_out=400, M=300, seed=0):
    d = pred.Predictor(n_in, hidden, n_out)
    rng = np.random.default_rng(seed)
    P = pred.net_param_count(d)
    th = np.concatenate([0.2 * rng.standard_normal(P), 0.1 * rng.standard_normal(n_in),
                         1.0 + 0.5 * rng.random(n_in)]).astype(np.float32)
    x = rng.standard_normal((M, n_in)).astype(np.float32)
    tgt = rng.standard_normal((M, n_out)).astype(np.float32)
    return d, th, x, tgt


def _standardised(th, x, d):
    P = th.shape[0] - 2 * d.n_in
    mu, sd = th[P:P + d.n_in].astype(np.float64), th[P + d.n_in:].astype(np.float64)
    return th[:P].astype(np.float64), (x.astype(np.float64) - mu) / sd


def test_predictor_forward_matches_reference(mods):
    pred, _ = mods
    d, th, x, _ = _case(pred)
    out = pred.forward(d, torch.tensor(th, device="cuda"), torch.tensor(x, device="cuda")).cpu().numpy()
    net, xs = _standardised(th, x, d)
    ref, _ = PR.forward(net, xs, d.n_in, d.hidden, d.n_out)
    assert np.abs(out - ref).max() <= 1e-5 * np.abs(ref).max()


def test_predictor_gradient_and_adam_match_reference(mods):
    pred, _ = mods
    d, th, x, tgt = _case(pred, M=256, seed=1)
    theta = torch.tensor(th, device="cuda")
    tr = pred.Trainer(d, theta, batch=256, lr=1e-3)
    loss = tr.step(torch.tensor(x, device="cuda"), torch.tensor(tgt, device="cuda"), lr=0.0)
    net, xs = _standardised(th, x, d)
    L, g = PR.loss_and_grad(net, xs, tgt.astype(np.float64), d.n_in, d.hidden, d.n_out)
    assert abs(float(loss.item()) - L) <= 1e-5 * L
    gg = tr.grad.cpu().numpy()
    assert np.abs(gg - g).max() <= 1e-4 * np.abs(g).max(), np.abs(gg - g).max() / np.abs(g).max()
    assert np.array_equal(theta.cpu().numpy(), th)  # lr = 0: no update
    # Adam: a few steps against the reference update rule on the GPU's own gradients
    tr2 = pred.Trainer(d, torch.tensor(th, device="cuda"), batch=256, lr=1e-3)
    ref_th, m, v = net.copy(), np.zeros_like(net), np.zeros_like(net)
    for step in range(1, 4):
        tr2.step(torch.tensor(x, device="cuda"), torch.tensor(tgt, device="cuda"))
        ref_th, m, v = PR.adam_step(ref_th, tr2.grad.cpu().numpy().astype(np.float64), m, v, step, 1e-3)
    got = tr2.theta.cpu().numpy()[:net.shape[0]]
    assert np.abs(got - ref_th).max() <= 1e-5 * np.abs(ref_th).max()


def test_predictor_training_reduces_loss(mods):
    pred, _ = mods
    d = pred.Predictor(10, 128, 40)
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.standard_normal((4096, 10)), dtype=torch.float32, device="cuda")
    A = torch.tensor(rng.standard_normal((10, 40)) / 3, dtype=torch.float32, device="cuda")
    tgt = torch.tanh(x @ A).contiguous()
    theta = pred.init_params(d, seed=1)
    theta = pred.set_standardisation(theta, d, x)
    hist = pred.Trainer(d, theta, batch=256, lr=3e-3).fit(x, tgt, epochs=8)
    assert hist[-1] < 0.2 * hist[0], hist


def test_trained_predictor_gains_over_extrapolation(mods):
    """Train on chunks the solver itself computed, then solve held-out series
    from the zero start, the extrapolated start and the learned start: all
    reach the same trajectory and the learned start is closer to the converged
    chunk.  The gain the method would need, fewer Newton corrections, is
    asserted last and reported as an expected failure while it does not hold:
    on this smooth problem every start needs exactly one correction per chunk."""
    pred, tvi = mods
    C, tol = 50, (1e-8, 1e-6)
    f32 = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")
    tr = W.mlp(B=96, N=2000, seed=105)
    y, st, _, _ = tvi.solve_forward("mlp", f32(tr["y0"]), f32(tr["times"]), f32(tr["params"]), chunk=C, tol=tol)
    assert (st.cpu().numpy() == 0).all()
    x, inc, dts = pred.chunk_samples(y, f32(tr["times"]), C)
    d = pred.dims(8, C)
    p = pred.corrections("mlp", x, inc, dts, f32(tr["params"]), 8)
    theta, hist = pred.fit_predictor(d, x, p, epochs=40, seed=3)
    assert hist[-1] < 0.2 * hist[0], hist

    ev = W.mlp(B=32, N=2000, seed=107)
    ev["params"] = tr["params"]
    args = (f32(ev["y0"]), f32(ev["times"]), f32(ev["params"]))
    yo, _, _ = oracle.forward("mlp", ev["y0"].astype(np.float32), ev["times"].astype(np.float32),
                              ev["params"].astype(np.float32), tol=(1e-12, 1e-12))
    its = {}
    for init in ("zero", "extrap", "predictor"):
        kw = dict(predictor=pred.solver_args(d, theta, 8, base=1)) if init == "predictor" else {}
        yy, st, it, _ = tvi.solve_forward("mlp", *args, chunk=C, tol=tol, init=init, **kw)
        assert (st.cpu().numpy() == 0).all()
        rel = np.abs(yy.cpu().numpy() - yo).max() / np.abs(yo).max()
        assert rel <= 1e-5, (init, rel)
        its[init] = int(it.sum().item())
    # initial-iterate error on the held-out chunks: learned vs extrapolated increments
    xe, ie, de = pred.chunk_samples(f32(yo), f32(ev["times"]), C)
    ext = pred.extrapolated("mlp", xe, de, args[2], 8)
    err_ext = float(((ext - ie) ** 2).mean().item())
    err_pred = float(((ext + pred.forward(d, theta, xe) - ie) ** 2).mean().item())
    print("Newton corrections: zero %d, extrapolation %d, predictor %d; initial iterate MSE: extrapolation "
          "%.3e, predictor %.3e" % (its["zero"], its["extrap"], its["predictor"], err_ext, err_pred))
    assert err_pred < 0.5 * err_ext
    assert its["predictor"] <= its["extrap"] < its["zero"]
    # with Algorithm 1's reference residual (that of dy = 0) a better start may stop sooner
    its0 = {}
    for init in ("extrap", "predictor"):
        kw = dict(predictor=pred.solver_args(d, theta, 8, base=1)) if init == "predictor" else {}
        yy, st, it, _ = tvi.solve_forward("mlp", *args, chunk=C, tol=tol, init=init, reference="zero", **kw)
        assert (st.cpu().numpy() == 0).all()
        rel = np.abs(yy.cpu().numpy() - yo).max() / np.abs(yo).max()
        assert rel <= 1e-5, (init, rel)
        its0[init] = int(it.sum().item())
    print("with the zero-increment reference: extrapolation %d, predictor %d" % (its0["extrap"], its0["predictor"]))
    assert its0["predictor"] <= its0["extrap"] <= its["extrap"]
    if not its["predictor"] < its["extrap"]:
        pytest.xfail("the learned start saves no Newton correction (%d against %d from the extrapolated start): "
                     "each start needs one correction per chunk" % (its["predictor"], its["extrap"]))


def _dev64(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_untrained_predictor_start_is_its_base(mods):
    """A network with a zero last layer proposes exactly its base start (the
    extrapolation, or zero), which is then kept: trajectories and iteration
    counts are bitwise equal to those of that start."""
    pred, tvi = mods
    for kind, w, C in (
            ("vanderpol", W.vanderpol(B=64, N=1000, mu_range=(1.0, 100.0)), 50),
            ("robertson", W.robertson(B=40, n_range=(100, 1500)), 64),
            ("linear", W.linear(B=8, N=200), 20)):
        n = w["y0"].shape[1]
        off = None if w["offsets"] is None else torch.as_tensor(w["offsets"], device="cuda")
        d = pred.dims(n, C)
        theta = pred.init_params(d, seed=2)
        args = (_dev64(w["y0"]), _dev64(w["times"]), _dev64(w["params"]))
        for base, init in ((1, "extrap"), (0, "zero")):
            ye, se, ie, _ = tvi.solve_forward(kind, *args, offsets=off, chunk=C, init=init)
            yp, sp, ip, _ = tvi.solve_forward(kind, *args, offsets=off, chunk=C, init="predictor",
                                              predictor=pred.solver_args(d, theta, n, base=base))
            assert torch.equal(se, sp) and torch.equal(ie, ip), (kind, init)
            assert torch.equal(torch.nan_to_num(ye), torch.nan_to_num(yp)), (kind, init)


def test_predictor_on_robertson(mods):
    """Train on ragged Robertson chunks the solver computed (corrections to the
    zero start: on log-spaced grids the extrapolation overshoots), then solve
    held-out series from the learned start: the oracle's trajectory, a smaller
    initial iterate error than the zero start, and the recomputing adjoint
    (which re-runs the predictor from every checkpoint) bitwise equal to the
    adjoint on the stored trajectory."""
    pred, tvi = mods
    from tests.helpers import PARITY_TOL, TIMING_TOL, series_rel_err
    C = 64
    tr = W.robertson(B=300, seed=106, n_range=(200, 4000))
    off = torch.as_tensor(tr["offsets"], device="cuda")
    y, st, _, _ = tvi.solve_forward("robertson", _dev64(tr["y0"]), _dev64(tr["times"]), _dev64(tr["params"]),
                                    offsets=off, chunk=C, tol=TIMING_TOL)
    assert (st.cpu().numpy() == 0).all()
    x, ys, inc, dts, series = pred.chunk_samples_ragged(y, _dev64(tr["times"]), off, C)
    d = pred.dims(3, C)
    theta, hist = pred.fit_predictor(d, x, inc.float().contiguous(), epochs=60, seed=1)
    assert hist[-1] < 0.5 * hist[0], hist
    args_p = pred.solver_args(d, theta, 3, base=0)

    ev = W.robertson(B=48, seed=108, n_range=(200, 4000))
    eoff = torch.as_tensor(ev["offsets"], device="cuda")
    args = (_dev64(ev["y0"]), _dev64(ev["times"]), _dev64(ev["params"]))
    yo, so, _ = oracle.forward("robertson", ev["y0"], ev["times"], ev["params"], offsets=ev["offsets"],
                               tol=PARITY_TOL)
    its = {}
    for init in ("zero", "predictor"):
        kw = dict(predictor=args_p) if init == "predictor" else {}
        yy, st, it, ck = tvi.solve_forward("robertson", *args, offsets=eoff, chunk=C, tol=PARITY_TOL, init=init,
                                           checkpoints=True, **kw)
        assert (st.cpu().numpy() == 0).all(), init
        assert series_rel_err(yy.cpu().numpy(), yo, ev["offsets"]).max() <= 1e-10, init
        its[init] = int(it.sum().item())
        if init == "predictor":
            g = yy / torch.sqrt((yy ** 2).sum())
            a1 = tvi.solve_adjoint("robertson", args[1], args[2], g, y=yy, offsets=eoff, chunk=C, tol=PARITY_TOL,
                                   init=init, **kw)
            a2 = tvi.solve_adjoint("robertson", args[1], args[2], g, ckpt=ck, offsets=eoff, chunk=C, tol=PARITY_TOL,
                                   init=init, **kw)
            assert torch.equal(a1[0], a2[0]) and torch.equal(a1[1], a2[1])
            y_ref = yy
    xe, yse, ie, de, se = pred.chunk_samples_ragged(y_ref, args[1], eoff, C)
    err_zero = float((ie ** 2).mean().item())
    err_pred = float(((ie - pred.forward(d, theta, xe).double()) ** 2).mean().item())
    print("Robertson Newton corrections: zero %d, predictor %d; initial iterate MSE: zero %.3e, predictor %.3e"
          % (its["zero"], its["predictor"], err_zero, err_pred))
    assert err_pred < err_zero
    if not its["predictor"] < its["zero"]:
        pytest.xfail("the learned start needs no fewer Newton corrections than the zero start (%d against %d): the "
                     "absolute tolerance binds on most chunks" % (its["predictor"], its["zero"]))
