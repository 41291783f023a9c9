"""One captured graph for forward + loss gradient + adjoint on ragged series:
every replay equals the eager run, and the eager run equals the oracle."""
import numpy as np
import pytest

import oracle
from paper_2310_08649_amd import workloads as W
from tests.helpers import PARITY_TOL, series_rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_08649_amd import graph, tvi
    tvi.load()
    return graph, tvi


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def test_loss_gradients_match_definitions(mods):
    graph, tvi = mods
    import ctypes
    lib = tvi.load()
    rng = np.random.default_rng(1)
    y = rng.standard_normal((1000, 3))
    obs = (rng.random(1000) < 0.1).astype(np.uint8)
    ws = torch.empty(lib.tvi_loss_workspace_bytes(), dtype=torch.uint8, device="cuda")
    for kind in (0, 1):
        yd, g, L = dev(y), torch.empty(1000, 3, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.float64,
                                                                                                   device="cuda")
        od = dev(obs, torch.uint8)
        rc = lib.tvi_loss_grad(kind, tvi.F64, 1000, 3, tvi._ptr(yd), tvi._ptr(od), int(obs.sum()), tvi._ptr(g),
                               tvi._ptr(L), tvi._ptr(ws), ws.numel(), tvi._stream())
        assert rc == 0
        if kind == 0:
            Lr = np.sqrt(np.sum(y ** 2))
            gr = y / Lr
        else:
            Lr = np.sum(y[obs == 1] ** 2) / (obs.sum() * 3)
            gr = np.where(obs[:, None] == 1, 2 * y / (obs.sum() * 3), 0.0)
        assert abs(L.item() - Lr) <= 1e-13 * Lr
        np.testing.assert_allclose(g.cpu().numpy(), gr, rtol=1e-13, atol=1e-16)


def test_captured_robertson_step_replays_exactly(mods):
    graph, tvi = mods
    w = W.robertson(B=64, n_range=(100, 3000))
    step = graph.CapturedStep("robertson", dev(w["y0"]), dev(w["times"]), dev(w["params"]),
                              offsets=dev(w["offsets"], torch.int64), chunk=64, tol=PARITY_TOL, loss="frobenius")
    step.run_eager()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (step.y, step.g, step.dLdp, step.dLdy0, step.status_fwd, step.status_adj)]
    step.capture()
    for rep in range(3):
        # eager work of the program between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        step.replay()
        torch.cuda.synchronize()
        got = (step.y, step.g, step.dLdp, step.dLdy0, step.status_fwd, step.status_adj)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), rep
        del junk
    assert (ref[4].cpu().numpy() == 0).all() and (ref[5].cpu().numpy() == 0).all()
    # and the eager run is the oracle's
    yo, so, _ = oracle.forward("robertson", w["y0"], w["times"], w["params"], offsets=w["offsets"], tol=PARITY_TOL)
    assert series_rel_err(ref[0].cpu().numpy(), yo, w["offsets"]).max() <= 1e-10
    g = ref[1].cpu().numpy()
    op, oy0, _ = oracle.adjoint("robertson", ref[0].cpu().numpy(), w["times"], w["params"], g, offsets=w["offsets"])
    dp = ref[2].cpu().numpy()
    assert (np.abs(dp - op).max(axis=1) / np.abs(op).max(axis=1)).max() <= 1e-10


def test_loss_gradients_float_storage(mods):
    """The float path of the loss kernels: value accumulated in double, gradient
    to float rounding, against the definitions in float64."""
    graph, tvi = mods
    lib = tvi.load()
    rng = np.random.default_rng(3)
    y = rng.standard_normal((5000, 8)).astype(np.float32)
    obs = (rng.random(5000) < 0.02).astype(np.uint8)
    ws = torch.empty(lib.tvi_loss_workspace_bytes(), dtype=torch.uint8, device="cuda")
    yd = dev(y, torch.float32)
    for kind in (0, 1):
        g = torch.empty(5000, 8, dtype=torch.float32, device="cuda")
        L = torch.empty(1, dtype=torch.float64, device="cuda")
        rc = lib.tvi_loss_grad(kind, tvi.F32, 5000, 8, tvi._ptr(yd), tvi._ptr(dev(obs, torch.uint8)),
                               int(obs.sum()), tvi._ptr(g), tvi._ptr(L), tvi._ptr(ws), ws.numel(), tvi._stream())
        assert rc == 0
        y64 = y.astype(np.float64)
        if kind == 0:
            Lr = np.sqrt(np.sum(y64 ** 2))
            gr = y64 / Lr
        else:
            Lr = np.sum(y64[obs == 1] ** 2) / (obs.sum() * 8)
            gr = np.where(obs[:, None] == 1, 2 * y64 / (obs.sum() * 8), 0.0)
        assert abs(L.item() - Lr) <= 1e-12 * Lr
        np.testing.assert_allclose(g.cpu().numpy(), gr, rtol=1e-6, atol=1e-7 * np.abs(gr).max())


@pytest.mark.parametrize("opts", [dict(scheme="forward_euler"), dict(jacobian="forward_ad"),
                                  dict(scheme="forward_euler", recompute=False)],
                         ids=["forward_euler", "forward_ad", "forward_euler_stored"])
def test_captured_step_with_solver_options_replays_exactly(mods, opts):
    """Forward Euler and AD Jacobians inside one captured graph:
    every replay, with eager work in between, equals the eager run bitwise."""
    graph, tvi = mods
    w = W.vanderpol(B=96, N=800, mu_range=(1.0, 10.0))
    step = graph.CapturedStep("vanderpol", dev(w["y0"]), dev(w["times"]), dev(w["params"]), chunk=40,
                              tol=PARITY_TOL, loss="frobenius", **opts)
    step.run_eager()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (step.y, step.g, step.dLdp, step.dLdy0, step.status_fwd, step.status_adj)]
    assert (ref[4].cpu().numpy() == 0).all() and (ref[5].cpu().numpy() == 0).all()
    step.capture()
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()
        step.replay()
        torch.cuda.synchronize()
        got = (step.y, step.g, step.dLdp, step.dLdy0, step.status_fwd, step.status_adj)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), rep
        del junk
    scheme = opts.get("scheme", "backward_euler")
    yo, so, _ = oracle.forward("vanderpol", w["y0"], w["times"], w["params"], tol=PARITY_TOL, scheme=scheme)
    assert series_rel_err(ref[0].cpu().numpy(), yo).max() <= 1e-10
    op, _, _ = oracle.adjoint("vanderpol", ref[0].cpu().numpy(), w["times"], w["params"], ref[1].cpu().numpy(),
                              scheme=scheme)
    dp = ref[2].cpu().numpy()
    assert (np.abs(dp - op).max(axis=1) / np.abs(op).max(axis=1)).max() <= 1e-10


@pytest.mark.parametrize("kind", ["mds", "mlp"])
def test_fused_frobenius_gradient_equals_the_formed_one(mods, kind):
    """The Frobenius loss's gradient read by the adjoint as y / L from the
    trajectory (tvi_options.g_divisor; the loss kernel computes L alone)
    against the graph that forms g = y / L in memory, for the block solver and
    the neural ODE: the same gradients to rounding (one reciprocal instead of
    a division per entry), every replay bitwise equal to the first."""
    graph, tvi = mods
    f64 = torch.float64
    if kind == "mds":
        w = W.mds(3, 4, n_time=300, t_max=0.05)
        kw = dict(chunk=100, steps_per_lane=10)
    else:
        w = W.mlp(B=6, N=400)
        f64 = torch.float32
        kw = dict(chunk=100)
    # the float network's Newton stops at the float tolerance
    tol = PARITY_TOL if f64 == torch.float64 else (1e-8, 1e-6)
    args = (dev(w["y0"], f64), dev(w["times"], f64), dev(w["params"], f64))
    for recompute in ((False, True) if kind == "mlp" else (False,)):
        runs = {}
        for fused in (False, True):
            step = graph.CapturedStep(kind, *args, tol=tol, loss="frobenius", recompute=recompute,
                                      fused=fused, **kw).capture()
            step.replay()
            torch.cuda.synchronize()
            first = (step.dLdp.clone(), step.dLdy0.clone())
            for _ in range(3):
                step.replay()
                torch.cuda.synchronize()
                assert torch.equal(step.dLdp, first[0]) and torch.equal(step.dLdy0, first[1])
            assert (step.status_fwd.cpu() == 0).all() and (step.status_adj.cpu() == 0).all()
            runs[fused] = first
        gate = 1e-13 if f64 == torch.float64 else 1e-5
        for a, b in zip(runs[True], runs[False]):
            a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
            assert np.abs(a - b).max() <= gate * np.abs(b).max(), (kind, recompute)


def test_fused_gradient_is_refused_by_the_register_solver(mods):
    """The register solver's adjoint reads the plain trajectory-shaped g: the
    fused graph is refused for its models."""
    graph, tvi = mods
    w = W.vanderpol(B=4, N=50, mu_range=(1.0, 5.0))
    args = (dev(w["y0"]), dev(w["times"]), dev(w["params"]))
    with pytest.raises(tvi.TviError):
        graph.CapturedStep("vanderpol", *args, chunk=10, loss="frobenius", fused=True)
