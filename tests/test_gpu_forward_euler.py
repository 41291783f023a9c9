"""Forward Euler (Eq. forward-euler) on the GPU: the chunked Newton solve of the
explicit scheme and its discrete adjoint against the oracle's plain sequential
recurrence, element by element on the same seeded inputs, through the C ABI.

Gates: FP64 <= 1e-10 relative per series; float storage <= 1e-5 against the
FP64 oracle run on the same float-rounded inputs."""
import numpy as np
import pytest

import oracle
from paper_2310_08649_amd import workloads as W
from tests.helpers import PARITY_TOL, TIMING_TOL, series_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
FE = "forward_euler"


@pytest.fixture(scope="module")
def tvi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_08649_amd import tvi as t
    t.load()
    return t


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def grad_err(a, b):
    return (np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)).max()


def ragged_grid(rng, B, n_range, dt):
    Nb = rng.integers(n_range[0], n_range[1] + 1, size=B)
    offsets = np.concatenate([[0], np.cumsum(Nb + 1)]).astype(np.int64)
    times = np.concatenate([dt * np.arange(N + 1) for N in Nb])
    return offsets, times, Nb


@pytest.mark.parametrize("chunk", [1, 7, 20, 64, 200])
def test_fe_linear_closed_form_one_correction_per_chunk(tvi, chunk):
    w = W.linear(B=8, N=200, lam_range=(0.1, 100.0))
    y, st, it, _ = tvi.solve_forward("linear", dev(w["y0"]), dev(w["times"]), dev(w["params"]), chunk=chunk,
                                     tol=TIMING_TOL, scheme=FE)
    y, st, it = host(y), host(st), host(it)
    assert (st == 0).all()
    h = w["times"][1] - w["times"][0]
    k = np.arange(201)
    c = np.einsum("bji,bj->bi", w["Q"], w["y0"])
    fac = (1.0 - h * w["lam"])[:, None, :] ** k[None, :, None]
    yc = np.einsum("bij,bkj,bj->bki", w["Q"], fac, c)
    assert series_rel_err(y, yc).max() <= 1e-10
    yo, _, _ = oracle.forward("linear", w["y0"], w["times"], w["params"], scheme=FE)
    assert series_rel_err(y, yo).max() <= 1e-10
    assert (it == -(-200 // chunk)).all()  # the explicit chunk system is linear in dy for a linear h


def test_fe_every_tiling_forward_and_adjoint(tvi):
    from paper_2310_08649_amd import autotune
    rng = np.random.default_rng(43)
    n, B, N = 3, 37, 130
    A = -2.0 * np.eye(n)[None] + rng.standard_normal((B, n, n))
    p = A.reshape(B, -1)
    y0 = rng.standard_normal((B, n))
    times = np.cumsum(np.r_[0.0, 0.005 + 0.01 * rng.random(N)])
    yo, so, _ = oracle.forward("linear", y0, times, p, scheme=FE)
    assert (so == 0).all()
    g = yo / np.sqrt(np.sum(yo ** 2))
    op, oy0, _ = oracle.adjoint("linear", yo, times, p, g, scheme=FE)
    cases = [(1, 1, 1)] + [(C, S, T) for C in (3, 16, 40, 130, 256) for S, T in autotune.tilings(C)]
    for C, S, T in cases:
        kw = dict(chunk=C, lanes=S, steps_per_lane=T, tol=PARITY_TOL, scheme=FE)
        y, st, _, ck = tvi.solve_forward("linear", dev(y0), dev(times), dev(p), checkpoints=True, **kw)
        assert (host(st) == 0).all(), (C, S, T)
        assert series_rel_err(host(y), yo).max() <= 1e-10, (C, S, T)
        for src in (dict(y=y), dict(ckpt=ck)):
            dp, dy0, sa = tvi.solve_adjoint("linear", dev(times), dev(p), dev(g), **src, **kw)
            assert (host(sa) == 0).all(), (C, S, T)
            assert grad_err(host(dp), op) <= 1e-10, (C, S, T, list(src))
            assert grad_err(host(dy0), oy0) <= 1e-10, (C, S, T, list(src))


@pytest.mark.parametrize("chunk", [1, 16, 50, 128, 500])
def test_fe_vanderpol_forward_and_adjoint(tvi, chunk):
    w = W.vanderpol(B=64, N=600, mu_range=(1.0, 10.0))
    times = np.linspace(0.0, 1.5, 601)
    yo, so, _ = oracle.forward("vanderpol", w["y0"], times, w["params"], scheme=FE)
    assert (so == 0).all()
    kw = dict(chunk=chunk, tol=PARITY_TOL, scheme=FE)
    y, st, it, ck = tvi.solve_forward("vanderpol", dev(w["y0"]), dev(times), dev(w["params"]), checkpoints=True,
                                      **kw)
    assert (host(st) == 0).all()
    assert series_rel_err(host(y), yo).max() <= 1e-10
    g = yo / np.sqrt(np.sum(yo ** 2))
    op, oy0, _ = oracle.adjoint("vanderpol", yo, times, w["params"], g, scheme=FE)
    dp, dy0, sa = tvi.solve_adjoint("vanderpol", dev(times), dev(w["params"]), dev(g), y=y, **kw)
    dp2, dy02, sa2 = tvi.solve_adjoint("vanderpol", dev(times), dev(w["params"]), dev(g), ckpt=ck, **kw)
    assert (host(sa) == 0).all() and (host(sa2) == 0).all()
    # recomputed interior states are bitwise the forward's
    assert torch.equal(dp, dp2) and torch.equal(dy0, dy02)
    assert grad_err(host(dp), op) <= 1e-10 and grad_err(host(dy0), oy0) <= 1e-10


def test_fe_robertson_ragged_with_empty_series(tvi):
    rng = np.random.default_rng(12)
    B = 40
    offsets, times, Nb = ragged_grid(rng, B, (0, 700), 1e-4)
    Nb[:3] = (0, 1, 2)
    offsets = np.concatenate([[0], np.cumsum(Nb + 1)]).astype(np.int64)
    times = np.concatenate([1e-4 * np.arange(N + 1) for N in Nb])
    params = 10.0 ** rng.uniform(np.log10(0.5), np.log10(2.0), size=(B, 3))
    y0 = np.tile([1.0, 0.0, 0.0], (B, 1))
    yo, so, _ = oracle.forward("robertson", y0, times, params, offsets=offsets, scheme=FE)
    assert (so == 0).all()
    g = yo / np.sqrt(np.sum(yo ** 2))
    op, oy0, _ = oracle.adjoint("robertson", yo, times, params, g, offsets=offsets, scheme=FE)
    off = dev(offsets, torch.int64)
    order = tvi.order_longest_first(off)
    for C, S, T in ((64, 64, 1), (100, 16, 8), (9, 4, 4)):
        kw = dict(offsets=off, chunk=C, lanes=S, steps_per_lane=T, tol=PARITY_TOL, scheme=FE, order=order)
        y, st, _, ck = tvi.solve_forward("robertson", dev(y0), dev(times), dev(params), checkpoints=True, **kw)
        assert (host(st) == 0).all(), (C, S, T)
        yh = host(y)
        assert series_rel_err(yh, yo, offsets).max() <= 1e-10, (C, S, T)
        assert np.abs(yh.sum(axis=1) - 1.0).max() <= 1e-13  # the rates sum to zero
        for src in (dict(y=y), dict(ckpt=ck)):
            dp, dy0, sa = tvi.solve_adjoint("robertson", dev(times), dev(params), dev(g), **src, **kw)
            assert (host(sa) == 0).all()
            assert grad_err(host(dp)[3:], op[3:]) <= 1e-10, (C, S, T, list(src))
            assert grad_err(host(dy0), oy0) <= 1e-10, (C, S, T, list(src))
            # the series without a step: dL/dy0 = g_0 exactly, no parameter gradient
            assert np.array_equal(host(dy0)[0], g[offsets[0]]) and (host(dp)[0] == 0).all()


def test_fe_float_storage(tvi):
    w = W.vanderpol(B=64, N=600, mu_range=(1.0, 10.0))
    times = np.linspace(0.0, 1.5, 601)
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    yo, so, _ = oracle.forward("vanderpol", r(w["y0"]), r(times), r(w["params"]), scheme=FE)
    f = lambda a: dev(a, torch.float32)
    y, st, _, _ = tvi.solve_forward("vanderpol", f(w["y0"]), f(times), f(w["params"]), chunk=50, tol=TIMING_TOL,
                                    scheme=FE)
    assert (host(st) == 0).all()
    assert series_rel_err(host(y).astype(np.float64), yo).max() <= 1e-5


def test_fe_odeint_adjoint_autograd(tvi):
    """torch autograd through odeint_adjoint with the explicit scheme gives the
    oracle's discrete-adjoint gradients."""
    w = W.vanderpol(B=8, N=300, mu_range=(1.0, 5.0))
    times = np.linspace(0.0, 1.0, 301)
    y0 = dev(w["y0"]).requires_grad_(True)
    p = dev(w["params"]).requires_grad_(True)
    y = tvi.odeint_adjoint("vanderpol", y0, dev(times), p, chunk=32, tol=PARITY_TOL, scheme=FE)
    loss = torch.sqrt((y ** 2).sum())
    loss.backward()
    yo, _, _ = oracle.forward("vanderpol", w["y0"], times, w["params"], scheme=FE)
    op, oy0, _ = oracle.adjoint("vanderpol", yo, times, w["params"], yo / np.sqrt(np.sum(yo ** 2)), scheme=FE)
    assert grad_err(host(p.grad), op) <= 1e-10 and grad_err(host(y0.grad), oy0) <= 1e-10


# --------------------------------------------------------------------------
# The neural ODE (MFMA path, float): gate 1e-5 against the float64 oracle on
# the same float-rounded inputs
# --------------------------------------------------------------------------
TOL32 = (1e-8, 1e-6)


def _f32(w):
    return (w[k].astype(np.float32) for k in ("y0", "times", "params"))


@pytest.fixture(scope="module")
def mlp_fe():
    w = W.mlp()  # 64 series x 10000 steps
    y0, times, theta = _f32(w)
    yo, so, _ = oracle.forward("mlp", y0, times, theta, scheme=FE)
    assert (so == 0).all()
    return y0, times, theta, yo


@pytest.mark.parametrize("chunk", [100, 1, 37, 128])
def test_fe_mlp_forward_full_size(tvi, mlp_fe, chunk):
    y0, times, theta, yo = mlp_fe
    f = lambda a: dev(a, torch.float32)
    y, st, it, _ = tvi.solve_forward("mlp", f(y0), f(times), f(theta), chunk=chunk, tol=TOL32, scheme=FE)
    assert (host(st) == 0).all()
    err = series_rel_err(host(y).astype(np.float64), yo)
    assert err.max() <= 1e-5, err.max()


def test_fe_mlp_adjoint_stored_and_recomputed(tvi):
    w = W.mlp(B=8, N=2000)
    y0, times, theta = _f32(w)
    f = lambda a: dev(a, torch.float32)
    y, st, _, ck = tvi.solve_forward("mlp", f(y0), f(times), f(theta), chunk=100, tol=TOL32, checkpoints=True,
                                     scheme=FE)
    assert (host(st) == 0).all()
    yh = host(y).astype(np.float64)
    obs = W.observed_steps(2000, every=100)
    g = np.zeros_like(yh)
    g[:, obs] = 2.0 * yh[:, obs] / (8 * len(obs) * 8)
    a1 = tvi.solve_adjoint("mlp", f(times), f(theta), f(g), ckpt=ck, chunk=100, tol=TOL32, scheme=FE)
    a2 = tvi.solve_adjoint("mlp", f(times), f(theta), f(g), y=y, chunk=100, tol=TOL32, scheme=FE)
    assert (host(a1[2]) == 0).all() and (host(a2[2]) == 0).all()
    assert torch.equal(a1[0], a2[0]) and torch.equal(a1[1], a2[1])
    oth, oy0, _ = oracle.adjoint("mlp", yh, times.astype(np.float64), theta.astype(np.float64), g, scheme=FE)
    e1 = np.abs(host(a1[0]) - oth).max() / np.abs(oth).max()
    e2 = np.abs(host(a1[1]) - oy0).max() / np.abs(oy0).max()
    assert e1 <= 1e-5 and e2 <= 1e-5, (e1, e2)
