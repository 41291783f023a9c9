"""Neural-ODE path (MFMA) against the CPU oracle, through the C ABI.

The network rate enters the residual as bf16x3 MFMA products (about float
accuracy) and the whole path computes in float, so the gate against the
float64 oracle is 1e-5 relative."""
import numpy as np
import pytest

import oracle
from paper_2310_08649_amd import workloads as W
from tests.helpers import series_rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL32 = (1e-8, 1e-6)


@pytest.fixture(scope="module")
def tvi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_08649_amd import tvi as t
    t.load()
    return t


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("scale", [0.1, 0.5])
def test_mlp_rate_and_jacobian_match_oracle(tvi, scale):
    rng = np.random.default_rng(3)
    theta = W.mlp_theta(rng, 8, 64, scale=scale).astype(np.float32)
    M = 300  # several workgroups of 128 states and a ragged tail
    y = rng.standard_normal((M, 8)).astype(np.float32)
    f, J = tvi.model_eval("mlp", dev(y), dev(theta))
    f, J = host(f), host(J)
    for q in range(M):
        fo, Jo = oracle.rhs("mlp", y[q], 0.0, theta.astype(np.float64))
        assert np.abs(f[q] - fo).max() <= 1e-5 * max(np.abs(fo).max(), 1e-3), q
        assert np.abs(J[q] - Jo).max() <= 1e-5 * max(np.abs(Jo).max(), 1e-3), q


@pytest.mark.parametrize("kind,n,P", [("linear", 4, 16), ("vanderpol", 2, 1), ("robertson", 3, 3)])
def test_analytic_rate_and_jacobian_match_oracle(tvi, kind, n, P):
    rng = np.random.default_rng(5)
    M = 257
    y = rng.standard_normal((M, n))
    p = np.abs(rng.standard_normal((M, P))) + 0.5
    f, J = tvi.model_eval(kind, dev(y, torch.float64), dev(p, torch.float64))
    f, J = host(f), host(J)
    for q in range(M):
        fo, Jo = oracle.rhs(kind, y[q], 0.0, p[q])
        np.testing.assert_allclose(f[q], fo, rtol=1e-13, atol=1e-13 * np.abs(fo).max())
        np.testing.assert_allclose(J[q], Jo, rtol=1e-13, atol=1e-13 * np.abs(Jo).max())


@pytest.fixture(scope="module")
def mlp_full():
    w = W.mlp()  # 64 series x 10000 steps
    y0, times, theta = (w[k].astype(np.float32) for k in ("y0", "times", "params"))
    yo, so, io = oracle.forward("mlp", y0, times, theta, tol=(1e-12, 1e-12))
    assert (so == 0).all()
    return y0, times, theta, yo


@pytest.mark.parametrize("chunk", [100, 1, 37, 128])
def test_mlp_forward_full_size_parity(tvi, mlp_full, chunk):
    y0, times, theta, yo = mlp_full
    y, st, it, _ = tvi.solve_forward("mlp", dev(y0), dev(times), dev(theta), chunk=chunk, tol=TOL32)
    assert (host(st) == 0).all()
    err = series_rel_err(host(y), yo)
    assert err.max() <= 1e-5, err.max()
    assert (host(it) >= -(-10000 // chunk)).all()


def test_mlp_forward_chip_filling_batch(tvi):
    """1024 series x 1000 steps of 1e-4 (the benchmark's chip-filling neural-ODE batch):
    one workgroup per series, four per CU."""
    w = W.mlp(B=1024, N=1000, seed=131, t_end=0.1)
    y0, times, theta = (w[k].astype(np.float32) for k in ("y0", "times", "params"))
    yo, so, _ = oracle.forward("mlp", y0, times, theta, tol=(1e-12, 1e-12))
    assert (so == 0).all()
    y, st, it, _ = tvi.solve_forward("mlp", dev(y0), dev(times), dev(theta), chunk=100, tol=TOL32)
    assert (host(st) == 0).all()
    err = series_rel_err(host(y), yo)
    assert err.max() <= 1e-5, err.max()


def test_mlp_forward_extrapolated_start_and_checkpoints(tvi):
    w = W.mlp(B=8, N=1000)
    y0, times, theta = (w[k].astype(np.float32) for k in ("y0", "times", "params"))
    yo, so, _ = oracle.forward("mlp", y0, times, theta, tol=(1e-12, 1e-12))
    y0d, td, thd = dev(y0), dev(times), dev(theta)
    yz, sz, iz, ck = tvi.solve_forward("mlp", y0d, td, thd, chunk=100, tol=TOL32, checkpoints=True)
    ye, se, ie, _ = tvi.solve_forward("mlp", y0d, td, thd, chunk=100, tol=TOL32, init="extrap")
    assert (host(sz) == 0).all() and (host(se) == 0).all()
    assert series_rel_err(host(yz), yo).max() <= 1e-5
    assert series_rel_err(host(ye), yo).max() <= 1e-5
    # the slope start is closer to the solution: no more Newton iterations than from zero
    assert host(ie).sum() <= host(iz).sum()
    ck = ck.cpu().numpy()
    assert np.allclose(ck[:, 0], y0) and np.allclose(ck[:, -1], host(yz)[:, -1], rtol=1e-6, atol=1e-7)


def _mlp_loss_grad(y, obs):
    """L = mean over series, observed steps and components of y^2; g = dL/dy."""
    B, n = y.shape[0], y.shape[2]
    g = np.zeros_like(y)
    g[:, obs] = 2.0 * y[:, obs] / (B * len(obs) * n)
    return g


@pytest.mark.parametrize("recompute", [True, False])
def test_mlp_adjoint_matches_oracle(tvi, recompute):
    w = W.mlp(B=8, N=2000)
    y0, times, theta = (w[k].astype(np.float32) for k in ("y0", "times", "params"))
    obs = W.observed_steps(2000, every=100)
    y, st, _, ck = tvi.solve_forward("mlp", dev(y0), dev(times), dev(theta), chunk=100, tol=TOL32, checkpoints=True)
    assert (host(st) == 0).all()
    yh = host(y)
    g = _mlp_loss_grad(yh, obs)
    kw = dict(ckpt=ck) if recompute else dict(y=y)
    dth, dy0, sa = tvi.solve_adjoint("mlp", dev(times), dev(theta), dev(g), chunk=100, tol=TOL32, **kw)
    assert (host(sa) == 0).all()
    oth, oy0, ost = oracle.adjoint("mlp", yh, times.astype(np.float64), theta.astype(np.float64), g)
    assert (ost == 0).all()
    e1 = np.abs(host(dth) - oth).max() / np.abs(oth).max()
    e2 = np.abs(host(dy0) - oy0).max() / np.abs(oy0).max()
    assert e1 <= 1e-5 and e2 <= 1e-5, (e1, e2)


def test_mlp_adjoint_recompute_is_bitwise_and_full_size(tvi, mlp_full):
    y0, times, theta, yo = mlp_full
    obs = W.observed_steps(10000, every=100)
    y, st, _, ck = tvi.solve_forward("mlp", dev(y0), dev(times), dev(theta), chunk=100, tol=TOL32, checkpoints=True)
    g = _mlp_loss_grad(host(y), obs)
    a1 = tvi.solve_adjoint("mlp", dev(times), dev(theta), dev(g), ckpt=ck, chunk=100, tol=TOL32)
    a2 = tvi.solve_adjoint("mlp", dev(times), dev(theta), dev(g), y=y, chunk=100, tol=TOL32)
    assert np.array_equal(host(a1[0]), host(a2[0])) and np.array_equal(host(a1[1]), host(a2[1]))
    oth, oy0, _ = oracle.adjoint("mlp", yo, times.astype(np.float64), theta.astype(np.float64),
                                 _mlp_loss_grad(yo, obs))
    e1 = np.abs(host(a1[0]) - oth).max() / np.abs(oth).max()
    assert e1 <= 1e-5, e1


def test_mlp_gradient_matches_central_differences(tvi):
    """dL/dtheta along random directions against central differences (eps = 1e-4)
    of the float64 oracle's loss."""
    w = W.mlp(B=4, N=400)
    y0, times, theta = w["y0"], w["times"], w["params"]
    obs = W.observed_steps(400, every=100)
    f32 = lambda a: a.astype(np.float32)
    y, st, _, ck = tvi.solve_forward("mlp", dev(f32(y0)), dev(f32(times)), dev(f32(theta)), chunk=100, tol=TOL32,
                                     checkpoints=True)
    g = _mlp_loss_grad(host(y), obs)
    dth, _, _ = tvi.solve_adjoint("mlp", dev(f32(times)), dev(f32(theta)), dev(g), ckpt=ck, chunk=100, tol=TOL32)
    dth = host(dth)

    def loss(th):
        yy, _, _ = oracle.forward("mlp", y0, times, th, tol=(1e-13, 1e-13))
        return np.sum(yy[:, obs] ** 2) / (yy.shape[0] * len(obs) * 8)

    rng = np.random.default_rng(17)
    for _ in range(4):
        d = rng.standard_normal(theta.shape)
        d /= np.linalg.norm(d)
        fd = (loss(theta + 1e-4 * d) - loss(theta - 1e-4 * d)) / 2e-4
        assert abs(dth @ d - fd) <= 1e-4 * max(abs(fd), 1e-6) + 1e-7, (dth @ d, fd)


def test_mlp_double_storage_forward_and_adjoint(tvi):
    """Double inputs and outputs (the network still computes in float): the
    trajectory and gradient at the float gate against the oracle on the same
    float-rounded inputs, and recomputation bitwise equal to the stored path."""
    w = W.mlp(B=6, N=1500)
    y0, times, theta = (w[k].astype(np.float32).astype(np.float64) for k in ("y0", "times", "params"))
    yo, so, _ = oracle.forward("mlp", y0, times, theta, tol=(1e-12, 1e-12))
    assert (so == 0).all()
    d = lambda a: dev(a, torch.float64)
    y, st, _, ck = tvi.solve_forward("mlp", d(y0), d(times), d(theta), chunk=64, tol=TOL32, checkpoints=True)
    assert y.dtype == torch.float64 and (host(st) == 0).all()
    assert series_rel_err(host(y), yo).max() <= 1e-5
    obs = W.observed_steps(1500, every=100)
    g = _mlp_loss_grad(host(y), obs)
    a1 = tvi.solve_adjoint("mlp", d(times), d(theta), d(g), ckpt=ck, chunk=64, tol=TOL32)
    a2 = tvi.solve_adjoint("mlp", d(times), d(theta), d(g), y=y, chunk=64, tol=TOL32)
    assert torch.equal(a1[0], a2[0]) and torch.equal(a1[1], a2[1])
    oth, oy0, _ = oracle.adjoint("mlp", host(y), times, theta, g)
    assert np.abs(host(a1[0]) - oth).max() <= 1e-5 * np.abs(oth).max()
    assert np.abs(host(a1[1]) - oy0).max() <= 1e-5 * np.abs(oy0).max()
