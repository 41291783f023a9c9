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
