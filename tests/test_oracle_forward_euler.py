"""Pins of the oracle's forward-Euler scheme (Section 2.2, Eq. forward-euler)
and of its discrete adjoint, against closed forms, an independent integrator's
order of accuracy and central finite differences of the forward map."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2310_08649_amd import workloads as W

FE = "forward_euler"


def ragged_grid(rng, B, n_range, dt):
    """Point offsets and times of B series of N_b uniform steps of dt from t = 0."""
    Nb = rng.integers(n_range[0], n_range[1] + 1, size=B)
    offsets = np.concatenate([[0], np.cumsum(Nb + 1)]).astype(np.int64)
    times = np.concatenate([dt * np.arange(N + 1) for N in Nb])
    return offsets, times


def test_fe_linear_closed_form():
    """y_k = (I + hA)^k y0 = Q diag((1 - h lam)^k) Q^T y0 for A = -Q diag(lam) Q^T."""
    w = W.linear(B=5, N=300, lam_range=(0.1, 100.0))  # h lam <= 1/3: a stable step
    y, st, it = oracle.forward("linear", w["y0"], w["times"], w["params"], scheme=FE)
    assert (st == 0).all() and (it == 0).all()
    h = w["times"][1] - w["times"][0]
    k = np.arange(301)
    c = np.einsum("bji,bj->bi", w["Q"], w["y0"])
    fac = (1.0 - h * w["lam"])[:, None, :] ** k[None, :, None]
    ref = np.einsum("bij,bkj,bj->bki", w["Q"], fac, c)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_fe_vdp_mu_zero_is_a_growing_rotation():
    """mu = 0: I + hA = sqrt(1 + h^2) R(-atan h), so y_k = (1 + h^2)^(k/2) R(-k atan h) y0."""
    N, T = 400, 4.0
    h = T / N
    times = np.linspace(0, T, N + 1)
    y0 = np.array([[1.2, -0.4], [-0.3, 0.9]])
    y, st, _ = oracle.forward("vanderpol", y0, times, np.zeros((2, 1)), scheme=FE)
    k = np.arange(N + 1)
    ang = -k * np.arctan(h)
    amp = (1.0 + h * h) ** (k / 2.0)
    ref = np.empty_like(y)
    ref[:, :, 0] = amp * (np.cos(ang) * y0[:, None, 0] - np.sin(ang) * y0[:, None, 1])
    ref[:, :, 1] = amp * (np.sin(ang) * y0[:, None, 0] + np.cos(ang) * y0[:, None, 1])
    assert np.abs(y - ref).max() <= 1e-12


@pytest.mark.parametrize("mu", [1.0, 3.0])
def test_fe_vdp_first_order_convergence(mu):
    y0 = np.array([1.5, 0.3])
    f = lambda t, y: np.array([y[1], mu * (1.0 - y[0] ** 2) * y[1] - y[0]])
    ref = solve_ivp(f, (0, 2), y0, method="Radau", rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for N in (800, 1600, 3200, 6400):
        y, st, _ = oracle.forward("vanderpol", y0[None], np.linspace(0, 2, N + 1), np.array([[mu]]), scheme=FE)
        errs.append(np.abs(y[0, -1] - ref).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 2.0) < 0.03), ratios


def test_fe_robertson_mass_conservation_on_a_stable_grid():
    rng = np.random.default_rng(7)
    offsets, times = ragged_grid(rng, 6, (50, 400), 1e-4)
    params = 10.0 ** rng.uniform(np.log10(0.5), np.log10(2.0), size=(6, 3))
    y0 = np.tile([1.0, 0.0, 0.0], (6, 1))
    y, st, _ = oracle.forward("robertson", y0, times, params, offsets=offsets, scheme=FE)
    assert (st == 0).all()
    assert np.abs(y.sum(axis=1) - 1.0).max() <= 1e-14


def test_fe_adjoint_linear_closed_form():
    """dL/dy0 = sum_k (S^k)^T g_k and dL/dA = sum_k h lam_k y_{k-1}^T with S = I + hA,
    lam_k = sum_{i >= k} (S^{i-k})^T g_i."""
    w = W.linear(B=3, N=40, lam_range=(0.1, 10.0))
    rng = np.random.default_rng(5)
    params = w["params"] + 3.0 * rng.standard_normal(w["params"].shape)  # non-symmetric
    y, st, _ = oracle.forward("linear", w["y0"], w["times"], params, scheme=FE)
    g = rng.standard_normal(y.shape)
    dLdp, dLdy0, ast = oracle.adjoint("linear", y, w["times"], params, g, scheme=FE)
    assert (ast == 0).all()
    h = w["times"][1] - w["times"][0]
    N = y.shape[1] - 1
    for b in range(3):
        S = np.eye(4) + h * params[b].reshape(4, 4)
        pw = [np.eye(4)]
        for _ in range(N):
            pw.append(S @ pw[-1])
        acc = sum(pw[k].T @ g[b, k] for k in range(N + 1))
        np.testing.assert_allclose(dLdy0[b], acc, rtol=1e-12, atol=1e-12)
        lam = [None] + [sum(pw[i - k].T @ g[b, i] for i in range(k, N + 1)) for k in range(1, N + 1)]
        dA = sum(h * np.outer(lam[k], y[b, k - 1]) for k in range(1, N + 1))
        np.testing.assert_allclose(dLdp[b].reshape(4, 4), dA, rtol=1e-11, atol=1e-12)


def _fd_case(kind, y0, times, params, offsets=None, hidden=64, dirs=6, eps=1e-6, dy_scale=1.0):
    shared = params.ndim == 1
    fwd = lambda y0_, p_: oracle.forward(kind, y0_, times, p_, offsets=offsets, hidden=hidden,
                                        params_shared=shared, scheme=FE)[0]
    loss = lambda y: np.sqrt(np.sum(y ** 2))
    y = fwd(y0, params)
    g = y / loss(y)
    dLdp, dLdy0, st = oracle.adjoint(kind, y, times, params, g, offsets=offsets, hidden=hidden,
                                     params_shared=shared, scheme=FE)
    assert (st == 0).all()
    rng = np.random.default_rng(22)
    for _ in range(dirs):
        dp = rng.standard_normal(params.shape) * np.maximum(np.abs(params), 1e-3)
        dy = rng.standard_normal(y0.shape) * dy_scale
        fd = (loss(fwd(y0 + eps * dy, params + eps * dp)) - loss(fwd(y0 - eps * dy, params - eps * dp))) / (2 * eps)
        an = np.sum(dLdp * dp) + np.sum(dLdy0 * dy)
        assert abs(an - fd) <= 1e-7 * max(abs(fd), 1e-8), (an, fd)


def test_fe_adjoint_fd_vanderpol():
    w = W.vanderpol(B=4, N=600, mu_range=(1.0, 10.0))
    _fd_case("vanderpol", w["y0"], np.linspace(0, 1.5, 601), w["params"])


def test_fe_adjoint_fd_robertson_ragged():
    rng = np.random.default_rng(8)
    offsets, times = ragged_grid(rng, 4, (30, 200), 1e-4)
    params = 10.0 ** rng.uniform(np.log10(0.5), np.log10(2.0), size=(4, 3))
    # y2 stays small: 2 k2 y2 h must stay below 2 for a stable step
    y0 = np.tile([1.0, 0.0, 0.0], (4, 1)) + rng.random((4, 3)) * np.array([0.01, 1e-6, 0.01])
    # directions in y0 sized to each component (y2 is of order 1e-5)
    _fd_case("robertson", y0, times, params, offsets=offsets, dy_scale=np.array([1.0, 1e-6, 1.0]))


def test_fe_adjoint_fd_mlp_shared_params():
    w = W.mlp(B=3, N=50, hidden=16)
    _fd_case("mlp", w["y0"], w["times"], w["params"], hidden=16, eps=1e-5)


def test_fe_ragged_equals_individual_runs_and_empty_series():
    rng = np.random.default_rng(9)
    offsets, times = ragged_grid(rng, 5, (0, 30), 1e-2)
    params = 10.0 ** rng.uniform(0, 1, size=(5, 1))
    y0 = rng.uniform(-2, 2, size=(5, 2))
    y, st, _ = oracle.forward("vanderpol", y0, times, params, offsets=offsets, scheme=FE)
    g = rng.standard_normal(y.shape)
    dp, dy0, _ = oracle.adjoint("vanderpol", y, times, params, g, offsets=offsets, scheme=FE)
    for b in range(5):
        a, e = offsets[b], offsets[b + 1]
        yb, _, _ = oracle.forward("vanderpol", y0[b:b + 1], times[a:e], params[b:b + 1], scheme=FE)
        assert np.array_equal(yb[0], y[a:e])
        pb, y0b, _ = oracle.adjoint("vanderpol", yb, times[a:e], params[b:b + 1], g[None, a:e], scheme=FE)
        assert np.array_equal(pb[0], dp[b]) and np.array_equal(y0b[0], dy0[b])
        if e - a == 1:  # no step: dL/dy0 = g_0 and no parameter gradient
            assert np.array_equal(dy0[b], g[a]) and (dp[b] == 0).all()


def test_fe_blowup_is_reported():
    """An unstable step (h lam = 3 on lam = 3000) grows without bound: NONFINITE and NaN."""
    w = W.linear(B=2, N=2000, lam_range=(3000.0, 3000.0), t_end=2.0)
    y, st, _ = oracle.forward("linear", w["y0"], w["times"], w["params"], scheme=FE)
    assert (st == 3).all()
    assert np.isnan(y[:, -1]).all()
