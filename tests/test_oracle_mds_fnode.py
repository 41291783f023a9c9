"""Pins of the oracle's mass-damper-spring chain and forced neural ODE
(Section 5.1.1), and of the coupled-neuron model at the study's larger sizes.

Mass-damper-spring: the model is linear, so its pins are physical identities
of the backward-Euler map that a wrong sign, index or mass would break:
momentum balance step by step (internal forces cancel pairwise, only the
applied force and the wall act), the exact energy identity of backward Euler
for a conservative or damped chain, the closed-form forced damped oscillator
for one unit (first-order convergence), and the rate, Jacobian and parameter
gradient against a stiffness-matrix assembly written element by element.
Forced neural ODE: rate, Jacobian and parameter gradient against a torch
transcription built from torch.nn.functional.linear with autograd, the
constant-rate special case (exact), first-order convergence to Radau.  Both:
the adjoint against central differences of the whole forward map."""
import math

import numpy as np
import pytest
import torch
from scipy.integrate import solve_ivp

import oracle
from paper_2310_08649_amd import workloads as W

TIGHT = (1e-14, 1e-13)


# --------------------------------------------------------------------------
# mass-damper-spring
# --------------------------------------------------------------------------
def mds_matrices(p, nu):
    """Stiffness and damping matrices by element assembly (torch, differentiable
    in p): spring i joins mass i and mass i+1 (the wall for the last one) and
    adds k [[1, -1], [-1, 1]] over its two ends; a wall end is dropped."""
    K, C = p[:nu], p[nu:2 * nu]
    rows_k, rows_c = [], []
    for a in range(nu):
        rk, rc = [], []
        for b in range(nu):
            sk = torch.zeros((), dtype=torch.float64)
            sc = torch.zeros((), dtype=torch.float64)
            for i in range(nu):
                ends = [i] + ([i + 1] if i + 1 < nu else [])
                if a in ends and b in ends:
                    sgn = 1.0 if a == b else -1.0
                    sk = sk + sgn * K[i]
                    sc = sc + sgn * C[i]
            rk.append(sk)
            rc.append(sc)
        rows_k.append(torch.stack(rk))
        rows_c.append(torch.stack(rc))
    return torch.stack(rows_k), torch.stack(rows_c)


def mds_ref(y, t, p):
    """Torch rate from the assembled matrices: M dv/dt = -K d - C v + M f."""
    nu = y.shape[0] // 2
    Km, Cm = mds_matrices(p, nu)
    d, v = y[0::2], y[1::2]
    M, fa, T = p[2 * nu:3 * nu], p[3 * nu], p[3 * nu + 1]
    force = torch.cat([(fa * torch.sin(2 * math.pi * t / T)).reshape(1), torch.zeros(nu - 1, dtype=torch.float64)])
    acc = -(Km @ d + Cm @ v) / M + force
    return torch.stack([v, acc], dim=1).reshape(-1)


def mds_split(p, nu):
    return p[:nu], p[nu:2 * nu], p[2 * nu:3 * nu], p[3 * nu], p[3 * nu + 1]


def _mds_params(nu, rng):
    p = W.mds(nu, 3)["params"][1].copy()
    p[:3 * nu] *= np.exp(0.3 * rng.standard_normal(3 * nu))  # off the linspace table
    return p


@pytest.mark.parametrize("nu", [1, 2, 3, 5, 10])
def test_mds_rate_and_jacobian_match_element_assembly(nu):
    rng = np.random.default_rng(41 + nu)
    p = _mds_params(nu, rng)
    y = 1e-4 * rng.standard_normal(2 * nu)
    t = 0.0123
    f, J = oracle.rhs("mds", y, t, p)
    ref = mds_ref(torch.tensor(y), t, torch.tensor(p)).numpy()
    np.testing.assert_allclose(f, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    Jt = torch.autograd.functional.jacobian(lambda v: mds_ref(v, t, torch.tensor(p)), torch.tensor(y)).numpy()
    np.testing.assert_allclose(J, Jt, rtol=1e-12, atol=1e-13 * np.abs(Jt).max())


@pytest.mark.parametrize("nu", [1, 3, 10])
def test_mds_parameter_gradient_matches_autograd(nu):
    """(dh/dp)^T w against autograd through the element-assembled rate."""
    rng = np.random.default_rng(7 + nu)
    p = _mds_params(nu, rng)
    y = 1e-4 * rng.standard_normal(2 * nu)
    t, w = 0.31, rng.standard_normal(2 * nu)
    pt = torch.tensor(p, requires_grad=True)
    mds_ref(torch.tensor(y), t, pt).backward(torch.tensor(w))
    ref = pt.grad.numpy()
    np.testing.assert_allclose(oracle.vjp_p("mds", y, t, p, w), ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("nu", [1, 2, 5])
def test_mds_momentum_balance_every_step(nu):
    """Internal spring and damper forces cancel in pairs, so every backward-Euler
    step satisfies sum_i M_i (v_i^k - v_i^{k-1}) = dt (M_1 f(t_k) - K_nu d_nu^k - C_nu v_nu^k):
    only the applied force and the wall spring and damper change the momentum."""
    w = W.mds(nu, 3, n_time=400, t_max=0.2)
    y, st, _ = oracle.forward("mds", w["y0"], w["times"], w["params"], tol=TIGHT)
    assert (st == 0).all()
    t = w["times"]
    h = t[1] - t[0]
    for b in range(3):
        K, C, M, fa, T = mds_split(w["params"][b], nu)
        v, d = y[b, :, 1::2], y[b, :, 0::2]
        lhs = (M[None, :] * np.diff(v, axis=0)).sum(axis=1)
        rhs = h * (M[0] * fa * np.sin(2 * np.pi * t[1:] / T) - K[-1] * d[1:, -1] - C[-1] * v[1:, -1])
        scale = h * M[0] * fa
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-9 * scale)


@pytest.mark.parametrize("nu", [2, 5])
@pytest.mark.parametrize("damped", [False, True])
def test_mds_backward_euler_energy_identity(nu, damped):
    """Unforced chain, energy E = 1/2 sum M_i v_i^2 + 1/2 sum K_i (d_i - d_{i+1})^2
    (d_{nu+1} = 0).  Backward Euler on this system satisfies exactly
    E_{k-1} - E_k = 1/2 |y_k - y_{k-1}|_E^2 + dt sum_i C_i (v_i^k - v_{i+1}^k)^2:
    numerical dissipation plus the dampers' work, each step."""
    rng = np.random.default_rng(11 * nu + damped)
    w = W.mds(nu, 1, n_time=300, t_max=0.05)
    p = w["params"].copy()
    p[0, 3 * nu] = 0.0            # no applied force
    if not damped:
        p[0, nu:2 * nu] = 0.0     # no dampers
    y0 = 1e-4 * rng.standard_normal((1, 2 * nu))
    y, st, _ = oracle.forward("mds", y0, w["times"], p, tol=TIGHT)
    assert (st == 0).all()
    K, C, M, _, _ = mds_split(p[0], nu)
    h = w["times"][1] - w["times"][0]

    def energy(s):
        d, v = s[..., 0::2], s[..., 1::2]
        dn = np.concatenate([d[..., 1:], np.zeros(d.shape[:-1] + (1,))], axis=-1)
        return 0.5 * (M * v ** 2).sum(-1) + 0.5 * (K * (d - dn) ** 2).sum(-1)

    def damper_work(s):
        v = s[..., 1::2]
        vn = np.concatenate([v[..., 1:], np.zeros(v.shape[:-1] + (1,))], axis=-1)
        return (C * (v - vn) ** 2).sum(-1)

    E = energy(y[0])
    lhs = E[:-1] - E[1:]
    rhs = energy(np.diff(y[0], axis=0)) + h * damper_work(y[0, 1:])
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-9 * E[0])
    assert np.all(lhs > 0)


def test_mds_single_unit_converges_to_forced_oscillator():
    """One unit is the forced damped oscillator d'' + (C/M) d' + (K/M) d = f_a sin(W t)
    from rest; backward Euler approaches its closed form at first order."""
    p = np.array([0.5, 2e-5, 1e-5, 1.0, 0.02])
    K, C, M, fa, T = p
    w0, zeta, Om = math.sqrt(K / M), C / (2 * M * math.sqrt(K / M)), 2 * math.pi / T
    den = (w0 ** 2 - Om ** 2) ** 2 + (2 * zeta * w0 * Om) ** 2
    A, Bc = fa * (w0 ** 2 - Om ** 2) / den, -fa * 2 * zeta * w0 * Om / den
    wd = w0 * math.sqrt(1 - zeta ** 2)
    c1 = -Bc
    c2 = (zeta * w0 * c1 - A * Om) / wd

    def exact(t):
        e = math.exp(-zeta * w0 * t)
        d = A * math.sin(Om * t) + Bc * math.cos(Om * t) + e * (c1 * math.cos(wd * t) + c2 * math.sin(wd * t))
        v = (A * Om * math.cos(Om * t) - Bc * Om * math.sin(Om * t)
             + e * ((-zeta * w0 * c1 + wd * c2) * math.cos(wd * t) + (-zeta * w0 * c2 - wd * c1) * math.sin(wd * t)))
        return np.array([d, v])

    t_end = 0.03
    ref = exact(t_end)
    errs = []
    for N in (4000, 8000, 16000, 32000):
        y, st, _ = oracle.forward("mds", np.zeros((1, 2)), np.linspace(0, t_end, N + 1), p[None], tol=TIGHT)
        assert (st == 0).all()
        errs.append(np.abs(y[0, -1] - ref).max() / np.abs(ref).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 2.0) < 0.1), (errs, ratios)


# --------------------------------------------------------------------------
# forced neural ODE
# --------------------------------------------------------------------------
def fnode_ref(y, t, p):
    """Torch transcription: three torch.nn.functional.linear layers on (y, f(t))."""
    n = y.shape[0]
    m = n + 1
    sizes = [("W1", (m, m)), ("b1", (m,)), ("W2", (m, m)), ("b2", (m,)), ("W3", (n, m)), ("b3", (n,))]
    q, o = {}, 0
    for name, sh in sizes:
        k = int(np.prod(sh))
        q[name] = p[o:o + k].reshape(sh)
        o += k
    fa, T = p[o], p[o + 1]
    x = torch.cat([y, (fa * torch.sin(2 * math.pi * t / T)).reshape(1)])
    F = torch.nn.functional
    a1 = torch.tanh(F.linear(x, q["W1"], q["b1"]))
    a2 = torch.tanh(F.linear(a1, q["W2"], q["b2"]))
    return torch.tanh(F.linear(a2, q["W3"], q["b3"]))


@pytest.mark.parametrize("nu", [1, 5, 10, 25])
def test_fnode_rate_jacobian_and_parameter_gradient_match_autograd(nu):
    rng = np.random.default_rng(60 + nu)
    p = W.fnode(nu, 3)["params"][2].copy()
    p[:-2] *= 1.0 + 0.5 * rng.standard_normal(p.shape[0] - 2)  # enter the tanh's curved range
    y = rng.standard_normal(nu)
    t = 0.137
    f, J = oracle.rhs("fnode", y, t, p)
    yt, pt = torch.tensor(y, requires_grad=True), torch.tensor(p, requires_grad=True)
    ref = fnode_ref(yt, t, pt)
    np.testing.assert_allclose(f, ref.detach().numpy(), rtol=1e-13, atol=1e-14)
    Jt = torch.autograd.functional.jacobian(lambda v: fnode_ref(v, t, torch.tensor(p)), torch.tensor(y)).numpy()
    np.testing.assert_allclose(J, Jt, rtol=1e-12, atol=1e-13 * np.abs(Jt).max())
    w = rng.standard_normal(nu)
    ref.backward(torch.tensor(w))
    np.testing.assert_allclose(oracle.vjp_p("fnode", y, t, p, w), pt.grad.numpy(), rtol=1e-12,
                               atol=1e-13 * max(1.0, np.abs(pt.grad.numpy()).max()))


def test_fnode_constant_rate_is_exact():
    """With W3 = 0 the rate is the constant tanh(b3): backward Euler reproduces
    y_k = y_0 + t_k tanh(b3) exactly (one Newton correction per step)."""
    nu = 5
    w = W.fnode(nu, 2, n_time=300)
    p = w["params"].copy()
    m = nu + 1
    o3 = 2 * m * m + 2 * m
    p[:, o3:o3 + nu * m] = 0.0
    b3 = p[0, o3 + nu * m:o3 + nu * m + nu]
    y0 = np.random.default_rng(3).standard_normal((2, nu))
    y, st, _ = oracle.forward("fnode", y0, w["times"], p, tol=TIGHT)
    assert (st == 0).all()
    ref = y0[:, None, :] + w["times"][None, :, None] * np.tanh(b3)[None, None, :]
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nu", [1, 5])
def test_fnode_first_order_convergence_to_radau(nu):
    w = W.fnode(nu, 3)
    p = w["params"][1]
    p = p.copy()
    p[:-2] *= 2.0  # a non-trivial trajectory
    y0 = 0.3 * np.ones(nu)
    t_end = 0.5
    fun = lambda t, y: fnode_ref(torch.tensor(y), t, torch.tensor(p)).numpy()
    ref = solve_ivp(fun, (0, t_end), y0, method="Radau", rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for N in (1000, 2000, 4000, 8000):
        y, st, _ = oracle.forward("fnode", y0[None], np.linspace(0, t_end, N + 1), p[None], tol=TIGHT)
        assert (st == 0).all()
        errs.append(np.abs(y[0, -1] - ref).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 2.0) < 0.05), ratios


# --------------------------------------------------------------------------
# the coupled-neuron model at the study's larger sizes (n = 4 n_unit up to 40)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("nu", [3, 6, 10])
def test_neuron_large_rate_jacobian_and_gradient_match_autograd(nu):
    from tests.test_oracle_paper_models import neuron_ref
    rng = np.random.default_rng(90 + nu)
    p = W.neuron(nu, 3)["params"][1].copy()
    p[:15 * nu] *= np.exp(0.2 * rng.standard_normal(15 * nu))
    y = rng.uniform(0.05, 1.0, size=4 * nu)
    t = 0.77
    f, J = oracle.rhs("neuron", y, t, p)
    yt, pt = torch.tensor(y, requires_grad=True), torch.tensor(p, requires_grad=True)
    ref = neuron_ref(yt, t, pt)
    np.testing.assert_allclose(f, ref.detach().numpy(), rtol=1e-13, atol=1e-14)
    Jt = torch.autograd.functional.jacobian(lambda v: neuron_ref(v, t, torch.tensor(p)), torch.tensor(y)).numpy()
    np.testing.assert_allclose(J, Jt, rtol=1e-12, atol=1e-13 * np.abs(Jt).max())
    w = rng.standard_normal(4 * nu)
    ref.backward(torch.tensor(w))
    np.testing.assert_allclose(oracle.vjp_p("neuron", y, t, p, w), pt.grad.numpy(), rtol=1e-12,
                               atol=1e-13 * max(1.0, np.abs(pt.grad.numpy()).max()))


# --------------------------------------------------------------------------
# adjoints against central differences
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind,nu,t_max,y0s", [("mds", 1, 0.05, 1e-5), ("mds", 3, 0.05, 1e-5),
                                                ("fnode", 1, 1.0, 0.1), ("fnode", 5, 1.0, 0.1),
                                                ("neuron", 3, 3.0, 0.05)])
def test_adjoint_matches_central_differences(kind, nu, t_max, y0s):
    w = getattr(W, kind)(nu, 3, n_time=300, t_max=t_max)
    times, params = w["times"], w["params"].copy()
    if kind == "fnode":
        # forcing periods the 300-step grid resolves: at T = 0.01 the loss varies
        # with T on a scale below the difference step
        params[:, -1] = np.linspace(0.25, 1.0, 3)
    y0 = y0s * np.random.default_rng(2).random(w["y0"].shape)

    def fwd(y0_, p_):
        return oracle.forward(kind, y0_, times, p_, tol=TIGHT)[0]

    y = fwd(y0, params)
    L = np.sqrt(np.sum(y ** 2))
    dp, dy0, st = oracle.adjoint(kind, y, times, params, y / L)
    assert (st == 0).all()
    rng = np.random.default_rng(23)
    for _ in range(4):
        d = rng.standard_normal(params.shape) * np.abs(params)
        dy = rng.standard_normal(y0.shape) * y0s
        eps = 1e-6
        fd = (np.sqrt(np.sum(fwd(y0 + eps * dy, params + eps * d) ** 2))
              - np.sqrt(np.sum(fwd(y0 - eps * dy, params - eps * d) ** 2))) / (2 * eps)
        an = np.sum(dp * d) + np.sum(dy0 * dy)
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-8 * L), (an, fd)
