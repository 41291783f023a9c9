"""Pins of the oracle's Chaboche and coupled-neuron models (Section 5.1.1)
against independent torch transcriptions (rate, state Jacobian and parameter
gradient by autograd), closed forms of special cases, first-order convergence
to scipy's Radau on the transcription, and central differences of the whole
forward map for the adjoint."""
import math

import numpy as np
import pytest
import torch
from scipy.integrate import solve_ivp

import oracle
from paper_2310_08649_amd import workloads as W

TIGHT = (1e-14, 1e-13)


# --------------------------------------------------------------------------
# Independent transcriptions (torch, float64) from the paper's equations
# --------------------------------------------------------------------------
def chaboche_ref(y, t, p):
    nu = y.shape[0] - 2
    E, ex, eta, s0, Kinf, tau = p[0], p[1], p[2], p[3], p[4], p[5]
    C, gam, eda, T = p[6:6 + nu], p[6 + nu:6 + 2 * nu], p[6 + 2 * nu], p[7 + 2 * nu]
    sig, K, X = y[0], y[1], y[2:]
    s = sig - X.sum()
    over = torch.clamp((torch.abs(s) - K - s0) / eta, min=0.0)
    rate = over ** ex                      # |plastic strain rate|
    ep = rate * torch.sign(s)
    edot = eda * torch.sin(2 * math.pi * t / T)
    return torch.cat([(E * (edot - ep)).reshape(1), (tau * (Kinf - K) * rate).reshape(1),
                      2.0 / 3.0 * C * ep - gam * X * rate])


def neuron_ref(y, t, p):
    nu = y.shape[0] // 4
    Ia = p[15 * nu]
    out = []
    V = y[0::4]
    for i in range(nu):
        q = p[15 * i:15 * (i + 1)]
        C, gNa, ENa, gK, EK, gL, EL, minf, tm, hinf, th, ninf, tn, gC, T = [q[k] for k in range(15)]
        v, m, h, n = y[4 * i], y[4 * i + 1], y[4 * i + 2], y[4 * i + 3]
        I = Ia * torch.sin(2 * math.pi * t / T)
        dv = (-gNa * m ** 3 * h * (v - ENa) - gK * n ** 4 * (v - EK) - gL * (v - EL) + I + gC * (v - V).sum()) / C
        out += [dv.reshape(1), ((minf - m) / tm).reshape(1), ((hinf - h) / th).reshape(1),
                ((ninf - n) / tn).reshape(1)]
    return torch.cat(out)


REF = {"chaboche": chaboche_ref, "neuron": neuron_ref}


def _cases():
    rng = np.random.default_rng(31)
    out = []
    for nu in (1, 2, 3):
        p = W.chaboche(nu, 2)["params"][1].copy()
        # plastic states: |s| well above K + sigma0, both signs of s
        for sgn in (1.0, -1.0):
            y = np.concatenate([[sgn * 3.0, 0.4], 0.1 * rng.standard_normal(nu)])
            out.append(("chaboche", y, 0.37, p))
        out.append(("chaboche", np.concatenate([[0.3, 0.4], 0.05 * rng.standard_normal(nu)]), 0.2, p))  # elastic
    for nu in (1, 2):
        p = W.neuron(nu, 3)["params"][2].copy()
        p[:15 * nu] *= np.exp(0.2 * rng.standard_normal(15 * nu))  # off the symmetric table values
        y = rng.uniform(0.05, 1.0, size=4 * nu)
        out.append(("neuron", y, 1.3, p))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: "%s-n%d" % (c[0], c[1].shape[0]))
def test_rate_jacobian_and_parameter_gradient_match_autograd(case):
    kind, y, t, p = case
    f, J = oracle.rhs(kind, y, t, p)
    yt, pt = torch.tensor(y, requires_grad=True), torch.tensor(p, requires_grad=True)
    ref = REF[kind](yt, t, pt)
    np.testing.assert_allclose(f, ref.detach().numpy(), rtol=1e-13, atol=1e-14)
    Jt = torch.autograd.functional.jacobian(lambda v: REF[kind](v, t, torch.tensor(p)), torch.tensor(y)).numpy()
    np.testing.assert_allclose(J, Jt, rtol=1e-12, atol=1e-13 * np.abs(Jt).max())
    w = np.random.default_rng(5).standard_normal(y.shape[0])
    ref.backward(torch.tensor(w))
    np.testing.assert_allclose(oracle.vjp_p(kind, y, t, p, w), pt.grad.numpy(), rtol=1e-12,
                               atol=1e-13 * max(1.0, np.abs(pt.grad.numpy()).max()))


def test_chaboche_elastic_closed_form():
    """Below the yield surface the plastic rate is zero: K and X stay put and
    backward Euler gives sigma_k = sigma_0 + sum_{i<=k} dt E edot(t_i) exactly."""
    w = W.chaboche(2, 3, n_time=500)
    p = w["params"].copy()
    p[:, 3] = 100.0  # sigma0: never reached
    y0 = np.array([[0.2, 0.5, 0.01, -0.02]] * 3)
    y, st, _ = oracle.forward("chaboche", y0, w["times"], p, tol=TIGHT)
    assert (st == 0).all()
    t = w["times"]
    h = t[1] - t[0]
    for b in range(3):
        edot = p[b, -2] * np.sin(2 * np.pi * t[1:] / p[b, -1])
        sig = y0[b, 0] + np.concatenate([[0.0], np.cumsum(h * p[b, 0] * edot)])
        np.testing.assert_allclose(y[b, :, 0], sig, rtol=1e-12, atol=1e-13)
        assert (y[b, :, 1:] == y0[b, 1:]).all()


def test_neuron_gating_closed_form():
    """The gating variables decay linearly to their constant targets: backward Euler
    gives x_k = x_inf + (x_0 - x_inf) (1 + dt / tau)^(-k) for m, h and n."""
    w = W.neuron(2, 2, n_time=400)
    y0 = np.array([[0.0, 0.9, 0.05, 0.7, 0.3, 0.2, 0.8, 0.1]] * 2)
    y, st, _ = oracle.forward("neuron", y0, w["times"], w["params"], tol=TIGHT)
    assert (st == 0).all()
    h = w["times"][1] - w["times"][0]
    k = np.arange(401)
    for b in range(2):
        for i in range(2):
            q = w["params"][b, 15 * i:15 * (i + 1)]
            for comp, (xinf, tau) in enumerate(((q[7], q[8]), (q[9], q[10]), (q[11], q[12])), start=1):
                ref = xinf + (y0[b, 4 * i + comp] - xinf) * (1.0 + h / tau) ** (-k)
                np.testing.assert_allclose(y[b, :, 4 * i + comp], ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("kind,nu", [("chaboche", 2), ("neuron", 2)])
@pytest.mark.parametrize("scheme", ["backward_euler", "forward_euler"])
def test_first_order_convergence_to_radau(kind, nu, scheme):
    w = getattr(W, kind)(nu, 2)
    p = w["params"][1]
    y0 = np.zeros(w["n"])
    t_end = 2.0
    fun = lambda t, y: REF[kind](torch.tensor(y), t, torch.tensor(p)).numpy()
    ref = solve_ivp(fun, (0, t_end), y0, method="Radau", rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for N in (1000, 2000, 4000, 8000):
        y, st, _ = oracle.forward(kind, y0[None], np.linspace(0, t_end, N + 1), p[None], tol=TIGHT, scheme=scheme)
        assert (st == 0).all()
        errs.append(np.abs(y[0, -1] - ref).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 2.0) < 0.05), ratios


@pytest.mark.parametrize("kind,nu", [("chaboche", 1), ("chaboche", 2), ("neuron", 1), ("neuron", 2)])
@pytest.mark.parametrize("scheme", ["backward_euler", "forward_euler"])
def test_adjoint_matches_central_differences(kind, nu, scheme):
    w = getattr(W, kind)(nu, 3, n_time=300, t_max=3.0)
    times, params = w["times"], w["params"]
    y0 = 0.05 * np.random.default_rng(2).random(w["y0"].shape)

    def fwd(y0_, p_):
        return oracle.forward(kind, y0_, times, p_, tol=TIGHT, scheme=scheme)[0]

    y = fwd(y0, params)
    L = np.sqrt(np.sum(y ** 2))
    dp, dy0, st = oracle.adjoint(kind, y, times, params, y / L, scheme=scheme)
    assert (st == 0).all()
    rng = np.random.default_rng(23)
    for _ in range(4):
        d = rng.standard_normal(params.shape) * np.abs(params)
        dy = rng.standard_normal(y0.shape) * 0.01
        eps = 1e-6
        fd = (np.sqrt(np.sum(fwd(y0 + eps * dy, params + eps * d) ** 2))
              - np.sqrt(np.sum(fwd(y0 - eps * dy, params - eps * d) ** 2))) / (2 * eps)
        an = np.sum(dp * d) + np.sum(dy0 * dy)
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-8), (an, fd)
