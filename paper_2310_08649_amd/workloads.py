"""Seeded synthetic workloads.

Input generators only: they draw initial states, time grids and model
parameters with ``numpy.random.default_rng(seed)`` in a fixed order and hold
none of the integration method's arithmetic.  The same arrays feed the HIP
library and the CPU oracle.

The paper measures on its own synthetic ODE problems (Section 5.1); there is
no dataset to stand in for.  The five workloads below are those the library
is benchmarked and tested on:

* ``linear``     stiff linear system dy/dt = A y, n = 4, A = -Q diag(lam) Q^T with
                 Q Haar-orthogonal and lam log-uniform in [0.1, 1000]
* ``vanderpol``  Van der Pol, n = 2, mu log-uniform in [1, 1000], y0 ~ U(-2, 2)
* ``mlp``        neural ODE dy/dt = MLP(y; theta), n = 8, two tanh layers of 64,
                 theta ~ N(0, 0.1^2), y0 ~ N(0, 1)
* ``robertson``  Robertson kinetics, n = 3, rate scale factors log-uniform in
                 [0.5, 2], series lengths log-uniform in [100, 20000] on
                 log-spaced grids over [1e-5, 1e4], y0 = (1, 0, 0)

and two of the paper's own example problems with its parameter tables
(Section 5.1.1; deterministic, no draws):

* ``chaboche``   Chaboche viscoplasticity, n = 2 + n_unit backstresses
* ``neuron``     coupled neurons, n = 4 n_unit
* ``mds``        mass-damper-spring chain, n = 2 n_unit
* ``fnode``      forced neural ODE, n = n_unit (weights drawn once, seeded)

Every generator returns a dict of contiguous numpy arrays in the library's
series-major layouts (see ``include/tvi.h``).
"""
from __future__ import annotations

import numpy as np


def haar_orthogonal(rng, n):
    """A Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the signs fixed by diag(R)."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))[None, :]


def linear(B=8, N=200, n=4, seed=101, t_end=1.0, lam_range=(0.1, 1000.0)):
    """Stiff linear system; returns A [B,n,n] (as params [B,n*n]) with its Q and lam."""
    rng = np.random.default_rng(seed)
    Q = np.empty((B, n, n))
    lam = np.empty((B, n))
    lo, hi = np.log10(lam_range[0]), np.log10(lam_range[1])
    for b in range(B):
        Q[b] = haar_orthogonal(rng, n)
        lam[b] = 10.0 ** rng.uniform(lo, hi, size=n)
    y0 = rng.standard_normal((B, n))
    A = -np.einsum("bij,bj,bkj->bik", Q, lam, Q)
    times = np.linspace(0.0, t_end, N + 1)
    return dict(kind="linear", n=n, y0=y0, times=times, params=A.reshape(B, n * n).copy(),
                Q=Q, lam=lam, offsets=None)


def vanderpol(B=512, N=5000, seed=102, t_end=10.0, mu_range=(1.0, 1000.0)):
    rng = np.random.default_rng(seed)
    mu = 10.0 ** rng.uniform(np.log10(mu_range[0]), np.log10(mu_range[1]), size=B)
    y0 = rng.uniform(-2.0, 2.0, size=(B, 2))
    times = np.linspace(0.0, t_end, N + 1)
    return dict(kind="vanderpol", n=2, y0=y0, times=times, params=mu.reshape(B, 1).copy(), offsets=None)


def mlp_theta(rng, n=8, hidden=64, scale=0.1):
    """theta packed as W1[H][n], b1[H], W2[H][H], b2[H], W3[n][H], b3[n], each drawn in that order."""
    parts = [
        scale * rng.standard_normal(hidden * n),
        scale * rng.standard_normal(hidden),
        scale * rng.standard_normal(hidden * hidden),
        scale * rng.standard_normal(hidden),
        scale * rng.standard_normal(n * hidden),
        scale * rng.standard_normal(n),
    ]
    return np.concatenate(parts)


def mlp(B=64, N=10000, n=8, hidden=64, seed=103, t_end=1.0):
    rng = np.random.default_rng(seed)
    theta = mlp_theta(rng, n, hidden)
    y0 = rng.standard_normal((B, n))
    times = np.linspace(0.0, t_end, N + 1)
    return dict(kind="mlp", n=n, hidden=hidden, y0=y0, times=times, params=theta, offsets=None)


def robertson(B=2000, seed=104, n_range=(100, 20000), t_range=(1e-5, 1e4), s_range=(0.5, 2.0)):
    """Ragged Robertson series: point offsets [B+1], times [points] (log-spaced per series)."""
    rng = np.random.default_rng(seed)
    s = 10.0 ** rng.uniform(np.log10(s_range[0]), np.log10(s_range[1]), size=(B, 3))
    Nb = np.rint(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]), size=B))).astype(np.int64)
    Nb = np.maximum(Nb, 1)
    offsets = np.zeros(B + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(Nb + 1)
    lt0, lt1 = np.log10(t_range[0]), np.log10(t_range[1])
    times = np.empty(int(offsets[-1]))
    for b in range(B):
        k = np.arange(Nb[b] + 1, dtype=np.float64)
        times[offsets[b]:offsets[b + 1]] = 10.0 ** (lt0 + (lt1 - lt0) * k / Nb[b])
    y0 = np.tile(np.array([1.0, 0.0, 0.0]), (B, 1))
    return dict(kind="robertson", n=3, y0=y0, times=times, params=s, offsets=offsets, steps=Nb)


def observed_steps(N, every=100):
    """Observed step indices of the sampled mean-squared loss: k = every, 2 every, ..., N."""
    return np.arange(every, N + 1, every, dtype=np.int64)


def chaboche(n_unit=1, n_batch=3, n_time=2000, t_max=10.0):
    """The Chaboche timing case: E = 10, n = 5, eta = 2, sigma0 = 1, K_inf = 10,
    tau = 1, C_i = linspace(0.1, 1, n_unit), gamma_i = linspace(0.1, 0.5, n_unit),
    edot_a = linspace(0.1, 1, n_batch) (one value per series), T = 1, t in
    [0, t_max] in n_time equal steps, zero initial state.  Parameter vector per
    series: (E, n, eta, sigma0, K_inf, tau, C_1..C_nu, gamma_1..gamma_nu, edot_a, T)."""
    nu = n_unit
    base = np.concatenate([[10.0, 5.0, 2.0, 1.0, 10.0, 1.0], np.linspace(0.1, 1.0, nu), np.linspace(0.1, 0.5, nu)])
    params = np.array([np.concatenate([base, [ea, 1.0]]) for ea in np.linspace(0.1, 1.0, n_batch)])
    n = 2 + nu
    return dict(kind="chaboche", n=n, y0=np.zeros((n_batch, n)), times=np.linspace(0.0, t_max, n_time + 1),
                params=params, offsets=None)


NEURON_TABLE = (  # per neuron: (lo, hi) of linspace over the neurons, in the parameter order
    ("C", 0.1, 1.0), ("g_Na", 0.1, 1.0), ("E_Na", 0.1, 1.0), ("g_K", 0.1, 1.0), ("E_K", 0.1, 1.0),
    ("g_L", 0.1, 1.0), ("E_L", 0.1, 1.0), ("m_inf", 0.1, 1.0), ("tau_m", 0.5, 5.0), ("h_inf", 0.1, 1.0),
    ("tau_h", 1.5, 15.0), ("n_inf", 0.1, 1.0), ("tau_n", 1.0, 10.0), ("g_C", 1e-3, 1e-2), ("T", 0.5, 2.0))


def neuron(n_unit=1, n_batch=3, n_time=2000, t_max=10.0):
    """The coupled-neuron timing case: each per-neuron parameter is
    linspace(lo, hi, n_unit) over the neurons (NEURON_TABLE), the current
    amplitude I_a = linspace(0.1, 1, n_batch) (one value per series), t in
    [0, t_max] in n_time equal steps, zero initial state.  Parameter vector per
    series: the 15 per-neuron values of neuron 1, ..., of neuron n_unit, then I_a."""
    per = np.stack([np.linspace(lo, hi, n_unit) for _, lo, hi in NEURON_TABLE], axis=1)  # [n_unit][15]
    params = np.array([np.concatenate([per.reshape(-1), [ia]]) for ia in np.linspace(0.1, 1.0, n_batch)])
    n = 4 * n_unit
    return dict(kind="neuron", n=n, y0=np.zeros((n_batch, n)), times=np.linspace(0.0, t_max, n_time + 1),
                params=params, offsets=None)


def mds(n_unit=1, n_batch=3, n_time=2000, t_max=1.0):
    """The mass-damper-spring timing case: K_i = linspace(1e-2, 1, n_unit),
    C_i = linspace(1e-6, 1e-4, n_unit), M_i = linspace(1e-7, 1e-5, n_unit),
    f_a = 1, T = linspace(1e-2, 1, n_batch) (one value per series), t in
    [0, t_max] in n_time equal steps, zero initial state.  State (d_1, v_1, ...,
    d_nu, v_nu); parameter vector per series (K_1..K_nu, C_1..C_nu, M_1..M_nu,
    f_a, T)."""
    nu = n_unit
    base = np.concatenate([np.linspace(1e-2, 1.0, nu), np.linspace(1e-6, 1e-4, nu), np.linspace(1e-7, 1e-5, nu)])
    params = np.array([np.concatenate([base, [1.0, T]]) for T in np.linspace(1e-2, 1.0, n_batch)])
    n = 2 * nu
    return dict(kind="mds", n=n, y0=np.zeros((n_batch, n)), times=np.linspace(0.0, t_max, n_time + 1),
                params=params, offsets=None)


def fnode_weights(n_unit, seed=140):
    """The forced neural ODE's layers: W1, b1 (n+1 -> n+1), W2, b2 (n+1 -> n+1),
    W3, b3 (n+1 -> n), every entry U(-sqrt(1/(n+1)), sqrt(1/(n+1))), drawn once
    in that order."""
    rng = np.random.default_rng(seed)
    m = n_unit + 1
    a = np.sqrt(1.0 / m)
    shapes = ((m, m), (m,), (m, m), (m,), (n_unit, m), (n_unit,))
    return np.concatenate([rng.uniform(-a, a, size=sh).reshape(-1) for sh in shapes])


def fnode(n_unit=1, n_batch=3, n_time=2000, t_max=1.0, seed=140):
    """The neural-ODE timing case: dy/dt = tanh(L3(tanh(L2(tanh(L1(y, f(t))))))),
    the layers from fnode_weights (fixed for every series), f(t) = f_a sin(2 pi t / T)
    with f_a = 1 and T = linspace(1e-2, 1, n_batch) (one value per series), t in
    [0, t_max] in n_time equal steps, zero initial state.  Parameter vector per
    series (W1, b1, W2, b2, W3, b3, f_a, T)."""
    w = fnode_weights(n_unit, seed)
    params = np.array([np.concatenate([w, [1.0, T]]) for T in np.linspace(1e-2, 1.0, n_batch)])
    return dict(kind="fnode", n=n_unit, y0=np.zeros((n_batch, n_unit)),
                times=np.linspace(0.0, t_max, n_time + 1), params=params, offsets=None)
