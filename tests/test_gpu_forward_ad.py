"""State Jacobians by forward-mode automatic differentiation (the forward AD
option of Section 2.2) in the chunked solver: trajectories and adjoint
gradients against the oracle (analytic Jacobians, sequential Newton) at the
FP64 parity gate, for every analytic model, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2310_08649_amd import workloads as W
from tests.helpers import PARITY_TOL, series_rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def _cases():
    rng = np.random.default_rng(71)
    out = []
    for n in (2, 3, 4):
        B, N = 12, 120
        A = -2.0 * np.eye(n)[None] + rng.standard_normal((B, n, n))
        out.append(("linear", rng.standard_normal((B, n)), np.linspace(0, 1, N + 1), A.reshape(B, -1), None))
    w = W.vanderpol(B=48, N=1000, mu_range=(1.0, 30.0))
    out.append(("vanderpol", w["y0"], w["times"], w["params"], None))
    w = W.robertson(B=24, n_range=(100, 1500))
    out.append(("robertson", w["y0"], w["times"], w["params"], w["offsets"]))
    for nu in (1, 2):
        w = W.chaboche(nu, 10)
        out.append(("chaboche", w["y0"], w["times"], w["params"], None))
    w = W.neuron(1, 10)
    out.append(("neuron", w["y0"], w["times"], w["params"], None))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: "%s-n%d" % (c[0], c[1].shape[1]))
def test_forward_ad_jacobian_parity(tvi, case):
    kind, y0, times, params, offsets = case
    yo, so, _ = oracle.forward(kind, y0, times, params, offsets=offsets, tol=PARITY_TOL)
    assert (so == 0).all()
    g = yo / np.sqrt(np.sum(yo ** 2))
    off = None if offsets is None else dev(offsets, torch.int64)
    for C, S, T in ((64, 64, 1), (32, 8, 4), (1, 1, 1)):
        kw = dict(offsets=off, chunk=C, lanes=S, steps_per_lane=T, tol=PARITY_TOL, jacobian="forward_ad")
        y, st, _, ck = tvi.solve_forward(kind, dev(y0), dev(times), dev(params), checkpoints=True, **kw)
        assert (host(st) == 0).all(), (C, S, T)
        assert series_rel_err(host(y), yo, offsets).max() <= 1e-10, (C, S, T)
        a1 = tvi.solve_adjoint(kind, dev(times), dev(params), dev(g), y=y, **kw)
        a2 = tvi.solve_adjoint(kind, dev(times), dev(params), dev(g), ckpt=ck, **kw)
        assert torch.equal(a1[0], a2[0]) and torch.equal(a1[1], a2[1]), (C, S, T)
        # the oracle's adjoint at the states this solve converged to: the stiff Van der Pol
        # series amplify the within-tolerance difference of the two stopping points
        op, oy0, _ = oracle.adjoint(kind, host(y), times, params, g, offsets=offsets)
        assert grad_err(host(a1[0]), op) <= 1e-10, (C, S, T, grad_err(host(a1[0]), op))
        assert np.abs(host(a1[1]) - oy0).max() <= 1e-10 * np.abs(oy0).max(), (C, S, T)
