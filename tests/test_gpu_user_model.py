"""Right-hand sides written as user models (include/tvi_user_model.hpp): only
the rate is written, the state Jacobian of the Newton blocks and the
parameter products of the adjoint come from forward-mode automatic
differentiation on the device.  The Van der Pol and Robertson rates of the
test workloads are written that way, compiled the way a user would
(tests/user_model/user_models.hip), and checked against the CPU oracle's
hand-written models: trajectories at the parity tolerance within 1e-10, and
adjoint gradients (stored and recomputed states) within 1e-10 of the oracle's
adjoint on the same trajectory, over several lane tilings."""
import os

import numpy as np
import pytest

import oracle
from paper_2310_08649_amd import workloads as W
from tests.helpers import PARITY_TOL, series_rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "user_model", "libtvi_user_models.so")


@pytest.fixture(scope="module")
def models():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_08649_amd import tvi
    return {"vanderpol": tvi.UserModel(LIB, "user_vanderpol", 2, 1),
            "robertson": tvi.UserModel(LIB, "user_robertson", 3, 3)}


def d(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


TILINGS = [(64, 64, 1), (64, 16, 4), (32, 4, 8), (1, 1, 1)]


@pytest.mark.parametrize("C,S,T", TILINGS)
def test_user_vanderpol_forward_and_adjoint_match_oracle(models, C, S, T):
    um = models["vanderpol"]
    w = W.vanderpol(B=32, N=1000, mu_range=(1.0, 20.0))
    print("user vanderpol chunk=%d S=%d T=%d" % (C, S, T), flush=True)
    y, st, _, ck = um.solve_forward(d(w["y0"]), d(w["times"]), d(w["params"]), chunk=C, lanes=S, steps_per_lane=T,
                                    tol=PARITY_TOL, checkpoints=True)
    yo, so, _ = oracle.forward("vanderpol", w["y0"], w["times"], w["params"], tol=PARITY_TOL)
    assert (so == 0).all() and (host(st) == 0).all()
    assert series_rel_err(host(y), yo).max() <= 1e-10
    yh = host(y)
    g = yh / np.sqrt(np.sum(yh ** 2))
    op, oy0, _ = oracle.adjoint("vanderpol", yh, w["times"], w["params"], g)
    for src in ("stored", "recompute"):
        kw = dict(y=y) if src == "stored" else dict(ckpt=ck)
        dp, dy0, sa = um.solve_adjoint(d(w["times"]), d(w["params"]), d(g), chunk=C, lanes=S, steps_per_lane=T,
                                       tol=PARITY_TOL, **kw)
        assert (host(sa) == 0).all()
        assert np.abs(host(dp) - op).max() <= 1e-10 * np.abs(op).max(), src
        assert np.abs(host(dy0) - oy0).max() <= 1e-10 * np.abs(oy0).max(), src


@pytest.mark.parametrize("C,S,T", TILINGS[:3])
def test_user_robertson_ragged_matches_oracle(models, C, S, T):
    um = models["robertson"]
    w = W.robertson(B=40, seed=17, n_range=(50, 2000))
    off = torch.as_tensor(w["offsets"], device="cuda")
    print("user robertson chunk=%d S=%d T=%d" % (C, S, T), flush=True)
    y, st, _, _ = um.solve_forward(d(w["y0"]), d(w["times"]), d(w["params"]), offsets=off, chunk=C, lanes=S,
                                   steps_per_lane=T, tol=PARITY_TOL)
    yo, so, _ = oracle.forward("robertson", w["y0"], w["times"], w["params"], offsets=w["offsets"], tol=PARITY_TOL)
    assert (so == 0).all() and (host(st) == 0).all()
    assert series_rel_err(host(y), yo, offsets=w["offsets"]).max() <= 1e-10
    yh = host(y)
    g = yh / np.sqrt(np.sum(yh ** 2))
    dp, dy0, sa = um.solve_adjoint(d(w["times"]), d(w["params"]), d(g), y=y, offsets=off, chunk=C, lanes=S,
                                   steps_per_lane=T, tol=PARITY_TOL)
    op, oy0, _ = oracle.adjoint("robertson", yh, w["times"], w["params"], g, offsets=w["offsets"])
    assert (host(sa) == 0).all()
    for b in range(w["y0"].shape[0]):
        assert np.abs(host(dp)[b] - op[b]).max() <= 1e-10 * np.abs(op[b]).max(), b
    assert np.abs(host(dy0) - oy0).max() <= 1e-10 * np.abs(oy0).max()


def test_user_model_refuses_options_it_does_not_take(models):
    from paper_2310_08649_amd import tvi
    um = models["vanderpol"]
    w = W.vanderpol(B=4, N=50)
    with pytest.raises(tvi.TviError):
        um.solve_forward(d(w["y0"]), d(w["times"]), d(w["params"]), chunk=16, init=7)
    with pytest.raises(tvi.TviError):
        um.solve_forward(d(w["y0"]), d(w["times"]), d(w["params"]), chunk=16, lanes=3, steps_per_lane=8)
