"""The block solver (state sizes up to 40: the paper's mass-damper-spring
chain, coupled neurons beyond two units and forced neural ODE) against the CPU
oracle, through the C ABI.

Every tiling is checked: T = chunk (Thomas's algorithm), T = 1 (pure PCR, up to
ten reduction levels at chunk 1000) and the hybrids in between, at the parity
tolerance where both sides iterate Newton to rounding level (gate 1e-10
relative, per series), on uniform and ragged grids with empty and one-step
series.  Adjoints are checked on the GPU's own trajectory (the kernel) and end
to end against the oracle's forward + adjoint (the pipeline)."""
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


def d(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _workload(kind, nu, B, N, t_max=None):
    kw = {} if t_max is None else {"t_max": t_max}
    w = getattr(W, kind)(nu, B, n_time=N, **kw)
    if kind == "fnode":
        w["y0"] = 0.2 * np.random.default_rng(nu).standard_normal(w["y0"].shape)
    if kind == "neuron":
        w["y0"] = np.random.default_rng(nu).uniform(0.05, 0.6, w["y0"].shape)
    return w


MODELS = [("mds", 1), ("mds", 3), ("mds", 10), ("mds", 20), ("neuron", 3), ("neuron", 10), ("fnode", 1),
          ("fnode", 5), ("fnode", 25)]


@pytest.mark.parametrize("kind,nu", MODELS, ids=lambda v: str(v))
def test_block_model_rate_and_jacobian_match_oracle(tvi, kind, nu):
    w = _workload(kind, nu, 3, 10)
    n = w["n"]
    rng = np.random.default_rng(7)
    M = 37  # several workgroups of 8 states and a ragged tail
    scale = 1e-4 if kind == "mds" else 0.5
    y = scale * rng.standard_normal((M, n))
    if kind == "neuron":
        y = rng.uniform(0.05, 1.0, (M, n))
    t = rng.uniform(0.0, 1.0, M)
    p = w["params"][rng.integers(0, 3, M)]
    f, J = tvi.model_eval(kind, d(y), d(p), times=d(t))
    f, J = host(f), host(J)
    for q in range(M):
        fo, Jo = oracle.rhs(kind, y[q], t[q], p[q])
        np.testing.assert_allclose(f[q], fo, rtol=1e-13, atol=1e-13 * np.abs(fo).max())
        np.testing.assert_allclose(J[q], Jo, rtol=1e-13, atol=1e-13 * np.abs(Jo).max())


def _tilings(C):
    out = {(C, C), (C, 1)}           # Thomas, PCR
    for T in (2, 8, 64):
        if T < C:
            out.add((C, T))          # hybrids
    return sorted(out)


CASES = []
for kind, nu, N in [("mds", 1, 300), ("mds", 10, 300), ("mds", 20, 200), ("neuron", 3, 300), ("neuron", 10, 200),
                    ("fnode", 1, 300), ("fnode", 5, 300), ("fnode", 25, 200)]:
    for C in (1, 7, 64, N):
        for C_, T in _tilings(C):
            CASES.append((kind, nu, N, C_, T))


@pytest.mark.parametrize("kind,nu,N,C,T", CASES, ids=lambda v: str(v))
def test_block_forward_matches_oracle(tvi, kind, nu, N, C, T):
    w = _workload(kind, nu, 3, N, t_max=3.0 if kind == "neuron" else None)
    yo, so, _ = oracle.forward(kind, w["y0"], w["times"], w["params"], tol=PARITY_TOL)
    assert (so == 0).all()
    print("block forward %s nu=%d N=%d chunk=%d T=%d" % (kind, nu, N, C, T), flush=True)
    y, st, it, _ = tvi.solve_forward(kind, d(w["y0"]), d(w["times"]), d(w["params"]), chunk=C, steps_per_lane=T,
                                     tol=PARITY_TOL)
    assert (host(st) == 0).all(), host(st)
    err = series_rel_err(host(y), yo)
    assert err.max() <= 1e-10, err


def test_block_chunk_1000_every_solver(tvi):
    """The study's largest chunk: 2000 steps in two chunks of 1000 (ten PCR levels
    for T = 1), n = 20."""
    w = _workload("mds", 10, 2, 2000)
    yo, so, _ = oracle.forward("mds", w["y0"], w["times"], w["params"], tol=PARITY_TOL)
    assert (so == 0).all()
    for T in (1000, 1, 8, 100):
        print("block chunk 1000 T=%d" % T, flush=True)
        y, st, _, _ = tvi.solve_forward("mds", d(w["y0"]), d(w["times"]), d(w["params"]), chunk=1000,
                                        steps_per_lane=T, tol=PARITY_TOL)
        assert (host(st) == 0).all()
        assert series_rel_err(host(y), yo).max() <= 1e-10, T


def _ragged(kind, nu, lens, seed=0):
    base = _workload(kind, nu, len(lens), 4)
    rng = np.random.default_rng(seed)
    times, offs = [], [0]
    for L in lens:
        times.append(np.sort(rng.uniform(0.0, 0.2, L + 1)))
        offs.append(offs[-1] + L + 1)
    return base["y0"], np.concatenate(times), base["params"], np.array(offs, dtype=np.int64)


@pytest.mark.parametrize("kind,nu", [("mds", 5), ("neuron", 4), ("fnode", 9)])
@pytest.mark.parametrize("C,T", [(64, 64), (64, 1), (64, 8), (16, 4)])
def test_block_ragged_with_empty_and_one_step_series(tvi, kind, nu, C, T):
    y0, times, p, offs = _ragged(kind, nu, [0, 1, 5, 130, 64, 2, 200, 0, 77])
    yo, so, _ = oracle.forward(kind, y0, times, p, offsets=offs, tol=PARITY_TOL)
    assert (so == 0).all()
    y, st, _, _ = tvi.solve_forward(kind, d(y0), d(times), d(p), offsets=torch.as_tensor(offs, device="cuda"),
                                    chunk=C, steps_per_lane=T, tol=PARITY_TOL)
    assert (host(st) == 0).all()
    err = series_rel_err(host(y), yo, offsets=offs)
    assert err.max() <= 1e-10, err


ADJ_CASES = [("mds", 3, 300, 64, 64), ("mds", 20, 200, 50, 1), ("mds", 10, 300, 100, 8), ("neuron", 3, 300, 64, 1),
             ("neuron", 10, 200, 40, 40), ("fnode", 5, 300, 64, 8), ("fnode", 25, 200, 30, 30), ("fnode", 1, 300, 7, 1)]


@pytest.mark.parametrize("kind,nu,N,C,T", ADJ_CASES, ids=lambda v: str(v))
def test_block_adjoint_matches_oracle(tvi, kind, nu, N, C, T):
    w = _workload(kind, nu, 3, N, t_max=3.0 if kind == "neuron" else None)
    print("block adjoint %s nu=%d chunk=%d T=%d" % (kind, nu, C, T), flush=True)
    y, st, _, _ = tvi.solve_forward(kind, d(w["y0"]), d(w["times"]), d(w["params"]), chunk=C, steps_per_lane=T,
                                    tol=PARITY_TOL)
    assert (host(st) == 0).all()
    yh = host(y)
    g = yh / np.sqrt(np.sum(yh ** 2))
    dp, dy0, sa = tvi.solve_adjoint(kind, d(w["times"]), d(w["params"]), d(g), y=y, chunk=C, steps_per_lane=T,
                                    tol=PARITY_TOL)
    assert (host(sa) == 0).all()
    # the kernel: the oracle's adjoint on the GPU's own trajectory
    op, oy0, so = oracle.adjoint(kind, yh, w["times"], w["params"], g)
    assert (so == 0).all()
    for b in range(3):
        assert np.abs(host(dp)[b] - op[b]).max() <= 1e-10 * np.abs(op[b]).max(), b
        assert np.abs(host(dy0)[b] - oy0[b]).max() <= 1e-10 * max(np.abs(oy0[b]).max(), 1e-300), b
    # the pipeline: the oracle's forward and adjoint on its own trajectory
    yo, _, _ = oracle.forward(kind, w["y0"], w["times"], w["params"], tol=PARITY_TOL)
    go = yo / np.sqrt(np.sum(yo ** 2))
    op2, oy02, _ = oracle.adjoint(kind, yo, w["times"], w["params"], go)
    for b in range(3):
        assert np.abs(host(dp)[b] - op2[b]).max() <= 1e-10 * np.abs(op2[b]).max(), b


def test_block_adjoint_ragged(tvi):
    y0, times, p, offs = _ragged("mds", 6, [3, 0, 90, 1, 140, 33])
    o = torch.as_tensor(offs, device="cuda")
    y, st, _, _ = tvi.solve_forward("mds", d(y0), d(times), d(p), offsets=o, chunk=32, steps_per_lane=4,
                                    tol=PARITY_TOL)
    yh = host(y)
    g = yh / np.sqrt(np.sum(yh ** 2))
    dp, dy0, sa = tvi.solve_adjoint("mds", d(times), d(p), d(g), y=y, offsets=o, chunk=32, steps_per_lane=4,
                                    tol=PARITY_TOL)
    assert (host(sa) == 0).all()
    op, oy0, _ = oracle.adjoint("mds", yh, times, p, g, offsets=offs)
    for b in range(len(offs) - 1):
        if offs[b + 1] - offs[b] > 1:
            assert np.abs(host(dp)[b] - op[b]).max() <= 1e-10 * np.abs(op[b]).max(), b
        np.testing.assert_allclose(host(dy0)[b], oy0[b], rtol=1e-10, atol=1e-14 * np.abs(oy0).max())


def test_block_timing_tolerance_and_extrapolated_start(tvi):
    """The paper's tolerances with both starts: every step satisfies the
    backward-Euler equation to the stopping test's bound, and the trajectory is
    within that bound of the oracle's."""
    w = _workload("neuron", 5, 3, 2000, t_max=10.0)
    yo, so, _ = oracle.forward("neuron", w["y0"], w["times"], w["params"], tol=(1e-8, 1e-6))
    for init in ("zero", "extrap"):
        y, st, it, _ = tvi.solve_forward("neuron", d(w["y0"]), d(w["times"]), d(w["params"]), chunk=100,
                                         steps_per_lane=100, tol=(1e-8, 1e-6), init=init)
        assert (host(st) == 0).all()
        yh = host(y)
        h = np.diff(w["times"])
        for b in range(3):
            f = np.array([oracle.rhs("neuron", yh[b, k], w["times"][k], w["params"][b])[0]
                          for k in range(1, yh.shape[1])])
            r = yh[b, 1:] - yh[b, :-1] - h[:, None] * f
            assert np.linalg.norm(r, axis=1).max() <= 1e-7, (init, b)
        assert series_rel_err(yh, yo).max() <= 1e-5
