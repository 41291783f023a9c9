"""The autotuner: every candidate it times is a valid tiling of its chunk, the
choice ranks failed series before time, the cache returns the same choice, and
the tuned solve is the oracle's trajectory."""
import json

import numpy as np
import pytest

import oracle
from paper_2310_08649_amd import workloads as W
from tests.helpers import PARITY_TOL, series_rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_08649_amd import autotune, tvi
    tvi.load()
    return autotune, tvi


def test_tune_forward_choice_cache_and_parity(mods, tmp_path, monkeypatch):
    autotune, tvi = mods
    monkeypatch.setattr(autotune, "_CACHE_PATH", str(tmp_path / "tune.json"))
    w = W.robertson(B=64, n_range=(100, 3000))
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    off = torch.as_tensor(w["offsets"], device="cuda")
    args = (d(w["y0"]), d(w["times"]), d(w["params"]))
    chunks = (8, 32, 100)
    res = autotune.tune_forward("robertson", *args, offsets=off, tol=PARITY_TOL, chunks=chunks,
                                inits=("zero",), reps=2)
    table, best = res["table"], res["best"]
    assert {(r["chunk"], r["lanes"], r["steps_per_lane"]) for r in table} == \
        {(C, S, T) for C in chunks for S, T in autotune.tilings(C)}
    for r in table:
        assert r["lanes"] * r["steps_per_lane"] >= r["chunk"] and r["ms"] > 0
    assert best == min(table, key=lambda r: (r["failed"], r["ms"]))
    # the cache answers the same question with the same choice, without timing
    again = autotune.tune_forward("robertson", *args, offsets=off, tol=PARITY_TOL, chunks=chunks,
                                  inits=("zero",), reps=2)
    assert again["best"] == json.loads(json.dumps(best))
    y, st, _, _ = tvi.solve_forward("robertson", *args, offsets=off, chunk=best["chunk"], lanes=best["lanes"],
                                    steps_per_lane=best["steps_per_lane"], init=best["init"], tol=PARITY_TOL)
    yo, so, _ = oracle.forward("robertson", w["y0"], w["times"], w["params"], offsets=w["offsets"], tol=PARITY_TOL)
    assert (st.cpu().numpy() == 0).all()
    assert series_rel_err(y.cpu().numpy(), yo, w["offsets"]).max() <= 1e-10


def test_tune_forward_over_iteration_limits(mods, tmp_path, monkeypatch):
    """The single-step iteration limit as a tuned dimension (Van der Pol with
    stiff members): every limit appears in the table with every tiling, the
    choice ranks failed series first, and with multi-step attempts capped
    below both limits a higher limit never gives up on more series (a series
    whose single steps all converged within the lower limit takes the same
    path under the higher one)."""
    autotune, tvi = mods
    monkeypatch.setattr(autotune, "_CACHE_PATH", str(tmp_path / "tune.json"))
    w = W.vanderpol(B=64, N=2000, mu_range=(1.0, 1000.0), t_end=20.0)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    args = (d(w["y0"]), d(w["times"]), d(w["params"]))
    res = autotune.tune_forward("vanderpol", *args, tol=(1e-8, 1e-6), chunks=(16, 50), inits=("zero",),
                                caps=(0, 5), limits=(10, 50), reps=2, use_cache=False)
    table, best = res["table"], res["best"]
    keys = {(r["chunk"], r["lanes"], r["steps_per_lane"], r["max_newton_chunk"], r["max_newton"]) for r in table}
    assert keys == {(C, S, T, c, l) for C in (16, 50) for S, T in autotune.tilings(C) for c in (0, 5)
                    for l in (10, 50)}
    assert best == min(table, key=lambda r: (r["failed"], r["ms"]))
    fails = {(r["chunk"], r["lanes"], r["steps_per_lane"], r["max_newton_chunk"], r["max_newton"]): r["failed"]
             for r in table}
    for (C, S, T, c, l), f in fails.items():
        if l == 10 and c == 5:
            assert fails[(C, S, T, c, 50)] <= f
