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
