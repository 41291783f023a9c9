"""Host-side logic on the CPU: the seeded input generators, the tiling
candidates of the autotuner and the option marshalling of the binding."""
import numpy as np
import pytest

import oracle
from paper_2310_08649_amd import workloads as W


def test_generators_are_seeded_and_shaped():
    for gen, kw in ((W.linear, {}), (W.vanderpol, dict(B=16, N=100)), (W.mlp, dict(B=4, N=50)),
                    (W.robertson, dict(B=30, n_range=(100, 500)))):
        a, b = gen(**kw), gen(**kw)
        for k in ("y0", "times", "params"):
            assert np.array_equal(a[k], b[k]), (gen.__name__, k)
        B, n = a["y0"].shape
        if a["offsets"] is None:
            assert a["times"].ndim == 1 and np.all(np.diff(a["times"]) > 0)
        else:
            off = a["offsets"]
            assert off.shape == (B + 1,) and off[0] == 0 and off[-1] == a["times"].shape[0]
            lens = np.diff(off) - 1
            assert np.array_equal(lens, a["steps"]) and lens.min() >= 1
            for i in range(B):  # each series' grid increases
                assert np.all(np.diff(a["times"][off[i]:off[i + 1]]) > 0)
        P = oracle.param_count(a["kind"], n, a.get("hidden", 64))
        assert a["params"].shape[-1] == P


def test_robertson_lengths_follow_the_recipe():
    w = W.robertson()
    assert w["steps"].min() >= 100 and w["steps"].max() <= 20000
    assert 6.5e6 < w["steps"].sum() < 8.5e6  # log-uniform lengths in [100, 2e4] over 2000 series
    t0 = w["times"][w["offsets"][:-1]]
    t1 = w["times"][w["offsets"][1:] - 1]
    np.testing.assert_allclose(t0, 1e-5, rtol=1e-12)
    np.testing.assert_allclose(t1, 1e4, rtol=1e-12)


@pytest.mark.parametrize("nu", [1, 2, 5])
def test_paper_problem_tables(nu):
    c = W.chaboche(nu, 7)
    assert c["params"].shape == (7, oracle.param_count("chaboche", 2 + nu))
    np.testing.assert_allclose(c["params"][:, -2], np.linspace(0.1, 1.0, 7))  # edot_a per series
    assert (c["params"][:, :6] == [10.0, 5.0, 2.0, 1.0, 10.0, 1.0]).all()
    nr = W.neuron(min(nu, 2), 5)
    assert nr["params"].shape == (5, oracle.param_count("neuron", 4 * min(nu, 2)))
    np.testing.assert_allclose(nr["params"][:, -1], np.linspace(0.1, 1.0, 5))  # I_a per series
    assert (c["y0"] == 0).all() and (nr["y0"] == 0).all()


def test_tiling_candidates():
    from paper_2310_08649_amd import autotune
    for C in range(1, 513):
        t = autotune.tilings(C)
        assert t, C
        for S, T in t:
            assert S in (1, 4, 8, 16, 32, 64) and T in (1, 2, 4, 8)
            assert S * T >= C, (C, S, T)
            if C > 1:
                assert S * T < 2 * max(C, 4) or (S, T) == (64, 8), (C, S, T)


def test_option_marshalling():
    pytest.importorskip("torch")
    from paper_2310_08649_amd import tvi
    import os
    if not os.path.exists(tvi.LIB_PATH):
        pytest.skip("libtvi.so not built")
    o = tvi.make_options(chunk=37, tol=(1e-9, 1e-7), max_newton=12, lanes=16, steps_per_lane=4, init="extrap",
                         halving=False, scheme="forward_euler", jacobian="forward_ad",
                         reference="zero")
    assert (o.chunk, o.max_newton, o.lanes, o.steps_per_lane, o.init, o.halving) == (37, 12, 16, 4, 1, 0)
    assert (o.tol_a, o.tol_r) == (1e-9, 1e-7)
    assert (o.scheme, o.jacobian, o.reference_residual) == (1, 1, 1)
    assert tvi.make_options(init="predictor").init == 2 and tvi.make_options(init="zero").init == 0
    assert tvi.make_options().max_newton_chunk == 0 and tvi.make_options(max_newton_chunk=9).max_newton_chunk == 9


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


@pytest.mark.parametrize("nu,nb", [(1, 3), (3, 10), (5, 50)])
def test_chaboche_workload_is_the_paper_table(nu, nb):
    g = _golden("chaboche_parameters.json")
    p = W.chaboche(nu, nb, n_time=_golden("chunk_study.json")["n_time"])
    assert p["times"][-1] == g["t_max"] and p["times"].shape[0] == 2001
    for b in range(nb):
        row = p["params"][b]
        assert list(row[:6]) == [g["E"], g["n"], g["eta"], g["sigma0"], g["K_inf"], g["tau"]]
        np.testing.assert_array_equal(row[6:6 + nu], np.linspace(*g["C"]["linspace"], nu))
        np.testing.assert_array_equal(row[6 + nu:6 + 2 * nu], np.linspace(*g["gamma"]["linspace"], nu))
        assert row[6 + 2 * nu] == np.linspace(*g["edot_a"]["linspace"], nb)[b] and row[7 + 2 * nu] == g["T"]


@pytest.mark.parametrize("nu,nb", [(1, 3), (2, 30)])
def test_neuron_workload_is_the_paper_table(nu, nb):
    g = _golden("neuron_parameters.json")
    p = W.neuron(nu, nb)
    assert p["times"][-1] == g["t_max"]
    names = list(g["per_neuron_linspace_over_n_unit"])
    for b in range(nb):
        row = p["params"][b]
        for i in range(nu):
            for k, name in enumerate(names):
                lo, hi = g["per_neuron_linspace_over_n_unit"][name]
                assert row[15 * i + k] == np.linspace(lo, hi, nu)[i], (name, i)
        assert row[15 * nu] == np.linspace(*g["I_a"]["linspace"], nb)[b]


# --------------------------------------------------------------------------
# Benchmark host logic (no GPU): the one-GPU contract, the algorithmic flop
# count, and the staleness gate on profiler traffic
# --------------------------------------------------------------------------
def _bench():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py")
    spec = importlib.util.spec_from_file_location("bench_under_test", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod, path


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    _, path = _bench()
    r = subprocess.run([sys.executable, path, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_reduction_levels_and_flop_count():
    import math
    b, _ = _bench()
    for c in range(1, 600):
        assert b.levels(c) == math.ceil(math.log2(c))
    # residual, Jacobian, inverse and update, plus one 2x2 affine composition per level
    assert b.vdp_flops_per_step_iter(50) == 44 + 24 * 6
    assert b.vdp_flops_per_step_iter(1) == 44


def test_bench_robertson_flop_counts():
    b, _ = _bench()
    # pure PCR over 64 lanes: six reduction levels per step
    assert b.rob_forward_flops_per_step(64, 1) == 26 + 24 + 72 + 6 * 72
    # hybrid: three serial compositions and six levels shared by four steps, plus the replay
    assert b.rob_forward_flops_per_step(64, 4) == 26 + 24 + 72 + 72 * (3 + 6) / 4 + 24
    # one lane per series (chunk 1): no composition at all
    assert b.rob_forward_flops_per_step(1, 1) == 26 + 24 + 72
    assert b.rob_adjoint_flops_per_step(1, 1) == 24 + 72 + 24 + 12
    # over 4 waves (256 lanes): six levels inside each wave, then the value entering the wave
    # applied to each lane's composed map (24 flops), no seventh composition
    assert b.rob_forward_flops_per_step(256, 4) == 26 + 24 + 72 + (72 * (3 + 6) + 24) / 4 + 24
    fwd, adj = b.kernel_names(256, 4, "zero", False)
    assert fwd == "tvi::wide::forward_kernel<tvi::Robertson, double, 4, 4>(tvi::SolveArgs<double>, double*)"
    assert adj == "tvi::wide::adjoint_kernel<tvi::Robertson, double, 4, 4>(tvi::SolveArgs<double>, double const*)"


def test_bench_traffic_is_reported_only_for_matching_kernel_code(monkeypatch, tmp_path):
    import json
    import os
    import shutil
    b, _ = _bench()
    srcs = ["solver.hpp", "device.hpp"]
    kernel = "tvi::forward_kernel<tvi::Robertson, double, 64, 4, false, false, false>(tvi::SolveArgs<double>)"
    table = {kernel: {"bytes_per_dispatch": 1.5e8, "sources": srcs, "source_hash": b.csrc_hash(srcs)}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(table))
    csrc = tmp_path / "paper_2310_08649_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in srcs:
        shutil.copy(os.path.join(b.ROOT, "paper_2310_08649_amd", "csrc", name), csrc / name)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic(kernel) == 1.5e8
    assert b.measured_traffic("no such kernel") is None
    # a change to a file the kernel is not built from leaves the counters valid
    (csrc / "unrelated.hip").write_text("int x;")
    assert b.measured_traffic(kernel) == 1.5e8
    # a change to one it is built from makes them stale
    (csrc / "device.hpp").write_text((csrc / "device.hpp").read_text() + "\nint changed;\n")
    assert b.measured_traffic(kernel) is None


def test_bench_line_is_compact_json():
    import argparse
    import json
    b, _ = _bench()
    args = argparse.Namespace(steps=20, warmup=5)
    cfg = {"workload": "x" * 300, "chunk": 256, "lanes": 64, "steps_per_lane": 4, "init": "zero",
           "adjoint_states": "stored", "series": 2000, "series_steps": 7710000, "series_failed": 0,
           "series_steps_counted": 7710000, "newton_corrections": 86000}
    roof = {"bound": "alu", "achieved": 11.2, "peak": 78.6, "unit": "TFLOP/s", "frac": 0.142, "traffic": 2.5e8,
            "kernel": "k" * 120, "avg_launch_ms": 0.63, "algorithmic_flops": 7.1e9, "algorithmic_bytes": 2.4e8,
            "hbm_gbs": 390.0, "hbm_frac": 0.05, "other_kernel": {"kernel": "k" * 120, "avg_launch_ms": 0.5,
                                                                   "tflops": 5.0, "hbm_gbs": 800.0},
            "loss_ms": 0.05, "loss_hbm_gbs": 3000.0}
    head = {"value": 6.4e9, "ms_per_step": 1.2, "replay": {"mean_ms": 1.2, "median_ms": 1.2, "min_ms": 1.19},
            "config": cfg, "roofline": roof, "peak_device_memory_bytes": 10 ** 9,
            "chunk1": {"value": 1e8, "ms_per_step": 80.0, "series_failed": 0, "speedup_of_chunked": 66.0},
            "other_adjoint_states": {"adjoint_states": "recompute", "value": 4e9, "ms_per_step": 1.8},
            "autotune_best": {"chunk": 256}, "autotune_candidates": 40}
    out = b.compose_line(args, head)
    out["cpu_baseline"] = {"value": 1e8, "unit": "series*steps/s", "cores": 16, "kind": "oracle",
                           "sample": "s" * 200, "one_core_value": 1e7, "one_core_sample": "s" * 60,
                           "cpu_model": "c" * 40, "nproc": 16}
    line = json.dumps(out, separators=(",", ":"))
    assert len(line) < 4096
    back = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in back
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in back["roofline"]
    assert "workload" in back["config"]


def test_bench_code_hash_ignores_comments_only(tmp_path, monkeypatch):
    import os
    import shutil
    b, _ = _bench()
    src = os.path.join(b.ROOT, "paper_2310_08649_amd", "csrc")
    dst = tmp_path / "paper_2310_08649_amd" / "csrc"
    shutil.copytree(src, dst)
    h0 = b.csrc_hash()
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.csrc_hash() == h0
    f = dst / "pcr.hip"
    text = f.read_text()
    f.write_text("// a new comment\n/* and a block\n   comment */\n\n" + text + "\n\n")
    assert b.csrc_hash() == h0
    f.write_text(text.replace("kWave", "kWave + 0", 1))
    assert b.csrc_hash() != h0


def test_bench_records_traffic_from_counter_csvs(monkeypatch, tmp_path):
    """The traffic record: per-kernel FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    scaled by what each counter reads for the plain copy of known size."""
    import json
    import os
    import shutil
    b, _ = _bench()
    kern = "tvi::forward_kernel<tvi::Robertson, double, 64, 8, false, false, false>(tvi::SolveArgs<double>)"
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"

    def csv(path, counter, copy_kib, k1, k2):
        path.mkdir()
        (path / "run_counter_collection.csv").write_text(
            hdr + '1,"__amd_rocclr_copyBuffer",%s,%r\n' % (counter, copy_kib)
            + '2,"void %s",%s,%r\n' % (kern, counter, k1) + '3,"void %s",%s,%r\n' % (kern, counter, k2))

    csv(tmp_path / "f", "FETCH_SIZE", 131072.0, 100.0, 300.0)   # fetch reads half the copy's bytes
    csv(tmp_path / "w", "WRITE_SIZE", 262144.0, 1000.0, 1000.0)
    (tmp_path / "profiles").mkdir()
    csrc = tmp_path / "paper_2310_08649_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in b.KERNEL_SOURCES["Robertson"]:
        shutil.copy(os.path.join(b.ROOT, "paper_2310_08649_amd", "csrc", name), csrc / name)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    table = b.record_traffic(str(tmp_path / "f"), str(tmp_path / "w"), 1 << 28)
    rec = table[kern]
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert rec["bytes_per_dispatch"] == (200.0 * 2.0 + 1000.0) * 1024.0
    assert json.loads((tmp_path / "profiles" / "traffic.json").read_text())[kern]["dispatches"] == 2
    assert b.measured_traffic(kern) == rec["bytes_per_dispatch"]
    assert "__amd_rocclr_copyBuffer" not in table


@pytest.mark.parametrize("nu,nb", [(1, 3), (5, 30), (10, 100)])
def test_mds_workload_is_the_paper_table(nu, nb):
    g = _golden("mds_parameters.json")
    p = W.mds(nu, nb, n_time=_golden("chunk_study.json")["n_time"])
    assert p["times"][-1] == g["t_max"] and p["times"].shape[0] == 2001 and p["n"] == 2 * nu
    assert (p["y0"] == 0).all()
    for b in range(nb):
        row = p["params"][b]
        np.testing.assert_array_equal(row[:nu], np.linspace(*g["K"]["linspace"], nu))
        np.testing.assert_array_equal(row[nu:2 * nu], np.linspace(*g["C"]["linspace"], nu))
        np.testing.assert_array_equal(row[2 * nu:3 * nu], np.linspace(*g["M"]["linspace"], nu))
        assert row[3 * nu] == g["f_a"] and row[3 * nu + 1] == np.linspace(*g["T"]["linspace"], nb)[b]


@pytest.mark.parametrize("nu,nb", [(1, 3), (25, 100)])
def test_neural_ode_workload_is_the_paper_table(nu, nb):
    g = _golden("neural_ode_parameters.json")
    p = W.fnode(nu, nb)
    m = nu + 1
    assert p["times"][-1] == g["t_max"] and p["n"] == nu and (p["y0"] == 0).all()
    P = 2 * m * m + 2 * m + nu * m + nu + 2
    assert p["params"].shape == (nb, P)
    w = p["params"][:, :-2]
    assert (w == w[0]).all()                      # one set of layers for every series
    assert np.abs(w).max() <= np.sqrt(1.0 / m)    # the uniform law's range
    for b in range(nb):
        assert p["params"][b, -2] == g["f_a"] and p["params"][b, -1] == np.linspace(*g["T"]["linspace"], nb)[b]
    study = _golden("chunk_study.json")
    assert study["n_unit"]["neural_ode"] == [1, 5, 10, 15, 20, 25]
    assert study["n_unit"]["mass_damper_spring"] == [1, 2, 3, 5, 10]
