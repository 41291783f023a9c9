"""The C-ABI library loads and exports every symbol tvi.h declares; host-side
argument checks reject bad calls synchronously, before any launch.  CPU only:
no call here reaches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvi.h")
LIB = os.path.join(ROOT, "paper_2310_08649_amd", "libtvi.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tvi_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libtvi.so not built")
    from paper_2310_08649_amd import tvi
    return tvi.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("tvi_pcr_solve", "tvi_solve_forward", "tvi_solve_adjoint", "tvi_adjoint_workspace_bytes",
              "tvi_default_options", "tvi_status_str", "tvi_version", "tvi_param_count"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults(lib):
    from paper_2310_08649_amd import tvi
    assert lib.tvi_status_str(0) == b"ok"
    assert lib.tvi_status_str(-1) == b"invalid argument"
    assert b"gfx950" in lib.tvi_version()
    o = tvi.make_options()
    assert o.chunk == 64 and o.tol_a == 1e-8 and o.tol_r == 1e-6 and o.halving == 1
    assert tvi.param_count("linear", 4) == 16
    assert tvi.param_count("vanderpol", 2) == 1
    assert tvi.param_count("robertson", 3) == 3
    assert tvi.param_count("mlp", 8, 64) == 5256


def _fake():
    return ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("field,value", [("chunk", 0), ("chunk", 2049), ("max_newton", 0), ("tol_a", -1.0),
                                         ("init", 7), ("lanes", 3), ("steps_per_lane", 16),
                                         ("max_newton_chunk", -1)])
def test_forward_rejects_bad_options(lib, field, value):
    from paper_2310_08649_amd import tvi
    m = tvi.Model(tvi.KINDS["vanderpol"], 2, tvi.F64, 0, 64)
    o = tvi.make_options(chunk=64)
    if field in ("lanes", "steps_per_lane"):
        o.lanes, o.steps_per_lane = 64, 1
    setattr(o, field, value)
    f = _fake()
    rc = lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None)
    assert rc == -1


def test_forward_rejects_bad_model_and_sizes(lib):
    from paper_2310_08649_amd import tvi
    o = tvi.make_options(chunk=16)
    f = _fake()
    bad_models = [tvi.Model(1, 3, tvi.F64, 0, 64),   # Van der Pol with n = 3
                  tvi.Model(2, 2, tvi.F64, 0, 64),   # Robertson with n = 2
                  tvi.Model(9, 2, tvi.F64, 0, 64),   # unknown kind
                  tvi.Model(1, 2, 5, 0, 64)]         # unknown dtype
    for m in bad_models:
        assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None,
                                     None) == -1
    m = tvi.Model(1, 2, tvi.F64, 0, 64)
    # negative sizes, missing outputs
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), -1, 10, None, f, f, f, f, None, f, None, None) == -1
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, None, None, f, None, None) == -1
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, None, None, None) == -1
    # linear model beyond the supported sizes
    m = tvi.Model(0, 8, tvi.F64, 0, 64)
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None) == -4
    # an empty batch is a no-op
    m = tvi.Model(1, 2, tvi.F64, 0, 64)
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 0, 10, None, None, None, None, None, None, None,
                                 None, None) == 0


def test_adjoint_and_pcr_reject_bad_arguments(lib):
    from paper_2310_08649_amd import tvi
    o = tvi.make_options(chunk=16)
    f = _fake()
    m = tvi.Model(1, 2, tvi.F64, 0, 64)
    # recomputation needs checkpoints and a large enough workspace
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, None, None, f, f, f, f, f, 10**9,
                                 None) == -1
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, None, f, f, f, f, f, f, 8,
                                 None) == -1
    assert lib.tvi_adjoint_workspace_bytes(ctypes.byref(m), ctypes.byref(o), 4) == 4 * 16 * 2 * 8
    # shared parameters are not supported by the analytic adjoint
    ms = tvi.Model(1, 2, tvi.F64, 1, 64)
    assert lib.tvi_solve_adjoint(ctypes.byref(ms), ctypes.byref(o), 4, 10, None, f, f, f, None, f, f, f, f, None, 0,
                                 None) == -4
    assert lib.tvi_pcr_solve(tvi.F64, 2, 4, 0, f, f, f, 0, None) == -1
    assert lib.tvi_pcr_solve(tvi.F64, 2, 4, 513, f, f, f, 0, None) == -1
    assert lib.tvi_pcr_solve(tvi.F64, 9, 4, 8, f, f, f, 0, None) == -4
    assert lib.tvi_pcr_solve(tvi.F64, 8, 4, 8, f, f, f, 0, None) == -4    # 8 x 8: float only
    assert lib.tvi_pcr_solve(tvi.F32, 8, 4, 129, f, f, f, 0, None) == -4  # and m <= 128
    assert lib.tvi_pcr_solve(7, 2, 4, 8, f, f, f, 0, None) == -1
    assert lib.tvi_pcr_solve(tvi.F64, 2, 4, 8, None, f, f, 0, None) == -1


def test_predictor_options_and_pack_reject_bad_arguments(lib):
    """The learned start: bad base, missing parameters, too few predicted steps,
    too narrow a segment or too many values per lane are refused before any
    launch; pack refuses aliasing and a bad shape."""
    from paper_2310_08649_amd import predictor as pred
    from paper_2310_08649_amd import tvi
    f = _fake()
    m = tvi.Model(tvi.KINDS["vanderpol"], 2, tvi.F64, 0, 64)

    def fwd(o):
        return lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None)

    class P:  # a stand-in for a device tensor: only its address is marshalled
        def data_ptr(self):
            return 0x1000

    o = tvi.make_options(chunk=16, init="predictor", predictor=(P(), 128, 16, 2))
    assert fwd(o) == -1                       # base must be 0 or 1
    o = tvi.make_options(chunk=16, init="predictor", predictor=(P(), 128, 8, 0))
    assert fwd(o) == -1                       # predicts fewer steps than the chunk
    o = tvi.make_options(chunk=16, init="predictor", predictor=(P(), 512, 16, 0))
    assert fwd(o) == -1                       # hidden width beyond 256
    o = tvi.make_options(chunk=16, init="predictor")
    assert fwd(o) == -1                       # no parameters
    o = tvi.make_options(chunk=4, lanes=1, steps_per_lane=4, init="predictor", predictor=(P(), 128, 4, 0))
    assert fwd(o) == -4                       # one lane per series cannot share the network
    o = tvi.make_options(chunk=64, lanes=8, steps_per_lane=8, init="predictor", predictor=(P(), 128, 64, 0))
    assert fwd(o) == -4                       # 8 steps x n = 2 per lane: not compiled
    d = pred.Predictor(4, 128, 32)
    assert lib.tvi_predictor_pack(ctypes.byref(d), f, f, None) == -1   # aliasing
    bad = pred.Predictor(0, 128, 32)
    assert lib.tvi_predictor_pack(ctypes.byref(bad), f, ctypes.c_void_p(0x2000), None) == -1


def test_scheme_option_is_checked(lib):
    """Forward Euler: an unknown scheme is invalid; the learned start is refused
    with it; the default is backward Euler."""
    from paper_2310_08649_amd import tvi
    f = _fake()
    assert tvi.make_options().scheme == 0
    m = tvi.Model(tvi.KINDS["vanderpol"], 2, tvi.F64, 0, 64)
    o = tvi.make_options(chunk=16, scheme=2)
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None) == -1
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, None, f, f, f, f, None, 0,
                                 None) == -1

    class P:
        def data_ptr(self):
            return 0x1000

    o = tvi.make_options(chunk=16, init="predictor", predictor=(P(), 128, 16, 0), scheme="forward_euler")
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None) == -4
    mm = tvi.Model(tvi.KINDS["mlp"], 8, tvi.F32, 1, 64)
    o = tvi.make_options(chunk=16, init="predictor", predictor=(P(), 128, 16, 0), scheme="forward_euler")
    assert lib.tvi_solve_forward(ctypes.byref(mm), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None) == -4


def test_paper_example_models_sizes(lib):
    """Chaboche with 1 to 5 backstresses and one or two neurons run in the
    register-resident solver; other sizes are refused before any launch."""
    from paper_2310_08649_amd import tvi
    assert tvi.param_count("chaboche", 3) == 10 and tvi.param_count("chaboche", 4) == 12
    assert tvi.param_count("neuron", 4) == 16
    o = tvi.make_options(chunk=16)
    f = _fake()

    def fwd(kind, n, dtype=tvi.F64):
        m = tvi.Model(tvi.KINDS[kind], n, dtype, 0, 64)
        return lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None)

    assert fwd("chaboche", 2) == -1
    assert fwd("chaboche", 8) == -4
    assert fwd("neuron", 6) == -1
    # more neurons, the mass-damper-spring chain and the forced neural ODE: the
    # block solver, up to n = 40, double storage, with its workspace
    assert fwd("neuron", 12) == -1          # no workspace given
    assert fwd("neuron", 44) == -4
    assert fwd("mds", 7) == -1 and fwd("mds", 42) == -4 and fwd("fnode", 41) == -4
    assert fwd("mds", 20, tvi.F32) == -4
    assert tvi.param_count("mds", 20) == 32
    assert tvi.param_count("fnode", 5) == 2 * 36 + 12 + 30 + 5 + 2


def test_block_solver_options_and_workspace(lib):
    """The block solver's checks: its workspace size, the segment length, chunk
    up to 1024, and the options it does not take."""
    from paper_2310_08649_amd import tvi
    f = _fake()
    m = tvi.Model(tvi.KINDS["mds"], 20, tvi.F64, 0, 64)

    def ws(o, B=3, adjoint=False):
        fn = lib.tvi_adjoint_workspace_bytes if adjoint else lib.tvi_forward_workspace_bytes
        return fn(ctypes.byref(m), ctypes.byref(o), B)

    thomas, pcr, hybrid = (tvi.make_options(chunk=1000, steps_per_lane=T) for T in (1000, 1, 8))
    NP = 24  # n = 20 padded
    blk = NP * NP
    per = 1000 * blk + 1000 * NP + 1001 * NP      # step maps, offsets, iterate
    assert ws(thomas) == 3 * 8 * per
    assert ws(pcr) == 3 * 8 * (per + 1000 * blk + 1000 * NP)  # one more buffer of maps for the levels
    assert ws(hybrid) == 3 * 8 * (per + 2 * 125 * (blk + NP))
    assert ws(thomas, adjoint=True) == 3 * 8 * (per + 1000 * (5 * 10 + 3))  # plus the per-step factors
    assert ws(tvi.make_options(chunk=1025)) == 0
    assert lib.tvi_forward_workspace_bytes(ctypes.byref(tvi.Model(1, 2, tvi.F64, 0, 64)),
                                           ctypes.byref(thomas), 3) == 0   # not a block model

    def fwd(o, wsb=None):
        o.workspace = 0x1000
        o.workspace_bytes = ws(o) if wsb is None else wsb
        return lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 3, 10, None, f, f, f, f, None, f, None, None)

    assert fwd(tvi.make_options(chunk=64), wsb=100) == -1                      # workspace too small
    assert fwd(tvi.make_options(chunk=64, scheme="forward_euler")) == -4
    assert fwd(tvi.make_options(chunk=64, jacobian="forward_ad")) == -4
    assert fwd(tvi.make_options(chunk=64, reference="zero")) == -4
    assert fwd(tvi.make_options(chunk=1025)) == -1
    o = tvi.make_options(chunk=64)
    o.steps_per_lane = -2
    assert fwd(o) == -1
    # the adjoint reads the stored trajectory: no recomputation from checkpoints
    o = tvi.make_options(chunk=64)
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 3, 10, None, f, f, None, f, f, f, f, f, f,
                                 ws(o, adjoint=True), None) == -4


def test_jacobian_option_is_checked(lib):
    from paper_2310_08649_amd import tvi
    f = _fake()

    def fwd(o, kind="vanderpol", n=2, dtype=tvi.F64, shared=0):
        m = tvi.Model(tvi.KINDS[kind], n, dtype, shared, 64)
        return lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None)

    assert tvi.make_options().jacobian == 0
    assert fwd(tvi.make_options(chunk=16, jacobian=2)) == -1
    assert fwd(tvi.make_options(chunk=16, jacobian="forward_ad", scheme="forward_euler")) == -4
    assert fwd(tvi.make_options(chunk=16, jacobian="forward_ad"), dtype=tvi.F32) == -4
    assert fwd(tvi.make_options(chunk=16, jacobian="forward_ad"), kind="mlp", n=8, dtype=tvi.F32, shared=1) == -4


def test_larger_chaboche_one_step_per_lane(lib):
    from paper_2310_08649_amd import tvi
    f = _fake()
    m = tvi.Model(tvi.KINDS["chaboche"], 7, tvi.F64, 0, 64)

    def fwd(o):
        return lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None)

    assert tvi.param_count("chaboche", 7) == 18
    assert fwd(tvi.make_options(chunk=128, lanes=64, steps_per_lane=2)) == -4   # one step per lane only
    assert fwd(tvi.make_options(chunk=16, scheme="forward_euler")) == -4
    assert fwd(tvi.make_options(chunk=16, jacobian="forward_ad")) == -4
    mb = tvi.Model(tvi.KINDS["chaboche"], 8, tvi.F64, 0, 64)
    assert lib.tvi_solve_forward(ctypes.byref(mb), ctypes.byref(tvi.make_options(chunk=16)), 4, 10, None, f, f, f, f,
                                 None, f, None, None) == -4


def test_reference_residual_option_is_checked(lib):
    from paper_2310_08649_amd import tvi
    f = _fake()
    m = tvi.Model(tvi.KINDS["vanderpol"], 2, tvi.F64, 0, 64)
    assert tvi.make_options().reference_residual == 0
    o = tvi.make_options(chunk=16, reference=2)
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None) == -1


def test_noalloc_adjoint_rejects_more_than_its_scratch_on_the_host(lib):
    """tvi_solve_adjoint_noalloc refuses a workspace above its static scratch
    (TVI_ESCRATCH) on the host, before any HIP call."""
    from paper_2310_08649_amd import tvi
    o = tvi.make_options(chunk=512)
    m = tvi.Model(2, 3, tvi.F64, 0, 64)
    assert lib.tvi_adjoint_workspace_bytes(ctypes.byref(m), ctypes.byref(o), 4096) > (32 << 20)
    f = _fake()
    assert lib.tvi_solve_adjoint_noalloc(ctypes.byref(m), ctypes.byref(o), 4096, 100, None, f, f, None, f, f, f, f, f,
                                         None) == -5
    assert lib.tvi_status_str(-5).startswith(b"workspace needed exceeds")
    # bad options are still refused first
    o.chunk = 0
    assert lib.tvi_solve_adjoint_noalloc(ctypes.byref(m), ctypes.byref(o), 4, 100, None, f, f, None, f, f, f, f, f,
                                         None) == -1


def test_observed_steps_option_is_checked(lib):
    """obs_idx needs n_obs >= 1 and a uniform grid."""
    from paper_2310_08649_amd import tvi
    f = _fake()
    m = tvi.Model(1, 2, tvi.F64, 0, 64)
    o = tvi.make_options(chunk=16)
    o.obs_idx = 0x1000
    o.n_obs = 0
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, None, f, f, f, f, None, 0,
                                 None) == -1
    o.n_obs = 3
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 4, 10, f, f, f, f, None, f, f, f, f, None, 0,
                                 None) == -1   # ragged (offsets given)


def test_register_solver_refuses_divided_or_observed_gradients(lib):
    """The divided gradient (g_divisor) and observed-step gradients (obs_idx)
    are offered by the neural-ODE and block solvers, and the divided gradient
    by the stored-trajectory adjoint over several waves (Robertson and Van der
    Pol in double); the one-wave register solver's adjoint, the recomputing
    adjoint and the other models refuse them with TVI_EUNSUPPORTED before any
    HIP call."""
    from paper_2310_08649_amd import tvi
    f = _fake()
    m = tvi.Model(1, 2, tvi.F64, 0, 64)
    o = tvi.make_options(chunk=16)
    o.g_divisor = 0x1000
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, None, f, f, f, f, None, 0,
                                 None) == -4
    o.g_divisor = None
    o.obs_idx = 0x1000
    o.n_obs = 3
    assert lib.tvi_solve_adjoint(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, None, f, f, f, f, None, 0,
                                 None) == -4

    def adj(kind, n, dtype=tvi.F64, stored=True, **kw):
        mm = tvi.Model(tvi.KINDS[kind], n, dtype, 0, 64)
        oo = tvi.make_options(**kw)
        oo.g_divisor = 0x1000
        return lib.tvi_solve_adjoint(ctypes.byref(mm), ctypes.byref(oo), 4, 10, None, f, f, f if stored else None,
                                     f, f, f, f, f, f, 1 << 30, None)

    wide = dict(chunk=1024, lanes=128, steps_per_lane=8)
    assert adj("robertson", 3, stored=False, **wide) == -4      # recomputing adjoint
    assert adj("linear", 2, **wide) == -4                       # no wide kernels for this model
    assert adj("vanderpol", 2, dtype=tvi.F32, **wide) == -4     # double storage only
    assert adj("robertson", 3, jacobian="forward_ad", **wide) == -4
    assert adj("robertson", 3, chunk=512, lanes=64, steps_per_lane=8) == -4   # one wave


def test_series_sums_are_checked(lib):
    """Per-series sums of squares (tvi_options.series_sumsq) come from the
    forward pass over several waves only; the loss from sums checks its
    arguments; both before any HIP call."""
    from paper_2310_08649_amd import tvi
    f = _fake()

    def fwd(kind, n, dtype=tvi.F64, **kw):
        m = tvi.Model(tvi.KINDS[kind], n, dtype, 1 if kind == "mlp" else 0, 64)
        o = tvi.make_options(**kw)
        o.series_sumsq = 0x1000
        return lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None)

    wide = dict(chunk=1024, lanes=128, steps_per_lane=8)
    assert fwd("robertson", 3, chunk=512, lanes=64, steps_per_lane=8) == -4     # one wave
    assert fwd("linear", 2, **wide) == -4
    assert fwd("vanderpol", 2, dtype=tvi.F32, **wide) == -4
    assert fwd("robertson", 3, jacobian="forward_ad", **wide) == -4
    assert fwd("mlp", 8, dtype=tvi.F32, chunk=100) == -4
    assert lib.tvi_loss_from_sums(None, 4, f, None) == -1
    assert lib.tvi_loss_from_sums(f, 0, f, None) == -1
    assert lib.tvi_loss_from_sums(f, 4, None, None) == -1


def test_tilings_over_several_waves_are_checked(lib):
    """128 or 256 lanes (2 or 4 waves) take 2, 4 or 8 steps per lane and chunks up
    to 2048; other combinations, and these tilings for models or options the
    wide kernels do not cover, are refused on the host."""
    from paper_2310_08649_amd import tvi
    f = _fake()

    def fwd(kind, n, **kw):
        m = tvi.Model(tvi.KINDS[kind], n, tvi.F64, 0, 64)
        o = tvi.make_options(**kw)
        return lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None, None)

    for S, T, C in [(128, 1, 128), (512, 8, 2048), (256, 16, 2048), (96, 8, 512), (128, 8, 1025), (256, 8, 2049)]:
        assert fwd("robertson", 3, chunk=C, lanes=S, steps_per_lane=T) == -1, (S, T, C)
    # the register solver's other models stop at one wave
    assert fwd("linear", 2, chunk=1024, lanes=128, steps_per_lane=8) == -4
    assert fwd("chaboche", 3, chunk=1024, lanes=128, steps_per_lane=8) == -4
    # options the wide kernels do not take
    assert fwd("robertson", 3, chunk=1024, lanes=128, steps_per_lane=8, scheme="forward_euler") == -4
    assert fwd("vanderpol", 2, chunk=2048, lanes=256, steps_per_lane=8, jacobian="forward_ad") == -4
    assert fwd("robertson", 3, chunk=1024, lanes=128, steps_per_lane=8, init="extrap", reference="zero") == -4
    m = tvi.Model(tvi.KINDS["robertson"], 3, tvi.F32, 0, 64)
    o = tvi.make_options(chunk=1024, lanes=128, steps_per_lane=8)
    assert lib.tvi_solve_forward(ctypes.byref(m), ctypes.byref(o), 4, 10, None, f, f, f, f, None, f, None,
                                 None) == -4                         # double storage only
