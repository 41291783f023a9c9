"""The allocation-free adjoint entry point (tvi_solve_adjoint_noalloc) against
tvi_solve_adjoint with a caller workspace, through the C ABI.

Both run the same kernels on the same inputs, so their outputs must be
bitwise equal.  Each case makes two calls in a row on the static scratch, the
second with a smaller batch (and a different chunk), so a stale byte left by
the first call would show up in the second.  The states are recomputed from
checkpoints (the scratch holds the recomputed chunk) and, for the neural ODE,
the scratch also holds the per-series parameter gradients."""
import numpy as np
import pytest

from paper_2310_08649_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tvi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_08649_amd import tvi as t
    t.load()
    return t


def _rob_case(tvi, B, seed, chunk, lanes, spl):
    w = W.robertson(B=B, seed=seed, n_range=(50, 3000))
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    y0, times, p = d(w["y0"]), d(w["times"]), d(w["params"])
    off = torch.as_tensor(w["offsets"], device="cuda")
    kw = dict(offsets=off, chunk=chunk, lanes=lanes, steps_per_lane=spl, tol=(1e-10, 1e-8))
    y, st, _, ck = tvi.solve_forward("robertson", y0, times, p, checkpoints=True, **kw)
    g = y / torch.sqrt((y * y).sum())
    ref = tvi.solve_adjoint("robertson", times, p, g, ckpt=ck, **kw)
    new = tvi.solve_adjoint("robertson", times, p, g, ckpt=ck, noalloc=True, **kw)
    return st, ref, new


def _mlp_case(tvi, B, N, chunk, seed):
    w = W.mlp(B=B, N=N, seed=seed)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    y0, times, theta = d(w["y0"]), d(w["times"]), d(w["params"])
    kw = dict(chunk=chunk, tol=(1e-8, 1e-6))
    y, st, _, ck = tvi.solve_forward("mlp", y0, times, theta, checkpoints=True, **kw)
    g = y / torch.sqrt((y.double() ** 2).sum()).float()
    ref = tvi.solve_adjoint("mlp", times, theta, g, ckpt=ck, **kw)
    new = tvi.solve_adjoint("mlp", times, theta, g, ckpt=ck, noalloc=True, **kw)
    return st, ref, new


def _same(ref, new):
    for a, b in zip(ref, new):
        assert torch.equal(a, b)


def test_noalloc_adjoint_equals_workspace_adjoint_robertson(tvi):
    # first call: 96 ragged series at chunk 64; second: 17 series at chunk 32
    for B, seed, chunk, lanes, spl in ((96, 301, 64, 16, 4), (17, 302, 32, 32, 1)):
        print("noalloc robertson B=%d chunk=%d" % (B, chunk), flush=True)
        st, ref, new = _rob_case(tvi, B, seed, chunk, lanes, spl)
        torch.cuda.synchronize()
        assert (st.cpu() == 0).all()
        assert (ref[2].cpu() == 0).all()
        _same(ref, new)


def test_noalloc_adjoint_equals_workspace_adjoint_mlp(tvi):
    for B, N, chunk, seed in ((12, 400, 100, 311), (5, 250, 64, 312)):
        print("noalloc mlp B=%d N=%d chunk=%d" % (B, N, chunk), flush=True)
        st, ref, new = _mlp_case(tvi, B, N, chunk, seed)
        torch.cuda.synchronize()
        assert (st.cpu() == 0).all()
        assert (ref[2].cpu() == 0).all()
        _same(ref, new)


def test_noalloc_adjoint_rejects_more_than_its_scratch(tvi):
    """A recomputation workspace above the static scratch is refused before
    anything is enqueued (TVI_ESCRATCH)."""
    import ctypes
    lib = tvi.load()
    o = tvi.make_options(chunk=512)
    m = tvi.Model(2, 3, tvi.F64, 0, 64)
    need = lib.tvi_adjoint_workspace_bytes(ctypes.byref(m), ctypes.byref(o), 4096)
    assert need > (32 << 20)
    f = ctypes.c_void_p(0x1000)
    assert lib.tvi_solve_adjoint_noalloc(ctypes.byref(m), ctypes.byref(o), 4096, 100, None, f, f, None, f, f, f, f,
                                         f, None) == -5
