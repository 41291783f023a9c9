"""Shared helpers of the GPU parity tests (numpy side; no method arithmetic
beyond the residual invariant checks)."""
import numpy as np

PARITY_TOL = (1e-13, 1e-13)  # both sides iterate Newton to rounding level
TIMING_TOL = (1e-8, 1e-6)    # the paper's tolerances (Section 2.3)


def series_rel_err(a, b, offsets=None):
    """Per series ||a - b||_inf / ||b||_inf over all steps and components."""
    if offsets is None:
        num = np.abs(a - b).reshape(a.shape[0], -1).max(axis=1)
        den = np.abs(b).reshape(b.shape[0], -1).max(axis=1)
    else:
        B = offsets.shape[0] - 1
        num = np.array([np.abs(a[offsets[i]:offsets[i + 1]] - b[offsets[i]:offsets[i + 1]]).max() for i in range(B)])
        den = np.array([np.abs(b[offsets[i]:offsets[i + 1]]).max() for i in range(B)])
    return num / np.maximum(den, 1e-300)


def rhs_np(kind, y, p):
    """Model rates evaluated with numpy over [..., n] states (p broadcast per series)."""
    if kind == "linear":
        n = y.shape[-1]
        A = p.reshape(p.shape[:-1] + (n, n))
        return np.einsum("...ik,...k->...i", A, y)
    if kind == "vanderpol":
        mu = p[..., 0]
        return np.stack([y[..., 1], mu * (1.0 - y[..., 0] ** 2) * y[..., 1] - y[..., 0]], -1)
    if kind == "robertson":
        k1, k2, k3 = 0.04 * p[..., 0], 3.0e7 * p[..., 1], 1.0e4 * p[..., 2]
        a, b, c = k1 * y[..., 0], k3 * y[..., 1] * y[..., 2], k2 * y[..., 1] ** 2
        return np.stack([-a + b, a - b - c, c], -1)
    raise ValueError(kind)


def be_step_residual(kind, y, times, params):
    """max_k ||y_k - y_{k-1} - dt_k h(y_k)||_2 per series for a uniform grid [B, N+1, n]."""
    dt = np.diff(times)[None, :, None]
    f = rhs_np(kind, y[:, 1:], params[:, None, :])
    r = y[:, 1:] - y[:, :-1] - dt * f
    return np.linalg.norm(r, axis=2).max(axis=1)


def be_step_residual_ragged(kind, y, times, params, offsets):
    B = offsets.shape[0] - 1
    out = np.zeros(B)
    for b in range(B):
        sl = slice(offsets[b], offsets[b + 1])
        yb, tb = y[sl], times[sl]
        if yb.shape[0] < 2:
            continue
        f = rhs_np(kind, yb[1:], params[b][None, :])
        r = yb[1:] - yb[:-1] - np.diff(tb)[:, None] * f
        out[b] = np.linalg.norm(r, axis=1).max()
    return out


def certify_alternate_root(kind, yg, yo, times, p, agree=1e-8, jump=1e-5, resid=1e-8):
    """True if two trajectories of one series [N+1, n] part at a step whose
    backward-Euler equation has (at least) two roots: they agree (to `agree`)
    up to step k-1, differ by more than `jump` at step k, and both y_k satisfy
    y_k - y_{k-1} - dt h(y_k) = 0 for that same y_{k-1}.  Exhibiting two
    distinct roots of one step's equation proves the step is not uniquely
    solvable, so neither trajectory is wrong."""
    scale = max(np.abs(yo).max(), 1e-300)
    d = np.abs(yg - yo).max(axis=1) / scale
    bad = np.nonzero(d > agree)[0]
    if bad.size == 0:
        return False
    k = int(bad[0])
    if k == 0 or d[k] <= jump:
        return False
    dt = times[k] - times[k - 1]
    rg = yg[k] - yo[k - 1] - dt * rhs_np(kind, yg[k][None], p[None])[0]
    ro = yo[k] - yo[k - 1] - dt * rhs_np(kind, yo[k][None], p[None])[0]
    tol = resid * max(1.0, np.abs(yo[k - 1]).max())
    return bool(np.abs(rg).max() <= tol and np.abs(ro).max() <= tol)
