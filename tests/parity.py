"""Shared helpers of the GPU parity tests (not a test module).

Every comparison with the FP64 oracle is entry by entry:

    |gpu_i - ref_i| <= atol + rtol * |ref_i|      for every entry i

with atol stated per quantity below.  The float32 path runs on the same
float32-rounded inputs as the oracle.

Tolerances (the solve stops at a scaled KKT residual of `tol`, 1e-5 unless a
test says otherwise):
  x          atol = 1e-4 * max(1, |x*|_inf),  rtol = 1e-4
  s          atol = tol * (1 + max(|G x*|_inf, |s*|_inf, |h|_inf))
                    + |G|_inf * 1e-4 * max(1, |x*|_inf),          rtol = 1e-4
             (s - s* = (s - (h - G x)) - G (x - x*): the primal residual the
             stopping test allows plus the image of the allowed x error)
  y, z       atol = 1e-3 * max(1, |d*|_inf),  rtol = 1e-3  (where unique)
  gradients  atol = 1e-3 * max(|g_block|_inf, 1e-3 * |g_all|_inf),  rtol = 1e-3
             per parameter block (dQ, dq, dA, db, dG, dh); a block that is
             numerically zero is compared against the scale of the others.
"""
from __future__ import annotations

import numpy as np

X_TOL = 1e-4
DUAL_TOL = 1e-3
GRAD_TOL = 1e-3
BLOCKS = ("Q", "q", "A", "b", "G", "h")


def torch_mod():
    import pytest
    return pytest.importorskip("torch")


def dev():
    import pytest
    torch = torch_mod()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(P):
    d = dev()
    torch = torch_mod()
    return [torch.from_numpy(a).to(d) for a in P.arrays()]


def npd(d):
    """Tensors of a (nested) result dict as numpy arrays."""
    return {k: (v if not hasattr(v, "cpu") else v.cpu().numpy()) if not isinstance(v, dict)
            else npd(v) for k, v in d.items()}


def outcome(status):
    """Per-QP outcome (low byte of the status word)."""
    return np.asarray(status) & 0xFF


def inf(a):
    a = np.asarray(a, np.float64)
    return float(np.max(np.abs(a))) if a.size else 0.0


def assert_close(what, got, ref, atol, rtol):
    """Entry-by-entry |got - ref| <= atol + rtol |ref|; returns the largest
    ratio |got - ref| / (atol + rtol |ref|) (<= 1 passes)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    if ref.size == 0:
        return 0.0
    assert np.all(np.isfinite(got)), (what, "non-finite entries")
    bound = atol + rtol * np.abs(ref)
    ratio = np.abs(got - ref) / bound
    k = int(np.argmax(ratio))
    worst = float(ratio.flat[k])
    assert worst <= 1.0, (f"{what}: entry {np.unravel_index(k, ref.shape)} off by "
                          f"{abs(got.flat[k] - ref.flat[k]):.3e} (bound {bound.flat[k]:.3e}, "
                          f"ref {ref.flat[k]:.3e})")
    return worst


def check_x(what, x, ref_x):
    return assert_close(what + " x", x, ref_x, X_TOL * max(1.0, inf(ref_x)), X_TOL)


def check_point(what, P, i, sol, ref, tol=1e-5, duals=True):
    """x, s (and y, z if `duals`) of QP i of `sol` against the oracle result
    `ref` (fields x, y, z, s)."""
    Q, q, A, b, G, h = P.one(i)
    w = check_x(what, sol["x"][i], ref.x)
    if G.shape[0]:
        gx = G @ ref.x
        atol_s = (tol * (1.0 + max(inf(gx), inf(ref.s), inf(h)))
                  + inf(np.sum(np.abs(G), axis=1)) * X_TOL * max(1.0, inf(ref.x)))
        w = max(w, assert_close(what + " s", sol["s"][i], ref.s, atol_s, X_TOL))
        if duals:
            w = max(w, assert_close(what + " z", sol["z"][i], ref.z,
                                    DUAL_TOL * max(1.0, inf(ref.z)), DUAL_TOL))
    if A.shape[0] and duals:
        w = max(w, assert_close(what + " y", sol["y"][i], ref.y,
                                DUAL_TOL * max(1.0, inf(ref.y)), DUAL_TOL))
    return w


def check_grads(what, g, i, ref):
    """The six gradient blocks of QP i (dicts of batched arrays `g`) against
    the oracle's (dict of per-QP arrays `ref`)."""
    scale_all = max(inf(ref[k]) for k in BLOCKS)
    w = 0.0
    for k in BLOCKS:
        r = np.asarray(ref[k])
        if r.size == 0:
            continue
        atol = GRAD_TOL * max(inf(r), 1e-3 * scale_all)
        w = max(w, assert_close(f"{what} d{k}", g[k][i], r, atol, GRAD_TOL))
    return w
