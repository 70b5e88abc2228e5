"""Algorithm 1 (solve_qp) and Algorithm 2 (relax_qp) with implicit
complementarity, in plain dense FP64.

Each Newton step solves the *uncondensed* system eq. implicit_kkt with dense
LU.  That form is what defines the step; the paper warns against it in low
precision (appendix B.2), which does not matter in float64.  The GPU path
solves the reduced form instead and shares none of this code.

Readings of passages the paper leaves open (each is listed in the design
notes as well):
  * initialize ("same as CVXOPT / CVXGEN"): solve the regularised KKT system
    [Q A' G'; A 0 0; G 0 -I][x; y; zt] = [-q; b; h], set s = -zt, z = zt, and
    shift each to be positive: if max(-s) >= 0 then s += 1 + max(-s) (same
    for z).
  * kappa = s'z / m with m the number of inequality rows.
  * stopping test: scaled residual norms (kkt.scaled_norms), the
    complementarity measure max(z*s) (= kappa on the manifold) and the
    implicit residuals r_z, r_s scaled by 1 + max(|z|, |s|), all < tol.
  * centering: fixed kappa_target = sigma*kappa (Algorithm 1 as printed), or,
    with pc=True, a predictor with kappa_target = 0 followed by a corrector
    with kappa_target = (kappa_aff / kappa)^3 kappa on the same matrix, where
    kappa_aff = (s + a ds)'(z + a dz) / m at the predictor's step length a.
    The implicit linearisation has no z*s product, so there is no
    second-order correction term.
  * line search: eq. linesearch as printed (no back-off).
  * relax: residual test with |z*s - kappa_relax| / kappa_relax in place of
    max(z*s); the matrix is refactored at every iterate.
  * m = 0 (no inequalities): the initial KKT solve is already the optimum.

Test infrastructure only (see package docstring).
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import kkt
from . import retraction as rt

CONVERGED, MAX_ITER, NONFINITE = 0, 1, 2


@dataclasses.dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    s: np.ndarray
    kappa: float
    iters: int
    status: int
    res: float


def linesearch(s, z, ds, dz):
    """eq. linesearch: largest alpha <= 1 keeping s + alpha ds >= 0 and
    z + alpha dz >= 0 (linearised)."""
    alpha = 1.0
    neg = ds < 0
    if np.any(neg):
        alpha = min(alpha, float(np.min(-s[neg] / ds[neg])))
    neg = dz < 0
    if np.any(neg):
        alpha = min(alpha, float(np.min(-z[neg] / dz[neg])))
    return alpha


def initialize(Q, q, A, b, G, h):
    """CVXOPT-style starting point (reading of 'initialize' in Algorithm 1)."""
    n, p, m = Q.shape[0], A.shape[0], G.shape[0]
    N = n + p + m
    K = np.zeros((N, N), dtype=Q.dtype)
    K[:n, :n] = Q
    K[:n, n:n + p] = A.T
    K[:n, n + p:] = G.T
    K[n:n + p, :n] = A
    K[n + p:, :n] = G
    K[n + p:, n + p:] = -np.eye(m)
    sol = np.linalg.solve(K, np.concatenate([-q, b, h]))
    x, y, zt = sol[:n], sol[n:n + p], sol[n + p:]
    s, z = -zt, zt.copy()
    if m:
        ap = float(np.max(-s))
        if ap >= 0:
            s = s + (1.0 + ap)
        ad = float(np.max(-z))
        if ad >= 0:
            z = z + (1.0 + ad)
    return x, y, z, s


def residual_measure(Q, q, A, b, G, h, x, y, z, s, v, kappa, kappa_relax=None):
    """Largest scaled residual (see module docstring)."""
    rt_s, ri_s, re_s = kkt.scaled_norms(Q, q, A, b, G, h, x, y, z, s)
    out = max(rt_s, ri_s, re_s)
    if G.shape[0]:
        r_z, r_s = kkt.implicit_residuals(z, s, v, kappa)
        rzs = max(np.max(np.abs(r_z)), np.max(np.abs(r_s))) / (
            1.0 + max(np.max(np.abs(z)), np.max(np.abs(s))))
        if kappa_relax is None:
            rc = float(np.max(z * s))
        else:
            rc = float(np.max(np.abs(z * s - kappa_relax))) / kappa_relax
        out = max(out, rzs, rc)
    return float(out)


def newton_direction(Q, q, A, b, G, h, x, y, z, s, v, kappa, kappa_target):
    """Solve eq. implicit_kkt for (dx, dy, dz, ds, dv, dkappa) with
    r_kappa = kappa - kappa_target."""
    r_t, _, r_i, r_e = kkt.kkt_residuals(Q, q, A, b, G, h, x, y, z, s)
    r_z, r_s = kkt.implicit_residuals(z, s, v, kappa)
    J, sl = kkt.implicit_jacobian(Q, A, G, v, kappa)
    rhs = -np.concatenate([r_t, r_e, r_i, r_z, r_s, [kappa - kappa_target]])
    d = np.linalg.solve(J, rhs)
    return tuple(d[k] for k in sl)


def _newton_loop(Q, q, A, b, G, h, x, y, z, s, *, tol, max_iter, target, kappa_relax=None):
    m = G.shape[0]
    dt = Q.dtype
    v = z - s
    kappa = float(s @ z) / m
    res = np.inf
    for it in range(max_iter):
        # manifold coordinates
        v = z - s
        kappa = float(s @ z) / m
        res = residual_measure(Q, q, A, b, G, h, x, y, z, s, v, kappa, kappa_relax)
        if not np.isfinite(res):
            return Result(x, y, z, s, kappa, it, NONFINITE, res)
        if res < tol:
            return Result(x, y, z, s, kappa, it, CONVERGED, res)
        kt = target(Q, q, A, b, G, h, x, y, z, s, v, kappa)
        dx, dy, dz, ds, dv, dk = newton_direction(Q, q, A, b, G, h, x, y, z, s, v, kappa, kt)
        alpha = linesearch(s, z, ds, dz)
        x = x + alpha * dx
        y = y + alpha * dy
        v = v + alpha * dv
        kappa = kappa + alpha * float(dk[0])
        z = rt.b(v, kappa).astype(dt)
        s = rt.b(-v, kappa).astype(dt)
    v = z - s
    kappa = float(s @ z) / m
    res = residual_measure(Q, q, A, b, G, h, x, y, z, s, v, kappa, kappa_relax)
    return Result(x, y, z, s, kappa, max_iter, CONVERGED if res < tol else MAX_ITER, res)


def solve_qp(Q, q, A, b, G, h, *, sigma=0.1, tol=1e-12, max_iter=100, pc=True,
             dtype=np.float64) -> Result:
    """Algorithm 1: implicit-complementarity primal-dual IPM."""
    Q, q, A, b, G, h = (np.asarray(a, dtype=dtype) for a in (Q, q, A, b, G, h))
    x, y, z, s = initialize(Q, q, A, b, G, h)
    m = G.shape[0]
    if m == 0:
        res = residual_measure(Q, q, A, b, G, h, x, y, z, s, z, 0.0)
        return Result(x, y, z, s, 0.0, 0, CONVERGED if res < max(tol, 1e-10) else MAX_ITER, res)

    def target(Q, q, A, b, G, h, x, y, z, s, v, kappa):
        if not pc:
            return sigma * kappa
        # predictor: aim at kappa = 0, measure how far the affine step gets
        _, _, dz, ds, _, _ = newton_direction(Q, q, A, b, G, h, x, y, z, s, v, kappa, 0.0)
        a = linesearch(s, z, ds, dz)
        kaff = float((s + a * ds) @ (z + a * dz)) / m
        return (kaff / kappa) ** 3 * kappa

    return _newton_loop(Q, q, A, b, G, h, x, y, z, s, tol=tol, max_iter=max_iter, target=target)


def relax_qp(Q, q, A, b, G, h, x, y, z, s, kappa_relax, *, tol=1e-12, max_iter=100,
             dtype=np.float64) -> Result:
    """Algorithm 2: warm-started from a solution, drive kappa to kappa_relax
    along the central path (kappa_target = kappa_relax every step)."""
    Q, q, A, b, G, h, x, y, z, s = (np.asarray(a, dtype=dtype)
                                    for a in (Q, q, A, b, G, h, x, y, z, s))
    if G.shape[0] == 0:
        return Result(x, y, z, s, 0.0, 0, CONVERGED, 0.0)
    return _newton_loop(Q, q, A, b, G, h, x, y, z, s, tol=tol, max_iter=max_iter,
                        target=lambda *a: kappa_relax, kappa_relax=kappa_relax)
