"""Standard (explicit-complementarity) primal-dual IPM: the ablation arm.

Mehrotra predictor-corrector in the CVXGEN style (the paper refers to
CVXGEN for the standard method's details and names its stages in the NaN
trace of appendix D.4: z/s scaling, affine predictor, centering (sigma, mu),
corrector, line search).  Each Newton step solves the uncondensed standard
system eq. explicit_uncondensed with dense LU.

Readings: the step length is 0.99 times the ratio-test step of eq.
linesearch, capped at 1 (CVXGEN convention; without a back-off s or z can
hit 0 exactly); sigma = (mu_aff / mu)^3; the corrector adds the second-order
term ds_aff * dz_aff.  The relaxation drives z*s to kappa_relax by Newton
steps on the perturbed system (section 2.2, eq. r_{c,kappa}).

Test infrastructure only (see package docstring).
"""
from __future__ import annotations

import numpy as np

from . import kkt
from .implicit import Result, initialize, linesearch, CONVERGED, MAX_ITER, NONFINITE


def _measure(Q, q, A, b, G, h, x, y, z, s, kappa_relax=None):
    rt_s, ri_s, re_s = kkt.scaled_norms(Q, q, A, b, G, h, x, y, z, s)
    out = max(rt_s, ri_s, re_s)
    if G.shape[0]:
        if kappa_relax is None:
            out = max(out, float(np.max(z * s)))
        else:
            out = max(out, float(np.max(np.abs(z * s - kappa_relax))) / kappa_relax)
    return float(out)


def _solve(Q, q, A, b, G, h, x, y, z, s, rc):
    r_t, _, r_i, r_e = kkt.kkt_residuals(Q, q, A, b, G, h, x, y, z, s)
    J = kkt.standard_jacobian(Q, A, G, z, s)
    d = np.linalg.solve(J, -np.concatenate([r_t, r_e, r_i, rc]))
    n, p, m = Q.shape[0], A.shape[0], G.shape[0]
    return d[:n], d[n:n + p], d[n + p:n + p + m], d[n + p + m:]


def solve_qp(Q, q, A, b, G, h, *, tol=1e-12, max_iter=100, backoff=0.99,
             dtype=np.float64) -> Result:
    """Mehrotra predictor-corrector on the standard KKT system."""
    Q, q, A, b, G, h = (np.asarray(a, dtype=dtype) for a in (Q, q, A, b, G, h))
    x, y, z, s = initialize(Q, q, A, b, G, h)
    m = G.shape[0]
    if m == 0:
        return Result(x, y, z, s, 0.0, 0, CONVERGED, _measure(Q, q, A, b, G, h, x, y, z, s))
    with np.errstate(all="ignore"):
        for it in range(max_iter):
            res = _measure(Q, q, A, b, G, h, x, y, z, s)
            if not np.isfinite(res):
                return Result(x, y, z, s, float(s @ z) / m, it, NONFINITE, res)
            if res < tol:
                return Result(x, y, z, s, float(s @ z) / m, it, CONVERGED, res)
            mu = float(s @ z) / m
            try:
                dxa, dya, dza, dsa = _solve(Q, q, A, b, G, h, x, y, z, s, z * s)
                aa = linesearch(s, z, dsa, dza)
                mu_aff = float((s + aa * dsa) @ (z + aa * dza)) / m
                sig = (mu_aff / mu) ** 3
                dx, dy, dz, ds = _solve(Q, q, A, b, G, h, x, y, z, s,
                                        z * s + dsa * dza - sig * mu)
            except np.linalg.LinAlgError:
                return Result(x, y, z, s, mu, it, NONFINITE, np.nan)
            alpha = min(1.0, backoff * linesearch(s, z, ds, dz))
            x, y, z, s = x + alpha * dx, y + alpha * dy, z + alpha * dz, s + alpha * ds
    res = _measure(Q, q, A, b, G, h, x, y, z, s)
    return Result(x, y, z, s, float(s @ z) / m, max_iter, CONVERGED if res < tol else MAX_ITER, res)


def relax_qp(Q, q, A, b, G, h, x, y, z, s, kappa_relax, *, tol=1e-12, max_iter=100,
             backoff=0.99, dtype=np.float64) -> Result:
    """Newton steps on Qx+q+G'z+A'y = 0, Ax = b, Gx+s = h, z*s = kappa_relax,
    warm-started at a solution (the standard arm's relaxation)."""
    Q, q, A, b, G, h, x, y, z, s = (np.asarray(a, dtype=dtype)
                                    for a in (Q, q, A, b, G, h, x, y, z, s))
    m = G.shape[0]
    if m == 0:
        return Result(x, y, z, s, 0.0, 0, CONVERGED, 0.0)
    with np.errstate(all="ignore"):
        for it in range(max_iter):
            res = _measure(Q, q, A, b, G, h, x, y, z, s, kappa_relax)
            if not np.isfinite(res):
                return Result(x, y, z, s, float(s @ z) / m, it, NONFINITE, res)
            if res < tol:
                return Result(x, y, z, s, float(s @ z) / m, it, CONVERGED, res)
            try:
                dx, dy, dz, ds = _solve(Q, q, A, b, G, h, x, y, z, s, z * s - kappa_relax)
            except np.linalg.LinAlgError:
                return Result(x, y, z, s, float(s @ z) / m, it, NONFINITE, np.nan)
            alpha = min(1.0, backoff * linesearch(s, z, ds, dz))
            x, y, z, s = x + alpha * dx, y + alpha * dy, z + alpha * dz, s + alpha * ds
    res = _measure(Q, q, A, b, G, h, x, y, z, s, kappa_relax)
    return Result(x, y, z, s, float(s @ z) / m, max_iter, CONVERGED if res < tol else MAX_ITER, res)
