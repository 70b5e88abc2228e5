"""Gradients of a loss l(x*(theta)) with respect to the QP data
theta = (Q, q, A, b, G, h), taken at the relaxed central-path point.

ift_vjp    Implicit function theorem (appendix A): with F(w, theta) = 0 the
           relaxed KKT conditions in w = (x, y, z, s), the vector-Jacobian
           product is lambda' dF/dtheta where J' lambda = -dl/dw and J is the
           standard Jacobian (eq. explicit_uncondensed) at the relaxed point.
           The parameter formulas are those of Algorithm 3 with
           (dx, dy, dz) = (lambda_x, lambda_y, lambda_z):
               grad_Q = (dx x' + x dx')/2   (symmetric parametrisation of Q)
               grad_q = dx
               grad_A = dy x' + y dx'
               grad_b = -dy
               grad_G = dz x' + z dx'
               grad_h = -dz
           Algorithm 3's own sign convention for the adjoint right-hand side is
           ambiguous; this is the definition, whose sign the finite-difference
           pins fix.
fd_vjp     central differences of l(x_relaxed(theta)) along a direction.

Test infrastructure only (see package docstring).
"""
from __future__ import annotations

import numpy as np

from . import kkt
from . import implicit


def ift_vjp(Q, q, A, b, G, h, x, y, z, s, gx, gy=None, gz=None):
    """Exact VJP at the point (x, y, z, s) for upstream (gx, gy, gz)."""
    Q, A, G = (np.asarray(a, dtype=np.float64) for a in (Q, A, G))
    n, p, m = Q.shape[0], A.shape[0], G.shape[0]
    J = kkt.standard_jacobian(Q, A, G, z, s)
    g = np.zeros(n + p + 2 * m)
    g[:n] = gx
    if gy is not None:
        g[n:n + p] = gy
    if gz is not None:
        g[n + p:n + p + m] = gz
    lam = np.linalg.solve(J.T, -g)
    dx, dy, dz = lam[:n], lam[n:n + p], lam[n + p:n + p + m]
    return {
        "Q": 0.5 * (np.outer(dx, x) + np.outer(x, dx)),
        "q": dx,
        "A": np.outer(dy, x) + np.outer(y, dx),
        "b": -dy,
        "G": np.outer(dz, x) + np.outer(z, dx),
        "h": -dz,
        "dx": dx, "dy": dy, "dz": dz,
    }


def relaxed_point(Q, q, A, b, G, h, kappa_relax, *, tol=1e-13, warm=None):
    """Solve (Algorithm 1) and relax (Algorithm 2) in FP64.  ``warm`` =
    (x, y, z, s) skips the solve and relaxes from that point."""
    if warm is None:
        r = implicit.solve_qp(Q, q, A, b, G, h, tol=1e-10, max_iter=200)
        warm = (r.x, r.y, r.z, r.s)
    rr = implicit.relax_qp(Q, q, A, b, G, h, *warm, kappa_relax, tol=tol, max_iter=200)
    return rr


def grad_at_relaxed(Q, q, A, b, G, h, kappa_relax, gx, gy=None, gz=None, warm=None):
    rr = relaxed_point(Q, q, A, b, G, h, kappa_relax, warm=warm)
    return ift_vjp(Q, q, A, b, G, h, rr.x, rr.y, rr.z, rr.s, gx, gy, gz), rr


def fd_vjp(Q, q, A, b, G, h, kappa_relax, gx, direction, step, warm, gy=None, gz=None):
    """Central difference (l(theta + t D) - l(theta - t D)) / 2t with
    l = gx' x + gy' y + gz' z at the relaxed point (gy, gz optional).
    ``direction`` is a dict with keys Q..h (Q's direction should be
    symmetric); ``warm`` is the relaxed point at theta, used to warm-start
    both perturbed relaxations."""
    base = dict(Q=Q, q=q, A=A, b=b, G=G, h=h)
    vals = []
    for sgn in (1.0, -1.0):
        th = {k: np.asarray(base[k], np.float64) + sgn * step * direction.get(k, 0.0)
              for k in base}
        rr = implicit.relax_qp(th["Q"], th["q"], th["A"], th["b"], th["G"], th["h"],
                               *warm, kappa_relax, tol=1e-13, max_iter=200)
        val = float(gx @ rr.x)
        if gy is not None:
            val += float(gy @ rr.y)
        if gz is not None:
            val += float(gz @ rr.z)
        vals.append(val)
    return (vals[0] - vals[1]) / (2.0 * step)
