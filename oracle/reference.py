"""Closed forms and brute force that pin the oracle's solver.

Test infrastructure only (see package docstring).
"""
from __future__ import annotations

import itertools
import numpy as np


def equality_qp(Q, q, A, b):
    """min 1/2 x'Qx + q'x s.t. Ax = b by its KKT system (p = 0 gives
    x = -Q^{-1} q)."""
    n, p = Q.shape[0], A.shape[0]
    K = np.zeros((n + p, n + p))
    K[:n, :n] = Q
    K[:n, n:] = A.T
    K[n:, :n] = A
    sol = np.linalg.solve(K, np.concatenate([-q, b]))
    return sol[:n], sol[n:]


def bruteforce(Q, q, A, b, G, h, feas_tol=1e-9):
    """Active-set enumeration for tiny strictly convex QPs: for every subset
    S of inequality rows with |S| + p <= n, solve the equality QP with rows
    S held at equality; return the (unique) candidate that is primal feasible
    and has non-negative multipliers on S."""
    n, p, m = Q.shape[0], A.shape[0], G.shape[0]
    for k in range(0, min(m, n - p) + 1):
        for S in itertools.combinations(range(m), k):
            S = list(S)
            AS = np.vstack([A, G[S]]) if k else A
            bS = np.concatenate([b, h[S]]) if k else b
            try:
                x, lam = equality_qp(Q, q, AS, bS)
            except np.linalg.LinAlgError:
                continue
            zS = lam[p:]
            if np.all(G @ x <= h + feas_tol) and np.all(zS >= -feas_tol):
                z = np.zeros(m)
                z[S] = zS
                return x, lam[:p], z
    raise RuntimeError("no active set satisfies the KKT conditions")


def box_solution(d, q, lo, hi):
    """Diagonal-Q box QP: x* = clip(-q/d, lo, hi)."""
    return np.clip(-q / d, lo, hi)


def box_relaxed(d, q, lo, hi, kappa, iters=200):
    """Box QP central-path point: per coordinate the barrier equation
    d x + q + kappa/(hi - x) - kappa/(x - lo) = 0, increasing in x on
    (lo, hi), solved by bisection."""
    a, bb = lo.copy(), hi.copy()
    for _ in range(iters):
        mid = 0.5 * (a + bb)
        f = d * mid + q + kappa / (hi - mid) - kappa / (mid - lo)
        bb = np.where(f > 0, mid, bb)
        a = np.where(f > 0, a, mid)
    return 0.5 * (a + bb)


def box_relaxed_dq(d, x, lo, hi, kappa):
    """d x_i / d q_i at the box central-path point: differentiating the
    barrier equation gives -1 / (d + kappa/(hi-x)^2 + kappa/(x-lo)^2), i.e.
    -1 / (d + z_u/s_u + z_l/s_l)."""
    return -1.0 / (d + kappa / (hi - x) ** 2 + kappa / (x - lo) ** 2)


def hard_projection_jacobian(G_act):
    """eq. hard-jacobian: J = I - G_A'(G_A G_A')^{-1} G_A, the orthogonal
    projector onto the tangent space of the active face (appendix D.2)."""
    n = G_act.shape[1]
    return np.eye(n) - G_act.T @ np.linalg.solve(G_act @ G_act.T, G_act)
