"""KKT residuals and Newton matrices, written out from their definitions.

Conventions (section 2.1): x in R^n, G in R^{m x n} (inequalities Gx <= h,
multipliers z, slacks s), A in R^{p x n} (equalities Ax = b, multipliers y).
The Lagrangian is 1/2 x'Qx + q'x + y'(Ax - b) + z'(Gx + s - h), which fixes
the signs of the multiplier terms.

Test infrastructure only (see package docstring).
"""
import numpy as np

from . import retraction as rt


def kkt_residuals(Q, q, A, b, G, h, x, y, z, s):
    """eq. kkt_conditions: stationarity r_t = Qx + q + G'z + A'y,
    complementarity r_c = z*s, inequality r_i = Gx + s - h, equality
    r_e = Ax - b."""
    r_t = Q @ x + q + G.T @ z + A.T @ y
    r_c = z * s
    r_i = G @ x + s - h
    r_e = A @ x - b
    return r_t, r_c, r_i, r_e


def implicit_residuals(z, s, v, kappa):
    """eq. implicit_complementarity_residuals: r_z = z - b_kappa(v),
    r_s = s - b_kappa(-v)."""
    return z - rt.b(v, kappa), s - rt.b(-v, kappa)


def scaled_norms(Q, q, A, b, G, h, x, y, z, s):
    """Scaled infinity norms of the KKT residuals used for the stopping test.

    The paper's test is ||r||_inf < tol without saying which residuals or how
    they are scaled.  Reading used here: each residual block is divided by one
    plus the largest infinity norm of the terms it sums, so the test is
    invariant to the data's scale and reachable in float32."""
    Qx, Gx, Ax = Q @ x, G @ x, A @ x
    Gz, Ay = G.T @ z, A.T @ y
    r_t = Qx + q + Gz + Ay
    r_i = Gx + s - h
    r_e = Ax - b
    ninf = lambda a: float(np.max(np.abs(a))) if a.size else 0.0
    rt_s = ninf(r_t) / (1.0 + max(ninf(Qx), ninf(q), ninf(Gz), ninf(Ay)))
    ri_s = ninf(r_i) / (1.0 + max(ninf(Gx), ninf(s), ninf(h))) if G.shape[0] else 0.0
    re_s = ninf(r_e) / (1.0 + max(ninf(Ax), ninf(b))) if A.shape[0] else 0.0
    return rt_s, ri_s, re_s


def standard_jacobian(Q, A, G, z, s):
    """Newton matrix of the standard (explicit) perturbed KKT system, eq.
    explicit_uncondensed.  Unknown order (dx, dy, dz, ds), row order
    (r_t, r_e, r_i, r_c):

        [ Q  A'  G'    0   ]
        [ A  0   0     0   ]
        [ G  0   0     I   ]
        [ 0  0   D(s)  D(z)]
    """
    n, p, m = Q.shape[0], A.shape[0], G.shape[0]
    N = n + p + 2 * m
    J = np.zeros((N, N), dtype=Q.dtype)
    ix, iy, iz, is_ = slice(0, n), slice(n, n + p), slice(n + p, n + p + m), slice(n + p + m, N)
    J[ix, ix] = Q
    J[ix, iy] = A.T
    J[ix, iz] = G.T
    J[iy, ix] = A
    J[iz, ix] = G
    J[iz, is_] = np.eye(m)
    J[is_, iz] = np.diag(s)
    J[is_, is_] = np.diag(z)
    return J


def implicit_jacobian(Q, A, G, v, kappa):
    """Uncondensed Newton matrix of the implicit-complementarity system,
    eq. implicit_kkt (derived in appendix B.1).  Unknown order
    (dx, dy, dz, ds, dv, dkappa), row order (r_t, r_e, r_i, r_z, r_s, r_kappa):

        [ Q  A'  G'  0   0        0  ]
        [ A  0   0   0   0        0  ]
        [ G  0   0   I   0        0  ]
        [ 0  0   I   0  -B(v)    -c  ]
        [ 0  0   0   I   B(-v)   -c  ]
        [ 0  0   0   0   0        1  ]

    with B(+-v) = Diag(b_kappa'(+-v)) and c = d b_kappa / d kappa (a vector,
    the same for +v and -v)."""
    n, p, m = Q.shape[0], A.shape[0], G.shape[0]
    N = n + p + 3 * m + 1
    J = np.zeros((N, N), dtype=Q.dtype)
    o = np.cumsum([0, n, p, m, m, m, 1])
    X, Y, Z, S, V, K = (slice(o[i], o[i + 1]) for i in range(6))
    J[X, X] = Q
    J[X, Y] = A.T
    J[X, Z] = G.T
    J[Y, X] = A
    J[Z, X] = G
    J[Z, S] = np.eye(m)
    c = rt.db_dkappa(v, kappa)
    J[S, Z] = np.eye(m)                      # row r_z, column dz
    J[S, V] = -np.diag(rt.db_dv(v, kappa))   # row r_z, column dv
    J[S, K] = -c[:, None]
    J[V, S] = np.eye(m)                      # row r_s, column ds
    J[V, V] = np.diag(rt.db_dv(-v, kappa))   # row r_s, column dv
    J[V, K] = -c[:, None]
    J[K, K] = 1.0
    return J, (X, Y, Z, S, V, K)


def reduced_matrix(Q, A, G, v, kappa):
    """Reduced symmetric system of eq. implicit_partially_condensed (appendix
    B.3, second form); unknown order (dx, dv, dy):

        [ Q - G'G   G'       A' ]
        [ G        -B(-v)    0  ]
        [ A         0        0  ]
    """
    n, p, m = Q.shape[0], A.shape[0], G.shape[0]
    K = np.zeros((n + m + p, n + m + p), dtype=Q.dtype)
    K[:n, :n] = Q - G.T @ G
    K[:n, n:n + m] = G.T
    K[:n, n + m:] = A.T
    K[n:n + m, :n] = G
    K[n:n + m, n:n + m] = -np.diag(rt.db_dv(-v, kappa))
    K[n + m:, :n] = A
    return K


def reduced_rhs(r_t, r_e, r_i, r_z, r_s, r_kappa, c, G):
    """Right-hand side of eq. implicit_partially_condensed:
    -[ r_t - G'(r_i + r_z - r_s);  r_i - r_s - c r_kappa;  r_e ]."""
    return -np.concatenate([r_t - G.T @ (r_i + r_z - r_s), r_i - r_s - c * r_kappa, r_e])
