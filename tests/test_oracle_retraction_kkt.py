"""Pins for the oracle's retraction map and KKT matrices.

Each check compares the oracle with something the mathematics fixes:
closed-form identities of the softplus retraction (section 4.1, appendix C),
finite-difference Jacobians of the residual maps (so any wrong sign, index
or transposed block in the Newton matrices fails), and the equivalence of
the uncondensed and reduced systems (section 4.2, appendix B.3).
"""
import numpy as np
import pytest

from oracle import retraction as rt, kkt
import qpgen

KAPPAS = [1e-12, 1e-8, 1e-4, 1e-2, 1.0]
VS = np.concatenate([-np.logspace(-6, 6, 49), [0.0], np.logspace(-6, 6, 49)])


@pytest.mark.parametrize("kappa", KAPPAS)
def test_product_identity(kappa):
    # eq. retraction_map: b(v) b(-v) = kappa
    prod = rt.b(VS, kappa) * rt.b(-VS, kappa)
    np.testing.assert_allclose(prod, kappa, rtol=1e-13)
    assert np.all(rt.b(VS, kappa) > 0)


@pytest.mark.parametrize("kappa", KAPPAS)
def test_branch_form_equals_definition(kappa):
    # appendix C: the branch form equals eq. softplus where the latter is exact
    v = VS[np.abs(VS) <= 10 * np.sqrt(kappa)]
    np.testing.assert_allclose(rt.b(v, kappa), rt.b_plain(v, kappa), rtol=1e-12)
    vp = VS[VS >= 0]
    np.testing.assert_array_equal(rt.b(vp, kappa), rt.b_plain(vp, kappa))
    # sum and difference: b(v) + b(-v) = sqrt(v^2+4k), b(v) - b(-v) = v
    np.testing.assert_allclose(rt.b(VS, kappa) - rt.b(-VS, kappa), VS, rtol=1e-12,
                               atol=1e-14 * np.sqrt(kappa))


@pytest.mark.parametrize("kappa", [1e-4, 1e-2, 1.0])
def test_derivatives_match_finite_differences(kappa):
    v = np.linspace(-3, 3, 61) * np.sqrt(kappa) * 4
    hv = 1e-6 * np.sqrt(kappa)
    fd_v = (rt.b_plain(v + hv, kappa) - rt.b_plain(v - hv, kappa)) / (2 * hv)
    np.testing.assert_allclose(rt.db_dv(v, kappa), fd_v, rtol=1e-7, atol=1e-12)
    hk = 1e-6 * kappa
    fd_k = (rt.b_plain(v, kappa + hk) - rt.b_plain(v, kappa - hk)) / (2 * hk)
    np.testing.assert_allclose(rt.db_dkappa(v, kappa), fd_k, rtol=1e-6)


@pytest.mark.parametrize("kappa", KAPPAS)
def test_derivative_properties(kappa):
    # eq. softplus_properties: db(v) + db(-v) = 1 and 0 < db <= 1
    d1, d2 = rt.db_dv(VS, kappa), rt.db_dv(-VS, kappa)
    np.testing.assert_allclose(d1 + d2, 1.0, rtol=1e-12)
    assert np.all(d1 > 0) and np.all(d1 <= 1)
    # at v = 0 both branches give 1/2 (continuity)
    assert rt.db_dv(np.array([0.0]), kappa)[0] == 0.5
    np.testing.assert_allclose(rt.db_dv(np.array([-1e-300]), kappa), 0.5, rtol=1e-12)


def _point(n=4, m=6, p=2, seed=0):
    P = qpgen.random_feasible(1, n, m, p, seed).one(0)
    rng = np.random.default_rng(seed + 100)
    x, y = rng.standard_normal(n), rng.standard_normal(p)
    z, s = rng.uniform(0.2, 2, m), rng.uniform(0.2, 2, m)
    v, kappa = rng.standard_normal(m), 0.3
    return P, x, y, z, s, v, kappa


def _fd_jacobian(f, w, h=1e-6):
    f0 = f(w)
    J = np.zeros((f0.size, w.size))
    for j in range(w.size):
        e = np.zeros_like(w)
        e[j] = h
        J[:, j] = (f(w + e) - f(w - e)) / (2 * h)
    return J


def test_implicit_jacobian_is_the_residual_jacobian():
    # eq. implicit_kkt must be the Jacobian of (r_t, r_e, r_i, r_z, r_s, r_kappa)
    # with respect to (x, y, z, s, v, kappa)
    (Q, q, A, b, G, h), x, y, z, s, v, kappa = _point()
    n, p, m = 4, 2, 6
    kt = 0.05

    def R(w):
        o = np.cumsum([0, n, p, m, m, m, 1])
        xx, yy, zz, ss, vv, kk = (w[o[i]:o[i + 1]] for i in range(6))
        r_t, _, r_i, r_e = kkt.kkt_residuals(Q, q, A, b, G, h, xx, yy, zz, ss)
        r_z, r_s = kkt.implicit_residuals(zz, ss, vv, kk[0])
        return np.concatenate([r_t, r_e, r_i, r_z, r_s, [kk[0] - kt]])

    w = np.concatenate([x, y, z, s, v, [kappa]])
    J, _ = kkt.implicit_jacobian(Q, A, G, v, kappa)
    np.testing.assert_allclose(J, _fd_jacobian(R, w), atol=1e-7)


def test_standard_jacobian_is_the_residual_jacobian():
    (Q, q, A, b, G, h), x, y, z, s, _, kappa = _point(seed=1)
    n, p, m = 4, 2, 6

    def R(w):
        o = np.cumsum([0, n, p, m, m])
        xx, yy, zz, ss = (w[o[i]:o[i + 1]] for i in range(4))
        r_t, r_c, r_i, r_e = kkt.kkt_residuals(Q, q, A, b, G, h, xx, yy, zz, ss)
        return np.concatenate([r_t, r_e, r_i, r_c - kappa])

    w = np.concatenate([x, y, z, s])
    np.testing.assert_allclose(kkt.standard_jacobian(Q, A, G, z, s), _fd_jacobian(R, w), atol=1e-7)


def test_stationarity_is_the_lagrangian_gradient():
    # r_t = grad_x L with L = 1/2 x'Qx + q'x + y'(Ax-b) + z'(Gx+s-h)
    (Q, q, A, b, G, h), x, y, z, s, _, _ = _point(seed=2)
    L = lambda xx: 0.5 * xx @ Q @ xx + q @ xx + y @ (A @ xx - b) + z @ (G @ xx + s - h)
    fd = _fd_jacobian(lambda xx: np.array([L(xx)]), x)[0]
    r_t, _, _, _ = kkt.kkt_residuals(Q, q, A, b, G, h, x, y, z, s)
    np.testing.assert_allclose(r_t, fd, atol=1e-7)


@pytest.mark.parametrize("seed", range(4))
def test_reduced_system_gives_the_uncondensed_step(seed):
    # appendix B.3: the reduced symmetric system yields the same Newton step
    (Q, q, A, b, G, h), x, y, z, s, v, kappa = _point(n=5, m=8, p=2, seed=seed)
    n, p, m = 5, 2, 8
    kt = 0.1 * kappa
    J, sl = kkt.implicit_jacobian(Q, A, G, v, kappa)
    r_t, _, r_i, r_e = kkt.kkt_residuals(Q, q, A, b, G, h, x, y, z, s)
    r_z, r_s = kkt.implicit_residuals(z, s, v, kappa)
    d = np.linalg.solve(J, -np.concatenate([r_t, r_e, r_i, r_z, r_s, [kappa - kt]]))
    K = kkt.reduced_matrix(Q, A, G, v, kappa)
    np.testing.assert_allclose(K, K.T)  # symmetric (section 4.2, property (i))
    c = rt.db_dkappa(v, kappa)
    red = np.linalg.solve(K, kkt.reduced_rhs(r_t, r_e, r_i, r_z, r_s, kappa - kt, c, G))
    np.testing.assert_allclose(red[:n], d[sl[0]], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(red[n:n + m], d[sl[4]], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(red[n + m:], d[sl[1]], rtol=1e-9, atol=1e-11)
    # the middle block is diagonal with entries in (0, 1)
    mid = -np.diag(K[n:n + m, n:n + m])
    assert np.all(mid > 0) and np.all(mid < 1)
