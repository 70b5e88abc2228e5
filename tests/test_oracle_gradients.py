"""Pins for the oracle's implicit-function-theorem gradients: closed forms
(unconstrained, box, projection), the hard-projection limit (appendix D.2)
and central finite differences of the relaxed map for all six blocks."""
import numpy as np
import pytest

import qpgen
from oracle import implicit, gradients, reference


def test_unconstrained_gradient_closed_form():
    P = qpgen.random_feasible(2, 6, 0, 0, seed=1)
    g = np.random.default_rng(0).standard_normal(6)
    for i in range(2):
        Q, q, A, b, G, h = P.one(i)
        x = -np.linalg.solve(Q, q)
        gr = gradients.ift_vjp(Q, q, A, b, G, h, x, np.zeros(0), np.zeros(0), np.zeros(0), g)
        dx = -np.linalg.solve(Q, g)  # x = -Q^{-1} q  =>  dl/dq = -Q^{-1} g
        np.testing.assert_allclose(gr["q"], dx, rtol=1e-10)
        np.testing.assert_allclose(gr["Q"], 0.5 * (np.outer(dx, x) + np.outer(x, dx)), rtol=1e-10)


@pytest.mark.parametrize("kappa_relax", [1e-1, 1e-3])
def test_box_gradient_closed_form(kappa_relax):
    P = qpgen.box_qp(3, 5, seed=2)
    g = np.random.default_rng(1).standard_normal(5)
    for i in range(3):
        Q, q, A, b, G, h = P.one(i)
        gr, rr = gradients.grad_at_relaxed(Q, q, A, b, G, h, kappa_relax, g)
        d, lo, hi = P.extra["d"][i], P.extra["lo"][i], P.extra["hi"][i]
        xr = reference.box_relaxed(d, q, lo, hi, kappa_relax)
        np.testing.assert_allclose(gr["q"], g * reference.box_relaxed_dq(d, xr, lo, hi, kappa_relax),
                                   rtol=1e-8)


def test_projection_gradient_tends_to_hard_jacobian():
    # Q = I, q = -x_query: d(v'Pi(x))/dx = -grad_q.  At kappa_relax -> 0 it
    # approaches J_hard v on a strictly complementary instance.
    P = qpgen.projection(2, 6, 8, 3, d=1.0, seed=4)
    vprobe = np.random.default_rng(3).standard_normal(6)
    for i in range(2):
        Q, q, A, b, G, h = P.one(i)
        Jh = reference.hard_projection_jacobian(G[:3])
        errs = []
        for kr in [1e-2, 1e-4, 1e-6, 1e-8]:
            gr, rr = gradients.grad_at_relaxed(Q, q, A, b, G, h, kr, vprobe)
            g_soft = -gr["q"]
            # closed form at the relaxed point: (I + G' diag(z/s) G)^{-1} v
            M = np.eye(6) + G.T @ np.diag(rr.z / rr.s) @ G
            np.testing.assert_allclose(g_soft, np.linalg.solve(M, vprobe), rtol=1e-6, atol=1e-10)
            errs.append(np.linalg.norm(g_soft - Jh @ vprobe))
        assert errs[-1] < 1e-5 and errs[0] > errs[-1]
        assert all(a >= b for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("seed", range(3))
def test_gradients_match_central_differences(seed):
    n, m, p = [(5, 8, 2), (6, 10, 1), (4, 7, 0)][seed]
    P = qpgen.random_feasible(1, n, m, p, seed=20 + seed)
    Q, q, A, b, G, h = P.one(0)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n)
    kr = 1e-2
    gr, rr = gradients.grad_at_relaxed(Q, q, A, b, G, h, kr, g)
    warm = (rr.x, rr.y, rr.z, rr.s)
    for key, shape in [("Q", (n, n)), ("q", (n,)), ("A", (p, n)), ("b", (p,)),
                       ("G", (m, n)), ("h", (m,))]:
        if 0 in shape:
            continue
        for _ in range(2):
            D = rng.standard_normal(shape)
            if key == "Q":
                D = 0.5 * (D + D.T)
            fd = gradients.fd_vjp(Q, q, A, b, G, h, kr, g, {key: D}, 1e-5, warm)
            an = float(np.sum(gr[key] * D))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (key, fd, an)


@pytest.mark.parametrize("seed", range(2))
def test_full_vjp_matches_central_differences(seed):
    # upstream on all three outputs: l = gx'x + gy'y + gz'z at the relaxed
    # point (the multipliers are unique there for kappa_relax > 0 and A of
    # full row rank)
    n, m, p = [(5, 8, 2), (6, 9, 1)][seed]
    P = qpgen.random_feasible(1, n, m, p, seed=40 + seed)
    Q, q, A, b, G, h = P.one(0)
    rng = np.random.default_rng(100 + seed)
    gx, gy, gz = rng.standard_normal(n), rng.standard_normal(p), rng.standard_normal(m)
    kr = 1e-2
    gr, rr = gradients.grad_at_relaxed(Q, q, A, b, G, h, kr, gx, gy, gz)
    warm = (rr.x, rr.y, rr.z, rr.s)
    for key, shape in [("Q", (n, n)), ("q", (n,)), ("A", (p, n)), ("b", (p,)),
                       ("G", (m, n)), ("h", (m,))]:
        D = rng.standard_normal(shape)
        if key == "Q":
            D = 0.5 * (D + D.T)
        fd = gradients.fd_vjp(Q, q, A, b, G, h, kr, gx, {key: D}, 1e-5, warm, gy=gy, gz=gz)
        an = float(np.sum(gr[key] * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (key, fd, an)


def test_safety_filter_shapes_and_feasibility():
    # appendix F shapes: 2 N_a variables, 4 N_a + 3 N_a + N_a (N_a - 1) / 2 rows
    for na in (1, 4, 9):
        P = qpgen.safety_filter(3, na, seed=na)
        n, m = 2 * na, 7 * na + na * (na - 1) // 2
        assert P.Q.shape == (3, n, n) and P.G.shape == (3, m, n) and P.A.shape == (3, 0, n)
        u0 = P.extra["u0"]
        slack = P.h.astype(np.float64) - np.einsum("bmn,bn->bm", P.G.astype(np.float64), u0)
        assert np.all(slack > 0.04)
        r = implicit.solve_qp(*P.one(0))
        assert r.status == implicit.CONVERGED


def test_scalar_qp_golden():
    # tests/golden/scalar_qp.json: a one-variable QP worked by hand
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "scalar_qp.json")))
    Q, q, G, h = (np.array(d[k], dtype=float) for k in ("Q", "q", "G", "h"))
    A, b = np.zeros((0, 1)), np.zeros(0)
    r = implicit.solve_qp(Q, q, A, b, G, h)
    np.testing.assert_allclose(r.x, d["x_star"], atol=1e-11)
    np.testing.assert_allclose(r.z, d["z_star"], atol=1e-11)
    for cp in d["central_path"]:
        gr, rr = gradients.grad_at_relaxed(Q, q, A, b, G, h, cp["kappa"], np.array([1.0]))
        np.testing.assert_allclose(rr.x, [cp["x"]], rtol=1e-12)
        np.testing.assert_allclose(rr.s, [cp["s"]], rtol=1e-10)
        np.testing.assert_allclose(gr["q"], [cp["dx_dq"]], rtol=1e-9)
        np.testing.assert_allclose(gr["h"], [cp["dx_dh"]], rtol=1e-9)


def test_ift_matches_finite_differences_at_differentiation_shape():
    # the differentiation workload's shape (n=100, m=200, p=20), at the step
    # the workload names for its finite-difference check (1e-3) and at
    # kappa_relax = 1e-4: central differences of the relaxed map along one
    # unit-norm random direction per parameter block (symmetric for Q)
    # agree with the IFT product to better than 1e-4 relative (measured
    # truncation at this step: <= 6e-5)
    P = qpgen.make_config("differentiation", seed=0, B=1)
    prob = P.one(0)
    gx = qpgen.upstream(1, P.n, seed=11)[0].astype(np.float64)
    ref, rr = gradients.grad_at_relaxed(*prob, 1e-4, gx)
    warm = (rr.x, rr.y, rr.z, rr.s)
    rng = np.random.default_rng(7)
    for k, key in enumerate(("Q", "q", "A", "b", "G", "h")):
        D = rng.standard_normal(np.shape(prob[k]))
        if key == "Q":
            D = 0.5 * (D + D.T)
        D /= np.linalg.norm(D)
        fd = gradients.fd_vjp(*prob, 1e-4, gx, {key: D}, 1e-3, warm)
        ift = float(np.sum(ref[key] * D))
        assert abs(fd - ift) <= 1e-4 * max(abs(ift), 1e-3 * np.linalg.norm(ref[key])), (key, fd, ift)
