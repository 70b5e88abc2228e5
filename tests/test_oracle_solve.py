"""Pins for the oracle's solvers (Algorithm 1, Algorithm 2, standard IPM)
against closed forms, brute-force active sets and KKT invariants."""
import numpy as np
import pytest

import qpgen
from oracle import implicit, standard, reference, retraction as rt, kkt


def _rel(a, b):
    return np.linalg.norm(a - b) / max(1.0, np.linalg.norm(b))


@pytest.mark.parametrize("pc", [True, False])
def test_unconstrained_closed_form(pc):
    P = qpgen.random_feasible(3, 7, 0, 0, seed=5)
    for i in range(3):
        Q, q, A, b, G, h = P.one(i)
        r = implicit.solve_qp(Q, q, A, b, G, h, pc=pc)
        np.testing.assert_allclose(r.x, -np.linalg.inv(Q) @ q, rtol=1e-9)


def test_equality_only_closed_form():
    P = qpgen.random_feasible(3, 7, 0, 3, seed=6)
    for i in range(3):
        Q, q, A, b, G, h = P.one(i)
        r = implicit.solve_qp(Q, q, A, b, G, h)
        x, y = reference.equality_qp(Q, q, A, b)
        np.testing.assert_allclose(r.x, x, rtol=1e-9)
        np.testing.assert_allclose(r.y, y, rtol=1e-9)
        np.testing.assert_allclose(A @ r.x, b, atol=1e-10)


@pytest.mark.parametrize("solver", ["implicit_pc", "implicit_sigma", "standard"])
def test_box_qp_clip(solver):
    P = qpgen.box_qp(6, 5, seed=7)
    for i in range(P.B):
        Q, q, A, b, G, h = P.one(i)
        if solver == "standard":
            r = standard.solve_qp(Q, q, A, b, G, h)
        else:
            r = implicit.solve_qp(Q, q, A, b, G, h, pc=(solver == "implicit_pc"))
        assert r.status == implicit.CONVERGED
        xs = reference.box_solution(P.extra["d"][i], q, P.extra["lo"][i], P.extra["hi"][i])
        np.testing.assert_allclose(r.x, xs, atol=1e-9)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("solver", ["implicit_pc", "implicit_sigma", "standard"])
def test_bruteforce_active_set(seed, solver):
    n, m, p = [(3, 6, 0), (4, 8, 1), (5, 10, 1), (6, 12, 2), (4, 12, 0), (6, 9, 3)][seed]
    P = qpgen.random_feasible(2, n, m, p, seed=100 + seed)
    for i in range(2):
        prob = P.one(i)
        if solver == "standard":
            r = standard.solve_qp(*prob)
        else:
            r = implicit.solve_qp(*prob, pc=(solver == "implicit_pc"))
        assert r.status == implicit.CONVERGED
        xb, yb, zb = reference.bruteforce(*prob)
        np.testing.assert_allclose(r.x, xb, atol=1e-8)
        np.testing.assert_allclose(r.z, zb, atol=1e-7)
        if p:
            np.testing.assert_allclose(r.y, yb, atol=1e-7)


def test_invariants_on_the_manifold():
    # after a retraction z*s = kappa elementwise and s'z = m kappa (eq. retraction_map)
    P = qpgen.make_config("plain", seed=0, B=8)
    for i in range(8):
        Q, q, A, b, G, h = P.one(i)
        r = implicit.solve_qp(Q, q, A, b, G, h, tol=1e-9)
        assert r.status == implicit.CONVERGED
        assert np.all(r.s > 0) and np.all(r.z > 0)
        np.testing.assert_allclose(r.z * r.s, np.mean(r.z * r.s), rtol=1e-9)
        r_t, r_c, r_i, r_e = kkt.kkt_residuals(Q, q, A, b, G, h, r.x, r.y, r.z, r.s)
        assert np.max(np.abs(r_t)) < 1e-7 and np.max(np.abs(r_i)) < 1e-8


def test_implicit_and_standard_agree():
    P = qpgen.random_feasible(4, 20, 40, 4, seed=11)
    for i in range(4):
        prob = P.one(i)
        a = implicit.solve_qp(*prob)
        s = standard.solve_qp(*prob)
        assert a.status == s.status == implicit.CONVERGED
        assert _rel(a.x, s.x) < 1e-9
        assert np.max(np.abs(a.z - s.z)) < 1e-7


def test_planted_optimum_of_the_degenerate_recipe():
    P = qpgen.ill_conditioned(2, 16, 32, 2, seed=3)
    for i in range(2):
        r = implicit.solve_qp(*P.one(i), tol=1e-11, max_iter=200)
        assert r.status == implicit.CONVERGED
        assert _rel(r.x, P.extra["x_star"][i]) < 1e-4  # inputs are float32-rounded


def test_projection_recipe_hits_the_planted_point():
    P = qpgen.projection(3, 8, 10, 4, d=1.0, seed=2)
    for i in range(3):
        r = implicit.solve_qp(*P.one(i), tol=1e-11)
        assert _rel(r.x, P.extra["y0"][i]) < 1e-5


@pytest.mark.parametrize("kappa_relax", [1e-1, 1e-2, 1e-4])
def test_relax_box_barrier_equation(kappa_relax):
    # Algorithm 2 lands on the central path point; for a box QP it solves
    # d x + q + k/(hi - x) - k/(x - lo) = 0 coordinate-wise
    P = qpgen.box_qp(4, 6, seed=9)
    for i in range(P.B):
        Q, q, A, b, G, h = P.one(i)
        r = implicit.solve_qp(Q, q, A, b, G, h)
        rr = implicit.relax_qp(Q, q, A, b, G, h, r.x, r.y, r.z, r.s, kappa_relax)
        assert rr.status == implicit.CONVERGED
        xr = reference.box_relaxed(P.extra["d"][i], q, P.extra["lo"][i], P.extra["hi"][i], kappa_relax)
        np.testing.assert_allclose(rr.x, xr, atol=1e-10)
        np.testing.assert_allclose(rr.z * rr.s, kappa_relax, rtol=1e-10)


def test_relax_implicit_equals_standard_central_path():
    P = qpgen.random_feasible(3, 10, 20, 2, seed=4)
    for i in range(3):
        prob = P.one(i)
        r = implicit.solve_qp(*prob)
        a = implicit.relax_qp(*prob, r.x, r.y, r.z, r.s, 1e-3)
        s = standard.relax_qp(*prob, r.x, r.y, r.z, r.s, 1e-3)
        assert a.status == s.status == implicit.CONVERGED
        np.testing.assert_allclose(a.x, s.x, atol=1e-9)
        np.testing.assert_allclose(a.z, s.z, atol=1e-9)


def test_linesearch_definition():
    s = np.array([1.0, 2.0, 0.5])
    z = np.array([1.0, 1.0, 1.0])
    ds = np.array([-2.0, 1.0, 0.0])
    dz = np.array([0.0, -4.0, 1.0])
    assert implicit.linesearch(s, z, ds, dz) == 0.25
    assert implicit.linesearch(s, z, np.abs(ds), np.abs(dz)) == 1.0


def test_infeasible_qp_is_not_reported_converged():
    # x <= -1 and -x <= -1 (x >= 1): empty feasible set
    Q = np.eye(1)
    q = np.zeros(1)
    G = np.array([[1.0], [-1.0]])
    h = np.array([-1.0, -1.0])
    r = implicit.solve_qp(Q, q, np.zeros((0, 1)), np.zeros(0), G, h, max_iter=50)
    assert r.status != implicit.CONVERGED
