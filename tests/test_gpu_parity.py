"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances (float32 path vs float64 oracle on identical float32 inputs):
  x        ||x - x*||_2 / max(1, ||x*||_2) <= 1e-4
  y, z     ||d - d*||_inf / max(1, ||d*||_inf) <= 1e-3 (duals are unique here)
  grads    ||g - g*||_2 / max(1e-3, ||g*||_2) <= 1e-3 per parameter block
The stopping tolerance is 1e-5 on the scaled residuals (the reading of the
paper's ||r||_inf < tol that float32 can reach).
"""
import numpy as np
import pytest

import qpgen
from oracle import implicit, standard, gradients

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _to_dev(P):
    d = _dev()
    return [torch.from_numpy(a).to(d) for a in P.arrays()]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(1.0, np.linalg.norm(b)))


def _oracle_solutions(P, idx, tol=1e-11):
    out = []
    for i in idx:
        r = implicit.solve_qp(*P.one(i), tol=tol, max_iter=200)
        assert r.status == implicit.CONVERGED
        out.append(r)
    return out


def _run(P, **kw):
    import paper_2605_17913_amd as qpx
    Q, q, A, b, G, h = _to_dev(P)
    sol = qpx.solve(Q, q, A, b, G, h, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in sol.items()}


def _check_solution(P, sol, idx, xtol=1e-4, dtol=1e-3):
    ref = _oracle_solutions(P, idx)
    worst = 0.0
    for k, i in enumerate(idx):
        r = ref[k]
        ex = _rel(sol["x"][i], r.x)
        worst = max(worst, ex)
        assert ex <= xtol, (i, ex)
        if P.m:
            ez = np.max(np.abs(sol["z"][i] - r.z)) / max(1.0, np.max(np.abs(r.z)))
            assert ez <= dtol, (i, ez)
        if P.p:
            ey = np.max(np.abs(sol["y"][i] - r.y)) / max(1.0, np.max(np.abs(r.y)))
            assert ey <= dtol, (i, ey)
    return worst


@pytest.mark.parametrize("pc", [True, False])
def test_plain_config_bounded(pc):
    P = qpgen.make_config("plain", seed=0)
    sol = _run(P, pc=pc)
    assert np.all(sol["status"] == 0), sol["status"]
    _check_solution(P, sol, range(P.B))


def test_plain_config_tail_and_ragged_sizes():
    # sizes that are not multiples of the tile / panel widths
    for (n, m, p, seed) in [(7, 13, 1, 1), (17, 35, 3, 2), (33, 70, 5, 3), (3, 1, 0, 4)]:
        P = qpgen.random_feasible(9, n, m, p, seed)
        sol = _run(P)
        assert np.all(sol["status"] == 0), (n, m, p, sol["status"])
        _check_solution(P, sol, range(P.B))


def test_box_qp_closed_form():
    P = qpgen.box_qp(32, 12, seed=3)
    sol = _run(P)
    assert np.all(sol["status"] == 0)
    for i in range(P.B):
        xs = np.clip(-P.q[i] / P.extra["d"][i], P.extra["lo"][i], P.extra["hi"][i])
        assert np.max(np.abs(sol["x"][i] - xs)) < 1e-4


def test_unconstrained_and_equality_only():
    P = qpgen.random_feasible(8, 12, 0, 0, seed=5)
    sol = _run(P)
    assert np.all(sol["status"] == 0)
    for i in range(P.B):
        Q, q, A, b, G, h = P.one(i)
        assert _rel(sol["x"][i], -np.linalg.solve(Q, q)) < 1e-4
    P = qpgen.random_feasible(8, 12, 0, 4, seed=6)
    sol = _run(P)
    assert np.all(sol["status"] == 0)
    _check_solution(P, sol, range(P.B))


def test_standard_arm_on_plain_config():
    # the explicit arm runs on the same inputs; in FP32 it may fail on some
    # QPs (the paper's point) but every converged QP must be right
    P = qpgen.make_config("plain", seed=0)
    sol = _run(P, form="standard")
    ok = np.where(sol["status"] == 0)[0]
    assert len(ok) > 0
    ref = _oracle_solutions(P, ok)
    for k, i in enumerate(ok):
        assert _rel(sol["x"][i], ref[k].x) <= 1e-3


def test_throughput_config_sampled():
    P = qpgen.make_config("throughput", seed=0)
    sol = _run(P)
    bad = np.where(sol["status"] != 0)[0]
    assert len(bad) == 0, [(int(i), int(sol["status"][i]), int(sol["iters"][i])) for i in bad[:8]]
    idx = np.random.default_rng(0).choice(P.B, 12, replace=False)
    _check_solution(P, sol, idx)


def test_deterministic_and_batch_order_invariant():
    P = qpgen.random_feasible(40, 20, 40, 4, seed=7)
    a = _run(P)
    b = _run(P)
    for k in ("x", "y", "z", "s", "iters"):
        assert np.array_equal(a[k], b[k]), k
    perm = np.random.default_rng(1).permutation(P.B)
    c = _run(P.subset(perm))
    for k in ("x", "z", "iters"):
        assert np.array_equal(a[k][perm], c[k]), k


def test_deterministic_global_factor_path():
    # n=100, m=200, p=20 puts the bordered factor in global memory
    P = qpgen.random_feasible(16, 100, 200, 20, seed=8)
    a = _run(P)
    b = _run(P)
    for k in ("x", "z", "iters", "status"):
        assert np.array_equal(a[k], b[k]), k
    assert np.all(a["status"] == 0)
    _check_solution(P, a, [0, 5, 15])


def test_empty_batch():
    import paper_2605_17913_amd as qpx
    d = _dev()
    Q = torch.zeros(0, 4, 4, device=d)
    sol = qpx.solve(Q, torch.zeros(0, 4, device=d), None, None,
                    torch.zeros(0, 3, 4, device=d), torch.zeros(0, 3, device=d))
    assert sol["x"].shape == (0, 4)


def _grads_check(P, kr, gtol=1e-3, idx=None):
    import paper_2605_17913_amd as qpx
    Q, q, A, b, G, h = _to_dev(P)
    sol = qpx.solve(Q, q, A, b, G, h, tol=1e-6)
    gx_np = qpgen.upstream(P.B, P.n, seed=11)
    gx = torch.from_numpy(gx_np).to(Q.device)
    g = qpx.backward(Q, q, A, b, G, h, sol, gx, kappa_relax=kr, relaxed=True)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if not isinstance(v, dict) else {kk: vv.cpu().numpy() for kk, vv in v.items()})
         for k, v in g.items()}
    idx = range(P.B) if idx is None else idx
    for i in idx:
        ref, rr = gradients.grad_at_relaxed(*P.one(i), kr, gx_np[i].astype(np.float64))
        assert _rel(g["relaxed"]["x"][i], rr.x) <= 1e-4
        for key in ("Q", "q", "A", "b", "G", "h"):
            if ref[key].size == 0:
                continue
            err = np.linalg.norm(g[key][i] - ref[key]) / max(1e-3, np.linalg.norm(ref[key]))
            assert err <= gtol, (i, key, err)


@pytest.mark.parametrize("kr", [1e-2, 1e-4])
def test_backward_plain_config(kr):
    P = qpgen.random_feasible(16, 10, 20, 2, seed=9)
    _grads_check(P, kr)


def test_backward_differentiation_shape_sampled():
    P = qpgen.random_feasible(64, 100, 200, 20, seed=2)
    _grads_check(P, 1e-4, idx=[0, 17, 63])
