"""Every compiled kernel configuration against the FP64 oracle.

The library instantiates its fused kernels per (threads per QP, rows per
lane in the solves, factor in LDS or in global memory); the launch plan
picks one from the problem size (and `block`, when given).  Each case below
is the smallest random feasible shape whose plan lands on one of the 18
reachable configurations (the plan is asserted, so the case keeps covering
the configuration it names).  For QP 0 of each batch: the solution entry by
entry (x, s, y, z), then the relaxed point and all six gradient blocks,
with the tolerances of tests/parity.py.  Then rescaled inputs (Q, G, A or
q multiplied by powers of ten): every QP converges and two match the
oracle.  Last, batches of tiny QPs (one or a few rows): every QP converges.
"""
import numpy as np
import pytest

import qpgen
from oracle import implicit, gradients

import parity as pt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (threads, rows per lane, factor in LDS) -> (n, m, p)
CASES = {
    (128, 1, True): (2, 1, 0),
    (128, 2, True): (26, 26, 13),
    (128, 2, False): (47, 47, 23),
    (128, 4, True): (56, 896, 28),
    (128, 4, False): (53, 53, 26),
    (128, 8, False): (104, 104, 52),
    (256, 1, True): (2, 1, 0),
    (256, 2, True): (26, 26, 13),
    (256, 2, False): (47, 500, 23),
    (256, 4, True): (53, 53, 26),
    (256, 4, False): (56, 56, 28),
    (256, 8, False): (104, 104, 52),
    (512, 1, True): (2, 1, 0),
    (512, 2, True): (26, 26, 13),
    (512, 4, True): (53, 53, 26),
    (512, 4, False): (146, 37, 73),
    (512, 8, False): (104, 104, 52),
    (512, 16, False): (95, 380, 47),
}
KR = 1e-4


def _rows_per_lane(N):
    r = (N + 63) // 64
    return 1 if r <= 1 else 2 if r <= 2 else 4 if r <= 4 else 8 if r <= 8 else 16


@pytest.mark.parametrize("key", sorted(CASES), ids=lambda k: f"T{k[0]}_rpl{k[1]}_{'lds' if k[2] else 'global'}")
def test_kernel_configuration_vs_oracle(key):
    import paper_2605_17913_amd as qpx
    T, rpl, lds = key
    n, m, p = CASES[key]
    pl = qpx.plan(n, m, p, block=T)
    assert (pl["threads"], _rows_per_lane(n + pl["kb"] + p), pl["factor_in_lds"]) == key, pl
    print(f"configuration {key}: n={n} m={m} p={p} B=3", flush=True)
    P = qpgen.random_feasible(3, n, m, p, seed=100 + n + m + p)
    Td = pt.to_dev(P)
    sol = qpx.solve(*Td, block=T)
    gx = qpgen.upstream(P.B, n, seed=7)
    g = qpx.backward(*Td, sol, torch.from_numpy(gx).to(Td[0].device), kappa_relax=KR,
                     relaxed=True, block=T)
    torch.cuda.synchronize()
    sol, g = pt.npd(sol), pt.npd(g)
    st = pt.outcome(sol["status"])
    assert np.all(st == 0), (key, st.tolist(), sol["iters"].tolist())
    rst = pt.outcome(g["relaxed"]["status"])
    assert np.all(rst == 0), (key, rst.tolist())
    r = implicit.solve_qp(*P.one(0), tol=1e-11, max_iter=200)
    assert r.status == implicit.CONVERGED
    worst = pt.check_point(f"{key} QP 0", P, 0, sol, r)
    ref, rr = gradients.grad_at_relaxed(*P.one(0), KR, gx[0].astype(np.float64))
    worst = max(worst, pt.check_point(f"{key} relaxed QP 0", P, 0, g["relaxed"], rr, tol=1e-6))
    worst = max(worst, pt.check_grads(f"{key} QP 0", g, 0, ref))
    print(f"  iters {sol['iters'].tolist()} worst entry at {worst:.2f} of its bound", flush=True)


# Rescaled inputs: Q multiplied by 1e3 moves the border's pivots (of order
# |A_j|^2 / |Q|) far below the H block's, which each block's own pivot
# scale in the regularisation test keeps from being taken for numerical
# zeros; G (with h) by 1e-2 and q by 1e3 stress the same scales.  G by 1e2
# or A (with b) by 1e-2 puts inequality and equality rows of norms 1e4
# apart in one border, whose equilibration keeps the equality rows' pivots
# from being taken for numerical zeros (without it most of these QPs ended
# at the iteration limit).
RESCALED = [
    ((5, 0, 4), "Q", 1e3),
    ((50, 100, 10), "Q", 1e3),
    ((20, 400, 2), "Q", 1e3),
    ((12, 40, 11), "G", 1e-2),
    ((150, 300, 15), "q", 1e3),
    ((50, 100, 10), "G", 1e2),
    ((150, 300, 15), "G", 1e2),
    ((20, 400, 2), "G", 1e2),
    ((12, 40, 11), "A", 1e-2),
]


@pytest.mark.parametrize("case", RESCALED, ids=lambda c: f"{c[0]}_{c[1]}x{c[2]:g}")
def test_rescaled_inputs_vs_oracle(case):
    import paper_2605_17913_amd as qpx
    (n, m, p), which, f = case
    print(f"rescaled {which} x {f:g}: n={n} m={m} p={p} B=4", flush=True)
    P = qpgen.random_feasible(4, n, m, p, seed=1000 + n + m + p)
    getattr(P, which)[...] *= np.float32(f)
    if which == "G":  # the planted point stays strictly feasible
        P.h[...] *= np.float32(f)
    if which == "A":  # and on the equality constraints
        P.b[...] *= np.float32(f)
    sol = pt.npd(qpx.solve(*pt.to_dev(P)))
    st = pt.outcome(sol["status"])
    assert np.all(st == 0), (case, st.tolist(), sol["iters"].tolist())
    for i in (0, 1):
        r = implicit.solve_qp(*P.one(i), tol=1e-11, max_iter=300)
        assert r.status == implicit.CONVERGED
        worst = pt.check_point(f"{case} QP {i}", P, i, sol, r)
        print(f"  QP {i}: worst entry at {worst:.2f} of its bound", flush=True)


# Tiny QPs: with one inactive row the corrector's target kappa_t can lie far
# below kappa's rounding unit, and a full step kappa + (kappa_t - kappa) then
# rounded to exactly zero (z of the inactive row became 0 and the next
# centering step divided by kappa = 0: "non-finite value" on about 0.5% of
# these QPs).  Every QP of these batches converges, and QP 0 of each matches
# the oracle.
@pytest.mark.parametrize("shape", [(1, 1, 0), (2, 1, 0), (1, 3, 0), (5, 5, 0)],
                         ids=lambda s: "n%d_m%d_p%d" % s)
def test_tiny_qps_converge(shape):
    import paper_2605_17913_amd as qpx
    n, m, p = shape
    print(f"tiny QPs n={n} m={m} p={p}: 20 batches of 64", flush=True)
    for seed in range(20):
        P = qpgen.random_feasible(64, n, m, p, seed=seed)
        sol = pt.npd(qpx.solve(*pt.to_dev(P)))
        st = pt.outcome(sol["status"])
        assert np.all(st == 0), (shape, seed, [qpx.result_string(int(s)) for s in sol["status"][st != 0]])
        if seed < 2:
            r = implicit.solve_qp(*P.one(0), tol=1e-11, max_iter=200)
            assert r.status == implicit.CONVERGED
            pt.check_point(f"{shape} seed {seed} QP 0", P, 0, sol, r)
