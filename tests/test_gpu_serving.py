"""GPU tests of the serving loop: continuous batching of single QPs of
uneven sizes over the serving workload's full range (n ~ U{8..256}, m = 2n,
p = floor(n/10)), which covers every size-class bucket: 128, 256 and
512 threads per QP, the factor in LDS and in global memory.

A request must give the same result alone and in a mix (bitwise: each QP's
arithmetic is independent, and resuming from the stored iterate and
arithmetic state repeats an uninterrupted solve), equal to qp_solve on a
batch of one (bitwise), and within the parity tolerances of the FP64 oracle
(entry by entry, tests/parity.py)."""
import numpy as np
import pytest

import qpgen
from oracle import implicit

import parity as pt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests(count, seed, n_lo=8, n_hi=256):
    reqs = []
    for (n, m, p, sd) in qpgen.serving_requests(count, seed, n_lo, n_hi):
        reqs.append(qpgen.random_feasible(1, n, m, p, sd % (2**31)))
    return reqs


def _args(P):
    return (P.Q[0], P.q[0], P.A[0] if P.p else None, P.b[0] if P.p else None,
            P.G[0] if P.m else None, P.h[0] if P.m else None)


def test_serving_alone_equals_mix_equals_batch_and_oracle():
    import paper_2605_17913_amd as qpx
    d = pt.dev()
    reqs = _requests(24, seed=3)
    # make sure the extremes of the range are in the mix
    reqs[0] = qpgen.random_feasible(1, 256, 512, 25, 901)
    reqs[1] = qpgen.random_feasible(1, 8, 16, 0, 902)
    plans = {(P.n, P.m, P.p): qpx.plan(P.n, P.m, P.p) for P in reqs}
    buckets = {(pl["threads"], pl["factor_in_lds"]) for pl in plans.values()}
    print(f"serving: {len(reqs)} requests, n {min(P.n for P in reqs)}..{max(P.n for P in reqs)}, "
          f"buckets (threads, factor in LDS) {sorted(buckets)}", flush=True)
    assert {128, 256, 512} <= {b[0] for b in buckets}
    assert {True, False} <= {b[1] for b in buckets}
    with qpx.Server(max_slots=8, iters_per_step=3, arena_bytes=256 << 20) as srv:
        alone = [srv.wait(srv.submit(*_args(P)), timeout=120) for P in reqs[:6]]
        tickets = [srv.submit(*_args(P)) for P in reqs]  # arrive while others run
        mix = [srv.wait(t, timeout=300) for t in tickets]
        st = srv.stats()
    assert st["peak_resident"] <= 8 and st["completed"] == 30
    for a, b in zip(alone, mix[:6]):
        for k in ("x", "y", "z", "s"):
            assert np.array_equal(a[k], b[k]), k
        assert a["iters"] == b["iters"] and a["status"] == b["status"]
    worst = 0.0
    for j, (P, r) in enumerate(zip(reqs, mix)):
        assert pt.outcome(r["status"]) == 0, (j, r["status"])
        sol = pt.npd(qpx.solve(*[torch.from_numpy(a).to(d) for a in P.arrays()]))
        for k in ("x", "y", "z", "s"):
            assert np.array_equal(sol[k][0], r[k]), (j, k)
        assert int(sol["iters"][0]) == r["iters"] and int(sol["status"][0]) == r["status"]
        ref = implicit.solve_qp(*P.one(0), tol=1e-11, max_iter=200)
        worst = max(worst, pt.check_point(f"request {j} (n={P.n})", P, 0,
                                          {k: r[k][None] for k in ("x", "y", "z", "s")}, ref))
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    print(f"serving: worst entry at {worst:.2f} of its bound", flush=True)


def test_serving_respects_max_iter():
    # a step may run several Newton iterations; no request runs more than
    # max_iter in total, and a request stopped by the limit reports it
    import paper_2605_17913_amd as qpx
    pt.dev()
    reqs = _requests(6, seed=8, n_lo=8, n_hi=40)
    with qpx.Server(max_slots=4, iters_per_step=5, max_iter=3) as srv:
        res = [srv.wait(srv.submit(*_args(P))) for P in reqs]
    for r in res:
        assert r["iters"] <= 3 and pt.outcome(r["status"]) == 1, (r["iters"], r["status"])


def test_serving_admission_respects_arena():
    import paper_2605_17913_amd as qpx
    pt.dev()
    reqs = _requests(12, seed=5, n_lo=40, n_hi=60)
    # footprint per request: its data, iterate and arithmetic state,
    # 256-byte aligned pieces
    def fp(P):
        n, m, p = P.n, P.m, P.p
        pieces = [n * n, n, p * n, p, m * n, m, n + p + 2 * m + 1]
        return sum(-(-4 * k // 256) * 256 for k in pieces)
    arena = 100 * 1024
    smallest = min(fp(P) for P in reqs)
    with qpx.Server(max_slots=64, iters_per_step=2, arena_bytes=arena) as srv:
        tickets = [srv.submit(*_args(P)) for P in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(pt.outcome(r["status"]) == 0 for r in res)
    assert 1 <= st["peak_resident"] <= arena // smallest
