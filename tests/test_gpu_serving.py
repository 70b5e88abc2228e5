"""GPU tests of the serving loop: continuous batching of QPs of uneven
sizes.  A request must give the same result alone and in a mix (bitwise:
each QP's arithmetic is independent and resuming from the stored iterate
repeats an uninterrupted solve), equal to qp_solve on a batch of one, and
within the parity tolerance of the FP64 oracle."""
import numpy as np
import pytest

import qpgen
from oracle import implicit

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests(count, seed, n_lo=8, n_hi=64):
    reqs = []
    for (n, m, p, sd) in qpgen.serving_requests(count, seed, n_lo, n_hi):
        P = qpgen.random_feasible(1, n, m, p, sd % (2**31))
        reqs.append(P)
    return reqs


def _args(P):
    return (P.Q[0], P.q[0], P.A[0] if P.p else None, P.b[0] if P.p else None,
            P.G[0] if P.m else None, P.h[0] if P.m else None)


def test_serving_alone_equals_mix_equals_batch_and_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_17913_amd as qpx
    reqs = _requests(24, seed=3)
    with qpx.Server(max_slots=8, iters_per_step=3) as srv:
        alone = []
        for P in reqs[:6]:
            alone.append(srv.wait(srv.submit(*_args(P))))
        tickets = [srv.submit(*_args(P)) for P in reqs]  # arrive while others run
        mix = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["peak_resident"] <= 8 and st["completed"] == 30
    for a, b in zip(alone, mix[:6]):
        for k in ("x", "y", "z", "s"):
            assert np.array_equal(a[k], b[k]), k
        assert a["iters"] == b["iters"]
    dev = torch.device("cuda:0")
    for P, r in zip(reqs, mix):
        assert r["status"] == 0, r["status"]
        T = [torch.from_numpy(a).to(dev) for a in P.arrays()]
        sol = qpx.solve(*T)
        torch.cuda.synchronize()
        assert np.array_equal(sol["x"][0].cpu().numpy(), r["x"])
        assert int(sol["iters"][0]) == r["iters"]
        ref = implicit.solve_qp(*P.one(0), tol=1e-11, max_iter=200)
        err = np.linalg.norm(r["x"] - ref.x) / max(1.0, np.linalg.norm(ref.x))
        assert err <= 1e-4, err
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_serving_admission_respects_arena():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_17913_amd as qpx
    reqs = _requests(12, seed=5, n_lo=40, n_hi=60)
    # footprint per request: its data + iterate, 256-byte aligned pieces
    def fp(P):
        n, m, p = P.n, P.m, P.p
        pieces = [n * n, n, p * n, p, m * n, m, n + p + 2 * m]
        return sum(-(-4 * k // 256) * 256 for k in pieces)
    arena = 100 * 1024
    smallest = min(fp(P) for P in reqs)
    with qpx.Server(max_slots=64, iters_per_step=2, arena_bytes=arena) as srv:
        tickets = [srv.submit(*_args(P)) for P in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(r["status"] == 0 for r in res)
    assert 1 <= st["peak_resident"] <= arena // smallest
