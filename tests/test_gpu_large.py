"""GPU parity on the large-size paths, against the FP64 oracle.

* The bordered factor in global memory: with n = 128, m = 256, p = 16 the
  factor (N up to 272 rows) needs about 161 KB, more than a workgroup's LDS,
  and the solves run with 8 rows per lane; with n = 256, m = 512, p = 32 the
  system has up to 544 rows and the solves run with 16 rows per lane.
* Each H-block assembly arithmetic (FP32 vector ALUs, BF16x3 split products
  on the matrix cores with refinement, FP32 on the matrix cores).
* The ill-conditioned, degenerate shape (Q with eigenvalues down to 1e-4,
  half of the 512 rows active, plus 32 equalities, in R^256): x is unique,
  the multipliers are not, so x is compared with the oracle's and with the
  planted optimum.

Tolerances as in test_gpu_parity: x within 1e-4 (relative, 2-norm) of the
oracle, and duals within 1e-3 where the duals are unique; for the
ill-conditioned shape also x within 1e-4 of the planted optimum.
"""
import numpy as np
import pytest

import qpgen
from oracle import implicit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _run(P, **kw):
    import paper_2605_17913_amd as qpx
    d = _dev()
    Q, q, A, b, G, h = [torch.from_numpy(a).to(d) for a in P.arrays()]
    sol = qpx.solve(Q, q, A, b, G, h, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in sol.items()}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(1.0, np.linalg.norm(b)))


def _parity(P, sol, idx, xtol, dtol):
    worst = 0.0
    for i in idx:
        r = implicit.solve_qp(*P.one(i), tol=1e-11, max_iter=200)
        assert r.status == implicit.CONVERGED
        ex = _rel(sol["x"][i], r.x)
        worst = max(worst, ex)
        assert ex <= xtol, (i, ex)
        if dtol is not None:
            ez = float(np.max(np.abs(sol["z"][i] - r.z)) / max(1.0, np.max(np.abs(r.z))))
            assert ez <= dtol, (i, ez)
    return worst


@pytest.mark.parametrize("assembly", ["fp32", "bf16x3", "mfma_fp32"])
def test_global_factor_path_n128(assembly):
    P = qpgen.random_feasible(8, 128, 256, 16, seed=9)
    print(f"global factor n=128 m=256 p=16 B=8 assembly={assembly}", flush=True)
    sol = _run(P, assembly=assembly)
    st = sol["status"] & 0xFF
    assert np.all(st == 0), (st.tolist(), sol["iters"].tolist())
    worst = _parity(P, sol, [0, 3, 7], 1e-4, 1e-3)
    print(f"  iters {sol['iters'].tolist()} worst x err {worst:.2e}", flush=True)


def test_sixteen_rows_per_lane_n256():
    P = qpgen.random_feasible(4, 256, 512, 32, seed=10)
    print("global factor n=256 m=512 p=32 B=4 (up to 544 rows)", flush=True)
    sol = _run(P)
    st = sol["status"] & 0xFF
    assert np.all(st == 0), (st.tolist(), sol["iters"].tolist())
    worst = _parity(P, sol, [0, 2], 1e-4, 1e-3)
    print(f"  iters {sol['iters'].tolist()} worst x err {worst:.2e}", flush=True)


def test_ill_conditioned_degenerate():
    P = qpgen.ill_conditioned(4, 256, 512, 32, seed=0)
    print("ill-conditioned degenerate n=256 m=512 p=32 B=4", flush=True)
    sol = _run(P)
    st = sol["status"] & 0xFF
    errs = [_rel(sol["x"][i], P.extra["x_star"][i]) for i in range(P.B)]
    print(f"  status {st.tolist()} iters {sol['iters'].tolist()} "
          f"x err vs planted {[f'{e:.1e}' for e in errs]}", flush=True)
    assert np.all(st == 0), st.tolist()
    assert max(errs) <= 1e-4, errs
    _parity(P, sol, [0], 1e-4, None)
