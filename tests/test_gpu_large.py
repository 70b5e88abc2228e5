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


def test_ill_conditioned_batch_all_converge():
    # the benchmark's 512-QP batch of the ill-conditioned shape: every QP
    # converges and matches the planted optimum (which the FP64 oracle
    # reproduces to 1e-7).  The scaled residual does not bound the error in
    # x on this shape (smallest eigenvalue of Q 1e-4): at tol 1e-5, 2 of the
    # 512 QPs are 1.6e-4 away; at 1e-6 (0.6 more iterations on average)
    # every QP is within 2e-5, so the test asks for 1e-6.
    P = qpgen.ill_conditioned(512, 256, 512, 32, seed=4)
    print("ill-conditioned degenerate n=256 m=512 p=32 B=512 tol=1e-6 (default assembly)",
          flush=True)
    sol = _run(P, tol=1e-6)
    st = sol["status"] & 0xFF
    errs = np.array([_rel(sol["x"][i], P.extra["x_star"][i]) for i in range(P.B)])
    print(f"  failed {np.nonzero(st)[0].tolist()} worst x err {errs.max():.2e}", flush=True)
    assert np.all(st == 0), np.nonzero(st)[0].tolist()
    assert errs.max() <= 1e-4, (int(errs.argmax()), float(errs.max()))


def test_ill_conditioned_gradients():
    # IFT gradients on the degenerate shape against the FP64 oracle at
    # kappa_relax = 1e-3 (the paper's FP32 setting for its hardest workload).
    # At 1e-4 the relaxation does not reach its tolerance within 30
    # iterations on this shape (status MAX_ITER) and the gradient is not
    # accurate; the status tells the caller.
    import paper_2605_17913_amd as qpx
    from oracle import gradients
    d = _dev()
    P = qpgen.ill_conditioned(2, 256, 512, 32, seed=1)
    print("ill-conditioned gradients n=256 m=512 p=32 B=2 kappa_relax=1e-3", flush=True)
    Q, q, A, b, G, h = [torch.from_numpy(a).to(d) for a in P.arrays()]
    sol = qpx.solve(Q, q, A, b, G, h, tol=1e-6)
    gx = qpgen.upstream(P.B, 256, seed=2)
    g = qpx.backward(Q, q, A, b, G, h, sol, torch.from_numpy(gx).to(d), kappa_relax=1e-3,
                     relaxed=True)
    torch.cuda.synchronize()
    # converged, or stopped at relax_max_iter just short of relax_tol (the
    # default refinement leaves the relaxed residual near 1e-7 on this shape;
    # refine_steps=8 converges it): the gradients are checked either way
    assert int(g["relaxed"]["status"][0].item()) & 0xFF <= 1
    ref, rr = gradients.grad_at_relaxed(*P.one(0), 1e-3, gx[0].astype(np.float64))
    assert _rel(g["relaxed"]["x"][0].cpu().numpy(), rr.x) <= 1e-4
    for key in ("Q", "q", "A", "b", "G", "h"):
        gg = g[key][0].cpu().numpy()
        err = np.linalg.norm(gg - ref[key]) / max(1e-3, np.linalg.norm(ref[key]))
        print(f"  d{key} err {err:.2e}", flush=True)
        assert err <= 1e-3, (key, err)


def test_workspace_shared_across_streams():
    # the context's global factor workspace is shared; solves enqueued on two
    # streams one after the other must not overlap on it
    import paper_2605_17913_amd as qpx
    d = _dev()
    P1 = qpgen.random_feasible(64, 128, 256, 16, seed=21)
    P2 = qpgen.random_feasible(64, 128, 256, 16, seed=22)
    T1 = [torch.from_numpy(a).to(d) for a in P1.arrays()]
    T2 = [torch.from_numpy(a).to(d) for a in P2.arrays()]
    ref1 = qpx.solve(*T1)["x"].cpu().numpy()
    ref2 = qpx.solve(*T2)["x"].cpu().numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(s1):
            a = qpx.solve(*T1)
        with torch.cuda.stream(s2):
            b = qpx.solve(*T2)
        torch.cuda.synchronize()
        assert np.array_equal(a["x"].cpu().numpy(), ref1)
        assert np.array_equal(b["x"].cpu().numpy(), ref2)
