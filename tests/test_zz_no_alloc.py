"""GPU test of qp_solve_noalloc (the allocation-free qp_solve), called
through the C-ABI with caller-allocated outputs: two calls in a row, the
second with a smaller input, each bitwise equal to qp_solve on the same
batch (same kernels; only the factor workspace differs), and a batch that
needs more workspace than the fixed array holds is refused."""
import ctypes

import numpy as np
import pytest

import qpgen

import parity as pt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _out(B, n, m, p, d):
    f = dict(dtype=torch.float32, device=d)
    return dict(x=torch.full((B, n), np.nan, **f), y=torch.full((B, p), np.nan, **f),
                z=torch.full((B, m), np.nan, **f), s=torch.full((B, m), np.nan, **f),
                status=torch.full((B,), -7, dtype=torch.int32, device=d),
                iters=torch.full((B,), -7, dtype=torch.int32, device=d),
                res=torch.full((B,), np.nan, **f))


def _call(P, out, **kw):
    import paper_2605_17913_amd as qpx
    d = pt.dev()
    T = [torch.from_numpy(a).to(d) for a in P.arrays()]
    st, keep, (B, n, m, p, dev) = qpx._batch(*T)
    o = qpx.make_opts(**kw)
    so = qpx._Out(qpx._ptr(out["x"]), qpx._ptr(out["y"]), qpx._ptr(out["z"]), qpx._ptr(out["s"]),
                  qpx._ptr(out["status"]), qpx._ptr(out["iters"]), qpx._ptr(out["res"]), None)
    rc = qpx.lib().qp_solve_noalloc(qpx._context(dev), ctypes.byref(st), ctypes.byref(o),
                                    ctypes.byref(so), qpx._stream(dev))
    torch.cuda.synchronize()
    return rc, T


def _same_as_solve(P, T, out):
    import paper_2605_17913_amd as qpx
    ref = pt.npd(qpx.solve(*T))
    got = pt.npd(out)
    for k in ("x", "y", "z", "s", "status", "iters", "res"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.all(pt.outcome(got["status"]) == 0)


def test_noalloc_two_calls_match_qp_solve():
    import paper_2605_17913_amd as qpx
    d = pt.dev()
    # 1) the differentiation shape: factors in the scratch array (6.9 MB)
    P1 = qpgen.random_feasible(64, 100, 200, 20, seed=41)
    assert not qpx.plan(100, 200, 20)["factor_in_lds"]
    out1 = _out(64, 100, 200, 20, d)
    rc, T1 = _call(P1, out1)
    assert rc == 0
    _same_as_solve(P1, T1, out1)
    # 2) a smaller input right after: fewer QPs with larger factors (2.7 MB)
    P2 = qpgen.random_feasible(8, 128, 256, 16, seed=42)
    out2 = _out(8, 128, 256, 16, d)
    rc, T2 = _call(P2, out2)
    assert rc == 0
    _same_as_solve(P2, T2, out2)
    # 3) a batch whose factors stay in LDS uses no scratch
    P3 = qpgen.random_feasible(16, 10, 20, 2, seed=43)
    out3 = _out(16, 10, 20, 2, d)
    rc, T3 = _call(P3, out3)
    assert rc == 0
    _same_as_solve(P3, T3, out3)


def test_noalloc_refuses_oversized_batch():
    import paper_2605_17913_amd as qpx
    d = pt.dev()
    per_qp = qpx.plan(100, 200, 20)["workspace_bytes"]
    B = qpx.NOALLOC_SCRATCH_BYTES // per_qp + 1
    P = qpgen.random_feasible(B, 100, 200, 20, seed=44)
    out = _out(B, 100, 200, 20, d)
    rc, _ = _call(P, out)
    assert rc == -5  # QPX_ERR_UNSUPPORTED, before anything is launched
    assert torch.all(out["status"] == -7)
