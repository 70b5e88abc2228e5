"""GPU tests of the torch.autograd wrapper (QPFunction / qp_layer): its
gradients are the library's backward pass (bitwise equal to calling
qp_backward directly) and match the FP64 oracle's implicit-function-theorem
product entry by entry (tests/parity.py), with and without equality and
inequality constraints; inputs given as None get no gradient; a QP that does
not converge raises."""
import numpy as np
import pytest

import qpgen
from oracle import gradients

import parity as pt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KR = 1e-3


def _leaf(a, d):
    return None if a is None else torch.from_numpy(a).to(d).requires_grad_(True)


@pytest.mark.parametrize("shape", [(10, 20, 2), (10, 20, 0), (10, 0, 3), (12, 0, 0)])
def test_qp_layer_gradients(shape):
    import paper_2605_17913_amd as qpx
    n, m, p = shape
    d = pt.dev()
    P = qpgen.random_feasible(8, n, m, p, seed=17 + m + p)
    arr = [P.Q, P.q, P.A if p else None, P.b if p else None, P.G if m else None,
           P.h if m else None]
    leaves = [_leaf(a, d) for a in arr]
    v_np = qpgen.upstream(P.B, n, seed=4)
    v = torch.from_numpy(v_np).to(d)
    x, status = qpx.qp_layer(*leaves, return_status=True, kappa_relax=KR)
    assert np.all(pt.outcome(status.cpu().numpy()) == 0)
    (x * v).sum().backward()
    for k, t in enumerate(leaves):
        if arr[k] is None:
            assert t is None
        else:
            assert t.grad is not None and t.grad.shape == t.shape
    # the same gradients as the direct backward call
    T = [None if a is None else torch.from_numpy(a).to(d) for a in arr]
    sol = qpx.solve(*T, kappa_relax=KR)
    g = qpx.backward(*T, sol, v, kappa_relax=KR)
    for k, key in enumerate(pt.BLOCKS):
        if leaves[k] is not None:
            assert torch.equal(leaves[k].grad, g[key]), key
    # and the oracle's IFT product at the relaxed point
    grads = {key: (leaves[k].grad.cpu().numpy() if leaves[k] is not None
                   else np.zeros((P.B,) + getattr(P, key).shape[1:], np.float32))
             for k, key in enumerate(pt.BLOCKS)}
    for i in (0, 5):
        ref, _ = gradients.grad_at_relaxed(*P.one(i), KR, v_np[i].astype(np.float64))
        pt.check_grads(f"qp_layer {shape} QP {i}", grads, i, ref)


def test_needs_input_grad_is_honoured():
    import paper_2605_17913_amd as qpx
    d = pt.dev()
    P = qpgen.random_feasible(4, 8, 16, 2, seed=3)
    Q, q, A, b, G, h = (torch.from_numpy(a).to(d) for a in P.arrays())
    q.requires_grad_(True)
    x = qpx.qp_layer(Q, q, A, b, G, h, kappa_relax=KR)
    x.sum().backward()
    assert q.grad is not None and Q.grad is None and G.grad is None


def test_failed_solve_raises():
    import paper_2605_17913_amd as qpx
    d = pt.dev()
    P = qpgen.random_feasible(4, 10, 20, 2, seed=1)
    T = [torch.from_numpy(a).to(d) for a in P.arrays()]
    with pytest.raises(qpx.QPError):
        qpx.qp_layer(*T, max_iter=1)  # one Newton iteration cannot converge
    x, st = qpx.qp_layer(*T, max_iter=1, check=False, return_status=True)
    assert np.all(pt.outcome(st.cpu().numpy()) == 1)
