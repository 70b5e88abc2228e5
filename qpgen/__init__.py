"""Seeded synthetic QP batches.

This module only draws problem data.  It holds none of the solver's
arithmetic, and both the FP64 oracle and the GPU path read their inputs from
here, so that both sides see bit-identical FP32 problems.

Problem form (paper section 2.1, QP in slack form):

    minimize  1/2 x^T Q x + q^T x   s.t.  A x = b,  G x <= h

Sizes follow one convention throughout: n variables, m inequality rows
(G is m x n), p equality rows (A is p x n).  Arrays are batch-major and
row-major: Q[B,n,n], q[B,n], A[B,p,n], b[B,p], G[B,m,n], h[B,m], all float32
and C-contiguous.

Recipes
-------
random_feasible      Q = M M^T + 1e-2 I with M ~ N(0,1)^{n x n}; q, G, A ~ N(0,1);
                     x0 ~ N(0,1), s0 ~ U(0.1,1), h = G x0 + s0, b = A x0, so x0 is
                     strictly feasible.
ill_conditioned      Q = U diag(lam) U^T, U Haar-orthogonal, lam = 10^U(-4,0);
                     x*, y*, z* constructed so that a random half of the G rows is
                     active at x* (degenerate: active + equality rows >= n).
projection           Euclidean projection onto a polytope, Q = I, no equalities,
                     with a prescribed active face (paper appendix D).
serving_sizes        n ~ U{8..256}, m = 2n, p = floor(n/10), Poisson arrivals.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "QPBatch", "random_feasible", "ill_conditioned", "projection",
    "box_qp", "safety_filter", "serving_requests", "upstream", "CONFIGS", "make_config", "concat",
]


@dataclasses.dataclass
class QPBatch:
    """A batch of QPs, float32, batch-major.  Extra fields carry the
    construction (e.g. a planted optimum) for reporting only."""
    Q: np.ndarray
    q: np.ndarray
    A: np.ndarray
    b: np.ndarray
    G: np.ndarray
    h: np.ndarray
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def B(self) -> int:
        return self.Q.shape[0]

    @property
    def n(self) -> int:
        return self.Q.shape[1]

    @property
    def m(self) -> int:
        return self.G.shape[1]

    @property
    def p(self) -> int:
        return self.A.shape[1]

    def subset(self, idx) -> "QPBatch":
        idx = np.asarray(idx)
        ex = {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == (self.B,) else v)
              for k, v in self.extra.items()}
        return QPBatch(*(np.ascontiguousarray(a[idx]) for a in
                         (self.Q, self.q, self.A, self.b, self.G, self.h)), extra=ex)

    def one(self, i: int):
        """Problem i as float64 arrays (exact upcast of the float32 data)."""
        return tuple(a[i].astype(np.float64) for a in
                     (self.Q, self.q, self.A, self.b, self.G, self.h))

    def arrays(self):
        return (self.Q, self.q, self.A, self.b, self.G, self.h)


def concat(batches) -> QPBatch:
    """Batches of the same sizes joined into one (extras are dropped)."""
    cat = lambda k: np.ascontiguousarray(np.concatenate([getattr(P, k) for P in batches]))
    return QPBatch(*(cat(k) for k in ("Q", "q", "A", "b", "G", "h")))


def _f32(*arrs):
    return tuple(np.ascontiguousarray(a, dtype=np.float32) for a in arrs)


def random_feasible(B: int, n: int, m: int, p: int, seed: int) -> QPBatch:
    """Random strictly feasible convex QPs (the plain / throughput /
    differentiation workloads)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = rng.standard_normal((B, n, n))
    Q = M @ np.swapaxes(M, 1, 2) + 1e-2 * np.eye(n)[None]
    q = rng.standard_normal((B, n))
    G = rng.standard_normal((B, m, n))
    A = rng.standard_normal((B, p, n))
    x0 = rng.standard_normal((B, n))
    s0 = rng.uniform(0.1, 1.0, (B, m))
    Q, q, G, A = _f32(Q, q, G, A)
    # right-hand sides from the float32-rounded matrices so x0 stays feasible
    h = np.einsum("bmn,bn->bm", G.astype(np.float64), x0) + s0
    b = np.einsum("bpn,bn->bp", A.astype(np.float64), x0)
    h, b = _f32(h, b)
    return QPBatch(Q, q, A, b, G, h, extra={"x0": x0})


def ill_conditioned(B: int, n: int, m: int, p: int, seed: int) -> QPBatch:
    """Ill-conditioned, degenerate QPs with a planted optimum x*.

    Q has eigenvalues log-uniform in [1e-4, 1]; a random half of the G rows is
    active at x* with multipliers U(0.1,1); the rest have slack U(0.1,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = rng.standard_normal((B, n, n))
    U, R = np.linalg.qr(Z)
    U = U * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    lam = 10.0 ** rng.uniform(-4.0, 0.0, (B, n))
    Q = (U * lam[:, None, :]) @ np.swapaxes(U, 1, 2)
    Q = 0.5 * (Q + np.swapaxes(Q, 1, 2))
    G = rng.standard_normal((B, m, n))
    A = rng.standard_normal((B, p, n))
    xs = rng.standard_normal((B, n))
    act = np.zeros((B, m), dtype=bool)
    for i in range(B):
        act[i, rng.permutation(m)[: m // 2]] = True
    slack = np.where(act, 0.0, rng.uniform(0.1, 1.0, (B, m)))
    zs = np.where(act, rng.uniform(0.1, 1.0, (B, m)), 0.0)
    ys = rng.standard_normal((B, p))
    Q, G, A = _f32(Q, G, A)
    Qd, Gd, Ad = (a.astype(np.float64) for a in (Q, G, A))
    h = np.einsum("bmn,bn->bm", Gd, xs) + slack
    b = np.einsum("bpn,bn->bp", Ad, xs)
    q = -(np.einsum("bij,bj->bi", Qd, xs) + np.einsum("bmn,bm->bn", Gd, zs)
          + np.einsum("bpn,bp->bn", Ad, ys))
    q, h, b = _f32(q, h, b)
    return QPBatch(Q, q, A, b, G, h, extra={"x_star": xs, "z_star": zs,
                                            "y_star": ys, "active": act})


def projection(B: int, n: int, n_ineq: int, n_active: int, d: float, seed: int) -> QPBatch:
    """Polytope projection instances (paper appendix D).

    Q = I, q = -x_query, no equalities.  A boundary point y0 is made the exact
    projection: the first n_active rows are active at y0 (h_A = G_A y0), the
    others have slack U(0.5, 1.5); the query is x = y0 + G_A^T (d xi) with
    xi ~ U(0.5, 1.5).  Rows of G are Gaussian, normalised to unit length.
    The appendix leaves the row distribution, the inactive margin and y0
    unspecified; these are this module's choices."""
    rng = np.random.Generator(np.random.PCG64(seed))
    G = rng.standard_normal((B, n_ineq, n))
    G /= np.linalg.norm(G, axis=2, keepdims=True)
    y0 = rng.standard_normal((B, n))
    margin = rng.uniform(0.5, 1.5, (B, n_ineq))
    margin[:, :n_active] = 0.0
    xi = rng.uniform(0.5, 1.5, (B, n_active))
    G32, = _f32(G)
    Gd = G32.astype(np.float64)
    h = np.einsum("bmn,bn->bm", Gd, y0) + margin
    xq = y0 + np.einsum("bmn,bm->bn", Gd[:, :n_active], d * xi)
    Q = np.broadcast_to(np.eye(n), (B, n, n))
    A = np.zeros((B, 0, n))
    bb = np.zeros((B, 0))
    Q, q, A, bb, h = _f32(Q, -xq, A, bb, h)
    return QPBatch(Q, q, A, bb, G32, h, extra={"y0": y0, "x_query": xq,
                                               "n_active": n_active})


def box_qp(B: int, n: int, seed: int) -> QPBatch:
    """Diagonal-Q box QPs: Q = diag(d), l <= x <= u as G = [I; -I],
    h = [u; -l].  The exact optimum is clip(-q/d, l, u)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.uniform(0.5, 2.0, (B, n))
    q = 2.0 * rng.standard_normal((B, n))
    lo = rng.uniform(-1.5, -0.5, (B, n))
    hi = rng.uniform(0.5, 1.5, (B, n))
    Q = np.zeros((B, n, n))
    Q[:, np.arange(n), np.arange(n)] = d
    G = np.concatenate([np.broadcast_to(np.eye(n), (B, n, n)),
                        -np.broadcast_to(np.eye(n), (B, n, n))], axis=1)
    h = np.concatenate([hi, -lo], axis=1)
    Q, q, G, h = _f32(Q, q, G, h)
    A = np.zeros((B, 0, n), np.float32)
    b = np.zeros((B, 0), np.float32)
    return QPBatch(Q, q, A, b, G, h, extra={"d": d.astype(np.float32).astype(np.float64),
                                            "lo": -h[:, n:].astype(np.float64),
                                            "hi": h[:, :n].astype(np.float64)})


def safety_filter(B: int, n_agents: int, seed: int) -> QPBatch:
    """Batches shaped like the paper's multi-agent safety filter (appendix F):
    2 N_a variables (a planar control per agent), Q = I, q = -u_nom, no
    equalities, and 4 N_a + 3 N_a + N_a (N_a - 1) / 2 inequality rows:
    per agent the four bounds |u_x|, |u_y| <= 1 and three half-planes
    a' u_i <= h (unit normals a), and per pair of agents one half-plane
    d' (u_i - u_j) <= h_ij.  The appendix trains a network to produce the
    constraint data, which is not available; the half-planes here are
    random, with offsets drawn so that u0 (|u0| < 0.5) is strictly feasible,
    and u_nom ~ N(0, 1) makes a share of the rows active at the optimum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    na = n_agents
    n = 2 * na
    m = 4 * na + 3 * na + na * (na - 1) // 2
    G = np.zeros((B, m, n))
    r = 0
    for i in range(na):
        for c in range(2):
            G[:, r, 2 * i + c] = 1.0
            G[:, r + 1, 2 * i + c] = -1.0
            r += 2
    for i in range(na):
        a = rng.standard_normal((B, 3, 2))
        a /= np.linalg.norm(a, axis=2, keepdims=True)
        G[:, r:r + 3, 2 * i:2 * i + 2] = a
        r += 3
    for i in range(na):
        for j in range(i + 1, na):
            d = rng.standard_normal((B, 2))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            G[:, r, 2 * i:2 * i + 2] = d
            G[:, r, 2 * j:2 * j + 2] = -d
            r += 1
    u0 = rng.uniform(-0.5, 0.5, (B, n))
    G = _f32(G)[0]
    gu = np.einsum("bmn,bn->bm", G.astype(np.float64), u0)
    h = np.empty((B, m))
    h[:, :4 * na] = 1.0
    h[:, 4 * na:] = gu[:, 4 * na:] + rng.uniform(0.05, 1.0, (B, m - 4 * na))
    Q = np.broadcast_to(np.eye(n), (B, n, n)).copy()
    q = -rng.standard_normal((B, n))
    Q, q, h = _f32(Q, q, h)
    A = np.zeros((B, 0, n), np.float32)
    b = np.zeros((B, 0), np.float32)
    return QPBatch(Q, q, A, b, G, h, extra={"u0": u0})


def upstream(B: int, n: int, seed: int) -> np.ndarray:
    """Upstream gradient dL/dx ~ N(0,1), float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((B, n)), dtype=np.float32)


def serving_requests(count: int, seed: int, n_lo: int = 8, n_hi: int = 256):
    """Sizes and per-request seeds of a serving stream: n ~ U{n_lo..n_hi},
    m = 2n, p = floor(n/10).  Arrival times are drawn by the caller from the
    exponential inter-arrival law at the chosen rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(n_lo, n_hi + 1, count)
    seeds = rng.integers(0, 2**62, count)
    return [(int(nn), 2 * int(nn), int(nn) // 10, int(sd)) for nn, sd in zip(ns, seeds)]


# Named workloads: (B, n, m, p, recipe)
CONFIGS = {
    "plain": (64, 10, 20, 2, "random_feasible"),
    "throughput": (4096, 50, 100, 10, "random_feasible"),
    "differentiation": (1024, 100, 200, 20, "random_feasible"),
    "illcond": (512, 256, 512, 32, "ill_conditioned"),
}


def make_config(name: str, seed: int = 0, B: int | None = None) -> QPBatch:
    b0, n, m, p, recipe = CONFIGS[name]
    fn = random_feasible if recipe == "random_feasible" else ill_conditioned
    return fn(B if B is not None else b0, n, m, p, seed)
