"""Benchmark: batched FP32 implicit-complementarity QP solves (+ backward)
on one MI355X.

Workload: 4096 random strictly feasible QPs, n=50, m=100 inequalities,
p=10 equalities (seeded synthetic, see qpgen.random_feasible), FP32, stopping
tolerance 1e-5 on the scaled KKT residuals.  One step = the whole hot path
on that batch: solve (Algorithm 1 with predictor-corrector centering), relax
to kappa_relax = 1e-4 (Algorithm 2), adjoint solve and parameter gradients
(Algorithm 3) for an upstream dL/dx ~ N(0,1).

Printed: one JSON line.  value = fwd+bwd QPs per second of the timed steps;
extra fields give forward-only solves/s, the roofline of the dominant kernel
(the fused solve kernel), the FP64 oracle timed on the host cores, the
standard-form ablation on the same inputs, the serving loop's throughput and
p50/p99 latency, and the rates of the differentiation (n=100) and
ill-conditioned (n=256) configurations.

--calibrate-copy runs only a device-to-device copy of a known size; its
FETCH_SIZE / WRITE_SIZE counters give the scale that turns those counters
into HBM bytes for the solve kernel's measured traffic.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import hashlib

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QP solves/s + fwd+bwd/s at 1e-5 KKT residual (FP32 vs plain); p50/p99 latency"
KERNEL_SRC = os.path.join(ROOT, "paper_2605_17913_amd", "csrc", "qp_kernel_impl.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_qp_solve_kernel_n50_m100_p10.json")

PEAK_ALU = 78.6      # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP32 FMA, unpacked)
PEAK_ALU_PACKED = 157.3
PEAK_HBM = 8000.0    # GB/s


def _oracle_worker(work):
    """One step of the workload per QP with the FP64 oracle: solve to 1e-5,
    relax to kappa_relax = 1e-4 from that point, IFT vector-Jacobian product."""
    import threadpoolctl
    from oracle import gradients, implicit
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        for prob, gx in work:
            r = implicit.solve_qp(*prob, tol=1e-5)
            gradients.grad_at_relaxed(*prob, 1e-4, gx, warm=(r.x, r.y, r.z, r.s))
        return time.perf_counter() - t0, len(work)


def cpu_baseline(P, gx, budget_s=15.0):
    """The FP64 oracle (Algorithm 1 with dense LU on the uncondensed system,
    Algorithm 2, the IFT product from the transposed standard Jacobian) on a
    bounded sample of the same workload, one QP per worker process."""
    import multiprocessing as mp
    cores = min(16, os.cpu_count() or 1)
    t, _ = _oracle_worker([(P.one(0), gx[0])])  # calibrate
    n_qp = int(min(P.B, max(cores, budget_s * cores / max(t, 1e-4))))
    chunks = [[(P.one(i), gx[i]) for i in range(c, n_qp, cores)] for c in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, [c for c in chunks if c])
    wall = time.perf_counter() - t0
    done = sum(r[1] for r in res)
    busy = max(r[0] for r in res)
    return {"value": round(done / busy, 2), "unit": "QPs/s", "cores": cores, "kind": "oracle",
            "sample": f"first {done} of the {P.B} QPs, FP64 oracle solve to tol 1e-5 + relax to "
                      f"kappa 1e-4 + IFT gradient, {cores} worker processes with 1 BLAS thread "
                      f"each ({wall:.1f} s wall)"}


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(launch_s):
    """HBM traffic of the solve kernel from the committed counter runs, or
    None when the kernel source has changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    byts = t["bytes_per_launch"]
    return {"bytes_per_launch": byts, "GB_per_s": round(byts / launch_s / 1e9, 1),
            "hbm_frac": round(byts / launch_s / 1e9 / PEAK_HBM, 4), "source": os.path.basename(TRAFFIC_FILE)}


def calibrate_copy(mib=512, reps=5):
    """Device-to-device copies of a known size (for the counter scale)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}


def config_rate(qpx, torch, P, steps=3, backward=True, **kw):
    """Solves/s (and fwd+bwd/s) of one extra configuration, inputs resident."""
    dev = torch.device("cuda:0")
    Q, q, A, b, G, h = (torch.from_numpy(a).to(dev) for a in P.arrays())
    import qpgen
    gx = torch.from_numpy(qpgen.upstream(P.B, P.Q.shape[1], 11)).to(dev)
    opts = qpx.make_opts(tol=1e-5, kappa_relax=1e-4, **kw)
    sol = qpx.solve(Q, q, A, b, G, h, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sol = qpx.solve(Q, q, A, b, G, h, opts=opts)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / steps
    out = {"solves_per_s": round(P.B / t_fwd, 1),
           "converged_frac": float(np.mean((sol["status"].cpu().numpy() & 0xFF) == 0)),
           "iters_mean": float(sol["iters"].float().mean().item())}
    if backward:
        t0 = time.perf_counter()
        for _ in range(steps):
            s2 = qpx.solve(Q, q, A, b, G, h, opts=opts)
            qpx.backward(Q, q, A, b, G, h, s2, gx, opts=opts)
        torch.cuda.synchronize()
        out["fwd_bwd_per_s"] = round(P.B / ((time.perf_counter() - t0) / steps), 1)
    return out


def serving_bench(n_requests=1200, seed=7, rates=(0.5, 0.9), max_slots=512, iters_per_step=4):
    """Serving workload: a stream of single QPs with n ~ U{8..256}, m = 2n,
    p = floor(n/10) (random feasible recipe).  Saturation throughput is
    measured closed-loop (all requests queued at once); latency
    (completion - submission, host monotonic clock) open-loop with Poisson
    arrivals at fractions of that rate."""
    import paper_2605_17913_amd as qpx
    import qpgen
    sizes = qpgen.serving_requests(n_requests, seed)
    probs = []
    for (n, m, p, sd) in sizes:
        P = qpgen.random_feasible(1, n, m, p, sd % (2**31))
        probs.append((P.Q[0], P.q[0], P.A[0] if p else None, P.b[0] if p else None,
                      P.G[0] if m else None, P.h[0] if m else None))
    out = {"requests": n_requests, "n_range": [8, 256], "max_slots": max_slots,
           "iters_per_step": iters_per_step}
    with qpx.Server(max_slots=max_slots, iters_per_step=iters_per_step,
                    arena_bytes=1 << 30) as srv:
        for P in probs[:16]:  # warm-up: first launches of every kernel variant
            srv.wait(srv.submit(*P))
        t0 = time.perf_counter()
        tickets = [srv.submit(*P) for P in probs]
        res = [srv.wait(t, timeout=300) for t in tickets]
        wall = time.perf_counter() - t0
        mu_sat = n_requests / wall
        out["saturation_solves_per_s"] = round(mu_sat, 1)
        out["converged_frac"] = float(np.mean([(r["status"] & 0xff) == 0 for r in res]))
        out["peak_resident"] = srv.stats()["peak_resident"]
        rng = np.random.default_rng(seed)
        for frac in rates:
            lam = frac * mu_sat
            arr = np.cumsum(rng.exponential(1.0 / lam, n_requests))
            pending = {}
            lat = []
            t0 = time.perf_counter()
            k = 0
            while k < n_requests or pending:
                now = time.perf_counter() - t0
                while k < n_requests and arr[k] <= now:
                    pending[srv.submit(*probs[k])] = None
                    k += 1
                for t in list(pending):
                    r = srv.poll(t)
                    if r is not None:
                        lat.append(r["t_done"] - r["t_submit"])
                        del pending[t]
                if k < n_requests and not pending:
                    time.sleep(max(0.0, min(1e-3, arr[k] - (time.perf_counter() - t0))))
            lat = np.array(lat) * 1e3
            out[f"rate_{frac:.2f}"] = {"offered_per_s": round(lam, 1),
                                       "p50_ms": round(float(np.percentile(lat, 50)), 3),
                                       "p99_ms": round(float(np.percentile(lat, 99)), 3)}
    return out


def projection_grad_errors(n, n_ineq, n_act, kappa_relax, tol, form, seeds=(0, 1, 2),
                           ds=None, device="cuda:0"):
    """Appendix D experiment on the GPU: Euclidean projection onto a polytope
    (Q = I, q = -x_query, no equalities) with a planted active face; the
    gradient of v'Pi(x) with respect to x (= -dl/dq for upstream v) is
    compared with the hard-projection reference J_hard v (eq. hard-jacobian),
    the error measured relative to |v|.
    All (seed, distance) instances of a cell run as one batch.  Returns
    per-instance relative errors (nan on failure) and the first failing
    solver stage of each failed instance."""
    import torch
    import paper_2605_17913_amd as qpx
    import qpgen
    ds = np.logspace(-2, 2, 21) if ds is None else ds
    insts, vs, ghs = [], [], []
    for seed in seeds:
        for k, d in enumerate(ds):
            P = qpgen.projection(1, n, n_ineq, n_act, float(d), seed * 1000 + k)
            rng = np.random.default_rng(seed * 7919 + k)
            v = rng.standard_normal(n).astype(np.float32)
            Ga = P.G[0, :n_act].astype(np.float64)
            Jh = np.eye(n) - Ga.T @ np.linalg.solve(Ga @ Ga.T, Ga)
            insts.append(P)
            vs.append(v)
            ghs.append(Jh @ v.astype(np.float64))
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(P, k) for P in insts])).to(device)
    Q, q, G, h = cat("Q"), cat("q"), cat("G"), cat("h")
    sol = qpx.solve(Q, q, None, None, G, h, form=form, tol=tol, max_iter=100)
    gv = torch.from_numpy(np.stack(vs)).to(device)
    g = qpx.backward(Q, q, None, None, G, h, sol, gv, form=form, tol=tol,
                     kappa_relax=kappa_relax, relax_tol=max(tol, 1e-7), relaxed=True)
    torch.cuda.synchronize()
    st = sol["status"].cpu().numpy()
    rs = g["relaxed"]["status"].cpu().numpy()
    gq = -g["q"].cpu().numpy().astype(np.float64)
    errs, stages = [], []
    for k in range(len(insts)):
        bad_s, bad_r = (st[k] & 0xff) >= 2, (rs[k] & 0xff) >= 2
        if bad_s or bad_r or not np.all(np.isfinite(gq[k])):
            errs.append(np.nan)
            code = st[k] if bad_s else rs[k]
            stage = (code >> 8) & 0xff if (bad_s or bad_r) else 7
            stages.append(qpx.STAGES[stage])
        else:
            # relative to |v| (|J_hard| <= 1; J_hard v vanishes at a vertex)
            errs.append(float(np.linalg.norm(gq[k] - ghs[k]) / np.linalg.norm(vs[k])))
    return np.array(errs), stages


def ablation():
    """Size sweep (kappa_relax = 1e-4, tol 1e-4, #ineq = 1.25 n, active ratio
    m_r in {0.2, 0.6, 0.8}) and kappa_relax sweep (n = 20, 25 inequalities,
    10/12/15 active, tol = min(kappa_relax, 1e-4)) in FP32, as in the paper's
    appendix D, for the bounded form, the standard form and the first
    partially condensed form (appendix B.3, the negative control); medians
    over 3 seeds x 21 distances."""
    out = {"size_sweep": [], "kappa_sweep": []}
    for n in (2, 6, 10, 14, 18, 22, 26, 30, 34, 38):
        for mr in (0.2, 0.6, 0.8):
            n_ineq = int(round(1.25 * n))
            n_act = max(1, int(round(mr * n)))
            row = {"n": n, "m_r": mr}
            for form in ("bounded", "standard", "condensed"):
                e, st = projection_grad_errors(n, n_ineq, n_act, 1e-4, 1e-4, form)
                row[form] = {"fail_rate": round(float(np.mean(np.isnan(e))), 3),
                             "median_err": (round(float(np.nanmedian(e)), 6)
                                            if np.any(~np.isnan(e)) else None)}
            out["size_sweep"].append(row)
    for n_act in (10, 12, 15):
        for kr in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9):
            row = {"n_active": n_act, "kappa_relax": kr}
            for form in ("bounded", "standard", "condensed"):
                e, st = projection_grad_errors(20, 25, n_act, kr, min(kr, 1e-4), form)
                counts = {}
                for x in st:
                    counts[x] = counts.get(x, 0) + 1
                row[form] = {"fail_rate": round(float(np.mean(np.isnan(e))), 3),
                             "median_err": (round(float(np.nanmedian(e)), 7)
                                            if np.any(~np.isnan(e)) else None),
                             "first_failing_stage": counts}
            out["kappa_sweep"].append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--ablation", action="store_true",
                    help="run the appendix D projection sweeps instead of the benchmark")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the differentiation and ill-conditioned configurations")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run device copies of a known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(QPs shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2605_17913_amd as qpx
    import qpgen

    if args.ablation:
        print(json.dumps({"ablation": ablation()}), flush=True)
        return
    if args.calibrate_copy:
        print(json.dumps({"calibrate_copy": calibrate_copy()}), flush=True)
        return

    B, n, m, p = args.batch, 50, 100, 10
    dev = torch.device("cuda:0")
    P = qpgen.random_feasible(B, n, m, p, args.seed)
    Q, q, A, b, G, h = (torch.from_numpy(a).to(dev) for a in P.arrays())
    gx_h = qpgen.upstream(B, n, args.seed + 1)
    gx = torch.from_numpy(gx_h).to(dev)
    opts = qpx.make_opts(tol=1e-5, kappa_relax=1e-4)

    def step(timing=None):
        if timing is not None:
            timing[0].record()
        sol = qpx.solve(Q, q, A, b, G, h, opts=opts, work=timing is not None)
        if timing is not None:
            timing[1].record()
        g = qpx.backward(Q, q, A, b, G, h, sol, gx, opts=opts, work=timing is not None)
        if timing is not None:
            timing[2].record()
        return sol, g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    sols = []
    for k in range(args.steps):
        sols.append(step(evs[k]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = [e[0].elapsed_time(e[1]) for e in evs]
    bwd_ms = [e[1].elapsed_time(e[2]) for e in evs]
    step_ms = [e[0].elapsed_time(e[2]) for e in evs]
    sol, g = sols[-1]
    status = sol["status"].cpu().numpy()
    iters = sol["iters"].cpu().numpy()
    work_fwd = float(sol["work"].sum().item())
    work_bwd = float(g["relaxed"]["work"].sum().item())
    fwd_avg = float(np.mean(fwd_ms)) * 1e-3
    bwd_avg = float(np.mean(bwd_ms)) * 1e-3
    ms_per_step = wall / args.steps * 1e3
    value = B * args.steps / wall
    achieved = work_fwd / fwd_avg / 1e12

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "QPs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"random feasible QPs B={B} n={n} m={m} p={p}, solve to 1e-5 "
                               "(scaled KKT residual) + relax to kappa 1e-4 + IFT backward; "
                               "value = fwd+bwd QPs/s", "batch": B, "n": n, "m": m, "p": p},
        "solves_per_s": round(B / fwd_avg, 1),
        "fwd_ms": round(fwd_avg * 1e3, 3), "bwd_ms": round(bwd_avg * 1e3, 3),
        "converged_frac": float(np.mean((status & 0xff) == 0)),
        "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_ALU,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_ALU, 4),
                     "traffic": measured_traffic(fwd_avg),
                     "kernel": "qp_solve_kernel<256, 2, true> (fused solve, one launch per step)",
                     "launch_ms": round(fwd_avg * 1e3, 3), "peak_packed_fp32": PEAK_ALU_PACKED},
    }
    if not args.no_ablation:
        std = qpx.solve(Q, q, A, b, G, h, form="standard", tol=1e-5)
        torch.cuda.synchronize()
        s2 = std["status"].cpu().numpy()
        out["standard_form"] = {"converged_frac": float(np.mean((s2 & 0xff) == 0)),
                                "nonfinite_or_factor_fail_frac": float(np.mean((s2 & 0xff) >= 2))}
    if not args.no_extra:
        out["other_configs"] = {
            "differentiation n=100 m=200 p=20 B=1024": config_rate(
                qpx, torch, qpgen.random_feasible(1024, 100, 200, 20, 3)),
            "ill-conditioned degenerate n=256 m=512 p=32 B=512": config_rate(
                qpx, torch, qpgen.ill_conditioned(512, 256, 512, 32, 4), steps=1, backward=False),
        }
    if not args.no_serving:
        out["serving"] = serving_bench()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(P, gx_h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
