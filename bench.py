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
(the fused solve kernel) and of every other hot kernel (`kernels`), the same
step under the FP64-residual policy (`precision`), the oracle timed on the
host cores in FP64 and in FP32 (the plain per-QP path), the standard-form
ablation on the same inputs, the serving loop's throughput and p50/p99
latency per size class, and the rates of the differentiation (n=100) and
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
CSRC = os.path.join(ROOT, "paper_2605_17913_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_kernels_bench_workloads.json")

PEAK_ALU = 78.6      # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP32 FMA, unpacked)
PEAK_ALU_PACKED = 157.3
PEAK_MFMA_FP32 = 157.3  # TFLOP/s, dense FP32 matrix cores
PEAK_HBM = 8000.0    # GB/s

# The ill-conditioned workload is solved to 1e-6 (at 1e-5 its scaled residual
# does not bound the error in x to 1e-4) and differentiated at
# kappa_relax = 1e-3 (float32 cannot resolve its relaxed system at 1e-4).
ILL_TOL = 1e-6
ILL_KAPPA_RELAX = 1e-3


def _oracle_worker(args):
    """One step of the workload per QP with the oracle: solve to 1e-5, relax
    to kappa_relax = 1e-4 from that point, IFT vector-Jacobian product.
    dtype float64 is the oracle as it stands; float32 runs the same code in
    single precision (the plain per-QP FP32 path; the IFT product itself is
    float64 in the oracle).  Returns (busy seconds, QPs, converged)."""
    work, dtype = args
    import threadpoolctl
    from oracle import gradients, implicit
    with threadpoolctl.threadpool_limits(1), np.errstate(all="ignore"):
        t0 = time.perf_counter()
        conv = 0
        for prob, gx in work:
            r = implicit.solve_qp(*prob, tol=1e-5, dtype=dtype)
            rr = implicit.relax_qp(*prob, r.x, r.y, r.z, r.s, 1e-4, tol=1e-6, dtype=dtype)
            if dtype == np.float64:
                gradients.ift_vjp(*prob, rr.x, rr.y, rr.z, rr.s, gx)
            elif np.all(np.isfinite(rr.x)):
                gradients.ift_vjp(*prob, rr.x, rr.y, rr.z, rr.s, gx)
            conv += int(r.status == 0 and rr.status == 0)
        return time.perf_counter() - t0, len(work), conv


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(P, gx, dtype, workers, budget_s):
    """QPs/s of the oracle step on `workers` processes (1 BLAS thread each),
    on the first QPs of the batch, sized to about budget_s seconds of work
    per worker."""
    import multiprocessing as mp
    t, _, _ = _oracle_worker(([(P.one(0), gx[0])], dtype))  # calibrate
    n_qp = int(min(P.B, max(workers, budget_s * workers / max(t, 1e-4))))
    chunks = [[(P.one(i), gx[i]) for i in range(c, n_qp, workers)] for c in range(workers)]
    if workers == 1:
        res = [_oracle_worker((chunks[0], dtype))]
    else:
        with mp.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_oracle_worker, [(c, dtype) for c in chunks if c])
    done = sum(r[1] for r in res)
    busy = max(r[0] for r in res)
    return {"value": round(done / busy, 2), "qps": done, "converged": sum(r[2] for r in res)}


def cpu_baseline(P, gx, budget_s=6.0):
    """The oracle on a bounded sample of the same workload: FP64 (the oracle
    as it stands) and FP32 (the plain per-QP path), each on one core and on
    every core of this process's CPU set, one QP per worker process."""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(16, cores))
    all64 = _oracle_rate(P, gx, np.float64, cores, budget_s)
    one64 = _oracle_rate(P, gx, np.float64, 1, budget_s)
    all32 = _oracle_rate(P, gx, np.float32, cores, budget_s)
    one32 = _oracle_rate(P, gx, np.float32, 1, budget_s)
    return {"value": all64["value"], "unit": "QPs/s", "cores": cores, "kind": "oracle",
            "sample": f"first {all64['qps']} of the {P.B} QPs (all cores) and {one64['qps']} "
                      f"(one core): oracle solve to tol 1e-5 + relax to kappa 1e-4 + IFT "
                      f"gradient, one QP per worker process with 1 BLAS thread",
            "one_core": one64["value"],
            "plain_fp32": {"all_cores": all32["value"], "one_core": one32["value"],
                           "converged_frac": round(all32["converged"] / max(1, all32["qps"]), 3),
                           "note": "the same oracle code in float32 (IFT product in float64)"},
            "nproc": os.cpu_count(), "cpu_set": cores, "cpu_model": _cpu_model()}


def kernel_source_hash():
    """Hash of every source the kernels are built from (csrc/ and the
    C-ABI header): a change to any of them invalidates stored counters."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hpp", ".hip", ".cpp", ".h")))
    for name in files + ["../../include/qpx.h"]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_name(kind, n, m, p, **kw):
    """Name of the fused kernel the library launches for one problem size
    (from its launch plan)."""
    import paper_2605_17913_amd as qpx
    pl = qpx.plan(n, m, p, **kw)
    rpl = (n + pl["kb"] + p + 63) // 64
    rpl = 1 if rpl <= 1 else 2 if rpl <= 2 else 4 if rpl <= 4 else 8 if rpl <= 8 else 16
    lds = "true" if pl["factor_in_lds"] else "false"
    return f"qp_{kind}_kernel<{pl['threads']}, {rpl}, {lds}>"


def measured_traffic(kernel, launch_s):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, scaled by a
    copy of known size) from the committed counter runs, or None when a
    kernel source has changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(kernel)
    if t.get("kernel_source_sha256_16") != kernel_source_hash() or k is None:
        return None
    byts = k["fetch_bytes"] + k["write_bytes"]
    return {"bytes_per_launch": byts, "fetch_bytes": k["fetch_bytes"],
            "write_bytes": k["write_bytes"], "GB_per_s": round(byts / launch_s / 1e9, 1),
            "hbm_frac": round(byts / launch_s / 1e9 / PEAK_HBM, 4),
            "source": os.path.basename(TRAFFIC_FILE)}


def grad_bytes(B, n, m, p):
    """Bytes of the parameter gradients one backward launch writes (a14)."""
    return 4 * B * (n * n + n + p * n + p + m * n + m)


def roofline_entry(kernel, bound, achieved, peak, unit, launch_ms, workload="", **extra):
    return dict(kernel=f"{kernel} {workload}".strip(), bound=bound, achieved=round(achieved, 3),
                peak=peak, unit=unit, frac=round(achieved / peak, 4),
                launch_ms=round(launch_ms, 3),
                traffic=measured_traffic(kernel, launch_ms * 1e-3), **extra)


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


def timed_config(qpx, torch, P, steps=3, backward=True, kappa_relax=1e-4, **kw):
    """Solves/s (and fwd+bwd/s) of one configuration with inputs resident,
    each launch timed with HIP events on its stream, plus the kernels'
    algorithmic flops (the `work` counters)."""
    import qpgen
    dev = torch.device("cuda:0")
    Q, q, A, b, G, h = (torch.from_numpy(a).to(dev) for a in P.arrays())
    gx = torch.from_numpy(qpgen.upstream(P.B, P.Q.shape[1], 11)).to(dev)
    opts = qpx.make_opts(kappa_relax=kappa_relax, **kw)
    sol = qpx.solve(Q, q, A, b, G, h, opts=opts)
    if backward:
        qpx.backward(Q, q, A, b, G, h, sol, gx, opts=opts)
    torch.cuda.synchronize()
    fwd, bwd = [], []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        sol = qpx.solve(Q, q, A, b, G, h, opts=opts, work=True)
        e[1].record()
        if backward:
            g = qpx.backward(Q, q, A, b, G, h, sol, gx, opts=opts, work=True)
        e[2].record()
        torch.cuda.synchronize()
        fwd.append(e[0].elapsed_time(e[1]) * 1e-3)
        bwd.append(e[1].elapsed_time(e[2]) * 1e-3)
    st = sol["status"].cpu().numpy()
    tf, tb = float(np.median(fwd)), float(np.median(bwd))
    out = {"solves_per_s": round(P.B / tf, 1),
           "converged_frac": float(np.mean((st & 0xFF) == 0)),
           "fp64_refinement_frac": float(np.mean((st >> 16) & 1)),
           "iters_mean": float(sol["iters"].float().mean().item()),
           "fwd_ms": round(tf * 1e3, 3), "fwd_flops": float(sol["work"].sum().item())}
    if kw.get("assembly") == "bf16x3":
        out["bf16x3_fallback_frac"] = float(np.mean((st >> 17) & 1))
    if backward:
        rst = g["relaxed"]["status"].cpu().numpy()
        out.update({"fwd_bwd_per_s": round(P.B / (tf + tb), 1), "bwd_ms": round(tb * 1e3, 3),
                    "relax_converged_frac": float(np.mean((rst & 0xFF) == 0)),
                    "bwd_flops": float(g["relaxed"]["work"].sum().item())})
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
                    pending[srv.submit(*probs[k])] = sizes[k][0]
                    k += 1
                for t in list(pending):
                    r = srv.poll(t)
                    if r is not None:
                        lat.append((r["t_done"] - r["t_submit"], pending[t]))
                        del pending[t]
                if k < n_requests and not pending:
                    time.sleep(max(0.0, min(1e-3, arr[k] - (time.perf_counter() - t0))))
            lat = np.array([l for l, _ in lat]) * 1e3, np.array([n for _, n in lat])
            row = {"offered_per_s": round(lam, 1),
                   "p50_ms": round(float(np.percentile(lat[0], 50)), 3),
                   "p99_ms": round(float(np.percentile(lat[0], 99)), 3), "by_n": {}}
            for lo, hi in ((8, 64), (65, 128), (129, 256)):
                sel = lat[0][(lat[1] >= lo) & (lat[1] <= hi)]
                if sel.size:
                    row["by_n"][f"{lo}-{hi}"] = {
                        "count": int(sel.size), "p50_ms": round(float(np.percentile(sel, 50)), 3),
                        "p99_ms": round(float(np.percentile(sel, 99)), 3)}
            out[f"rate_{frac:.2f}"] = row
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

    def run_steps(opts, steps, warmup):
        """`steps` timed steps (solve + relax + backward) after `warmup`
        untimed ones; HIP events on the launch stream around each launch."""
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
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        t0 = time.perf_counter()
        sols = [step(evs[k]) for k in range(steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fwd = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) * 1e-3
        bwd = float(np.mean([e[1].elapsed_time(e[2]) for e in evs])) * 1e-3
        return sols[-1], wall, fwd, bwd

    opts = qpx.make_opts(tol=1e-5, kappa_relax=1e-4)
    (sol, g), wall, fwd_avg, bwd_avg = run_steps(opts, args.steps, args.warmup)
    status = sol["status"].cpu().numpy()
    rstatus = g["relaxed"]["status"].cpu().numpy()
    iters = sol["iters"].cpu().numpy()
    work_fwd = float(sol["work"].sum().item())
    work_bwd = float(g["relaxed"]["work"].sum().item())
    ms_per_step = wall / args.steps * 1e3
    value = B * args.steps / wall
    achieved = work_fwd / fwd_avg / 1e12
    solve_k = kernel_name("solve", n, m, p)
    bwd_k = kernel_name("backward", n, m, p)

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
        "relax_converged_frac": float(np.mean((rstatus & 0xff) == 0)),
        "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_ALU,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_ALU, 4),
                     "traffic": measured_traffic(solve_k, fwd_avg),
                     "kernel": f"{solve_k} (fused solve, one launch per step)",
                     "launch_ms": round(fwd_avg * 1e3, 3), "peak_packed_fp32": PEAK_ALU_PACKED},
    }
    kernels = [
        roofline_entry(solve_k, "alu", achieved, PEAK_ALU, "TFLOP/s", fwd_avg * 1e3, "n=50"),
        roofline_entry(bwd_k, "alu", work_bwd / bwd_avg / 1e12, PEAK_ALU, "TFLOP/s",
                       bwd_avg * 1e3, "n=50"),
        roofline_entry(bwd_k, "hbm", grad_bytes(B, n, m, p) / bwd_avg / 1e9, PEAK_HBM, "GB/s",
                       bwd_avg * 1e3, "n=50 (gradient writes, a14)",
                       note="gradient bytes written / whole backward launch (relax + adjoint "
                            "+ writes): a lower bound on the write bandwidth of a14"),
    ]
    out["kernels"] = kernels
    # the same step with FP64-accumulated residuals everywhere (the other
    # precision policy), for comparison with the FP32-first default
    (sol64, g64), wall64, f64, b64 = run_steps(qpx.make_opts(tol=1e-5, kappa_relax=1e-4,
                                                             residual="fp64"),
                                               max(2, args.steps // 2), 1)
    out["precision"] = {
        "default": {"policy": "FP32 residuals; FP64 refinement residuals for QPs whose FP32 "
                              "refinement stalls",
                    "solves_per_s": round(B / fwd_avg, 1), "fwd_bwd_per_s": round(value, 1),
                    "fp64_refinement_frac_fwd": float(np.mean((status >> 16) & 1)),
                    "fp64_refinement_frac_bwd": float(np.mean((rstatus >> 16) & 1))},
        "fp64_residual": {"solves_per_s": round(B / f64, 1),
                          "fwd_bwd_per_s": round(B * max(2, args.steps // 2) / wall64, 1),
                          "converged_frac": float(np.mean(
                              (sol64["status"].cpu().numpy() & 0xff) == 0))},
    }
    if not args.no_ablation:
        std = qpx.solve(Q, q, A, b, G, h, form="standard", tol=1e-5)
        torch.cuda.synchronize()
        s2 = std["status"].cpu().numpy()
        out["standard_form"] = {"converged_frac": float(np.mean((s2 & 0xff) == 0)),
                                "nonfinite_or_factor_fail_frac": float(np.mean((s2 & 0xff) >= 2))}
    if not args.no_extra:
        c3 = timed_config(qpx, torch, qpgen.make_config("differentiation", seed=3))
        ill = qpgen.make_config("illcond", seed=4)
        c5 = timed_config(qpx, torch, ill, steps=2, tol=ILL_TOL, kappa_relax=ILL_KAPPA_RELAX)
        c5b = timed_config(qpx, torch, ill, steps=2, backward=False, tol=ILL_TOL,
                           assembly="bf16x3")
        out["other_configs"] = {
            "differentiation n=100 m=200 p=20 B=1024 (tol 1e-5, kappa_relax 1e-4)": c3,
            f"ill-conditioned degenerate n=256 m=512 p=32 B=512 (tol {ILL_TOL}, "
            f"kappa_relax {ILL_KAPPA_RELAX}, FP32 matrix-core assembly)": c5,
            f"ill-conditioned degenerate n=256 m=512 p=32 B=512 (tol {ILL_TOL}, "
            "BF16x3 split-product assembly + refinement)": c5b,
        }
        k3s, k3b = kernel_name("solve", 100, 200, 20), kernel_name("backward", 100, 200, 20)
        k5 = kernel_name("solve", 256, 512, 32)
        kernels += [
            roofline_entry(k3s, "alu", c3["fwd_flops"] / c3["fwd_ms"] / 1e9,
                           PEAK_ALU, "TFLOP/s", c3["fwd_ms"], "n=100"),
            roofline_entry(k3b, "alu", c3["bwd_flops"] / c3["bwd_ms"] / 1e9,
                           PEAK_ALU, "TFLOP/s", c3["bwd_ms"], "n=100"),
            roofline_entry(k3b, "hbm", grad_bytes(1024, 100, 200, 20) / c3["bwd_ms"] / 1e6,
                           PEAK_HBM, "GB/s", c3["bwd_ms"], "n=100 (gradient writes, a14)"),
            roofline_entry(k5, "mfma", c5["fwd_flops"] / c5["fwd_ms"] / 1e9, PEAK_MFMA_FP32,
                           "TFLOP/s", c5["fwd_ms"], "n=256 FP32 MFMA assembly"),
            roofline_entry(k5, "mfma", c5b["fwd_flops"] / c5b["fwd_ms"] / 1e9, PEAK_MFMA_FP32,
                           "TFLOP/s", c5b["fwd_ms"], "n=256 BF16x3 assembly"),
        ]
    if not args.no_serving:
        out["serving"] = serving_bench()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(P, gx_h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
