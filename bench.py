#!/usr/bin/env python3
"""Throughput benchmark of the second-order adjoint evaluation on one MI355X.

One step = cost + exact gradient + exact Hessian (every row of the hot path: controls,
eigen-data, forward sweep, terminal residual, backward sweep, U'' contraction, assembly)
for a batch of independent control-coefficient vectors theta on the molecule-sized
workload (N=36, J=4000 steps of dt=0.02, Fourier model with K=16 harmonics, P=32).
Inputs are synthetic (seeded generators) and resident in HBM before timing starts.

Prints one JSON line.  --gpus N with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2505_00529_amd import inputs, qoc  # noqa: E402

PEAK_FP64 = 78.6e12          # MI355X FP64 vector (= FP64 matrix) peak, FLOP/s
PEAK_HBM = 8.0e12            # bytes/s


def alg_flops_per_step(kernel: str, n: int, p: int) -> float:
    """Algorithmic FLOPs per (theta, time step) of each kernel (method's nominal counts)."""
    return {
        "eig": 9.0 * n ** 3 + 4.0 * n ** 3,   # eigendecomposition + Mt = V^T M V
        "forward": 8.0 * n * n * p,           # N x N . N x P complex tangent product
        "backward": 8.0 * n * n * p,          # N x N . N x P complex second-adjoint product
        "sterm": 8.0 * n ** 3,                # U'' contraction (two N x N complex-real products)
    }.get(kernel, 0.0)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_molecule_b256.json")


# the sources that decide what the single-problem evaluation kernels do and how they are launched
# (the solvers, the batch layer and the network do not enter a counter run of the evaluation)
KERNEL_SOURCES = ("qoc_api.hip", "qoc_api_internal.h", "qoc_device.h", "qoc_internal.h", "qoc_kernels.hip")


def kernel_source_digest() -> str:
    """SHA-256 over the evaluation kernels' sources (ties a counter measurement to the code)."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2505_00529_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, batch: int):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE counter runs,
    each scaled by the factor a reference copy of known size gave; None when the kernel sources
    have changed since, or the measurement was for another kernel or batch."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("batch") != batch or t.get("source_sha256") != kernel_source_digest():
        return None
    return 1024.0 * (t["fetch_kib_per_dispatch"] * t["fetch_scale"] + t["write_kib_per_dispatch"] * t["write_scale"])


def log(msg: str) -> None:
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(w, single_thread_steps: int = 1000) -> dict:
    """The CPU oracle timed on the host cores: one theta of the same workload (full cost + grad +
    Hessian) with every BLAS thread, and the first `single_thread_steps` steps of it on one
    thread (the oracle's time is linear in the steps; the rate is scaled to the full horizon)."""
    from oracle import qoc_oracle as O
    from threadpoolctl import threadpool_info, threadpool_limits

    threads = max([int(x.get("num_threads", 1)) for x in threadpool_info()] or [1])
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    th = inputs.draw_thetas(w.p, 1, w.seed)[0]
    t0 = time.perf_counter()
    O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th, w.gamma, w.rho)
    dt = time.perf_counter() - t0
    ns = min(single_thread_steps, w.nt)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis[:ns], w.dt, th, w.gamma, w.rho)
        dt1 = (time.perf_counter() - t0) * w.nt / ns
    return {"value": 1.0 / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"1 theta of the same workload (N={s.n}, J={w.nt}, P={w.p}), full cost+grad+Hessian, "
                      f"{dt:.1f} s on {threads} BLAS threads; forward-over-forward oracle with "
                      "block-triangular exponentials",
            "single_thread": {"value": 1.0 / dt1, "unit": "evals/s", "cores": 1,
                              "sample": f"the first {ns} of the {w.nt} steps of the same theta on one thread, "
                                        f"{dt1 * ns / w.nt:.1f} s, scaled to the full horizon"}}


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
PARITY_TOL = 1e-10


def parity_vs_oracle(workload: str, costs, grads, hess) -> dict:
    """Normwise relative error of the timed batch's thetas 0 and 1 (the benchmark draws the
    stored oracle cases first) against the CPU oracle's values for them."""
    path = os.path.join(GOLDEN_DIR, f"{workload}_oracle.json")
    with open(path) as f:
        doc = json.load(f)

    def rel(a, b):
        b = np.asarray(b)
        return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))

    errs = {}
    for case in doc["cases"]:
        i = case["theta_index"]
        errs[f"theta{i}"] = {"cost": rel(costs[i], case["cost"]), "grad": rel(grads[i], case["grad"]),
                             "hess": rel(hess[i], case["hess"])}
    worst = max(v for e in errs.values() for v in e.values())
    return {"max_rel_err": worst, "tolerance": PARITY_TOL, "ok": worst < PARITY_TOL, "per_theta": errs,
            "reference": f"oracle values of thetas 0 and 1 (tests/golden/{workload}_oracle.json)"}


KERNELS = ["controls", "eig", "boundary", "forward", "terminal", "backward", "sterm", "assemble"]


def timed_batch(prob, thetas, steps: int, warmup: int, stream, label: str):
    """Warm up, then time `steps` Hessian evaluations of the batch `thetas` (device tensor) with
    HIP events on `stream`; per-kernel averages from the library's own events on the same stream."""
    import torch

    B, P = thetas.shape
    costs = torch.empty(B, dtype=torch.float64, device="cuda")
    grads = torch.empty(B, P, dtype=torch.float64, device="cuda")
    hess = torch.empty(B, P, P, dtype=torch.float64, device="cuda")

    def step():
        prob.hess_many_dev(B, thetas.data_ptr(), costs.data_ptr(), grads.data_ptr(), hess.data_ptr())

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"bench: {label} warmup {i + 1}/{warmup} done")
    prob.sync()
    prob.jacobi_stats(reset=True)
    prob.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prob.sync()
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    log(f"bench: {label}: {steps} timed steps in {t1 - t0:.3f} s")
    ktimes = {}
    for k in KERNELS:
        ms, cnt = prob.profile_kernel_ms(k)
        if cnt:
            ktimes[k] = (ms / cnt, cnt)
    prob.profile_enable(False)
    eig_steps, eig_sweeps = prob.jacobi_stats(reset=True)
    return {"elapsed": t1 - t0, "step_ms": step_ms, "ktimes": ktimes,
            "sweeps_per_step": eig_sweeps / max(eig_steps, 1),
            "costs": costs.cpu().numpy(), "grads": grads.cpu().numpy(), "hess": hess.cpu().numpy()}


def eig_roofline(ktimes, n, P, nt, B):
    avg_ms = ktimes["eig"][0]
    achieved = alg_flops_per_step("eig", n, P) * nt * B / (avg_ms * 1e-3) / 1e12
    return achieved, achieved / (PEAK_FP64 / 1e12)


def secondary_system(name: str, B: int, steps: int, stream) -> dict:
    """Throughput of a second system (same measurement, fewer steps), reported beside the
    headline line."""
    import torch

    w = inputs.make_workload(name)
    n, P, nt = w.system.n, w.p, w.nt
    log(f"bench: secondary workload {name} n={n} nt={nt} P={P} batch={B}")
    prob = qoc.problem_from_workload(w, device=0)
    prob.set_stream(stream.cuda_stream)
    thetas = torch.tensor(inputs.draw_thetas(P, B, w.seed), dtype=torch.float64, device="cuda")
    r = timed_batch(prob, thetas, steps, 1, stream, name)
    prob.close()
    value = B * steps / r["elapsed"]
    f_alg = sum(alg_flops_per_step(k, n, P) for k in ("eig", "forward", "backward", "sterm")) * nt
    ach, frac = eig_roofline(r["ktimes"], n, P, nt, B)
    par = parity_vs_oracle(name, r["costs"], r["grads"], r["hess"])
    log(f"bench: {name}: {value:.1f} evals/s, parity {par['max_rel_err']:.2e}")
    return {"workload": f"{name}: N={n}, J={nt}, dt={w.dt}, Fourier K={w.k} (P={P}), {B} theta ~ N(0, 0.1^2)",
            "evals_per_s": value, "steps": steps, "ms_per_step": 1e3 * r["elapsed"] / steps,
            "kernel_ms": {k: round(v[0], 3) for k, v in r["ktimes"].items()},
            "path_alg_flops_per_eval": f_alg, "path_roofline_frac": f_alg * value / PEAK_FP64,
            "eig_roofline": {"achieved": ach, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": frac,
                             "bound": "alu"},
            "jacobi_sweeps_per_step": r["sweeps_per_step"], "parity": par}


WARM_MODEL = os.path.join(ROOT, "paper_2505_00529_amd", "data", "warm_c5_mlp.npz")


def tr_plain_vs_warm(count: int) -> dict:
    """Trust-region solves per second on the 64-level system (N=64, J=4000, K=32) for `count`
    held-out targets: from theta = 0 (plain) and from the learned warm start (network inference
    included), with the plain solve judging the final cost (same minimum within 1e-8)."""
    from paper_2505_00529_amd import warmstart as W

    w = inputs.make_workload("warm")
    prob = qoc.problem_from_workload(w, device=0)
    targets = inputs.warm_targets(w.system.n, count, spawn=1)
    ws = W.WarmStart.load(prob, WARM_MODEL)
    log(f"bench: {count} trust-region solves on the 64-level system, plain and warm-started ...")
    th, c, its, conv, ps = W.solve_plain(prob, targets, 1e-8, 1000)
    wr = ws.solve(targets, 1e-8, 1000)
    cmp = W.compare(c, wr["cost"])
    meta = np.load(WARM_MODEL)
    prob.close()
    log(f"bench: plain {count / ps:.2f} solves/s, warm {count / wr['seconds']:.2f} solves/s")
    return {"workload": "warm: N=64, J=4000, dt=0.02, Fourier K=32 (P=64); held-out targets in the lowest-8 "
                        "eigenspace", "solves": count,
            "plain": {"solves_per_s": count / ps, "seconds": ps, "iters_mean": float(its.mean()),
                      "converged": int(conv.sum())},
            "warm": {"solves_per_s": count / wr["seconds"], "seconds": wr["seconds"],
                     "iters_mean": float(wr["iters"].mean()), "converged": int(wr["converged"].sum()),
                     "fallback": int(wr["fallback"].sum())},
            "same_final_cost_1e-8": cmp["match"], "warm_lower": cmp["lower"], "warm_higher": cmp["higher"],
            "network": f"trained on the zero-start iterate after {int(meta['target_iters'])} iterations of "
                       f"{int(meta['train'])} training targets (paper_2505_00529_amd/data/warm_c5_mlp.npz)",
            "note": "gradient norm < 1e-8 on the controllable subspace; lockstep batches of 256"}


def run_batched(args) -> int:
    """Uneven-problem batch: 256 problems (N in {8,16,36,64,128}, J in [2000, 8000], K in
    {8,16,32}); one step = cost+grad+Hessian of every problem.  Batched (queue launches under a
    HIP graph, autotuned) against one launch sequence per problem."""
    import torch

    torch.cuda.set_device(0)
    ws = inputs.batched_workloads(args.count)
    log(f"bench: batched workload, {len(ws)} problems")
    probs = [qoc.problem_from_workload(w) for w in ws]
    b = qoc.Batch(probs)
    for p in probs:
        p.close()
    log(f"bench: batch workspace {b.memory() / 2**30:.1f} GiB")
    th = [inputs.draw_thetas(w.p, 1, 1000 + i)[0] for i, w in enumerate(ws)]
    f_alg = sum(sum(alg_flops_per_step(k, w.system.n, w.p) for k in ("eig", "forward", "backward", "sterm")) * w.nt
                for w in ws)
    if not args.no_autotune:
        t0 = time.perf_counter()
        b.autotune(th)
        log(f"bench: autotune {time.perf_counter() - t0:.1f} s")
    for i in range(args.warmup):
        b.hess(th)
        log(f"bench: warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    for i in range(args.steps):
        b.hess(th)
        dev_ms.append(b.last_ms())
        log(f"bench: batched step {i + 1}/{args.steps}: {dev_ms[-1]:.1f} ms")
    t1 = time.perf_counter()
    un_ms = []
    for i in range(args.unbatched_steps):
        b.hess_unbatched(th)
        un_ms.append(b.last_ms())
        log(f"bench: per-problem step {i + 1}/{args.unbatched_steps}: {un_ms[-1]:.1f} ms")
    elapsed = t1 - t0
    value = len(ws) * args.steps / elapsed
    achieved = f_alg * args.steps / (sum(dev_ms) * 1e-3) / 1e12
    out = {
        "metric": "aggregate grad+Hessian evals/s, 256 uneven problems",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {len(ws)} problems, N in {{8,16,36,64,128}}, J in [2000, 8000], "
                               "K in {8,16,32}, dt=0.02; one theta ~ N(0, 0.1^2) per problem",
                   "problems": len(ws), "parallelism": "single GPU"},
        "roofline": {"kernel": "whole batched path", "bound": "alu", "achieved": achieved, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / (PEAK_FP64 / 1e12), "traffic": None},
        "batched_device_ms": sorted(dev_ms)[len(dev_ms) // 2],
        "per_problem_device_ms": sorted(un_ms)[len(un_ms) // 2] if un_ms else None,
        "speedup_vs_per_problem": (sorted(un_ms)[len(un_ms) // 2] / sorted(dev_ms)[len(dev_ms) // 2]) if un_ms else None,
        "path_alg_flops_per_step": f_alg,
        "batch_workspace_bytes": b.memory(),
    }
    print(json.dumps(out), flush=True)
    b.close()
    return 0


def multi_flops_per_step(kernel: str, n: int, p: int, ndir: int) -> float:
    """Algorithmic FLOPs per (theta, time step) with ndir control directions: one
    eigendecomposition and ndir products M~_k = V^T M_k V; per direction one S_k mat-vec in each
    sweep beside the N x N . N x P tangent product; one U'' contraction per direction pair."""
    return {
        "eig": 9.0 * n ** 3 + 4.0 * ndir * n ** 3,
        "forward": 8.0 * n * n * p + 8.0 * ndir * n * n,
        "backward": 8.0 * n * n * p + 8.0 * ndir * n * n,
        "sterm": 8.0 * n ** 3 * ndir * (ndir + 1) / 2,
    }.get(kernel, 0.0)


def run_multi(args) -> int:
    """Three control directions (Sec. II with the x, y, z dipoles; the mixed second derivatives of
    eq. d2Ldf2): one step = cost + gradient + Hessian of a batch of theta on the molecule workload
    with two further dipole operators and a Fourier block of 32 parameters per direction
    (P = 96).  Rows 0 and 1 of the timed batch are checked against stored oracle values."""
    import torch

    torch.cuda.set_device(0)
    w, ms = inputs.multi_direction_workload()
    s = w.system
    ndir, n, nt, B = len(ms), w.system.n, w.nt, args.multi_batch
    prob = qoc.Problem(0)
    prob.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    prob.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, w.dt, w.k)
    prob.set_weights(w.gamma, w.rho)
    P = prob.P
    log(f"bench: three-direction workload n={n} nt={nt} P={P} batch={B}")
    stream = torch.cuda.current_stream()
    prob.set_stream(stream.cuda_stream)
    thetas = torch.tensor(inputs.draw_thetas(P, B, w.seed), dtype=torch.float64, device="cuda")
    r = timed_batch(prob, thetas, args.steps, args.warmup, stream, "multi")
    ktimes = r["ktimes"]
    dom = max(ktimes, key=lambda k: ktimes[k][0])
    achieved = multi_flops_per_step(dom, n, P, ndir) * nt * B / (ktimes[dom][0] * 1e-3) / 1e12
    peak = PEAK_FP64 / 1e12
    parity = parity_vs_oracle("multi", r["costs"], r["grads"], r["hess"])
    log(f"bench: parity of the timed batch against the oracle: max rel err {parity['max_rel_err']:.2e}")
    value = B * args.steps / r["elapsed"]
    f_alg = sum(multi_flops_per_step(k, n, P, ndir) for k in ("eig", "forward", "backward", "sterm")) * nt
    out = {
        "metric": f"grad+Hessian evals/s (FP64, N={n}, {ndir} control directions, P={P})",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"multi: molecule N={n}, J={nt}, dt={w.dt}, {ndir} dipole operators, Fourier "
                               f"K={w.k} per direction (P={P}), {B} independent theta ~ N(0, 0.1^2) per step",
                   "n": n, "nt": nt, "P": P, "directions": ndir, "batch": B, "parallelism": "single GPU"},
        "roofline": {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None},
        "kernel_ms": {k: round(v[0], 4) for k, v in ktimes.items()},
        "step_ms_median": float(np.median(r["step_ms"])),
        "jacobi_sweeps_per_step": r["sweeps_per_step"],
        "path_alg_flops_per_eval": f_alg,
        "path_roofline_frac": f_alg * value / PEAK_FP64,
        "parity": parity,
    }
    prob.close()
    if not args.no_cpu_baseline:
        from oracle import qoc_oracle as O
        from threadpoolctl import threadpool_info

        log("bench: timing the CPU oracle on a sample of one theta ...")
        threads = max([int(x.get("num_threads", 1)) for x in threadpool_info()] or [1])
        ns = min(args.multi_oracle_steps, nt)
        b0 = O.fourier_basis(nt, w.dt, w.k)[:ns]
        p0 = b0.shape[1]
        bases = np.zeros((ndir, ns, ndir * p0))
        for c in range(ndir):
            bases[c, :, c * p0:(c + 1) * p0] = b0
        th = inputs.draw_thetas(P, 1, w.seed)[0]
        t0 = time.perf_counter()
        O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, w.dt, th, w.gamma, w.rho)
        dt_s = (time.perf_counter() - t0) * nt / ns
        out["cpu_baseline"] = {"value": 1.0 / dt_s, "unit": "evals/s", "cores": threads, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"the first {ns} of the {nt} steps of one theta (cost+grad+Hessian, "
                                         f"{ndir} directions, P={P}) on {threads} BLAS threads, "
                                         f"{dt_s * ns / nt:.1f} s, scaled to the full horizon"}
    print(json.dumps(out), flush=True)
    if not parity["ok"]:
        log(f"bench: PARITY FAILURE: max rel err {parity['max_rel_err']:.3e} above {PARITY_TOL:g}")
        return 1
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["molecule", "warm", "batched", "multi"], default="molecule",
                    help="molecule: the headline evals/s line (N=36, P=32); warm: the 64-level system "
                         "(N=64, P=64); batched: 256 uneven problems; multi: three control directions "
                         "(N=36, P=96)")
    ap.add_argument("--multi-batch", type=int, default=256, help="theta per step of the multi workload")
    ap.add_argument("--multi-oracle-steps", type=int, default=400,
                    help="steps of the multi workload's oracle sample (its time is linear in the steps)")
    ap.add_argument("--n64-steps", type=int, default=4,
                    help="with the molecule workload, also time this many steps of the 64-level system "
                         "(256 theta) and report them beside the headline (0: skip)")
    ap.add_argument("--count", type=int, default=256, help="problems in the batched workload")
    ap.add_argument("--unbatched-steps", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=256, help="independent theta per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-calls", type=int, default=30, help="single-theta calls timed for the latency")
    ap.add_argument("--tr-solves", type=int, default=32, help="plain trust-region solves timed after the steps")
    ap.add_argument("--tr-warm", type=int, default=128,
                    help="held-out targets of the 64-level system solved plain and warm-started (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB (a reference "
                         "dispatch of known traffic for HBM byte counters; use more than the last-level "
                         "cache so that its source is read from HBM)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU only (one process, one MI355X); "
              "--gpus above 1 is not supported", file=sys.stderr)
        return 2

    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "multi":
        return run_multi(args)

    import torch

    torch.cuda.set_device(0)
    wl = args.workload
    w = inputs.make_workload(wl)
    n, P, nt, B = w.system.n, w.p, w.nt, args.batch
    log(f"bench: workload {wl} n={n} nt={nt} P={P} batch={B}")
    prob = qoc.problem_from_workload(w, device=0)
    stream = torch.cuda.current_stream()
    prob.set_stream(stream.cuda_stream)

    thetas = torch.tensor(inputs.draw_thetas(P, B, w.seed), dtype=torch.float64, device="cuda")
    r = timed_batch(prob, thetas, args.steps, args.warmup, stream, wl)
    t0, t1 = 0.0, r["elapsed"]
    step_ms, ktimes = r["step_ms"], r["ktimes"]
    eig_sweeps_per_step = r["sweeps_per_step"]
    dom = max(ktimes, key=lambda k: ktimes[k][0])
    avg_ms = ktimes[dom][0]
    flops_launch = alg_flops_per_step(dom, n, P) * nt * B
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_FP64 / 1e12

    h, c_np, g_np = r["hess"], r["costs"], r["grads"]
    assert np.all(np.isfinite(h)) and np.all(np.isfinite(c_np))
    parity = parity_vs_oracle(wl, c_np, g_np, h)
    log(f"bench: parity of the timed batch against the oracle: max rel err {parity['max_rel_err']:.2e}")

    # single-problem latency (B = 1) on its own handle, so the batch workspace stays in place
    single = qoc.problem_from_workload(w, device=0)
    single.set_stream(stream.cuda_stream)
    th1 = thetas[:1].clone()
    c1 = torch.empty(1, dtype=torch.float64, device="cuda")
    g1 = torch.empty(1, P, dtype=torch.float64, device="cuda")
    h1 = torch.empty(1, P, P, dtype=torch.float64, device="cuda")
    n_lat = max(args.latency_calls, 1)
    for _ in range(3):
        single.hess_many_dev(1, th1.data_ptr(), c1.data_ptr(), g1.data_ptr(), h1.data_ptr())
    single.sync()
    lev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * n_lat)]
    for i in range(n_lat):
        lev[2 * i].record(stream)
        single.hess_many_dev(1, th1.data_ptr(), c1.data_ptr(), g1.data_ptr(), h1.data_ptr())
        lev[2 * i + 1].record(stream)
    single.sync()
    lat_ms = np.array([lev[2 * i].elapsed_time(lev[2 * i + 1]) for i in range(n_lat)])
    th1_host = th1.cpu().numpy()[0]
    hw = []
    for _ in range(5):
        ta = time.perf_counter()
        single.hess(th1_host)
        hw.append(time.perf_counter() - ta)
    single.close()
    latency = {"ms_median": float(np.median(lat_ms)),
               "ms_iqr": [float(np.percentile(lat_ms, 25)), float(np.percentile(lat_ms, 75))],
               "calls": n_lat, "evals_per_s": 1e3 / float(np.median(lat_ms)),
               "path_roofline_frac": None,
               "host_wall_ms_per_abi_call": 1e3 * float(np.median(hw))}
    log(f"bench: single-theta latency {latency['ms_median']:.2f} ms (device), "
        f"{latency['host_wall_ms_per_abi_call']:.2f} ms per host ABI call")

    # gradient only (cost + adjoint gradient, same thetas): the Hessian-to-gradient time ratio
    th_host = thetas.cpu().numpy()
    prob.grad_many(th_host)
    g_steps = max(1, min(args.steps, 3))
    tg0 = time.perf_counter()
    for _ in range(g_steps):
        prob.grad_many(th_host)
    tg = (time.perf_counter() - tg0) / g_steps
    log(f"bench: gradient-only {tg * 1e3:.1f} ms per batch")

    # plain trust-region solves from theta = 0 on per-theta targets of the same system
    tr = None
    if args.tr_solves > 0:
        tgs = inputs.warm_targets(n, args.tr_solves, spawn=2, dim=6)
        tt0 = time.perf_counter()
        th_out, _, its, conv = prob.tr_solve_many(np.zeros((args.tr_solves, P)), tgs, gtol=1e-8, max_iter=1000)
        tt = time.perf_counter() - tt0
        _, g_out, _ = prob.hess_many_targets(th_out, tgs)
        gn, pn = prob.gradient_norms(g_out)
        tr = {"solves": args.tr_solves, "seconds": tt, "solves_per_s": args.tr_solves / tt,
              "iters_mean": float(its.mean()), "iters_median": float(np.median(its)),
              "converged": int(conv.sum()),
              "grad_norm_max": float(gn.max()), "grad_norm_median": float(np.median(gn)),
              "projected_grad_norm_max": float(pn.max()),
              "below_1e-8_grad_norm": int((gn < 1e-8).sum()),
              "below_1e-8_projected": int((pn < 1e-8).sum()),
              "note": "zero start; 'converged' counts ||V_r^T g||_2 < 1e-8 (the directions of the control "
                      "basis with singular value above 1e-7 of the largest); ||g||_2 reported beside it; "
                      "lockstep batch"}
        log(f"bench: {args.tr_solves} trust-region solves in {tt:.1f} s")

    elapsed = t1 - t0
    value = B * args.steps / elapsed
    f_alg = sum(alg_flops_per_step(k, n, P) for k in ("eig", "forward", "backward", "sterm")) * nt
    out = {
        "metric": f"grad+Hessian evals/s (FP64, N={n}, P={P})",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{wl}: N={n}, J={nt}, dt={w.dt}, Fourier K={w.k} (P={P}), "
                        f"{B} independent theta ~ N(0, 0.1^2) per step",
            "n": n, "nt": nt, "P": P, "batch": B, "parallelism": "single GPU",
        },
        "roofline": {
            "kernel": dom,
            "bound": "alu" if dom == "eig" else "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(dom, B),
        },
        "kernel_ms": {k: round(v[0], 4) for k, v in ktimes.items()},
        "step_ms_median": float(np.median(step_ms)),
        "step_ms_iqr": [float(np.percentile(step_ms, 25)), float(np.percentile(step_ms, 75))],
        "grad_only_evals_per_s": B / tg,
        "hess_to_grad_time_ratio": (elapsed / args.steps) / tg,
        "tr_plain": tr,
        "jacobi_sweeps_per_step": eig_sweeps_per_step,
        "path_alg_flops_per_eval": f_alg,
        "path_roofline_frac": f_alg * value / PEAK_FP64,
        "parity": parity,
        "single_theta_latency": latency,
    }
    latency["path_roofline_frac"] = f_alg * latency["evals_per_s"] / PEAK_FP64
    if args.calib_copy_mib > 0:
        nel = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = int(nel * 8)
        del src, dst
    prob.close()
    if wl == "molecule" and args.n64_steps > 0:
        out["n64_system"] = secondary_system("warm", 256, args.n64_steps, stream)
        if not out["n64_system"]["parity"]["ok"]:
            parity["ok"] = False
    if args.tr_warm > 0:
        out["tr_solves_per_s_plain_vs_warm"] = tr_plain_vs_warm(args.tr_warm)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on one theta ...")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)
    if not parity["ok"]:
        log(f"bench: PARITY FAILURE: max rel err {parity['max_rel_err']:.3e} above {PARITY_TOL:g}")
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
