"""Wall time of one gradient evaluation (Alg. 1) and of one gradient + Hessian evaluation (Alg. 2)
against the number of time steps J, on the paper's timing protocol (Sec. IV-A, Fig. 1).

Protocol: maximal model f_j = theta_j (P = J), J = 2^kappa for kappa = 2..10, theta ~ N(0, I) drawn
afresh for every trial, alpha = e_0 and beta = e_{N-1}; both evaluations run on the same theta, in
turn, through the host-pointer C ABI (inputs on the host, results back on the host), after one
untimed call per (N, J) that sizes the workspaces.  Systems: N = 4 and 16 stand in for the paper's
full-CI molecules (the real transfer systems of the optimiser comparison); N = 64 and 144 use a
random diagonal H0 and a random complex Hermitian M, evaluated through the real embedding of size
128 and 288.
The time step is 0.1 and the weights 1 and rho = 1e6, as in the optimiser comparison (the paper
states neither for its timing runs; they do not change the work).  With theta ~ N(0, I) consecutive
steps are far apart, so warm-started eigen chains save little: by default every step is its own
chain (--chunk 1), decomposed from scratch and in parallel with the others.

Reported per (N, J): mean and standard deviation of both wall times over the trials and their
ratio; per N, the OLS slopes of log2(mean time) against log2(J) for both algorithms.

    python -m paper_2505_00529_amd.jscaling [--n 4 16 64 144] [--trials 1000] [--trials-large 100]
                                            [--trials-xl 10] [--kmax 10]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs
from . import qoc

DT, RHO = 0.1, 1e6


def _say(msg: str) -> None:
    print(f"[jscaling] {msg}", flush=True)


def make_problem(n: int, nt: int, chunk: int = 0, device: int = 0) -> qoc.Problem:
    p = qoc.Problem(device)
    p.set_eig_chunk(chunk)
    if n >= 64:
        s = inputs.hermitian_system(n)
        p.set_system_hermitian(s.h0, s.m, s.psi0, s.psi_target)
    else:
        s = inputs.transfer_system(n)
        p.set_system(s.h0, s.m, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_IDENTITY, nt, DT, 0)
    p.set_weights(1.0, RHO)
    return p


def time_pair(p: qoc.Problem, nt: int, trials: int, seed: int):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, nt])))
    p.grad(rng.normal(size=nt))
    p.hess(rng.normal(size=nt))
    tg = np.zeros(trials)
    th = np.zeros(trials)
    for i in range(trials):
        theta = rng.normal(size=nt)
        t0 = time.perf_counter()
        p.grad(theta)
        t1 = time.perf_counter()
        p.hess(theta)
        t2 = time.perf_counter()
        tg[i], th[i] = t1 - t0, t2 - t1
    return tg, th


def ols_slope(x: np.ndarray, y: np.ndarray) -> float:
    a = np.vstack([x, np.ones_like(x)]).T
    return float(np.linalg.lstsq(a, y, rcond=None)[0][0])


def run(n: int, kmin: int, kmax: int, trials: int, seed: int, chunk: int = 0) -> dict:
    rows = []
    for kappa in range(kmin, kmax + 1):
        nt = 2 ** kappa
        p = make_problem(n, nt, chunk)
        tg, th = time_pair(p, nt, trials, seed)
        p.close()
        rows.append({"J": nt, "grad_ms_mean": 1e3 * tg.mean(), "grad_ms_std": 1e3 * tg.std(),
                     "hess_ms_mean": 1e3 * th.mean(), "hess_ms_std": 1e3 * th.std(),
                     "hess_over_grad": float(th.mean() / tg.mean())})
        _say(f"N={n} J={nt} chain {chunk}: gradient {1e3 * tg.mean():.3f} ms, gradient + Hessian {1e3 * th.mean():.3f} ms")
    lj = np.log2([r["J"] for r in rows])
    return {"n": n, "complex_hermitian": n >= 64, "trials": trials, "eig_chunk": chunk, "rows": rows,
            "ols_slope_alg1_grad": ols_slope(lj, np.log2([r["grad_ms_mean"] for r in rows])),
            "ols_slope_alg2_hess": ols_slope(lj, np.log2([r["hess_ms_mean"] for r in rows]))}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, nargs="+", default=[4, 16, 64, 144])
    ap.add_argument("--trials", type=int, default=1000)
    ap.add_argument("--trials-large", type=int, default=100,
                    help="trials per J for the complex N = 64 system (its evaluations take 5-220 ms)")
    ap.add_argument("--trials-xl", type=int, default=10,
                    help="trials per J for complex N > 64 (N = 144: 0.27-4 s per evaluation)")
    ap.add_argument("--kmin", type=int, default=2)
    ap.add_argument("--kmax", type=int, default=10)
    ap.add_argument("--seed", type=int, default=14)
    ap.add_argument("--chunk", type=int, default=1,
                    help="length of the warm-started eigen chains (0: automatic; 1: every step from "
                         "scratch and in parallel, the better choice when the steps are cold anyway)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    def trials(n):
        return a.trials if n < 64 else (a.trials_large if n == 64 else a.trials_xl)

    res = [run(n, a.kmin, a.kmax, trials(n), a.seed, a.chunk) for n in a.n]
    line = json.dumps({"protocol": "J scaling of one evaluation, maximal model", "dt": DT, "rho": RHO,
                       "systems": res})
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
