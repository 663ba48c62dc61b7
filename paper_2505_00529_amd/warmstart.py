"""Learned warm start for the exact-Hessian trust-region solver.

A small network (``n_in = 2n`` target features -> 512 -> 512 -> P, erf-GELU between) proposes
the starting control for a new target state.  It is trained on optimal controls that the
trust-region solver itself produced from the zero start, and it runs entirely in the library's
BF16 matrix-core kernels (``qoc_mlp_*``: forward, backward and Adam, FP32 accumulation and
master weights).  The network regresses the trust-region metric coordinates
c = diag(sigma_r) V_r^T theta (``qoc_control_coords``), which are isometric to the sampled
control f = B theta; a half-period Fourier basis is numerically rank-deficient, so the raw
coefficients are not identifiable and make poor regression targets.

The regression target is the zero-start solver's own iterate after k iterations (k =
``target_iters``; 0 means the final optimum).  The optimum reached from theta = 0 is a
discontinuous function of the target (the plain solve lands in one of many nearby local
minima), so it cannot be learned from a few thousand samples; the early iterate is a smooth
function of the target away from the few targets where a ratio test decides differently, and a
warm solve started close to it continues along the plain solve's path into the same minimum,
skipping about k iterations.

The plain zero-start solve stays the reference and the fallback: a warm solve that does not
converge is rerun from theta = 0, and its final cost is compared with the plain solve's.

Command line (one GPU): ``python -m paper_2505_00529_amd.warmstart --train 2000 --test 200``
generates the training set, trains, and reports iterations, wall time and cost agreement of
plain against warm-started solves on held-out targets as one JSON line.
"""
from __future__ import annotations

import argparse
import json
import time
from typing import Optional

import numpy as np

from . import qoc


def target_features(targets) -> np.ndarray:
    """(count, n) complex targets -> (count, 2n) float32 [Re beta, Im beta]."""
    t = np.asarray(targets, dtype=np.complex128)
    return np.concatenate([t.real, t.imag], axis=1).astype(np.float32)


def init_params(n_in: int, n_hidden: int, n_out: int, seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, packed like qoc_mlp."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_out, fan_in in ((n_hidden, n_in), (n_hidden, n_hidden), (n_out, n_hidden)):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, size=fan_out * fan_in))
        parts.append(rng.uniform(-b, b, size=fan_out))
    return np.concatenate(parts).astype(np.float32)


class WarmStart:
    """Network + output normalisation for one configured problem (system, basis, weights)."""

    def __init__(self, problem: "qoc.Problem", n_hidden: int = 512, max_batch: int = 256, seed: int = 0):
        self.problem = problem
        self.n_in = 2 * problem.n
        self.n_out = problem.P
        self.max_batch = max_batch
        self.mlp = qoc.Mlp(self.n_in, n_hidden, self.n_out, max_batch)
        self.mlp.set_params(init_params(self.n_in, n_hidden, self.n_out, seed))
        self.mean = np.zeros(self.n_out)
        self.scale = np.ones(self.n_out)
        self.rank = self.n_out

    # -- training
    def fit(self, targets, thetas, epochs: int = 200, lr: float = 1e-3, batch: int = 128, seed: int = 0,
            lr_final: float = 1e-5, verbose: bool = False):
        """Train on (target, optimal theta) pairs; returns the mean loss of each epoch."""
        import torch

        coords, self.rank = self.problem.control_coords(thetas)
        self.mean = coords.mean(axis=0)
        sd = coords.std(axis=0)
        self.scale = np.where(sd > 1e-12, sd, 1.0)
        y = ((coords - self.mean) / self.scale).astype(np.float32)
        x = target_features(targets)
        xd = torch.from_numpy(x).cuda()
        yd = torch.from_numpy(y).cuda()
        loss = torch.zeros((), dtype=torch.float32, device="cuda")
        rng = np.random.Generator(np.random.PCG64(seed))
        batch = min(batch, self.max_batch)
        count = x.shape[0]
        history = []
        steps_per_epoch = max(1, count // batch)
        total = epochs * steps_per_epoch
        step = 0
        for _ in range(epochs):
            perm = torch.from_numpy(rng.permutation(count)).cuda()
            xs = xd.index_select(0, perm).contiguous()
            ys = yd.index_select(0, perm).contiguous()
            acc = 0.0
            for k in range(steps_per_epoch):
                # cosine decay from lr to lr_final
                cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * step / total))
                xb = xs[k * batch:(k + 1) * batch]
                yb = ys[k * batch:(k + 1) * batch]
                self.mlp.train_step(batch, xb.data_ptr(), yb.data_ptr(), float(cur), loss_ptr=loss.data_ptr())
                acc += loss.item()
                step += 1
            history.append(acc / steps_per_epoch)
            if verbose and len(history) % 50 == 0:
                print(f"[warmstart]   epoch {len(history)}/{epochs}: loss {history[-1]:.4f}", flush=True)
        return history

    # -- persistence
    def save(self, path: str, **extra):
        """Trained parameters and output normalisation (.npz)."""
        np.savez_compressed(path, params=self.mlp.get_params(), mean=self.mean, scale=self.scale,
                            rank=np.int64(self.rank), n_hidden=np.int64(self.mlp.n_hidden), **extra)

    @classmethod
    def load(cls, problem: "qoc.Problem", path: str, max_batch: int = 256) -> "WarmStart":
        d = np.load(path)
        ws = cls(problem, n_hidden=int(d["n_hidden"]), max_batch=max_batch)
        ws.mlp.set_params(d["params"])
        ws.mean, ws.scale, ws.rank = d["mean"], d["scale"], int(d["rank"])
        return ws

    # -- inference
    def predict_coords(self, targets) -> np.ndarray:
        import torch

        x = torch.from_numpy(target_features(targets)).cuda()
        count = x.shape[0]
        y = torch.empty((count, self.n_out), dtype=torch.float32, device="cuda")
        for s in range(0, count, self.max_batch):
            e = min(count, s + self.max_batch)
            xb = x[s:e].contiguous()
            yb = torch.empty((e - s, self.n_out), dtype=torch.float32, device="cuda")
            self.mlp.forward(e - s, xb.data_ptr(), yb.data_ptr())
            y[s:e] = yb
        c = y.cpu().numpy().astype(np.float64) * self.scale + self.mean
        c[:, self.rank:] = 0.0
        return c

    def predict(self, targets) -> np.ndarray:
        """Starting parameters theta_0 (count x P) for the given targets."""
        return self.problem.params_from_coords(self.predict_coords(targets))

    def solve(self, targets, gtol: float = 1e-8, max_iter: int = 10000, chunk: int = 256, verbose: bool = False):
        """Warm-started solves with the zero-start fallback, in lockstep chunks of `chunk` targets.
        Returns a dict of per-target arrays (theta, cost, iters, converged, fallback) and the wall
        time (network inference included)."""
        targets = np.asarray(targets)
        count = targets.shape[0]
        t0 = time.perf_counter()
        th0 = self.predict(targets)
        th = np.zeros((count, self.n_out))
        c = np.zeros(count)
        its = np.zeros(count, dtype=np.int32)
        conv = np.zeros(count, dtype=bool)
        for s in range(0, count, chunk):
            e = min(count, s + chunk)
            th[s:e], c[s:e], its[s:e], conv[s:e] = self.problem.tr_solve_many(th0[s:e], targets[s:e], gtol=gtol,
                                                                              max_iter=max_iter)
            if verbose:
                print(f"[warmstart]   warm solved {e}/{count} ({time.perf_counter() - t0:.1f} s)", flush=True)
        fb = ~conv
        if fb.any():
            idx = np.flatnonzero(fb)
            th2, c2, its2, conv2 = solve_plain(self.problem, targets[idx], gtol, max_iter, chunk)[:4]
            th[idx], c[idx], conv[idx] = th2, c2, conv2
            its[idx] += its2
        return dict(theta=th, cost=c, iters=its, converged=conv, fallback=fb, seconds=time.perf_counter() - t0)


def early_iterates(problem: "qoc.Problem", targets, k: int, gtol: float = 1e-8, chunk: int = 256):
    """The zero-start trust-region iterate after k iterations for every target (the solver is
    deterministic, so this is the plain solve's own path; a solve that converges earlier gives
    its optimum)."""
    return solve_plain(problem, targets, gtol, k, chunk)


def solve_plain(problem: "qoc.Problem", targets, gtol: float = 1e-8, max_iter: int = 10000, chunk: int = 256,
                verbose: bool = False):
    """Zero-start solves in lockstep chunks; returns (theta, cost, iters, converged, seconds)."""
    targets = np.asarray(targets)
    count = targets.shape[0]
    th = np.zeros((count, problem.P))
    c = np.zeros(count)
    its = np.zeros(count, dtype=np.int32)
    conv = np.zeros(count, dtype=bool)
    t0 = time.perf_counter()
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        th[s:e], c[s:e], its[s:e], conv[s:e] = problem.tr_solve_many(np.zeros((e - s, problem.P)), targets[s:e],
                                                                      gtol=gtol, max_iter=max_iter)
        if verbose:
            print(f"[warmstart]   solved {e}/{count} ({time.perf_counter() - t0:.1f} s)", flush=True)
    return th, c, its, conv, time.perf_counter() - t0


def regression_baselines(problem: "qoc.Problem", train_targets, train_thetas, test_targets, test_thetas) -> dict:
    """How well plain regressors predict the network's regression target from the target state,
    in the same metric coordinates: median relative error on the held-out targets of the
    training mean, ridge regression (linear and quadratic features) and k-nearest neighbours.
    A map no better than the mean is not learnable from that many samples."""
    from sklearn.linear_model import Ridge
    from sklearn.neighbors import KNeighborsRegressor

    def feats(t):
        return target_features(t).astype(np.float64)

    def quad(x):
        iu = np.triu_indices(x.shape[1])
        return np.concatenate([x, (x[:, :, None] * x[:, None, :])[:, iu[0], iu[1]]], axis=1)

    ctr, r = problem.control_coords(train_thetas)
    cte, _ = problem.control_coords(test_thetas)
    ctr, cte = ctr[:, :r], cte[:, :r]
    xtr, xte = feats(train_targets), feats(test_targets)
    keep = np.abs(xtr).max(axis=0) > 0   # the target's nonzero components
    xtr, xte = xtr[:, keep], xte[:, keep]

    def err(pred):
        return float(np.median(np.linalg.norm(pred - cte, axis=1) / np.linalg.norm(cte, axis=1)))

    out = {"mean": err(np.tile(ctr.mean(axis=0), (cte.shape[0], 1))),
           "ridge": err(Ridge(alpha=1e-3).fit(xtr, ctr).predict(xte)),
           "ridge_quadratic": err(Ridge(alpha=1e-3).fit(quad(xtr), ctr).predict(quad(xte)))}
    for k in (1, 5, 20):
        out[f"knn{k}"] = err(KNeighborsRegressor(k).fit(xtr, ctr).predict(xte))
    return out


def compare(plain_cost, warm_cost, tol: float = 1e-8) -> dict:
    """Same final cost within tol counts as a match; otherwise a miss, reported as lower or higher."""
    d = np.asarray(warm_cost) - np.asarray(plain_cost)
    return dict(match=int((np.abs(d) <= tol).sum()), lower=int((d < -tol).sum()), higher=int((d > tol).sum()),
                max_abs_diff_matched=float(np.abs(d[np.abs(d) <= tol]).max()) if (np.abs(d) <= tol).any() else None)


def main(argv: Optional[list] = None):
    from . import inputs

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="warm")
    ap.add_argument("--n", type=int, default=None, help="override the system dimension of the workload")
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--gtol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--target-iters", type=int, default=8,
                    help="regress the zero-start iterate after this many iterations (0: the final optimum)")
    ap.add_argument("--save", default=None, help="write the training set and trained parameters (.npz)")
    ap.add_argument("--load", default=None, help="training set from an earlier --save instead of solving")
    ap.add_argument("--save-model", default=None, help="write only the trained network (.npz, for WarmStart.load)")
    args = ap.parse_args(argv)

    w = inputs.make_workload(args.workload, n=args.n)
    p = qoc.problem_from_workload(w)
    tr_t = inputs.warm_targets(w.system.n, args.train, spawn=0)
    te_t = inputs.warm_targets(w.system.n, args.test, spawn=1)
    if args.load:
        d = np.load(args.load)
        tr_t, tr_th, tr_c, tr_it = d["train_targets"], d["train_thetas"], d["train_costs"], d["train_iters"]
        tr_conv = d["train_converged"].astype(bool) if "train_converged" in d else np.ones(len(tr_t), bool)
        tr_s = float(d["train_seconds"]) if "train_seconds" in d else 0.0
        args.train = len(tr_t)
        print(f"[warmstart] loaded {args.train} training pairs from {args.load}", flush=True)
    else:
        k = args.target_iters
        print(f"[warmstart] {args.workload}: n={w.system.n} nt={w.nt} P={w.p}; "
              + (f"zero-start iterates after {k} iterations for" if k > 0 else "solving")
              + f" {args.train} training targets", flush=True)
        tr_th, tr_c, tr_it, tr_conv, tr_s = solve_plain(p, tr_t, args.gtol, k if k > 0 else args.max_iter,
                                                        verbose=True)
        if k > 0:
            tr_conv = np.ones(args.train, dtype=bool)   # an early iterate is a target whether or not converged
    print(f"[warmstart] training set: {tr_s:.1f} s, mean iters {tr_it.mean():.1f}", flush=True)
    ws = WarmStart(p)
    t0 = time.perf_counter()
    hist = ws.fit(tr_t[tr_conv], tr_th[tr_conv], epochs=args.epochs, lr=args.lr, batch=args.batch, verbose=True)
    fit_s = time.perf_counter() - t0
    print(f"[warmstart] trained {args.epochs} epochs in {fit_s:.1f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}",
          flush=True)
    pl_th, pl_c, pl_it, pl_conv, pl_s = solve_plain(p, te_t, args.gtol, args.max_iter, verbose=True)
    print(f"[warmstart] plain held-out: {pl_s:.1f} s, mean iters {pl_it.mean():.1f}", flush=True)
    wr = ws.solve(te_t, args.gtol, args.max_iter, verbose=True)
    print(f"[warmstart] warm held-out: {wr['seconds']:.1f} s, mean iters {wr['iters'].mean():.1f}", flush=True)
    cmp = compare(pl_c, wr["cost"])
    # the held-out values of the regression target: early iterates, or the plain optima
    ref_th = early_iterates(p, te_t, args.target_iters, args.gtol)[0] if args.target_iters > 0 else pl_th
    print("[warmstart] regression baselines ...", flush=True)
    base = regression_baselines(p, tr_t[tr_conv], tr_th[tr_conv], te_t, ref_th)
    pred_c = ws.predict_coords(te_t)
    true_c, _ = p.control_coords(ref_th)
    out = dict(
        workload=args.workload, n=w.system.n, nt=w.nt, P=w.p, rank=ws.rank, train=args.train, test=args.test,
        target_iters=args.target_iters,
        train_converged=int(tr_conv.sum()), train_seconds=round(tr_s, 2), fit_seconds=round(fit_s, 2),
        loss_first=hist[0], loss_last=hist[-1],
        coord_rel_err_median=float(np.median(np.linalg.norm(pred_c - true_c, axis=1) / np.linalg.norm(true_c, axis=1))),
        plain=dict(seconds=round(pl_s, 3), solves_per_s=args.test / pl_s, iters_mean=float(pl_it.mean()),
                   iters_median=float(np.median(pl_it)), converged=int(pl_conv.sum())),
        warm=dict(seconds=round(wr["seconds"], 3), solves_per_s=args.test / wr["seconds"],
                  iters_mean=float(wr["iters"].mean()), iters_median=float(np.median(wr["iters"])),
                  converged=int(wr["converged"].sum()), fallback=int(wr["fallback"].sum())),
        cost_agreement=cmp,
        regression_baselines_rel_err=base,
    )
    print(json.dumps(out), flush=True)
    if args.save:
        np.savez(args.save, train_targets=tr_t, train_thetas=tr_th, train_costs=tr_c, train_iters=tr_it,
                 train_converged=tr_conv, train_seconds=tr_s, params=ws.mlp.get_params(), mean=ws.mean,
                 scale=ws.scale, rank=ws.rank, target_iters=args.target_iters)
    if args.save_model:
        ws.save(args.save_model, target_iters=np.int64(args.target_iters), train=np.int64(args.train))
    return out


if __name__ == "__main__":
    main()
