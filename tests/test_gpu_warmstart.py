"""Learned warm start: trained on solver-generated optima, it must cut trust-region iterations on
held-out targets while the zero-start solve stays the reference for the final cost."""
import sys

import numpy as np
import pytest

from paper_2505_00529_amd import inputs, qoc
from paper_2505_00529_amd import warmstart as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_control_coords_round_trip_and_isometry():
    w = inputs.make_workload("warm", n=8, nt=300, k=8)
    p = qoc.problem_from_workload(w)
    th = inputs.draw_thetas(w.p, 5, 9, sigma=0.3)
    c, r = p.control_coords(th)
    assert 0 < r <= w.p and np.all(c[:, r:] == 0.0)
    back = p.params_from_coords(c)
    c2, _ = p.control_coords(back)
    assert np.abs(c2 - c).max() < 1e-10 * np.abs(c).max()
    # same sampled control, hence the same cost, from the minimum-norm representative
    for i in range(2):
        assert abs(p.cost(back[i]) - p.cost(th[i])) < 1e-9
    # ||c|| equals ||B theta||: the field-energy term of the cost with rho = 0 is (gamma/2) ||c||^2
    p.set_weights(w.gamma, 0.0)
    for i in range(2):
        assert abs(p.cost(th[i]) - 0.5 * w.gamma * np.dot(c[i], c[i])) < 1e-10 * p.cost(th[i])
    p.close()


def test_warm_start_reduces_iterations_with_same_final_cost():
    w = inputs.make_workload("warm", n=16, nt=400, k=8)
    p = qoc.problem_from_workload(w)
    tr = inputs.warm_targets(w.system.n, 192, spawn=0)
    te = inputs.warm_targets(w.system.n, 48, spawn=1)
    _say(f"warm start test: n={w.system.n} nt={w.nt} P={w.p}")
    th, c, its, conv = W.solve_plain(p, tr, max_iter=500)[:4]
    _say(f"  training solves: converged {conv.sum()}/{conv.size}, mean iters {its.mean():.1f}")
    assert conv.mean() > 0.95
    ws = W.WarmStart(p, max_batch=64)
    hist = ws.fit(tr[conv], th[conv], epochs=300, lr=2e-3, batch=32)
    _say(f"  loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    assert hist[-1] < 0.2 * hist[0]
    pth, pc, pit, pconv, _ = W.solve_plain(p, te, max_iter=500)
    wr = ws.solve(te, max_iter=500)
    cmp = W.compare(pc, wr["cost"])
    _say(f"  plain mean iters {pit.mean():.2f}, warm {wr['iters'].mean():.2f}, fallback {wr['fallback'].sum()}, "
         f"cost agreement {cmp}")
    assert wr["converged"].all()
    assert wr["iters"].mean() < pit.mean()
    # the two starts may end in different local minima (a miss); most land in the same one
    assert cmp["match"] >= 0.75 * te.shape[0]
    p.close()
