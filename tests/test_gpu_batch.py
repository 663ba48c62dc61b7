"""Batched evaluation of uneven problems (persistent queue launches under a HIP graph) against
per-problem launches and the oracle; graph replays; autotuner."""
import sys

import numpy as np
import pytest

from oracle import qoc_oracle as O
from paper_2505_00529_amd import inputs, qoc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _small_batch(count=12, seed=31):
    # uneven shapes covering every eigen kernel variant (wave 4/8/16/36, block kernel at
    # odd n, 64 and 128) and both sweep variants, with short horizons
    ws = inputs.batched_workloads(count, seed=seed, sizes=(4, 5, 8, 16, 36, 64, 128), nt_range=(40, 160),
                                  ks=(1, 2, 4, 8))
    return ws


def _make(ws):
    probs = [qoc.problem_from_workload(w) for w in ws]
    return probs, qoc.Batch(probs)


def test_batched_matches_per_problem_and_oracle():
    ws = _small_batch()
    _say("shapes: " + ", ".join(f"(n={w.system.n}, J={w.nt}, P={w.p})" for w in ws))
    probs, b = _make(ws)
    th = [inputs.draw_thetas(w.p, 1, 100 + i, sigma=0.3)[0] for i, w in enumerate(ws)]
    c, g, h = b.hess(th)
    cu, gu, hu = b.hess_unbatched(th)
    for i, w in enumerate(ws):
        assert _rel(c[i], cu[i]) < 1e-13 and _rel(g[i], gu[i]) < 1e-13 and _rel(h[i], hu[i]) < 1e-13, i
        # the handle's own path agrees too (its eigen chunking differs, so only to rounding)
        ci, gi, hi = probs[i].hess(th[i])
        assert _rel(c[i], ci) < 1e-10 and _rel(g[i], gi) < 1e-10 and _rel(h[i], hi) < 1e-10, i
    for i in range(len(ws)):
        w = ws[i]
        s = w.system
        basis = O.fourier_basis(w.nt, w.dt, w.k)
        cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th[i], w.gamma, w.rho)
        _say(f"  problem {i} n={s.n}: dC={_rel(c[i], cr):.2e} dg={_rel(g[i], gr):.2e} dH={_rel(h[i], hr):.2e}")
        assert _rel(c[i], cr) < 1e-10 and _rel(g[i], gr) < 1e-10 and _rel(h[i], hr) < 1e-10
    b.close()
    for p in probs:
        p.close()


def test_graph_replays_with_changing_inputs():
    ws = _small_batch(8, seed=32)
    probs, b = _make(ws)
    for rep in range(3):
        th = [inputs.draw_thetas(w.p, 1, 200 + 10 * rep + i, sigma=0.2)[0] for i, w in enumerate(ws)]
        c, g, h = b.hess(th)
        # eager work between replays
        cu, gu, hu = b.hess_unbatched(th)
        errs = [max(_rel(c[i], cu[i]), _rel(g[i], gu[i]), _rel(h[i], hu[i])) for i in range(len(ws))]
        _say(f"  replay {rep}: max rel diff to per-problem launches {max(errs):.2e}")
        assert max(errs) < 1e-13
    b.close()
    for p in probs:
        p.close()


def test_autotune_changes_nothing_but_speed():
    ws = _small_batch(10, seed=33)
    probs, b = _make(ws)
    th = [inputs.draw_thetas(w.p, 1, 300 + i)[0] for i, w in enumerate(ws)]
    c0, g0, h0 = b.hess(th)
    b.autotune(th)
    cfg = [b.config(i) for i in range(len(ws))]
    _say("  tuned (pg, chunk): " + ", ".join(f"n={w.system.n},P={w.p}:{cfg[i]}" for i, w in enumerate(ws)))
    c1, g1, h1 = b.hess(th)
    for i in range(len(ws)):
        pg, chunk = cfg[i]
        assert 1 <= pg <= max(1, ws[i].p) and 8 <= chunk <= 32
        # a different chunking changes rounding only
        assert _rel(c1[i], c0[i]) < 1e-12 and _rel(g1[i], g0[i]) < 1e-10 and _rel(h1[i], h0[i]) < 1e-10
    b.set_config(0, 1, 32)
    assert b.config(0)[0] == 1
    c2, g2, h2 = b.hess(th)
    assert _rel(h2[0], h0[0]) < 1e-10
    with pytest.raises(qoc.QocError):
        b.set_config(0, 0, 32)
    with pytest.raises(qoc.QocError):
        b.set_config(0, 1, 64)
    b.close()
    for p in probs:
        p.close()


def test_batch_copies_problem_state():
    ws = _small_batch(3, seed=34)
    probs, b = _make(ws)
    th = [inputs.draw_thetas(w.p, 1, 400 + i)[0] for i, w in enumerate(ws)]
    c0, _, _ = b.hess(th, with_hessian=False)
    # changing and closing the source handles does not affect the batch
    probs[0].set_weights(1.0, 5.0)
    for p in probs:
        p.close()
    c1, _, _ = b.hess(th, with_hessian=False)
    assert np.array_equal(c0, c1)
    b.close()


def test_batch_rejects_problems_above_its_size_limit():
    """Single problems go up to n = 288; a batch takes n <= 128 and says so."""
    ws = _small_batch(2, seed=35)
    big = inputs.make_workload("molecule", n=150, nt=24, dt=0.02, k=2, seed=36)
    probs = [qoc.problem_from_workload(w) for w in ws] + [qoc.problem_from_workload(big)]
    with pytest.raises(qoc.QocError) as ei:
        qoc.Batch(probs)
    assert ei.value.status == qoc.QOC_ERR_UNSUPPORTED
    for p in probs:
        p.close()
