"""Several control directions (Sec. II, H0 + sum_k f^k M_k; the mixed second derivatives of
eq. d2Ldf2) on the GPU, against the oracle's K-direction functions (tolerance 1e-10 normwise
relative), and, at horizons the oracle does not reach, against properties that hold at any
size: a duplicated operator equals the single-direction path at the summed parameters, and
rotating two directions into each other changes nothing."""
import sys

import numpy as np
import pytest

from oracle import qoc_oracle as O
from paper_2505_00529_amd import inputs, qoc

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ops(n, k, seed, scale=0.4):
    """The molecule recipe's H0 and M, plus k - 1 further random symmetric operators."""
    s = inputs.transfer_system(n, seed=seed)
    rng = np.random.default_rng(seed + 100)
    ms = [s.m]
    for _ in range(k - 1):
        a = rng.normal(size=(n, n))
        ms.append(scale * 0.5 * (a + a.T) / np.sqrt(n))
    return s, ms


def _fourier_stack(nt, dt, kf, ndir):
    b0 = O.fourier_basis(nt, dt, kf)
    p0 = b0.shape[1]
    bases = np.zeros((ndir, nt, ndir * p0))
    for c in range(ndir):
        bases[c, :, c * p0:(c + 1) * p0] = b0
    return bases


@pytest.mark.parametrize("n,ndir", [(4, 2), (7, 3), (16, 3), (35, 3), (36, 2), (64, 2), (80, 3)])
def test_fourier_directions_against_oracle(n, ndir):
    """Fourier model per direction (a block of theta each); n = 7 pads the Jacobi players; n = 35
    (padded) and 36 run the circle-slot eigen kernel at NP = 36, n = 64 the one at NP = 64; n = 80
    keeps the generic eigen kernel's matrices in global memory."""
    nt, dt, kf = 24, 0.05, 2
    s, ms = _ops(n, ndir, 60 + n)
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, dt, kf)
    p.set_weights(0.3, 2.0)
    assert p.P == ndir * 2 * kf
    bases = _fourier_stack(nt, dt, kf, ndir)
    ths = inputs.draw_thetas(p.P, 2, 900 + n, sigma=0.8)
    _say(f"multi n={n} K={ndir} P={p.P} nt={nt}")
    c, g, h = p.hess_many(ths)
    for i, th in enumerate(ths):
        cr, gr, hr = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, th, 0.3, 2.0)
        _say(f"  theta {i}: dC={_rel(c[i], cr):.2e} dg={_rel(g[i], gr):.2e} dH={_rel(h[i], hr):.2e}")
        assert _rel(c[i], cr) < TOL and _rel(g[i], gr) < TOL and _rel(h[i], hr) < TOL
    c1, g1 = p.grad_many(ths)
    assert _rel(c1, c) < 1e-13 and _rel(g1, g) < 1e-12
    v = inputs.draw_directions(p.P, 1, 950 + n)[0]
    hv = p.hvp(ths[0], v)
    hr0 = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, ths[0], 0.3, 2.0)[2]
    _say(f"  hvp: {_rel(hv, hr0 @ v):.2e}")
    assert _rel(hv, hr0 @ v) < TOL
    p.close()


@pytest.mark.parametrize("n,ndir,nt", [(130, 2, 24), (120, 3, 16)])
def test_above_128_levels(n, ndir, nt):
    """n = 130, two directions: the eigen kernel's matrices in global memory, sweeps reading O and
    S_k from global memory (too large to stage), rows past 128 in the U'' moments (kept in LDS for
    all pairs).  n = 120, three directions: the U'' moments of three directions no longer fit in
    LDS, so each pair builds its own (the per-pair kernel)."""
    dt, kf = 0.05, 1
    s, ms = _ops(n, ndir, 190 + ndir)
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, dt, kf)
    p.set_weights(0.3, 2.0)
    bases = _fourier_stack(nt, dt, kf, ndir)
    th = inputs.draw_thetas(p.P, 1, 191, sigma=0.8)[0]
    c, g, h = p.hess(th)
    cr, gr, hr = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, th, 0.3, 2.0)
    _say(f"n={n} K={ndir}: dC={_rel(c, cr):.2e} dg={_rel(g, gr):.2e} dH={_rel(h, hr):.2e}")
    assert _rel(c, cr) < TOL and _rel(g, gr) < TOL and _rel(h, hr) < TOL
    p.close()


def test_wide_spectral_spread_takes_the_direct_form():
    """dt = 0.8: every step's spread needs more series terms than the U'' contraction keeps, so
    the pair values come from the divided differences of every triple."""
    n, nt, dt, kf = 6, 12, 0.8, 1
    s, ms = _ops(n, 2, 75)
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, dt, kf)
    p.set_weights(0.3, 2.0)
    bases = _fourier_stack(nt, dt, kf, 2)
    th = inputs.draw_thetas(p.P, 1, 76, sigma=0.8)[0]
    c, g, h = p.hess(th)
    cr, gr, hr = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, th, 0.3, 2.0)
    _say(f"wide spread K=2: dC={_rel(c, cr):.2e} dg={_rel(g, gr):.2e} dH={_rel(h, hr):.2e}")
    assert _rel(c, cr) < TOL and _rel(g, gr) < TOL and _rel(h, hr) < TOL
    p.close()


def test_dense_models_move_every_direction():
    """A dense nt x P model per direction (every parameter moves all three directions)."""
    n, nt, dt, P = 8, 30, 0.05, 5
    s, ms = _ops(n, 3, 71)
    rng = np.random.default_rng(72)
    bases = rng.normal(size=(3, nt, P)) * 0.5
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_DENSE, nt, dt, P, bases)
    p.set_weights(0.2, 3.0)
    ths = inputs.draw_thetas(P, 2, 73, sigma=0.7)
    c, g, h = p.hess_many(ths)
    for i, th in enumerate(ths):
        cr, gr, hr = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, th, 0.2, 3.0)
        _say(f"dense K=3 theta {i}: dC={_rel(c[i], cr):.2e} dg={_rel(g[i], gr):.2e} dH={_rel(h[i], hr):.2e}")
        assert _rel(c[i], cr) < TOL and _rel(g[i], gr) < TOL and _rel(h[i], hr) < TOL
    tg = rng.normal(size=(2, n)) + 1j * rng.normal(size=(2, n))
    tg /= np.linalg.norm(tg, axis=1, keepdims=True)
    ct, gt, ht = p.hess_many_targets(ths, tg)
    cr, gr, hr = O.cost_grad_hess_multi(s.h0, ms, s.psi0, tg[1], bases, dt, ths[1], 0.2, 3.0)
    assert _rel(ct[1], cr) < TOL and _rel(gt[1], gr) < TOL and _rel(ht[1], hr) < TOL
    p.close()


@pytest.mark.parametrize("ndir,P,nt", [(3, 45, 50), (2, 70, 37)])
def test_hessian_tiles_ragged_against_oracle(ndir, P, nt):
    """Dense models with P spanning several 32-column Hessian tiles, the last one ragged, and a
    horizon that is not a whole number of the assembly's step chunks (16 steps at K = 3, 24 at
    K = 2): the tiled Hessian against the oracle, exactly symmetric (upper tiles mirrored), and
    the gradient and a Hessian-vector product through their own kernels."""
    n, dt = 8, 0.05
    s, ms = _ops(n, ndir, 170 + P)
    rng = np.random.default_rng(171 + P)
    bases = rng.normal(size=(ndir, nt, P)) * 0.3
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_DENSE, nt, dt, P, bases)
    p.set_weights(0.3, 2.0)
    ths = inputs.draw_thetas(P, 2, 172 + P, sigma=0.5)
    c, g, h = p.hess_many(ths)
    for i, th in enumerate(ths):
        cr, gr, hr = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, th, 0.3, 2.0)
        _say(f"tiles K={ndir} P={P} nt={nt} theta {i}: dC={_rel(c[i], cr):.2e} dg={_rel(g[i], gr):.2e} "
             f"dH={_rel(h[i], hr):.2e}")
        assert _rel(c[i], cr) < TOL and _rel(g[i], gr) < TOL and _rel(h[i], hr) < TOL
        assert np.array_equal(h[i], h[i].T)
    v = rng.normal(size=P)
    hv = p.hvp(ths[0], v)
    _say(f"  hvp against H v: {_rel(hv, h[0] @ v):.2e}")
    assert _rel(hv, h[0] @ v) < TOL
    p.close()


def test_one_direction_through_the_multi_setter_is_the_single_path():
    w = inputs.make_workload("tiny", nt=80)
    s = w.system
    p1 = qoc.problem_from_workload(w)
    p2 = qoc.Problem(0)
    p2.set_system_multi(s.h0, [s.m], s.psi0, s.psi_target)
    p2.set_control_basis(qoc.QOC_BASIS_FOURIER, w.nt, w.dt, w.k)
    p2.set_weights(w.gamma, w.rho)
    ths = inputs.draw_thetas(w.p, 2, 5)
    assert np.array_equal(np.asarray(p1.hess_many(ths)[2]), np.asarray(p2.hess_many(ths)[2]))
    p1.close()
    p2.close()


def test_duplicated_operator_equals_single_direction_path_long_horizon():
    """M_2 = M_1 with a block of theta each acts as one control at theta_1 + theta_2: with
    gamma = 0 the K = 2 gradient repeats the single-direction gradient and every Hessian block is
    the single-direction Hessian (independent kernels on both sides), at J = 1000, n = 36."""
    w = inputs.make_workload("molecule", n=36, nt=1000, dt=0.02, k=8, seed=81)
    s = w.system
    p1 = qoc.Problem(0)
    p1.set_system(s.h0, s.m, s.psi0, s.psi_target)
    p1.set_control_basis(qoc.QOC_BASIS_FOURIER, w.nt, w.dt, w.k)
    p1.set_weights(0.0, w.rho)
    p2 = qoc.Problem(0)
    p2.set_system_multi(s.h0, [s.m, s.m], s.psi0, s.psi_target)
    p2.set_control_basis(qoc.QOC_BASIS_FOURIER, w.nt, w.dt, w.k)
    p2.set_weights(0.0, w.rho)
    p0 = w.p
    rng = np.random.default_rng(82)
    th = rng.normal(size=2 * p0) * 0.15
    c1, g1, h1 = p1.hess(th[:p0] + th[p0:])
    c2, g2, h2 = p2.hess(th)
    _say(f"duplicated operator J=1000: dC={_rel(c2, c1):.2e} dg={_rel(g2, np.concatenate([g1, g1])):.2e}")
    assert _rel(c2, c1) < TOL
    assert _rel(g2, np.concatenate([g1, g1])) < TOL
    for a in range(2):
        for b in range(2):
            blk = h2[a * p0:(a + 1) * p0, b * p0:(b + 1) * p0]
            assert _rel(blk, h1) < TOL, (a, b, _rel(blk, h1))
    p1.close()
    p2.close()


def test_rotated_directions_change_nothing_long_horizon():
    """f1 M1 + f2 M2 = f1' M1' + f2' M2' with (M1', M2') and (theta_1', theta_2') rotated by the
    same angle: cost, Q^T g' and Q^T H' Q are unchanged (field energy included), J = 800."""
    n, nt, dt, kf = 16, 800, 0.02, 4
    s, ms = _ops(n, 2, 91)
    ang = 0.6
    cs, sn = np.cos(ang), np.sin(ang)
    pa = qoc.Problem(0)
    pa.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    pa.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, dt, kf)
    pa.set_weights(0.5, 2.0)
    pb = qoc.Problem(0)
    pb.set_system_multi(s.h0, [cs * ms[0] + sn * ms[1], -sn * ms[0] + cs * ms[1]], s.psi0, s.psi_target)
    pb.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, dt, kf)
    pb.set_weights(0.5, 2.0)
    p0 = 2 * kf
    q = np.block([[cs * np.eye(p0), sn * np.eye(p0)], [-sn * np.eye(p0), cs * np.eye(p0)]])
    th = np.random.default_rng(92).normal(size=2 * p0) * 0.3
    c, g, h = pa.hess(th)
    c2, g2, h2 = pb.hess(q @ th)
    _say(f"rotation J=800: dC={_rel(c2, c):.2e} dg={_rel(q.T @ g2, g):.2e} dH={_rel(q.T @ h2 @ q, h):.2e}")
    assert _rel(c2, c) < TOL and _rel(q.T @ g2, g) < TOL and _rel(q.T @ h2 @ q, h) < TOL
    pa.close()
    pb.close()


def test_trust_region_with_three_directions():
    """The exact-Hessian trust region runs on the K-direction evaluations (its control-space
    whitening uses the stacked model) and reaches a stationary point of the oracle's cost."""
    n, nt, dt, kf = 4, 40, 0.1, 2
    s, ms = _ops(n, 3, 95)
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, dt, kf)
    p.set_weights(0.1, 2.0)
    res = p.tr_solve(np.zeros(p.P), gtol=1e-8, max_iter=200)
    theta = res[0]
    bases = _fourier_stack(nt, dt, kf, 3)
    c0 = O.cost_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, np.zeros(p.P), 0.1, 2.0)
    c, g = O.cost_grad_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, theta, 0.1, 2.0)
    _say(f"TR K=3: cost {c0:.4e} -> {c:.4e}, |g| {np.linalg.norm(g):.2e}")
    assert c < c0 and np.linalg.norm(g) < 1e-6
    p.close()


def test_multi_direction_limits_are_reported():
    s, ms = _ops(4, 3, 97)
    p = qoc.Problem(0)
    with pytest.raises(qoc.QocError):
        p.set_system_multi(s.h0, ms + [ms[0]], s.psi0, s.psi_target)   # four directions
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_FOURIER, 20, 0.05, 1)
    th = np.zeros(p.P)
    with pytest.raises(qoc.QocError) as ei:
        p.step_propagators(th, 0)
    assert ei.value.status == qoc.QOC_ERR_UNSUPPORTED
    p.set_checkpoint_interval(5)
    with pytest.raises(qoc.QocError) as ei:
        p.grad(th)
    assert ei.value.status == qoc.QOC_ERR_UNSUPPORTED
    p.set_checkpoint_interval(0)
    with pytest.raises(qoc.QocError) as ei:
        qoc.Batch([p])
    assert ei.value.status == qoc.QOC_ERR_UNSUPPORTED
    c, g = p.grad(th)
    assert np.isfinite(c) and np.all(np.isfinite(g))
    p.close()


def test_benchmark_configuration_against_stored_oracle():
    """The three-direction workload at full size, in the launch configuration the benchmark times
    (256 theta, J = 4000, P = 96): rows 0 and 1 against the oracle's stored values
    (tests/golden/multi_oracle.json, written by make_golden_multi.py)."""
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "multi_oracle.json")) as fh:
        doc = json.load(fh)
    w, ms = inputs.multi_direction_workload()
    s = w.system
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_FOURIER, w.nt, w.dt, w.k)
    p.set_weights(w.gamma, w.rho)
    ths = inputs.draw_thetas(p.P, 256, w.seed)
    c, g, h = p.hess_many(ths)
    for case in doc["cases"]:
        i = case["theta_index"]
        dc, dg, dh = _rel(c[i], case["cost"]), _rel(g[i], case["grad"]), _rel(h[i], case["hess"])
        _say(f"multi bench config theta {i}: dC={dc:.2e} dg={dg:.2e} dH={dh:.2e}")
        assert dc < TOL and dg < TOL and dh < TOL
    p.close()


def test_autograd_with_three_directions():
    """The torch.autograd layer (device entry points on torch's stream) on a three-direction
    problem: cost, gradient and a Hessian-vector product by double backward against the oracle."""
    import torch
    from paper_2505_00529_amd import autograd as QA

    n, nt, dt, kf = 6, 40, 0.05, 2
    s, ms = _ops(n, 3, 96)
    p = qoc.Problem(0)
    p.set_system_multi(s.h0, ms, s.psi0, s.psi_target)
    p.set_control_basis(qoc.QOC_BASIS_FOURIER, nt, dt, kf)
    p.set_weights(0.3, 2.0)
    bases = _fourier_stack(nt, dt, kf, 3)
    th_np = inputs.draw_thetas(p.P, 1, 97, sigma=0.6)[0]
    v_np = inputs.draw_directions(p.P, 1, 97)[0]
    th = torch.tensor(th_np, dtype=torch.float64, device="cuda", requires_grad=True)
    c = QA.cost(th, p)
    (g,) = torch.autograd.grad(c, th, create_graph=True)
    (hv,) = torch.autograd.grad(g, th, torch.tensor(v_np, dtype=torch.float64, device="cuda"))
    p.sync()
    cr, gr, hr = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, dt, th_np, 0.3, 2.0)
    _say(f"autograd K=3: dC={_rel(c.item(), cr):.2e} dg={_rel(g.detach().cpu().numpy(), gr):.2e} "
         f"dHv={_rel(hv.cpu().numpy(), hr @ v_np):.2e}")
    assert _rel(c.item(), cr) < TOL
    assert _rel(g.detach().cpu().numpy(), gr) < TOL
    assert _rel(hv.cpu().numpy(), hr @ v_np) < TOL
    p.close()
