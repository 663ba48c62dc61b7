"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerance (normwise relative per output, at random theta, not at an optimum):
cost, gradient, Hessian and Hessian-vector product within 1e-10.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import qoc_oracle as O
from paper_2505_00529_amd import inputs
from paper_2505_00529_amd import qoc

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "molecule_oracle.json")


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem(s, nt, dt, basis_kind, k_or_p, b=None, gamma=None, rho=None):
    p = qoc.Problem(0)
    p.set_system(s.h0, s.m, s.psi0, s.psi_target)
    p.set_control_basis(basis_kind, nt, dt, k_or_p, b)
    if gamma is not None:
        p.set_weights(gamma, rho)
    return p


CASES = [
    # name, workload, overrides, sigma
    ("tiny-full", "tiny", {}, 0.1),
    ("tiny-odd5-ragged", "tiny", dict(n=5, nt=37, k=3), 0.3),
    ("molecule-short", "molecule", dict(nt=300), 0.1),
    ("warm-short", "warm", dict(nt=60, k=8), 0.1),
    # odd n padded to the workgroup eigen kernels' sizes (36 and 64): the padding must stay
    # decoupled through the rotations and the first-order finish
    ("molecule-odd35-padded", "molecule", dict(n=35, nt=200), 0.1),
    ("warm-odd63-padded", "warm", dict(n=63, nt=50, k=8), 0.1),
    # dt * spectral radius far beyond the moment-series range: pairwise U'' fallback
    ("wide-spread-dt0.8", "tiny", dict(n=6, nt=20, dt=0.8, k=2), 0.5),
    # n above the LDS staging limit of the sweeps, odd, ragged chunks
    ("n67-unstaged", "tiny", dict(n=67, nt=21, k=2), 0.2),
    # sweep product and staging paths by n: three-row tiles with n = 2 mod 4 (18), four-row
    # paired tiles with a partly filled last staging slot (44), the generic tile path (22), and
    # the register-staged mode with even n (50)
    ("dbuf-n18-tiles3", "tiny", dict(n=18, nt=40, k=3), 0.2),
    ("dbuf-n44-pairs", "tiny", dict(n=44, nt=30, k=2), 0.2),
    ("dbuf-n22-generic", "tiny", dict(n=22, nt=30, k=2), 0.2),
    ("regs-n50-even", "tiny", dict(n=50, nt=25, k=2), 0.2),
]


@pytest.mark.parametrize("name,wl,over,sigma", CASES, ids=[c[0] for c in CASES])
def test_cost_grad_hess_against_oracle(name, wl, over, sigma):
    w = inputs.make_workload(wl, **over)
    s = w.system
    _say(f"case {name}: n={s.n} nt={w.nt} P={w.p}")
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    p = qoc.problem_from_workload(w)
    for i, th in enumerate(inputs.draw_thetas(w.p, 2, w.seed + 100, sigma=sigma)):
        c, g, h = p.hess(th)
        cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th, w.gamma, w.rho)
        _say(f"  theta {i}: dC={_rel(c, cr):.2e} dg={_rel(g, gr):.2e} dH={_rel(h, hr):.2e}")
        assert _rel(c, cr) < TOL
        assert _rel(g, gr) < TOL
        assert _rel(h, hr) < TOL
        assert np.linalg.norm(h - h.T) <= 1e-13 * np.linalg.norm(h)
        c2, g2 = p.grad(th)
        assert _rel(c2, cr) < TOL and _rel(g2, gr) < TOL
        assert _rel(p.cost(th), cr) < TOL
    p.close()


def test_hvp_against_oracle():
    w = inputs.make_workload("molecule", nt=200)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    p = qoc.problem_from_workload(w)
    th = inputs.draw_thetas(w.p, 1, 77)[0]
    for v in inputs.draw_directions(w.p, 3, 78):
        hv, g = p.hvp(th, v, with_grad=True)
        ref = O.hvp(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th, v, w.gamma, w.rho)
        _say(f"  hvp rel {_rel(hv, ref):.2e}")
        assert _rel(hv, ref) < TOL
    _, gr = O.cost_grad(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th, w.gamma, w.rho)
    assert _rel(g, gr) < TOL
    p.close()


def test_full_molecule_workload_against_stored_oracle():
    """N=36, J=4000, K=16: the workload the throughput benchmark times."""
    doc = json.load(open(GOLDEN))
    w = inputs.make_workload("molecule")
    assert doc["nt"] == w.nt and doc["n"] == w.system.n
    thetas = inputs.draw_thetas(w.p, 2, w.seed)
    vs = inputs.draw_directions(w.p, 1, w.seed)
    p = qoc.problem_from_workload(w)
    costs, grads, hess = p.hess_many(thetas)
    for case in doc["cases"]:
        i = case["theta_index"]
        _say(f"  theta {i}: dC={_rel(costs[i], case['cost']):.2e} dg={_rel(grads[i], case['grad']):.2e} "
             f"dH={_rel(hess[i], case['hess']):.2e}")
        assert _rel(costs[i], case["cost"]) < TOL
        assert _rel(grads[i], case["grad"]) < TOL
        assert _rel(hess[i], case["hess"]) < TOL
        if "hvp" in case:
            hv = p.hvp(thetas[i], vs[case["v_index"]])
            _say(f"  hvp: {_rel(hv, case['hvp']):.2e}")
            assert _rel(hv, case["hvp"]) < TOL
    c1, g1, h1 = p.hess(thetas[0])
    assert _rel(h1, hess[0]) < 1e-12 and _rel(g1, grads[0]) < 1e-12
    p.close()


def test_benchmark_configuration_against_stored_oracle():
    """The throughput benchmark's exact evaluation: the molecule workload with the batch of 256
    thetas it times (16 tangent columns per sweep workgroup, 32-step eigen chunks, 125 chunks per
    theta).  Its first two thetas are the stored oracle cases."""
    doc = json.load(open(GOLDEN))
    w = inputs.make_workload("molecule")
    thetas = inputs.draw_thetas(w.p, 256, w.seed)
    ref = inputs.draw_thetas(w.p, 2, w.seed)
    assert np.array_equal(thetas[:2], ref)
    p = qoc.problem_from_workload(w)
    costs, grads, hess = p.hess_many(thetas)
    for case in doc["cases"]:
        i = case["theta_index"]
        _say(f"  batch 256, theta {i}: dC={_rel(costs[i], case['cost']):.2e} "
             f"dg={_rel(grads[i], case['grad']):.2e} dH={_rel(hess[i], case['hess']):.2e}")
        assert _rel(costs[i], case["cost"]) < TOL
        assert _rel(grads[i], case["grad"]) < TOL
        assert _rel(hess[i], case["hess"]) < TOL
    # every theta of the batch: finite and symmetric; two more sampled rows against the oracle
    # computed here, and three rows against their evaluation in a batch of 2 (8 columns per
    # workgroup, 8-step chunks: a different rounding history, so equal within the tolerance)
    assert np.all(np.isfinite(hess)) and np.all(np.isfinite(grads))
    sym = np.linalg.norm(hess - hess.transpose(0, 2, 1), axis=(1, 2)) / np.linalg.norm(hess, axis=(1, 2))
    assert sym.max() <= 1e-13
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    for i in (131, 255):
        cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, thetas[i], w.gamma, w.rho)
        _say(f"  batch 256, theta {i}: dC={_rel(costs[i], cr):.2e} dg={_rel(grads[i], gr):.2e} dH={_rel(hess[i], hr):.2e}")
        assert _rel(costs[i], cr) < TOL and _rel(grads[i], gr) < TOL and _rel(hess[i], hr) < TOL
    for i in (17, 128, 255):
        c2, g2, h2 = p.hess_many(thetas[[i, 0]])
        _say(f"  theta {i}: batch 256 vs batch 2: dC={_rel(costs[i], c2[0]):.2e} dH={_rel(hess[i], h2[0]):.2e}")
        assert _rel(costs[i], c2[0]) < TOL and _rel(grads[i], g2[0]) < TOL and _rel(hess[i], h2[0]) < TOL
    p.close()


def test_step_propagators_against_block_exponential():
    w = inputs.make_workload("molecule", n=6, nt=50)
    s = w.system
    p = qoc.problem_from_workload(w)
    th = inputs.draw_thetas(w.p, 1, 5, sigma=0.5)[0]
    f = O.fourier_basis(w.nt, w.dt, w.k) @ th
    for j in (0, 17, 49):
        u, u1, u2 = p.step_propagators(th, j)
        r0, r1, r2 = O.step_propagators(s.h0, s.m, f[j], w.dt)
        assert _rel(u, r0) < 1e-13
        assert _rel(u1, r1) < 1e-12
        assert _rel(u2, r2) < 1e-11
    p.close()


def test_step_propagators_degenerate_spectrum():
    """H0 = 0 and theta = 0: every eigenvalue of H_j coincides (fully confluent divided
    differences); U = I, U' = -i dt M, U'' = -dt^2 M^2."""
    n, nt, dt = 5, 10, 0.1
    rng = np.random.default_rng(3)
    mm = rng.normal(size=(n, n))
    mm = mm + mm.T
    sysm = inputs.System(np.zeros((n, n)), mm, np.eye(n)[0].astype(complex), np.eye(n)[1].astype(complex))
    p = _problem(sysm, nt, dt, qoc.QOC_BASIS_FOURIER, 2)
    u, u1, u2 = p.step_propagators(np.zeros(4), 3)
    assert np.allclose(u, np.eye(n), atol=1e-15)
    assert np.allclose(u1, -1j * dt * mm, atol=1e-15)
    assert np.allclose(u2, -dt * dt * mm @ mm, atol=1e-14)
    p.close()


def test_large_dimension_global_scratch_path():
    w = inputs.make_workload("diff", nt=12, k=2)
    s = w.system
    _say(f"n={s.n} nt={w.nt}")
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    p = qoc.problem_from_workload(w)
    th = inputs.draw_thetas(w.p, 1, 3, sigma=0.3)[0]
    c, g, h = p.hess(th)
    cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th, w.gamma, w.rho)
    _say(f"  dC={_rel(c, cr):.2e} dg={_rel(g, gr):.2e} dH={_rel(h, hr):.2e}")
    assert _rel(c, cr) < TOL and _rel(g, gr) < TOL and _rel(h, hr) < TOL
    p.close()


def test_identity_and_dense_bases():
    w = inputs.make_workload("tiny", nt=20)
    s = w.system
    p = _problem(s, w.nt, w.dt, qoc.QOC_BASIS_IDENTITY, 0, gamma=1.0, rho=10.0)
    assert p.P == w.nt
    th = np.random.default_rng(4).normal(0, 0.3, w.nt)
    c, g, h = p.hess(th)
    cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, np.eye(w.nt), w.dt, th, 1.0, 10.0)
    assert _rel(c, cr) < TOL and _rel(g, gr) < TOL and _rel(h, hr) < TOL
    p.close()
    # single step, dense basis with two columns
    b = np.array([[0.7, -0.2]])
    p = _problem(s, 1, 0.3, qoc.QOC_BASIS_DENSE, 2, b=b)
    th = np.array([0.4, 1.1])
    c, g, h = p.hess(th)
    cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, b, 0.3, th, 0.6, 2.0)
    assert _rel(c, cr) < TOL and _rel(g, gr) < TOL and _rel(h, hr) < TOL
    p.close()


def test_rabi_two_level_closed_form():
    e0, e1, mm = -1.1, -0.4, 0.6
    nt, dt, c = 60, 0.05, 0.37
    sysm = inputs.System(np.diag([e0, e1]), np.array([[0, mm], [mm, 0.0]]),
                         np.array([1, 0], complex), np.array([0, 1], complex))
    p = _problem(sysm, nt, dt, qoc.QOC_BASIS_DENSE, 1, b=np.ones((nt, 1)))
    cost = p.cost([c])
    d, om = (e1 - e0) / 2, c * mm
    omr = np.hypot(d, om)
    T = nt * dt
    a1 = abs(om / omr * np.sin(omr * T)) ** 2
    # |a(T) - e1|^2 = |a0|^2 + |a1 - 1|^2 with a1 = -i e^{-i ebar T} (om/omr) sin(omr T)
    ebar = (e0 + e1) / 2
    a0 = np.exp(-1j * ebar * T) * (np.cos(omr * T) + 1j * d / omr * np.sin(omr * T))
    a1c = np.exp(-1j * ebar * T) * (-1j * om / omr * np.sin(omr * T))
    ref = dt * nt * c * c + abs(a0) ** 2 + abs(a1c - 1) ** 2
    assert abs(abs(a1c) ** 2 - a1) < 1e-15
    assert abs(cost - ref) < 1e-12
    p.close()


def test_zero_rho_hessian_is_field_energy():
    w = inputs.make_workload("tiny", nt=64)
    p = qoc.problem_from_workload(w)
    p.set_weights(w.gamma, 0.0)
    th = inputs.draw_thetas(w.p, 1, 9)[0]
    _, _, h = p.hess(th)
    b = O.fourier_basis(w.nt, w.dt, w.k)
    assert _rel(h, w.gamma * b.T @ b) < 1e-13
    p.close()


def test_many_thetas_match_single_calls():
    w = inputs.make_workload("molecule", nt=120)
    p = qoc.problem_from_workload(w)
    ths = inputs.draw_thetas(w.p, 5, 31)
    c, g, h = p.hess_many(ths)
    for i in range(5):
        ci, gi, hi = p.hess(ths[i])
        assert _rel(ci, c[i]) < 1e-12 and _rel(gi, g[i]) < 1e-12 and _rel(hi, h[i]) < 1e-12
    cg, gg = p.grad_many(ths)
    assert _rel(gg, g) < 1e-12 and _rel(cg, c) < 1e-12
    p.close()


def _sentinels(P):
    return np.full(1, 7.0), np.full(P, 7.0), np.full((P, P), 7.0)


def test_invalid_arguments_leave_outputs_untouched():
    w = inputs.make_workload("tiny", nt=10)
    p = qoc.problem_from_workload(w)
    bad = np.full(w.p, np.nan)
    with pytest.raises(qoc.QocError) as ei:
        p.cost(bad)
    assert ei.value.status == qoc.QOC_ERR_INVALID_ARG
    lib = qoc.lib()
    c, g, h = _sentinels(w.p)
    st = lib.qoc_hess(p.handle, qoc._ptr(bad), qoc._ptr(c), qoc._ptr(g), qoc._ptr(h))
    assert st == qoc.QOC_ERR_INVALID_ARG
    assert np.all(c == 7.0) and np.all(g == 7.0) and np.all(h == 7.0)
    hv = np.full(w.p, 7.0)
    st = lib.qoc_hvp(p.handle, qoc._ptr(np.zeros(w.p)), None, qoc._ptr(hv), qoc._ptr(g))
    assert st == qoc.QOC_ERR_INVALID_ARG
    assert np.all(hv == 7.0) and np.all(g == 7.0)
    st = lib.qoc_grad_many(p.handle, 0, qoc._ptr(np.zeros(w.p)), qoc._ptr(c), qoc._ptr(g))
    assert st == qoc.QOC_ERR_INVALID_ARG
    assert np.all(c == 7.0) and np.all(g == 7.0)
    asym = w.system.m.copy()
    asym[0, 1] += 1e-3
    with pytest.raises(qoc.QocError) as ei:
        p.set_system(w.system.h0, asym, w.system.psi0, w.system.psi_target)
    assert ei.value.status == qoc.QOC_ERR_NOT_SYMMETRIC
    q = qoc.Problem(0)
    with pytest.raises(qoc.QocError) as ei:
        q.cost(np.zeros(1)) if q.P else q._check(qoc.lib().qoc_cost(q.handle, None, None))
    assert ei.value.status in (qoc.QOC_ERR_STATE, qoc.QOC_ERR_INVALID_ARG)
    q.close()
    p.close()


def test_sweep_cap_reports_nonconvergence():
    """A Jacobi step that reaches the sweep cap ends its kernel normally; the call reports
    QOC_ERR_NOCONV and leaves the outputs untouched.  The status belongs to that call only: the
    next evaluation with the default cap succeeds and matches an evaluation never capped."""
    w = inputs.make_workload("molecule", nt=64)
    p = qoc.problem_from_workload(w)
    th = inputs.draw_thetas(w.p, 1, 51)[0]
    c0, g0, h0 = p.hess(th)
    lib = qoc.lib()
    p.set_jacobi_sweep_cap(0)
    c, g, h = _sentinels(w.p)
    st = lib.qoc_hess(p.handle, qoc._ptr(th), qoc._ptr(c), qoc._ptr(g), qoc._ptr(h))
    assert st == qoc.QOC_ERR_NOCONV
    assert np.all(c == 7.0) and np.all(g == 7.0) and np.all(h == 7.0)
    with pytest.raises(qoc.QocError) as ei:
        p.grad(th)
    assert ei.value.status == qoc.QOC_ERR_NOCONV
    p.set_jacobi_sweep_cap(40)
    c1, g1, h1 = p.hess(th)
    assert c1 == c0 and np.array_equal(g1, g0) and np.array_equal(h1, h0)
    with pytest.raises(qoc.QocError):
        p.set_jacobi_sweep_cap(-1)
    p.close()


def test_sweep_cap_on_device_entry_points_and_autograd():
    """*_dev calls report the capped step through qoc_sync; the autograd layer raises in the call
    whose evaluation failed, and a later evaluation with the default cap is unaffected."""
    import torch
    from paper_2505_00529_amd import autograd as QA

    w = inputs.make_workload("molecule", n=16, nt=40, k=2)
    p = qoc.problem_from_workload(w)
    th = torch.tensor(inputs.draw_thetas(w.p, 1, 52)[0], dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.empty(w.p, dtype=torch.float64, device="cuda")
    p.set_stream(torch.cuda.current_stream().cuda_stream)
    p.set_jacobi_sweep_cap(0)
    p.grad_dev(th.detach().data_ptr(), None, g.data_ptr())
    with pytest.raises(qoc.QocError) as ei:
        p.sync()
    assert ei.value.status == qoc.QOC_ERR_NOCONV
    with pytest.raises(qoc.QocError) as ei:
        QA.cost(th, p)
    assert ei.value.status == qoc.QOC_ERR_NOCONV
    p.set_jacobi_sweep_cap(40)
    c = QA.cost(th, p)
    (gt,) = torch.autograd.grad(c, th)
    _, gr = p.grad(th.detach().cpu().numpy())
    assert _rel(gt.cpu().numpy(), gr) < 1e-13
    p.close()


@pytest.mark.parametrize("n", [72, 100, 127, 128, 200])
def test_large_n_eigen_kernel_against_oracle(n):
    """Sizes past one LDS tile: A in LDS and V in global memory (72, 100, odd 127), the slot-order
    kernel (128), all matrices in global memory with sweeps of more rows than the phase waves
    (200); five eigen chunks of 8 steps, against the oracle."""
    nt, dt, k = 40, 0.02, 2
    w = inputs.make_workload("molecule", n=n, nt=nt, dt=dt, k=k, seed=40 + n)
    s = w.system
    p = qoc.problem_from_workload(w)
    ths = inputs.draw_thetas(w.p, 2, 700 + n, sigma=0.3)
    c, g, h = p.hess_many(ths)
    basis = O.fourier_basis(nt, dt, k)
    for i in range(2):
        cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, dt, ths[i], w.gamma, w.rho)
        print(f"n={n} theta {i}: dC={_rel(c[i], cr):.2e} dg={_rel(g[i], gr):.2e} dH={_rel(h[i], hr):.2e}",
              flush=True)
        assert _rel(c[i], cr) < TOL and _rel(g[i], gr) < TOL and _rel(h[i], hr) < TOL
    p.close()


@pytest.mark.parametrize("n", [4, 36, 100])
def test_eig_chain_length_setting(n):
    """Fixed chain lengths 1, 3 and 32 give the automatic setting's results to rounding and the
    oracle's to the parity tolerance; lengths outside [0, 32] are rejected."""
    nt, dt, k = 40, 0.02, 2
    w = inputs.make_workload("molecule", n=n, nt=nt, dt=dt, k=k, seed=50 + n)
    s = w.system
    p = qoc.problem_from_workload(w)
    ths = inputs.draw_thetas(w.p, 2, 800 + n, sigma=0.3)
    c0, g0, h0 = p.hess_many(ths)
    basis = O.fourier_basis(nt, dt, k)
    cr, gr, hr = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, dt, ths[0], w.gamma, w.rho)
    for chain in (1, 3, 32):
        p.set_eig_chunk(chain)
        c, g, h = p.hess_many(ths)
        print(f"n={n} chain {chain}: vs auto dH={_rel(h, h0):.2e}, vs oracle dH={_rel(h[0], hr):.2e}", flush=True)
        assert _rel(c, c0) < 1e-12 and _rel(g, g0) < 1e-11 and _rel(h, h0) < 1e-11
        assert _rel(c[0], cr) < TOL and _rel(g[0], gr) < TOL and _rel(h[0], hr) < TOL
    for bad in (-1, 33):
        with pytest.raises(qoc.QocError):
            p.set_eig_chunk(bad)
    p.close()
