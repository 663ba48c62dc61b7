"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each check is independent of the oracle's own formulas: library routines
(scipy.linalg.expm / expm_frechet, numpy.linalg.eigh), closed forms (Rabi
two-level problem, commuting H0 = 0 case, field-free propagation, first-order
tangent at theta = 0), invariants of unitary propagation, finite differences and a
50-digit mpmath re-propagation on tiny inputs.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import qoc_oracle as O
from oracle import brute
from paper_2505_00529_amd import inputs


def _rand_sym(rng, n, scale=1.0):
    a = rng.normal(size=(n, n)) * scale
    return (a + a.T) / 2


# ------------------------------------------------------------ propagator pins

@pytest.mark.parametrize("n,dt,f", [(3, 0.05, 0.3), (6, 0.3, -1.2), (5, 2.0, 0.7)])
def test_block_exponential_matches_scipy(n, dt, f):
    """exp of the 3N x 3N block matrix: dense scipy expm and expm_frechet agree."""
    rng = np.random.default_rng(11 + n)
    h0 = np.diag(np.sort(rng.uniform(-2, 0, n)))
    m = _rand_sym(rng, n)
    u, u1, u2 = O.step_propagators(h0, m, f, dt)
    x = -1j * dt * (h0 + f * m)
    e = -1j * dt * m
    z = np.zeros_like(x)
    big = np.block([[x, e, z], [z, x, e], [z, z, x]])
    ex = sla.expm(big)
    assert np.allclose(u, ex[:n, :n], atol=1e-13, rtol=0)
    assert np.allclose(u1, ex[:n, n:2 * n], atol=1e-13, rtol=0)
    assert np.allclose(u2, 2 * ex[:n, 2 * n:], atol=1e-13, rtol=0)
    uf, frechet = sla.expm_frechet(x, e)
    assert np.allclose(u, uf, atol=1e-13, rtol=0)
    assert np.allclose(u1, frechet, atol=1e-13, rtol=0)


def test_propagators_commuting_case():
    """H0 = 0: U = exp(-i dt f M), U' = -i dt M U, U'' = -dt^2 M^2 U (eigh of M)."""
    rng = np.random.default_rng(5)
    n, dt, f = 5, 0.07, 0.9
    m = _rand_sym(rng, n)
    w, v = np.linalg.eigh(m)
    uref = (v * np.exp(-1j * dt * f * w)) @ v.T
    u, u1, u2 = O.step_propagators(np.zeros((n, n)), m, f, dt)
    assert np.allclose(u, uref, atol=1e-14)
    assert np.allclose(u1, -1j * dt * m @ uref, atol=1e-14)
    assert np.allclose(u2, -dt ** 2 * m @ m @ uref, atol=1e-14)


def test_propagators_unitarity_invariants():
    """Derivatives of U^H U = I: U^H U' + U'^H U = 0 and U''^H U + 2 U'^H U' + U^H U'' = 0."""
    rng = np.random.default_rng(6)
    n, dt, f = 7, 0.2, 0.4
    h0 = np.diag(np.sort(rng.uniform(-3, 0, n)))
    m = _rand_sym(rng, n, 0.3)
    u, u1, u2 = O.step_propagators(h0, m, f, dt)
    h = lambda a: a.conj().T
    assert np.allclose(h(u) @ u, np.eye(n), atol=1e-14)
    assert np.allclose(h(u) @ u1 + h(u1) @ u, 0, atol=1e-14)
    assert np.allclose(h(u2) @ u + 2 * h(u1) @ u1 + h(u) @ u2, 0, atol=1e-14)


def test_propagators_central_difference_in_f():
    rng = np.random.default_rng(7)
    n, dt, f, hstep = 4, 0.1, 0.25, 1e-4
    h0 = np.diag(np.sort(rng.uniform(-1.5, 0, n)))
    m = _rand_sym(rng, n, 0.5)
    u, u1, u2 = O.step_propagators(h0, m, f, dt)
    up = O.step_propagators(h0, m, f + hstep, dt)
    um = O.step_propagators(h0, m, f - hstep, dt)
    assert np.allclose((up[0] - um[0]) / (2 * hstep), u1, atol=1e-9)
    assert np.allclose((up[1] - um[1]) / (2 * hstep), u2, atol=1e-9)
    assert np.allclose((up[0] - 2 * u + um[0]) / hstep ** 2, u2, atol=1e-6)


# ------------------------------------------------------------------ Rabi pin

def _rabi_state(e0, e1, mm, c, t):
    """Exact two-level solution for constant field c (U^J = exp(-i H J dt) exactly)."""
    ebar = (e0 + e1) / 2
    d = (e1 - e0) / 2
    om = c * mm
    omr = mp.sqrt(d * d + om * om)
    ph = mp.exp(-1j * ebar * t)
    a0 = ph * (mp.cos(omr * t) + 1j * (d / omr) * mp.sin(omr * t))
    a1 = ph * (-1j * (om / omr) * mp.sin(omr * t))
    return a0, a1


def test_rabi_closed_form_cost_grad_hess():
    e0, e1, mm = -1.1, -0.4, 0.6
    nt, dt = 60, 0.05
    gamma, rho = 2 * dt, 2.0
    h0 = np.diag([e0, e1])
    m = np.array([[0.0, mm], [mm, 0.0]])
    psi0 = np.array([1, 0], dtype=complex)
    beta = np.array([0.3, 0.8 + 0.2j]) / np.linalg.norm([0.3, 0.8 + 0.2j])
    basis = np.ones((nt, 1))
    T = nt * dt

    def closed(c):
        a0, a1 = _rabi_state(mp.mpf(e0), mp.mpf(e1), mp.mpf(mm), c, mp.mpf(T))
        err = abs(a0 - complex(beta[0])) ** 2 + abs(a1 - complex(beta[1])) ** 2
        return mp.mpf(gamma) / 2 * nt * c * c + mp.mpf(rho) / 2 * err

    for c in (0.0, 0.37, -1.3):
        with mp.workdps(40):
            cref = closed(mp.mpf(c))
            gref = mp.diff(closed, mp.mpf(c))
            href = mp.diff(closed, mp.mpf(c), 2)
        cc, g, hh = O.cost_grad_hess(h0, m, psi0, beta, basis, dt, np.array([c]), gamma, rho)
        assert abs(cc - float(cref)) < 1e-13 * max(1, abs(float(cref)))
        assert abs(g[0] - float(gref)) < 1e-11 * max(1, abs(float(gref)))
        assert abs(hh[0, 0] - float(href)) < 1e-10 * max(1, abs(float(href)))
        # population transfer |a1(T)|^2 = (Om/Om_R)^2 sin^2(Om_R T)
        a = O.propagate_state(h0, m, psi0, basis, dt, np.array([c]))
        d = (e1 - e0) / 2
        om = c * mm
        omr = math.sqrt(d * d + om * om)
        assert abs(abs(a[1]) ** 2 - (om / omr) ** 2 * math.sin(omr * T) ** 2) < 1e-13


# ------------------------------------------------------------- special cases

def test_field_free_propagation():
    """theta = 0 and diagonal H0: a_J = diag(exp(-i T e)) alpha."""
    w = inputs.make_workload("tiny", nt=50)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    a = O.propagate_state(s.h0, s.m, s.psi0, basis, w.dt, np.zeros(w.p))
    e = np.diag(s.h0)
    assert np.allclose(a, np.exp(-1j * w.nt * w.dt * e) * s.psi0, atol=1e-13)


def test_commuting_case_cost_grad_hess():
    """H0 = 0: a_J = exp(-i dt S M) alpha with S = 1^T B theta; closed-form g and H."""
    rng = np.random.default_rng(9)
    n, nt, dt, k = 4, 40, 0.05, 2
    m = _rand_sym(rng, n, 0.5)
    psi0 = np.zeros(n, complex)
    psi0[0] = 1
    beta = np.zeros(n, complex)
    beta[1] = 1
    basis = O.fourier_basis(nt, dt, k)
    theta = rng.normal(0, 0.3, 2 * k)
    gamma, rho = 0.7, 3.0
    w, v = np.linalg.eigh(m)
    s_vec = basis.sum(axis=0)
    S = s_vec @ theta
    a_j = (v * np.exp(-1j * dt * S * w)) @ v.T @ psi0
    r = a_j - beta
    f = basis @ theta
    cref = gamma / 2 * f @ f + rho / 2 * np.vdot(r, r).real
    gref = gamma * basis.T @ f + rho * dt * np.real(np.vdot(r, -1j * m @ a_j)) * s_vec
    href = gamma * basis.T @ basis + rho * dt ** 2 * (
        np.vdot(m @ a_j, m @ a_j).real - np.vdot(r, m @ m @ a_j).real) * np.outer(s_vec, s_vec)
    c, g, h = O.cost_grad_hess(np.zeros((n, n)), m, psi0, beta, basis, dt, theta, gamma, rho)
    assert abs(c - cref) < 1e-13
    assert np.allclose(g, gref, atol=1e-12)
    assert np.allclose(h, href, atol=1e-11)


def test_first_order_tangent_at_zero_field():
    """theta = 0: U_j = D = diag(exp(-i dt e)), U'_j = Phi(e) o M with first divided
    differences of exp(-i dt x); A'_J[:, l] = sum_i D^{J-1-i} U' D^i alpha B_il."""
    w = inputs.make_workload("tiny", nt=30)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    e = np.diag(s.h0)
    ph = np.exp(-1j * w.dt * e)
    n = len(e)
    phi = np.empty((n, n), complex)
    for p in range(n):
        for q in range(n):
            if p == q:
                phi[p, q] = -1j * w.dt * ph[p]
            else:
                phi[p, q] = (ph[p] - ph[q]) / (e[p] - e[q])
    u1 = phi * s.m
    ref = np.zeros((n, w.p), complex)
    for i in range(w.nt):
        vec = np.diag(ph ** (w.nt - 1 - i)) @ u1 @ (ph ** i * s.psi0)
        ref += np.outer(vec, basis[i])
    _, a1 = O.trajectory_with_tangents(s.h0, s.m, s.psi0, basis, w.dt, np.zeros(w.p), order=1)
    assert np.allclose(a1, ref, atol=1e-13)


def test_zero_rho_gives_field_energy_hessian():
    w = inputs.make_workload("tiny", nt=40)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    th = inputs.draw_thetas(w.p, 1, 3)[0]
    _, _, h = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th, w.gamma, 0.0)
    assert np.allclose(h, w.gamma * basis.T @ basis, atol=1e-14, rtol=0)


# ---------------------------------------------------------------- invariants

def test_norm_and_tangent_invariants():
    """|a_j| = |alpha|; Re(a^H a'_l) = 0; Re(a'_l^H a'_m + a^H a''_lm) = 0 at every step."""
    w = inputs.make_workload("tiny", nt=60)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    th = inputs.draw_thetas(w.p, 1, 4, sigma=0.5)[0]
    worst = [0.0, 0.0, 0.0]

    def obs(j, a, a1, a2):
        worst[0] = max(worst[0], abs(np.linalg.norm(a) - 1.0))
        worst[1] = max(worst[1], np.abs(np.real(a.conj() @ a1)).max())
        sec = np.real(a1.conj().T @ a1) + np.real(np.einsum("n,nlm->lm", a.conj(), a2))
        worst[2] = max(worst[2], np.abs(sec).max())

    O.trajectory_with_tangents(s.h0, s.m, s.psi0, basis, w.dt, th, order=2, observer=obs)
    assert worst[0] < 1e-13 and worst[1] < 1e-12 and worst[2] < 1e-11


# ------------------------------------------------------------ finite differences

def test_gradient_and_hessian_central_differences():
    w = inputs.make_workload("tiny", nt=80)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    th = inputs.draw_thetas(w.p, 1, 5, sigma=0.3)[0]
    args = (s.h0, s.m, s.psi0, s.psi_target, basis, w.dt)
    c, g, h = O.cost_grad_hess(*args, th, w.gamma, w.rho)
    step = 1e-6
    gfd = np.zeros(w.p)
    hfd = np.zeros((w.p, w.p))
    for l in range(w.p):
        e = np.zeros(w.p)
        e[l] = step
        gfd[l] = (O.cost(*args, th + e, w.gamma, w.rho) - O.cost(*args, th - e, w.gamma, w.rho)) / (2 * step)
        gp = O.cost_grad(*args, th + e, w.gamma, w.rho)[1]
        gm = O.cost_grad(*args, th - e, w.gamma, w.rho)[1]
        hfd[:, l] = (gp - gm) / (2 * step)
    assert np.linalg.norm(g - gfd) < 1e-8 * np.linalg.norm(g)
    assert np.linalg.norm(h - hfd) < 1e-7 * np.linalg.norm(h)
    assert np.linalg.norm(h - h.T) < 1e-13 * np.linalg.norm(h)


def test_hvp_matches_hessian_times_vector():
    w = inputs.make_workload("tiny", nt=50)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    th = inputs.draw_thetas(w.p, 1, 6)[0]
    v = inputs.draw_directions(w.p, 1, 6)[0]
    args = (s.h0, s.m, s.psi0, s.psi_target, basis, w.dt)
    _, _, h = O.cost_grad_hess(*args, th, w.gamma, w.rho)
    hv = O.hvp(*args, th, v, w.gamma, w.rho)
    assert np.allclose(hv, h @ v, atol=1e-13)


# --------------------------------------------------------------- brute force

@pytest.mark.slow
def test_brute_force_mpmath_tiny():
    """50-digit re-propagation with mpmath.expm; gradient and Hessian by FD at 50 digits."""
    w = inputs.make_workload("tiny", n=3, nt=10, k=1)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    basis = np.concatenate([basis, np.ones((w.nt, 1))], axis=1)  # P = 3 (dense basis)
    th = np.array([0.4, -0.7, 0.25])
    args = (s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th, w.gamma, w.rho)
    c, g, h = O.cost_grad_hess(*args)
    cref = float(brute.mp_cost(*args))
    gref = brute.mp_grad(*args)
    href = brute.mp_hess(*args)
    assert abs(c - cref) < 1e-15 * abs(cref) + 1e-16
    assert np.linalg.norm(g - gref) < 1e-13 * np.linalg.norm(gref)
    assert np.linalg.norm(h - href) < 1e-12 * np.linalg.norm(href)


# --------------------------------------------------------------- model / inputs

def test_fourier_model_values():
    """Sine columns vanish at t_0; at t = T/2 the cosine of harmonic k is cos(k pi / 2);
    the Gram matrix follows the finite cosine sums on the left-end-point grid."""
    nt, dt, k = 40, 0.05, 5
    b = O.fourier_basis(nt, dt, k)
    assert b.shape == (nt, 2 * k)
    assert np.all(b[0, k:] == 0) and np.all(b[0, :k] == 1)
    half = b[nt // 2, :k]
    assert np.allclose(half, [0, -1, 0, 1, 0], atol=1e-15)
    # sum_{j<J} cos(pi m j / J) = J (m = 0), 0 (m even != 0), 1 (m odd), |m| < 2J
    def csum(mm):
        if mm == 0:
            return nt
        return 0.0 if mm % 2 == 0 else 1.0
    gram = b[:, :k].T @ b[:, :k]
    for a in range(1, k + 1):
        for c in range(1, k + 1):
            ref = 0.5 * (csum(abs(a - c)) + csum(a + c))
            assert abs(gram[a - 1, c - 1] - ref) < 1e-12


def test_generators_deterministic():
    a = inputs.make_workload("molecule")
    b = inputs.make_workload("molecule")
    for x, y in ((a.system.h0, b.system.h0), (a.system.m, b.system.m),
                 (a.system.psi_target, b.system.psi_target)):
        assert x.tobytes() == y.tobytes()
    e = np.diag(a.system.h0)
    assert e.min() >= -3.0 and e.max() <= 0.0 and np.diff(e).min() >= 1e-3 - 1e-15
    assert abs(np.linalg.norm(a.system.psi_target) - 1) < 1e-15
    assert np.all(a.system.psi_target[6:] == 0)
    t1 = inputs.draw_thetas(32, 4, 2)
    t2 = inputs.draw_thetas(32, 4, 2)
    assert t1.tobytes() == t2.tobytes()
    tiny = inputs.make_workload("tiny")
    assert np.all(np.diag(tiny.system.m) == 0)
    ws = inputs.batched_workloads(8)
    assert [x.system.n for x in ws] == [x.system.n for x in inputs.batched_workloads(8)]
