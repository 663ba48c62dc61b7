"""Pins of the CPU oracle on complex Hermitian systems (H0, M complex Hermitian, as in the paper's
timing runs with random Hermitian dipole matrices).  The oracle's formulas are written for any
Hermitian H0 and M; these checks fix the complex case against facts that do not come from the
oracle itself:

* gauge invariance: for a diagonal unitary D, the system (D H0 D^H, D M D^H, D alpha, D beta) has
  the same cost, gradient and Hessian as (H0, M, alpha, beta); with a real system on one side the
  complex side is pinned by the real-case pins;
* H0 = 0 closed forms with a genuinely complex M: a_J = V exp(-i dt S Lambda) V^H alpha from
  numpy's eigh of M, and the commuting-case gradient and Hessian;
* unitarity invariants of U, U', U'' for complex Hermitian H0 and M;
* central differences of the cost (gradient) and of the gradient (Hessian).
"""
import numpy as np

from oracle import qoc_oracle as O


def _herm(rng, n, scale):
    a = rng.normal(0, scale, (n, n)) + 1j * rng.normal(0, scale, (n, n))
    return 0.5 * (a + a.conj().T)


def _unit(n, i):
    v = np.zeros(n, complex)
    v[i] = 1.0
    return v


def test_gauge_transform_of_a_real_system():
    rng = np.random.default_rng(21)
    n, nt, dt, k = 5, 30, 0.05, 2
    h0 = np.diag(np.sort(rng.uniform(-1.5, 0, n)))
    m = rng.normal(0, 0.5, (n, n))
    m = 0.5 * (m + m.T)
    alpha, beta = _unit(n, 0), _unit(n, 3)
    d = np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    hc = (d[:, None] * h0) * d.conj()[None, :]
    mc = (d[:, None] * m) * d.conj()[None, :]
    assert np.abs(mc.imag).max() > 0.1          # genuinely complex
    basis = O.fourier_basis(nt, dt, k)
    th = rng.normal(0, 0.4, 2 * k)
    cr, gr, hr = O.cost_grad_hess(h0, m, alpha, beta, basis, dt, th, 0.3, 2.0)
    cc, gc, hc2 = O.cost_grad_hess(hc, mc, d * alpha, d * beta, basis, dt, th, 0.3, 2.0)
    assert abs(cc - cr) < 1e-13 * abs(cr)
    assert np.linalg.norm(gc - gr) < 1e-12 * np.linalg.norm(gr)
    assert np.linalg.norm(hc2 - hr) < 1e-12 * np.linalg.norm(hr)


def test_commuting_case_with_complex_dipole():
    rng = np.random.default_rng(22)
    n, nt, dt, k = 4, 40, 0.05, 2
    m = _herm(rng, n, 0.5)
    psi0 = (rng.normal(size=n) + 1j * rng.normal(size=n))
    psi0 /= np.linalg.norm(psi0)
    beta = _unit(n, 2)
    basis = O.fourier_basis(nt, dt, k)
    theta = rng.normal(0, 0.3, 2 * k)
    gamma, rho = 0.7, 3.0
    w, v = np.linalg.eigh(m)
    s_vec = basis.sum(axis=0)
    a_j = (v * np.exp(-1j * dt * (s_vec @ theta) * w)) @ v.conj().T @ psi0
    r = a_j - beta
    f = basis @ theta
    cref = gamma / 2 * f @ f + rho / 2 * np.vdot(r, r).real
    gref = gamma * basis.T @ f + rho * dt * np.real(np.vdot(r, -1j * m @ a_j)) * s_vec
    href = gamma * basis.T @ basis + rho * dt ** 2 * (
        np.vdot(m @ a_j, m @ a_j).real - np.vdot(r, m @ m @ a_j).real) * np.outer(s_vec, s_vec)
    c, g, h = O.cost_grad_hess(np.zeros((n, n), complex), m, psi0, beta, basis, dt, theta, gamma, rho)
    assert abs(c - cref) < 1e-13
    assert np.allclose(g, gref, atol=1e-12)
    assert np.allclose(h, href, atol=1e-11)


def test_unitarity_invariants_complex():
    rng = np.random.default_rng(23)
    n, dt, f = 6, 0.2, 0.4
    h0 = _herm(rng, n, 1.0)
    m = _herm(rng, n, 0.3)
    u, u1, u2 = O.step_propagators(h0, m, f, dt)
    h = lambda a: a.conj().T
    assert np.allclose(h(u) @ u, np.eye(n), atol=1e-14)
    assert np.allclose(h(u) @ u1 + h(u1) @ u, 0, atol=1e-14)
    assert np.allclose(h(u2) @ u + 2 * h(u1) @ u1 + h(u) @ u2, 0, atol=1e-14)


def test_central_differences_complex():
    rng = np.random.default_rng(24)
    n, nt, dt, k = 4, 25, 0.08, 2
    h0 = _herm(rng, n, 1.0)
    m = _herm(rng, n, 0.5)
    alpha, beta = _unit(n, 0), _unit(n, n - 1)
    basis = O.fourier_basis(nt, dt, k)
    th = rng.normal(0, 0.5, 2 * k)
    args = (h0, m, alpha, beta, basis, dt)
    c, g, hs = O.cost_grad_hess(*args, th, 1.0, 5.0)
    eps = 1e-5
    for l in range(2 * k):
        e = np.zeros(2 * k)
        e[l] = eps
        cp = O.cost(*args, th + e, 1.0, 5.0)
        cm = O.cost(*args, th - e, 1.0, 5.0)
        assert abs((cp - cm) / (2 * eps) - g[l]) < 1e-7 * max(1.0, abs(g[l]))
        gp = O.cost_grad(*args, th + e, 1.0, 5.0)[1]
        gm = O.cost_grad(*args, th - e, 1.0, 5.0)[1]
        assert np.linalg.norm((gp - gm) / (2 * eps) - hs[:, l]) < 1e-6 * max(1.0, np.linalg.norm(hs[:, l]))
