"""Pins of the oracle's K-direction functions (Sec. II, eq. matrixTDSE with three directions;
eq. d2Ldf2's sums over k and k, n) against facts that do not use its formulas:

* one direction reproduces the single-direction oracle;
* two directions with the same operator act as one control with f = f^1 + f^2, so the gradient
  blocks repeat and every Hessian block is the single-direction Hessian at the summed parameters;
* diagonal H0 and M_k (commuting) have a closed-form phase, hence closed-form cost, gradient and
  Hessian with mixed direction terms;
* rotating two directions into each other (and their parameters with them) changes nothing;
* finite differences on a non-commuting three-direction system, with a dense model per direction.
"""
import numpy as np
import pytest

from oracle import qoc_oracle as O


def _sym(rng, n, scale=1.0):
    a = rng.normal(size=(n, n))
    return scale * 0.5 * (a + a.T)


def _states(n):
    a = np.zeros(n, complex)
    a[0] = 1.0
    b = np.zeros(n, complex)
    b[-1] = 1.0
    return a, b


def test_one_direction_matches_single_direction_oracle():
    rng = np.random.default_rng(1)
    n, nt, dt = 4, 7, 0.2
    h0, m = _sym(rng, n), _sym(rng, n, 0.5)
    psi0, beta = _states(n)
    basis = O.fourier_basis(nt, dt, 2)
    th = rng.normal(size=4)
    c1, g1, h1 = O.cost_grad_hess(h0, m, psi0, beta, basis, dt, th, 0.3, 2.0)
    c2, g2, h2 = O.cost_grad_hess_multi(h0, [m], psi0, beta, basis[None], dt, th, 0.3, 2.0)
    assert abs(c1 - c2) < 1e-14 * abs(c1)
    assert np.abs(g1 - g2).max() < 1e-13 * np.abs(g1).max()
    assert np.abs(h1 - h2).max() < 1e-13 * np.abs(h1).max()
    v = rng.normal(size=4)
    assert np.abs(O.hvp_multi(h0, [m], psi0, beta, basis[None], dt, th, v, 0.3, 2.0) - h1 @ v).max() < 1e-12


def test_duplicated_operator_is_one_control_at_the_summed_parameters():
    rng = np.random.default_rng(2)
    n, nt, dt = 3, 6, 0.25
    h0, m = _sym(rng, n), _sym(rng, n, 0.7)
    psi0, beta = _states(n)
    basis = O.fourier_basis(nt, dt, 1)          # J x 2
    p0 = basis.shape[1]
    bases = np.zeros((2, nt, 2 * p0))
    bases[0, :, :p0] = basis
    bases[1, :, p0:] = basis
    th = rng.normal(size=2 * p0)
    c, g, h = O.cost_grad_hess_multi(h0, [m, m], psi0, beta, bases, dt, th, 0.0, 3.0)
    cs, gs, hs = O.cost_grad_hess(h0, m, psi0, beta, basis, dt, th[:p0] + th[p0:], 0.0, 3.0)
    assert abs(c - cs) < 1e-13
    assert np.abs(g - np.concatenate([gs, gs])).max() < 1e-12
    for a in range(2):
        for b in range(2):
            blk = h[a * p0:(a + 1) * p0, b * p0:(b + 1) * p0]
            assert np.abs(blk - hs).max() < 1e-11, (a, b)


def _closed_form(hd, md, psi0, beta, bases, dt, th, gamma, rho):
    """Diagonal system: a_J[p] = alpha_p exp(i phi_p), phi_p = -dt sum_j (h_p + sum_k f^k_j m_kp)."""
    f = np.einsum("kjl,l->kj", bases, th)
    phi = -dt * (hd * bases.shape[1] + np.einsum("kp,kj->p", md, f))
    dphi = -dt * np.einsum("kp,kjl->pl", md, bases)            # d phi_p / d theta_l
    a = psi0 * np.exp(1j * phi)
    r = a - beta
    c = 0.5 * gamma * (f * f).sum() + 0.5 * rho * np.vdot(r, r).real
    da = 1j * a[:, None] * dphi                                 # d a_p / d theta_l
    g = gamma * np.einsum("kjl,kj->l", bases, f) + rho * np.real(r.conj() @ da)
    d2a = -a[:, None, None] * dphi[:, :, None] * dphi[:, None, :]
    h = gamma * np.einsum("kjl,kjm->lm", bases, bases) + rho * np.real(da.conj().T @ da) \
        + rho * np.real(np.einsum("p,plm->lm", r.conj(), d2a))
    return c, g, h


def test_commuting_three_directions_closed_form():
    rng = np.random.default_rng(3)
    n, nt, dt, p = 4, 6, 0.3, 5
    hd = rng.normal(size=n)
    md = rng.normal(size=(3, n))
    psi0 = rng.normal(size=n) + 1j * rng.normal(size=n)
    psi0 /= np.linalg.norm(psi0)
    beta = rng.normal(size=n) + 1j * rng.normal(size=n)
    beta /= np.linalg.norm(beta)
    bases = rng.normal(size=(3, nt, p))                        # dense: every theta moves every direction
    th = rng.normal(size=p)
    c, g, h = O.cost_grad_hess_multi(np.diag(hd), [np.diag(x) for x in md], psi0, beta, bases, dt, th, 0.4, 2.5)
    cr, gr, hr = _closed_form(hd, md, psi0, beta, bases, dt, th, 0.4, 2.5)
    assert abs(c - cr) < 1e-12 * abs(cr)
    assert np.abs(g - gr).max() < 1e-11 * np.abs(gr).max()
    assert np.abs(h - hr).max() < 1e-11 * np.abs(hr).max()


def test_rotating_two_directions_changes_nothing():
    rng = np.random.default_rng(4)
    n, nt, dt = 4, 6, 0.2
    h0, m1, m2 = _sym(rng, n), _sym(rng, n, 0.6), _sym(rng, n, 0.6)
    psi0, beta = _states(n)
    basis = O.fourier_basis(nt, dt, 1)
    p0 = basis.shape[1]
    bases = np.zeros((2, nt, 2 * p0))
    bases[0, :, :p0] = basis
    bases[1, :, p0:] = basis
    th = rng.normal(size=2 * p0)
    ang = 0.7
    cs, sn = np.cos(ang), np.sin(ang)
    # f1 M1 + f2 M2 = f1' M1' + f2' M2' with M1' = c M1 + s M2, M2' = -s M1 + c M2,
    # f1' = c f1 + s f2, f2' = -s f1 + c f2; theta transforms the same way (Q orthogonal)
    q = np.block([[cs * np.eye(p0), sn * np.eye(p0)], [-sn * np.eye(p0), cs * np.eye(p0)]])
    c, g, h = O.cost_grad_hess_multi(h0, [m1, m2], psi0, beta, bases, dt, th, 0.5, 2.0)
    c2, g2, h2 = O.cost_grad_hess_multi(h0, [cs * m1 + sn * m2, -sn * m1 + cs * m2], psi0, beta, bases, dt,
                                        q @ th, 0.5, 2.0)
    assert abs(c - c2) < 1e-13
    assert np.abs(g - q.T @ g2).max() < 1e-12
    assert np.abs(h - q.T @ h2 @ q).max() < 1e-11


def test_three_directions_against_finite_differences():
    rng = np.random.default_rng(5)
    n, nt, dt, p = 3, 5, 0.3, 4
    h0 = _sym(rng, n)
    ms = [_sym(rng, n, 0.8) for _ in range(3)]
    psi0, beta = _states(n)
    bases = rng.normal(size=(3, nt, p))
    th = rng.normal(size=p)
    gamma, rho = 0.2, 3.0
    c, g, h = O.cost_grad_hess_multi(h0, ms, psi0, beta, bases, dt, th, gamma, rho)
    eps = 1e-5
    gf = np.zeros(p)
    hf = np.zeros((p, p))
    for l in range(p):
        e = np.zeros(p)
        e[l] = eps
        gf[l] = (O.cost_multi(h0, ms, psi0, beta, bases, dt, th + e, gamma, rho)
                 - O.cost_multi(h0, ms, psi0, beta, bases, dt, th - e, gamma, rho)) / (2 * eps)
        hf[:, l] = (O.cost_grad_multi(h0, ms, psi0, beta, bases, dt, th + e, gamma, rho)[1]
                    - O.cost_grad_multi(h0, ms, psi0, beta, bases, dt, th - e, gamma, rho)[1]) / (2 * eps)
    assert np.abs(g - gf).max() < 1e-8 * np.abs(g).max()
    assert np.abs(h - hf).max() < 1e-7 * np.abs(h).max()
    assert np.abs(h - h.T).max() < 1e-13 * np.abs(h).max()
    v = rng.normal(size=p)
    assert np.abs(O.hvp_multi(h0, ms, psi0, beta, bases, dt, th, v, gamma, rho) - h @ v).max() < 1e-12 * np.abs(h).max()
