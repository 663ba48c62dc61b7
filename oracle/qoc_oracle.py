"""Plain CPU FP64 oracle for the discretised quantum optimal-control objective.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.

What it computes (paper, Sec. II and Sec. III-A/B):

* the unwound cost (eq. costunwind, with eq. discretecost's field-energy term)
      C(theta) = (gamma/2) sum_j f_j^2 + (rho/2) || U_{J-1} ... U_1 U_0 alpha - beta ||^2,
  with U_j = exp(Z_j), Z_j = -i dt (H0 + f_j M) (eq. Zdef, eq. discTDSE), f_j = (B theta)_j
  the control model sampled at t_j = j dt (eq. eom), one control direction (the functions
  ending in _multi at the end of the module take K directions, H0 + sum_k f^k M_k);
* its gradient and Hessian, which the paper's adjoint methods reproduce exactly
  (eq. gradagree for the gradient; the Hessian is defined as the theta-Hessian of
  the unwound cost at the start of Sec. III-B);
* Hessian-vector products.

How: by the plain definition, with FORWARD-MODE sensitivities of the unwound
product, never by adjoints.  The per-step propagator and its first and second
f-derivatives come from one matrix exponential of the block upper-triangular matrix

      A = [[X, E, 0],
           [0, X, E],      X = -i dt (H0 + f M),   E = -i dt M,
           [0, 0, X]]

whose exponential is [[U, U', U''/2], [0, U, U'], [0, 0, U]] (Van Loan 1978, "Computing
integrals involving the matrix exponential"; Najfeld & Havel 1995, "Derivatives of the
matrix exponential and their computation").  This route shares no formula with an
eigendecomposition / divided-difference evaluation of the same derivatives.  The
exponential is a truncated Taylor series with scaling and squaring (Moler & Van Loan
2003, "Nineteen dubious ways to compute the exponential of a matrix", method 3).
Block upper-triangular Toeplitz matrices are closed under multiplication, so A and
its powers are carried as their three distinct blocks; a product of two such
matrices is (P0 Q0, P0 Q1 + P1 Q0, P0 Q2 + P1 Q1 + P2 Q0).

Conventions (readings of the paper where it is silent or inconsistent):
* f is sampled at left end points t_j = j dt, j = 0..J-1, T = J dt.
* Fourier model: B[j, k-1] = cos(k pi t_j / T), B[j, K+k-1] = sin(k pi t_j / T), k=1..K.
* gamma, rho are explicit weights; the paper's eq. discretecost has gamma = 1.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "fourier_basis",
    "identity_basis",
    "controls",
    "exp_block3",
    "step_propagators",
    "propagate_state",
    "cost",
    "cost_grad",
    "cost_grad_hess",
    "hvp",
    "trajectory_with_tangents",
    "controls_multi",
    "step_propagators_multi",
    "trajectory_with_tangents_multi",
    "cost_multi",
    "cost_grad_multi",
    "cost_grad_hess_multi",
    "hvp_multi",
]

_TAYLOR_TOL = 2.0 ** -60


# ----------------------------------------------------------------------------- model

def fourier_basis(nt: int, dt: float, k: int) -> np.ndarray:
    """J x 2K half-period Fourier model evaluated at t_j = j dt (model f(j dt; theta), Sec. II)."""
    t = dt * np.arange(nt)
    period = nt * dt
    harmonics = np.arange(1, k + 1)
    arg = np.pi * np.outer(t, harmonics) / period
    return np.concatenate([np.cos(arg), np.sin(arg)], axis=1)


def identity_basis(nt: int) -> np.ndarray:
    """Maximal (piecewise-constant) model f_j = theta_j (eq. maximal, one control)."""
    return np.eye(nt)


def controls(basis: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """f_j = sum_k B[j, k] theta_k."""
    return basis @ theta


# ----------------------------------------------------------------- block exponential

def _tmul(p, q):
    """Product of two block upper-triangular Toeplitz matrices given by their blocks."""
    return (p[0] @ q[0], p[0] @ q[1] + p[1] @ q[0], p[0] @ q[2] + p[1] @ q[1] + p[2] @ q[0])


def _tnorm1(p) -> float:
    """1-norm (max column sum) of the full 3N x 3N matrix with blocks (P0, P1, P2)."""
    c0 = np.abs(p[0]).sum(axis=0)
    c1 = np.abs(p[1]).sum(axis=0)
    c2 = np.abs(p[2]).sum(axis=0)
    return float(np.max(np.concatenate([c0, c0 + c1, c0 + c1 + c2])))


def exp_block3(x: np.ndarray, e: np.ndarray):
    """exp of [[X,E,0],[0,X,E],[0,0,X]] returned as its blocks (F0, F1, F2).

    F0 = exp(X), F1 = d/ds exp(X + sE)|0, F2 = (1/2) d^2/ds^2 exp(X + sE)|0.
    Taylor series with scaling and squaring: scale so that ||A||_1 / 2^s <= 1/2, sum
    terms until the term's 1-norm drops below 2^-60 times the running sum's, square s times.
    """
    n = x.shape[0]
    z = np.zeros((n, n), dtype=np.complex128)
    a = (x.astype(np.complex128), e.astype(np.complex128), z)
    nrm = _tnorm1(a)
    s = 0
    if nrm > 0.5:
        s = int(np.ceil(np.log2(nrm / 0.5)))
    scale = 2.0 ** (-s)
    a = (a[0] * scale, a[1] * scale, z)
    ident = np.eye(n, dtype=np.complex128)
    total = (ident.copy(), z.copy(), z.copy())
    term = (ident.copy(), z.copy(), z.copy())
    k = 0
    while True:
        k += 1
        term = _tmul(term, a)
        term = (term[0] / k, term[1] / k, term[2] / k)
        total = (total[0] + term[0], total[1] + term[1], total[2] + term[2])
        if _tnorm1(term) < _TAYLOR_TOL * _tnorm1(total) or k > 200:
            break
    for _ in range(s):
        total = _tmul(total, total)
    return total


def step_propagators(h0: np.ndarray, m: np.ndarray, f: float, dt: float):
    """(U, U', U'') of U(f) = exp(-i dt (H0 + f M)) and its first two f-derivatives."""
    x = -1j * dt * (h0 + f * m)
    e = -1j * dt * m
    f0, f1, f2 = exp_block3(x, e)
    return f0, f1, 2.0 * f2


# -------------------------------------------------------------------- forward mode

def propagate_state(h0, m, psi0, basis, dt, theta):
    """a_J = U_{J-1} ... U_0 alpha (eq. discTDSE, product ordered as in eq. costunwind)."""
    f = controls(basis, theta)
    a = np.asarray(psi0, dtype=np.complex128).copy()
    for j in range(basis.shape[0]):
        u = step_propagators(h0, m, f[j], dt)[0]
        a = u @ a
    return a


def cost(h0, m, psi0, psi_target, basis, dt, theta, gamma, rho) -> float:
    """Unwound cost (eq. costunwind) with field-energy weight gamma."""
    f = controls(basis, theta)
    a = propagate_state(h0, m, psi0, basis, dt, theta)
    r = a - psi_target
    return 0.5 * gamma * float(f @ f) + 0.5 * rho * float(np.vdot(r, r).real)


def trajectory_with_tangents(h0, m, psi0, basis, dt, theta, order=1, direction=None,
                             observer=None):
    """Forward sweep of the state and its theta-derivatives.

    order=1: returns (a_J, A'_J) with A'_J[:, l] = d a_J / d theta_l.
    order=2: also A''_J[:, l, m] = d^2 a_J / d theta_l d theta_m.
    direction=v (with order=2): returns (a_J, A'_J, a'_J[v], A''_J[:, :, v]) instead of the
    full second-order tensor, i.e. only second derivatives contracted with v.

    Recurrences (total derivatives of a_{j+1} = U(f_j) a_j, d a_0 = 0, eq. gradatheta):
      a'_{j+1}  = U a'_j + U' a_j b_j
      a''_{j+1} = U a''_j + U'(a'_j b_j^T + b_j a'_j^T) + U'' a_j b_j b_j^T
    observer(j, a_j, A'_j, A''_j) is called before each step (for invariant tests).
    """
    basis = np.asarray(basis, dtype=np.float64)
    nt, p = basis.shape
    n = h0.shape[0]
    f = controls(basis, theta)
    a = np.asarray(psi0, dtype=np.complex128).copy()
    a1 = np.zeros((n, p), dtype=np.complex128)
    if direction is not None:
        u = basis @ np.asarray(direction, dtype=np.float64)
        av = np.zeros(n, dtype=np.complex128)
        a2 = np.zeros((n, p), dtype=np.complex128)
    elif order >= 2:
        a2 = np.zeros((n, p, p), dtype=np.complex128)
    for j in range(nt):
        if observer is not None:
            observer(j, a, a1, a2 if order >= 2 else None)
        uj, u1, u2 = step_propagators(h0, m, f[j], dt)
        b = basis[j]
        if order >= 2 and direction is None:
            w = u1 @ a1
            a2_next = (uj @ a2.reshape(n, p * p)).reshape(n, p, p)
            a2_next += w[:, :, None] * b[None, None, :] + w[:, None, :] * b[None, :, None]
            a2_next += (u2 @ a)[:, None, None] * np.outer(b, b)[None, :, :]
            a2 = a2_next
        elif direction is not None:
            w = u1 @ a1
            wv = u1 @ av
            a2 = uj @ a2 + w * u[j] + np.outer(wv, b) + np.outer(u2 @ a, b) * u[j]
            av = uj @ av + (u1 @ a) * u[j]
        a1_next = uj @ a1 + np.outer(u1 @ a, b)
        a = uj @ a
        a1 = a1_next
    if direction is not None:
        return a, a1, av, a2
    if order >= 2:
        return a, a1, a2
    return a, a1


def cost_grad(h0, m, psi0, psi_target, basis, dt, theta, gamma, rho):
    """(C, dC/dtheta) by forward-mode tangents of the unwound cost."""
    basis = np.asarray(basis, dtype=np.float64)
    f = controls(basis, theta)
    a, a1 = trajectory_with_tangents(h0, m, psi0, basis, dt, theta, order=1)
    r = a - psi_target
    c = 0.5 * gamma * float(f @ f) + 0.5 * rho * float(np.vdot(r, r).real)
    g = gamma * (basis.T @ f) + rho * np.real(r.conj() @ a1)
    return c, g


def cost_grad_hess(h0, m, psi0, psi_target, basis, dt, theta, gamma, rho):
    """(C, g, H) by first- and second-order forward-mode tangents of the unwound cost.

    H_lm = gamma (B^T B)_lm + rho Re( a'_l^H a'_m + r^H a''_lm ),   r = a_J - beta.
    """
    basis = np.asarray(basis, dtype=np.float64)
    f = controls(basis, theta)
    a, a1, a2 = trajectory_with_tangents(h0, m, psi0, basis, dt, theta, order=2)
    r = a - psi_target
    c = 0.5 * gamma * float(f @ f) + 0.5 * rho * float(np.vdot(r, r).real)
    g = gamma * (basis.T @ f) + rho * np.real(r.conj() @ a1)
    h = gamma * (basis.T @ basis) + rho * np.real(a1.conj().T @ a1) \
        + rho * np.real(np.einsum("n,nlm->lm", r.conj(), a2))
    return c, g, h


def hvp(h0, m, psi0, psi_target, basis, dt, theta, v, gamma, rho):
    """H v by directional second-order forward mode (no full Hessian formed).

    (H v)_l = gamma (B^T B v)_l + rho Re( a'_l^H a'[v] + r^H a''_l[v] ).
    """
    basis = np.asarray(basis, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    a, a1, av, a2v = trajectory_with_tangents(h0, m, psi0, basis, dt, theta, order=2,
                                              direction=v)
    r = a - psi_target
    return gamma * (basis.T @ (basis @ v)) + rho * np.real(a1.conj().T @ av) \
        + rho * np.real(r.conj() @ a2v)


# ------------------------------------------------------------- several control directions
#
# Sec. II with K control directions (eq. matrixTDSE: H0 + sum_k f^k(t) M_k, K <= 3 in the paper):
# Z_j = -i dt (H0 + sum_k f^k_j M_k), f^k_j = (B_k theta)_j with one J x P model matrix per
# direction (a model with a block of theta per direction has zero columns elsewhere).  The
# theta-derivatives of the unwound cost follow by the chain rule through every direction (the
# sums over k in the gradient and over k, n in the Hessian, eq. d2Ldf2).  The per-step
# derivatives come from the same block exponential: U'_k = dU/df^k is its first block for
# E = -i dt M_k, and the mixed second derivative U''_kn, a symmetric bilinear form in the
# directions, follows by polarisation from second derivatives along single directions:
#   U''_kn = (U''[M_k + M_n] - U''[M_k] - U''[M_n]) / 2,   U''[D] = d^2/ds^2 exp(X + s E_D).


def controls_multi(bases: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """f^k_j = sum_l B_k[j, l] theta_l for every direction k: K x J."""
    return np.einsum("kjl,l->kj", np.asarray(bases, dtype=np.float64), np.asarray(theta, dtype=np.float64))


def step_propagators_multi(h0, ms, fvec, dt):
    """(U, [U'_k], [[U''_kn]]) of U = exp(-i dt (H0 + sum_k f_k M_k))."""
    K = len(ms)
    x = -1j * dt * (np.asarray(h0) + sum(fvec[k] * ms[k] for k in range(K)))
    first, second_single = [], []
    u = None
    for k in range(K):
        f0, f1, f2 = exp_block3(x, -1j * dt * ms[k])
        u = f0
        first.append(f1)
        second_single.append(2.0 * f2)
    second = [[None] * K for _ in range(K)]
    for k in range(K):
        second[k][k] = second_single[k]
        for n in range(k + 1, K):
            both = 2.0 * exp_block3(x, -1j * dt * (ms[k] + ms[n]))[2]
            mixed = 0.5 * (both - second_single[k] - second_single[n])
            second[k][n] = mixed
            second[n][k] = mixed
    return u, first, second


def trajectory_with_tangents_multi(h0, ms, psi0, bases, dt, theta, order=1, direction=None):
    """Forward sweep with K directions; returns as trajectory_with_tangents.

      a'_{j+1}  = U a'_j + sum_k U'_k a_j b_kj^T
      a''_{j+1} = U a''_j + sum_k U'_k (a'_j b_kj^T + b_kj a'_j^T) + sum_kn U''_kn a_j b_kj b_nj^T
    with b_kj = B_k[j, :].
    """
    bases = np.asarray(bases, dtype=np.float64)
    K, nt, p = bases.shape
    n = h0.shape[0]
    f = controls_multi(bases, theta)
    a = np.asarray(psi0, dtype=np.complex128).copy()
    a1 = np.zeros((n, p), dtype=np.complex128)
    if direction is not None:
        u = np.einsum("kjl,l->kj", bases, np.asarray(direction, dtype=np.float64))
        av = np.zeros(n, dtype=np.complex128)
        a2 = np.zeros((n, p), dtype=np.complex128)
    elif order >= 2:
        a2 = np.zeros((n, p, p), dtype=np.complex128)
    for j in range(nt):
        uj, u1, u2 = step_propagators_multi(h0, ms, f[:, j], dt)
        b = bases[:, j, :]
        if order >= 2 and direction is None:
            a2_next = (uj @ a2.reshape(n, p * p)).reshape(n, p, p)
            for k in range(K):
                w = u1[k] @ a1
                a2_next += w[:, :, None] * b[k][None, None, :] + w[:, None, :] * b[k][None, :, None]
                for m in range(K):
                    a2_next += (u2[k][m] @ a)[:, None, None] * np.outer(b[k], b[m])[None, :, :]
            a2 = a2_next
        elif direction is not None:
            a2_next = uj @ a2
            av_next = uj @ av
            for k in range(K):
                a2_next += (u1[k] @ a1) * u[k, j] + np.outer(u1[k] @ av, b[k])
                for m in range(K):
                    a2_next += np.outer(u2[k][m] @ a, b[k]) * u[m, j]
                av_next += (u1[k] @ a) * u[k, j]
            a2, av = a2_next, av_next
        a1_next = uj @ a1
        for k in range(K):
            a1_next += np.outer(u1[k] @ a, b[k])
        a = uj @ a
        a1 = a1_next
    if direction is not None:
        return a, a1, av, a2
    if order >= 2:
        return a, a1, a2
    return a, a1


def _field_terms(bases, f):
    """sum_k B_k^T f^k and sum_k B_k^T B_k."""
    return np.einsum("kjl,kj->l", bases, f), np.einsum("kjl,kjm->lm", bases, bases)


def cost_multi(h0, ms, psi0, psi_target, bases, dt, theta, gamma, rho) -> float:
    """Unwound cost with K directions; the field energy sums over directions."""
    bases = np.asarray(bases, dtype=np.float64)
    f = controls_multi(bases, theta)
    a, _ = trajectory_with_tangents_multi(h0, ms, psi0, bases, dt, theta, order=1)
    r = a - psi_target
    return 0.5 * gamma * float((f * f).sum()) + 0.5 * rho * float(np.vdot(r, r).real)


def cost_grad_multi(h0, ms, psi0, psi_target, bases, dt, theta, gamma, rho):
    """(C, dC/dtheta) with K directions."""
    bases = np.asarray(bases, dtype=np.float64)
    f = controls_multi(bases, theta)
    a, a1 = trajectory_with_tangents_multi(h0, ms, psi0, bases, dt, theta, order=1)
    r = a - psi_target
    c = 0.5 * gamma * float((f * f).sum()) + 0.5 * rho * float(np.vdot(r, r).real)
    bf, _ = _field_terms(bases, f)
    return c, gamma * bf + rho * np.real(r.conj() @ a1)


def cost_grad_hess_multi(h0, ms, psi0, psi_target, bases, dt, theta, gamma, rho):
    """(C, g, H) with K directions: H = gamma sum_k B_k^T B_k + rho Re(A'^H A' + r^H A'')."""
    bases = np.asarray(bases, dtype=np.float64)
    f = controls_multi(bases, theta)
    a, a1, a2 = trajectory_with_tangents_multi(h0, ms, psi0, bases, dt, theta, order=2)
    r = a - psi_target
    c = 0.5 * gamma * float((f * f).sum()) + 0.5 * rho * float(np.vdot(r, r).real)
    bf, bb = _field_terms(bases, f)
    g = gamma * bf + rho * np.real(r.conj() @ a1)
    h = gamma * bb + rho * np.real(a1.conj().T @ a1) + rho * np.real(np.einsum("n,nlm->lm", r.conj(), a2))
    return c, g, h


def hvp_multi(h0, ms, psi0, psi_target, bases, dt, theta, v, gamma, rho):
    """H v with K directions by directional second-order forward mode."""
    bases = np.asarray(bases, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    a, a1, av, a2v = trajectory_with_tangents_multi(h0, ms, psi0, bases, dt, theta, order=2, direction=v)
    r = a - psi_target
    _, bb = _field_terms(bases, np.zeros(bases.shape[:2]))
    return gamma * (bb @ v) + rho * np.real(a1.conj().T @ av) + rho * np.real(r.conj() @ a2v)
