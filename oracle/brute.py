"""Brute-force high-precision re-propagation (oracle of the oracle), tiny inputs only.

TEST INFRASTRUCTURE ONLY.

The unwound cost (paper eq. costunwind) is evaluated in mpmath at 50 significant
digits with mpmath's own matrix exponential for every step, and its gradient and
Hessian are taken by central finite differences in that precision (step 1e-12:
truncation ~1e-24, rounding ~1e-26).  Intended for N <= 4, J <= 40, P <= 4.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

__all__ = ["mp_cost", "mp_grad", "mp_hess"]

_DPS = 50


def _mpmat(a):
    a = np.asarray(a)
    return mp.matrix([[mp.mpc(complex(a[i, j])) for j in range(a.shape[1])]
                      for i in range(a.shape[0])])


def _mpvec(v):
    return mp.matrix([mp.mpc(complex(x)) for x in np.asarray(v)])


def mp_cost(h0, m, psi0, psi_target, basis, dt, theta, gamma, rho):
    """Cost at 50 digits; basis, theta may be numpy arrays or lists of mpf."""
    with mp.workdps(_DPS):
        nt, p = np.asarray(basis).shape
        H0 = _mpmat(h0)
        M = _mpmat(m)
        a = _mpvec(psi0)
        beta = _mpvec(psi_target)
        th = [mp.mpf(x) if not isinstance(x, mp.mpf) else x for x in theta]
        B = [[mp.mpf(float(basis[j, k])) for k in range(p)] for j in range(nt)]
        energy = mp.mpf(0)
        dtm = mp.mpf(dt)
        for j in range(nt):
            f = mp.fsum(B[j][k] * th[k] for k in range(p))
            energy += f * f
            z = (H0 + f * M) * (-1j * dtm)
            a = mp.expm(z) * a
        r = a - beta
        err = mp.fsum(abs(r[i]) ** 2 for i in range(r.rows))
        return mp.mpf(gamma) / 2 * energy + mp.mpf(rho) / 2 * err


def mp_grad(h0, m, psi0, psi_target, basis, dt, theta, gamma, rho, h=1e-12):
    with mp.workdps(_DPS):
        th = [mp.mpf(float(x)) for x in theta]
        hh = mp.mpf(h)
        g = []
        for l in range(len(th)):
            tp = list(th)
            tm = list(th)
            tp[l] += hh
            tm[l] -= hh
            cp = mp_cost(h0, m, psi0, psi_target, basis, dt, tp, gamma, rho)
            cm = mp_cost(h0, m, psi0, psi_target, basis, dt, tm, gamma, rho)
            g.append((cp - cm) / (2 * hh))
        return np.array([float(x) for x in g])


def mp_hess(h0, m, psi0, psi_target, basis, dt, theta, gamma, rho, h=1e-12):
    """Mixed central differences; symmetric by construction."""
    with mp.workdps(_DPS):
        th = [mp.mpf(float(x)) for x in theta]
        hh = mp.mpf(h)
        p = len(th)

        def c(t):
            return mp_cost(h0, m, psi0, psi_target, basis, dt, t, gamma, rho)

        c0 = c(th)
        out = np.zeros((p, p))
        for l in range(p):
            tp = list(th)
            tm = list(th)
            tp[l] += hh
            tm[l] -= hh
            out[l, l] = float((c(tp) - 2 * c0 + c(tm)) / (hh * hh))
            for k in range(l + 1, p):
                vals = []
                for sl, sk in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                    t = list(th)
                    t[l] += sl * hh
                    t[k] += sk * hh
                    vals.append(c(t))
                hv = (vals[0] - vals[1] - vals[2] + vals[3]) / (4 * hh * hh)
                out[l, k] = out[k, l] = float(hv)
        return out
