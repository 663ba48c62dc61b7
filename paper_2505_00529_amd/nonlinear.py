"""Control models that are not linear in their parameters.

Sec. II lets the control be any smooth model f(t; theta), and the paper names neural networks of t
as the models to try next.  For such a model the derivatives of C(theta) = C(f(theta)) follow from
the chain rule:

    grad = J^T dC/df,    Hess = J^T (d2C/df2) J + sum_j (dC/df_j) d2f_j/dtheta2,

with J = df/dtheta (nt x P).  The second-order adjoint kernels give the first term of each (they
take J as a dense control basis and the samples f directly, `qoc_eval_controls`) and dC/df; the
model supplies J and the last term, its own curvature weighted by dC/df.  Here the model is a
small tanh network of the normalised time, differentiated with torch.func in float64 on the host
(the model's derivatives, not the propagation, are what the host computes).
"""
from __future__ import annotations

import numpy as np
import torch

from . import qoc


class NeuralControl:
    """f(t_j; theta) = sum_k w2_k tanh(W1_k s_j + b1_k) + b2 with s_j = t_j / T = j / nt (left end
    points, as for the other models); theta = [W1, b1, w2, b2], P = 3 hidden + 1."""

    def __init__(self, nt: int, dt: float, hidden: int = 8):
        self.nt, self.dt, self.hidden = nt, dt, hidden
        self.P = 3 * hidden + 1
        self.s = torch.arange(nt, dtype=torch.float64) / nt

    def _f(self, th: torch.Tensor) -> torch.Tensor:
        h = self.hidden
        z = torch.tanh(self.s[:, None] * th[None, :h] + th[None, h:2 * h])
        return z @ th[2 * h:3 * h] + th[3 * h]

    @staticmethod
    def _t(theta) -> torch.Tensor:
        return torch.as_tensor(np.asarray(theta, dtype=np.float64))

    def init_params(self, seed: int = 0, scale: float = 0.5) -> np.ndarray:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 8191])))
        return rng.normal(0.0, scale, self.P)

    def samples(self, theta) -> np.ndarray:
        """f(t_j; theta), nt values."""
        with torch.no_grad():
            return self._f(self._t(theta)).numpy()

    def jacobian(self, theta) -> np.ndarray:
        """df/dtheta, nt x P, in forward mode (P tangents instead of nt cotangents: P << nt)."""
        return torch.func.jacfwd(self._f)(self._t(theta)).numpy()

    def curvature(self, theta, w) -> np.ndarray:
        """sum_j w_j d2f_j/dtheta2, P x P."""
        wt = torch.as_tensor(np.asarray(w, dtype=np.float64))
        return torch.func.hessian(lambda th: (self._f(th) * wt).sum())(self._t(theta)).numpy()


def evaluate(problem: qoc.Problem, model: NeuralControl, theta, hessian: bool = True):
    """(cost, gradient, Hessian or None) of C(f(theta)) for a handle whose system and weights are
    set; its control basis is replaced by the model's Jacobian at theta."""
    f = model.samples(theta)
    jac = model.jacobian(theta)
    problem.set_control_basis(qoc.QOC_BASIS_DENSE, model.nt, model.dt, model.P, jac)
    c, g, h_adj, dcdf = problem.eval_controls(f, hessian)
    if not hessian:
        return c, g, None
    return c, g, h_adj + model.curvature(theta, dcdf)
