"""A control model that is not linear in its parameters (a small tanh network of t) through the
second-order adjoint kernels (`qoc_eval_controls`), against the CPU oracle:

* dC/df and the cost against the oracle at the same samples (maximal model, f = theta);
* the gradient against J^T dC/df from the oracle, and against central differences of the
  oracle's cost of the composite model;
* the Hessian against J^T H_f J + sum_j (dC/df_j) d2f_j/dtheta2 with the oracle's H_f, and against
  central differences of the composite gradient built from the oracle."""
import sys

import numpy as np
import pytest

from oracle import qoc_oracle as O
from paper_2505_00529_amd import inputs, nonlinear, qoc

pytestmark = pytest.mark.gpu


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def test_neural_control_against_oracle():
    w = inputs.make_workload("tiny", nt=60)
    s = w.system
    model = nonlinear.NeuralControl(w.nt, w.dt, hidden=4)
    th = model.init_params(seed=3)
    p = qoc.Problem(0)
    p.set_system(s.h0, s.m, s.psi0, s.psi_target)
    p.set_weights(w.gamma, w.rho)
    c, g, h = nonlinear.evaluate(p, model, th)
    f = model.samples(th)
    jac = model.jacobian(th)
    eye = np.eye(w.nt)
    args = (s.h0, s.m, s.psi0, s.psi_target, eye, w.dt)
    cf, gf, hf = O.cost_grad_hess(*args, f, w.gamma, w.rho)
    _, _, _, dcdf = p.eval_controls(f, hessian=False)
    print(f"dC={_rel(c, cf):.2e} dcdf={_rel(dcdf, gf):.2e}", flush=True)
    assert _rel(c, cf) < 1e-12 and _rel(dcdf, gf) < 1e-10
    g_ref = jac.T @ gf
    h_ref = jac.T @ hf @ jac + model.curvature(th, gf)
    print(f"dg={_rel(g, g_ref):.2e} dH={_rel(h, h_ref):.2e}", flush=True)
    assert _rel(g, g_ref) < 1e-10 and _rel(h, h_ref) < 1e-10
    # central differences of the composite model through the oracle
    eps = 1e-5
    gfd = np.zeros(model.P)
    hfd = np.zeros((model.P, model.P))
    for l in range(model.P):
        e = np.zeros(model.P)
        e[l] = eps
        cp, gp = O.cost_grad(*args, model.samples(th + e), w.gamma, w.rho)
        cm, gm = O.cost_grad(*args, model.samples(th - e), w.gamma, w.rho)
        gfd[l] = (cp - cm) / (2 * eps)
        hfd[:, l] = (model.jacobian(th + e).T @ gp - model.jacobian(th - e).T @ gm) / (2 * eps)
    print(f"FD: dg={_rel(g, gfd):.2e} dH={_rel(h, hfd):.2e}", flush=True)
    sys.stdout.flush()
    assert _rel(g, gfd) < 1e-7 and _rel(h, hfd) < 1e-6
    p.close()
