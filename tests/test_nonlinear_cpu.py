"""The neural control model's own derivatives (host logic of the nonlinear-model layer): its
Jacobian against central differences of its samples, and its weighted curvature against central
differences of the weighted Jacobian."""
import numpy as np

from paper_2505_00529_amd.nonlinear import NeuralControl


def test_jacobian_and_curvature_against_central_differences():
    m = NeuralControl(nt=30, dt=0.05, hidden=4)
    th = m.init_params(seed=1)
    jac = m.jacobian(th)
    assert jac.shape == (30, m.P)
    h = 1e-6
    for l in range(m.P):
        e = np.zeros(m.P)
        e[l] = h
        fd = (m.samples(th + e) - m.samples(th - e)) / (2 * h)
        assert np.abs(fd - jac[:, l]).max() < 1e-8
    w = np.random.default_rng(2).normal(size=30)
    cur = m.curvature(th, w)
    assert np.abs(cur - cur.T).max() < 1e-12
    for l in range(m.P):
        e = np.zeros(m.P)
        e[l] = h
        fd = (m.jacobian(th + e).T @ w - m.jacobian(th - e).T @ w) / (2 * h)
        assert np.abs(fd - cur[:, l]).max() < 1e-7 * max(1.0, np.abs(cur).max())


def test_model_values():
    m = NeuralControl(nt=4, dt=0.1, hidden=1)
    th = np.array([2.0, -0.5, 3.0, 0.25])   # W1, b1, w2, b2
    s = np.arange(4) / 4
    assert np.allclose(m.samples(th), 3.0 * np.tanh(2.0 * s - 0.5) + 0.25, atol=1e-15)
