"""Pins of the CPU reference MLP used to check the device network."""
import numpy as np
import torch

from oracle import mlp_ref as R


def test_bf16_round_matches_torch_and_known_values():
    rng = np.random.Generator(np.random.PCG64(11))
    x = np.concatenate([rng.normal(size=4000).astype(np.float32) * np.float32(10.0) ** rng.integers(-6, 6, 4000),
                        np.array([0.0, -0.0, 1.0, -2.5, 3.0e38, 1e-40], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(R.bf16_round(x), ref)
    # ties go to even: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7
    assert R.bf16_round(np.float32(1 + 2.0 ** -8)) == 1.0
    assert R.bf16_round(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6


def test_fp64_mlp_gradient_matches_central_differences():
    n_in, h, n_out, batch = 5, 7, 3, 4
    rng = np.random.Generator(np.random.PCG64(12))
    p = R.init_params(n_in, h, n_out, 3).astype(np.float64)
    x = rng.normal(size=(batch, n_in))
    t = rng.normal(size=(batch, n_out))
    loss, g, _ = R.loss_and_grads(p, x, t, n_in, h, n_out)
    fd = np.zeros_like(p)
    eps = 1e-6
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        fd[i] = (R.loss_and_grads(p + e, x, t, n_in, h, n_out)[0] - R.loss_and_grads(p - e, x, t, n_in, h, n_out)[0]) / (2 * eps)
    assert np.abs(g - fd).max() < 1e-8 * max(1.0, np.abs(fd).max())
    assert loss > 0


def test_gelu_special_values_and_linear_identity():
    # one hidden unit per layer with unit weights and zero biases: y = gelu(gelu(x));
    # gelu(0) = 0 and gelu(z) -> z for large z, -> 0 for very negative z
    p = R.pack([np.ones((1, 1)), np.zeros(1), np.ones((1, 1)), np.zeros(1), np.ones((1, 1)), np.zeros(1)])
    y = R.forward(p, np.array([[0.0], [40.0], [-40.0]]), 1, 1, 1)["y"].ravel()
    assert y[0] == 0.0 and abs(y[1] - 40.0) < 1e-12 and abs(y[2]) < 1e-12
    # gelu(1) = 0.5 (1 + erf(1/sqrt 2)) = Phi(1) = 0.8413447460685429
    p1 = R.pack([np.ones((1, 1)), np.zeros(1), np.eye(1), np.full(1, -10.0), np.zeros((1, 1)), np.zeros(1)])
    z1 = R.forward(p1, np.array([[1.0]]), 1, 1, 1)
    assert abs(z1["a1"][0, 0] - 0.8413447460685429) < 1e-15


def test_adam_first_step_is_signed_learning_rate():
    # after one bias-corrected step m_hat = g and v_hat = g^2, so the update is -lr * sign(g)
    # (up to eps), and a zero gradient leaves the parameter where it is
    g = np.array([3.0, -1e-3, 0.0])
    p1, m, v = R.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, [-0.01, 0.01, 0.0], rtol=1e-4, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_bias_correction_over_several_steps():
    # A constant gradient g gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so with the bias
    # correction every step moves by -lr * sign(g) (up to eps), not only the first.
    g = np.array([2.0, -0.5, 1e-3])
    lr, b1, b2 = 0.01, 0.9, 0.999
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 8):
        p_new, m, v = R.adam_step(p, g, m, v, t, lr, b1, b2)
        assert np.allclose(p_new - p, -lr * np.sign(g), rtol=1e-4, atol=0), t
        assert np.allclose(m, (1 - b1 ** t) * g) and np.allclose(v, (1 - b2 ** t) * g * g)
        p = p_new
    # a sign flip at the second step: m_2 = -(1 - b1)^2 g, bias-corrected -(1 - b1)/(1 + b1) g,
    # and v_2 = (1 - b2)(1 + b2) g^2, bias-corrected g^2: the second step is
    # +lr (1 - b1)/(1 + b1) sign(g)
    p1, m, v = R.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr, b1, b2)
    p2, m, v = R.adam_step(p1, -g, m, v, 2, lr, b1, b2)
    assert np.allclose(p2 - p1, lr * (1 - b1) / (1 + b1) * np.sign(g), rtol=1e-4, atol=0)
