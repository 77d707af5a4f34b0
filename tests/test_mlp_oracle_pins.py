"""Pins of the warm-start network oracle: finite differences of the loss,
a closed-form single-layer case, and Adam's first step."""
import numpy as np

from oracle import mlp_oracle as mo


def test_gradient_matches_finite_differences():
    g = np.random.default_rng(0)
    F, H, n = 5, 8, 40
    theta = mo.init_params(F, H, g) + 0.05 * g.standard_normal(mo.n_params(F, H))
    X = g.standard_normal((n, F))
    t = g.standard_normal(n)
    loss, grad = mo.loss_and_grad(theta, X, t, H)
    for k in g.choice(theta.size, 40, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mo.loss_and_grad(tp, X, t, H)[0] - mo.loss_and_grad(tm, X, t, H)[0]) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, grad[k], fd)


def test_network_with_identity_hidden_path_is_linear():
    """With all hidden units active and identity-like weights the network is
    the affine map X a + c: its output is checked against that closed form."""
    F, H, n = 3, 4, 10
    P = {"W1": np.zeros((F, H)), "b1": np.full(H, 5.0), "W2": np.eye(H), "b2": np.zeros(H),
         "W3": np.eye(H), "b3": np.zeros(H), "w4": np.array([1.0, 0.0, 0.0, 0.0]), "b4": np.array([-5.0])}
    P["W1"][:, 0] = [0.1, -0.2, 0.3]
    theta = np.concatenate([P[name].ravel() for name, _ in mo.shapes(F, H)])
    X = np.random.default_rng(1).uniform(-1, 1, size=(n, F))
    out, _ = mo.forward(theta, X, H)
    np.testing.assert_allclose(out, X @ np.array([0.1, -0.2, 0.3]), atol=1e-12)


def test_adam_first_step_moves_each_parameter_by_lr():
    """Bias-corrected Adam's first step is -lr * sign(g) (up to eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mo.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-8)
