"""Pins of the FP64 estimator oracle (27 -> 64 -> 64 -> 4 tanh network).

* gradient = central finite differences of the loss (relative 1e-6);
* a network with a single active path computes the closed form
  w3 tanh(w2 tanh(w1.x + b1) + b2) + b3;
* Adam's first bias-corrected step moves every parameter by lr * sign(g),
  and Adam minimises a quadratic.
"""
import numpy as np

from oracle import oracle as O

NP = 6212


def split(p):
    out, o = {}, 0
    for name, shp in O.MLP_SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def random_params(rng, scale=0.3):
    return scale * rng.standard_normal(NP)


def random_batch(rng, n):
    x = rng.uniform(-0.5, 0.5, (n, 27))
    t = rng.standard_normal((n, 4))
    t[:, :3] /= np.linalg.norm(t[:, :3], axis=1, keepdims=True)
    t[:, 3] *= 0.1
    return x, t


def test_parameter_count():
    assert O.mlp_nparam() == NP == 27 * 64 + 64 + 64 * 64 + 64 + 4 * 64 + 4


def test_single_path_closed_form():
    rng = np.random.default_rng(0)
    p = np.zeros(NP)
    q = split(p)
    w1 = rng.standard_normal(27)
    q["W1"][5] = w1
    q["b1"][5] = 0.3
    q["W2"][9, 5] = -1.7
    q["b2"][9] = 0.2
    q["W3"][3, 9] = 2.5
    q["W3"][1, 9] = -0.5
    q["b3"][:] = [0.1, 0.2, 0.3, 0.4]
    x = rng.uniform(-0.5, 0.5, (7, 27))
    y = O.mlp_forward(p, x)
    h = np.tanh(-1.7 * np.tanh(x @ w1 + 0.3) + 0.2)
    # unused hidden units still carry tanh(b) = tanh(0) = 0
    assert np.allclose(y[:, 3], 2.5 * h + 0.4, atol=1e-15, rtol=0)
    assert np.allclose(y[:, 1], -0.5 * h + 0.2, atol=1e-15, rtol=0)
    assert np.allclose(y[:, 0], 0.1, atol=1e-15) and np.allclose(y[:, 2], 0.3, atol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = random_params(rng)
    x, t = random_batch(rng, 16)
    loss, g = O.mlp_loss_grad(p, x, t)
    idx = rng.choice(NP, 200, replace=False)
    idx = np.concatenate([idx, [0, 27 * 64, 27 * 64 + 64, NP - 4, NP - 1, NP - 260]])
    for i in idx:
        h = 1e-5 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (O.mlp_loss_grad(pp, x, t, False)[0] - O.mlp_loss_grad(pm, x, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_loss_is_zero_at_perfect_prediction():
    rng = np.random.default_rng(2)
    p = np.zeros(NP)
    q = split(p)
    q["b3"][:] = [0.0, 0.0, 1.0, 0.8]   # predicts n = +z, 4 kappa = 0.8
    x, _ = random_batch(rng, 5)
    t = np.tile([0.0, 0.0, 1.0, 0.2], (5, 1))
    loss, g = O.mlp_loss_grad(p, x, t)
    assert loss == 0.0 and np.all(g == 0.0)


def test_adam_first_step_and_quadratic():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(NP)
    g = rng.standard_normal(NP)
    m, v = np.zeros(NP), np.zeros(NP)
    p0 = p.copy()
    O.mlp_adam(p, m, v, g, 1, lr=1e-3, eps=0.0)
    assert np.allclose(p0 - p, 1e-3 * np.sign(g), rtol=1e-12, atol=0)
    # minimise sum (p - c)^2
    c = rng.standard_normal(NP)
    p = np.zeros(NP)
    m, v = np.zeros(NP), np.zeros(NP)
    for t in range(1, 3001):
        O.mlp_adam(p, m, v, 2 * (p - c), t, lr=1e-2)
    assert np.max(np.abs(p - c)) < 1e-2
