"""Pins of the oracle MLP: gradients by finite differences, Adam, features."""

import numpy as np

import scenes
from oracle import contacts, mlp


def init(seed=0):
    return scenes.tensors.mlp_init(mlp.LAYERS, seed)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    params = init(3)
    X = rng.standard_normal((17, 11))
    Y = rng.standard_normal((17, 3))
    loss, grads = mlp.loss_and_grad(params, X, Y)
    h = 1e-6
    for pi in range(len(params)):
        p = params[pi]
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grad(params, X, Y)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grad(params, X, Y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[pi].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)) + 1e-9, (pi, idx, fd, g)


def test_adam_first_step_is_signed_learning_rate():
    # after one step from zero moments, every parameter moves by lr*sign(g)
    params = init(4)
    before = [p.copy() for p in params]
    grads = [np.full_like(p, 0.3) for p in params]
    grads[0][0, 0] = -2.0
    state = ([np.zeros_like(p) for p in params], [np.zeros_like(p) for p in params], 0)
    mlp.adam_step(params, grads, state, lr=1e-3)
    for b, p, g in zip(before, params, grads):
        assert np.allclose(b - p, 1e-3 * np.sign(g), atol=1e-9)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((256, 11))
    Y = np.stack([np.sin(X[:, 0]), 0.5 * X[:, 1], np.tanh(X[:, 2])], axis=1)
    params = init(5)
    state = ([np.zeros_like(p) for p in params], [np.zeros_like(p) for p in params], 0)
    l0, _ = mlp.loss_and_grad(params, X, Y)
    for _ in range(200):
        _, g = mlp.loss_and_grad(params, X, Y)
        state = mlp.adam_step(params, g, state)
    l1, _ = mlp.loss_and_grad(params, X, Y)
    assert l1 < 0.1 * l0


def test_prediction_is_strictly_inside_the_cone():
    rng = np.random.default_rng(3)
    params = init(6)
    g = mlp.predict_gamma(params, 3 * rng.standard_normal((500, 11)), mu=0.4)
    assert np.all(g[:, 0] > 0)
    assert np.all(np.hypot(g[:, 1], g[:, 2]) <= 0.9 * 0.4 * g[:, 0] * (1 + 1e-12))


def test_features_of_a_resting_sphere():
    sc = scenes.sphere_on_plane()
    c = contacts.detect(sc)
    F = mlp.features(sc, c)
    assert F.shape == (1, 11)
    assert np.allclose(F[0], [0, 0, 0, 0, 0, 0, 1, 1, 0, 1, 0], atol=1e-12)


def test_targets_round_trip_through_the_prediction_map():
    g = np.array([[2.0, 0.3, -0.1], [0.5, 0.0, 0.0]])
    y = mlp.targets(g.reshape(-1), mu=0.5)
    assert np.allclose(np.exp(y[:, 0]), g[:, 0])
    assert np.allclose(y[:, 1:] * 0.5 * g[:, :1], g[:, 1:])
