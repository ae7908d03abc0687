"""Pins of the selector-network oracle: gradients against central finite
differences, the Adam step against its closed form on a quadratic, and a fit of
a smooth function to show the pieces work together."""
import numpy as np

from oracle import mlp
from workloads.rng import SplitMix64


def _setup(m=37, seed=3):
    g = SplitMix64(seed)
    params = mlp.init_params(g.uniform)
    X = g.uniform(m * 5, -1, 1).reshape(m, 5)
    Y = g.uniform(m * 9, -2, 2).reshape(m, 9)
    M = (g.uniform(m * 9) < 0.8).astype(np.float64).reshape(m, 9)
    return params, X, Y, M


def test_gradients_match_central_differences():
    params, X, Y, M = _setup()
    _, grads = mlp.loss_and_grads(params, X, Y, M)
    g = SplitMix64(99)
    h = 1e-6
    for li, p in enumerate(params):
        for _ in range(6):
            idx = tuple(int(g.uniform(1)[0] * s) for s in p.shape)
            old = p[idx]
            p[idx] = old + h
            lp, _ = mlp.loss_and_grads(params, X, Y, M)
            p[idx] = old - h
            lm, _ = mlp.loss_and_grads(params, X, Y, M)
            p[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[li][idx]) <= 1e-7 * max(1.0, abs(fd)), (li, idx, fd, grads[li][idx])


def test_masked_entries_do_not_contribute():
    params, X, Y, M = _setup()
    Y2 = Y.copy()
    Y2[M == 0] += 100.0
    l1, g1 = mlp.loss_and_grads(params, X, Y, M)
    l2, g2 = mlp.loss_and_grads(params, X, Y2, M)
    assert l1 == l2 and all(np.array_equal(a, b) for a, b in zip(g1, g2))


def test_adam_first_step_is_lr_times_sign():
    # after one step from zero moments, m_hat = g and v_hat = g^2, so the update is
    # lr * g / (|g| + eps) = lr * sign(g) up to eps
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    st = {}
    mlp.adam_step(p, g, st, lr=0.1)
    np.testing.assert_allclose(p[0], [0.9, -1.9, 2.9], atol=1e-6)


def test_training_fits_a_smooth_target():
    g = SplitMix64(5)
    params = mlp.init_params(g.uniform)
    X = g.uniform(2000 * 5, -1, 1).reshape(2000, 5)
    Y = np.stack([np.sin(X[:, 0] + k * X[:, 1]) * X[:, 2] for k in range(9)], axis=1)
    M = np.ones_like(Y)
    st = {}
    l0, _ = mlp.loss_and_grads(params, X, Y, M)
    for _ in range(300):
        _, gr = mlp.loss_and_grads(params, X, Y, M)
        mlp.adam_step(params, gr, st, lr=3e-3)
    l1, _ = mlp.loss_and_grads(params, X, Y, M)
    assert l1 < 0.05 * l0
