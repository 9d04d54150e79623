"""Pins for the float64 selector-MLP reference: central finite differences
for the backward pass, hand-computed forward values, mask semantics, and the
closed form of Adam under a constant gradient."""
import numpy as np

import oracle


def rand_params(rng, scale=0.3):
    flat = rng.standard_normal(oracle.MLP_N_PARAMS) * scale
    return oracle.mlp_unflatten(flat)


def test_param_count_matches_architecture():
    # 8->32->32->4: 8*32+32 + 32*32+32 + 32*4+4
    assert oracle.MLP_N_PARAMS == 1476


def test_forward_hand_computed():
    p = oracle.mlp_unflatten(np.zeros(oracle.MLP_N_PARAMS))
    p["W1"][0, 0] = 2.0
    p["W1"][1, 0] = -1.0          # negative pre-activation -> ReLU blocks it
    p["W2"][0, 0] = 3.0
    p["W2"][1, 1] = 5.0
    p["W3"][:, 0] = [0.0, 1.0, 2.0, 3.0]
    p["W3"][:, 1] = [7.0, 7.0, 7.0, 7.0]
    p["b3"][:] = [0.5, -0.5, 0.0, 1.0]
    X = np.zeros((1, 8))
    X[0, 0] = 1.0
    Y, _ = oracle.mlp_forward(p, X)
    # h1 = [2, 0, ...]; h2 = [6, 0, ...]; Y = 6*[0,1,2,3] + b3
    np.testing.assert_allclose(Y[0], [0.5, 5.5, 12.0, 19.0])


def test_zero_hidden_gives_bias():
    rng = np.random.default_rng(0)
    p = rand_params(rng)
    p["W3"][:] = 0.0
    X = rng.standard_normal((5, 8))
    Y, _ = oracle.mlp_forward(p, X)
    np.testing.assert_allclose(Y, np.tile(p["b3"], (5, 1)))


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    p = rand_params(rng)
    X = rng.standard_normal((16, 8))
    T = rng.standard_normal((16, 4))
    M = (rng.random((16, 4)) < 0.8).astype(np.float64)
    _, g = oracle.mlp_backward(p, X, T, M)
    flat = oracle.mlp_flatten(p)
    gflat = oracle.mlp_flatten(g)
    eps = 1e-6
    idx = rng.choice(flat.shape[0], 200, replace=False)
    for i in idx:
        a, b = flat.copy(), flat.copy()
        a[i] += eps
        b[i] -= eps
        num = (oracle.mlp_loss(oracle.mlp_unflatten(a), X, T, M)
               - oracle.mlp_loss(oracle.mlp_unflatten(b), X, T, M)) / (2 * eps)
        assert abs(num - gflat[i]) <= 1e-6 * max(1.0, abs(num)), (i, num, gflat[i])


def test_mask_excludes_entries():
    rng = np.random.default_rng(2)
    p = rand_params(rng)
    X = rng.standard_normal((4, 8))
    T = rng.standard_normal((4, 4))
    M = np.ones((4, 4))
    M[:, 3] = 0.0
    T2 = T.copy()
    T2[:, 3] += 100.0                     # masked targets must not matter
    l1, g1 = oracle.mlp_backward(p, X, T, M)
    l2, g2 = oracle.mlp_backward(p, X, T2, M)
    assert l1 == l2
    for k in g1:
        np.testing.assert_array_equal(g1[k], g2[k])
    np.testing.assert_array_equal(g1["b3"][3], 0.0)
    # mean over the 12 unmasked entries
    Y, _ = oracle.mlp_forward(p, X)
    assert np.isclose(l1, ((Y[:, :3] - T[:, :3]) ** 2).sum() / 12.0)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g, the bias-corrected moments are exactly g and
    # g^2 at every step, so each step moves by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    x = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        x_new, m, v = oracle.adam_step(x, g, m, v, t, lr=lr, eps=eps)
        np.testing.assert_allclose(x_new - x, -lr * g / (np.abs(g) + eps), rtol=1e-10, atol=1e-15)
        x = x_new


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    p = rand_params(rng)
    X = rng.standard_normal((64, 8))
    true = rand_params(np.random.default_rng(4), 0.5)
    T, _ = oracle.mlp_forward(true, X)
    M = np.ones_like(T)
    flat = oracle.mlp_flatten(p)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    l0 = oracle.mlp_loss(p, X, T, M)
    for t in range(1, 301):
        _, g = oracle.mlp_backward(oracle.mlp_unflatten(flat), X, T, M)
        flat, m, v = oracle.adam_step(flat, oracle.mlp_flatten(g), m, v, t, lr=1e-2)
    assert oracle.mlp_loss(oracle.mlp_unflatten(flat), X, T, M) < 0.2 * l0
