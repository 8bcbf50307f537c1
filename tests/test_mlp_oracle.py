"""Pins of the FP64 cost-model oracle (CPU): finite differences, closed
forms, a hand-computed tiny network, Adam's first step, and the pick rule."""
import numpy as np
import pytest

from oracle import mlp


def rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.NPARAMS)


def test_parameter_count_and_layout():
    assert mlp.NPARAMS == 5121
    p = np.arange(mlp.NPARAMS, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    assert W1.shape == (64, 13) and W1[0, 1] == 1 and W1[1, 0] == 13
    assert b1[0] == 832 and W2[0, 0] == 896 and W2[1, 0] == 960
    assert b2[0] == 4992 and w3[0] == 5056 and b3[0] == 5120


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = rand_params(1)
    X = rng.normal(0, 1, (9, 13))
    t = rng.normal(0, 1, 9)

    def loss(q):
        y, _ = mlp.forward(q, X)
        return mlp.mse(y, t)[0]

    y, cache = mlp.forward(p, X)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(p, cache, dy)
    h = 1e-6
    idx = list(range(0, 832, 37)) + list(range(832, 896, 7)) + list(range(896, 4992, 211)) + \
        list(range(4992, 5121, 5)) + [5120]
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_weights_closed_form():
    p = np.zeros(mlp.NPARAMS)
    p[-1] = 0.75                         # b3
    X = np.random.default_rng(2).normal(0, 1, (5, 13))
    t = np.arange(5.0)
    y, cache = mlp.forward(p, X)
    assert np.all(y == 0.75)
    L, dy = mlp.mse(y, t)
    g = mlp.backward(p, cache, dy)
    assert g[-1] == pytest.approx(2 * np.mean(0.75 - t))
    assert not np.any(g[:-1])            # every path through a ReLU is dead


def test_linear_region_matches_least_squares_gradient():
    """With every pre-activation positive the network is the affine map
    y = c . x + d, c = W1^T W2^T w3; the gradient wrt b3 is then the
    least-squares residual sum and wrt w3 is h2^T dy."""
    rng = np.random.default_rng(3)
    p = np.abs(rand_params(4, 0.1))       # positive weights and inputs
    X = np.abs(rng.normal(0, 1, (7, 13)))
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    c = W1.T @ W2.T @ w3
    d = w3 @ (W2 @ b1 + b2) + b3[0]
    y, cache = mlp.forward(p, X)
    assert np.allclose(y, X @ c + d, rtol=1e-12)
    t = rng.normal(0, 1, 7)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(p, cache, dy)
    assert g[-1] == pytest.approx(2 * np.mean(y - t))
    h2 = cache[4]
    assert np.allclose(g[5056:5120], h2.T @ dy)


def test_tiny_network_by_hand():
    """One active path: x0 -> unit 0 -> unit 0 -> output, everything else 0."""
    p = np.zeros(mlp.NPARAMS)
    p[0] = 2.0          # W1[0][0]
    p[832] = -1.0       # b1[0]
    p[896] = 3.0        # W2[0][0]
    p[4992] = 0.5       # b2[0]
    p[5056] = -2.0      # w3[0]
    p[5120] = 1.0       # b3
    X = np.zeros((2, 13))
    X[0, 0] = 1.5       # z1 = 2, h1 = 2, z2 = 6.5, y = -13 + 1 = -12
    X[1, 0] = 0.25      # z1 = -0.5 -> dead, z2 = 0.5, y = -1 + 1 = 0
    y, cache = mlp.forward(p, X)
    assert np.allclose(y, [-12.0, 0.0])
    g = mlp.backward(p, cache, np.array([1.0, 1.0]))
    # d y0 / d W1[0][0] = w3[0] * W2[0][0] * x0 = -2 * 3 * 1.5 = -9 (row 1 dead)
    assert g[0] == pytest.approx(-9.0)
    # d(y0 + y1)/d w3[0] = h2_0 + h2_1 = 6.5 + 0.5
    assert g[5056] == pytest.approx(7.0)
    assert g[5120] == pytest.approx(2.0)


def test_adam_first_step_is_signed_lr():
    p = np.ones(10)
    g = np.array([3.0, -2.0, 0.5, 0, 1e-3, -1e-3, 7, -7, 1, -1])
    p1, m, v = mlp.adam(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01)
    # bias-corrected m/sqrt(v) = g/|g| on the first step (up to eps)
    expect = np.where(g == 0, 1.0, 1.0 - 0.01 * np.sign(g))
    assert np.allclose(p1, expect, atol=1e-7)


def test_pick_rule_and_ties():
    p = np.zeros(mlp.NPARAMS)
    p[5056] = 1.0                  # y = h2_0 (unit 0 of layer 2)
    p[896] = 1.0                   # z2_0 = h1_0
    p[0] = 1.0                     # z1_0 = x_0 standardised
    feats = np.array([[5.0] + [0] * 12, [2.0] + [0] * 12, [2.0] + [0] * 12, [9.0] + [0] * 12])
    mean = np.zeros(13)
    std = np.zeros(13)             # std 0 counts as 1
    assert mlp.pick(p, feats, mean, std) == 1   # 2.0 twice: lowest index
    std[0] = 2.0
    mean[0] = 3.0                  # (x-3)/2 -> ReLU: 1, 0, 0, 3 -> min 0 at index 1
    assert mlp.pick(p, feats, mean, std) == 1


MLP_MUTANTS = [
    ("backward_W2_not_transposed", "dz1 = (dz2 @ W2) * (z1 > 0)", "dz1 = (dz2 @ W2.T) * (z1 > 0)"),
    ("relu_grad_ignored", "dz2 = np.outer(dy, w3) * (z2 > 0)", "dz2 = np.outer(dy, w3)"),
    ("dropped_b1_grad", "g_b1 = dz1.sum(axis=0)", "g_b1 = 0 * dz1.sum(axis=0)"),
    ("mse_grad_not_scaled", "return float(np.mean(d * d)), 2.0 * d / len(d)",
     "return float(np.mean(d * d)), 2.0 * d"),
    ("adam_no_bias_correction", "mh = m / (1 - beta1 ** step)", "mh = m"),
    ("forward_missing_b2", "z2 = h1 @ W2.T + b2", "z2 = h1 @ W2.T"),
    ("pick_argmax", "return int(np.argmin(y))", "return int(np.argmax(y))"),
]


@pytest.mark.parametrize("name,old,new", MLP_MUTANTS, ids=[m[0] for m in MLP_MUTANTS])
def test_mlp_mutant_fails_a_pin(tmp_path, monkeypatch, name, old, new):
    import importlib.util
    src = open(mlp.__file__).read()
    assert old in src, name
    f = tmp_path / "mlp_mut.py"
    f.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("mlp_mut", f)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(__import__("tests.test_mlp_oracle", fromlist=["mlp"]), "mlp", mod)
    pins = [test_parameter_count_and_layout, test_gradient_matches_central_differences,
            test_zero_weights_closed_form, test_linear_region_matches_least_squares_gradient,
            test_tiny_network_by_hand, test_adam_first_step_is_signed_lr, test_pick_rule_and_ties]
    failed = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed, f"mutant {name} passed every pin"
