"""Pins of the network oracle (oracle/mlp.py) against closed forms, special
cases and central finite differences (float64)."""
import numpy as np
import pytest

from oracle import mlp


def rand_params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, mlp.NPAR).astype(np.float32)


def test_bf16_rounding_points():
    one = np.float32(1.0)
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,                    # halfway, ties to even (mantissa 0)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,    # halfway, ties to even (mantissa 2)
        1.0 + 2.0 ** -8 + 2.0 ** -20: 1.0 + 2.0 ** -7,
        -2.5: -2.5,
        0.0: 0.0,
        65536.0 + 256.0: 65536.0,                # spacing 512 at 2^16: tie goes to even
        65536.0 + 257.0: 65536.0 + 512.0,
    }
    for x, want in cases.items():
        assert mlp.bf16(np.float32(x)) == np.float32(want), x
    assert np.isinf(mlp.bf16(np.float32(np.inf)))
    big = np.array([0x7F7FFFFF], np.uint32).view(np.float32)   # largest float32 rounds past bf16's range
    assert np.isinf(mlp.bf16(big))[0]
    assert np.isnan(mlp.bf16(np.float32(np.nan)))
    assert mlp.bf16(one) == 1.0


def test_layout_size():
    assert mlp.NPAR == 64 * 12 + 64 + 64 * 64 + 64 + 5 * 64 + 5 == 5317
    p = rand_params(1)
    assert np.allclose(mlp.pack(mlp.unpack(p)), p)


def test_forward_special_cases():
    x = np.random.default_rng(2).uniform(-1, 1, (7, 12))
    # all weights zero: the logits are the (rounded) output bias
    q = {k: np.zeros(s) for k, s in mlp.SHAPES}
    q["b3"] = np.array([0.5, -1.0, 2.0, 0.25, -0.125])
    z, h1, h2 = mlp.forward(mlp.pack(q), x)
    assert np.all(z == q["b3"]) and np.all(h1 == 0) and np.all(h2 == 0)
    # a single path: h1[0] = relu(x0), h2[0] = 2 h1[0], logit0 = 3 h2[0] - 1
    q = {k: np.zeros(s) for k, s in mlp.SHAPES}
    q["W1"][0, 0] = 1.0
    q["W2"][0, 0] = 2.0
    q["W3"][0, 0] = 3.0
    q["b3"][0] = -1.0
    xs = np.array([[0.75] + [0] * 11, [-0.5] + [0] * 11])
    z, _, _ = mlp.forward(mlp.pack(q), xs)
    assert z[0, 0] == 3 * 2 * 0.75 - 1 and z[1, 0] == -1.0


def test_loss_closed_forms():
    B = 6
    z = np.zeros((B, 5))
    labels = np.array([0, 1, 2, 0 | (1 << 8), 2 | (2 << 8), 1 | (0 << 8)])
    L, d = mlp.loss(z, labels)
    assert np.isclose(L, 2 * np.log(2) + np.log(3))
    y0, y1, dc = mlp.targets(labels)
    assert np.allclose(d[:, 0], (0.5 - y0) / B) and np.allclose(d[:, 1], (0.5 - y1) / B)
    onehot = np.eye(3)[dc]
    assert np.allclose(d[:, 2:], (1 / 3 - onehot) / B)
    # very confident correct predictions cost almost nothing
    z = np.zeros((1, 5))
    z[0, :] = [-40, 40, -40, -40, 40]
    L, _ = mlp.loss(z, np.array([1 | (2 << 8)]))
    assert L < 1e-15


def test_loss_gradient_by_finite_differences():
    rng = np.random.default_rng(3)
    z = rng.normal(size=(5, 5))
    labels = np.array([0, 1, 2, 1 | (1 << 8), 2 | (2 << 8)])
    _, d = mlp.loss(z, labels)
    h = 1e-6
    for i in range(5):
        for k in range(5):
            zp, zm = z.copy(), z.copy()
            zp[i, k] += h
            zm[i, k] -= h
            fd = (mlp.loss(zp, labels)[0] - mlp.loss(zm, labels)[0]) / (2 * h)
            assert abs(fd - d[i, k]) < 1e-8


@pytest.mark.parametrize("seed", [4, 5])
def test_backward_by_finite_differences(seed):
    """Without the bf16 rounding the network is piecewise linear in each
    parameter; central differences of sum(c * logits) pin every gradient."""
    rng = np.random.default_rng(seed)
    p = rand_params(seed).astype(np.float64)
    x = rng.uniform(-1, 1, (3, 12))
    c = rng.normal(size=(3, 5))
    z, h1, h2 = mlp.forward(p, x, rounding=False)
    g = mlp.backward(p, x, h1, h2, c, rounding=False)

    def f(pp):
        return np.sum(c * mlp.forward(pp, x, rounding=False)[0])

    h = 1e-6
    idx = rng.choice(mlp.NPAR, 400, replace=False)
    idx = np.concatenate([idx, np.arange(mlp.NPAR - 5, mlp.NPAR), [0, 64 * 12, 64 * 12 + 64]])
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)), i


def test_adam_first_step_is_signed_lr():
    g = np.array([2.0, -3.0, 0.5, 0.0])
    p = np.zeros(4)
    p1, m1, m2 = mlp.adam(g, p, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p1[:3], -0.01 * np.sign(g[:3]), rtol=1e-6) and p1[3] == 0
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)
