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


# ---------------------------------------------------------------- bf16 branch
# The rounded network (the one the GPU kernels compute) is pinned two ways
# that do not reuse the oracle's code: its forward pass against exact
# rational arithmetic with a round-to-nearest-even written from the
# definition, and its straight-through gradient against central differences
# of the unrounded network at the rounded parameters, at a point where every
# activation is a bfloat16 value (so rounding them is the identity).

from fractions import Fraction  # noqa: E402


def rne8(q):
    """Nearest rational with 8 significant bits (bfloat16's precision), ties
    to even; exact, for magnitudes far from bfloat16's exponent limits."""
    q = Fraction(q)
    if q == 0:
        return q
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    ulp = Fraction(2) ** (e - 7)          # 2^e <= a < 2^(e+1): 8 bits from 2^e down to 2^(e-7)
    k = a / ulp
    fl = k.numerator // k.denominator
    rem = k - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return (fl * ulp) if q > 0 else -(fl * ulp)


def test_rne8_reference_points():
    assert rne8(1 + Fraction(1, 256)) == 1                      # halfway, even mantissa stays
    assert rne8(1 + Fraction(3, 256)) == 1 + Fraction(1, 64)     # halfway, odd mantissa rounds up
    assert rne8(Fraction(255, 128) + Fraction(1, 256)) == 2       # carry into the next binade
    assert rne8(-Fraction(3, 1024) - Fraction(1, 10 ** 9)) == -Fraction(3, 1024)
    for x in np.random.default_rng(9).uniform(-4, 4, 200).astype(np.float32):
        assert float(rne8(Fraction(float(x)))) == mlp.bf16(x)


def _exact_forward(p, x):
    """The rounded network in exact rationals: every weight, input and hidden
    activation rounded by rne8, products and sums exact."""
    q = mlp.unpack(p)
    R = {k: [[rne8(Fraction(float(v))) for v in np.atleast_2d(q[k])[i]] for i in range(np.atleast_2d(q[k]).shape[0])]
         for k in ("W1", "W2", "W3")}
    B = {k: [rne8(Fraction(float(v))) for v in q[k]] for k in ("b1", "b2", "b3")}
    out = []
    for row in x:
        xr = [rne8(Fraction(float(v))) for v in row]
        h1 = [rne8(max(sum(w * a for w, a in zip(R["W1"][j], xr)) + B["b1"][j], 0)) for j in range(mlp.NH)]
        h2 = [rne8(max(sum(w * a for w, a in zip(R["W2"][j], h1)) + B["b2"][j], 0)) for j in range(mlp.NH)]
        z = [sum(w * a for w, a in zip(R["W3"][o], h2)) + B["b3"][o] for o in range(mlp.NO)]
        out.append((z, h1, h2))
    return out


def _signed_uniform(rng, n, lo=0.125, hi=1.0):
    return (rng.uniform(lo, hi, n) * rng.choice([-1.0, 1.0], n)).astype(np.float32)


def test_rounded_forward_matches_exact_rationals():
    """Parameters and inputs of 24-bit precision (not bfloat16 values), so
    every rounding point of the forward pass is exercised; magnitudes in
    [1/8, 1] keep the float64 sums exact, so the oracle must agree with the
    rational computation exactly on h1, h2 and to rounding on the logits."""
    rng = np.random.default_rng(21)
    p = _signed_uniform(rng, mlp.NPAR)
    x = _signed_uniform(rng, 3 * mlp.NI).reshape(3, mlp.NI)
    z, h1, h2 = mlp.forward(p, x, rounding=True)
    for b, (ze, h1e, h2e) in enumerate(_exact_forward(p, x)):
        assert h1[b].tolist() == [float(v) for v in h1e]
        assert h2[b].tolist() == [float(v) for v in h2e]
        assert np.allclose(z[b], [float(v) for v in ze], rtol=0, atol=1e-12)
    # the rounding points matter here: without them the activations differ
    _, u1, _ = mlp.forward(p, x, rounding=False)
    assert not np.array_equal(u1, h1)


def _dyadic_point(seed):
    """Parameters p_r and inputs x_r made of bfloat16 values such that every
    pre-activation of the unrounded network at (p_r, x_r) is a bfloat16
    value at least 1/16 away from the ReLU kink, and W1, W2 rows are sparse
    enough for that; then (p, x) = (p_r, x_r) plus perturbations below half a
    bfloat16 unit, so bf16(p) = p_r and bf16(x) = x_r exactly."""
    rng = np.random.default_rng(seed)
    for _ in range(2000):
        q = {k: np.zeros(s) for k, s in mlp.SHAPES}
        xr = rng.choice([-1.0, -0.5, 0.5, 1.0], (2, mlp.NI))
        for j in range(mlp.NH):
            cols = rng.choice(mlp.NI, 2, replace=False)
            q["W1"][j, cols] = rng.choice([-1.0, -0.5, 0.5, 1.0], 2)
            cols = rng.choice(mlp.NH, 2, replace=False)
            q["W2"][j, cols] = rng.choice([-1.0, -0.5, 0.5, 1.0], 2)
        q["b1"] = rng.choice([-0.375, -0.125, 0.125, 0.375, 0.625], mlp.NH)
        q["b2"] = rng.choice([-0.1875, 0.0625, 0.3125, 0.5625], mlp.NH)
        q["W3"] = rng.choice([-1.5, -0.75, -0.25, 0.25, 0.75, 1.25], (mlp.NO, mlp.NH))
        q["b3"] = rng.choice([-0.5, 0.5], mlp.NO)
        pr = mlp.pack(q)
        a1 = xr @ q["W1"].T + q["b1"]
        h1 = np.maximum(a1, 0)
        a2 = h1 @ q["W2"].T + q["b2"]
        ok = all(np.all(np.abs(a) >= 1 / 16) and np.array_equal(mlp.bf16(a), a) for a in (a1, a2))
        if ok and (a1 > 0).mean() > 0.3 and (a2 > 0).mean() > 0.3:
            break
    else:
        raise AssertionError("no dyadic point found")
    # perturb every nonzero value by a fraction of half its bfloat16 unit
    def perturb(v):
        v = np.asarray(v, np.float64)
        # the spacing below a power of two is half the one above: use the smaller
        ulp = 2.0 ** (np.floor(np.log2(np.where(v == 0, 1.0, np.abs(v)))) - 8)
        return (v + np.where(v == 0, 0.0, rng.uniform(-0.45, 0.45, v.shape) * ulp)).astype(np.float32)
    p, x = perturb(pr), perturb(xr)
    assert np.array_equal(mlp.bf16(p), pr) and np.array_equal(mlp.bf16(x), xr)
    assert np.all((p != pr)[pr != 0]) and np.all((x != xr)[xr != 0])
    return p, x, pr, xr


def _fd_gradient(pr, xr, c, h=1e-6):
    """Central differences of sum(c * logits) of the unrounded network at (pr, xr)."""
    def f(pp):
        return np.sum(c * mlp.forward(pp, xr, rounding=False)[0])
    g = np.empty(mlp.NPAR)
    for i in range(mlp.NPAR):
        pp, pm = pr.copy(), pr.copy()
        pp[i] += h
        pm[i] -= h
        g[i] = (f(pp) - f(pm)) / (2 * h)
    return g


def _straight_through_pin(backward, seed):
    p, x, pr, xr = _dyadic_point(seed)
    pr = pr.astype(np.float64)
    c = np.random.default_rng(seed + 1).normal(size=(2, mlp.NO))
    z, h1, h2 = mlp.forward(p, x, rounding=True)
    zr = mlp.forward(pr, xr, rounding=False)[0]
    assert np.array_equal(z, zr)                # every rounding point is exact at this point
    g = backward(p, x, h1, h2, c, rounding=True)
    fd = _fd_gradient(pr, xr, c)
    return np.max(np.abs(g - fd))


@pytest.mark.parametrize("seed", [31, 32])
def test_rounded_backward_is_gradient_at_rounded_point(seed):
    """With every activation a bfloat16 value at the rounded parameters, the
    straight-through gradient of the rounded network at p is the true
    gradient of the unrounded network at bf16(p); the perturbations (below
    half a unit) make any use of an unrounded weight or input visible."""
    assert _straight_through_pin(mlp.backward, seed) < 1e-8


def _mutant(old, new):
    """A copy of the oracle's backward with one planted mistake."""
    import inspect
    src = inspect.getsource(mlp.backward)
    assert old in src, old
    ns = dict(vars(mlp))
    exec(src.replace(old, new), ns)
    return ns["backward"]


@pytest.mark.parametrize("old,new", [
    ('W2, W3 = rnd(q["W2"]), rnd(q["W3"])', 'W2, W3 = rnd(q["W2"]), q["W3"]'),      # unrounded W3
    ('W2, W3 = rnd(q["W2"]), rnd(q["W3"])', 'W2, W3 = q["W2"], rnd(q["W3"])'),      # unrounded W2
    ("x = rnd(np.asarray(x, np.float64))", "x = np.asarray(x, np.float64)"),        # unrounded input
    ("dz1 = (dz2 @ W2) * (h1 > 0)", "dz1 = (dz2 @ W2.T) * (h1 > 0)"),               # transposed operand
    ('g["W2"] = dz2.T @ h1', 'g["W2"] = dz2.T @ h2'),                                # wrong activation
])
def test_planted_slips_fail_the_pin(old, new):
    assert _straight_through_pin(_mutant(old, new), 31) > 1e-6
