"""Pins of the refinement-network oracle against facts it does not compute
itself: finite differences of the loss, closed forms of Adam, BF16 rounding
cases fixed by the format, and invariances of the features."""
import numpy as np
import pytest

from oracle import refine_net as R
from paper_1610_00823_amd import inputs as I


def _batch(seed, B=24):
    rng = np.random.default_rng(seed)
    x = R.features(rng.standard_normal((B, 16, 16)) * np.exp(rng.uniform(-30, 2, B))[:, None, None],
                   rng.integers(0, 15, B))
    y = (rng.random(B) < 0.4).astype(np.float64)
    return x, y


def test_bf16_rounding_cases():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1);
    # 1 + 3 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6.
    assert R.bf16(1.0 + 2.0 ** -8) == 1.0
    assert R.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert R.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert R.bf16(-3.0) == -3.0 and R.bf16(0.0) == 0.0
    assert R.bf16(np.pi) == 3.140625                       # 8 significant bits of pi
    x = np.random.default_rng(0).standard_normal(1000)
    r = R.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)  # half an ulp of an 8-bit significand
    assert np.array_equal(R.bf16(r), r)


def test_features_invariances():
    rng = np.random.default_rng(3)
    s = rng.standard_normal((5, 16, 16))
    lv = np.array([0, 3, 7, 12, 16])
    x = R.features(s, lv)
    # a positive power-of-two scale of the samples leaves the shape features
    # unchanged and moves the amplitude feature by log10(scale) / 10
    x2 = R.features(s * 2.0 ** -20, lv)
    assert np.array_equal(x[:, :256], x2[:, :256])
    A = np.abs(s.reshape(5, -1)).max(1)
    assert np.allclose(x2[:, 257], R.bf16((np.log10(A * 2.0 ** -20) + 10) / 10), rtol=0, atol=0)
    assert np.all(np.abs(x[:, :256]).max(1) == 1.0)
    assert np.array_equal(x[:, 256], lv / 16.0) and np.all(x[:, 259:] == 0)
    z = R.features(np.zeros((1, 16, 16)), [4])
    assert np.all(z[0, :256] == 0) and z[0, 257] == -1.0 and z[0, 258] == -1.0
    big = R.features(np.full((1, 16, 16), 1e30), [0])
    assert big[0, 257] == 2.0 and big[0, 258] == R.bf16(30 / 320)
    # a faint trace (all samples near 1e-200) saturates the first amplitude
    # feature but not the second
    faint = R.features(np.full((1, 16, 16), 1e-200), [0])
    assert faint[0, 257] == -1.0 and faint[0, 258] == R.bf16(-200 / 320)


@pytest.mark.parametrize("emulate", [False, True])
def test_gradient_matches_finite_differences(emulate):
    # Central differences of the loss in random directions and in single
    # coordinates of every parameter block.  In FP64 the match is to O(h^2);
    # with BF16 rounding the loss is piecewise constant in W1 and W2 at
    # the ulp scale, so there only the unrounded parameters are probed.
    x, y = _batch(1)
    theta = I.refine_net_init(5)
    theta[R.N_HID * R.N_IN:R.N_HID * R.N_IN + R.N_HID] = 0.05        # b1 != 0: some units active, some not
    L0, g = R.loss_and_grad(theta, x, y, emulate)
    rng = np.random.default_rng(2)
    offs, o = {}, 0
    for name, shp in R.SHAPES:
        offs[name] = (o, o + int(np.prod(shp)))
        o += int(np.prod(shp))
    probe = ["b2", "w3", "b3"] if emulate else [name for name, _ in R.SHAPES]
    h = 1e-6
    for name in probe:
        a, b = offs[name]
        for k in rng.choice(np.arange(a, b), min(6, b - a), replace=False):
            e = np.zeros_like(theta)
            e[k] = h
            fd = (R.loss_and_grad(theta + e, x, y, emulate)[0] - R.loss_and_grad(theta - e, x, y, emulate)[0]) / (2 * h)
            assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (name, k, fd, g[k])
    if not emulate:
        d = rng.standard_normal(theta.size)
        d /= np.linalg.norm(d)
        fd = (R.loss_and_grad(theta + h * d, x, y, False)[0] - R.loss_and_grad(theta - h * d, x, y, False)[0]) / (2 * h)
        assert abs(fd - g @ d) <= 1e-7


def test_loss_closed_forms():
    # zero weights: logit = b3 for every box, loss = softplus(b3) - b3 mean(y)
    x, y = _batch(4)
    theta = np.zeros(R.N_PARAMS)
    theta[-1] = 0.7
    L, g = R.loss_and_grad(theta, x, y, emulate=False)
    assert np.isclose(L, np.log1p(np.exp(0.7)) - 0.7 * y.mean(), rtol=1e-15)
    assert np.isclose(g[-1], 1 / (1 + np.exp(-0.7)) - y.mean(), rtol=1e-14)
    assert np.all(g[:-1] == 0)
    assert np.allclose(R.bce(np.array([-800.0, 800.0]), np.array([0.0, 1.0])), 0.0)


def test_adam_closed_forms():
    rng = np.random.default_rng(6)
    w0, g = rng.standard_normal(50), rng.standard_normal(50)
    m = v = np.zeros(50)
    w = w0
    # a constant gradient: the bias-corrected moments equal g and g^2 at every
    # step, so each step moves w by lr g / (|g| + eps)
    for t in range(1, 6):
        w, m, v = R.adam_step(w, g, m, v, t, 1e-2, eps=1e-8)
        assert np.allclose(w, w0 - t * 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)
    # zero gradient after one step: m decays by beta1 and v by beta2
    w1, m1, v1 = R.adam_step(w0, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    _, m2, v2 = R.adam_step(w1, np.zeros(50), m1, v1, 2, 1e-3)
    assert np.allclose(m2, 0.9 * 0.1 * g) and np.allclose(v2, 0.999 * 0.001 * g * g)


def test_emulated_forward_is_close_to_fp64():
    # BF16 rounding of W1, W2 and h1 moves the logits by a few 2^-8 relative
    x, _ = _batch(7, 64)
    theta = I.refine_net_init(8)
    a, b = R.forward(theta, x, emulate=True), R.forward(theta, x, emulate=False)
    assert np.abs(a - b).max() <= 0.05 * np.abs(b).max()
    assert not np.array_equal(a, b)
