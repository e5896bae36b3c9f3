"""Pins of the network oracle (oracle/cnn_oracle.py) against definitions
written out as loops, adjoint identities and FP64 central differences."""

import numpy as np
import pytest

from oracle import cnn_oracle as co


def test_bf16_rounding_cases():
    one = 1.0
    ulp = 2.0 ** -7  # bfloat16 spacing just above 1
    cases = {
        one: one,
        one + ulp: one + ulp,
        one + ulp / 2: one,                     # tie -> even (1.0)
        one + 3 * ulp / 2: one + 2 * ulp,       # tie -> even (1 + 2^-6)
        one + ulp / 2 + 2.0 ** -20: one + ulp,  # above the tie
        -(one + ulp / 2 + 2.0 ** -20): -(one + ulp),
        0.0: 0.0,
        3.0e38: 226.0 / 128.0 * 2.0 ** 127,       # mantissa 225.7 / 128 rounds to 226 / 128
    }
    for x, want in cases.items():
        got = float(co.bf16(np.array([x]))[0])
        assert got == pytest.approx(want, rel=1e-4, abs=0), (x, got, want)
    # every bf16 value is exactly representable: rounding is idempotent
    r = co.bf16(np.random.default_rng(0).standard_normal(1000) * 10)
    assert np.array_equal(co.bf16(r), r)


def _conv3_loops(x, w, b):
    B, H, W, C = x.shape
    O = w.shape[3]
    y = np.zeros((B, H, W, O))
    for bb in range(B):
        for i in range(H):
            for j in range(W):
                for o in range(O):
                    s = b[o]
                    for p in range(3):
                        for q in range(3):
                            for c in range(C):
                                s += x[bb, (i + p - 1) % H, (j + q - 1) % W, c] * w[p, q, c, o]
                    y[bb, i, j, o] = s
    return y


def _down3_loops(x, w, b):
    B, H, W, C = x.shape
    O = w.shape[3]
    y = np.zeros((B, H // 3, W // 3, O))
    for bb in range(B):
        for i in range(H // 3):
            for j in range(W // 3):
                for o in range(O):
                    s = b[o]
                    for p in range(3):
                        for q in range(3):
                            for c in range(C):
                                s += x[bb, 3 * i + p, 3 * j + q, c] * w[p, q, c, o]
                    y[bb, i, j, o] = s
    return y


def test_conv3_matches_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 4, 3))
    w = rng.standard_normal((3, 3, 3, 2))
    b = rng.standard_normal(2)
    np.testing.assert_allclose(co.conv3(x, w, b), _conv3_loops(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv3_identity_and_shift_kernels():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 6, 7, 2))
    w = np.zeros((3, 3, 2, 2))
    w[1, 1] = np.eye(2)
    np.testing.assert_array_equal(co.conv3(x, w, np.zeros(2)), x)
    # tap (p, q) = (2, 0) reads x[i + 1, j - 1]
    w = np.zeros((3, 3, 2, 2))
    w[2, 0] = np.eye(2)
    np.testing.assert_array_equal(co.conv3(x, w, np.zeros(2)), np.roll(x, shift=(-1, 1), axis=(1, 2)))


def test_down3_up3_match_loops():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 6, 9, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(co.down3(x, w, b), _down3_loops(x, w, b), rtol=1e-13, atol=1e-13)
    u = co.up3(x)
    assert u.shape == (2, 18, 27, 3)
    for i in range(18):
        for j in range(27):
            np.testing.assert_array_equal(u[:, i, j], x[:, i // 3, j // 3])


@pytest.mark.parametrize("layer", ["conv3", "down3", "conv1"])
def test_layer_adjoints(layer):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 6, 9, 3))
    if layer == "conv1":
        w = rng.standard_normal((3, 4))
    else:
        w = rng.standard_normal((3, 3, 3, 4))
    f = {"conv3": co.conv3, "down3": co.down3, "conv1": co.conv1}[layer]
    fb = {"conv3": co.conv3_backward, "down3": co.down3_backward, "conv1": co.conv1_backward}[layer]
    y0 = f(x, w, np.zeros(4))
    gy = rng.standard_normal(y0.shape)
    gx, gw, gb = fb(x, w, gy)
    # <f(x), gy> = <x, gx> (linear in x without bias)
    assert np.vdot(y0, gy) == pytest.approx(np.vdot(x, gx), rel=1e-12)
    # linear in w as well: <f(x; w), gy> = <w, gw>
    assert np.vdot(y0, gy) == pytest.approx(np.vdot(w, gw), rel=1e-12)
    # bias gradient is the sum of gy over positions
    np.testing.assert_allclose(gb, gy.sum(axis=(0, 1, 2)), rtol=1e-13)
    # up3 adjoint
    u = rng.standard_normal((2, 18, 27, 3))
    assert np.vdot(co.up3(x), u) == pytest.approx(np.vdot(x, co.up3_backward(u)), rel=1e-12)


def test_layer_specs_product_size():
    n = 0
    for name, kind, ci, co_ in co.layer_specs(32):
        n += (ci * co_ if kind == "conv1" else 9 * ci * co_) + co_
    # the four-level 32/64/128/256 U-Net has about 2.9 M parameters
    assert 2.8e6 < n < 3.0e6


def test_network_gradients_central_differences():
    rng = np.random.default_rng(5)
    c0 = 2
    params = co.init_params(c0, seed=3)
    for name in params:  # nonzero biases exercise the bias gradients
        params[name][1] = rng.standard_normal(params[name][1].shape) * 0.1
    x = rng.standard_normal((2, 27, 27, 2))
    t = rng.standard_normal((2, 27, 27, 2))

    def loss_of(p, xx):
        y, _ = co.forward(p, xx, c0)
        return co.rel_mse(y, t)[0]

    y, acts = co.forward(params, x, c0)
    _, gy = co.rel_mse(y, t)
    grads = co.backward(params, acts, gy, c0)
    eps = 1e-6
    checked = 0
    for name in ["enc0a", "enc0b", "down0", "enc1b", "down2", "bot_b", "up2", "dec2a", "up0", "dec0a",
                 "dec0b", "head"]:
        for which in (0, 1):
            arr = params[name][which]
            for _ in range(2):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + eps
                lp = loss_of(params, x)
                arr[idx] = old - eps
                lm = loss_of(params, x)
                arr[idx] = old
                fd = (lp - lm) / (2 * eps)
                an = grads[name][which][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, which, idx, fd, an)
                checked += 1
    for _ in range(4):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        old = x[idx]
        x[idx] = old + eps
        lp = loss_of(params, x)
        x[idx] = old - eps
        lm = loss_of(params, x)
        x[idx] = old
        assert abs((lp - lm) / (2 * eps) - grads["x"][idx]) <= 1e-6 * max(1.0, abs(lp - lm) / (2 * eps)) + 1e-8
    assert checked == 48


def test_gradient_rounding_points():
    """round_grad acts on each layer's pre-activation gradient after the ReLU
    mask: for the head (no ReLU) its weight and bias gradients are the
    products with the rounded output gradient, and for dec0b the bias
    gradient is the sum of the rounded, masked product of that rounded
    gradient with the head's weights."""
    rng = np.random.default_rng(8)
    c0 = 2
    params = co.init_params(c0, seed=4)
    x = rng.standard_normal((1, 27, 27, 2))
    y, acts = co.forward(params, x, c0)
    gy = rng.standard_normal(y.shape) * (1.0 + 2.0 ** -12)  # not bf16-representable
    g = co.backward(params, acts, gy, c0, round_grad=co.bf16)
    g_exact = co.backward(params, acts, gy, c0)
    gq = co.bf16(gy)
    h = acts["dec0b"]
    wh = params["head"][0]
    # head: products with the rounded gradient, by explicit sums
    np.testing.assert_allclose(g["head"][1], gq.sum(axis=(0, 1, 2)), rtol=1e-13)
    np.testing.assert_allclose(g["head"][0], np.einsum("bijc,bijo->co", h, gq), rtol=1e-12)
    assert np.abs(g["head"][1] - g_exact["head"][1]).max() > 0
    # dec0b: rounding after the mask of its ReLU
    pre = co.bf16(np.where(h > 0, gq @ wh.T, 0.0))
    np.testing.assert_allclose(g["dec0b"][1], pre.sum(axis=(0, 1, 2)), rtol=1e-12)


def test_rel_mse_and_adam():
    rng = np.random.default_rng(6)
    y = rng.standard_normal((3, 4, 4, 2))
    t = rng.standard_normal((3, 4, 4, 2))
    loss, g = co.rel_mse(y, t)
    want = np.mean([np.sum((y[b] - t[b]) ** 2) / np.sum(t[b] ** 2) for b in range(3)])
    assert loss == pytest.approx(want, rel=1e-14)
    eps = 1e-6
    idx = (1, 2, 3, 1)
    y2 = y.copy()
    y2[idx] += eps
    lp = co.rel_mse(y2, t)[0]
    y2[idx] -= 2 * eps
    lm = co.rel_mse(y2, t)[0]
    assert (lp - lm) / (2 * eps) == pytest.approx(g[idx], rel=1e-7)
    # first Adam step moves every weight by about lr against the sign of g
    w = rng.standard_normal(10)
    gr = rng.standard_normal(10)
    w1, m, v = co.adam_step(w, gr, np.zeros(10), np.zeros(10), 1, lr=1e-3)
    np.testing.assert_allclose(w1, w - 1e-3 * gr / (np.abs(gr) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * gr)
    np.testing.assert_allclose(v, 0.001 * gr * gr)
