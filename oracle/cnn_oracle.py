"""Plain FP64 CPU reference for the warm-start network.

TEST INFRASTRUCTURE ONLY: used by the tests to check the HIP network kernels;
nothing in the product path imports it, and it shares no code with the GPU
path.

The paper solves every problem from e = E (Sec. 2.3); a learned initial
guess is a system pattern on top of it.  This module fixes what the network
computes, in the simplest form that can be checked by eye:

* Tensors are NHWC, ``[batch, height, width, channels]``, on periodic grids.
* ``conv3``: 3x3 convolution with circular padding, stride 1,
  ``y[b, i, j, o] = bias[o] + sum_{p, q, c} x[b, (i + p - 1) % H, (j + q - 1) % W, c] w[p, q, c, o]``.
* ``down3``: 3x3 convolution with stride 3 over non-overlapping cells,
  ``y[b, I, J, o] = bias[o] + sum_{p, q, c} x[b, 3I + p, 3J + q, c] w[p, q, c, o]``.
* ``up3``: nearest-neighbour upsampling by 3 in both directions.
* ``conv1``: 1x1 convolution (the head).
* ReLU after every convolution except the head.
* U-Net of four levels with widths ``(c0, 2 c0, 4 c0, 8 c0)`` (c0 = 32 in the
  product): two ``conv3`` per level on the way down, ``down3`` between levels,
  two ``conv3`` at the bottom, and on the way up ``up3`` -> ``conv3`` -> concat
  with the skip of that level (up-path channels first) -> two ``conv3``;
  then the ``conv1`` head to 2 channels.
* Loss: mean over the batch of ``||y - t||^2 / ||t||^2``.
* Adam (Kingma and Ba, 2015) with bias correction.
* ``bf16``: round-to-nearest-even to bfloat16 (8 exponent, 7 fraction bits).

Every backward function is the hand-written adjoint of its forward; the
tests pin them against central differences in FP64.
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Rounding
# ---------------------------------------------------------------------------

def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Layers: forward and adjoint
# ---------------------------------------------------------------------------

def conv3(x, w, b):
    out = np.zeros(x.shape[:3] + (w.shape[3],))
    for p in range(3):
        for q in range(3):
            # shifted[i, j] = x[(i + p - 1) % H, (j + q - 1) % W]
            shifted = np.roll(x, shift=(1 - p, 1 - q), axis=(1, 2))
            out += shifted @ w[p, q]
    return out + b


def conv3_backward(x, w, gy):
    """Gradients of sum(gy * conv3(x, w, b)) with respect to x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for p in range(3):
        for q in range(3):
            shifted = np.roll(x, shift=(1 - p, 1 - q), axis=(1, 2))
            gw[p, q] = np.einsum("bijc,bijo->co", shifted, gy)
            gx += np.roll(gy @ w[p, q].T, shift=(p - 1, q - 1), axis=(1, 2))
    gb = gy.sum(axis=(0, 1, 2))
    return gx, gw, gb


def down3(x, w, b):
    B, H, W, C = x.shape
    cells = x.reshape(B, H // 3, 3, W // 3, 3, C)
    return np.einsum("bipjqc,pqco->bijo", cells, w) + b


def down3_backward(x, w, gy):
    B, H, W, C = x.shape
    cells = x.reshape(B, H // 3, 3, W // 3, 3, C)
    gw = np.einsum("bipjqc,bijo->pqco", cells, gy)
    gx = np.einsum("bijo,pqco->bipjqc", gy, w).reshape(B, H, W, C)
    return gx, gw, gy.sum(axis=(0, 1, 2))


def up3(x):
    return np.repeat(np.repeat(x, 3, axis=1), 3, axis=2)


def up3_backward(gy):
    B, H, W, C = gy.shape
    return gy.reshape(B, H // 3, 3, W // 3, 3, C).sum(axis=(2, 4))


def conv1(x, w, b):
    return x @ w + b


def conv1_backward(x, w, gy):
    return gy @ w.T, np.einsum("bijc,bijo->co", x, gy), gy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


# ---------------------------------------------------------------------------
# The network
# ---------------------------------------------------------------------------

def layer_specs(c0: int = 32, cin: int = 2, cout: int = 2):
    """(name, kind, in_channels, out_channels) in execution order."""
    c = [c0, 2 * c0, 4 * c0, 8 * c0]
    s = [("enc0a", "conv3", cin, c[0]), ("enc0b", "conv3", c[0], c[0]),
         ("down0", "down3", c[0], c[1]),
         ("enc1a", "conv3", c[1], c[1]), ("enc1b", "conv3", c[1], c[1]),
         ("down1", "down3", c[1], c[2]),
         ("enc2a", "conv3", c[2], c[2]), ("enc2b", "conv3", c[2], c[2]),
         ("down2", "down3", c[2], c[3]),
         ("bot_a", "conv3", c[3], c[3]), ("bot_b", "conv3", c[3], c[3])]
    for lev in (2, 1, 0):
        s += [(f"up{lev}", "conv3", c[lev + 1], c[lev]),
              (f"dec{lev}a", "conv3", 2 * c[lev], c[lev]),
              (f"dec{lev}b", "conv3", c[lev], c[lev])]
    s.append(("head", "conv1", c[0], cout))
    return s


def init_params(c0: int = 32, seed: int = 0, cin: int = 2):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, kind, ci, co in layer_specs(c0, cin):
        if kind == "conv1":
            w = rng.standard_normal((ci, co)) * np.sqrt(1.0 / ci)
        else:
            w = rng.standard_normal((3, 3, ci, co)) * np.sqrt(2.0 / (9 * ci))
        params[name] = [w, np.zeros(co)]
    return params


def forward(params, x, c0: int = 32, round_act=None):
    """Network output and the activations the backward pass needs.
    round_act: optional function applied to every stored activation (e.g.
    bf16, to follow a low-precision implementation)."""
    rnd = round_act or (lambda a: a)
    acts = {"x": x}

    def conv(name, kind, inp, act=True):
        w, b = params[name]
        y = {"conv3": conv3, "down3": down3, "conv1": conv1}[kind](inp, w, b)
        y = relu(y) if act else y
        y = rnd(y)
        acts[name] = y
        return y

    h = conv("enc0a", "conv3", x)
    s0 = conv("enc0b", "conv3", h)
    h = conv("down0", "down3", s0)
    h = conv("enc1a", "conv3", h)
    s1 = conv("enc1b", "conv3", h)
    h = conv("down1", "down3", s1)
    h = conv("enc2a", "conv3", h)
    s2 = conv("enc2b", "conv3", h)
    h = conv("down2", "down3", s2)
    h = conv("bot_a", "conv3", h)
    h = conv("bot_b", "conv3", h)
    skips = {0: s0, 1: s1, 2: s2}
    for lev in (2, 1, 0):
        h = conv(f"up{lev}", "conv3", up3(h))
        cat = np.concatenate([h, skips[lev]], axis=-1)
        acts[f"cat{lev}"] = cat
        h = conv(f"dec{lev}a", "conv3", cat)
        h = conv(f"dec{lev}b", "conv3", h)
    y = conv("head", "conv1", h, act=False)
    return y, acts


def _input_of(name, acts):
    order = ["x", "enc0a", "enc0b", "down0", "enc1a", "enc1b", "down1", "enc2a", "enc2b", "down2",
             "bot_a", "bot_b"]
    if name in order[1:]:
        return acts[order[order.index(name) - 1]]
    if name.startswith("up"):
        lev = int(name[2])
        prev = "bot_b" if lev == 2 else f"dec{lev + 1}b"
        return up3(acts[prev])
    if name.startswith("dec"):
        lev = int(name[3])
        return acts[f"cat{lev}"] if name.endswith("a") else acts[f"dec{lev}a"]
    if name == "head":
        return acts["dec0b"]
    raise KeyError(name)


def backward(params, acts, gy, c0: int = 32, round_grad=None):
    """Gradients of sum(gy * forward(params, x)) for every parameter (and x).
    round_grad: optional function applied to the gradient at each layer's
    pre-activation output (after the ReLU mask), the operand of that layer's
    weight- and input-gradient products (e.g. bf16, to follow a
    low-precision implementation)."""
    grads = {}
    specs = {n: k for n, k, _, _ in layer_specs(c0, acts["x"].shape[-1])}
    rnd = round_grad or (lambda a: a)

    def back(name, g_out, act=True):
        w, _ = params[name]
        if act:
            g_out = g_out * (acts[name] > 0)
        g_out = rnd(g_out)
        inp = _input_of(name, acts)
        fn = {"conv3": conv3_backward, "down3": down3_backward, "conv1": conv1_backward}[specs[name]]
        gx, gw, gb = fn(inp, w, g_out)
        grads[name] = [gw, gb]
        return gx

    g = back("head", gy, act=False)
    g_skip = {}
    for lev in (0, 1, 2):
        g = back(f"dec{lev}b", g)
        g = back(f"dec{lev}a", g)
        c_up = params[f"up{lev}"][0].shape[-1]
        g_up, g_skip[lev] = g[..., :c_up], g[..., c_up:]
        g = up3_backward(back(f"up{lev}", g_up))
    g = back("bot_b", g)
    g = back("bot_a", g)
    g = back("down2", g)
    g = back("enc2b", g + g_skip[2])
    g = back("enc2a", g)
    g = back("down1", g)
    g = back("enc1b", g + g_skip[1])
    g = back("enc1a", g)
    g = back("down0", g)
    g = back("enc0b", g + g_skip[0])
    g = back("enc0a", g)
    grads["x"] = g
    return grads


# ---------------------------------------------------------------------------
# Loss and optimiser
# ---------------------------------------------------------------------------

def rel_mse(y, t):
    """Mean over the batch of ||y_b - t_b||^2 / ||t_b||^2, and its gradient."""
    B = y.shape[0]
    d = (y - t).reshape(B, -1)
    tn = np.maximum((t.reshape(B, -1) ** 2).sum(axis=1), 1e-30)
    loss = float(((d ** 2).sum(axis=1) / tn).mean())
    grad = (2.0 * d / tn[:, None] / B).reshape(y.shape)
    return loss, grad


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def network_input(phase, log10_rho):
    """[1, N, N, 2] input: phase indicator and log10(contrast) / 4."""
    ph = np.asarray(phase, dtype=np.float64)
    return np.stack([ph, np.full_like(ph, log10_rho / 4.0)], axis=-1)[None]
