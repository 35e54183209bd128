"""Oracle side: FP64 reference of the convolutional warm-start surrogate.

Test infrastructure only (see ``oracle/__init__.py``).  Plain NumPy, float64,
written for clarity: every layer is a loop over the 3 x 3 taps with einsum.
The GPU library's BF16/FP32 kernels are checked against it layer by layer
and end to end; it is itself pinned by finite differences and by the
adjoint identities of its layers.

Network (a U-Net; the same layer list the library builds):
  input   B x H x W x cin (NHWC), H and W divisible by 16
  block   conv3x3(pad 1) + bias + ReLU, twice
  down    2 x 2 average pool
  up      nearest-neighbour x2, then concat [up, skip] along channels
  encoder channels c, 2c, 4c, 8c; bottleneck 8c; decoder back to c
  head    1 x 1 conv to cout, no activation
Parameters are one flat vector: for each layer in order, W[cout, kh, kw, cin]
then b[cout].  The loss is the mean squared error over all outputs.
"""
from __future__ import annotations

import numpy as np


def layer_list(base: int, cin: int, cout: int):
    c0, c1, c2, c3 = base, 2 * base, 4 * base, 8 * base
    return [
        ("e1a", cin, c0, 3), ("e1b", c0, c0, 3),
        ("e2a", c0, c1, 3), ("e2b", c1, c1, 3),
        ("e3a", c1, c2, 3), ("e3b", c2, c2, 3),
        ("e4a", c2, c3, 3), ("e4b", c3, c3, 3),
        ("ba", c3, c3, 3), ("bb", c3, c3, 3),
        ("d4a", c3 + c3, c3, 3), ("d4b", c3, c3, 3),
        ("d3a", c3 + c2, c2, 3), ("d3b", c2, c2, 3),
        ("d2a", c2 + c1, c1, 3), ("d2b", c1, c1, 3),
        ("d1a", c1 + c0, c0, 3), ("d1b", c0, c0, 3),
        ("head", c0, cout, 1),
    ]


def param_count(base: int, cin: int, cout: int) -> int:
    return sum(co * k * k * ci + co for _, ci, co, k in layer_list(base, cin, cout))


def unpack(theta, base, cin, cout):
    out, off = {}, 0
    for name, ci, co, k in layer_list(base, cin, cout):
        nW = co * k * k * ci
        out[name] = (theta[off:off + nW].reshape(co, k, k, ci), theta[off + nW:off + nW + co])
        off += nW + co
    assert off == theta.size
    return out


# ---------------------------------------------------------------- layers

def conv(x, W, b):
    """x (B,H,W,ci), W (co,k,k,ci), same-size output, zero padding."""
    k = W.shape[1]
    r = k // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    H, Wd = x.shape[1], x.shape[2]
    y = np.zeros(x.shape[:3] + (W.shape[0],))
    for dy in range(k):
        for dx in range(k):
            y += np.einsum("bhwc,oc->bhwo", xp[:, dy:dy + H, dx:dx + Wd, :], W[:, dy, dx, :])
    return y + b


def conv_backward(x, W, dy):
    """Gradients of conv(x, W, b) w.r.t. x, W and b given dL/dy."""
    k = W.shape[1]
    r = k // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    H, Wd = x.shape[1], x.shape[2]
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(k):
        for kx in range(k):
            dW[:, ky, kx, :] = np.einsum("bhwo,bhwc->oc", dy, xp[:, ky:ky + H, kx:kx + Wd, :])
            dxp[:, ky:ky + H, kx:kx + Wd, :] += np.einsum("bhwo,oc->bhwc", dy, W[:, ky, kx, :])
    dx = dxp[:, r:r + H, r:r + Wd, :]
    db = dy.sum(axis=(0, 1, 2))
    return dx, dW, db


def pool(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


def bf16_round(a):
    """Round to the nearest bfloat16 (IEEE binary32 with the significand cut
    to 8 bits, ties to even), returned as float64.  The value is first
    rounded to float32, the precision in which the kernels form what they
    store, then the low 16 bits of the float32 pattern are dropped with
    round-to-nearest-even (finite values only)."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


# ---------------------------------------------------------------- network

class ReferenceUNet:
    """store: None (every activation kept in float64) or a rounding applied
    to each activation a network keeps in memory (the output of every
    conv + bias + ReLU and of every pooling), so that a check of a network
    that stores them at lower precision takes its ReLU decisions on the same
    stored values; the backward pass is the same code either way."""

    def __init__(self, base: int, cin: int, cout: int, store=None):
        self.base, self.cin, self.cout = base, cin, cout
        self.store = store if store is not None else (lambda a: a)

    def forward(self, theta, x):
        P = unpack(theta, self.base, self.cin, self.cout)
        cache = {"x": x}
        st = self.store

        def block(h, a, b_):
            h1 = st(relu(conv(h, *P[a])))
            h2 = st(relu(conv(h1, *P[b_])))
            cache[a] = (h, h1)
            cache[b_] = (h1, h2)
            return h2

        e1 = block(x, "e1a", "e1b")
        e2 = block(st(pool(e1)), "e2a", "e2b")
        e3 = block(st(pool(e2)), "e3a", "e3b")
        e4 = block(st(pool(e3)), "e4a", "e4b")
        bt = block(st(pool(e4)), "ba", "bb")
        d4 = block(np.concatenate([up(bt), e4], axis=3), "d4a", "d4b")
        d3 = block(np.concatenate([up(d4), e3], axis=3), "d3a", "d3b")
        d2 = block(np.concatenate([up(d3), e2], axis=3), "d2a", "d2b")
        d1 = block(np.concatenate([up(d2), e1], axis=3), "d1a", "d1b")
        y = conv(d1, *P["head"])
        cache["head"] = (d1, y)
        cache["skips"] = (e1, e2, e3, e4)
        return y, cache

    def backward(self, theta, cache, dy):
        """Gradient of the loss w.r.t. theta (flat) and the input x."""
        P = unpack(theta, self.base, self.cin, self.cout)
        grads = {}

        def conv_b(name, dout):
            inp, out = cache[name]
            W = P[name][0]
            if name != "head":
                dout = dout * (out > 0)
            dx, dW, db = conv_backward(inp, W, dout)
            grads[name] = (dW, db)
            return dx

        def block_b(a, b_, dout):
            return conv_b(a, conv_b(b_, dout))

        e1, e2, e3, e4 = cache["skips"]
        g = conv_b("head", dy)
        g = block_b("d1a", "d1b", g)
        du, de1 = g[..., :2 * self.base], g[..., 2 * self.base:]
        g = block_b("d2a", "d2b", up_backward(du))
        du, de2 = g[..., :4 * self.base], g[..., 4 * self.base:]
        g = block_b("d3a", "d3b", up_backward(du))
        du, de3 = g[..., :8 * self.base], g[..., 8 * self.base:]
        g = block_b("d4a", "d4b", up_backward(du))
        du, de4 = g[..., :8 * self.base], g[..., 8 * self.base:]
        g = block_b("ba", "bb", up_backward(du))
        g = block_b("e4a", "e4b", pool_backward(g) + de4)
        g = block_b("e3a", "e3b", pool_backward(g) + de3)
        g = block_b("e2a", "e2b", pool_backward(g) + de2)
        dx = block_b("e1a", "e1b", pool_backward(g) + de1)
        flat = []
        for name, ci, co, k in layer_list(self.base, self.cin, self.cout):
            dW, db = grads[name]
            flat.append(dW.reshape(-1))
            flat.append(db)
        return np.concatenate(flat), dx

    @staticmethod
    def mse(y, t):
        d = y - t
        return float((d * d).mean()), 2.0 * d / d.size


def he_init(base, cin, cout, seed):
    """Seeded He-normal weights, zero biases (the same recipe the tests use
    for both sides; weights are inputs, not expected values)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, k in layer_list(base, cin, cout):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (k * k * ci)), size=co * k * k * ci))
        parts.append(np.zeros(co))
    return np.concatenate(parts)
