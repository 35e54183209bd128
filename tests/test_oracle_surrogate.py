"""Pins of the FP64 reference surrogate (CPU only): special cases of its
layers, their adjoint identities, and central finite differences of the whole
network's loss against its backward pass."""
import numpy as np
import pytest

from oracle import surrogate as S


def test_conv_identity_kernel_returns_input():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 8, 6, 3))
    W = np.zeros((3, 3, 3, 3))
    for c in range(3):
        W[c, 1, 1, c] = 1.0
    assert np.array_equal(S.conv(x, W, np.zeros(3)), x)
    # a pure shift: output(y, x) = input(y, x + 1), zero past the edge
    W2 = np.zeros((3, 3, 3, 3))
    for c in range(3):
        W2[c, 1, 2, c] = 1.0
    y = S.conv(x, W2, np.zeros(3))
    assert np.array_equal(y[:, :, :-1], x[:, :, 1:]) and not y[:, :, -1].any()


def test_layer_adjoints():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 8, 8, 5))
    W = rng.normal(size=(4, 3, 3, 5))
    y = rng.normal(size=(2, 8, 8, 4))
    dx, dW, db = S.conv_backward(x, W, y)
    lhs = (S.conv(x, W, np.zeros(4)) * y).sum()
    assert abs(lhs - (x * dx).sum()) < 1e-10 * abs(lhs)
    V = rng.normal(size=W.shape)
    assert abs((S.conv(x, V, np.zeros(4)) * y).sum() - (V * dW).sum()) < 1e-10 * abs(lhs)
    assert np.allclose(db, y.sum(axis=(0, 1, 2)))
    p = rng.normal(size=(2, 4, 4, 5))
    assert abs((S.pool(x) * p).sum() - (x * S.pool_backward(p)).sum()) < 1e-12
    u = rng.normal(size=(2, 16, 16, 5))
    assert abs((S.up(x) * u).sum() - (x * S.up_backward(u)).sum()) < 1e-10


def test_param_count_of_the_production_network():
    # base 16, 16 (padded) input channels, 3 outputs: about one million parameters
    n = S.param_count(16, 16, 3)
    assert 1.0e6 < n < 1.4e6, n


@pytest.mark.parametrize("seed", [0, 1])
def test_network_gradient_matches_finite_differences(seed):
    base, cin, cout = 2, 3, 2
    net = S.ReferenceUNet(base, cin, cout)
    rng = np.random.default_rng(seed)
    theta = S.he_init(base, cin, cout, seed) + 0.05 * rng.normal(size=S.param_count(base, cin, cout))
    x = rng.normal(size=(2, 16, 16, cin))
    t = rng.normal(size=(2, 16, 16, cout))

    def loss(th, xx):
        y, _ = net.forward(th, xx)
        return S.ReferenceUNet.mse(y, t)[0]

    y, cache = net.forward(theta, x)
    _, dy = S.ReferenceUNet.mse(y, t)
    g, gx = net.backward(theta, cache, dy)
    h = 1e-6
    idx = rng.choice(theta.size, 60, replace=False)
    for q in idx:
        e = np.zeros_like(theta)
        e[q] = h
        fd = (loss(theta + e, x) - loss(theta - e, x)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1e-3, abs(g[q])) + 1e-9, (q, fd, g[q])
    for _ in range(10):
        i = tuple(rng.integers(0, s) for s in x.shape)
        e = np.zeros_like(x)
        e[i] = h
        fd = (loss(theta, x + e) - loss(theta, x - e)) / (2 * h)
        assert abs(fd - gx[i]) <= 1e-6 * max(1e-3, abs(gx[i])) + 1e-9, (i, fd, gx[i])


def test_bf16_round_matches_torch_conversion():
    """The reference's bfloat16 rounding against torch's CPU conversion (a
    library routine with round-to-nearest-even): random values over many
    magnitudes, both signs, zero, and exact ties with even and odd kept
    bits."""
    import torch

    rng = np.random.default_rng(5)
    a = rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, size=4000)
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0xBF818000, 0x4049_8000, 0x0080_8000],
                    dtype=np.uint32).view(np.float32).astype(np.float64)
    a = np.concatenate([a, ties, [0.0, -0.0, 1.0, -2.5]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = S.bf16_round(a)
    assert np.array_equal(got, ref)
    # ties go to the even pattern
    assert S.bf16_round(ties[:2]).tolist() == [1.0, 1.015625]


def test_stored_rounding_only_rounds_what_is_stored():
    """With the identity as the store rounding the network is the plain FP64
    one bit for bit; with bfloat16 every kept activation is a bfloat16 value
    and the output stays within bfloat16 rounding of the FP64 output."""
    base, cin, cout = 4, 3, 2
    rng = np.random.default_rng(2)
    theta = S.he_init(base, cin, cout, 2)
    x = S.bf16_round(rng.normal(size=(2, 32, 32, cin)))
    y0, _ = S.ReferenceUNet(base, cin, cout).forward(theta, x)
    y1, _ = S.ReferenceUNet(base, cin, cout, store=lambda v: v).forward(theta, x)
    assert np.array_equal(y0, y1)
    yb, cache = S.ReferenceUNet(base, cin, cout, store=S.bf16_round).forward(theta, x)
    for name, _, _, _ in S.layer_list(base, cin, cout)[:-1]:
        out = cache[name][1]
        assert np.array_equal(S.bf16_round(out), out), name
    assert np.abs(yb - y0).max() <= 2e-2 * np.abs(y0).max()
    assert not np.array_equal(yb, y0)
