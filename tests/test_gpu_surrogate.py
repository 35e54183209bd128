"""GPU tests of the surrogate's BF16 kernels against the FP64 reference net.

Every kernel is compared on inputs that are first rounded to BF16 on the
host, so both sides see the same operands: a single convolution then differs
only by FP32 accumulation order plus the final BF16 rounding of its output
(relative 2^-9), the weight gradient only by FP32 accumulation.  Through the
whole network every activation is re-rounded to BF16, so end-to-end outputs
and gradients are compared at the percent level.  A short Adam run on a
fixed batch must drive the loss down.
"""
import numpy as np
import pytest

from oracle import surrogate as S

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def _bf16_round(a):
    """Round float64 -> bfloat16 -> float64 (torch implements RNE)."""
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _dev_bf16(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda().contiguous()


def _host(t):
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("ci,co,relu", [(16, 16, True), (48, 32, False), (64, 16, True), (32, 48, False)])
def test_conv3x3_forward_matches_reference(ci, co, relu):
    import paper_1804_02418_amd as rl

    torch = _torch()
    rng = np.random.default_rng(ci * 100 + co)
    B, H, W = 2, 24, 40
    x = _bf16_round(rng.normal(size=(B, H, W, ci)))
    w = _bf16_round(rng.normal(size=(co, 3, 3, ci)) / np.sqrt(9 * ci))
    b = rng.normal(size=co).astype(np.float32)
    y = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
    rl.conv3x3_forward(_dev_bf16(x), _dev_bf16(w), torch.from_numpy(b).cuda(), y, relu=relu)
    torch.cuda.synchronize()
    ref = S.conv(x, w, b.astype(np.float64))
    if relu:
        ref = np.maximum(ref, 0)
    got = _host(y)
    err = np.abs(got - ref).max()
    print("conv fwd", ci, co, relu, "max err", err, "max |ref|", np.abs(ref).max(), flush=True)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("ci,co,relu,H,W", [(16, 16, True, 6, 256), (48, 32, False, 5, 200), (32, 16, True, 4, 130),
                                           (16, 16, True, 34, 130), (64, 32, False, 33, 64)])
def test_conv3x3_forward_wide_images(ci, co, relu, H, W):
    """Images wider than one 64-pixel tile of the forward kernel, also with a
    ragged last tile: the halo between tiles comes from the neighbour's
    pixels, zero only outside the image.  From 16 rows on, a block computes
    four rows (here with a ragged last group of rows)."""
    import paper_1804_02418_amd as rl

    torch = _torch()
    rng = np.random.default_rng(ci + co + W)
    x = _bf16_round(rng.normal(size=(1, H, W, ci)))
    w = _bf16_round(rng.normal(size=(co, 3, 3, ci)) / np.sqrt(9 * ci))
    b = rng.normal(size=co).astype(np.float32)
    y = torch.empty((1, H, W, co), dtype=torch.bfloat16, device="cuda")
    rl.conv3x3_forward(_dev_bf16(x), _dev_bf16(w), torch.from_numpy(b).cuda(), y, relu=relu)
    torch.cuda.synchronize()
    ref = S.conv(x, w, b.astype(np.float64))
    if relu:
        ref = np.maximum(ref, 0)
    got = _host(y)
    print("conv fwd wide", ci, co, W, "max err", np.abs(got - ref).max(), flush=True)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("ci,co,B,H,W", [(16, 32, 2, 16, 32), (48, 16, 2, 16, 32), (80, 32, 3, 20, 48),
                                         (128, 16, 2, 160, 16), (16, 16, 1, 6, 256), (32, 16, 2, 3, 200),
                                         (16, 32, 1, 34, 70), (64, 64, 8, 64, 16), (128, 128, 8, 30, 16),
                                         (16, 16, 8, 256, 16)])
def test_conv3x3_backward_kernels_match_reference(ci, co, B, H, W):
    """Also partial 64-channel blocks, widths that are not a multiple of the
    32-pixel segment, and several row chunks (320 rows of 16 pixels); the
    last three shapes make the weight gradient take two or four rows per
    step (batch 8), the second with a last chunk that runs past the image."""
    import paper_1804_02418_amd as rl

    torch = _torch()
    rng = np.random.default_rng(7 + ci)
    x = _bf16_round(rng.normal(size=(B, H, W, ci)))
    w = _bf16_round(rng.normal(size=(co, 3, 3, ci)) / np.sqrt(9 * ci))
    dy = _bf16_round(rng.normal(size=(B, H, W, co)))
    rdx, rdw, rdb = S.conv_backward(x, w, dy)
    dx = torch.empty((B, H, W, ci), dtype=torch.bfloat16, device="cuda")
    rl.conv3x3_backward_data(_dev_bf16(dy), _dev_bf16(w), dx)
    gw = torch.zeros((co, 3, 3, ci), dtype=torch.float32, device="cuda")
    gb = torch.zeros(co, dtype=torch.float32, device="cuda")
    rl.conv3x3_backward_weight(_dev_bf16(dy), _dev_bf16(x), gw, gb)
    torch.cuda.synchronize()
    gdx, gdw, gdb = _host(dx), _host(gw), _host(gb)
    print("bwd data err", np.abs(gdx - rdx).max(), "weight err", np.abs(gdw - rdw).max() / np.abs(rdw).max(), flush=True)
    assert np.all(np.abs(gdx - rdx) <= 2.0 ** -8 * np.abs(rdx) + 1e-5 * np.abs(rdx).max())
    assert np.abs(gdw - rdw).max() <= 1e-5 * np.abs(rdw).max()
    assert np.abs(gdb - rdb).max() <= 1e-5 * np.abs(rdb).max()


def _net_case(seed=3, B=2, H=32, W=32):
    base, cin, cout = 16, 16, 3
    rng = np.random.default_rng(seed)
    theta = S.he_init(base, cin, cout, seed).astype(np.float32)
    theta[-cout:] = rng.normal(size=cout)  # non-zero head bias
    x = rng.normal(size=(B, H, W, cin))
    x[..., 5:] = 0.0
    t = rng.normal(size=(B, H, W, cout))
    return base, cin, cout, theta, x, t


@pytest.mark.parametrize("H,W", [(32, 32), (48, 48)])
def test_network_forward_and_backward_match_reference(H, W):
    """32 x 32: every pooling, concatenation and the head are fused into the
    convolutions.  48 x 48: the full-resolution convolutions take one-row
    patches of 64 pixels, so their pooled copies come from the separate
    pooling kernel instead."""
    import paper_1804_02418_amd as rl

    torch = _torch()
    base, cin, cout, theta, x, t = _net_case(H=H, W=W)
    B, H, W = x.shape[:3]
    net = rl.UNet(base, cin, cout, H, W, max_batch=B)
    net.set_params(theta)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    y = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    net.forward(xd, y)
    loss = net.mse(y, td, dy)
    net.zero_grad()
    net.backward(dy)
    g = net.get_grads().astype(np.float64)
    # reference on the BF16-rounded parameters and input (the GPU computes with those)
    ref = S.ReferenceUNet(base, cin, cout)
    theta_b = _bf16_round(theta)
    yr, cache = ref.forward(theta_b, _bf16_round(x))
    lr_, dyr = S.ReferenceUNet.mse(yr, t)
    gr, _ = ref.backward(theta_b, cache, dyr)
    got = y.cpu().numpy().astype(np.float64)
    fwd_err = np.abs(got - yr).max() / np.abs(yr).max()
    cos = float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr)))
    rel = float(np.linalg.norm(g - gr) / np.linalg.norm(gr))
    print("unet fwd rel err", fwd_err, "loss", loss, lr_, "grad cosine", cos, "grad rel L2", rel, flush=True)
    assert fwd_err < 3e-2
    assert abs(loss - lr_) < 2e-2 * lr_
    assert cos > 0.999 and rel < 5e-2


def test_conditioned_network_gradient_element_by_element():
    """The same 32 x 32 network conditioned so that it takes no ReLU decision
    near zero (weights x 1/8, biases +1; every reference activation above
    0.05): its gradient must match the reference's, which stores every
    activation in bfloat16 as the kernels do, element by element -- within
    2% of each element plus 0.5% of the layer's largest (the floor covers
    elements whose terms cancel down to the size of their rounding)."""
    import paper_1804_02418_amd as rl

    torch = _torch()
    base, cin, cout, theta, x, t = _net_case()
    off = 0
    for _, ci, co, k in S.layer_list(base, cin, cout):
        n = co * k * k * ci
        theta[off:off + n] *= 0.125
        theta[off + n:off + n + co] = 1.0
        off += n + co
    B, H, W = x.shape[:3]
    net = rl.UNet(base, cin, cout, H, W, max_batch=B)
    net.set_params(theta.astype(np.float32))
    xb = _bf16_round(x)
    y = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    net.forward(torch.from_numpy(xb.astype(np.float32)).cuda(), y)
    dy = np.random.default_rng(3).normal(size=(B, H, W, cout)) + 0.5
    dx = torch.empty((B, H, W, cin), dtype=torch.float32, device="cuda")
    net.zero_grad()
    net.backward(torch.from_numpy(dy.astype(np.float32)).cuda(), dx)
    g = net.get_grads().astype(np.float64)
    net.close()
    ref = S.ReferenceUNet(base, cin, cout, store=S.bf16_round)
    tb = _kernel_params(theta, base, cin, cout)
    yr, cache = ref.forward(tb, xb)
    names = [l[0] for l in S.layer_list(base, cin, cout)]
    amin = min(float(cache[n][1].min()) for n in names[:-1])
    assert amin > 0.05, amin
    gr, dxr = ref.backward(tb, cache, dy)
    worst = _elementwise(g, gr, base, cin, cout, rtol=2e-2, floor=5e-3)
    gdx = dx.cpu().numpy().astype(np.float64)
    wdx = float(np.max(np.abs(gdx - dxr) / (2e-2 * np.abs(dxr) + 5e-3 * np.abs(dxr).max())))
    print("32x32 conditioned: min activation", amin, "element-wise worst ratio per layer",
          {k: round(v, 3) for k, v in worst.items()}, "input", round(wdx, 3), flush=True)
    assert max(worst.values()) <= 1.0, worst
    assert wdx <= 1.0


def _elementwise(g, gr, base, cin, cout, rtol, floor):
    """Per layer, weights and biases apart: every element of the gradient g
    within rtol of the reference's element plus floor times the layer's
    largest reference element (the floor covers the elements whose terms
    cancel down to the size of their rounding).  Returns the worst ratio of
    error to allowance per layer."""
    Pg, Pr = S.unpack(g, base, cin, cout), S.unpack(gr, base, cin, cout)
    worst = {}
    for n in Pr:
        for j, tag in ((0, "w"), (1, "b")):
            a, r = Pg[n][j], Pr[n][j]
            allow = rtol * np.abs(r) + floor * np.abs(r).max()
            worst[f"{n}.{tag}"] = float(np.max(np.abs(a - r) / allow))
    return worst


def _kernel_params(theta, base, cin, cout):
    """Parameters as the kernels use them: weights in bfloat16, biases in FP32."""
    out = theta.astype(np.float64).copy()
    off = 0
    for _, ci, co, k in S.layer_list(base, cin, cout):
        n = co * k * k * ci
        out[off:off + n] = _bf16_round(out[off:off + n])
        off += n + co
    return out


def _bench_size_run(theta, x, dy):
    """Forward of the batch x, then the backward of dy; returns the output,
    the parameter gradient and the input gradient (host, float64)."""
    import paper_1804_02418_amd as rl

    torch = _torch()
    B, H, W, cin = x.shape
    cout = dy.shape[-1]
    net = rl.UNet(16, cin, cout, H, W, max_batch=B)
    net.set_params(theta)
    y = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    net.forward(torch.from_numpy(x.astype(np.float32)).cuda(), y)
    dx = torch.empty((B, H, W, cin), dtype=torch.float32, device="cuda")
    net.zero_grad()
    net.backward(torch.from_numpy(dy.astype(np.float32)).cuda(), dx)
    g = net.get_grads().astype(np.float64)
    out = y.cpu().numpy().astype(np.float64), g, dx.cpu().numpy().astype(np.float64)
    net.close()
    return out


def test_network_at_bench_size_matches_reference():
    """The production network (base 16, 16 input and 3 output channels) at
    the bench's launch configuration, a batch of 8 images of 256 x 256,
    against the reference, which keeps its activations in bfloat16 as the
    network does (FP64 arithmetic otherwise) so that both sides take their
    ReLU decisions on the same stored values.

    Outputs: two images of a He-initialised network.  Gradients: that
    network's are chaotic under rounding (one-ulp changes to 0.1% of the
    inputs move the reference's own gradient by 7-9%, because pre-activations
    within rounding of zero switch sides and gradients sum terms of random
    sign), so they are checked on a network that takes no decision near
    zero: weights scaled by 1/8 and biases of +1 keep every activation of
    the reference above 0.05 (its gradient moves by under 0.1% under the same
    perturbation).  The output gradient is non-zero on one image only; the
    other seven must add nothing."""
    base, cin, cout, B, H, W = 16, 16, 3, 8, 256, 256
    rng = np.random.default_rng(11)
    x = _bf16_round(rng.normal(size=(B, H, W, cin)))
    dy = np.zeros((B, H, W, cout))
    # with a mean (as the loss gradient of a biased prediction has), so that
    # the sums over pixels that every bias and, in a network whose
    # activations sit near 1, every weight gradient contain do not cancel
    # (a zero-mean draw can leave them several times below the size of their
    # terms, and their rounding error then looks large beside them)
    dy[3] = rng.normal(size=(H, W, cout)) + 0.5
    ref = S.ReferenceUNet(base, cin, cout, store=S.bf16_round)

    theta = S.he_init(base, cin, cout, 11).astype(np.float32)
    theta[-cout:] = rng.normal(size=cout)
    got, _, _ = _bench_size_run(theta, x, dy)
    for k in (0, 3):
        yr, _ = ref.forward(_kernel_params(theta, base, cin, cout), x[k:k + 1])
        fwd_err = np.abs(got[k] - yr[0]).max() / np.abs(yr).max()
        print("image", k, "fwd rel err", fwd_err, flush=True)
        assert fwd_err < 3e-2

    theta = S.he_init(base, cin, cout, 12).astype(np.float32)
    off = 0
    for _, ci, co, k in S.layer_list(base, cin, cout):
        n = co * k * k * ci
        theta[off:off + n] *= 0.125
        theta[off + n:off + n + co] = 1.0
        off += n + co
    got, g, gdx = _bench_size_run(theta, x, dy)
    tb = _kernel_params(theta, base, cin, cout)
    yr, cache = ref.forward(tb, x[3:4])
    names = [l[0] for l in S.layer_list(base, cin, cout)]
    amin = min(float(cache[n][1].min()) for n in names[:-1])
    assert amin > 0.05, amin
    assert np.abs(got[3] - yr[0]).max() <= 1e-2 * np.abs(yr).max()
    gr, dxr = ref.backward(tb, cache, dy[3:4])
    Pg, Pr = S.unpack(g, base, cin, cout), S.unpack(gr, base, cin, cout)
    errs = {n: tuple(round(float(np.linalg.norm(Pg[n][j] - Pr[n][j]) / np.linalg.norm(Pr[n][j])), 5) for j in (0, 1))
            for n in names}
    edx = float(np.linalg.norm(gdx[3] - dxr[0]) / np.linalg.norm(dxr))
    print("256x256 conditioned: min activation", amin, "input gradient", edx, "per layer (weights, biases)", errs,
          flush=True)
    worst = _elementwise(g, gr, base, cin, cout, rtol=2e-2, floor=5e-3)
    wdx = float(np.max(np.abs(gdx[3] - dxr[0]) / (2e-2 * np.abs(dxr[0]) + 5e-3 * np.abs(dxr).max())))
    print("element-wise worst ratio per layer", {k: round(v, 3) for k, v in worst.items()}, "input", wdx,
          flush=True)
    for n, e in errs.items():
        assert max(e) <= 2e-2, (n, e)
    assert edx <= 2e-2
    assert max(worst.values()) <= 1.0, worst
    assert wdx <= 1.0
    assert not np.any(np.delete(gdx, 3, axis=0))


def test_adam_training_reduces_loss():
    import paper_1804_02418_amd as rl

    torch = _torch()
    base, cin, cout, theta, x, t = _net_case(seed=5, B=4, H=32, W=32)
    t = 0.1 * np.tanh(t)
    B, H, W = x.shape[:3]
    net = rl.UNet(base, cin, cout, H, W, max_batch=B)
    net.set_params(theta)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    y = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    losses = []
    for _ in range(60):
        net.forward(xd, y)
        losses.append(net.mse(y, td, dy))
        net.zero_grad()
        net.backward(dy)
        net.adam_step(1e-3)
    print("losses", losses[0], losses[10], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_trained_surrogate_warm_start_saves_steps():
    """What the trained network gains over the method without it: eight
    held-out 256 x 256 samples (seeds outside the training set) run to a
    1e-8 residual from the network's prediction and from the uniform start;
    the warm starts must converge, and take fewer steps at the median.  The
    plain solver decides convergence in both cases (the network only sets
    the initial state)."""
    import os

    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import surrogate as SU
    from paper_1804_02418_amd import workloads

    path = os.path.join(os.path.dirname(rl.__file__), "data", "unet_graphene256.npz")
    d = np.load(path)
    size = int(d["size"])
    held = workloads.batch_samples(7000 + 8, fixed_size=(size, size))[7000:]
    net = rl.UNet(int(d["base"]), int(d["cin"]), int(d["cout"]), size, size, max_batch=8)
    net.set_params(d["theta"])
    preds = SU.predict(net, np.stack([SU.encode(w) for w in held]), 8) * d["scale"]
    net.close()
    inits = SU.warm_start_inits(held, preds)
    assert all(i is not None for i in inits)
    _, steps_w, r_w, _ = SU.solve_batch(held, 400_000, tol=1e-8, init=inits)
    _, steps_c, r_c, _ = SU.solve_batch(held, 400_000, tol=1e-8)
    print("warm steps", steps_w, "cold steps", steps_c, flush=True)
    assert (r_w < 1e-8).all() and (r_c < 1e-8).all()
    assert np.median(steps_w) < np.median(steps_c)


def test_rejected_predictions_start_cold():
    """Predictions with a non-finite value, a density n <= 0 or a speed
    |v| >= 1 are rejected and those samples run from the cold start: the
    checked warm solve then gives, bit for bit, the plain solver's run."""
    from paper_1804_02418_amd import surrogate as SU
    from paper_1804_02418_amd import workloads

    held = workloads.batch_samples(3, fixed_size=(256, 128))
    preds = np.zeros((3, 128, 256, 3), dtype=np.float32)
    preds[0, 40, 100, 1] = np.nan
    preds[1, ..., 0] = -2.0 / SU.drive(held[1])                              # n = -1
    preds[2, 7, 9, 1] = 1.5 * (held[2]["tau"] - 0.5) / SU.drive(held[2])   # |v| = 1.5
    inits = SU.warm_start_inits(held, preds)
    assert inits == [None, None, None]
    fw, steps_w, r_w, _, restart = SU.solve_warm(held, inits, 1500, tol=1e-30)
    fc, steps_c, r_c, _ = SU.solve_batch(held, 1500, tol=1e-30)
    assert list(restart) == [-1, -1, -1]
    assert list(steps_w) == list(steps_c) == [1500] * 3
    for a, b in zip(fw, fc):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(r_w, r_c)


def test_failing_warm_start_restarts_cold():
    """A prediction that passes the checks but throws the lattice off (a
    checkerboard of +-0.9 c) fails the health check within the first
    interval; that sample restarts from the cold start, and from there its
    run is the plain solver's run of the remaining steps, bit for bit.  The
    well-predicted sample beside it (the uniform state, an exact warm start
    of nothing) is untouched."""
    from paper_1804_02418_amd import surrogate as SU
    from paper_1804_02418_amd import workloads

    held = workloads.batch_samples(2, fixed_size=(256, 128))
    ny, nx = 128, 256
    yy, xx = np.mgrid[0:ny, 0:nx]
    wild = (0.9 * np.where((xx + yy) % 2 == 0, 1.0, -1.0), np.zeros((ny, nx)))
    inits = [(np.ones((ny, nx)), *wild), (np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))]
    fw, steps_w, _, _, restart = SU.solve_warm(held, inits, 1200, tol=1e-30)
    print("restart steps", restart, "steps", steps_w, flush=True)
    assert restart[0] == 100 and restart[1] == -1
    assert list(steps_w) == [1200, 1200]
    fc, _, _, _ = SU.solve_batch([held[0]], 1200 - 100, tol=1e-30)
    for k in fc[0]:
        assert np.array_equal(fw[0][k], fc[0][k]), k
    fu, _, _, _ = SU.solve_batch([held[1]], 1200, tol=1e-30)
    for k in fu[0]:
        assert np.array_equal(fw[1][k], fu[0][k]), k
