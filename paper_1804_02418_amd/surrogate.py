"""Warm-start surrogate pipeline: data from the solver, training, warm start.

Everything numerical runs in librlbm.so (the batched FP64 solver for data,
the BF16 U-Net kernels for training and inference); this module only
arranges batches and bookkeeping.

* Encoding of a sample (``encode``): an H x W x 16 float32 image with
  channels 0: fluid mask (1), 1: source contact (1 on the bottom row inside
  its span), 2: drain contact, 3: tau, 4: log10(drive) + 5, 5: x / (W - 1),
  6: y / (H - 1), 7..15: 0.  The coordinates let the network place a pixel
  in the closed box: under a uniform drive the density settles into a ramp
  along the drive, which zero padding alone locates poorly.
* Targets (``targets``): the steady state in linear response, scaled the
  way slow viscous flow scales: ((n - 1)/F, vx (tau - 1/2)/F,
  vy (tau - 1/2)/F), with F the drive magnitude (the velocity of a Stokes
  flow driven by F goes as F / viscosity, and the viscosity as tau - 1/2).
  The network is trained on these divided by per-channel scales (the
  training set's standard deviations).
* Warm start (``decode``): n = 1 + F p0, v = F (p1, p2) / (tau - 1/2),
  T = 1; the prediction is rejected (cold start instead) if any value is
  non-finite, n <= 0 or |v| >= 1.
* Fallback during the solve (``solve_warm``): the plain solver judges every
  warm start.  A warm-started sample whose residual rises above ``growth``
  (default 100) times the smallest residual it has reached, or that fails
  the health check, is restarted from the cold start (the steps it spent
  count).  The early transient of a sound warm start can raise its residual
  more than tenfold before it settles, so a smaller factor restarts starts
  that would have converged sooner than a cold one.
"""
from __future__ import annotations

import time

import numpy as np

from . import _binding as B
from . import workloads

CIN = 16
COUT = 3


def encode(w) -> np.ndarray:
    H, W = w["ny"], w["nx"]
    x = np.zeros((H, W, CIN), dtype=np.float32)
    x[..., 0] = 1.0
    for k, c in enumerate(w["contacts"][:2]):
        if c["edge"] == "bottom":
            x[0, c["start"]:c["start"] + c["width"], 1 + k] = 1.0
    x[..., 3] = w["tau"]
    x[..., 4] = np.log10(abs(w["F"][0]) + abs(w["F"][1])) + 5.0
    x[..., 5] = np.linspace(0.0, 1.0, W, dtype=np.float32)[None, :]
    x[..., 6] = np.linspace(0.0, 1.0, H, dtype=np.float32)[:, None]
    return x


def drive(w) -> float:
    return float(np.hypot(*w["F"]))


def targets(w, fields) -> np.ndarray:
    F = drive(w)
    g = w["tau"] - 0.5
    return np.stack([(fields["n"] - 1.0) / F, fields["vx"] * g / F, fields["vy"] * g / F],
                    axis=-1).astype(np.float32)


def decode(w, pred: np.ndarray):
    """(n, vx, vy) from an (unscaled) prediction, or None when it is unusable."""
    F = drive(w)
    g = w["tau"] - 0.5
    n = 1.0 + F * pred[..., 0].astype(np.float64)
    vx = F / g * pred[..., 1].astype(np.float64)
    vy = F / g * pred[..., 2].astype(np.float64)
    if not (np.isfinite(n).all() and np.isfinite(vx).all() and np.isfinite(vy).all()):
        return None
    if (n <= 0).any() or (vx * vx + vy * vy >= 1.0).any():
        return None
    return n, vx, vy


def solve_batch(samples, max_steps, check_every=100, tol=1e-8, storage="f64", init=None):
    """Run samples to steady state with the batched solver.  init: optional
    per-sample (n, vx, vy) warm starts (None entries start cold).  Returns
    (fields list, steps array, residuals array, seconds)."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = B.Batch(samples, storage)
    if init is not None:
        for L, st in zip(bt.lattices, init):
            if st is not None:
                n, vx, vy = st
                L.init_fields(n, np.ones_like(n), vx, vy)
    steps, r = bt.step_until(max_steps, check_every, tol)
    fields = [L.read_fields() for L in bt.lattices]
    bt.close()
    torch.cuda.synchronize()
    return fields, steps, r, time.perf_counter() - t0


def solve_warm(samples, inits, max_steps, check_every=100, tol=1e-8, growth=100.0, storage="f64"):
    """Batched solve from warm starts with the plain solver as the fallback.

    inits: per sample (n, vx, vy) or None (a rejected prediction: cold
    start).  See warm_loop for the schedule and the fallback rule.  Returns
    (fields list, steps array (counting steps spent before a restart),
    residuals array, seconds, restart step per sample (-1: none))."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = B.Batch(samples, storage)
    for L, st in zip(bt.lattices, inits):
        if st is not None:
            nn, vx, vy = st
            L.init_fields(nn, np.ones_like(nn), vx, vy)
    warm = np.array([st is not None for st in inits], dtype=bool)
    steps, res, restart = warm_loop(bt, samples, warm, max_steps, check_every, tol, growth)
    fields = [L.read_fields() for L in bt.lattices]
    bt.close()
    torch.cuda.synchronize()
    return fields, steps, res, time.perf_counter() - t0, restart


def warm_loop(bt, samples, warm, max_steps, check_every, tol, growth):
    """The checked solve of solve_warm on an initialised batch bt.

    Every check_every steps the batch residuals are read; a sample stops (is
    frozen) once its residual over a full interval is below tol.  A
    warm-started sample is restarted cold -- the uniform equilibrium of its
    description -- when its residual exceeds growth times the smallest it
    has reached, or when it fails the health check; it is restarted at most
    once.  A sample failing the health check from a cold start raises
    Unstable.  Returns (steps, residuals, restart step or -1) per sample."""
    n = len(samples)
    steps = np.zeros(n, dtype=np.int64)
    res = np.full(n, np.inf)
    best = np.full(n, np.inf)
    restart = np.full(n, -1, dtype=np.int64)
    active = np.ones(n, dtype=bool)
    done = 0
    while active.any() and done < max_steps:
        k = min(check_every, max_steps - done)
        bt.set_active(active.astype(np.uint8))
        bt.step(k)
        done += k
        sick = np.zeros(n, dtype=bool)
        try:
            r = bt.residual()
        except B.Unstable:
            # which samples failed: each active lattice's own health check
            r = np.array(res)
            for s in np.flatnonzero(active):
                try:
                    r[s] = bt.lattices[s].residual()
                except B.Unstable:
                    r[s], sick[s] = np.inf, True
        for s in np.flatnonzero(active):
            steps[s] += k
            res[s] = r[s]
            if warm[s] and restart[s] < 0 and (sick[s] or r[s] > growth * best[s]):
                i = samples[s].get("init", {})
                bt.lattices[s].init_uniform(i.get("n", 1.0), i.get("T", 1.0), i.get("vx", 0.0), i.get("vy", 0.0))
                restart[s] = steps[s]
                res[s] = best[s] = np.inf
                continue
            if sick[s]:
                raise B.Unstable(B.EUNSTABLE, f"sample {s} failed the health check from a cold start")
            best[s] = min(best[s], r[s])
            if k == check_every and r[s] < tol:
                active[s] = False
    bt.set_active(np.ones(n, dtype=np.uint8))
    return steps, res, restart


def generate(count, size=256, seed_offset=0, max_steps=300_000, tol=1e-8, chunk=256, log=print):
    """Steady states of `count` samples of the uneven-sample generator at a
    fixed size (FP64, residual tol over 100 steps)."""
    all_samples = workloads.batch_samples(seed_offset + count, fixed_size=(size, size))[seed_offset:]
    X, Y, info = [], [], []
    for i in range(0, count, chunk):
        part = all_samples[i:i + chunk]
        fields, steps, r, secs = solve_batch(part, max_steps, tol=tol)
        log(f"generated {i + len(part)}/{count}: steps median {int(np.median(steps))} max {int(steps.max())}, "
            f"converged {(r < tol).sum()}/{len(part)}, {secs:.1f} s")
        for w, f, s, rr in zip(part, fields, steps, r):
            X.append(encode(w))
            Y.append(targets(w, f))
            info.append(dict(steps=int(s), residual=float(rr), tau=w["tau"], F=drive(w)))
    return np.stack(X), np.stack(Y), info


def train(net, X, Y, epochs, batch, lr=1e-3, log=print, seed=0):
    """Minibatch Adam on (X, Y) held on the device; returns the loss curve."""
    import torch

    rng = np.random.default_rng(seed)
    n = X.shape[0]
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    out = torch.empty((batch,) + Y.shape[1:], dtype=torch.float32, device="cuda")
    dy = torch.empty_like(out)
    curve = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot = 0.0
        nb = 0
        for k in range(0, n - batch + 1, batch):
            idx = torch.from_numpy(order[k:k + batch]).cuda()
            xb = Xd.index_select(0, idx).contiguous()
            yb = Yd.index_select(0, idx).contiguous()
            net.forward(xb, out)
            tot += net.mse(out, yb, dy)
            nb += 1
            net.zero_grad()
            net.backward(dy)
            net.adam_step(lr * (0.5 * (1 + np.cos(np.pi * ep / epochs))))
        curve.append(tot / max(nb, 1))
        log(f"epoch {ep}: loss {curve[-1]:.4g}")
    return curve


def predict(net, X, batch):
    import torch

    preds = []
    out = torch.empty((batch,) + X.shape[1:3] + (COUT,), dtype=torch.float32, device="cuda")
    for k in range(0, X.shape[0], batch):
        xb = torch.from_numpy(X[k:k + batch]).cuda()
        nb = xb.shape[0]
        if nb < batch:
            xb = torch.cat([xb, torch.zeros((batch - nb,) + xb.shape[1:], device="cuda")])
        net.forward(xb.contiguous(), out)
        preds.append(out[:nb].cpu().numpy())
    return np.concatenate(preds)


# Layer plan of the library's U-Net (level = resolution halvings, input and
# output channels, kernel size), in the library's order: encoder, bottleneck,
# decoder (its first conv of each level sees the concatenated skip), head.
def layer_plan(base: int, cin: int, cout: int):
    c0, c1, c2, c3 = base, 2 * base, 4 * base, 8 * base
    return [(0, cin, c0, 3), (0, c0, c0, 3), (1, c0, c1, 3), (1, c1, c1, 3), (2, c1, c2, 3), (2, c2, c2, 3),
            (3, c2, c3, 3), (3, c3, c3, 3), (4, c3, c3, 3), (4, c3, c3, 3), (3, 2 * c3, c3, 3), (3, c3, c3, 3),
            (2, c3 + c2, c2, 3), (2, c2, c2, 3), (1, c2 + c1, c1, 3), (1, c1, c1, 3), (0, c1 + c0, c0, 3),
            (0, c0, c0, 3), (0, c0, cout, 1)]


def forward_flops(base: int, cin: int, cout: int, H: int, W: int) -> int:
    """Multiply-add FLOPs (2 per MAC) of the convolutions of one forward pass
    of one sample; a training step does about three times as many (forward,
    gradient of the data, gradient of the weights)."""
    return sum(2 * (H >> lv) * (W >> lv) * ci * co * k * k for lv, ci, co, k in layer_plan(base, cin, cout))


def channel_scales(Y) -> np.ndarray:
    return np.maximum(Y.reshape(-1, Y.shape[-1]).std(axis=0), 1e-12).astype(np.float32)


def warm_start_inits(samples, preds):
    """Decoded warm starts, None where the prediction is rejected."""
    return [decode(w, p) for w, p in zip(samples, preds)]
