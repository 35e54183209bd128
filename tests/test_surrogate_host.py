"""Host logic of the surrogate warm start (CPU only).

* encode() lays out the sample's description and the pixel coordinates in
  the network's input channels.
* decode() rejects a prediction with a non-finite value, a density n <= 0 or
  a speed |v| >= 1 (the sample then starts cold) and scales the others.
* warm_loop(), the checked solve behind solve_warm(), driven by a scripted
  stand-in for the batch: samples freeze once converged; a warm start whose
  residual rises above `growth` times its best, or that fails the health
  check, restarts from the cold start once, its spent steps counted; a cold
  start that fails the health check raises.
"""
import numpy as np
import pytest

from paper_1804_02418_amd import _binding as B
from paper_1804_02418_amd import surrogate as S


def _sample(F=1e-5, tau=0.8):
    return dict(nx=4, ny=3, tau=tau, F=(F, 0.0), contacts=[], init=dict(n=1.0, T=1.0, vx=0.0, vy=0.0))


def test_encode_channels():
    w = dict(nx=5, ny=3, tau=0.9, F=(1e-5, 0.0),
             contacts=[dict(edge="bottom", start=1, width=2), dict(edge="bottom", start=3, width=1)])
    x = S.encode(w)
    assert x.shape == (3, 5, S.CIN) and x.dtype == np.float32
    assert np.all(x[..., 0] == 1) and np.all(x[..., 3] == np.float32(0.9))
    assert np.allclose(x[..., 4], 0.0, atol=1e-6)  # log10(1e-5) + 5
    assert list(np.flatnonzero(x[0, :, 1])) == [1, 2] and list(np.flatnonzero(x[0, :, 2])) == [3]
    assert not x[1:, :, 1:3].any()
    assert np.allclose(x[1, :, 5], [0, 0.25, 0.5, 0.75, 1]) and np.allclose(x[:, 2, 6], [0, 0.5, 1])
    assert not x[..., 7:].any()


def test_decode_scales_and_rejects():
    w = _sample(F=2e-5, tau=0.9)
    pred = np.zeros((3, 4, 3), dtype=np.float32)
    pred[..., 0] = 0.5
    pred[..., 1] = 0.25
    n, vx, vy = S.decode(w, pred)
    assert np.allclose(n, 1 + 2e-5 * 0.5) and np.allclose(vx, 2e-5 / 0.4 * 0.25) and np.all(vy == 0)
    for k, v in ((0, np.nan), (1, np.inf), (0, -1.0 / 2e-5), (0, -2.0 / 2e-5), (1, 0.4 / 2e-5), (2, -0.5 / 2e-5)):
        bad = pred.copy()
        bad[1, 2, k] = v
        assert S.decode(w, bad) is None, (k, v)
    # |v| just below 1 is still a valid start
    ok = pred.copy()
    ok[1, 2, 1] = 0.999 * 0.4 / 2e-5
    assert S.decode(w, ok) is not None


class _Lattice:
    def __init__(self, batch, s):
        self.b, self.s = batch, s

    def residual(self):
        v = self.b.current[self.s]
        if v == "sick":
            raise B.Unstable(B.EUNSTABLE, "scripted")
        return v

    def init_uniform(self, n, T, vx, vy):
        self.b.restarts.append((self.s, self.b.checks))
        self.b.script[self.s] = list(self.b.after_restart[self.s])


class _Batch:
    """Scripted residuals: each step call consumes one value per active sample."""

    def __init__(self, script, after_restart=None):
        self.script = [list(v) for v in script]
        self.after_restart = after_restart or [[] for _ in script]
        self.current = [None] * len(script)
        self.active = np.ones(len(script), dtype=np.uint8)
        self.lattices = [_Lattice(self, s) for s in range(len(script))]
        self.restarts, self.checks, self.stepped = [], 0, []

    def set_active(self, a):
        self.active = np.array(a, dtype=np.uint8)

    def step(self, k):
        self.checks += 1
        self.stepped.append(k)
        for s in np.flatnonzero(self.active):
            self.current[s] = self.script[s].pop(0)

    def residual(self):
        if any(self.current[s] == "sick" for s in np.flatnonzero(self.active)):
            raise B.Unstable(B.EUNSTABLE, "scripted")
        return np.array([np.nan if v in (None, "sick") else v for v in self.current], dtype=float)


def test_warm_loop_freezes_and_falls_back():
    tol = 1e-8
    script = [
        [1e-5, 1e-6, 1e-7, 5e-9, 1.0],                # 0 cold: converges at check 4
        [1e-4, 1e-6, 2e-6, 2e-5, 9.0],                # 1 warm: 2e-5 > 10 x 1e-6 at check 4 -> restart
        [1e-4, "sick", 9.0],                          # 2 warm: health check fails at check 2 -> restart
        [1e-5, 1e-7, 6e-7, 3e-8, 9e-9, 1.0],          # 3 warm: grows 6x (< 10x): no restart, converges at 5
        [1e-3, 1e-4] + [5e-7] * 20,                   # 4 cold: never converges within the budget
    ]
    after = [[], [1e-4, 1e-6, 2e-5, 1e-7, 2e-9, 1.0], [1e-3, 1e-6, 9e-9, 1.0], [], []]
    bt = _Batch(script, after)
    warm = np.array([False, True, True, True, False])
    steps, res, restart = S.warm_loop(bt, [_sample()] * 5, warm, max_steps=1000, check_every=100, tol=tol, growth=10.0)
    assert bt.restarts == [(2, 2), (1, 4)]
    assert list(restart) == [-1, 400, 200, -1, -1]
    # sample 1 grows again after its restart (2e-5 > 10 x 1e-6) but restarts only once
    assert list(steps) == [400, 900, 500, 500, 1000]
    assert res[0] < tol and res[1] < tol and res[2] < tol and res[3] < tol and res[4] == 5e-7
    assert bt.stepped == [100] * 10
    assert list(bt.active) == [1] * 5  # every sample active again at the end


def test_warm_loop_partial_interval_does_not_converge():
    """A last interval shorter than check_every is not a convergence check."""
    bt = _Batch([[1e-6, 1e-9]])
    steps, res, restart = S.warm_loop(bt, [_sample()], np.array([False]), max_steps=150, check_every=100,
                                      tol=1e-8, growth=10.0)
    assert bt.stepped == [100, 50] and steps[0] == 150 and restart[0] == -1


def test_warm_loop_cold_failure_raises():
    bt = _Batch([[1e-5, "sick"], [1e-5, 1e-6]])
    with pytest.raises(B.Unstable):
        S.warm_loop(bt, [_sample()] * 2, np.array([False, True]), max_steps=1000, check_every=100, tol=1e-8,
                    growth=10.0)
