"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

Shared by the tests, the benchmark and the smoke check.  Each workload is a
plain dict: lattice size, boundaries, contacts, tau, drive, initial fields
and step count.  Contacts use the lattice convention of include/rlbm.h
(edge, start, width, reservoir n, T, vx, vy).

* ``shear_wave``: periodic 64 x 64, uniform n = T = 1 plus a shear wave
  u_x = 1e-3 sin(2 pi y / 64), tau = 1, no force, 500 steps (FP64).
* ``graphene_sample``: the source/drain geometry.  W x H lattice with
  bounce-back walls on every edge, two contacts on the bottom edge (source
  and drain reservoirs at n = T = 1, u = 0) whose centres sit symmetrically
  about the middle, a uniform drive F along +x (from source to drain), tau,
  uniform equilibrium start n = T = 1, u = 0.
    - 1024 x 512: contacts 32 wide, centres 256 apart, F = 1e-5, tau = 0.8,
      20 000 steps (FP32).
    - 4096 x 2048: the same scaled by 4: contacts 128 wide, centres 1024 apart.
* ``injector_setup``: the validation geometry of Sec. 3 (its figure is not
  available, so the layout is this module's): an L x W channel (2000 x 500,
  L/W = 4) with bounce-back walls, an injector contact w_in = 8 sites wide at
  the middle of the bottom edge held at f^eq(n0, T0, (0, v_in)) and both
  channel ends (the full left and right edges) held as drains at
  f^eq(n0, T0, 0); uniform start n0 = 1.5, T0 = 1.25, v = 0; the deviation
  storage references (n0, T0); local-capacitance force with C_g.
* ``batch_samples``: 256 uneven samples, sizes uniform over
  {128, 192, ..., 1024} x {128, ..., 512}, tau ~ U[0.55, 2], contact width ~
  U{8..64}, centre gap ~ U{64..384} (redrawn until gap + width <= nx - 16),
  drive 10^U[-6, -4] along +x; sample s draws from
  numpy.random.default_rng(SeedSequence(180402418).spawn(256)[s]).
"""
from __future__ import annotations

import numpy as np

SEED = 180402418


def _contact_pair(nx: int, width: int, gap: int, n=1.0, T=1.0):
    c1 = nx // 2 - gap // 2
    c2 = c1 + gap
    return [dict(edge="bottom", start=c1 - width // 2, width=width, n=n, T=T, vx=0.0, vy=0.0),
            dict(edge="bottom", start=c2 - width // 2, width=width, n=n, T=T, vx=0.0, vy=0.0)]


def shear_wave(L: int = 64, amplitude: float = 1e-3, tau: float = 1.0, steps: int = 500):
    y = np.arange(L, dtype=np.float64)[:, None] * np.ones((1, L))
    return dict(name=f"shear_wave_{L}x{L}", nx=L, ny=L, periodic_x=True, periodic_y=True, contacts=[],
                tau=tau, F=(0.0, 0.0), steps=steps, storage="f64",
                init=dict(n=np.ones((L, L)), T=np.ones((L, L)), vx=amplitude * np.sin(2 * np.pi * y / L),
                          vy=np.zeros((L, L))))


def graphene_sample(nx: int = 1024, ny: int = 512, storage: str = "f32", steps: int = 20000):
    s = nx // 1024 if nx >= 1024 else 1
    width, gap = 32 * s, 256 * s
    return dict(name=f"graphene_sample_{nx}x{ny}", nx=nx, ny=ny, periodic_x=False, periodic_y=False,
                contacts=_contact_pair(nx, width, gap), tau=0.8, F=(1e-5, 0.0), steps=steps, storage=storage,
                init=dict(n=1.0, T=1.0, vx=0.0, vy=0.0))


def batch_samples(count: int = 256, fixed_size=None):
    """The uneven-size sample generator; fixed_size=(nx, ny) pins the size."""
    seqs = np.random.SeedSequence(SEED).spawn(count)
    out = []
    for s in range(count):
        rng = np.random.default_rng(seqs[s])
        nx = int(rng.integers(2, 17)) * 64
        ny = int(rng.integers(2, 9)) * 64
        if fixed_size is not None:
            nx, ny = fixed_size
        tau = float(rng.uniform(0.55, 2.0))
        while True:
            width = int(rng.integers(8, 65))
            gap = int(rng.integers(64, 385))
            if gap + width <= nx - 16:
                break
        drive = float(10.0 ** rng.uniform(-6.0, -4.0))
        out.append(dict(name=f"sample_{s}", nx=nx, ny=ny, periodic_x=False, periodic_y=False,
                        contacts=_contact_pair(nx, width, gap), tau=tau, F=(drive, 0.0),
                        init=dict(n=1.0, T=1.0, vx=0.0, vy=0.0)))
    return out


def small_device(nx: int = 203, ny: int = 77, steps: int = 120, seed: int = 5):
    """Ragged walls + contacts on three edges + drive + smooth random start."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    ph = rng.uniform(0, 2 * np.pi, 4)
    n = 1 + 0.02 * np.sin(2 * np.pi * x / nx + ph[0]) * np.cos(2 * np.pi * y / ny + ph[1])
    T = 1 + 0.01 * np.cos(2 * np.pi * x / nx + ph[2])
    vx = 0.01 * np.sin(2 * np.pi * y / ny + ph[3])
    vy = 0.005 * np.cos(2 * np.pi * x / nx)
    # contact spans scale with the lattice (203 x 77: bottom [30, 54) and
    # [140, 180), top [0, 16), left [20, 50))
    contacts = [dict(edge="bottom", start=int(0.15 * nx), width=max(1, int(0.12 * nx)), n=1.02, T=1.0),
                dict(edge="bottom", start=int(0.69 * nx), width=max(1, int(0.2 * nx)), n=0.99, T=1.01, vx=0.002),
                dict(edge="top", start=0, width=max(1, int(0.08 * nx)), n=1.0, T=0.98),
                dict(edge="left", start=int(0.26 * ny), width=max(1, int(0.39 * ny)), n=1.01, T=1.0, vx=0.003,
                     vy=-0.001)]
    return dict(name=f"small_device_{nx}x{ny}", nx=nx, ny=ny, periodic_x=False, periodic_y=False,
                contacts=contacts, tau=0.75, F=(2e-4, -1e-4), steps=steps, storage="f64",
                init=dict(n=n, T=T, vx=vx, vy=vy))


def injector_setup(nx: int = 2000, ny: int = 500, tau: float = 1.0, cg: float = 10.0, v_in: float = 1e-5,
                   w_in: int = 8, n0: float = 1.5, T0: float = 1.25, storage: str = "f64", steps: int = 200_000):
    """Injector into a channel drained at both ends (see the module notes)."""
    start = nx // 2 - w_in // 2
    contacts = [dict(edge="bottom", start=start, width=w_in, n=n0, T=T0, vx=0.0, vy=v_in),
                dict(edge="left", start=0, width=ny, n=n0, T=T0, vx=0.0, vy=0.0),
                dict(edge="right", start=0, width=ny, n=n0, T=T0, vx=0.0, vy=0.0)]
    return dict(name=f"injector_{nx}x{ny}_tau{tau:g}_cg{cg:g}", nx=nx, ny=ny, periodic_x=False, periodic_y=False,
                contacts=contacts, tau=tau, F=(0.0, 0.0), cg=cg, reference=(n0, T0), steps=steps, storage=storage,
                v_in=v_in, w_in=w_in, injector_centre=(start + (w_in - 1) / 2.0, -0.5),
                init=dict(n=n0, T=T0, vx=0.0, vy=0.0))
