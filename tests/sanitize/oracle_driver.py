"""Runs the oracle's C code, built with -fsanitize=address,undefined, through
every lattice feature on small lattices.  Started by tests/test_sanitizers.py
in a process of its own with the AddressSanitizer runtime preloaded; argv:
the sanitized float64 and long double builds.  Prints one checksum line per
case (the parent compares them with the ordinary build's)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1804_02418_amd import workloads  # noqa: E402


def cases():
    w = workloads.small_device(nx=37, ny=23, steps=6)
    yield "device", w
    w = workloads.small_device(nx=41, ny=19, steps=6, seed=2)
    w["contacts"] = [dict(edge="bottom", start=0, width=12, n=1.02), dict(edge="left", start=0, width=9, n=0.99),
                     dict(edge="right", start=10, width=9, n=1.01), dict(edge="top", start=29, width=12, n=1.0)]
    mask = np.zeros((19, 41), dtype=np.uint8)
    mask[6:11, 15:19] = 1
    mask[2, 30:36] = 1
    w["mask"] = mask
    yield "corners_mask", w
    for nx, ny in ((1, 6), (3, 7), (5, 2)):
        w = workloads.small_device(nx=nx, ny=ny, steps=6)
        w.update(periodic_x=True, periodic_y=True, contacts=[])
        yield f"tiny_{nx}x{ny}", w
    w = workloads.small_device(nx=30, ny=20, steps=6, seed=3)
    w["cg"] = 2.0
    yield "lca", w


def run(w, long_double):
    st = oracle.Stencil(long_double=long_double)
    L = oracle.Lattice(st, w["nx"], w["ny"], periodic_x=w["periodic_x"], periodic_y=w["periodic_y"],
                       contacts=w["contacts"], solid=w.get("mask"), tau=w["tau"], F=w["F"], cg=w.get("cg"))
    i = w["init"]
    shp = (w["ny"], w["nx"])
    L.init_fields(*[np.broadcast_to(np.asarray(i[k], dtype=np.float64), shp) for k in ("n", "T", "vx", "vy")])
    L.run(w["steps"])
    f = L.fields()
    fs = L.post_collision()
    back = L.stream(fs)
    return float(np.sum(np.asarray(f["n"], dtype=np.float64))), float(np.sum(np.asarray(back, dtype=np.float64)))


def main():
    oracle._LIB, oracle._LIB_LD = sys.argv[1], sys.argv[2]
    for name, w in cases():
        for ld in (False, True):
            a, b = run(w, ld)
            print(name, "ld" if ld else "f64", repr(a), repr(b), flush=True)
    # per-site functions on one site
    st = oracle.Stencil()
    U = oracle.four_velocity(0.1, -0.05)
    feq = st.feq(1.1, 0.9, U)
    out = st.collide(feq * (1 + 1e-3 * np.arange(48) / 48), 0.8, 1e-3, 2e-4)
    print("site", repr(float(out.sum())), repr(float(oracle.projections(1.1, 0.9, U).sum())), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
