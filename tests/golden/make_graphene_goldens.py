"""Stored oracle fields of the graphene sample, for the long-run GPU parity
tests and the benchmark's precision report.

Runs the oracle (and only the oracle: ``oracle/`` plus the input recipe of
``paper_1804_02418_amd.workloads``) on the graphene sample from its uniform
start -- walls on every edge, two bottom contacts, drive F = (1e-5, 0),
tau = 0.8 -- and stores, at each checkpoint step, the fields n, vx, vy, eps at
a fixed subset of sites: every 16th row and column (every 32nd at 4096 x
2048), the five rows and columns next to each edge, and the 8 (16) rows
above the two contacts, which hold the largest velocities.

Two builds of the oracle run side by side: the float64 oracle (the parity
reference, fields ``n``, ``vx``, ...) and, where ``--long-double`` covers the
checkpoint, the same source built with long double arithmetic and state
(fields ``n_ld``, ``vx_ld``, ...).  Both use the same float64 quadrature, so
they solve the same discrete problem and differ only by rounding; the
metadata records that difference over every site (``floor``), which is the
float64 rounding floor of this computation after that many steps.

At 4096 x 2048 the file also holds the 8 x 8 block means of n - 1, vx and vy
(512 x 256, float32) for the precision report of the three storages.

Usage (from the repository root; several minutes to hours of CPU):
    python tests/golden/make_graphene_goldens.py --size 1024x512 --steps 200,1000,20000 --long-double 200,1000
    python tests/golden/make_graphene_goldens.py --size 4096x2048 --steps 200 --long-double 200
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1804_02418_amd import workloads  # noqa: E402


def site_subset(w):
    """Flat indices (y * nx + x) of the stored sites, sorted."""
    nx, ny = w["nx"], w["ny"]
    stride = 16 if nx <= 1024 else 32
    xs = np.unique(np.concatenate([np.arange(0, nx, stride), np.arange(5), nx - 1 - np.arange(5)]))
    ys = np.unique(np.concatenate([np.arange(0, ny, stride), np.arange(5), ny - 1 - np.arange(5)]))
    grid = (ys[:, None] * nx + xs[None, :]).ravel()
    rows = 8 if nx <= 1024 else 16
    lo = min(c["start"] for c in w["contacts"]) - 16
    hi = max(c["start"] + c["width"] for c in w["contacts"]) + 16
    band = (np.arange(rows)[:, None] * nx + np.arange(max(lo, 0), min(hi, nx))[None, :]).ravel()
    return np.unique(np.concatenate([grid, band])).astype(np.int64)


def oracle_lattice(w, long_double):
    st = oracle.stencil(long_double=long_double)
    L = oracle.Lattice(st, w["nx"], w["ny"], periodic_x=w["periodic_x"], periodic_y=w["periodic_y"],
                       contacts=w["contacts"], tau=w["tau"], F=w["F"])
    i = w["init"]
    L.init_fields(i["n"], i["T"], i["vx"], i["vy"])
    return L


def errors(f, ref):
    """err_n = max |n - n_ref| / |n_ref|; err_u = max |u - u_ref| / max |u_ref|."""
    du = np.hypot(f["vx"] - ref["vx"], f["vy"] - ref["vy"])
    return {"err_n": float(np.max(np.abs(f["n"] - ref["n"]) / np.abs(ref["n"]))),
            "err_u": float(du.max() / np.hypot(ref["vx"], ref["vy"]).max()),
            "abs_u": float(du.max())}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", default="1024x512")
    ap.add_argument("--steps", default="200")
    ap.add_argument("--long-double", default="", help="checkpoints also run with the long double oracle")
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args(argv)
    nx, ny = (int(v) for v in a.size.split("x"))
    steps = sorted(int(s) for s in a.steps.split(",") if s)
    ld_steps = sorted(int(s) for s in a.long_double.split(",") if s)
    w = workloads.graphene_sample(nx, ny, storage="f64")
    idx = site_subset(w)
    D = oracle_lattice(w, False)
    LD = oracle_lattice(w, True) if ld_steps else None
    t0 = time.time()
    for t in steps:
        D.run(t - D.t)
        fd = {k: np.asarray(v, dtype=np.float64) for k, v in D.fields().items()}
        rec = {"workload": w["name"], "steps": t, "threads": oracle.lib().orc_get_threads(),
               "umax": float(np.hypot(fd["vx"], fd["vy"]).max())}
        arrays = {"sites": idx}
        for k in ("n", "vx", "vy", "eps"):
            arrays[k] = fd[k].ravel()[idx]
        if LD is not None and t in ld_steps:
            LD.run(t - LD.t)
            fl = LD.fields()
            for k in ("n", "vx", "vy", "eps"):
                arrays[k + "_ld"] = np.asarray(fl[k].ravel()[idx], dtype=np.float64)
            rec["floor"] = errors(fd, {k: np.asarray(v, dtype=np.float64) for k, v in fl.items()})
        if nx > 1024:
            b = 8

            def down(v):
                return v.reshape(ny // b, b, nx // b, b).mean(axis=(1, 3))

            arrays["down_n1"] = down(fd["n"] - 1.0).astype(np.float32)
            arrays["down_vx"] = down(fd["vx"]).astype(np.float32)
            arrays["down_vy"] = down(fd["vy"]).astype(np.float32)
        rec["seconds"] = round(time.time() - t0, 1)
        path = os.path.join(a.out, f"graphene_{nx}x{ny}_t{t}.npz")
        np.savez_compressed(path, meta=np.array(json.dumps(rec)), **arrays)
        print(path, json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
