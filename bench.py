#!/usr/bin/env python3
"""Benchmark of the fused relativistic LB step on one MI355X.

Workload (default): the 4096 x 2048 graphene sample -- bounce-back walls on
every edge, source and drain contacts 128 wide on the bottom edge with
centres 1024 apart, uniform drive F = 1e-5 along +x, tau = 0.8, FP32
populations, uniform equilibrium start -- stepped K times after W warm-up
steps.  Its two population arrays (3.2 GB) are far larger than the 256 MB
Infinity Cache, so the step streams from HBM.  One step = one pass of the
whole per-site update (pull with boundary rules, moments, Landau frame,
equilibrium, force, relaxation, store) over every site.

Prints one JSON line: MLUPS (million lattice-site updates per second), the
HBM roofline of the step kernel (algorithmic bytes per launch over the
average launch time measured with HIP events on the kernel's stream), the
same over a longer sustained run, the other storages and the 1024 x 512
sample (whose FP32 and FP16 arrays stay in the Infinity Cache), the
precision of every storage against the FP64 oracle (stored oracle fields
after 200 steps, 8 x 8 block means) and against the FP64 path after 20 000
steps, the aggregate throughput of the 256-sample uneven batch, the
surrogate's warm- vs cold-start time to a steady state, and the FP64 CPU
oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_POP = {"f64": 8, "f32": 4, "f16dev": 2}
KERNEL_SOURCES = ["paper_1804_02418_amd/csrc/step_impl.h", "paper_1804_02418_amd/csrc/rlbm_math.h",
                  "paper_1804_02418_amd/csrc/rlbm_kernels.h"]


def kernel_source_sha() -> str:
    """Hash of the step kernel's code (comments and blank lines left out, so
    that a comment edit does not orphan the counter records taken on it)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(HERE, p), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
        h.update("\n".join(lines).encode())
    return h.hexdigest()[:16]


def measured_traffic(name: str, sites: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(HERE, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != kernel_source_sha() or rec.get("sites") != sites:
        return None
    return rec.get("bytes_per_launch")


def make_lattice(w, storage, stream):
    import paper_1804_02418_amd as rl

    L = rl.Lattice(w["nx"], w["ny"], storage, stream=stream)
    L.set_boundaries(w["periodic_x"], w["periodic_y"], w["contacts"])
    L.set_tau(w["tau"])
    L.set_drive(*w["F"])
    i = w["init"]
    L.init_uniform(i["n"], i["T"], i["vx"], i["vy"])
    return L


def run_gpu(w, storage, steps, warmup, autotune=True):
    """Returns (seconds for `steps` steps, average launch ms, residual)
    timed with HIP events on the lattice's stream (torch's current stream).
    The library's autotuner picks the launch shape and memory form first
    (its trials are rolled back, so the timed steps start from the same
    state); the pick is left in run_gpu.launch."""
    import torch

    stream = torch.cuda.current_stream()
    L = make_lattice(w, storage, stream.cuda_stream)
    launch = None
    if autotune:
        # about 250 GB of algorithmic traffic per candidate run (45 ms at
        # 5.5 TB/s: 78 steps of FP32 at 4096 x 2048, 621 of FP64 at 1024 x 512),
        # so that every candidate is timed at the clocks a long run settles at
        ms = L.autotune(max(10, 250_000_000_000 // (2 * 48 * BYTES_PER_POP[storage] * w["nx"] * w["ny"])))
        nts, ntl = L.memory_form()
        launch = {"tile_x": L.launch_shape()[0], "streaming_stores": nts, "nontemporal_loads": ntl,
                  "trial_ms": [round(float(v), 4) for v in ms]}
    L.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    L.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    r = None
    try:
        r = L.residual()
    except Exception as exc:  # health check failure is reported, not hidden
        r = f"unstable: {exc}"
    L.close()
    run_gpu.launch = launch
    return ms / 1e3, ms / max(steps, 1), r


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps: int):
    """The FP64 oracle on this host's cores: `steps` steps of the workload
    from its uniform start on every thread, then one more on one thread.
    Returns (record, oracle fields after `steps` steps)."""
    import oracle

    st = oracle.stencil()
    O = oracle.Lattice(st, w["nx"], w["ny"], periodic_x=w["periodic_x"], periodic_y=w["periodic_y"],
                       contacts=w["contacts"], tau=w["tau"], F=w["F"])
    i = w["init"]
    O.init_fields(i["n"], i["T"], i["vx"], i["vy"])
    lib = oracle.lib()
    cores = lib.orc_get_threads()
    t0 = time.perf_counter()
    O.run(steps)
    dt = time.perf_counter() - t0
    ref = O.fields()
    lib.orc_set_threads(1)
    t1 = time.perf_counter()
    O.run(1)
    d1 = time.perf_counter() - t1
    lib.orc_set_threads(cores)
    sites = w["nx"] * w["ny"]
    base = {"value": round(sites * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{w['nx']}x{w['ny']} graphene sample, {steps} steps from the uniform start, FP64, "
                      f"{cores} threads, {dt:.1f} s",
            "single_thread": {"value": round(sites / d1 / 1e6, 3), "unit": "MLUPS",
                              "sample": f"the next step on one thread, {d1:.1f} s"}}
    return base, ref


def errors_vs_oracle(w, steps: int, ref):
    """The library's step in every storage, `steps` steps from the same
    uniform start as the oracle's fields `ref`: max-relative error in n (per
    site) and in u (of the largest oracle velocity) over the fluid sites."""
    import numpy as np
    import torch

    fluid = ~w["mask"].astype(bool) if w.get("mask") is not None else np.ones((w["ny"], w["nx"]), bool)
    rn = ref["n"][fluid]
    ru = np.hypot(ref["vx"], ref["vy"])[fluid]
    out = {"steps": steps, "reference": "FP64 oracle"}
    for st in ("f64", "f32", "f16dev"):
        L = make_lattice(w, st, torch.cuda.current_stream().cuda_stream)
        L.step(steps)
        g = L.read_fields()
        L.close()
        du = np.hypot(g["vx"] - ref["vx"], g["vy"] - ref["vy"])[fluid]
        out[st] = {"err_n": float(np.max(np.abs(g["n"][fluid] - rn) / np.abs(rn))),
                   "err_u": float(du.max() / ru.max())}
    out["max_u"] = float(ru.max())
    return out


GOLDEN = os.path.join(HERE, "tests", "golden")


def _field_errors(g, ref, sel=None):
    """err_n = max |n - n_ref| / |n_ref|; err_u = max |u - u_ref| / max |u_ref|;
    abs_u = max |u - u_ref| (early in a run the largest velocity is small, and
    err_u then magnifies differences at the level of the populations' rounding)."""
    sel = np.ones_like(ref["n"], dtype=bool) if sel is None else sel
    du = np.hypot(g["vx"] - ref["vx"], g["vy"] - ref["vy"])[sel]
    return {"err_n": float(np.max(np.abs(g["n"][sel] - ref["n"][sel]) / np.abs(ref["n"][sel]))),
            "err_u": float(du.max() / np.hypot(ref["vx"], ref["vy"])[sel].max()), "abs_u": float(du.max())}


def precision_vs_oracle(w, steps: int = 200, block: int = 8):
    """Every storage after `steps` steps from the uniform start against the
    FP64 oracle's fields of the same run (stored by
    tests/golden/make_graphene_goldens.py, which calls only the oracle): at
    the stored sites, and on the block-mean downsample (8 x 8 blocks: 512 x
    256 at 4096 x 2048).  None if the file is missing."""
    import torch

    path = os.path.join(GOLDEN, f"graphene_{w['nx']}x{w['ny']}_t{steps}.npz")
    if not os.path.exists(path):
        return None
    gd = np.load(path)
    meta = json.loads(str(gd["meta"]))
    sites = gd["sites"]
    ref = {k: gd[k] for k in ("n", "vx", "vy")}
    umax = meta["umax"]
    nx, ny = w["nx"], w["ny"]

    def down(a):
        return a.reshape(ny // block, block, nx // block, block).mean(axis=(1, 3))

    dref = {"n": 1.0 + gd["down_n1"].astype(np.float64), "vx": gd["down_vx"].astype(np.float64),
            "vy": gd["down_vy"].astype(np.float64)} if "down_n1" in gd else None
    out = {"steps": steps, "reference": "FP64 oracle (stored fields)", "stored_sites": int(sites.size),
           "oracle_float64_vs_long_double": meta.get("floor"),
           "downsample_reference": "8 x 8 block means of the oracle's fields stored in float32: errors below "
                                   "about 1e-7 there are the stored reference's rounding"}
    for st in ("f64", "f32", "f16dev"):
        L = make_lattice(w, st, torch.cuda.current_stream().cuda_stream)
        L.step(steps)
        g = L.read_fields()
        L.close()
        at = {k: g[k].ravel()[sites] for k in ("n", "vx", "vy")}
        du = np.hypot(at["vx"] - ref["vx"], at["vy"] - ref["vy"])
        rec = {"sites": {"err_n": float(np.max(np.abs(at["n"] - ref["n"]) / np.abs(ref["n"]))),
                         "err_u": float(du.max() / umax), "abs_u": float(du.max())}}
        if dref is not None:
            gdn = {k: down(g[k]) for k in ("n", "vx", "vy")}
            rec["downsample"] = _field_errors(gdn, dref)
        out[st] = rec
    return out


def precision_long_run(w, steps: int = 20000, block: int = 8):
    """FP32 and FP16-deviation storage against the FP64 path after `steps`
    steps (the FP64 path is tied to the FP64 oracle by the parity tests and
    the stored-oracle comparison): full fields and 8 x 8 block means."""
    import torch

    nx, ny = w["nx"], w["ny"]

    def down(a):
        return a.reshape(ny // block, block, nx // block, block).mean(axis=(1, 3))

    fields = {}
    for st in ("f64", "f32", "f16dev"):
        L = make_lattice(w, st, torch.cuda.current_stream().cuda_stream)
        L.step(steps)
        fields[st] = L.read_fields()
        L.close()
    ref = fields["f64"]
    dref = {k: down(ref[k]) for k in ("n", "vx", "vy")}
    out = {"steps": steps, "reference": "FP64 storage on the GPU", "downsample": [ny // block, nx // block],
           "max_u": float(np.hypot(ref["vx"], ref["vy"]).max())}
    for st in ("f32", "f16dev"):
        g = fields[st]
        out[st] = {"full": _field_errors(g, ref),
                   "downsample": _field_errors({k: down(g[k]) for k in ("n", "vx", "vy")}, dref)}
    return out


def copy_calibration(nbytes: int, reps: int = 20):
    """Plain device-to-device copy of nbytes (torch), timed with HIP events:
    the practical HBM bandwidth, and the kernel whose FETCH_SIZE / WRITE_SIZE
    counters calibrate the step kernel's measured traffic."""
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_bytes": nbytes, "read_plus_write_GBs": round(2 * nbytes / (ms / 1e3) / 1e9, 1),
            "ms_per_copy": round(ms, 4)}


def bandwidth_probes():
    """Practical bandwidth ceilings for the step: read, copy and the 48-plane
    pull pattern (trivial arithmetic) on arrays the size of one population
    array, plus torch's device copy, HIP events (include/rlbm_probe.h)."""
    from paper_1804_02418_amd import _binding as B

    rows = []
    for nx, ny, reps in ((4096, 2048, 20), (1024, 512, 200)):
        for pattern, nt in (("read", False), ("copy", False), ("copy", True)):
            g, u = B.bandwidth_probe(pattern, 4, nx, ny, nt, reps)
            rows.append({"pattern": pattern, "nontemporal": nt, "array_bytes": 48 * 4 * nx * ny, "GBs": round(g, 1),
                         "us": round(u, 2)})
    for pattern in ("pull48", "pull48_pair", "pull12_tuple", "pull24_tuple"):
        for elem, nx, ny, reps in ((4, 4096, 2048, 20), (2, 4096, 2048, 20), (8, 4096, 2048, 10), (4, 1024, 512, 200)):
            for nt in (False, True):
                g, u = B.bandwidth_probe(pattern, elem, nx, ny, nt, reps)
                rows.append({"pattern": pattern, "elem_bytes": elem, "nx": nx, "ny": ny, "nontemporal": nt,
                             "GBs": round(g, 1), "us": round(u, 2)})
    # 64 x 4 blocks, also on narrow lattices of about the same site count (a
    # batch's samples are a few hundred sites wide)
    for pattern in ("pull48_t64", "pull24_tuple_t64", "pull12_tuple_t64"):
        for elem, nx, ny, reps in ((4, 4096, 2048, 20), (4, 320, 26214, 20), (4, 192, 43690, 20), (2, 4096, 2048, 20),
                                   (2, 320, 26214, 20), (8, 4096, 2048, 10)):
            for nt in (False, True):
                g, u = B.bandwidth_probe(pattern, elem, nx, ny, nt, reps)
                rows.append({"pattern": pattern, "elem_bytes": elem, "nx": nx, "ny": ny, "nontemporal": nt,
                             "GBs": round(g, 1), "us": round(u, 2)})
    rows.append(dict(pattern="torch device copy", **copy_calibration(1 << 30)))
    return rows


WEIGHTS = os.path.join(HERE, "paper_1804_02418_amd", "data", "unet_graphene256.npz")


def main_precision(argv):
    """--precision-report: the long-run precision leg alone (any size, steps)."""
    from paper_1804_02418_amd import workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=20000)
    a = ap.parse_args(argv)
    w = workloads.graphene_sample(a.nx, a.ny)
    print(json.dumps({"precision_long_run": precision_long_run(w, a.steps)}), flush=True)
    return 0


def warm_vs_cold(path: str, count: int = 64, first_index: int = 6000, tol: float = 1e-8,
                 max_steps: int = 400_000):
    """Time to a 1e-8 residual of `count` held-out 256 x 256 samples (seeds
    disjoint from the training set), started cold (uniform equilibrium) and
    warm (the trained surrogate's prediction, with the plain solver as the
    fallback), each as one batched FP64 run.  Warm wall time includes the
    network's inference."""
    import torch

    from paper_1804_02418_amd import _binding as B
    from paper_1804_02418_amd import surrogate as S
    from paper_1804_02418_amd import workloads

    d = np.load(path)
    size = int(d["size"])
    held = workloads.batch_samples(first_index + count, fixed_size=(size, size))[first_index:]
    net = B.UNet(int(d["base"]), int(d["cin"]), int(d["cout"]), size, size, max_batch=8)
    net.set_params(d["theta"])
    X = np.stack([S.encode(w) for w in held])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    preds = S.predict(net, X, 8) * d["scale"]
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    inits = S.warm_start_inits(held, preds)
    fw, steps_w, r_w, t_w, restart = S.solve_warm(held, inits, max_steps, tol=tol)
    fc, steps_c, r_c, t_c = S.solve_batch(held, max_steps, tol=tol)
    net.close()
    # prediction error against the converged cold solution, relative RMS of the velocity
    rel = [float(np.sqrt(np.mean((np.hypot(*(S.decode(w, p)[1:]) ) - np.hypot(c["vx"], c["vy"])) ** 2)) /
                 np.sqrt(np.mean(np.hypot(c["vx"], c["vy"]) ** 2)))
           for w, p, c in zip(held, preds, fc) if S.decode(w, p) is not None]
    ratio = steps_w / np.maximum(steps_c, 1)
    return {"samples": count, "size": size, "tol": tol, "first_seed": first_index,
            "cold": {"steps_median": float(np.median(steps_c)), "steps_mean": float(np.mean(steps_c)),
                     "seconds": round(t_c, 3), "converged": int((r_c < tol).sum())},
            "warm": {"steps_median": float(np.median(steps_w)), "steps_mean": float(np.mean(steps_w)),
                     "seconds_incl_inference": round(t_w + t_inf, 3), "inference_seconds": round(t_inf, 4),
                     "converged": int((r_w < tol).sum()),
                     "rejected_predictions": sum(1 for i in inits if i is None),
                     "restarted_cold": int((restart >= 0).sum())},
            "steps_ratio_warm_over_cold": {"median": round(float(np.median(ratio)), 4),
                                           "p10": round(float(np.percentile(ratio, 10)), 4),
                                           "p90": round(float(np.percentile(ratio, 90)), 4)},
            "prediction_rel_rms_velocity_median": round(float(np.median(rel)), 4) if rel else None,
            "speedup_wall": round(t_c / (t_w + t_inf), 3)}


def batch_throughput(storage: str = "f32", count: int = 256, steps: int = 100, warmup: int = 10, rounds: int = 3):
    """Aggregate throughput of the uneven-sample batch (`count` samples of the
    batch generator, about 50 M sites at 256) advanced by the batched kernel,
    one launch per step over every sample's blocks: default launch shapes
    without the step graph, then two batches of the same samples, one with
    the default shapes and one after the batch autotuner, timed alternately
    with the step graph for `rounds` rounds (the medians are reported, so
    that a drift of the clock over the run falls on both alike).  HIP events
    on the batches' stream; each timed call includes the per-call copy of the
    previous velocities and the field write of its last step."""
    import statistics

    import torch

    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import workloads

    # a stream of its own: the batch must not run on a null stream the events would not order
    stream = torch.cuda.Stream()
    samples = workloads.batch_samples(count)
    per_site = 2 * 48 * BYTES_PER_POP[storage]

    def timed(B, graph):
        B.step(warmup, graph)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        B.step(steps, graph)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    def entry(ms):
        return {"ms_per_step": round(ms, 4), "mlups": round(sites / (ms / 1e3) / 1e6, 1),
                "roofline_frac": round(sites * per_site / (ms / 1e3) / (PEAK_HBM_GBS * 1e9), 4)}

    default = rl.Batch(samples, storage, stream=stream.cuda_stream)
    sites = default.sites()
    out = {"samples": count, "sites": sites, "storage": storage, "steps": steps, "rounds": rounds}
    out["default_shape_no_graph"] = entry(timed(default, False))
    tuned = rl.Batch(samples, storage, stream=stream.cuda_stream)
    tuned.autotune(20)

    def tiles_by_class(B):
        """Tile shapes in use per width class (multiple of 256, of 128 only, other)."""
        out = {}
        for w, L in zip(samples, B.lattices):
            k = "w%256==0" if w["nx"] % 256 == 0 else "w%128==0" if w["nx"] % 128 == 0 else "other"
            t, r = L.launch_shape()
            out.setdefault(k, {}).setdefault(f"{t}x{r}", 0)
            out[k][f"{t}x{r}"] += 1
        return out

    out["tiles_default"] = tiles_by_class(default)
    out["tiles_autotuned"] = tiles_by_class(tuned)
    t_default, t_tuned = [], []
    for _ in range(rounds):
        t_default.append(timed(default, True))
        t_tuned.append(timed(tuned, True))
    out["default_shape_graph"] = entry(statistics.median(t_default))
    out["autotuned_graph"] = entry(statistics.median(t_tuned))
    default.close()
    tuned.close()
    return out


PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak


def surrogate_throughput(batch: int = 8, size: int = 256, steps: int = 20, warmup: int = 3):
    """Training-step and inference throughput of the warm-start U-Net (base
    16, 16 input and 3 output channels) on a batch of random 256 x 256
    images: forward, loss, backward and Adam per training step, HIP events
    on the network's stream (torch's current stream).  FLOPs are the
    convolutions' multiply-adds (3 x forward for a training step)."""
    import torch

    from paper_1804_02418_amd import _binding as B
    from paper_1804_02418_amd import surrogate as S

    torch.manual_seed(0)
    net = B.UNet(16, S.CIN, S.COUT, size, size, max_batch=batch)
    x = torch.randn((batch, size, size, S.CIN), device="cuda")
    y = torch.randn((batch, size, size, S.COUT), device="cuda")
    out = torch.empty_like(y)
    dy = torch.empty_like(y)
    stream = torch.cuda.current_stream()

    def train_step():
        net.forward(x, out)
        net.mse(out, y, dy)
        net.zero_grad()
        net.backward(dy)
        net.adam_step(1e-4)

    def timed(fn, n):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(n):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / n

    ms_train = timed(train_step, steps)
    ms_infer = timed(lambda: net.forward(x, out), steps)
    nparam = net.nparam
    net.close()
    fwd = S.forward_flops(16, S.CIN, S.COUT, size, size) * batch
    return {"batch": batch, "size": size, "params": int(nparam),
            "ms_per_train_step": round(ms_train, 3), "ms_per_forward": round(ms_infer, 3),
            "train_tflops": round(3 * fwd / (ms_train / 1e3) / 1e12, 2),
            "forward_tflops": round(fwd / (ms_infer / 1e3) / 1e12, 2),
            "peak_bf16_tflops": PEAK_BF16_TFLOPS,
            "forward_frac": round(fwd / (ms_infer / 1e3) / 1e12 / PEAK_BF16_TFLOPS, 4)}


def surrogate_layers(batch: int = 8, size: int = 256, reps: int = 50):
    """Each 3x3 convolution of the U-Net alone (rlbm_conv3x3_forward on random
    BF16 tensors of the layer's shape, ReLU on): microseconds per call (HIP
    events over `reps` calls after 3 untimed), TFLOP/s of its multiply-adds and
    GB/s of its input plus output."""
    import torch

    from paper_1804_02418_amd import _binding as B
    from paper_1804_02418_amd import surrogate as S

    torch.manual_seed(0)
    stream = torch.cuda.current_stream()
    names = ["e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "e4a", "e4b", "ba", "bb", "d4a", "d4b", "d3a", "d3b", "d2a",
             "d2b", "d1a", "d1b"]
    rows = []
    for name, (lv, ci, co, k) in zip(names, S.layer_plan(16, S.CIN, S.COUT)):
        H = W = size >> lv
        x = torch.randn((batch, H, W, ci), device="cuda").to(torch.bfloat16)
        w = (torch.randn((co, 3, 3, ci), device="cuda") / (9 * ci) ** 0.5).to(torch.bfloat16)
        b = torch.randn(co, device="cuda")
        y = torch.empty((batch, H, W, co), device="cuda", dtype=torch.bfloat16)
        for _ in range(3):
            B.conv3x3_forward(x, w, b, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            B.conv3x3_forward(x, w, b, y)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        rows.append({"layer": name, "level": lv, "ci": ci, "co": co, "us": round(us, 2),
                     "tflops": round(2.0 * batch * H * W * ci * co * 9 / us / 1e6, 1),
                     "gbs": round(2.0 * batch * H * W * (ci + co) / us / 1e3, 1)})
    return {"batch": batch, "size": size, "layers": rows, "sum_us": round(sum(r["us"] for r in rows), 1)}


def cache_resident(w, storage) -> bool:
    """Both population arrays fit the 256 MB Infinity Cache (the step then
    need not stream from HBM)."""
    return 2 * 48 * BYTES_PER_POP[storage] * w["nx"] * w["ny"] <= 256 * 2 ** 20


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16dev"])
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--cpu-steps", type=int, default=16, help="oracle steps for the CPU baseline (0 = skip)")
    ap.add_argument("--sustained-steps", type=int, default=1000,
                    help="steps of the separately timed sustained run (0 = skip)")
    ap.add_argument("--long-run-steps", type=int, default=20000,
                    help="steps of the FP32 / FP16 vs FP64 precision leg (0 = skip)")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the surrogate warm- vs cold-start timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-sample batched-kernel throughput")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate network throughput")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision legs")
    ap.add_argument("--surrogate-only", action="store_true", help="only time the surrogate network")
    ap.add_argument("--surrogate-layers", action="store_true", help="only time each convolution of the network alone")
    ap.add_argument("--batch-only", action="store_true", help="only time the 256-sample batch")
    ap.add_argument("--bandwidth-probes", action="store_true",
                    help="only measure read, copy and 48-plane pull bandwidth (the practical ceilings)")
    ap.add_argument("--batch-steps", type=int, default=100, help="timed steps per batch configuration")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other storages at this size and the 1024 x 512 sample")
    ap.add_argument("--copy-bytes", type=int, default=0, help="only run the copy-bandwidth calibration")
    ap.add_argument("--no-autotune", action="store_true", help="time the default launch shape")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; y-slab sharding across GPUs is "
                                   "designed but not implemented", "n_gpus": args.gpus}), flush=True)
        return 2
    if args.copy_bytes:
        print(json.dumps(copy_calibration(args.copy_bytes)), flush=True)
        return 0
    if args.surrogate_only:
        print(json.dumps({"surrogate": surrogate_throughput()}), flush=True)
        return 0
    if args.surrogate_layers:
        print(json.dumps({"surrogate_layers": surrogate_layers()}), flush=True)
        return 0
    if args.bandwidth_probes:
        for row in bandwidth_probes():
            print(json.dumps(row), flush=True)
        return 0
    if args.batch_only:
        print(json.dumps({"batch_256": batch_throughput(steps=args.batch_steps)}), flush=True)
        return 0

    from paper_1804_02418_amd import workloads

    w = workloads.graphene_sample(args.nx, args.ny, storage=args.storage, steps=args.steps)
    sites = w["nx"] * w["ny"]
    per_site = 2 * 48 * BYTES_PER_POP[args.storage]
    secs, launch_ms, resid = run_gpu(w, args.storage, args.steps, args.warmup, not args.no_autotune)
    mlups = sites * args.steps / secs / 1e6
    achieved = per_site * sites / (launch_ms / 1e3) / 1e9
    out = {
        "metric": "MLUPS & % HBM roofline; warm-start vs cold time-to-steady at 1e-8 residual",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs * 1e3 / args.steps, 5),
        "timed_seconds": round(secs, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16dev": "f16 storage / f32 math"}[args.storage],
        "data": "synthetic",
        "config": {"workload": w["name"], "nx": w["nx"], "ny": w["ny"], "storage": args.storage, "tau": w["tau"],
                   "drive": w["F"][0], "contacts": [[c["start"], c["width"]] for c in w["contacts"]],
                   "cache_resident": cache_resident(w, args.storage), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(f"step_{args.storage}_{w['nx']}x{w['ny']}", sites)},
        "residual_last_call": resid,
        "launch": run_gpu.launch,
    }
    print(f"headline {mlups:.1f} MLUPS, {achieved / PEAK_HBM_GBS:.4f} of HBM peak", file=sys.stderr, flush=True)
    if args.sustained_steps > 0:
        s2, l2, _ = run_gpu(w, args.storage, args.sustained_steps, args.warmup, not args.no_autotune)
        g2 = per_site * sites / (l2 / 1e3) / 1e9
        out["sustained"] = {"steps": args.sustained_steps, "mlups": round(sites * args.sustained_steps / s2 / 1e6, 1),
                            "hbm_gbs": round(g2, 1), "frac": round(g2 / PEAK_HBM_GBS, 4)}
    if not args.no_variants:
        # the other storages at this size, and the 1024 x 512 sample in all three
        extra = {}

        def variant(wv, st, steps, warmup):
            s3, l3, _ = run_gpu(wv, st, steps, warmup)
            n = wv["nx"] * wv["ny"]
            gbs = 2 * 48 * BYTES_PER_POP[st] * n / (l3 / 1e3) / 1e9
            extra[f"{wv['name']}_{st}"] = {"mlups": round(n * steps / s3 / 1e6, 1), "hbm_gbs": round(gbs, 1),
                                           "frac": round(gbs / PEAK_HBM_GBS, 4),
                                           "cache_resident": cache_resident(wv, st), "steps": steps,
                                           "launch": run_gpu.launch}

        for st in ("f64", "f32", "f16dev"):
            if st != args.storage:
                variant(w, st, 2000, 100)
        small = workloads.graphene_sample(1024, 512)
        for st in ("f64", "f32", "f16dev"):
            variant(small, st, 4000, 200)
        out["variants"] = extra
        print("variants done", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batch_256"] = batch_throughput(args.storage if args.storage != "f64" else "f32")
        print("batch done", file=sys.stderr, flush=True)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_throughput()
    if not args.no_warm_start and os.path.exists(WEIGHTS):
        out["time_to_steady"] = warm_vs_cold(WEIGHTS)
        print("time to steady done", file=sys.stderr, flush=True)
    if not args.no_precision:
        out["precision_vs_oracle"] = precision_vs_oracle(w)
        if args.long_run_steps > 0:
            out["precision_long_run"] = precision_long_run(w, args.long_run_steps)
        print("precision done", file=sys.stderr, flush=True)
    if args.cpu_steps > 0:
        out["cpu_baseline"], ref = cpu_baseline(w, args.cpu_steps)
        out["errors_vs_oracle"] = errors_vs_oracle(w, args.cpu_steps, ref)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--precision-report":
        sys.exit(main_precision(sys.argv[2:]))
    sys.exit(main())
