"""GPU tests of the residual (reading R14) and of the caller-owned device
field paths of the binding.

The residual over the last call of K steps is
    r = ||u(t) - u(t - K)||_2 / (K ||u(t)||_2)   over the fluid sites,
the quantity every time-to-steady figure stops at.  Here it is written out
with numpy from two field snapshots K steps apart -- taken from the library
itself (the reduction) and from the oracle (the whole chain) -- and compared
with rlbm_residual and rlbm_batch_residual.
"""
import numpy as np
import pytest

from harness import gpu_lattice, oracle_lattice
from paper_1804_02418_amd import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _r(a, b, K, mask=None):
    sel = np.ones_like(a["vx"], dtype=bool) if mask is None else (np.asarray(mask) == 0)
    du = np.hypot(b["vx"] - a["vx"], b["vy"] - a["vy"])[sel]
    u = np.hypot(b["vx"], b["vy"])[sel]
    return float(np.sqrt(np.sum(du * du)) / (K * np.sqrt(np.sum(u * u))))


def _masked_device():
    w = workloads.small_device(nx=130, ny=50, steps=60)
    mask = np.zeros((50, 130), dtype=np.uint8)
    mask[18:30, 40:47] = 1
    w["mask"] = mask
    return w


@pytest.mark.parametrize("case", ["device", "masked", "graphene"])
def test_residual_matches_numpy_and_oracle(case):
    if case == "device":
        w, t0, K = workloads.small_device(), 10, 25
    elif case == "masked":
        w, t0, K = _masked_device(), 7, 13
    else:
        w, t0, K = workloads.graphene_sample(storage="f64"), 40, 100
    G = gpu_lattice(w, "f64")
    G.step(t0)
    ga = G.read_fields()
    G.step(K)
    gb = G.read_fields()
    r_lib = G.residual()
    r_np = _r(ga, gb, K, w.get("mask"))
    O = oracle_lattice(w)
    O.run(t0)
    oa = O.fields()
    O.run(K)
    ob = O.fields()
    r_or = _r(oa, ob, K, w.get("mask"))
    G.close()
    _say(case, "r library", r_lib, "numpy on library fields", r_np, "numpy on oracle fields", r_or)
    assert r_lib == pytest.approx(r_np, rel=1e-12, abs=0)
    assert r_lib == pytest.approx(r_or, rel=1e-12, abs=0)


def test_batch_residual_matches_numpy_and_oracle():
    """A batch of three samples of different sizes and parameters: every
    sample's batched residual is the numpy residual of its own fields and of
    the oracle's."""
    import paper_1804_02418_amd as rl

    ws = []
    for k, (nx, ny) in enumerate([(96, 40), (150, 64), (70, 90)]):
        w = workloads.small_device(nx=nx, ny=ny, steps=1, seed=7 + k)
        w["contacts"] = w["contacts"][:3]
        w["tau"] = 0.7 + 0.2 * k
        w["F"] = (2e-4 * (k + 1), -3e-5 * k)
        w["init"] = dict(n=1.0 + 0.01 * k, T=1.0, vx=0.002 * k, vy=0.0)
        ws.append(w)
    B = rl.Batch(ws, "f64")
    t0, K = 9, 31
    B.step(t0)
    fa = [bl.read_fields() for bl in B.lattices]
    B.step(K)
    fb = [bl.read_fields() for bl in B.lattices]
    r = B.residual()
    for k, w in enumerate(ws):
        O = oracle_lattice(w)
        O.run(t0)
        oa = O.fields()
        O.run(K)
        r_or = _r(oa, O.fields(), K)
        r_np = _r(fa[k], fb[k], K)
        _say("sample", k, "batch", r[k], "numpy", r_np, "oracle", r_or)
        assert r[k] == pytest.approx(r_np, rel=1e-12, abs=0)
        assert r[k] == pytest.approx(r_or, rel=1e-12, abs=0)
    B.close()


def test_torch_device_field_paths_match_host_paths():
    """init_fields and read_fields_device with caller-owned torch tensors give
    what the host-array paths give; tensors of the wrong dtype, size or
    device are refused before the library sees them."""
    import torch

    w = workloads.small_device(nx=90, ny=40, steps=5)
    shp = (w["ny"], w["nx"])
    host = {k: np.ascontiguousarray(np.broadcast_to(np.asarray(w["init"][k], dtype=np.float64), shp))
            for k in ("n", "T", "vx", "vy")}
    A = gpu_lattice(w, "f64")          # host-array init
    B = gpu_lattice(w, "f64")
    dev = {k: torch.from_numpy(v.copy()).cuda() for k, v in host.items()}
    B.init_fields(dev["n"], dev["T"], dev["vx"], dev["vy"])
    del dev                            # the binding has finished with them
    torch.cuda.synchronize()
    for L in (A, B):
        L.step(5)
    assert np.array_equal(A.read_populations(), B.read_populations())
    ref = A.read_fields()
    outs = {k: torch.full(shp, -1.0, dtype=torch.float64, device="cuda") for k in ("n", "vx", "vy", "eps")}
    B.read_fields_device(outs["n"], outs["vx"], None, outs["eps"])
    for k in ("n", "vx", "eps"):
        assert np.array_equal(outs[k].cpu().numpy(), ref[k]), k
    assert bool((outs["vy"] == -1.0).all())
    bad = [torch.zeros(shp, dtype=torch.float32, device="cuda"),
           torch.zeros((shp[0], shp[1] - 1), dtype=torch.float64, device="cuda"),
           torch.zeros(shp, dtype=torch.float64),
           torch.zeros((shp[1], 2 * shp[0]), dtype=torch.float64, device="cuda")[:, ::2]]
    ok = torch.ones(shp, dtype=torch.float64, device="cuda")
    for t in bad:
        with pytest.raises(ValueError):
            B.read_fields_device(t, None, None, None)
        with pytest.raises(ValueError):
            B.init_fields(t, ok, ok, ok)
    A.close()
    B.close()
