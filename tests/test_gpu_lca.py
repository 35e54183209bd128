"""GPU parity of the local-capacitance force (Sec. 3, Eq. lca) against the
FP64 oracle, through the C ABI.

The force -(1/C_g) grad n of the previous density is on at the paper's
coupling C_g = 10 and at C_g = 2, close to the strongest at which the lagged
term stays stable on these devices (at C_g = 0.5 the oracle itself loses its
Landau frame within 40 steps on the ragged device), on the ragged device (walls, contacts on three edges, drive), on a masked
obstacle (solid neighbours), on tiny periodic lattices (wrapping
neighbours) and with FP32 storage; FP64 must match to 1e-12 element by
element, populations included.  Also: checkpoints carry the previous
density, the term cannot ride in a batch, and C_g = infinity is the plain
kernel bit for bit.
"""
import numpy as np
import pytest

from harness import field_errors, gpu_lattice, oracle_lattice
from paper_1804_02418_amd import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)


def _compare(w, checkpoints, storage="f64", tol=(TOL, TOL), pops=True):
    O = oracle_lattice(w)
    G = gpu_lattice(w, storage)
    vs = None
    for t in checkpoints:
        O.run(t - O.t)
        G.step(t - G.time)
        ref = O.fields()
        got = G.read_fields()
        if vs is None:
            vs = float(np.max(np.hypot(ref["vx"], ref["vy"]))) or 1.0
        e = field_errors(got, ref, vscale=vs, mask=w.get("mask"))
        _say(w["name"], storage, "cg", w["cg"], "t", t, e)
        assert e["err_n"] <= tol[0] and e["err_u"] <= tol[1] and e["err_eps"] <= tol[0], (t, e)
    if pops:
        fo = O.post_collision()
        fg = G.read_populations()
        sel = np.ones((w["ny"], w["nx"]), dtype=bool) if w.get("mask") is None else (w["mask"] == 0)
        err = np.abs(fg[:, sel] - fo[:, sel]).max() / np.abs(fo[:, sel]).max()
        _say(w["name"], "populations rel err", err)
        assert err <= tol[0]
    G.close()


@pytest.mark.parametrize("cg", [2.0, 10.0])
def test_small_device_with_lca_matches_oracle(cg):
    w = workloads.small_device()
    w["cg"] = cg
    _compare(w, [0, 1, 2, 5, 40, 120])


def test_lca_changes_the_flow():
    """The term is not a no-op at this coupling (guards a silently ignored flag)."""
    w = workloads.small_device(steps=40)
    a = gpu_lattice(w)
    a.step(40)
    w["cg"] = 2.0
    b = gpu_lattice(w)
    b.step(40)
    fa, fb = a.read_fields(), b.read_fields()
    assert np.abs(fa["n"] - fb["n"]).max() > 1e-4


def test_masked_obstacle_with_lca_matches_oracle():
    w = workloads.small_device(nx=130, ny=50, steps=60)
    w["periodic_x"] = True
    w["contacts"] = [c for c in w["contacts"] if c["edge"] in ("bottom", "top")]
    mask = np.zeros((50, 130), dtype=np.uint8)
    mask[18:30, 40:47] = 1
    mask[5:9, 100:128] = 1
    w["mask"] = mask
    w["cg"] = 2.0
    _compare(w, [0, 1, 3, 60])


@pytest.mark.parametrize("nx,ny", [(1, 6), (3, 7), (70, 3)])
def test_tiny_periodic_lattices_with_lca_match_oracle(nx, ny):
    w = workloads.small_device(nx=nx, ny=ny, steps=10)
    w.update(periodic_x=True, periodic_y=True, contacts=[], cg=2.0)
    _compare(w, [0, 1, 10])


def test_fp32_storage_with_lca():
    w = workloads.small_device(steps=120)
    w["cg"] = 2.0
    _compare(w, [1, 120], storage="f32", tol=(2e-7, 2e-4), pops=False)


def test_fp16_storage_with_lca():
    """FP16 deviation storage (four-shell tuples) with the local-capacitance
    force, against the FP64 oracle: the bounds of the reduced-storage test
    in test_gpu_precision.py, set by the float16 rounding of the stored
    deviation."""
    w = workloads.small_device(steps=120)
    w["cg"] = 2.0
    _compare(w, [1, 120], storage="f16dev", tol=(2e-5, 5e-2), pops=False)


def test_infinite_capacitance_is_plain_kernel():
    w = workloads.small_device(nx=96, ny=40, steps=20)
    a = gpu_lattice(w)
    a.step(20)
    w["cg"] = np.inf
    b = gpu_lattice(w)
    b.step(20)
    assert np.array_equal(a.read_populations(), b.read_populations())


def test_checkpoint_with_lca_is_bit_identical():
    w = workloads.small_device(nx=96, ny=40, steps=20)
    w["cg"] = 2.0
    G = gpu_lattice(w)
    G.step(7)
    blob = G.get_state()
    G.step(13)
    a = G.read_populations()
    H = gpu_lattice(w)
    H.set_state(blob)
    H.step(13)
    assert np.array_equal(a, H.read_populations())


def test_lca_errors():
    import paper_1804_02418_amd as rl

    w = workloads.small_device(nx=64, ny=16, steps=4)
    G = gpu_lattice(w)
    for bad in (-1.0, np.nan):
        with pytest.raises(rl.RlbmError) as ei:
            rl.check(rl.lib().rlbm_set_lca(G._h, float(bad)))
        assert ei.value.status == -1
    blob = G.get_state()
    G.set_lca(2.0)
    with pytest.raises(rl.RlbmError):
        G.set_state(blob)  # saved without the term
    # a batch refuses a sample with the term on
    bt = rl.Batch(workloads.batch_samples(2, fixed_size=(128, 128)), "f64")
    bt.lattices[0].set_lca(10.0)
    with pytest.raises(rl.RlbmError):
        bt.step(2)
    bt.close()
