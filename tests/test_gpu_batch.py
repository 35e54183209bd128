"""GPU tests of the batched launch (all samples in one launch per step).

Every sample of a batch must evolve bit-identically to the same lattice
stepped alone (the step of a site is a pure function of the previous state,
whatever block or launch computes it), through eager launches and through
graph replays; frozen samples must not change; the batched residual must
equal the single-lattice residual; the batch autotuner must leave every
state as it found it.
"""
import numpy as np
import pytest

from harness import field_errors, gpu_lattice, oracle_lattice
from paper_1804_02418_amd import workloads

pytestmark = pytest.mark.gpu


def _samples():
    out = []
    for k, (nx, ny) in enumerate([(64, 48), (200, 90), (128, 128), (75, 31), (320, 64), (9, 40)]):
        w = workloads.small_device(nx=nx, ny=ny, steps=1)
        w["contacts"] = w["contacts"][:3]
        w["tau"] = 0.6 + 0.15 * k
        w["F"] = (1e-4 * (k + 1), -2e-5 * k)
        w["init"] = dict(n=1.0 + 0.01 * k, T=1.0 - 0.01 * k, vx=0.001 * k, vy=0.0)
        if k == 2:
            w.update(periodic_x=True, periodic_y=True, contacts=[])
        if k == 5:
            w.update(periodic_x=True, contacts=[c for c in w["contacts"] if c["edge"] != "left"])
        out.append(w)
    return out


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("xcd", [False, True])
def test_batch_matches_single_lattices(storage, graph, xcd):
    """Also across block orders: the batch in one, the single lattices in the other."""
    import paper_1804_02418_amd as rl

    ws = _samples()
    B = rl.Batch(ws, storage)
    B.set_block_order(xcd)
    singles = [gpu_lattice(w, storage) for w in ws]
    for L in singles:
        L.set_block_order(not xcd)
    for n in (1, 70):
        B.step(n, graph=graph)
        for L in singles:
            L.step(n)
    for k, (L, bl) in enumerate(zip(singles, B.lattices)):
        assert bl.time == L.time == 71
        assert np.array_equal(bl.read_populations(), L.read_populations()), k
        fa, fb = bl.read_fields(), L.read_fields()
        for key in fa:
            assert np.array_equal(fa[key], fb[key]), (k, key)
    r = B.residual()
    for k, L in enumerate(singles):
        assert r[k] == pytest.approx(L.residual(), rel=1e-12, abs=0)
    print(storage, "graph" if graph else "eager", "sites", B.sites(), "residuals", r, flush=True)
    B.close()


def test_frozen_samples_keep_their_state():
    import paper_1804_02418_amd as rl

    ws = _samples()
    B = rl.Batch(ws, "f64")
    B.step(5)
    before = [bl.read_populations() for bl in B.lattices]
    active = np.ones(len(ws), dtype=np.uint8)
    active[[1, 4]] = 0
    B.set_active(active)
    B.step(40)
    for k, bl in enumerate(B.lattices):
        if active[k]:
            assert bl.time == 45 and not np.array_equal(bl.read_populations(), before[k])
        else:
            assert bl.time == 5 and np.array_equal(bl.read_populations(), before[k])
    # reactivated samples continue exactly as if never frozen
    B.set_active(np.ones(len(ws), dtype=np.uint8))
    B.step(3)
    ref = gpu_lattice(ws[1], "f64")
    ref.step(8)
    assert np.array_equal(B.lattices[1].read_populations(), ref.read_populations())


def test_batch_autotune_restores_state():
    import paper_1804_02418_amd as rl

    ws = _samples()
    B = rl.Batch(ws, "f32")
    B.step(4)
    snap = [bl.read_populations() for bl in B.lattices]
    ms = B.autotune(3)
    print("batch autotune ms/step", ms, [bl.launch_shape() for bl in B.lattices], flush=True)
    assert (ms > 0).all()
    # the chosen decomposition is a valid one for every sample
    for bl in B.lattices:
        t, r = bl.launch_shape()
        assert t in (64, 128, 256) and t * r == 256
    for k, bl in enumerate(B.lattices):
        assert bl.time == 4 and np.array_equal(bl.read_populations(), snap[k])
    B.step(6)
    single = gpu_lattice(ws[3], "f32")
    single.step(10)
    assert np.array_equal(B.lattices[3].read_populations(), single.read_populations())


def test_batch_step_until_freezes_converged_samples():
    import paper_1804_02418_amd as rl

    ws = _samples()[:3]
    B = rl.Batch(ws, "f64")
    steps, r = B.step_until(400, 50, 1e-3)
    print("step_until steps", steps, "r", r, flush=True)
    assert ((r < 1e-3) | (steps == 400)).all()
    for k, bl in enumerate(B.lattices):
        assert bl.time == steps[k]


def test_full_batch_sampled_samples_against_oracle():
    """The 256-sample uneven batch (about 50 M sites, FP32) as the bench runs
    it (batch autotuner, graph replays of the step): after 40 steps, samples
    of the extreme and awkward shapes (fewest and most sites, widths 128 and
    192, height 128, widths that are not a multiple of 256) are each checked
    for one step at every site against the oracle (FP64) applied to the
    decoded GPU state, to the FP32 rounding of the stored deviations."""
    import oracle
    import paper_1804_02418_amd as rl

    ws = workloads.batch_samples(256)
    sites = [w["nx"] * w["ny"] for w in ws]
    pick = {int(np.argmin(sites)), int(np.argmax(sites))}
    for cond in (lambda w: w["nx"] == 128, lambda w: w["nx"] == 192, lambda w: w["ny"] == 128,
                 lambda w: w["nx"] % 256 == 64 and w["nx"] > 256):
        pick.add(next(k for k, w in enumerate(ws) if cond(w)))
    B = rl.Batch(ws, "f32")
    B.autotune(5)
    B.step(40, graph=True)
    fstar = {k: B.lattices[k].read_populations() for k in sorted(pick)}
    B.step(1, graph=True)
    wfull = np.array(oracle.stencil().w)[:, None, None]
    for k in sorted(pick):
        got = B.lattices[k].read_fields()
        got_f = B.lattices[k].read_populations()
        O = oracle_lattice(ws[k])
        fpre = np.empty_like(fstar[k])
        oracle.lib().orc_lattice_stream(O._h, oracle._ptr(np.ascontiguousarray(fstar[k])), oracle._ptr(fpre))
        O.f = fpre
        ref = O.fields()
        exp_f = O.post_collision()
        e = field_errors(got, ref)
        perr = np.abs(got_f - exp_f).max() / np.abs(exp_f - wfull).max()
        print("batch sample", k, (ws[k]["nx"], ws[k]["ny"]), e, "populations", perr, flush=True)
        assert e["err_n"] <= 1e-9 and e["err_u"] <= 1e-5 and perr <= 1e-5, (k, e, perr)
    B.close()


def test_degenerate_batches_and_zero_steps():
    """Zero steps change nothing (single lattice and batch); a batch whose
    samples are all frozen launches nothing and changes nothing; a batch of
    one sample is the single lattice bit for bit."""
    import paper_1804_02418_amd as rl

    ws = _samples()
    L = gpu_lattice(ws[1], "f32")
    L.step(3)
    f0 = L.read_populations()
    L.step(0)
    assert L.time == 3 and np.array_equal(L.read_populations(), f0)

    B = rl.Batch(ws, "f32")
    B.step(2)
    snap = [bl.read_populations() for bl in B.lattices]
    B.step(0)
    B.set_active(np.zeros(len(ws), dtype=np.uint8))
    B.step(5)
    for k, bl in enumerate(B.lattices):
        assert bl.time == 2 and np.array_equal(bl.read_populations(), snap[k]), k
    B.close()

    one = rl.Batch(ws[3:4], "f64")
    one.step(40, graph=True)
    ref = gpu_lattice(ws[3], "f64")
    ref.step(40)
    assert np.array_equal(one.lattices[0].read_populations(), ref.read_populations())
    one.close()
