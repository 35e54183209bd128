"""GPU tests of the reduced-precision storages and of the launch autotuner.

FP32 and FP16-deviation storage run the same geometry as the FP64 path,
which is itself held to the FP64 oracle at 1e-12 (test_gpu_parity.py); their
max-relative errors in n and u are printed and bounded.  Bounds follow from
the storage rounding: every step re-rounds each stored deviation
eta_i = (f_i - f_ref_i)/(w_i * scale) to 2^-24 (FP32) or 2^-11 (FP16)
relative, the arithmetic on it is FP32 (2^-24), and the moments go to the
Landau solve in FP64, so the per-step error is a few units of that rounding
of the deviation; over the run it accumulates like a random walk that the
collision damps.  The bench configuration (1024 x 512 FP32) is also checked
one step at a time against the oracle at every site.
"""
import numpy as np
import pytest

from harness import field_errors, gpu_lattice, oracle_lattice
from paper_1804_02418_amd import workloads

pytestmark = pytest.mark.gpu


def _small_sample():
    w = workloads.graphene_sample(256, 128)
    w["contacts"] = workloads._contact_pair(256, 16, 96)
    return w


@pytest.mark.parametrize("storage,tol_n,tol_u", [("f32", 2e-7, 2e-4), ("f16dev", 2e-5, 5e-2)])
def test_reduced_storage_error_against_fp64(storage, tol_n, tol_u):
    w = _small_sample()
    ref = gpu_lattice(w, "f64")
    G = gpu_lattice(w, storage)
    for t in (1, 100, 3000):
        ref.step(t - ref.time)
        G.step(t - G.time)
        e = field_errors(G.read_fields(), ref.read_fields())
        print(storage, "t", t, e, flush=True)
    assert e["err_n"] <= tol_n and e["err_u"] <= tol_u, e


def test_bench_configuration_one_step_against_oracle():
    """1024 x 512 graphene sample, FP32 storage, the launch shape bench.py
    uses: after 500 GPU steps, the oracle (FP64) streams and collides the
    decoded GPU state; the GPU's FP32 step must agree at every site to the
    FP32 rounding of the deviations."""
    import oracle

    w = workloads.graphene_sample()
    G = gpu_lattice(w, "f32")
    G.step(500)
    fstar = G.read_populations()
    G.step(1)
    got = G.read_fields()
    got_f = G.read_populations()
    O = oracle_lattice(w)
    fpre = np.empty_like(fstar)
    oracle.lib().orc_lattice_stream(O._h, oracle._ptr(np.ascontiguousarray(fstar)), oracle._ptr(fpre))
    O.f[...] = fpre
    ref = O.fields()
    exp_f = O.post_collision()
    e = field_errors(got, ref)
    # population error relative to the deviation scale (the stored quantity)
    wfull = np.array(oracle.stencil().w)[:, None, None]
    dev = np.abs(exp_f - wfull).max()
    perr = np.abs(got_f - exp_f).max() / dev
    print("f32 one step", e, "populations / max deviation", perr, flush=True)
    assert e["err_n"] <= 1e-9 and e["err_u"] <= 1e-5 and perr <= 1e-5


@pytest.mark.parametrize("storage,tol_f", [("f64", 1e-12), ("f32", 1e-5), ("f16dev", 1e-3)])
def test_large_sample_one_step_against_oracle(storage, tol_f):
    """4096 x 2048 graphene sample (contacts 128 wide, 512 from the centre) in
    the launch configuration the autotuner picks at that size (row tiles of
    256 sites, streaming stores): after 200 GPU steps, the oracle (FP64)
    streams and collides the decoded GPU state, and the GPU's next step must
    agree at every site.  FP64 to the parity bound; FP32 and FP16 deviations
    to the rounding of the stored deviation (2^-24 and 2^-11 of it: bounds
    1e-5 and 1e-3 of the largest deviation), their fields (FP32 moment sums
    of the same decoded values, FP64 Landau solve) as in the 1024 x 512
    check."""
    import oracle

    w = workloads.graphene_sample(4096, 2048)
    G = gpu_lattice(w, storage)
    G.set_launch_shape(256, 1)
    G.set_streaming_stores(True)
    G.step(200)
    fstar = G.read_populations()
    G.step(1)
    got = G.read_fields()
    got_f = G.read_populations()
    G.close()
    O = oracle_lattice(w)
    fpre = np.empty_like(fstar)
    oracle.lib().orc_lattice_stream(O._h, oracle._ptr(np.ascontiguousarray(fstar)), oracle._ptr(fpre))
    del fstar
    O.f = fpre
    ref = O.fields()
    exp_f = O.post_collision()
    e = field_errors(got, ref)
    if storage == "f64":
        perr = np.abs(got_f - exp_f).max() / np.abs(exp_f).max()
        bound_n = bound_u = 1e-12
    else:
        wfull = np.array(oracle.stencil().w)[:, None, None]
        perr = np.abs(got_f - exp_f).max() / np.abs(exp_f - wfull).max()
        bound_n, bound_u = 1e-9, 1e-5
    print(storage, "4096x2048 one step", e, "populations", perr, flush=True)
    assert e["err_n"] <= bound_n and e["err_u"] <= bound_u and perr <= tol_f, (e, perr)


def test_autotune_keeps_state_and_results():
    w = workloads.small_device(nx=300, ny=60, steps=5)
    a = gpu_lattice(w, "f32")
    a.step(3)
    b = gpu_lattice(w, "f32")
    b.step(3)
    ms = b.autotune(5)
    print("autotune ms/step (64, 128, 256):", ms, flush=True)
    assert b.time == 3 and (ms > 0).any()
    fa, fb = a.read_fields(), b.read_fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k])
    a.step(4)
    b.step(4)
    assert np.array_equal(a.read_populations(), b.read_populations())
