"""The injector validation of Sec. 3 (Eq. phi-approx-inlet, Fig. phi-inlet,
Fig. phi-vs-cg) on the GPU library, at 1000 x 400 (the 2000 x 500 runs are
the validation CLI's; both are in the design notes).

Physics bounds, not parity: the potential near a point injector follows
A cos(2 theta)/r^2 with A = 6 T0 nu Q / pi only between the kinetic layer
of the injector (r of a few mean free paths 5 tau) and the channel scale,
and the lattice's bounce-back walls slip by a few sites, which lowers A by
O(slip/r).  Measured at this size: ring amplitudes 3.43-3.88e-4 over
r = 60..100 (spread 12%), 0.85 of the analytic value, cos 2 theta misfit
2% and 1% at r = 80, 100; C_g = 10 moves the potential by 1.4% of its
largest value near the injector, C_g = 1e4 by 1.3e-5.  The bounds below
leave room around those values.  Also: the injector geometry (velocity
contact, full-edge drains, reference state n0 = 1.5, T0 = 1.25, C_g = 10)
against the FP64 oracle at 1e-12.
"""
import numpy as np
import pytest

from harness import field_errors, gpu_lattice, oracle_lattice
from paper_1804_02418_amd import validation as V
from paper_1804_02418_amd import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _steady(cg, tau=1.0):
    w = workloads.injector_setup(1000, 400, tau=tau, cg=cg)
    fields, steps, r, secs = V.run_to_steady(w, 100_000, tol=1e-9)
    _say(w["name"], "steps", steps, "residual", r, "seconds", round(secs, 2))
    assert r < 1e-9
    return w, fields


def test_injector_potential_follows_the_stokes_law():
    w, f = _steady(10.0)
    rep = V.analyse(w, f, [60, 80, 100])
    _say({k: v for k, v in rep.items() if k != "rings"}, rep["rings"])
    amps = np.array([g["A"] for g in rep["rings"]])
    assert (amps.max() - amps.min()) / amps.mean() < 0.2
    assert 0.75 < rep["A_mean_over_analytic"] < 1.0
    assert max(g["misfit"] for g in rep["rings"][1:]) < 0.05
    # incompressible near field: the same flux through every half circle
    q = [V.injected_flux(f, w["injector_centre"], r, w["reference"][0]) for r in (60, 80, 100)]
    assert max(q) / min(q) - 1 < 0.01, q


def test_potential_barely_depends_on_capacitance():
    phis, flux = {}, {}
    for cg in (10.0, 1e4, np.inf):
        w, f = _steady(cg)
        phis[cg] = V.potential(f, *w["reference"], cg)
        flux[cg] = V.injected_flux(f, w["injector_centre"], 80.0, w["reference"][0])
    rep = V.compare_potentials(phis, flux, w)
    _say(rep)
    assert rep["10.0"]["max_rel_diff"] < 0.03
    assert rep["10000.0"]["max_rel_diff"] < 1e-4


def test_injector_geometry_matches_oracle():
    w = workloads.injector_setup(120, 60, tau=0.9, cg=10.0, v_in=1e-2)
    O = oracle_lattice(w)
    G = gpu_lattice(w, "f64")
    for t in (1, 20, 150):
        O.run(t - O.t)
        G.step(t - G.time)
        e = field_errors(G.read_fields(), O.fields())
        _say("injector 120x60 t", t, e)
        assert e["err_n"] <= 1e-12 and e["err_u"] <= 1e-12 and e["err_eps"] <= 1e-12
