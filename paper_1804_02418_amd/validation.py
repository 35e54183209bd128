"""The paper's validation of the solver near a current injector (Sec. 3,
Eq. phi-approx-inlet, Fig. phi-inlet) and its C_g sweep (Fig. phi-vs-cg).

    python -m paper_1804_02418_amd.validation --tau 0.8 1.0 1.2 --cg 10
    python -m paper_1804_02418_amd.validation --tau 1.0 --cg-sweep 10 1e4 inf

Every run steps the injector channel (``workloads.injector_setup``) to a
steady state on the GPU library and analyses its fields here on the host.

Electrochemical potential.  With the local-capacitance force, the force
per carrier is -(c grad P)/n - (1/C_g) grad n (pressure P = eps/2 of the
massless gas, c = 5 sites/step converting the pressure gradient per site to
a force per step, e = 1).  Linearised about (n0, T0) it is -grad Phi with

    Phi = c (P - P0) / n0 + (n - n0) / C_g .

The steady slow flow obeys Stokes' equations n0 grad Phi = eta lap(beta)
with eta = 3 n0 T0 nu (enthalpy 3 n T, nu = 6.25 (tau - 1/2)
sites^2/step, beta = v/c), so a point injector of flux Q = v_in w_in into a
half plane gives

    Phi(r, theta) = A cos(2 theta) / r^2,   A = 6 T0 nu Q / pi,

theta measured from the injection direction: the form of Eq.
phi-approx-inlet with I = e n0 Q and the shear viscosity of the lattice.
In the finite channel Phi also carries the slowly varying potential of the
current flowing to the drains; on each ring it is close to a constant plus
a uniform gradient, which the ring fit of ``collapse`` takes out before
r^2 Phi is compared across rings.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

C_LATTICE = 5.0  # sites per step


def run_to_steady(w, max_steps=None, check_every=1000, tol=1e-9, stream=None):
    """Build the lattice of workload `w`, step it until the velocity residual
    over `check_every` steps drops below tol; returns (fields, steps, r, s)."""
    from . import _binding as B

    L = B.Lattice(w["nx"], w["ny"], w.get("storage", "f64"), stream=stream)
    L.set_boundaries(w["periodic_x"], w["periodic_y"], w["contacts"])
    L.set_tau(w["tau"])
    L.set_drive(*w["F"])
    if w.get("cg") is not None:
        L.set_lca(w["cg"])
    if w.get("reference") is not None:
        L.set_reference(*w["reference"])
    i = w["init"]
    L.init_uniform(i["n"], i["T"], i["vx"], i["vy"])
    t0 = time.perf_counter()
    steps, r = L.step_until(max_steps or w["steps"], check_every, tol)
    fields = L.read_fields()
    secs = time.perf_counter() - t0
    L.close()
    return fields, steps, r, secs


def potential(fields, n0, T0, cg):
    """Electrochemical potential Phi per carrier (module notes)."""
    P = 0.5 * fields["eps"]
    phi = C_LATTICE * (P - n0 * T0) / n0
    if cg is not None and np.isfinite(cg):
        phi = phi + (fields["n"] - n0) / cg
    return phi


def bilinear(a, x, y):
    """a[y, x] at fractional points (x, y) inside the lattice."""
    x0 = np.floor(x).astype(int)
    y0 = np.floor(y).astype(int)
    fx, fy = x - x0, y - y0
    x1 = np.minimum(x0 + 1, a.shape[1] - 1)
    y1 = np.minimum(y0 + 1, a.shape[0] - 1)
    return ((1 - fy) * ((1 - fx) * a[y0, x0] + fx * a[y0, x1]) + fy * ((1 - fx) * a[y1, x0] + fx * a[y1, x1]))


def ring_points(centre, r, thetas):
    """Points at distance r from the injector, theta from the inward normal (+y)."""
    return centre[0] + r * np.sin(thetas), centre[1] + r * np.cos(thetas)


def collapse(phi, centre, radii, n_theta=61, theta_max=np.radians(75.0)):
    """Per ring r: least-squares fit of r^2 Phi(r, theta) on the arc
    |theta| <= theta_max by A_r cos 2 theta + B_r + C_r cos theta +
    D_r sin theta.  B, C, D absorb the smooth potential of the current on
    its way to the drains (constant and uniform-gradient terms on the
    ring); A_r is the injector's amplitude, constant in r if Phi falls as
    1/r^2.  misfit: rms of what the fit leaves, relative to |A_r|."""
    th = np.linspace(-theta_max, theta_max, n_theta)
    M = np.stack([np.cos(2 * th), np.ones_like(th), np.cos(th), np.sin(th)], axis=1)
    out = []
    for r in radii:
        x, y = ring_points(centre, r, th)
        v = bilinear(phi, x, y) * r * r
        coef, *_ = np.linalg.lstsq(M, v, rcond=None)
        A = float(coef[0])
        mis = float(np.sqrt(((v - M @ coef) ** 2).mean()) / abs(A)) if A != 0 else float("inf")
        out.append({"r": float(r), "A": A, "misfit": mis})
    return out


def injected_flux(fields, centre, r, n0, n_theta=181):
    """Flux of beta = v/c through the half circle of radius r around the
    injector, weighted by n / n0 (number flux over n0)."""
    th = np.linspace(-np.pi / 2, np.pi / 2, n_theta)
    x, y = ring_points(centre, r, th)
    inside = y >= 0
    vx = bilinear(fields["vx"], x[inside], np.maximum(y[inside], 0))
    vy = bilinear(fields["vy"], x[inside], np.maximum(y[inside], 0))
    nn = bilinear(fields["n"], x[inside], np.maximum(y[inside], 0)) / n0
    vr = nn * (vx * np.sin(th[inside]) + vy * np.cos(th[inside]))
    return float(np.trapezoid(vr, th[inside]) * r)


def analyse(w, fields, radii):
    n0, T0 = w["reference"]
    nu = 6.25 * (w["tau"] - 0.5)
    phi = potential(fields, n0, T0, w.get("cg"))
    rings = collapse(phi, w["injector_centre"], radii)
    q_nominal = w["v_in"] * w["w_in"]
    q_meas = injected_flux(fields, w["injector_centre"], float(np.median(radii)), n0)
    A_nom = 6.0 * T0 * nu * q_nominal / np.pi
    A_meas = 6.0 * T0 * nu * q_meas / np.pi
    amps = np.array([g["A"] for g in rings])
    return {
        "rings": rings,
        "A_analytic_nominal_flux": A_nom,
        "A_analytic_measured_flux": A_meas,
        "flux_nominal": q_nominal,
        "flux_measured": q_meas,
        "collapse_spread": float((amps.max() - amps.min()) / abs(amps.mean())),
        "A_mean_over_analytic": float(amps.mean() / A_meas),
        "max_misfit": float(max(g["misfit"] for g in rings)),
    }


def compare_potentials(phis, fluxes, w, half_window=200):
    """Max difference of each run's potential from the last run's over the
    injector's neighbourhood (|x - x_c| < half_window, y < half_window, the
    injector's own 10 rows left out), relative to the last run's largest
    value there; also after dividing each potential by its run's measured
    flux (the potential per unit injected current)."""
    keys = list(phis)
    ref_k = keys[-1]
    cx = int(round(w["injector_centre"][0]))
    win = (slice(10, min(w["ny"], half_window)), slice(max(0, cx - half_window), min(w["nx"], cx + half_window)))
    ref = phis[ref_k][win]
    refq = ref / fluxes[ref_k]
    out = {}
    for k in keys[:-1]:
        d = phis[k][win]
        out[str(k)] = {"vs": str(ref_k), "max_rel_diff": float(np.abs(d - ref).max() / np.abs(ref).max()),
                       "max_rel_diff_per_flux": float(np.abs(d / fluxes[k] - refq).max() / np.abs(refq).max()),
                       "flux_ratio": float(fluxes[k] / fluxes[ref_k])}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nx", type=int, default=2000)
    ap.add_argument("--ny", type=int, default=500)
    ap.add_argument("--w-in", type=int, default=8)
    ap.add_argument("--tau", type=float, nargs="+", default=[0.8, 1.0, 1.2])
    ap.add_argument("--cg", type=float, default=10.0)
    ap.add_argument("--cg-sweep", type=float, nargs="*", default=None,
                    help="run the first tau at these C_g (inf allowed) and compare their potentials")
    ap.add_argument("--storage", default="f64", choices=["f64", "f32", "f16dev"])
    ap.add_argument("--max-steps", type=int, default=400_000)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--radii", type=float, nargs="+", default=[40, 60, 80, 100, 120])
    ap.add_argument("--out", default="")
    ap.add_argument("--save-fields", default="",
                    help="npz prefix: write each run's fields as float32 deviations dn, deps and vx, vy")
    args = ap.parse_args(argv)

    import torch  # noqa: F401  (loads the HIP runtime the library shares)

    from . import workloads

    report = {"runs": []}
    cgs = args.cg_sweep if args.cg_sweep else [args.cg]
    taus = args.tau[:1] if args.cg_sweep else args.tau
    phis = {}
    for tau in taus:
        for cg in cgs:
            w = workloads.injector_setup(args.nx, args.ny, tau=tau, cg=cg, w_in=args.w_in, storage=args.storage)
            fields, steps, r, secs = run_to_steady(w, args.max_steps, tol=args.tol)
            rec = {"workload": w["name"], "tau": tau, "cg": cg, "steps": int(steps), "residual": r,
                   "seconds": round(secs, 2)}
            rec.update(analyse(w, fields, args.radii))
            report["runs"].append(rec)
            print(json.dumps(rec), flush=True)
            phis[cg] = potential(fields, *w["reference"], cg)
            if args.save_fields:
                n0, T0 = w["reference"]
                np.savez(f"{args.save_fields}_{w['name']}.npz", dn=(fields["n"] - n0).astype(np.float32),
                         deps=(fields["eps"] - 2 * n0 * T0).astype(np.float32),
                         vx=fields["vx"].astype(np.float32), vy=fields["vy"].astype(np.float32))
    if args.cg_sweep and len(cgs) > 1:
        report["cg_sweep"] = compare_potentials(phis, {r["cg"]: r["flux_measured"] for r in report["runs"]},
                                                workloads.injector_setup(args.nx, args.ny, w_in=args.w_in))
        print(json.dumps({"cg_sweep": report["cg_sweep"]}), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
