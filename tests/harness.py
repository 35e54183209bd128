"""Test helpers: build the same workload on the oracle and on the GPU library
and compare their fields.  Inputs come only from paper_1804_02418_amd.workloads."""
from __future__ import annotations

import numpy as np


def oracle_lattice(w, use_printed=False):
    import oracle

    st = oracle.Stencil(shells=w["quadrature"]) if w.get("quadrature") is not None else oracle.stencil(use_printed)
    L = oracle.Lattice(st, w["nx"], w["ny"], periodic_x=w["periodic_x"],
                       periodic_y=w["periodic_y"], contacts=w["contacts"], solid=w.get("mask"), tau=w["tau"],
                       F=w["F"], cg=w.get("cg"))
    i = w["init"]
    L.init_fields(i["n"], i["T"], i["vx"], i["vy"])
    return L


def gpu_lattice(w, storage=None, shape=None, table=True):
    import paper_1804_02418_amd as rl

    L = rl.Lattice(w["nx"], w["ny"], storage or w.get("storage", "f64"))
    if not table:
        L.set_gather_table(False)
    if w.get("quadrature") is not None:
        L.set_quadrature(*w["quadrature"])
    L.set_boundaries(w["periodic_x"], w["periodic_y"], w["contacts"])
    if w.get("mask") is not None:
        L.set_mask(w["mask"])
    L.set_tau(w["tau"])
    L.set_drive(*w["F"])
    if w.get("cg") is not None:
        L.set_lca(w["cg"])
    if w.get("reference") is not None:
        L.set_reference(*w["reference"])
    i = w["init"]
    if all(np.isscalar(v) for v in i.values()):
        L.init_uniform(i["n"], i["T"], i["vx"], i["vy"])
    else:
        shp = (w["ny"], w["nx"])
        L.init_fields(*[np.broadcast_to(np.asarray(i[k], dtype=np.float64), shp) for k in ("n", "T", "vx", "vy")])
    return L


def field_errors(got, ref, vscale=None, mask=None):
    """Max-relative errors (S20 normalisation): err_n = max|n - n_ref| / |n_ref|;
    err_u = max|u - u_ref| / vscale (vscale = max|u_ref| unless given)."""
    sel = np.ones_like(ref["n"], dtype=bool) if mask is None else (np.asarray(mask) == 0)
    err_n = float(np.max(np.abs(got["n"][sel] - ref["n"][sel]) / np.abs(ref["n"][sel])))
    du = np.hypot(got["vx"] - ref["vx"], got["vy"] - ref["vy"])[sel]
    umax = float(np.max(np.hypot(ref["vx"], ref["vy"])[sel]))
    vs = umax if vscale is None else vscale
    err_u = float(np.max(du) / vs) if vs > 0 else float(np.max(du))
    err_eps = float(np.max(np.abs(got["eps"][sel] - ref["eps"][sel]) / np.abs(ref["eps"][sel])))
    return dict(err_n=err_n, err_u=err_u, err_eps=err_eps, umax=umax)
