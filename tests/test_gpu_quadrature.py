"""A lattice running another member of the massless quadrature family
(rlbm_set_quadrature) against the FP64 oracle on the same quadrature, at
1e-12, and the library's refusal of tables that are not quadratures.  The
family member is the oracle's own (tests/golden/m0_family_member.txt)."""
import numpy as np
import pytest

from harness import field_errors, gpu_lattice, oracle_lattice
from paper_1804_02418_amd import workloads
from test_oracle_quadrature_search import read_family_member

pytestmark = pytest.mark.gpu


def test_family_member_matches_oracle():
    w = workloads.small_device(nx=120, ny=50, steps=40)
    w["quadrature"] = read_family_member()
    O = oracle_lattice(w)
    G = gpu_lattice(w, "f64")
    for t in (1, 10, 40):
        O.run(t - O.t)
        G.step(t - G.time)
        e = field_errors(G.read_fields(), O.fields())
        print("family member t", t, e, flush=True)
        assert e["err_n"] <= 1e-12 and e["err_u"] <= 1e-12 and e["err_eps"] <= 1e-12
    fo, fg = O.post_collision(), G.read_populations()
    assert np.abs(fg - fo).max() / np.abs(fo).max() <= 1e-12


def test_family_member_differs_from_default():
    w = workloads.small_device(nx=120, ny=50, steps=40)
    a = gpu_lattice(w)
    a.step(40)
    w["quadrature"] = read_family_member()
    b = gpu_lattice(w)
    b.step(40)
    assert np.abs(a.read_fields()["vx"] - b.read_fields()["vx"]).max() > 1e-9


def test_set_quadrature_rejects_non_quadratures():
    import paper_1804_02418_amd as rl

    w1, w2, p0 = read_family_member()
    L = rl.Lattice(16, 16, "f64")
    bad_p0 = list(p0)
    bad_p0[1] *= 1 + 1e-6
    for args in ((w1, w2, bad_p0), ([-w1[0]] + w1[1:], w2, p0), (w1, w2, [0.0] + p0[1:])):
        with pytest.raises(rl.RlbmError) as ei:
            L.set_quadrature(*args)
        assert ei.value.status == -1
    L.set_quadrature(w1, w2, p0)  # accepted
    L.close()
