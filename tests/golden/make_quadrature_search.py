"""Writes m5_quadrature.txt: the third-order quadrature of the 45-vector
stencil printed for mbar = 5 (Sec. 2.3, Fig. `stencil`, left), found by the
oracle alone.  The weights depend on v0; non-negative ones exist only in a
narrow window, and the file keeps the v0 that maximises the smallest weight
(golden-section search of the extended-precision solve over [0.2200, 0.2215]).

    python tests/golden/make_quadrature_search.py
"""
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import quadrature_search as Q  # noqa: E402


NL = chr(10)


def mp_str(v):
    import mpmath as mp

    return mp.nstr(v, 20)


def main():
    vec = Q.full_symmetric(Q.M5_ORBIT_REPS)

    def margin(v0):
        return min(Q.orbit_weights_mp(5.0, v0, vec)[1])

    a, b = 0.2200, 0.2215
    g = (math.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = margin(c), margin(d)
    for _ in range(80):
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = margin(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = margin(d)
    v0 = 0.5 * (a + b)
    orbs, w, res = Q.orbit_weights_mp(5.0, v0, vec)
    with open(os.path.join(HERE, "m5_quadrature.txt"), "w") as fh:
        fh.write("# Third-order quadrature of the mbar = 5 stencil of Sec. 2.3 (Fig. stencil, left),\n")
        fh.write("# 45 vectors in 10 (+-x,+-y)_FS orbits.  Written by make_quadrature_search.py\n")
        fh.write("# (oracle only).  Line 1: mbar, v0 maximising the smallest weight, that weight,\n")
        fh.write("# residual norm of the scaled monomial conditions of degree <= 6.  Then one line\n")
        fh.write("# per orbit: representative x y, orbit size, weight of each of its nodes.\n")
        fh.write(f"5.0 {v0!r} {min(w)!r} {res:.3e}\n")
        for orb, wk in zip(orbs, w):
            fh.write(f"{orb[0][0]} {orb[0][1]} {len(orb)} {wk!r}\n")
    print("v0", v0, "min weight", min(w), "residual", res)

    # another member of the massless family: the conditions solved from the
    # printed values with the fourth shell moved from 0.9358 to 1.0
    from oracle import quadrature as OQ

    start = list(OQ.PRINTED_W1 + OQ.PRINTED_W2 + OQ.PRINTED_P0)
    start[11] = "1.0"
    sol = OQ.solve_from(tuple(start))
    with open(os.path.join(HERE, "m0_family_member.txt"), "w") as fh:
        fh.write("# A second massless third-order quadrature on the 48-node stencil (Sec. 2.3):" + NL)
        fh.write("# the conditions solved (minimum-norm Gauss-Newton, 50 digits) from the printed" + NL)
        fh.write("# values with p0_4 = 1.0.  Written by make_quadrature_search.py (oracle only)." + NL)
        fh.write("# Rows: w1[4] (+-3,+-4)_FS, w2[4] (+-5,0)_FS, p0[4]; then the residual." + NL)
        for key in ("w1", "w2", "p0"):
            fh.write(" ".join(mp_str(v) for v in sol[key]) + NL)
        fh.write(f"{sol['residual']:.3e}" + NL)
    print("family member", [float(v) for v in sol["p0"]], "residual", sol["residual"])


if __name__ == "__main__":
    main()
