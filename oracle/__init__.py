"""FP64 CPU oracle of the (2+1)-D relativistic lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  The GPU library never calls it, and the two share no code:
the oracle has its own quadrature polish (``quadrature.py``), its own
Appendix A transcription and force matrices (``appendix.py``) and its own
plain-C step (``rlbm_oracle.c``).

Every function is pinned by a ``-m "not gpu"`` test against something the
paper or the mathematics fixes (printed weights, exact continuum moments,
orthonormality, closed-form Maxwell-Juttner moments, conservation laws,
LAPACK eigenvectors, the shear viscosity).  One part is "parity unpinned":
the higher (non-conserved) moments of the forcing term, which no closed form
fixes; only its number, energy and momentum sources are pinned.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

from . import appendix, quadrature

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rlbm_oracle.c")
_LIB = os.path.join(_HERE, "librlbm_oracle.so")
# The same source built with long double arithmetic and state (-DORC_LONG_DOUBLE):
# the same discrete problem with about 2^-11 of the rounding error, used to
# measure the rounding floor of the float64 build.
_LIB_LD = os.path.join(_HERE, "librlbm_oracle_ld.so")

Q = quadrature.Q
K = 16


def build(force: bool = True, long_double: bool = False) -> str:
    """Compile the plain-C oracle (gcc, -O2, OpenMP).  Returns the .so path."""
    out = _LIB_LD if long_double else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                        *(["-DORC_LONG_DOUBLE"] if long_double else []), "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, out)
    return out


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_ldp = ctypes.POINTER(ctypes.c_longdouble)


@functools.lru_cache(maxsize=2)
def lib(long_double: bool = False) -> ctypes.CDLL:
    path = build(force=False, long_double=long_double)
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    rp = _ldp if long_double else _dp          # pointer to the arithmetic type
    rv = ctypes.c_longdouble if long_double else ctypes.c_double
    L.orc_real_bytes.restype = ctypes.c_int
    if L.orc_real_bytes() != ctypes.sizeof(rv):
        raise RuntimeError(f"{path}: built for another arithmetic type")
    L.orc_stencil_new.restype = vp
    L.orc_stencil_new.argtypes = [_dp, _dp, _dp, _dp, _ip, _ip, _ip, _dp, _dp, _dp]
    L.orc_stencil_free.argtypes = [vp]
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = None
    L.orc_get_threads.argtypes = []
    L.orc_get_threads.restype = ctypes.c_int
    L.orc_projections.argtypes = [rv, rv, rp, rp]
    L.orc_moments.argtypes = [vp, rp, rp, rp]
    L.orc_landau.argtypes = [rp, rp, rp]
    L.orc_landau.restype = ctypes.c_int
    L.orc_macro.argtypes = [vp, rp, rp, rp, rp, rp]
    L.orc_macro.restype = ctypes.c_int
    L.orc_feq.argtypes = [vp, rv, rv, rp, rp]
    L.orc_force_term.argtypes = [vp, rv, rv, rp, rv, rv, rp]
    L.orc_collide.argtypes = [vp, rp, rv, rv, rv, rp]
    L.orc_collide.restype = ctypes.c_int
    L.orc_lattice_new.restype = vp
    L.orc_lattice_new.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, _ip, _ip, _ip, _dp, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.orc_lattice_free.argtypes = [vp]
    L.orc_lattice_collide.argtypes = [vp, rp, rp]
    L.orc_lattice_collide.restype = ctypes.c_int
    L.orc_lattice_stream.argtypes = [vp, rp, rp]
    L.orc_lattice_run.argtypes = [vp, rp, ctypes.c_int64]
    L.orc_lattice_run.restype = ctypes.c_int
    L.orc_lattice_fields.argtypes = [vp, rp, rp, rp, rp, rp, rp]
    L.orc_lattice_fields.restype = ctypes.c_int
    L.orc_lattice_init.argtypes = [vp, _dp, _dp, _dp, _dp, rp]
    L.orc_lattice_set_lca.argtypes = [vp, ctypes.c_double]
    return L


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _rptr(a: np.ndarray):
    """Pointer to a float64 or long double array (the arithmetic type of a build)."""
    assert a.flags.c_contiguous
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    assert a.dtype == np.longdouble
    return a.ctypes.data_as(_ldp)


def _iptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


class Stencil:
    """The 48-node quadrature with its Appendix A table and force matrices.

    long_double: use the long double build of the oracle (state, fields and
    per-site arguments are numpy.longdouble arrays) on the same float64
    constants."""

    def __init__(self, use_printed: bool = False, shells=None, long_double: bool = False):
        nodes = quadrature.node_table(use_printed, shells)
        self.nodes = nodes
        self.long_double = bool(long_double)
        self.real = np.longdouble if long_double else np.float64
        self._lib = lib(self.long_double)
        self.w = np.array(nodes["w"], dtype=np.float64)
        self.p0 = np.array(nodes["p0"], dtype=np.float64)
        self.px = np.array(nodes["px"], dtype=np.float64)
        self.py = np.array(nodes["py"], dtype=np.float64)
        self.cx = np.array(nodes["cx"], dtype=np.int32)
        self.cy = np.array(nodes["cy"], dtype=np.int32)
        self.opp = np.array(nodes["opp"], dtype=np.int32)
        self.J = np.ascontiguousarray(appendix.node_J_table(nodes))
        Cx, Cy = appendix.force_matrices()
        self.Cx = np.ascontiguousarray(Cx)
        self.Cy = np.ascontiguousarray(Cy)
        self._h = self._lib.orc_stencil_new(_ptr(self.w), _ptr(self.p0), _ptr(self.px), _ptr(self.py),
                                            _iptr(self.cx), _iptr(self.cy), _iptr(self.opp),
                                            _ptr(self.J), _ptr(self.Cx), _ptr(self.Cy))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_stencil_free(h)
            self._h = None

    def _arr(self, a):
        return np.ascontiguousarray(a, dtype=self.real)

    # ---- per-site operations (each a thin call into the C oracle) ----
    def moments(self, f):
        f = self._arr(f)
        N = np.zeros(3, dtype=self.real)
        T = np.zeros(9, dtype=self.real)
        self._lib.orc_moments(self._h, _rptr(f), _rptr(N), _rptr(T))
        return N, T.reshape(3, 3)

    def macro(self, f):
        """(n, T, eps, U) of one site's populations."""
        f = self._arr(f)
        out = np.zeros(3, dtype=self.real)
        U = np.zeros(3, dtype=self.real)
        rc = self._lib.orc_macro(self._h, _rptr(f), _rptr(out[0:1]), _rptr(out[1:2]), _rptr(out[2:3]), _rptr(U))
        if rc:
            raise ArithmeticError("no timelike Landau eigenvector")
        return out[0], out[1], out[2], U

    def feq(self, n, T, U):
        U = self._arr(U)
        out = np.zeros(Q, dtype=self.real)
        self._lib.orc_feq(self._h, n, T, _rptr(U), _rptr(out))
        return out

    def force_term(self, n, T, U, Fx, Fy):
        U = self._arr(U)
        out = np.zeros(Q, dtype=self.real)
        self._lib.orc_force_term(self._h, n, T, _rptr(U), Fx, Fy, _rptr(out))
        return out

    def collide(self, f, tau, Fx=0.0, Fy=0.0):
        f = self._arr(f)
        out = np.zeros(Q, dtype=self.real)
        if self._lib.orc_collide(self._h, _rptr(f), tau, Fx, Fy, _rptr(out)):
            raise ArithmeticError("collision failed (no Landau frame)")
        return out


def projections(n, T, U):
    """Appendix B projections a^(k) times n/T, App. A order."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    a = np.zeros(K)
    lib().orc_projections(float(n), float(T), _ptr(U), _ptr(a))
    return a


def landau(Tm):
    """(eps, U) of a 3x3 contravariant T^{ab}."""
    Tm = np.ascontiguousarray(Tm, dtype=np.float64).reshape(9)
    eps = np.zeros(1)
    U = np.zeros(3)
    rc = lib().orc_landau(_ptr(Tm), _ptr(eps), _ptr(U))
    if rc:
        raise ArithmeticError("no timelike Landau eigenvector")
    return eps[0], U


def four_velocity(vx, vy):
    g = 1.0 / np.sqrt(1.0 - vx * vx - vy * vy)
    return np.array([g, g * vx, g * vy])


EDGES = {"bottom": 0, "top": 1, "left": 2, "right": 3}


class Lattice:
    """nx x ny lattice holding the pre-collision populations f (SoA, float64,
    or long double with a long double stencil).

    contacts: iterable of dicts {edge, start, width, n, T, vx, vy}; edge is
    'bottom' | 'top' | 'left' | 'right' (or 0..3).  Non-periodic edges are
    bounce-back walls except where a contact's ghost span lies.
    """

    def __init__(self, stencil: Stencil, nx: int, ny: int, *, periodic_x=False, periodic_y=False,
                 contacts=(), solid=None, tau=1.0, F=(0.0, 0.0), cg=None):
        self.st = stencil
        self.nx, self.ny = int(nx), int(ny)
        self.tau = float(tau)
        self.F = (float(F[0]), float(F[1]))
        contacts = list(contacts)
        edge = np.array([EDGES.get(c["edge"], c["edge"]) if isinstance(c["edge"], str) else c["edge"]
                         for c in contacts] or [0], dtype=np.int32)
        start = np.array([c["start"] for c in contacts] or [0], dtype=np.int32)
        width = np.array([c["width"] for c in contacts] or [0], dtype=np.int32)
        state = np.array([[c.get("n", 1.0), c.get("T", 1.0), c.get("vx", 0.0), c.get("vy", 0.0)]
                          for c in contacts] or [[0, 0, 0, 0]], dtype=np.float64).reshape(-1)
        self._solid = None
        sp = None
        if solid is not None:
            self._solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.ny, self.nx)
            sp = self._solid.ctypes.data_as(ctypes.c_void_p)
        self._lib = stencil._lib
        self._h = self._lib.orc_lattice_new(stencil._h, self.nx, self.ny, int(periodic_x), int(periodic_y),
                                            len(contacts), _iptr(edge), _iptr(start), _iptr(width),
                                            _ptr(state), sp, self.tau, self.F[0], self.F[1])
        if not self._h:
            raise ValueError("invalid lattice description")
        # local-capacitance force -(1/C_g) grad n (None or inf: off)
        if cg is not None and np.isfinite(cg):
            self._lib.orc_lattice_set_lca(self._h, 1.0 / float(cg))
        self.f = np.zeros((Q, self.ny, self.nx), dtype=stencil.real)
        self.t = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_lattice_free(h)
            self._h = None

    def init_fields(self, n, T, vx, vy):
        shape = (self.ny, self.nx)
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))
                for a in (n, T, vx, vy)]
        self._lib.orc_lattice_init(self._h, *[_ptr(a) for a in arrs], _rptr(self.f))
        self.t = 0

    def run(self, nsteps: int) -> None:
        bad = self._lib.orc_lattice_run(self._h, _rptr(self.f), int(nsteps))
        self.t += int(nsteps)
        if bad:
            raise ArithmeticError(f"{bad} site updates without a Landau frame")

    def post_collision(self) -> np.ndarray:
        out = np.empty_like(self.f)
        if self._lib.orc_lattice_collide(self._h, _rptr(self.f), _rptr(out)):
            raise ArithmeticError("collision failed")
        return out

    def fields(self):
        """dict of n, vx, vy, eps, T arrays (ny, nx) of the current state."""
        out = {k: np.empty((self.ny, self.nx), dtype=self.st.real) for k in ("n", "vx", "vy", "eps", "T")}
        self._lib.orc_lattice_fields(self._h, _rptr(self.f), _rptr(out["n"]), _rptr(out["vx"]),
                                     _rptr(out["vy"]), _rptr(out["eps"]), _rptr(out["T"]))
        return out

    def stream(self, fstar: np.ndarray) -> np.ndarray:
        """Streaming with the boundary rules alone: the pre-collision state
        that the post-collision populations fstar (Q, ny, nx) lead to."""
        fstar = np.ascontiguousarray(fstar, dtype=self.st.real)
        out = np.empty_like(fstar)
        self._lib.orc_lattice_stream(self._h, _rptr(fstar), _rptr(out))
        return out

    def totals(self):
        """Lattice sums of N^0, T^00, T^0x, T^0y and N^x, N^y of the current state."""
        f = self.f.reshape(Q, -1)
        st = self.st
        fs = f.sum(axis=1)
        return {
            "N0": float(fs @ st.p0), "Nx": float(fs @ st.px), "Ny": float(fs @ st.py),
            "T00": float(fs @ (st.p0 * st.p0)), "T0x": float(fs @ (st.p0 * st.px)),
            "T0y": float(fs @ (st.p0 * st.py)),
        }


@functools.lru_cache(maxsize=4)
def stencil(use_printed: bool = False, long_double: bool = False) -> Stencil:
    return Stencil(use_printed, long_double=long_double)
