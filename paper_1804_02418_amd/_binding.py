"""ctypes binding of librlbm.so (argument marshalling only; every step of the
method runs in the library's HIP kernels).  Names follow include/rlbm.h."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlbm.so")
ABI_VERSION = 2

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSTABLE, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
F64, F32, F16DEV = 0, 1, 2
STORAGE = {"f64": F64, "f32": F32, "f16dev": F16DEV, F64: F64, F32: F32, F16DEV: F16DEV}
EDGE = {"bottom": 0, "top": 1, "left": 2, "right": 3}


class RlbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"rlbm status {status}: {message}")
        self.status = status


class Unstable(RlbmError):
    pass


class rlbm_contact(ctypes.Structure):
    _fields_ = [("edge", ctypes.c_int), ("start", ctypes.c_int), ("width", ctypes.c_int),
                ("n", ctypes.c_double), ("T", ctypes.c_double), ("vx", ctypes.c_double), ("vy", ctypes.c_double)]


class rlbm_sample(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("periodic_x", ctypes.c_int), ("periodic_y", ctypes.c_int),
                ("tau", ctypes.c_double), ("Fx", ctypes.c_double), ("Fy", ctypes.c_double),
                ("ncontacts", ctypes.c_int), ("contacts", rlbm_contact * 4),
                ("n0", ctypes.c_double), ("T0", ctypes.c_double), ("vx0", ctypes.c_double), ("vy0", ctypes.c_double)]


def _contact(c) -> rlbm_contact:
    e = c["edge"]
    return rlbm_contact(EDGE.get(e, e) if isinstance(e, str) else int(e), int(c["start"]), int(c["width"]),
                        float(c.get("n", 1.0)), float(c.get("T", 1.0)), float(c.get("vx", 0.0)),
                        float(c.get("vy", 0.0)))


_lib = None

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_ip = ctypes.POINTER(ctypes.c_int)

# name -> (argtypes, restype); restype None = rlbm_status (int)
SIGNATURES = {
    "rlbm_last_error": ([], ctypes.c_char_p),
    "rlbm_version": ([], ctypes.c_int),
    "rlbm_quadrature": ([_dp, _dp, _dp], None),
    "rlbm_force_matrices": ([_dp, _dp], None),
    "rlbm_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp)], None),
    "rlbm_destroy": ([_vp], "void"),
    "rlbm_set_boundaries": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(rlbm_contact), ctypes.c_int], None),
    "rlbm_set_mask": ([_vp, _vp], None),
    "rlbm_set_tau": ([_vp, ctypes.c_double], None),
    "rlbm_set_drive": ([_vp, ctypes.c_double, ctypes.c_double], None),
    "rlbm_set_lca": ([_vp, ctypes.c_double], None),
    "rlbm_set_quadrature": ([_vp, _dp, _dp, _dp], None),
    "rlbm_mj_moment": ([ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp], None),
    "rlbm_quadrature_massive": ([ctypes.c_double, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp],
                                None),
    "rlbm_quadrature_massless": ([ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_uint64,
                                  ctypes.c_int, _dp, _dp, _dp, _dp], None),
    "rlbm_bandwidth_probe": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                              _dp, _dp], None),
    "rlbm_set_block_order": ([_vp, ctypes.c_int], None),
    "rlbm_batch_set_block_order": ([_vp, ctypes.c_int], None),
    "rlbm_set_reference": ([_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double], None),
    "rlbm_init_uniform": ([_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double], None),
    "rlbm_init_fields": ([_vp, _vp, _vp, _vp, _vp, ctypes.c_int], None),
    "rlbm_step": ([_vp, _i64], None),
    "rlbm_get_time": ([_vp, ctypes.POINTER(_i64)], None),
    "rlbm_read_fields": ([_vp, _vp, _vp, _vp, _vp, ctypes.c_int], None),
    "rlbm_residual": ([_vp, _dp], None),
    "rlbm_residual_noalloc": ([_vp, _dp], None),
    "rlbm_step_until": ([_vp, _i64, _i64, ctypes.c_double, ctypes.POINTER(_i64), _dp], None),
    "rlbm_read_populations": ([_vp, _vp, ctypes.c_int], None),
    "rlbm_state_bytes": ([_vp, ctypes.POINTER(ctypes.c_size_t)], None),
    "rlbm_get_state": ([_vp, _vp, ctypes.c_size_t], None),
    "rlbm_set_state": ([_vp, _vp, ctypes.c_size_t], None),
    "rlbm_set_launch_shape": ([_vp, ctypes.c_int, ctypes.c_int], None),
    "rlbm_get_launch_shape": ([_vp, _ip, _ip], None),
    "rlbm_autotune": ([_vp, ctypes.c_int, _dp], None),
    "rlbm_set_streaming_stores": ([_vp, ctypes.c_int], None),
    "rlbm_set_streaming_loads": ([_vp, ctypes.c_int], None),
    "rlbm_get_memory_form": ([_vp, _ip, _ip], None),
    "rlbm_set_gather_table": ([_vp, ctypes.c_int], None),
    "rlbm_synchronize": ([_vp], None),
    "rlbm_batch_create": ([_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp)], None),
    "rlbm_batch_destroy": ([_vp], "void"),
    "rlbm_batch_lattice": ([_vp, ctypes.c_int, ctypes.POINTER(_vp)], None),
    "rlbm_batch_step": ([_vp, _i64, ctypes.c_int], None),
    "rlbm_batch_set_active": ([_vp, _vp], None),
    "rlbm_batch_residual": ([_vp, _dp], None),
    "rlbm_batch_step_until": ([_vp, _i64, _i64, ctypes.c_double, _vp, _dp], None),
    "rlbm_batch_autotune": ([_vp, ctypes.c_int, _dp], None),
    "rlbm_batch_sites": ([_vp, ctypes.POINTER(_i64)], None),
    # surrogate (include/rlbm_surrogate.h)
    "rlbm_unet_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_uint64, _vp, ctypes.POINTER(_vp)], None),
    "rlbm_unet_destroy": ([_vp], "void"),
    "rlbm_unet_param_count": ([_vp, ctypes.POINTER(_i64)], None),
    "rlbm_unet_set_params": ([_vp, _vp], None),
    "rlbm_unet_get_params": ([_vp, _vp], None),
    "rlbm_unet_get_grads": ([_vp, _vp], None),
    "rlbm_unet_forward": ([_vp, _vp, _vp, ctypes.c_int], None),
    "rlbm_unet_mse": ([_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_float), _vp], None),
    "rlbm_unet_backward": ([_vp, _vp, ctypes.c_int, _vp], None),
    "rlbm_unet_zero_grad": ([_vp], None),
    "rlbm_unet_adam_step": ([_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float], None),
    "rlbm_conv3x3_forward": ([_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, _vp], None),
    "rlbm_conv3x3_backward_data": ([_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, _vp], None),
    "rlbm_conv3x3_backward_weight": ([_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _vp], None),
}


def lib() -> ctypes.CDLL:
    """Load the in-tree librlbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname as the system
        # one; load it first so that torch and librlbm share one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1804_02418_amd.build.build() "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None if res == "void" else (ctypes.c_int if res is None else res)
        if L.rlbm_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.rlbm_version()}, this binding {ABI_VERSION}: rebuild it")
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != OK:
        msg = lib().rlbm_last_error().decode(errors="replace")
        raise (Unstable if status == EUNSTABLE else RlbmError)(status, msg)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def quadrature():
    """(w1[4], w2[4], p0[4]) polished by the library on the host."""
    w1, w2, p0 = np.zeros(4), np.zeros(4), np.zeros(4)
    check(lib().rlbm_quadrature(w1.ctypes.data_as(_dp), w2.ctypes.data_as(_dp), p0.ctypes.data_as(_dp)))
    return w1, w2, p0


def force_matrices():
    Cx, Cy = np.zeros(256), np.zeros(256)
    check(lib().rlbm_force_matrices(Cx.ctypes.data_as(_dp), Cy.ctypes.data_as(_dp)))
    return Cx.reshape(16, 16), Cy.reshape(16, 16)


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class Lattice:
    """One nx x ny lattice owned by the library (see include/rlbm.h)."""

    def __init__(self, nx: int, ny: int, storage="f64", stream=None):
        self.nx, self.ny = int(nx), int(ny)
        self.storage = STORAGE[storage]
        h = _vp()
        s = _vp(stream) if stream is not None else None
        check(lib().rlbm_create(self.nx, self.ny, self.storage, s, ctypes.byref(h)))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().rlbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- set-up ----
    def set_boundaries(self, periodic_x=False, periodic_y=False, contacts=()):
        contacts = list(contacts)
        arr = (rlbm_contact * max(1, len(contacts)))()
        for k, c in enumerate(contacts):
            arr[k] = _contact(c)
        check(lib().rlbm_set_boundaries(self._h, int(bool(periodic_x)), int(bool(periodic_y)), arr, len(contacts)))

    def set_mask(self, mask):
        if mask is None:
            check(lib().rlbm_set_mask(self._h, None))
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(self.ny, self.nx)
        check(lib().rlbm_set_mask(self._h, m.ctypes.data))

    def set_tau(self, tau):
        check(lib().rlbm_set_tau(self._h, float(tau)))

    def set_drive(self, Fx, Fy=0.0):
        check(lib().rlbm_set_drive(self._h, float(Fx), float(Fy)))

    def set_block_order(self, xcd_contiguous: bool):
        check(lib().rlbm_set_block_order(self._h, int(bool(xcd_contiguous))))

    def set_quadrature(self, w1, w2, p0):
        """Another member of the massless third-order quadrature family (then init again)."""
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (w1, w2, p0)]
        check(lib().rlbm_set_quadrature(self._h, *[x.ctypes.data_as(_dp) for x in a]))

    def set_lca(self, cg):
        """Local-capacitance force with capacitance C_g (None or inf: off)."""
        inv = 0.0 if cg is None or not np.isfinite(cg) else 1.0 / float(cg)
        check(lib().rlbm_set_lca(self._h, inv))

    def set_reference(self, n_ref=1.0, T_ref=1.0, scale=1.0):
        check(lib().rlbm_set_reference(self._h, float(n_ref), float(T_ref), float(scale)))

    def init_uniform(self, n=1.0, T=1.0, vx=0.0, vy=0.0):
        check(lib().rlbm_init_uniform(self._h, float(n), float(T), float(vx), float(vy)))

    def _device_field(self, a, name):
        """A caller-owned field on the device: a contiguous float64 CUDA tensor
        of nx * ny elements (checked here; the library reads or writes exactly
        that many)."""
        import torch

        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
                and a.numel() == self.nx * self.ny):
            raise ValueError(f"{name}: need a contiguous float64 CUDA tensor of {self.nx} x {self.ny} elements, got "
                             f"{getattr(a, 'dtype', type(a))} {tuple(getattr(a, 'shape', ()))} "
                             f"on {getattr(a, 'device', '?')}")
        return a

    def init_fields(self, n, T, vx, vy):
        if any(_is_torch(a) for a in (n, T, vx, vy)):
            import torch

            fields = [self._device_field(a, k) for a, k in zip((n, T, vx, vy), ("n", "T", "vx", "vy"))]
            # the init kernel runs on the lattice's stream: order it after the
            # work that produced the fields, and let it finish before the
            # caller may free them
            torch.cuda.current_stream(fields[0].device).synchronize()
            check(lib().rlbm_init_fields(self._h, *[a.data_ptr() for a in fields], 1))
            check(lib().rlbm_synchronize(self._h))
            return
        shape = (self.ny, self.nx)
        arrs = [np.ascontiguousarray(np.broadcast_to(_f64(a), shape)) for a in (n, T, vx, vy)]
        check(lib().rlbm_init_fields(self._h, *[a.ctypes.data for a in arrs], 0))

    # ---- time stepping ----
    def step(self, nsteps: int):
        check(lib().rlbm_step(self._h, int(nsteps)))

    @property
    def time(self) -> int:
        t = _i64()
        check(lib().rlbm_get_time(self._h, ctypes.byref(t)))
        return t.value

    def step_until(self, max_steps: int, check_every: int, tol: float):
        taken, r = _i64(), ctypes.c_double()
        check(lib().rlbm_step_until(self._h, int(max_steps), int(check_every), float(tol), ctypes.byref(taken),
                                    ctypes.byref(r)))
        return taken.value, r.value

    # ---- observation ----
    def read_fields(self):
        """dict n, vx, vy, eps of numpy arrays (ny, nx)."""
        out = {k: np.empty((self.ny, self.nx)) for k in ("n", "vx", "vy", "eps")}
        check(lib().rlbm_read_fields(self._h, *[out[k].ctypes.data for k in ("n", "vx", "vy", "eps")], 0))
        return out

    def read_fields_device(self, n, vx, vy, eps):
        """Copy the fields into caller-owned device buffers (contiguous float64
        CUDA tensors of nx * ny elements, or None); returns once the copies
        are done."""
        outs = [None if a is None else self._device_field(a, k) for a, k in zip((n, vx, vy, eps),
                                                                                 ("n", "vx", "vy", "eps"))]
        check(lib().rlbm_read_fields(self._h, *[None if a is None else a.data_ptr() for a in outs], 1))
        check(lib().rlbm_synchronize(self._h))

    def residual(self) -> float:
        r = ctypes.c_double()
        check(lib().rlbm_residual(self._h, ctypes.byref(r)))
        return r.value

    def residual_noalloc(self) -> float:
        """rlbm_residual_noalloc: the same residual, with no allocation."""
        r = ctypes.c_double()
        check(lib().rlbm_residual_noalloc(self._h, ctypes.byref(r)))
        return r.value

    def read_populations(self) -> np.ndarray:
        f = np.empty((48, self.ny, self.nx))
        check(lib().rlbm_read_populations(self._h, f.ctypes.data, 0))
        return f

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        check(lib().rlbm_state_bytes(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        check(lib().rlbm_get_state(self._h, buf, n.value))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().rlbm_set_state(self._h, buf, len(blob)))

    def set_launch_shape(self, tile_x: int, rows: int):
        check(lib().rlbm_set_launch_shape(self._h, int(tile_x), int(rows)))

    def launch_shape(self):
        """(tile_x, rows) of the step's work decomposition."""
        t, r = ctypes.c_int(), ctypes.c_int()
        check(lib().rlbm_get_launch_shape(self._h, ctypes.byref(t), ctypes.byref(r)))
        return t.value, r.value

    def set_streaming_stores(self, on: bool):
        check(lib().rlbm_set_streaming_stores(self._h, int(bool(on))))

    def set_streaming_loads(self, on: bool):
        check(lib().rlbm_set_streaming_loads(self._h, int(bool(on))))

    def memory_form(self):
        """(streaming stores, non-temporal loads) of the next step."""
        a, b = ctypes.c_int(), ctypes.c_int()
        check(lib().rlbm_get_memory_form(self._h, ctypes.byref(a), ctypes.byref(b)))
        return bool(a.value), bool(b.value)

    def set_gather_table(self, enabled: bool):
        """False: resolve every boundary source in place, as lattices of 4 GiB
        and more do (include/rlbm.h)."""
        check(lib().rlbm_set_gather_table(self._h, int(bool(enabled))))

    def autotune(self, trial_steps: int = 20):
        """Pick the fastest launch shape and memory form; returns ms/step for
        tile_x 64, 128, 256 in the ordinary form, then with streaming stores,
        with non-temporal loads, and with both."""
        ms = np.zeros(12)
        check(lib().rlbm_autotune(self._h, int(trial_steps), ms.ctypes.data_as(_dp)))
        return ms

    def synchronize(self):
        check(lib().rlbm_synchronize(self._h))


class _BorrowedLattice(Lattice):
    """A sample lattice owned by a Batch (not destroyed from Python)."""

    def __init__(self, handle, nx, ny, storage):
        self.nx, self.ny, self.storage, self._h = nx, ny, storage, handle

    def close(self) -> None:
        self._h = None


class Batch:
    """Many uneven lattices advanced together, one launch per step over all
    samples' work items (see rlbm_batch_* in include/rlbm.h)."""

    def __init__(self, samples, storage="f32", stream=None):
        n = len(samples)
        arr = (rlbm_sample * n)()
        for k, w in enumerate(samples):
            cs = list(w["contacts"])
            if len(cs) > 4:
                raise ValueError("at most 4 contacts per sample")
            q = arr[k]
            q.nx, q.ny = int(w["nx"]), int(w["ny"])
            q.periodic_x, q.periodic_y = int(bool(w["periodic_x"])), int(bool(w["periodic_y"]))
            q.tau, q.Fx, q.Fy = float(w["tau"]), float(w["F"][0]), float(w["F"][1])
            q.ncontacts = len(cs)
            for j, c in enumerate(cs):
                q.contacts[j] = _contact(c)
            i = w.get("init", {})
            q.n0, q.T0 = float(i.get("n", 1.0)), float(i.get("T", 1.0))
            q.vx0, q.vy0 = float(i.get("vx", 0.0)), float(i.get("vy", 0.0))
        self.storage = STORAGE[storage]
        self.n = n
        h = _vp()
        s = _vp(stream) if stream is not None else None
        check(lib().rlbm_batch_create(arr, n, self.storage, s, ctypes.byref(h)))
        self._h = h
        self.lattices = []
        for k in range(n):
            lh = _vp()
            check(lib().rlbm_batch_lattice(self._h, k, ctypes.byref(lh)))
            self.lattices.append(_BorrowedLattice(lh, arr[k].nx, arr[k].ny, self.storage))

    def close(self) -> None:
        if getattr(self, "_h", None):
            for L in self.lattices:
                L.close()
            lib().rlbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps: int, graph: bool = True):
        check(lib().rlbm_batch_step(self._h, int(nsteps), int(bool(graph))))

    def set_active(self, active):
        a = np.ascontiguousarray(active, dtype=np.uint8)
        check(lib().rlbm_batch_set_active(self._h, a.ctypes.data))

    def residual(self) -> np.ndarray:
        r = np.zeros(self.n)
        check(lib().rlbm_batch_residual(self._h, r.ctypes.data_as(_dp)))
        return r

    def step_until(self, max_steps: int, check_every: int, tol: float):
        steps = np.zeros(self.n, dtype=np.int64)
        r = np.zeros(self.n)
        check(lib().rlbm_batch_step_until(self._h, int(max_steps), int(check_every), float(tol), steps.ctypes.data,
                                          r.ctypes.data_as(_dp)))
        return steps, r

    def autotune(self, trial_steps: int = 10) -> np.ndarray:
        ms = np.zeros(6)
        check(lib().rlbm_batch_autotune(self._h, int(trial_steps), ms.ctypes.data_as(_dp)))
        return ms

    def set_block_order(self, xcd_contiguous: bool):
        check(lib().rlbm_batch_set_block_order(self._h, int(bool(xcd_contiguous))))

    def sites(self) -> int:
        n = _i64()
        check(lib().rlbm_batch_sites(self._h, ctypes.byref(n)))
        return n.value


class NotFound(RlbmError):
    pass


PROBE_PATTERNS = {"read": 0, "copy": 1, "pull48": 2, "pull48_pair": 3, "pull12_tuple": 4, "pull24_tuple": 5,
                  "pull48_t64": 6, "pull24_tuple_t64": 7, "pull12_tuple_t64": 8}


def bandwidth_probe(pattern: str, elem_bytes: int, nx: int, ny: int, nontemporal: bool = False, reps: int = 10,
                    stream=None):
    """(GB/s, us per launch) of a read, copy or 48-plane pull over arrays the
    size of one population array of an nx x ny lattice (include/rlbm_probe.h)."""
    g, u = ctypes.c_double(), ctypes.c_double()
    check(lib().rlbm_bandwidth_probe(PROBE_PATTERNS[pattern], int(elem_bytes), int(nx), int(ny), int(bool(nontemporal)),
                                     int(reps), _vp(stream) if stream else None, ctypes.byref(g), ctypes.byref(u)))
    return g.value, u.value


def mj_moment(mbar: float, a: int, b: int, c: int) -> float:
    """<p0^a px^b py^c> of the rest Maxwell-Juttner weight (include/rlbm_quadrature.h)."""
    v = ctypes.c_double()
    check(lib().rlbm_mj_moment(float(mbar), int(a), int(b), int(c), ctypes.byref(v)))
    return v.value


def quadrature_massive(mbar: float, vectors, order: int = 3, nscan: int = 0):
    """Search of Sec. 2.3 for massive particles: (v0, per-node weights,
    smallest weight, residual).  Raises NotFound (carrying the best attempt
    in .result) when no v0 gives non-negative weights."""
    vec = np.ascontiguousarray(np.asarray(vectors, dtype=np.int32).reshape(-1, 2))
    n = vec.shape[0]
    w = np.zeros(n)
    v0, mw, res = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib().rlbm_quadrature_massive(float(mbar), int(order), vec.ctypes.data, n, int(nscan), ctypes.byref(v0),
                                       w.ctypes.data_as(_dp), ctypes.byref(mw), ctypes.byref(res))
    out = (v0.value, w, mw.value, res.value)
    if st == ENOTFOUND:
        e = NotFound(st, lib().rlbm_last_error().decode(errors="replace"))
        e.result = out
        raise e
    check(st)
    return out


def quadrature_massless(directions, nshells: int, order: int = 3, start=None, seed: int = 1, max_starts: int = 64):
    """Search of Sec. 2.3 for massless particles: (p0[nshells] ascending,
    weights[nshells, ndir], smallest weight, residual).  start = (p0, w) with
    w shaped (nshells, ndir) starts from there instead of random starts."""
    d = np.ascontiguousarray(np.asarray(directions, dtype=np.int32).reshape(-1, 2))
    nd = d.shape[0]
    p0 = np.zeros(nshells)
    w = np.zeros((nshells, nd))
    mw, res = ctypes.c_double(), ctypes.c_double()
    sp = sw = None
    if start is not None:
        sp = np.ascontiguousarray(start[0], dtype=np.float64)
        sw = np.ascontiguousarray(start[1], dtype=np.float64).reshape(nshells, nd)
    st = lib().rlbm_quadrature_massless(int(order), d.ctypes.data, nd, int(nshells),
                                        None if sp is None else sp.ctypes.data,
                                        None if sw is None else sw.ctypes.data, int(seed), int(max_starts),
                                        p0.ctypes.data_as(_dp), w.ctypes.data_as(_dp), ctypes.byref(mw),
                                        ctypes.byref(res))
    out = (p0, w, mw.value, res.value)
    if st == ENOTFOUND:
        e = NotFound(st, lib().rlbm_last_error().decode(errors="replace"))
        e.result = out
        raise e
    check(st)
    return out


def _ptr(t):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    assert t.is_contiguous()
    return t.data_ptr()


def _stream_ptr(stream):
    return None if stream is None else _vp(stream)


class UNet:
    """The warm-start surrogate network (include/rlbm_surrogate.h).  Inputs
    and outputs are device float32 torch tensors in NHWC layout."""

    def __init__(self, base=16, cin=16, cout=3, height=256, width=256, max_batch=8, seed=1, stream=None):
        h = _vp()
        check(lib().rlbm_unet_create(int(base), int(cin), int(cout), int(height), int(width), int(max_batch),
                                     int(seed), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.base, self.cin, self.cout, self.height, self.width, self.max_batch = base, cin, cout, height, width, max_batch
        n = _i64()
        check(lib().rlbm_unet_param_count(self._h, ctypes.byref(n)))
        self.nparam = n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().rlbm_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.nparam
        check(lib().rlbm_unet_set_params(self._h, a.ctypes.data))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparam, dtype=np.float32)
        check(lib().rlbm_unet_get_params(self._h, a.ctypes.data))
        return a

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.nparam, dtype=np.float32)
        check(lib().rlbm_unet_get_grads(self._h, a.ctypes.data))
        return a

    def forward(self, x, y):
        check(lib().rlbm_unet_forward(self._h, _ptr(x), _ptr(y), int(x.shape[0])))

    def mse(self, y, t, dy=None) -> float:
        loss = ctypes.c_float()
        check(lib().rlbm_unet_mse(self._h, _ptr(y), _ptr(t), int(y.shape[0]), ctypes.byref(loss), _ptr(dy)))
        return loss.value

    def backward(self, dy, dx=None):
        check(lib().rlbm_unet_backward(self._h, _ptr(dy), int(dy.shape[0]), _ptr(dx)))

    def zero_grad(self):
        check(lib().rlbm_unet_zero_grad(self._h))

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        check(lib().rlbm_unet_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps)))


def conv3x3_forward(x, w, b, y, relu=True, stream=None):
    B, H, W, ci = x.shape
    co = w.shape[0]
    check(lib().rlbm_conv3x3_forward(_ptr(x), _ptr(w), _ptr(b), _ptr(y), B, H, W, ci, co, int(bool(relu)),
                                     _stream_ptr(stream)))


def conv3x3_backward_data(dy, w, dx, stream=None):
    B, H, W, co = dy.shape
    ci = w.shape[3]
    check(lib().rlbm_conv3x3_backward_data(_ptr(dy), _ptr(w), _ptr(dx), B, H, W, ci, co, _stream_ptr(stream)))


def conv3x3_backward_weight(dy, x, gw, gb=None, stream=None):
    B, H, W, co = dy.shape
    ci = x.shape[3]
    check(lib().rlbm_conv3x3_backward_weight(_ptr(dy), _ptr(x), _ptr(gw), _ptr(gb), B, H, W, ci, co,
                                             _stream_ptr(stream)))
