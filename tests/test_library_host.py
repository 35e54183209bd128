"""CPU checks of the GPU library: it loads, exports every symbol of
include/rlbm.h, and its host-side constants (quadrature polish and force
matrices, computed independently of the oracle) agree with the oracle's.
No call here touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(rlbm_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    import paper_1804_02418_amd as rl

    L = rl.lib()
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in sorted(declared):
        assert hasattr(L, name), name
    # the binding covers the same set
    from paper_1804_02418_amd import _binding

    assert declared <= set(_binding.SIGNATURES), declared - set(_binding.SIGNATURES)


def test_library_quadrature_matches_oracle():
    import paper_1804_02418_amd as rl
    from oracle import quadrature

    w1, w2, p0 = rl.quadrature()
    o1, o2, op = quadrature.shell_tables()
    # both polishes solve for 12 unknowns of order 1e-4..8 jointly; agreement
    # is to ~1e-19 in absolute terms (the tiny shell p0_1 ~ 1.6e-5 included)
    np.testing.assert_allclose(w1, o1, rtol=4e-16, atol=1e-18)
    np.testing.assert_allclose(w2, o2, rtol=4e-16, atol=1e-18)
    np.testing.assert_allclose(p0, op, rtol=4e-16, atol=1e-18)


def test_library_force_matrices_match_oracle():
    import paper_1804_02418_amd as rl
    from oracle import appendix

    Cx, Cy = rl.force_matrices()
    ox, oy = appendix.force_matrices()
    assert np.abs(Cx - ox).max() < 1e-15
    assert np.abs(Cy - oy).max() < 1e-15


@pytest.mark.parametrize("nx,ny,storage", [(0, 8, 0), (8, -1, 1), (8, 8, 7)])
def test_create_rejects_invalid_arguments(nx, ny, storage):
    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import _binding

    h = ctypes.c_void_p()
    st = rl.lib().rlbm_create(nx, ny, storage, None, ctypes.byref(h))
    assert st == _binding.EINVAL
    assert rl.lib().rlbm_last_error()


def test_null_handle_is_rejected():
    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import _binding

    assert rl.lib().rlbm_set_tau(None, 1.0) == _binding.EINVAL
    assert rl.lib().rlbm_step(None, 1) == _binding.EINVAL
    assert rl.lib().rlbm_set_lca(None, 0.1) == _binding.EINVAL
    rl.lib().rlbm_destroy(None)


@pytest.mark.parametrize("nx,ny,storage", [(65536, 8192, 0), (65536, 32769, 2)])
def test_create_rejects_oversized_lattices(nx, ny, storage):
    """A population plane must stay below 4 GiB (the kernels address each
    plane with a 32-bit byte offset) and the site count below 2^31; both are
    refused before any device call."""
    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import _binding

    h = ctypes.c_void_p()
    assert rl.lib().rlbm_create(nx, ny, storage, None, ctypes.byref(h)) == _binding.EINVAL
    assert not h.value


def test_conv_entry_points_reject_misaligned_tensors():
    """The surrogate's convolution kernels move 8 BF16 channels (16 bytes)
    per access: tensors that do not start on a 16-byte boundary are refused
    on the host."""
    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import _binding

    L = rl.lib()
    good, bad = ctypes.c_void_p(1 << 20), ctypes.c_void_p((1 << 20) + 2)
    assert L.rlbm_conv3x3_forward(bad, good, None, good, 1, 16, 16, 16, 16, 1, None) == _binding.EINVAL
    assert L.rlbm_conv3x3_backward_data(good, good, bad, 1, 16, 16, 16, 16, None) == _binding.EINVAL
    assert L.rlbm_conv3x3_backward_weight(bad, good, good, None, 1, 16, 16, 16, 16, None) == _binding.EINVAL
    assert L.rlbm_conv3x3_backward_weight(good, good, good, None, 1, 16, 16, 24, 16, None) == _binding.EINVAL


def test_store_form_and_block_order_reject_bad_arguments():
    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import _binding

    assert rl.lib().rlbm_set_streaming_stores(None, 1) == _binding.EINVAL
    assert rl.lib().rlbm_set_streaming_loads(None, 1) == _binding.EINVAL
    assert rl.lib().rlbm_get_memory_form(None, None, None) == _binding.EINVAL
    assert rl.lib().rlbm_version() == _binding.ABI_VERSION
    assert rl.lib().rlbm_set_block_order(None, 0) == _binding.EINVAL
    assert rl.lib().rlbm_set_gather_table(None, 1) == _binding.EINVAL


def test_bandwidth_probe_rejects_bad_arguments():
    """Checked before any device call: unknown pattern, element size, sizes
    too small for the pull's interior, too many rows, no repetitions."""
    import paper_1804_02418_amd as rl
    from paper_1804_02418_amd import _binding as B

    for args in ((9, 4, 64, 64, 0, 1), (-1, 4, 64, 64, 0, 1), (0, 3, 64, 64, 0, 1), (2, 4, 10, 64, 0, 1), (2, 4, 64, 10, 0, 1),
                 (2, 4, 64, 70000, 0, 1), (1, 4, 64, 64, 0, 0)):
        st = rl.lib().rlbm_bandwidth_probe(*args, None, None, None)
        assert st == B.EINVAL, (args, st)
