"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code.

* The oracle (oracle/rlbm_oracle.c, both its float64 and long double builds)
  is compiled with gcc -fsanitize=address,undefined and driven through every
  lattice feature -- contacts on every edge and at the corners, a solid
  mask, tiny periodic lattices whose hops wrap several times, the
  local-capacitance force, streaming alone, per-site calls -- in a process
  with the AddressSanitizer runtime preloaded.  Any report fails the test,
  and the results must equal the ordinary build's.
* The library's host-only code (the quadrature polish and force matrices,
  the quadrature searches: csrc/host_constants.cpp, csrc/quadrature_search.cpp)
  is compiled with g++ and the same sanitizers into tests/sanitize/host_driver,
  which runs every entry point of that code, error paths included; its
  results must equal the library's.
The GPU code is not built here: device sanitizers are not part of this
build, and the lattice runtime needs a device.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} is not available to gcc")
    return os.path.realpath(path)


def _env(extra=None):
    env = dict(os.environ)
    env.update(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    env.update(extra or {})
    return env


def _check_clean(res):
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    src = os.path.join(ROOT, "oracle", "rlbm_oracle.c")
    libs = []
    for tag, flags in (("f64", []), ("ld", ["-DORC_LONG_DOUBLE"])):
        out = str(tmp_path / f"librlbm_oracle_{tag}_san.so")
        subprocess.run(["gcc", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", *SAN, *flags, "-o", out, src,
                        "-lm"], check=True)
        libs.append(out)
    driver = os.path.join(ROOT, "tests", "sanitize", "oracle_driver.py")
    res = subprocess.run([sys.executable, driver, *libs], capture_output=True, text=True, timeout=600,
                         env=_env({"LD_PRELOAD": asan}), cwd=ROOT)
    _check_clean(res)
    san = [line.split() for line in res.stdout.splitlines()]
    # the same driver on the ordinary builds
    import oracle

    oracle.build(force=False)
    oracle.build(force=False, long_double=True)
    ref = subprocess.run([sys.executable, driver, oracle._LIB, oracle._LIB_LD], capture_output=True, text=True,
                         timeout=600, env=_env(), cwd=ROOT)
    assert ref.returncode == 0, ref.stderr[-2000:]
    plain = [line.split() for line in ref.stdout.splitlines()]
    assert len(san) == len(plain) >= 13
    for a, b in zip(san, plain):
        assert a[:2] == b[:2]
        for x, y in zip(a[2:], b[2:]):
            assert abs(float(x) - float(y)) <= 1e-12 * max(1.0, abs(float(y))), (a, b)


def test_host_code_under_address_and_undefined_sanitizers(tmp_path):
    from oracle import quadrature_search as Q

    import paper_1804_02418_amd as rl

    csrc = os.path.join(ROOT, "paper_1804_02418_amd", "csrc")
    exe = str(tmp_path / "host_driver")
    subprocess.run(["g++", "-std=c++17", "-Wall", *SAN, "-o", exe,
                    os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                    os.path.join(csrc, "host_constants.cpp"), os.path.join(csrc, "quadrature_search.cpp")], check=True)
    vec = Q.full_symmetric(Q.M5_ORBIT_REPS)
    res = subprocess.run([exe, "5.0", *[str(v) for xy in vec for v in xy]], capture_output=True, text=True,
                         timeout=900, env=_env())
    _check_clean(res)
    got = {}
    for line in res.stdout.splitlines():
        k, *v = line.split()
        got.setdefault(k, []).append(v)
    # the same computations through the library
    w1, w2, p0 = rl.quadrature()
    for k, ref in (("w1", w1), ("w2", w2), ("p0", p0)):
        assert np.allclose([float(x) for x in got[k][0]], ref, rtol=1e-15, atol=0), k
    assert float(got["massless_residual"][0][0]) < 1e-13
    for m, a, b, c, v in got["moment"]:
        assert abs(float(v) - rl.mj_moment(float(m), int(a), int(b), int(c))) <= 1e-13 * max(1.0, abs(float(v)))
    st, v0, wmin, _ = got["massive"][0]
    v0_lib, _, wmin_lib, _ = rl.quadrature_massive(5.0, vec, nscan=2000)
    assert int(st) == 0 and abs(float(v0) - v0_lib) < 1e-12 and abs(float(wmin) - wmin_lib) < 1e-12
    assert int(got["massless"][0][0]) == 0
    for k in ("massive_bad", "massless_bad", "order_bad"):
        assert int(got[k][0][0]) == -1, k
