"""The autotuner's cache file, named by RLBM_TUNE_CACHE.

The library reads it at the first lattice creation of a process: one entry
per line, `arch storage nx ny mask tile_x form` (form: bit 0 streaming
stores, bit 1 non-temporal loads).  Lines of another shape (the six-field
lines of ABI version 1), of another architecture, or with a tile width or
form out of range are skipped, and such a lattice starts with the default
launch.  An autotuned lattice appends its pick, and a later process starts
a lattice of the same description with it.

Each check runs in a child process of its own, since the file is read once
per process.
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# prints [(tile_x, streaming stores, non-temporal loads), ...] for FP32
# lattices 300 wide of the given heights; with "tune", autotunes the last
CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import paper_1804_02418_amd as rl
heights, tune = json.loads(sys.argv[2]), sys.argv[3] == "tune"
out = []
for ny in heights:
    L = rl.Lattice(300, ny, "f32")
    if tune and ny == heights[-1]:
        L.init_uniform(1.0, 1.0, 0.0, 0.0)
        L.autotune(3)
    out.append((L.launch_shape()[0],) + tuple(L.memory_form()))
    L.close()
print(json.dumps(out))
"""


def _child(cache, heights, tune=False):
    env = dict(os.environ, RLBM_TUNE_CACHE=str(cache))
    print("child: heights", heights, "tune" if tune else "", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, json.dumps(heights), "tune" if tune else "-"],
                       env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    return [tuple(v) for v in json.loads(r.stdout.strip().splitlines()[-1])]


def _arch():
    import torch

    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def test_cache_entries_are_validated(tmp_path):
    arch = _arch()
    cache = tmp_path / "tune.txt"
    cache.write_text("\n".join([
        f"{arch} 1 300 40 0 64",          # six fields: skipped
        f"{arch} 1 300 41 0 32 1",        # tile width out of range: skipped
        f"{arch} 1 300 42 0 64 3",        # valid
        f"{arch} 1 300 43 0 128 4",       # form out of range: skipped
        "gfx000 1 300 44 0 128 1",        # another architecture
        "not an entry",
    ]) + "\n")
    got = _child(cache, [40, 41, 42, 43, 44])
    default = (256, False, False)  # 300 wide: 256-wide tiles; 4.6 MB of populations: ordinary stores
    assert got == [default, default, (64, True, True), default, default], got


def test_autotuned_pick_is_reused_by_a_later_process(tmp_path):
    cache = tmp_path / "tune.txt"
    picked = _child(cache, [45], tune=True)[0]
    lines = cache.read_text().split("\n")
    assert len([ln for ln in lines if ln.strip()]) == 1 and len(lines[0].split()) == 7, lines
    assert _child(cache, [45]) == [picked]
