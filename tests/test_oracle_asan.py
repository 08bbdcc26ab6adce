"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
oracle.c compiled with both, loaded into a child Python process (the ASan
runtime preloaded), runs every pin of tests/oracle_pins.py and the selection
and per-pixel entry points on small scans.  Any out-of-bounds access, use
after free or undefined behaviour aborts the child."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g"]

CHILD = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import numpy as np
import oracle, oracle_pins, synth
lib = oracle.load({lib!r})
for pin in oracle_pins.ALL_PINS:
    pin(lib)
    print("pin", pin.__name__, flush=True)
s = synth.tiny(37, 5, 19, 43, seed=3, n_src=6, dark=100.0)
act = oracle.activity(s.images, lib=lib)
for k in (0, 1, 7, act.shape[0]):
    sel = oracle.select_top(act, k, lib=lib)
    assert sel.shape[0] == k
pix = np.array([0, 36, 37, 184], dtype=np.int64)
out, bins, u = oracle.reconstruct_pixels(s, pix, want_bins=True, want_u=True, lib=lib)
_, _, u_only = oracle.reconstruct_pixels(s, pix, images=None, want_bins=False, want_u=True, lib=lib)
full, tot, _ = oracle.reconstruct(s, row0=2, nrows=3, want_bins=True, lib=lib)
print("entry points ok", flush=True)
"""


def _asan_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    src = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
    subprocess.run(["gcc", *oracle.CFLAGS, *SAN, src, "-o", lib, "-lm"], check=True,
                   capture_output=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=900)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert "entry points ok" in r.stdout
