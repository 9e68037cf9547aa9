"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, g++): tracking in float and double with both candidate scans, the
margin check, the FP64 replay, the refit (both map modes) with its gradient,
the ambiguity solving, the three-iteration fit and the rebuild, on a single
sector that includes non-finite clusters.  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from synth import geometry as G

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    srcs = [os.path.join(HERE, "oracle_sanitize_main.cpp")] + oracle.SOURCES
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", *srcs, "-o", str(exe)], check=True)
    cs = synth.single_sector(seed=2, n_tracks=120)
    y, z = cs.y.copy(), cs.z.copy()
    y[::997] = np.nan
    z[5::1009] = np.inf
    inp = tmp_path / "input.bin"
    with open(inp, "wb") as f:
        f.write(np.array([G.N_ROWS, cs.n_units], np.int32).tobytes())
        f.write(np.array([cs.n_clusters], np.int64).tobytes())
        f.write(G.row_x().astype(np.float32).tobytes())
        f.write(cs.row_begin.astype(np.int64).tobytes())
        f.write(y.astype(np.float32).tobytes())
        f.write(z.astype(np.float32).tobytes())
        f.write(G.sector_alpha(cs.unit_sector).astype(np.float32).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe), str(inp)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "kept" in r.stdout
