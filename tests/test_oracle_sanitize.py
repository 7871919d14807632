"""The oracle under the host sanitizers: tests/native/oracle_sanitize_driver.c
and oracle/rhg_oracle.c built with gcc -fsanitize=address,undefined (no GPU
code involved), run on a small graph; any memory error or undefined
behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_is_clean_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fopenmp",
           os.path.join(HERE, "native", "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "rhg_oracle.c"),
           "-o", exe, "-lquadmath", "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "sanitizer" in (b.stderr or "").lower() and "cannot find" in (b.stderr or "").lower():
        pytest.skip("sanitizer runtime libraries are not installed: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-1000:], r.stderr[-4000:])
    assert r.stdout.startswith("ok")
