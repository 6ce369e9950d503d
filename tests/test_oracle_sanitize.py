"""The three CPU oracles built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc) and driven through every boundary kind,
source terms and the sampled step (tests/sanitize_driver.c): no
out-of-bounds access, no leak, no undefined behaviour, finite results."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracles_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "driver")
    srcs = [os.path.join(HERE, "sanitize_driver.c")] + [
        os.path.join(ROOT, "oracle", f) for f in ("dugks_oracle.c", "dugks_oracle1d.c", "dugks_oracle3d.c")]
    build = subprocess.run([gcc, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=all", "-ffp-contract=off", *srcs, "-lm", "-o", exe],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "ok" in run.stdout
