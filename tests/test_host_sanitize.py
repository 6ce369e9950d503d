"""The host side of libdugks (2-D, batch, 3-D and 1-D families) built with
AddressSanitizer and UndefinedBehaviorSanitizer for the host code only (each
-fsanitize after -Xarch_host; the device code and the kernel objects are
the library's own build) and driven without a GPU through argument checks,
state errors and format checks (tests/host_sanitize_driver.cpp): every call
returns its documented code, with no memory error, leak or undefined
behaviour."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_1906_11036_amd")
CSRC = os.path.join(PKG, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-g"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def test_host_library_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC) or shutil.which("ld") is None:
        pytest.skip("hipcc not found")
    from paper_1906_11036_amd import build as B
    kernels = [os.path.join(B.OBJ, f) for f in ("dugks_kernels.hip.o", "dugks3d_kernels.hip.o")]
    if not all(os.path.exists(k) for k in kernels):
        B.build(incremental=True)
    srcs = [os.path.join(CSRC, f) for f in ("dugks_host.cpp", "dugks3d_host.cpp", "dugks1d.hip")]
    srcs.append(os.path.join(HERE, "host_sanitize_driver.cpp"))
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]

    def compile_one(pair):
        s, o = pair
        return subprocess.run([HIPCC] + FLAGS + SAN + ["-c", s, "-o", o], capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(compile_one, zip(srcs, objs)))
    for s, r in zip(srcs, results):
        assert r.returncode == 0, f"{os.path.basename(s)}: {r.stderr[-3000:]}"
    exe = str(tmp_path / "driver")
    link = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined"] + objs + kernels + ["-o", exe],
                          capture_output=True, text=True)
    assert link.returncode == 0, link.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "ok" in run.stdout
