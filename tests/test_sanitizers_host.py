"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle through every topology, model and solver entry, and the library's
host paths (argument validation, footprints, the coupling-matrix compression,
the server's queue, the tuning cache) built from the library sources with host
code only.  Drivers: tests/sanitize/."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2410_19075_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host code only (no device compilation); each sanitizer flag applies to the host pass
HOST_SAN = ["--offload-host-only", "-fgpu-rdc", "-O1", "-g", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"],
        str(tmp_path))
    r = run([exe], str(tmp_path))
    assert "oracle clean" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_paths_under_sanitizers(tmp_path):
    from paper_2410_19075_amd import build as nd_build
    inc = ["-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    srcs = [os.path.join(CSRC, s) for s in nd_build.SOURCES] + [os.path.join(SAN, "host_driver.cpp")]
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]

    def compile_one(a):
        src, obj = a
        run([HIPCC, *HOST_SAN, *inc, "-c", "-x", "hip", src, "-o", obj], str(tmp_path))

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(compile_one, zip(srcs, objs)))
    exe = str(tmp_path / "host_san")
    run([HIPCC, *HOST_SAN, *objs, "-o", exe], str(tmp_path))
    r = run([exe], str(tmp_path))
    assert "host paths clean" in r.stdout
