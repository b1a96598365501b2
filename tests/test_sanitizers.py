"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Builds tests/sanitize_driver.cpp with the FP64 oracle (oracle/oracle.c) and
the library's host-only sources (the system-kernel builder and the geometry
validation) using g++/gcc with -fsanitize=address,undefined, and runs it: any
out-of-bounds access, use after free, leak or undefined behaviour aborts the
driver, and the driver itself checks identities, the dot test of the oracle
and the error codes of the validation.  The device code is not built here."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2609_29253_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    objs = []
    o = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", *SAN, "-c",
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", o], check=True)
    objs.append(o)
    for src in ("kernel_builder.cpp", "geometry.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run(["g++", "-std=c++17", *SAN, *inc, "-c", os.path.join(csrc, src), "-o", o], check=True)
        objs.append(o)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", "-std=c++17", *SAN, *inc, os.path.join(ROOT, "tests", "sanitize_driver.cpp"), *objs,
                    "-fopenmp", "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(res.stdout[-2000:], res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr
    assert "sanitized host checks passed" in res.stdout
