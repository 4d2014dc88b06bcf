"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU.

* The oracle (plain C) built with both sanitizers and driven through its entry
  points on small inputs in every n and dimension (tests/sanitize/oracle_driver.c).
* The host side of the C ABI (mbo_api.cpp) built with the sanitizers on its host
  code only, linked with the library's kernel objects, and driven through the
  argument checks that run before any device work, without a GPU
  (tests/sanitize/abi_driver.cpp).

A sanitizer report makes the program exit non-zero (-fno-sanitize-recover).
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-std=c11", "-fopenmp"] + SAN + ["-o", exe, os.path.join(ROOT, "oracle", "mbo_oracle.c"),
                                                  os.path.join(HERE, "oracle_driver.c"), "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="2"))
    assert "oracle driver done rc=0" in r.stdout


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not installed")
def test_abi_argument_checks_under_address_and_ub_sanitizers(tmp_path):
    from paper_1711_01365_amd import build as hip_build
    objs = [o for o in glob.glob(os.path.join(hip_build.BUILD_DIR, "*.o"))
            if not o.endswith("mbo_api.o")]
    if len(objs) < len(hip_build.SOURCES) - 1:
        hip_build.build()
        objs = [o for o in glob.glob(os.path.join(hip_build.BUILD_DIR, "*.o")) if not o.endswith("mbo_api.o")]
    hipcc = hip_build.hipcc()
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f] if f.startswith("-fsanitize") or f.startswith("-fno-sanitize") else [f]
    api_o = str(tmp_path / "mbo_api_san.o")
    _run([hipcc] + hip_build.flags() + host_san + ["-x", "hip", "-c",
                                                   os.path.join(hip_build.CSRC, "mbo_api.cpp"), "-o", api_o])
    drv_o = str(tmp_path / "abi_driver.o")
    _run(["g++", "-std=c++17", "-I", hip_build.INCLUDE] + SAN + ["-c", os.path.join(HERE, "abi_driver.cpp"),
                                                                  "-o", drv_o])
    exe = str(tmp_path / "abi_asan")
    _run([hipcc, "--offload-arch=gfx950", "-fsanitize=address,undefined", "-o", exe, drv_o, api_o] + objs)
    r = _run([exe], env=ENV)
    assert "abi driver done bad=0" in r.stdout
