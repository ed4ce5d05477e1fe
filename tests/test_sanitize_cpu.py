"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU: the FP64
oracle (tests/sanitize/oracle_driver.c, gcc) and the library's host runtime
(tests/sanitize/host_driver.cpp against a build of libvpmc whose host code,
and only its host code, carries the sanitizers).  Each driver exits 0 only
if every call returned what it should and no sanitizer reported."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2307_01416_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe,
          os.path.join(SAN, "oracle_driver.c"), "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="2"))
    assert "ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_runtime_under_sanitizers(tmp_path):
    lib = str(tmp_path / "libvpmc_san.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    srcs = [os.path.join(CSRC, s) for s in
            ("vpmc_kernels.hip", "vpmc_mlp.hip", "vpmc_opt.hip", "vpmc_api.cpp", "tables.cpp")]
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san + ["-o", lib] + srcs)
    exe = str(tmp_path / "host_driver")
    _run([HIPCC, "-O1", "-g", "-std=c++17"] + san +
         ["-o", exe, os.path.join(SAN, "host_driver.cpp"), "-L" + str(tmp_path), "-lvpmc_san",
          "-Wl,-rpath," + str(tmp_path)])
    r = _run([exe], env=dict(ENV, VPMC_SANITIZE_TMP=str(tmp_path)))
    assert "ok" in r.stdout
