"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

* The FP64 oracle (oracle/mrt_oracle.c), built with gcc -fsanitize=address,undefined,
  runs every boundary kind, a porosity field with a free-fluid cell, a per-node J plane
  and the thermal coupling (tests/sanitize/oracle_driver.c).
* The library's C ABI (lbm_abi.cpp, its host code built with the sanitizers, linked with
  the kernel objects of the normal build) takes valid and invalid descriptors, workspace
  sizing, the refusal paths of lbm_create and lbm_create_batch, and calls on NULL
  contexts (tests/sanitize/abi_driver.cpp).
Leak detection is on in both. Each driver exits 0 only when every call returned what
the header promises; a sanitizer report aborts it."""
import os
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent
SAN = ROOT / "tests" / "sanitize"
CSRC = ROOT / "paper_1311_7239_amd" / "csrc"
BUILD = ROOT / "paper_1311_7239_amd" / "_build"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    r = _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-fopenmp", "-I", str(ROOT / "oracle"),
              str(ROOT / "oracle" / "mrt_oracle.c"), str(SAN / "oracle_driver.c"), "-lm", "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failing cases" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_host_code_under_address_and_ub_sanitizers(tmp_path):
    kernels = [BUILD / "lbm_kernels.hip.o", BUILD / "lbm_adjoint.hip.o"]
    if not all(k.exists() for k in kernels):
        pytest.skip("kernel objects not built (run paper_1311_7239_amd.build first)")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    common = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-I", str(ROOT / "include")]
    abi_o, drv_o, exe = tmp_path / "abi.o", tmp_path / "drv.o", tmp_path / "abi_asan"
    r = _run([HIPCC, "--offload-arch=gfx950", *common, "-fPIC", "-ffp-contract=off", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", *san, "-x", "hip", "-I", str(CSRC), "-c",
              str(CSRC / "lbm_abi.cpp"), "-o", str(abi_o)])
    assert r.returncode == 0, r.stderr
    r = _run([HIPCC, *common, *san, "-c", str(SAN / "abi_driver.cpp"), "-o", str(drv_o)])
    assert r.returncode == 0, r.stderr
    r = _run([HIPCC, "--offload-arch=gfx950", *san, str(drv_o), str(abi_o), *map(str, kernels), "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
