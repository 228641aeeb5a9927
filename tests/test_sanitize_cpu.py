"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

* The FP64 oracle (oracle/mrt_oracle.c), built with gcc -fsanitize=address,undefined,
  runs every boundary kind, a porosity field with a free-fluid cell, a per-node J plane
  and the thermal coupling (tests/sanitize/oracle_driver.c).
* The library's C ABI (lbm_abi.cpp, its host code built with the sanitizers, linked with
  the kernel objects of the normal build) takes valid and invalid descriptors, workspace
  sizing, the refusal paths of lbm_create and lbm_create_batch, and calls on NULL
  contexts (tests/sanitize/abi_driver.cpp).
* Fault injection through a null device (tests/sanitize/null_device.cpp, test code only):
  the same host code and the kernel objects' launch stubs run on a fake HIP runtime in host
  memory, where launches are recorded and not executed. A NaN injected into a population
  gives LBM_EUNSTABLE, an injected HIP failure poisons the context, calls out of order get
  the status the header names, and a second lbm_destroy is refused
  (tests/sanitize/null_driver.cpp).
Leak detection is on in all three. Each driver exits 0 only when every call returned what
the header promises; a sanitizer report aborts it."""
import os
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent
SAN_DIR = ROOT / "tests" / "sanitize"
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
              str(ROOT / "oracle" / "mrt_oracle.c"), str(SAN_DIR / "oracle_driver.c"), "-lm", "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failing cases" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


HAVE_HIPCC = bool(shutil.which(HIPCC)) or os.path.exists(HIPCC)
KERNELS = [BUILD / "lbm_kernels.hip.o", BUILD / "lbm_adjoint.hip.o"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
COMMON = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-I", str(ROOT / "include")]
CLANG = pathlib.Path(HIPCC).resolve().parent.parent / "llvm" / "bin" / "clang++"


@pytest.fixture(scope="module")
def abi_asan_object(tmp_path_factory):
    """lbm_abi.cpp with its host code built under the sanitizers (device code as usual)."""
    if not HAVE_HIPCC:
        pytest.skip("hipcc not available")
    if not all(k.exists() for k in KERNELS):
        pytest.skip("kernel objects not built (run paper_1311_7239_amd.build first)")
    obj = tmp_path_factory.mktemp("abi") / "abi.o"
    r = _run([HIPCC, "--offload-arch=gfx950", *COMMON, "-fPIC", "-ffp-contract=off", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", *SAN, "-x", "hip", "-I", str(CSRC), "-c",
              str(CSRC / "lbm_abi.cpp"), "-o", str(obj)])
    assert r.returncode == 0, r.stderr
    return obj


def test_abi_host_code_under_address_and_ub_sanitizers(tmp_path, abi_asan_object):
    drv_o, exe = tmp_path / "drv.o", tmp_path / "abi_asan"
    r = _run([HIPCC, *COMMON, *SAN, "-c", str(SAN_DIR / "abi_driver.cpp"), "-o", str(drv_o)])
    assert r.returncode == 0, r.stderr
    r = _run([HIPCC, "--offload-arch=gfx950", *SAN, str(drv_o), str(abi_asan_object), *map(str, KERNELS),
              "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_fault_injection_through_the_null_device(tmp_path, abi_asan_object):
    if not CLANG.exists():
        pytest.skip("ROCm clang++ not found")
    dev_o, drv_o, exe = tmp_path / "null_device.o", tmp_path / "null_driver.o", tmp_path / "null_asan"
    r = _run([HIPCC, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", *COMMON, "-fPIC", *SAN,
              "-I", str(CSRC), "-c", str(SAN_DIR / "null_device.cpp"), "-o", str(dev_o)])
    assert r.returncode == 0, r.stderr
    r = _run([str(CLANG), *COMMON, "-fsanitize=address,undefined", "-c", str(SAN_DIR / "null_driver.cpp"),
              "-o", str(drv_o)])
    assert r.returncode == 0, r.stderr
    # linked without the HIP runtime: every HIP symbol resolves to the null device
    r = _run([str(CLANG), "-fsanitize=address,undefined", str(drv_o), str(abi_asan_object), str(dev_o),
              *map(str, KERNELS), "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "null-device driver: 0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
