"""The library's host C++ under AddressSanitizer and UndefinedBehaviorSanitizer.

The host k-means (csrc/kmeans.hip, compiled host-only), community cores and
the block CG's dense algebra (csrc/dense.cpp) are built with both sanitizers
into a small program (tests/sanitize_host.cpp) that runs them on random and
degenerate inputs; any memory error, leak or undefined behaviour aborts it.
The step kernels' gather loop and work orders, host-callable in
csrc/device.hpp, get the same treatment (tests/step_host.cpp).
CPU only: no GPU code is built or run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1602_02018_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-ffp-contract=off"]


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    out = tmp_path_factory.mktemp("san")
    km = str(out / "kmeans.o")
    # host-only build of the k-means translation unit; the sanitizers apply
    # to the host code only
    subprocess.run([HIPCC, "--offload-host-only", *FLAGS,
                    "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined",
                    "-I", os.path.join(ROOT, "include"),
                    "-c", os.path.join(CSRC, "kmeans.hip"), "-o", km],
                   check=True, capture_output=True)
    objs = [km]
    for src, obj in ((os.path.join(CSRC, "dense.cpp"), "dense.o"),
                     (os.path.join(HERE, "sanitize_host.cpp"), "harness.o")):
        objs.append(str(out / obj))
        subprocess.run([CLANG, *FLAGS, "-fsanitize=address,undefined", "-c", src, "-o", objs[-1]],
                       check=True, capture_output=True)
    exe = str(out / "sanitize_host")
    subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", exe, *objs, "-lpthread"],
                   check=True, capture_output=True)
    return exe


@pytest.fixture(scope="module")
def step_host(tmp_path_factory):
    """Host build of the step kernels' gather loop and work orders
    (csrc/device.hpp's host-callable parts) with both sanitizers."""
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    out = tmp_path_factory.mktemp("step")
    obj, exe = str(out / "step_host.o"), str(out / "step_host")
    subprocess.run([HIPCC, "--offload-host-only", "-x", "hip", *FLAGS,
                    "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined",
                    "-I", os.path.join(ROOT, "include"),
                    "-c", os.path.join(HERE, "step_host.cpp"), "-o", obj],
                   check=True, capture_output=True)
    subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", exe, obj],
                   check=True, capture_output=True)
    return exe


def test_step_gather_loop_and_work_orders_under_sanitizers(step_host):
    """Every read of the gather loop stays inside its row's CSR segment and
    the gathered block, its sums equal a plain CSR-order loop bit for bit,
    and every XCD work order is a bijection (tests/step_host.cpp)."""
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([step_host], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "step host checks passed" in r.stdout


def test_host_code_is_clean_under_sanitizers(sanitized):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sanitized], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "sanitized host checks passed" in r.stdout


def test_sanitizer_build_catches_an_overflow(tmp_path):
    """The same flags turn an out-of-bounds read into a failed run."""
    if not os.path.exists(CLANG):
        pytest.skip("ROCm compilers not found")
    src = tmp_path / "oob.cpp"
    src.write_text("#include <vector>\nint main() { std::vector<int> v(4); return v.data()[4]; }\n")
    exe = tmp_path / "oob"
    subprocess.run([CLANG, "-O0", "-fsanitize=address,undefined", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr
