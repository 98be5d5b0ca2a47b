"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the FP64 oracle driven
through every routine, and the host side of libsal (argument validation, stencil resolution,
line templates, constant-table building) driven through its C ABI with the device launches
stubbed out.  Any out-of-bounds access, leak or undefined operation fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    return r.returncode, r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_asan")
    rc, out = _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "sal_oracle.c"), os.path.join(HERE, "oracle_driver.c"), "-o", exe,
                    "-lm"])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="2")
    rc, out = _run([exe], env=env, timeout=300)
    print(out[-3000:])
    assert rc == 0 and "ORACLE_SANITIZE_OK" in out and "runtime error" not in out


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_libsal_host_code_under_sanitizers(tmp_path):
    """libsal's host files (sal_host.cpp, sal_api.cpp) with the sanitizers on the host side
    only (each -fsanitize behind -Xarch_host; the device code is built as usual), linked with
    stand-ins for the device launches and driven through the C ABI."""
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    from concurrent.futures import ThreadPoolExecutor
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san
    srcs = [os.path.join(ROOT, "paper_2201_06174_amd", "csrc", "sal_host.cpp"),
            os.path.join(ROOT, "paper_2201_06174_amd", "csrc", "sal_api.cpp"),
            os.path.join(HERE, "host_stubs.cpp"), os.path.join(HERE, "host_driver.cpp")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        return _run([HIPCC] + flags + ["-c", src, "-o", obj]) + (obj,)

    with ThreadPoolExecutor(4) as ex:
        results = list(ex.map(compile_one, srcs))
    for rc, out, _ in results:
        assert rc == 0, out
    exe = str(tmp_path / "host_asan")
    rc, out = _run([HIPCC, "--offload-arch=gfx950"] + san + [r[2] for r in results] +
                   ["-o", exe, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    assert rc == 0, out
    # the HIP runtime keeps allocations for the process's lifetime; leaks are the oracle test's job
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    rc, out = _run([exe], env=env, timeout=300)
    print(out[-3000:])
    assert rc == 0 and "HOST_SANITIZE_OK" in out and "runtime error" not in out
