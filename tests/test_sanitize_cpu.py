"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C code driven over small problems of every kind
(tests/sanitize/oracle_driver.c), and the library's host-only paths --
configuration checks, level shapes, workspace layout and the argument
checks made before any device work (tests/sanitize/abi_driver.cpp) -- with
the library's host code instrumented and its device code untouched."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ("address", "undefined")


def _run(exe, leaks=True):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={1 if leaks else 0}:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=" + ",".join(SAN), "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), "-o", exe,
           os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "tomg_oracle.c"),
           "-lm"]
    subprocess.run(cmd, check=True, timeout=300)
    r = _run(exe)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all cases ran" in r.stdout


def test_library_host_paths_under_sanitizers(tmp_path):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hip = os.path.join(rocm, "bin", "hipcc")
    clang = os.path.join(rocm, "llvm", "bin", "clang++")
    if not (os.path.exists(hip) and os.path.exists(clang)):
        pytest.skip("no ROCm toolchain")
    from paper_2602_01888_amd import build
    objdir = os.path.join(ROOT, "paper_2602_01888_amd", "_build")
    others = [os.path.join(objdir, s + ".o") for s in ("kernels.hip", "fused.hip", "tail.hip")]
    if not all(os.path.exists(o) for o in others):
        build.build()
    host_san = []
    for s in SAN:  # host code only: the device code is built as usual
        host_san += ["-Xarch_host", "-fsanitize=" + s]
    api = str(tmp_path / "api.o")
    subprocess.run([hip, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san +
                   ["-Xarch_host", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2602_01888_amd", "csrc"),
                    "-c", os.path.join(ROOT, "paper_2602_01888_amd", "csrc", "api.hip"),
                    "-o", api], check=True, timeout=600)
    drv = str(tmp_path / "abi_driver.o")
    san = "-fsanitize=" + ",".join(SAN)
    subprocess.run([clang, "-O1", "-g", "-std=c++17", san, "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(HERE, "abi_driver.cpp"), "-o", drv], check=True, timeout=300)
    exe = str(tmp_path / "abi_driver")
    subprocess.run([clang, san, "-o", exe, drv, api] + others +
                   ["-L", os.path.join(rocm, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + os.path.join(rocm, "lib")], check=True, timeout=300)
    r = _run(exe)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks ran" in r.stdout
