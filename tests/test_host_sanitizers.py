"""The FP64 oracle and the host code of libjd under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

* The host library (argument validation, workspace sizing, the line-search
  driver, the request server's arena and failure paths) is compiled with g++
  and the sanitizers against host stand-ins for the HIP runtime and the kernel
  launchers (tests/sanitize/host_stubs.cpp) and driven by
  tests/sanitize/host_driver.cpp.
* The oracle is compiled with the sanitizers and its pin suites run against
  that build (the sanitizer runtime preloaded into the Python process).
* A planted heap overflow in a copy of the oracle must be reported, which shows
  that the sanitizer is live in these runs."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_04328_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]
PIN_SUITES = ["tests/test_oracle_model.py", "tests/test_oracle_rng.py", "tests/test_oracle_fb.py",
              "tests/test_oracle_adapted.py", "tests/test_oracle_coupled.py"]


def _runtime(name):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not found")
    return path


def _preload_env(lib):
    env = dict(os.environ, JD_ORACLE_LIB=lib, OMP_NUM_THREADS="4",
               LD_PRELOAD=f"{_runtime('libasan.so')} {_runtime('libubsan.so')}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return env


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    return tmp_path_factory.mktemp("san")


def test_host_library_under_sanitizers(tmp):
    if not shutil.which("g++") or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the HIP headers not found")
    exe = str(tmp / "host_driver")
    srcs = [os.path.join(CSRC, f) for f in ("jd_api.cpp", "jd_feedback.cpp", "jd_server.cpp",
                                             "jd_shapes.cpp")]
    srcs += [os.path.join(ROOT, "tests", "sanitize", f) for f in ("host_stubs.cpp",
                                                                  "host_driver.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-Wno-ignored-attributes", *srcs, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
                                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host checks passed" in r.stdout


def test_oracle_pins_under_sanitizers(tmp):
    from oracle import build
    lib = build.build(out=str(tmp / "liboracle_san.so"), extra=SAN)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *PIN_SUITES], cwd=ROOT, env=_preload_env(lib), capture_output=True,
                       text=True, timeout=900)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_sanitizer_reports_a_planted_overflow(tmp):
    """A copy of the oracle whose path buffers are one element short: the
    sanitized build must stop with a heap-buffer-overflow report."""
    from oracle import build
    src = open(os.path.join(ROOT, "oracle", "jd_oracle.c")).read()
    old = "double* Xs = (double*)malloc(stride * sizeof(double));"
    assert src.count(old) >= 1
    bad = tmp / "jd_oracle_overflow.c"
    bad.write_text(src.replace(old, "double* Xs = (double*)malloc((stride - 1) * sizeof(double));"))
    lib = build.build(src=[str(bad), os.path.join(ROOT, "oracle", "fb_oracle.c")],
                      out=str(tmp / "liboracle_overflow.so"),
                      extra=[*SAN, "-I" + os.path.join(ROOT, "oracle")])
    code = ("from oracle import ref\n"
            "from paper_2505_04328_amd import workloads as wl\n"
            "p = wl.general_problem(2, 10, seed=1)\n"
            "ref.cost_grad(p, 50, 1, 0, nthreads=1)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=_preload_env(lib),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
