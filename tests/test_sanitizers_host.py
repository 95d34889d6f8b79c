"""Sanitizer runs on the CPU (no GPU needed).

- the serving loop's admission rules (csrc/admission.h) checked with a fake
  clock and budget by tests/cpp/admission_check.cpp, built by g++ with
  AddressSanitizer and UndefinedBehaviorSanitizer;
- the oracle's own pin tests against an ASan/UBSan build of the oracle;
- the host runtime (argument checks, sensor validation, planning-free entry
  points, status strings) through tests/test_abi_host.py against
  libhabmi_san.so, the library with its host code instrumented.
Any sanitizer report fails the run (no recovery)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1904_01201_amd", "csrc")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout, cwd=ROOT)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_admission_rules_under_sanitizers(tmp_path):
    exe = str(tmp_path / "admission_check")
    _run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-Wall", "-Wextra", f"-I{CSRC}",
          os.path.join(ROOT, "tests", "cpp", "admission_check.cpp"), "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert r.stdout.strip() == "ok"


def _preload(compiler_args):
    out = subprocess.run(compiler_args, capture_output=True, text=True).stdout.strip()
    if not out or not os.path.exists(out):
        pytest.skip(f"sanitizer runtime not found ({compiler_args})")
    return out


def test_oracle_pins_under_sanitizers():
    asan = _preload(["gcc", "-print-file-name=libasan.so"])
    env = dict(os.environ, ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
          "tests/test_oracle_pins.py", "tests/test_oracle_nav.py", "tests/test_oracle_actuation.py",
          "tests/test_oracle_texture.py", "tests/test_oracle_noise.py"], env=env, timeout=900)


def test_host_runtime_under_sanitizers():
    from paper_1904_01201_amd import build as hb
    lib = hb.build(sanitize=True)
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    asan = _preload([clang, "-print-file-name=libclang_rt.asan-x86_64.so"])
    env = dict(os.environ, HABMI_LIBRARY=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
          "tests/test_abi_host.py"], env=env, timeout=900)
