"""Host code under sanitizers (CPU): the cut (heap path and the threaded,
lock-free forest path) and the CPU oracle, built from source with g++ / gcc
and AddressSanitizer + UndefinedBehaviorSanitizer, and with ThreadSanitizer,
then run on seeded random inputs (tests/sanitize/san_main.cpp).  Only host
sources are compiled here; no GPU code is built with a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "sanitize", "san_main.cpp")
CUT = [os.path.join(ROOT, "paper_1402_3789_amd", "csrc", f) for f in ("cut.cpp", "capi.cpp")]
ORACLE = os.path.join(ROOT, "oracle", "oracle.c")


def _build_and_run(tmp_path, flags, name, omp):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    obj = tmp_path / f"oracle_{name}.o"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", *flags, *omp, "-c", ORACLE,
                    "-o", str(obj)], check=True)
    exe = tmp_path / f"san_{name}"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *flags, "-I", os.path.join(ROOT, "include"),
                    HARNESS, *CUT, str(obj), "-o", str(exe), *omp, "-lpthread", "-lm"], check=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    r = subprocess.run([str(exe), "4" if omp else "1"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitizer harness ok" in r.stdout
    assert "runtime error" not in r.stderr and "WARNING: ThreadSanitizer" not in r.stderr, r.stderr


def test_cut_and_oracle_under_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                              "-fno-sanitize-recover=undefined"], "asan", ["-fopenmp"])


def test_cut_and_oracle_under_tsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], "tsan", [])
