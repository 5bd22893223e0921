"""Host code under sanitizers (CPU): the cut (heap path and the threaded,
lock-free forest path) and the CPU oracle, built from source with g++ / gcc
and AddressSanitizer + UndefinedBehaviorSanitizer, and with ThreadSanitizer,
then run on seeded random inputs (tests/sanitize/san_main.cpp); and the
boundary and oracle-pin test files run against ASan+UBSan builds of the C ABI,
the cut and the oracle.  Only host sources are compiled with a sanitizer
here; no GPU code is."""
import os
import shutil
import subprocess
import sys

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


def test_boundary_and_oracle_pins_under_asan_ubsan(tmp_path):
    """tests/test_boundary.py and tests/test_oracle_pins.py against builds
    whose host code is instrumented: the C ABI and the cut (g++ with ASan and
    UBSan, linked with the GPU objects of the ordinary build, which are not
    rebuilt) and the oracle (gcc, OpenMP), loaded through NNM_LIB and
    ORACLE_LIB under a preloaded ASan runtime (the interpreter itself is not
    instrumented, so leak checking is off)."""
    build = os.path.join(ROOT, "paper_1402_3789_amd", "_build")
    gpu_objs = [os.path.join(build, f + ".o") for f in
                ("stage", "cand_mfma", "cand_fp32", "rescore", "merge", "sort_scan", "spatial",
                 "driver", "allpairs", "cut_dev", "autotune")]
    if not all(os.path.exists(o) for o in gpu_objs):
        pytest.skip("GPU objects not built (paper_1402_3789_amd/build.py)")
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined"]
    host_objs = []
    for f in CUT:
        o = tmp_path / (os.path.basename(f) + ".o")
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fPIC", *san, "-I",
                        os.path.join(ROOT, "include"), "-c", f, "-o", str(o)], check=True)
        host_objs.append(str(o))
    lib = tmp_path / "libnnm_san.so"
    subprocess.run(["g++", "-shared", *san, *host_objs, *gpu_objs, "-L/opt/rocm/lib",
                    "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", str(lib)], check=True)
    olib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", *san, ORACLE, "-o", str(olib), "-lm"], check=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True, check=True).stdout.strip()
    env = dict(os.environ)
    env.update(NNM_LIB=str(lib), ORACLE_LIB=str(olib), LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = ("import paper_1402_3789_amd._native as N, oracle; N.lib(); oracle._load(); "
             "m = open('/proc/self/maps').read(); "
             f"assert {str(lib)!r} in m and {str(olib)!r} in m")
    subprocess.run([sys.executable, "-c", probe], env=env, check=True, timeout=300)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_boundary.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
