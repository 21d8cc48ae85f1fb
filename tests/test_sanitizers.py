"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (no GPU).

Two host-only parts are rebuilt with the sanitizers and driven by their own
CPU tests in a child process: the server's scheduling core (serve_core.h,
through the simulated-device driver serve_sim.cpp) and the FP64 oracle's
projector (siddon.c, OpenMP).  Any out-of-bounds access, use after free or
undefined behaviour aborts the child with a sanitizer report.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def san_libs(tmp_path_factory):
    if shutil.which("gcc") is None or shutil.which("g++") is None or not _runtime("libasan.so"):
        pytest.skip("gcc with the sanitizer runtimes is not available")
    d = tmp_path_factory.mktemp("san")
    sim = str(d / "libcbct_sim_san.so")
    orc = str(d / "liboracle_san.so")
    subprocess.run(["g++", "-std=c++17", "-fPIC", "-shared", *SAN,
                    f"-I{os.path.join(ROOT, 'include')}",
                    os.path.join(ROOT, "paper_2509_08574_amd", "csrc", "serve_sim.cpp"),
                    "-o", sim], check=True)
    subprocess.run(["gcc", "-std=c11", "-fPIC", "-shared", "-fopenmp", *SAN,
                    os.path.join(ROOT, "oracle", "siddon.c"), "-o", orc, "-lm"], check=True)
    return sim, orc


def test_host_code_is_clean_under_asan_and_ubsan(san_libs):
    sim, orc = san_libs
    env = dict(os.environ)
    # the sanitizer runtime first; libstdc++ up front too, so that its exception
    # entry points exist when the runtime's interceptors resolve them (the
    # scheduler's tests throw and catch simulated launch failures)
    env["LD_PRELOAD"] = " ".join(p for p in (_runtime("libasan.so"),
                                             _runtime("libstdc++.so.6")) if p)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["CBCT_SIM_LIB"] = sim
    env["CBCT_ORACLE_LIB"] = orc
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_serve_core.py"),
                        os.path.join(ROOT, "tests", "test_oracle_projector.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
