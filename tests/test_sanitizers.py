"""CPU AddressSanitizer and UndefinedBehaviorSanitizer builds (no GPU):

* the oracle (g++ with -fsanitize=address,undefined), driven through every
  entry point on small problems;
* the HIP library with its host code sanitized (hipcc -Xarch_host
  -fsanitize=...; the device code is unchanged), driven through the
  host-side plan validation and packing, the refusals of bad input and the
  Monte Carlo plan's host factor.

Each runs in a child process with the sanitizer runtime preloaded; any
report aborts it."""
import os
import shutil
import subprocess
import sys

import pytest

from conftest import ROOT

DRIVER = os.path.join(ROOT, "tests", "sanitized_driver.py")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer"]


def _runtime():
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True,
                           text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"{name} not available")
        libs.append(p)
    return libs


def _run(kind, lib, tmp_path):
    env = dict(os.environ)
    env["LD_PRELOAD"] = ":".join(_runtime())
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, DRIVER, kind, str(lib)], capture_output=True, text=True,
                       env=env, cwd=str(tmp_path), timeout=600)
    assert r.returncode == 0 and f"{kind} ok" in r.stdout, r.stdout[-3000:] + r.stderr[-6000:]
    assert "runtime error" not in r.stderr, r.stderr[-6000:]


def test_oracle_under_asan_ubsan(tmp_path):
    _runtime()
    lib = tmp_path / "liboracle_san.so"
    src = os.path.join(ROOT, "oracle", "sabr_oracle.cpp")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-fno-fast-math", *SAN, "-o", str(lib), src],
                   check=True)
    _run("oracle", lib, tmp_path)


def test_hip_host_code_under_asan_ubsan(tmp_path):
    _runtime()
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_2408_01470_amd import build as B
    objs = [os.path.join(B.OBJDIR, s + ".o") for s in B.SOURCES if s != "sabr_api.cpp"]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built")
    api_obj = tmp_path / "sabr_api_san.o"
    flags = [f for f in B.HIPCC_FLAGS]
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    subprocess.run([hipcc, *flags, *host_san, "-c", "-o", str(api_obj),
                    os.path.join(B.CSRC, "sabr_api.cpp")], check=True, capture_output=True)
    lib = tmp_path / "libsabr_hip_san.so"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *host_san, "-o",
                    str(lib), str(api_obj), *objs], check=True, capture_output=True)
    _run("host", lib, tmp_path)
