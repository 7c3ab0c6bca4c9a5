"""Build the HIP library (gfx950) in-tree: ``libsabr_hip.so`` next to this file.

Each source compiles to its own object (in parallel, under ``_build/``) and
the objects link into the shared library; no device code crosses a source
file, so no relocatable device code is needed."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsabr_hip.so")
OBJDIR = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["sabr_kernels.hip", "sabr_adjoint.hip", "sabr_nm.hip", "sabr_mc.hip", "sabr_api.cpp"]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere (the kernels are FP64)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


LAUNCH_MARKER = b"// Launch wrappers"


def source_digest() -> str:
    """SHA-256 over the device code of the annealing kernels: every header
    under csrc/ and sabr_kernels.hip up to its host-side launch wrappers, in
    name order.  Identifies the kernel build that a set of hardware counters
    of those kernels belongs to (the adjoint's kernels, the host runtime and
    the pricing program do not enter)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if not (name.endswith(".hpp") or name == "sabr_kernels.hip") or name == "sabr_adjoint.hpp":
            continue
        with open(os.path.join(CSRC, name), "rb") as fh:
            text = fh.read()
        if name == "sabr_kernels.hip":
            cut = text.find(LAUNCH_MARKER)
            assert cut > 0, "launch wrapper marker missing"
            text = text[:cut]
        h.update(name.encode())
        h.update(text)
    return h.hexdigest()


CALIB_SRC = os.path.join(CSRC, "elementary_calib.hip")
CALIB_BIN = os.path.join(HERE, "elementary_calib")


def build_calib(hipcc: str | None = None) -> str:
    """The elementary-function pricing program (profiling only; not part of
    build())."""
    hipcc = hipcc or os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    res = subprocess.run([hipcc, *HIPCC_FLAGS, "-o", CALIB_BIN + ".tmp", CALIB_SRC],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(CALIB_BIN + ".tmp", CALIB_BIN)
    return CALIB_BIN


def _compile(hipcc: str, src: str) -> tuple[str, str]:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    res = subprocess.run([hipcc, *HIPCC_FLAGS, "-c", "-o", obj + ".tmp", src],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n" + res.stdout + res.stderr)
    os.replace(obj + ".tmp", obj)
    return obj, res.stderr


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    jobs = min(len(srcs), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        done = list(ex.map(lambda s: _compile(hipcc, s), srcs))
    if verbose:
        for _, err in done:
            print(err)
    tmp = LIB + ".tmp"
    res = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp,
                          *[o for o, _ in done]], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
