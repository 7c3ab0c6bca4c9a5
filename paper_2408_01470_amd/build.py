"""Build the HIP library (gfx950) in-tree: ``libsabr_hip.so`` next to this file."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsabr_hip.so")
SOURCES = ["sabr_kernels.hip", "sabr_adjoint.hip", "sabr_nm.hip", "sabr_mc.hip", "sabr_api.cpp"]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
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


def build_calib(hipcc: str) -> str:
    """The elementary-function pricing program (profiling only)."""
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    res = subprocess.run([hipcc, *flags, "-o", CALIB_BIN + ".tmp", CALIB_SRC], capture_output=True,
                         text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(CALIB_BIN + ".tmp", CALIB_BIN)
    return CALIB_BIN


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    build_calib(hipcc)
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *srcs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
