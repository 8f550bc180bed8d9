"""Build the HIP library libdtn.so for gfx950 (in-tree)."""
import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdtn.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dtn.h")
SOURCES = ["dtn_wos.hip", "dtn_patch.hip", "dtn_points.hip", "dtn_tree.hip", "dtn_operators.cpp", "dtn_capi.cpp", "dtn_server.cpp"]


def hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


CALIB = os.path.join(HERE, "libdtn_calib.so")


def build_calib(verbose: bool = False, arch: str = "gfx950") -> str:
    """The issue-rate microbenchmarks (measurement support, own library)."""
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           os.path.join(CSRC, "calib.hip"), "-o", CALIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CALIB + ".tmp", CALIB)
    return CALIB


def header_digest(path: str = None) -> str:
    """First 16 hex digits of the SHA-256 of the C-ABI header.  The library
    carries the digest of the header it was built against (in
    dtn_version()), and the binding refuses a library whose digest differs
    from the header beside it: a stale build would otherwise be called with
    the argument lists of a newer header."""
    with open(HEADER if path is None else path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def build(verbose: bool = False, arch: str = "gfx950", extra=()) -> str:
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-pthread", f"-DDTN_HEADER_DIGEST=\"{header_digest()}\"",
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", LIB + ".tmp", *extra]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_calib(verbose=True))
