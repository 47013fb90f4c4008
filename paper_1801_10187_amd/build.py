"""Build libmpcd.so in-tree with hipcc for gfx950.

    python -m paper_1801_10187_amd.build        (or build() from Python)

Flags that matter for results:
  -ffp-contract=off   every floating-point operation rounds once, in the
                      order written (stream, binning and the fixed-point
                      split rely on it);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "mpcd.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "mpcd_kernels.hpp"),
        os.path.join(HERE, "csrc", "mpcd_device.hpp"),
        os.path.join(ROOT, "include", "mpcd.h"),
        os.path.join(HERE, "csrc", "mpcd_md.hpp"),
        os.path.join(HERE, "csrc", "mpcd_emb.hpp")]
LIB = os.path.join(HERE, "libmpcd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def source_hash():
    """SHA-256 over the library sources and header (identifies the kernels a
    measurement was taken on)."""
    import hashlib
    h = hashlib.sha256()
    for f in DEPS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_hash():
    """SHA-256 over the device-code sources only (the kernels and their
    launch shapes): identifies the kernels a counter measurement was taken
    on, unchanged by host-side edits."""
    import hashlib
    h = hashlib.sha256()
    for f in DEPS[1:3]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose=False):
    """Compile the library (always; a fresh build each call)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmpcd.so")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
