"""Build the gfx950 shared library libdugks.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libdugks.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# every HIP source of the library (csrc/*.hip)
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
HEADERS = ["dugks_common.h", "dugks_kernels.h", "dugks_plan.h", "dugks_batch_impl.h"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # every a*b+c rounds as written or through an explicit fma(): the same
    # expression gives the same bits in every inlined copy, so results do not
    # depend on the tile shape (or on a grid being alone or in a batch)
    "-ffp-contract=off",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def _messages(text: str) -> list:
    # the host pass warns that it does not know the device-only feature flag
    return [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]


def build(verbose: bool = False) -> str:
    """Compile every source into libdugks.so (always rebuilds): the sources
    are compiled in parallel to objects, then linked."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        procs.append(_run([HIPCC, *FLAGS, "-c", *inc, os.path.join(CSRC, src), "-o", obj],
                          verbose))
    failed = False
    for pr in procs:
        out, _ = pr.communicate()
        msgs = _messages(out or "")
        if pr.returncode != 0:
            failed = True
            sys.stderr.write("\n".join(msgs) + "\n")
        elif verbose and msgs:
            print("\n".join(msgs))
    if failed:
        raise RuntimeError("hipcc failed building libdugks.so")
    tmp = LIB + ".tmp"
    link = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    out, _ = link.communicate()
    if link.returncode != 0:
        sys.stderr.write("\n".join(_messages(out or "")) + "\n")
        raise RuntimeError("hipcc failed linking libdugks.so")
    for obj in objs:
        os.remove(obj)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
