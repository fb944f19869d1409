"""Compile the HIP library librkc.so for gfx950 (hipcc, in-tree).

Every translation unit under csrc/ is compiled in parallel, then linked into
paper_1309_2710_amd/librkc.so.  The packed-FP32 instructions are disabled for
all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librkc.so")
PROBE_SRC = os.path.join(CSRC, "probe", "fp64_peak.hip")
PROBE_LIB = os.path.join(HERE, "librkc_probe.so")
ARCH = os.environ.get("RKC_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -ffp-contract=on: a multiply and an add are fused only inside one source
# expression, so every kernel variant that shares an expression rounds it the
# same way (the default also fuses across statements, depending on context).
CFLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=on",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall",
          "-Wno-unused-variable", "-Wno-unused-function"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
    if verbose and r.stderr.strip():
        print(r.stderr[-3000:], flush=True)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # the FP64 throughput probe of the roofline (bench.py --peak), its own library
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, *CFLAGS, "-shared", PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, PROBE_LIB)
    return LIB


def ensure_built():
    """Build the library only if none is built (the tests, the smoke check and
    the benchmark load what is there; build() always recompiles)."""
    if not os.path.exists(LIB) or not os.path.exists(PROBE_LIB):
        print("librkc.so not found: building it for %s" % ARCH, flush=True)
        build()
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
