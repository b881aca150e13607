"""Build libdpd.so (HIP, gfx950) in-tree.

    python -m paper_1612_09001_amd.build

Every translation unit is compiled by hipcc for gfx950 only, in parallel, then
linked into ``paper_1612_09001_amd/libdpd.so``.  Packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdpd.so")
OBJDIR = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I" + INCLUDE, "-I" + CSRC,
]

# (source, extra defines, object name)
UNITS = [("dpd_api.hip", [], "dpd_api.o")]
UNITS += [("dpd_fwd_inst.hip", ["-DDPD_NI=%d" % k], "dpd_fwd_ni%d.o" % k) for k in range(1, 9)]
UNITS += [("dpd_bwd_inst.hip", ["-DDPD_NI=%d" % k], "dpd_bwd_ni%d.o" % k) for k in range(1, 9)]
UNITS += [("dpd_bwd.hip", [], "dpd_bwd.o")]
UNITS += [("dpd_batch_inst.hip", ["-DDPD_BATCH_S=%d" % s], "dpd_batch_s%d.o" % s) for s in (2, 4, 8)]
UNITS += [("dpd_batch.hip", [], "dpd_batch.o")]
UNITS += [("dpd_train.hip", [], "dpd_train.o")]
UNITS += [("dpd_transmit.hip", [], "dpd_transmit.o")]
UNITS += [("dpd_transmit_bwd.hip", [], "dpd_transmit_bwd.o")]
UNITS += [("dpd_ls.hip", [], "dpd_ls.o")]


def _compile(unit):
    src, defs, obj = unit
    out = os.path.join(OBJDIR, obj)
    cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return out


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
