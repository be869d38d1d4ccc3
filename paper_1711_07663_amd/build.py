"""Compile the HIP library (gfx950) into paper_1711_07663_amd/liboc.so, and
its checked variant (OC_CHECKED: the CSR walks validate every index against
the array it reads and record violations in the context's check word) into
liboc_checked.so.

Each translation unit is compiled with hipcc in parallel, then linked into
one shared library.  Packed FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liboc.so")
LIB_CHECKED = os.path.join(HERE, "liboc_checked.so")
SOURCES = ["oc_api.hip", "k_cut.hip", "k_donor.hip", "k_scan.hip", "k_unblank.hip", "k_ab.hip", "k_heur.hip",
           "oc_service.hip", "k_refined.hip"]
ARCH = os.environ.get("OC_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-Wno-pass-failed"]


def _compile(job):
    src, checked = job
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ("_checked.o" if checked else ".o"))
    cmd = [hipcc(), *FLAGS, *(["-DOC_CHECKED"] if checked else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj, r.stderr


def _link(objs, lib):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, lib)


def build(verbose=False):
    """Both variants; returns the path of the product library."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(s, False) for s in SOURCES] + [(s, True) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=min(len(jobs), 16)) as ex:
        res = list(ex.map(_compile, jobs))
    if verbose:
        for obj, err in res:
            if err.strip():
                sys.stderr.write(err)
    n = len(SOURCES)
    _link([o for o, _ in res[:n]], LIB)
    _link([o for o, _ in res[n:]], LIB_CHECKED)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
