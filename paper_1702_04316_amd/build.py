"""Build the HIP library ``libnuma_hevi.so`` in-tree for gfx950 with hipcc.

Each source is compiled to its own object in parallel (the sources share no
device symbols, so no relocatable device code is needed), then the objects
are linked into the shared library.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnuma_hevi.so")
SOURCES = ["abi.cpp", "setup.cpp", "ensemble.cpp", "kernels.hip", "rhs_alt.hip", "imex3d.hip", "learned.hip",
           "colstd.hip"]
ARCH = "gfx950"
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the GPU-only feature flag; that warning is noise
    lines = [l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l]
    return res.returncode, "\n".join(lines)


def build(verbose=False, extra=(), jobs=None):
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="numa_build_")
    try:
        objs, cmds = [], []
        for s in SOURCES:
            o = os.path.join(tmp, os.path.splitext(s)[0] + ".o")
            objs.append(o)
            cmds.append([cc] + FLAGS + list(extra) + ["-c", os.path.join(CSRC, s), "-o", o])
        jobs = jobs or min(len(cmds), os.cpu_count() or 1, 16)
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), cmds))
        failed = False
        for (rc, text), s in zip(results, SOURCES):
            if text:
                print(text, flush=True)
            if rc != 0:
                print(f"hipcc failed on {s} with exit code {rc}", flush=True)
                failed = True
        if failed:
            raise RuntimeError("hipcc failed")
        out = LIB + ".tmp"
        rc, text = _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + objs, verbose)
        if text:
            print(text, flush=True)
        if rc != 0:
            raise RuntimeError(f"hipcc link failed with exit code {rc}")
        os.replace(out, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
