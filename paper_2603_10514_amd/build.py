"""Build libchase.so (the gfx950 HIP library behind include/chase.h) in place.

    python paper_2603_10514_amd/build.py        (or __graft_entry__.build())

(Run as a script: `python -m` would import the package, which loads the
previous libchase.so.)

Compiles every source under csrc/ with hipcc for gfx950 (no vendor math
library is linked).  Always recompiles; the output lands next to this file."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchase.so")
SOURCES = ["kernels.hip", "eig.hip", "solver.cpp", "abi.cpp", "noalloc.cpp"]
ARCH = os.environ.get("CHASE_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=3, defines=(), out=None):
    cc = hipcc()
    flags = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
             "-Wno-unused-result",
             # MFMA accumulators in arch VGPRs: no AGPR round trips per K chunk
             "-mllvm", "--amdgpu-mfma-vgpr-form"] + ["-D" + d for d in defines]
    lib = out or LIB
    objdir = os.path.join(HERE, "_build", os.path.basename(lib))
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".", "_") + ".o")
        objs.append(obj)
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [cc] + flags + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs, verbose)
    _drain(procs, verbose)
    tmp = lib + ".tmp"
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    _run(cmd, verbose)
    os.replace(tmp, lib)
    return lib


def _run(cmd, verbose):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if verbose or r.returncode != 0:
        sys.stdout.write(_filter(r.stdout))
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd))


def _drain(procs, verbose):
    failed = None
    for cmd, p in procs:
        out, _ = p.communicate()
        out = out.decode(errors="replace")
        if verbose or p.returncode != 0:
            sys.stdout.write(_filter(out))
        if p.returncode != 0 and failed is None:
            failed = cmd
    procs.clear()
    if failed:
        raise RuntimeError("compile failed: " + " ".join(failed))


def _filter(text):
    # hipcc's host pass does not know the packed-fp32 target feature; harmless
    return "".join(l for l in text.splitlines(True) if "packed-fp32-ops" not in l)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
