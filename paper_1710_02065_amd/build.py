"""Build the HIP library liblbm_hip.so for gfx950 (in-tree).

hipcc cross-compiles without a GPU.  All HIP sources are compiled with packed
FP32 instructions disabled.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = ["kernels.hip", "msweep.hip", "runtime.hip", "refine.hip", "serve.hip"]
ARCH = os.environ.get("HRLBM_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "-O3", "--offload-arch=" + ARCH, "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(HERE, "..", "include")]


def build(jobs: int = 4) -> str:
    """Compile every source and link the shared library; always rebuilds."""
    objs = []
    tmpdir = tempfile.mkdtemp(prefix="hrlbm_build_")
    procs = []
    for src in SOURCES:
        obj = os.path.join(tmpdir, src.replace(".hip", ".o"))
        log = open(obj + ".log", "w")  # a file, not a pipe: no back-pressure
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
        objs.append(obj)
        while len([p for p in procs if p[1].poll() is None]) >= jobs:
            next(p for p in procs if p[1].poll() is None)[1].wait()
    failed = []
    for src, p, log in procs:
        p.wait()
        log.close()
        with open(log.name, errors="replace") as f:
            lines = [l for l in f.read().splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write("\n".join(lines[-200:]) + "\n")
    if failed:
        raise RuntimeError("HIP compilation failed: %s" % ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs, check=True)
    os.replace(tmp, LIB)
    shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build())
