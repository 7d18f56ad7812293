"""Build libhexval.so (HIP for gfx950) in-tree.

    python -m paper_1706_01613_amd.build

Every source is compiled with hipcc for gfx950 only, packed FP32 disabled, no
floating-point contraction (the kernels' error bounds assume exactly the
roundings written in the source; fused operations are explicit fma calls).
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhexval.so")
EMUL = os.path.join(HERE, "libhexval_emul.so")
LOADGEN = os.path.join(HERE, "libhexval_loadgen.so")
CALIB = os.path.join(HERE, "libhexval_calib.so")

SOURCES = ["hexval_kernels.hip", "hexval_runtime.hip", "hexval_exact.cpp", "hexval_server.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=4):
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="hexval_build_")
    try:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [cc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, *lang, "-c",
                   os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd), src))
            objs.append(obj)
        for p, src in procs:
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {src}")
        out = LIB + ".tmp"
        cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out, "-lpthread"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(out, LIB)
        # CPU replay of the kernels' per-element arithmetic (test support only)
        out = EMUL + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
               "-I", CSRC, os.path.join(CSRC, "host_emul.cpp"), os.path.join(CSRC, "hexval_exact.cpp"),
               "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(out, EMUL)
        # open-loop request generator for the server (benchmark/test driver)
        out = LOADGEN + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", INCLUDE,
               os.path.join(CSRC, "hexval_loadgen.cpp"), "-L", HERE, "-lhexval",
               "-Wl,-rpath,$ORIGIN", "-lpthread", "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(out, LOADGEN)
        # machine ceilings (HBM read, copy, FP64 FMA) for the benchmark
        out = CALIB + ".tmp"
        cmd = [cc, *HIPCC_FLAGS, "-I", INCLUDE, "-shared", "-x", "hip",
               os.path.join(CSRC, "hexval_calib.hip"), "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(out, CALIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
