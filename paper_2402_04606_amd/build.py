"""Build libsbt.so (HIP kernels + host engine + C ABI) for gfx950 with hipcc."""
import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
LIB = os.path.join(_HERE, "libsbt.so")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose=False, jobs=2):
    csrc = os.path.join(_HERE, "csrc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    objs = []
    procs = []
    for src in ("sbt_kernels.hip", "sbt_persist.hip", "sbt_stats.hip", "sbt3d.hip", "sbt3f.hip", "sbt_static.hip",
                "sbt_host.cpp"):
        obj = os.path.join(csrc, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = ["hipcc", *HIP_FLAGS, *inc, *lang, "-c", os.path.join(csrc, src), "-o", obj]
        if src.endswith(".cpp"):
            # host-only translation unit (uses the HIP runtime API)
            cmd = ["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-Wall", *inc, "-c",
                   os.path.join(csrc, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError(f"hipcc failed: {rc}")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
