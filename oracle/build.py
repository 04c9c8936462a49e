"""Build the oracle shared library (plain gcc, FP64, no FMA contraction)."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
         "-shared", "-Wall", "-Wno-unused-function"]


def build(verbose=False):
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liborc.so")
    tmp = out + ".tmp"
    cmd = ["gcc", *FLAGS, src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_variant(edits, out_dir, name):
    """Build a copy of oracle.c with textual edits [(old, new), ...] applied,
    each of which must match exactly once: the tests plant a mistake in the
    oracle this way and check that a pin catches it.  Returns the path."""
    text = open(os.path.join(_HERE, "oracle.c")).read()
    for old, new in edits:
        n = text.count(old)
        if n != 1:
            raise ValueError(f"edit target found {n} times: {old!r}")
        text = text.replace(old, new)
    src = os.path.join(out_dir, name + ".c")
    with open(src, "w") as fh:
        fh.write(text)
    out = os.path.join(out_dir, "lib" + name + ".so")
    subprocess.run(["gcc", *FLAGS, "-I", _HERE, src, "-o", out, "-lm"], check=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
