"""CPU runs of the host code under AddressSanitizer and UndefinedBehavior-
Sanitizer: the oracle (gcc) through a set of its pins, and the host-side
forest builder and planner of the library (hipcc, host code only) through
the descriptors of every workload shape and a set of invalid ones.  Each
runs in a child process with the sanitizer runtime preloaded; any report
aborts it."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_04606_amd", "csrc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

ORACLE_PINS = ("tgv_closed_form or poiseuille or couette or refined_band or uniform_flow or mdf or peskin or spread "
               "or interpolation or flap or ramp or triangular or pitching_bodies or force_stats or velocity_change "
               "or ibb_half_way or ibb_short or host_markers or rejected or d3q19_conservation "
               "or 3d_moving or symmetric_body or open_boundaries or closed_box")


def _run(cmd, env_extra, timeout):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    return r.stdout


def test_oracle_pins_under_asan_ubsan(tmp_path):
    from oracle import build as B
    so = str(tmp_path / "liborc_san.so")
    subprocess.run(["gcc", *B.FLAGS, "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "oracle.c"), "-o", so, "-lm"],
                   check=True)
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    driver = ("import sys, oracle, pytest; oracle.LIB_PATH = sys.argv[1]; "
              "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '-m', 'not gpu and not slow', "
              "'tests/test_oracle_pins.py', 'tests/test_oracle_interface_pins.py', "
              "'tests/test_oracle_forest3d.py', '-k', sys.argv[2]]))")
    out = _run([sys.executable, "-c", driver, so, ORACLE_PINS + " or chapman or outflow_at or 3d_pitch_plunge_pose or invariant_forest "
                                           "or single_level_forest or uniform_stream_on or permutation"],
               {"LD_PRELOAD": libasan, "OMP_NUM_THREADS": "4"}, 900)
    assert " passed" in out and "failed" not in out, out[-2000:]


def test_host_planner_under_asan_ubsan(tmp_path):
    lib = os.path.join(ROOT, "paper_2402_04606_amd", "libsbt.so")
    if not os.path.exists(lib):
        pytest.skip("libsbt.so not built")
    runtime = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not runtime:
        pytest.skip("no clang ASan runtime")
    obj, so = str(tmp_path / "sbt_host.o"), str(tmp_path / "libsbt_san.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
                    *san, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
                    os.path.join(CSRC, "sbt_host.cpp"), "-o", obj], check=True, capture_output=True)
    # the sanitized planner, with the kernels' host stubs taken from the built library
    subprocess.run(["hipcc", "-shared", "-fPIC", *san[:4], obj, "-L" + os.path.dirname(lib), "-l:libsbt.so",
                    "-Wl,-rpath," + os.path.dirname(lib), "-o", so], check=True, capture_output=True)
    driver = """
import sys
import paper_2402_04606_amd as P
import workloads as W
P.LIB_PATH = sys.argv[1]
n = 0
for wls, st in (([W.tgv(64)], P.F64), ([W.cavity()], P.F16S), ([W.cavity_ibb()], P.F32), (W.batch_sweep(), P.F16S),
                ([W.flapping_ellipse()], P.F32), ([W.pitch_up_plate()], P.F16S), ([W.small_refined_flap()], P.F64),
                ([W.tgv_patch(m=3)], P.BF16S), ([W.ibb_channel()], P.F64)):
    n += P.plan(wls, st) > 0
for bad in (dict(boxes=[(1, 0, 0, 4, 4)], n_levels=2, body=None), dict(boxes=[(1, 12, 12, 20, 20), (2, 22, 22, 42, 42)]),
            dict(boxes=[(1, 12, 12, 20, 20), (2, 24, 24, 40, 40)]), dict(boxes=[(3, 1, 1, 2, 2)]),
            dict(tau0=0.5), dict(nx0=250), dict(bc=(0, 1, 1, 1))):
    try:
        P.plan([W.cavity().replace(**bad)])
    except P.SbtError:
        n += 1
print("planned", n)
"""
    out = _run([sys.executable, "-c", driver, so], {"LD_PRELOAD": runtime[0]}, 600)
    assert "planned 16" in out, out
