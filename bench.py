#!/usr/bin/env python3
"""Throughput of the LBM-IBM hot path (arXiv 2402.04606) on one MI355X.

One step = one virtual-level-0 step of the whole batch: every level of every
case sub-cycled per Algorithm 1, with the multi-direct-forcing IBM before
every finest substep.  Prints one JSON line: MLUPS (cell updates per second),
the level kernel's achieved bandwidth against the 8 TB/s HBM peak, the other
storage forms with their error against FP64, and the FP64 CPU oracle timed on
a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import subprocess
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
Q = 9


def workload_list(name):
    import workloads as W
    if name == "sweep":
        return W.batch_sweep(), "batch_sweep_64_flapping_ellipses"
    if name == "cylinder":
        return [W.cylinder()], "cylinder_1024x512_D40_126markers"
    if name == "cavity":
        return [W.cavity()], "cavity_256_3levels_D32_lid0.1_rescale"
    if name == "cavity_ibb":
        return [W.cavity_ibb()], "cavity_256_3levels_D32_lid0.1_rescale_solid_cylinder_ibb"
    if name == "flap":
        return [W.flapping_ellipse()], "flapping_ellipse_512x256_4levels_200markers"
    if name == "pitch_up":
        return [W.pitch_up_plate()], "pitch_up_plate_1120x640_3levels_chord64_ramp"
    if name == "pitching_airfoil":
        return [W.pitching_airfoil()], "pitching_airfoil_1120x640_3levels_chord64_tri"
    if name == "tgv64":
        return [W.tgv(64, tau=0.8, u0=0.02)], "tgv_64x64_single_level"
    if name == "flap_re1000":
        return [W.flapping_ellipse(Re=1000.0)], "flapping_ellipse_512x256_4levels_200markers_re1000"
    if name == "tgv8192":
        return [W.tgv(8192, tau=0.8, u0=0.02)], "tgv_8192x8192_single_level"
    raise SystemExit(f"unknown workload {name}")


def measured_traffic_3d(storage):
    """HBM bytes per launch of the 3D kernel from its committed counter
    summary (same method as measured_traffic), or None."""
    path = os.path.join(ROOT, "profiles", f"step3_kernel_box3d_{storage}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2402_04606_amd", "csrc", "sbt3d.hip")
    if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec.get("hbm_bytes_per_launch")


def measured_traffic_forest(storage):
    """HBM bytes per coarse step of the 3D forest's step launches from the
    committed counter summary, or None (none, or the kernel source changed)."""
    path = os.path.join(ROOT, "profiles", f"forest3_kernel_forest3d_{storage}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2402_04606_amd", "csrc", "sbt3f.hip")
    if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec.get("hbm_bytes_per_step")


def measured_traffic(workload, storage):
    """HBM bytes per launch of the level kernel from the committed counter
    summary of this workload and storage form (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, each scaled by the same counter's reading for a plain copy
    of known size), or None when there is none or the kernel source changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", f"level_tile_kernel_{workload}_{storage}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2402_04606_amd", "csrc", "sbt_kernels.hip")
    if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec.get("hbm_bytes_per_launch")


def rel_l2_vs(ref, sim, wls):
    """Relative L2 of velocity of `sim` against `ref` over all cases and levels."""
    import numpy as np
    num = den = 0.0
    worst = 0.0
    for c, wl in enumerate(wls):
        cn = cd = 0.0
        for l in range(wl.n_levels):
            a = ref.fields_blocks(c, l)
            b = sim.fields_blocks(c, l)
            m = ~np.isnan(a[:, 0])
            du = (b[:, 1][m] - a[:, 1][m]) ** 2 + (b[:, 2][m] - a[:, 2][m]) ** 2
            w = 0.25 ** l
            cn += w * float(np.nansum(du))
            cd += w * float(((a[:, 1][m]) ** 2 + (a[:, 2][m]) ** 2).sum())
        num += cn
        den += cd
        worst = max(worst, math.sqrt(cn / max(cd, 1e-300)))
    return math.sqrt(num / max(den, 1e-300)), worst


def time_form(P, wls, storage, steps, warmup, tile=None, autotune=False, persistent=False):
    import torch
    sim = P.Sim(wls, storage)
    if tile is not None:
        sim.set_option(P.OPT_TILE, tile)
    if persistent:
        sim.set_option(P.OPT_PERSISTENT, 1)
    if autotune:
        # blocks per workgroup per level: the autotuner's cached choice for
        # this workload shape, or timed trials when the shape is new
        sim.autotune(steps=2, cache_path=os.path.join(ROOT, "paper_2402_04606_amd", "tune_cache.json"))
    sim.step(warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ups = sim.updates_per_step()
    return sim, dt, ups


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(wls, budget_s, V, per_case=8):
    """(cell updates, seconds, cases used) of the FP64 oracle on the cases of
    the workload, smallest first, each for whole batch steps (2^(V-m) coarse
    steps) until budget_s / per_case is used on it (at least one), until the
    budget is used.  Only stepping is timed (the oracle's set-up of its dense
    per-level arrays is not)."""
    import oracle
    order = sorted(range(len(wls)), key=lambda c: wls[c].nx0 * wls[c].ny0 * 4 ** wls[c].n_levels)
    ups, t_used, used = 0, 0.0, []
    for c in order:
        wl = wls[c]
        o = oracle.OracleSim(wl)
        n = 2 ** (V - wl.n_levels)
        cells = sum(int((o.kinds(l) == 1).sum()) * 2 ** l for l in range(wl.n_levels))
        t_case = 0.0
        while t_case < budget_s / per_case or t_case == 0.0:
            t0 = time.perf_counter()
            o.step(n)
            t_case += time.perf_counter() - t0
            ups += cells * n
        t_used += t_case
        used.append(c)
        del o
        if t_used >= budget_s:
            break
    return ups, t_used, used


def cpu_baseline(wls, budget_s, V, name, mrt=False):
    """The FP64 oracle on every case of the workload (whole batch steps of
    each, the budget split evenly over the cases), on all the host's threads
    and, in a child process, on one thread."""
    import oracle
    ups, t_used, used = _oracle_rate(wls, budget_s, V)
    out = dict(value=round(ups / t_used / 1e6, 3), unit="MLUPS", cores=oracle.num_threads(),
               kind="oracle", host_cpus=os.cpu_count(), cpu_model=_cpu_model(),
               sample=f"cases {used} of the same workload (smallest first), whole batch steps each, "
                      f"{ups} cell updates in {t_used:.1f} s of stepping, FP64, OpenMP")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import json, sys; sys.path.insert(0, %r); import bench, workloads as W; "
            "w, _ = bench.workload_list(%r); w = [c.replace(collision=W.COLL_MRT) for c in w] if %r else w; "
            "u, t, c = bench._oracle_rate(w, %r, %d); print(json.dumps([u, t]))") % (ROOT, name, mrt, budget_s / 2, V)
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=60 + 4 * budget_s)
        u1, t1 = json.loads(r.stdout.strip().splitlines()[-1])
        out["single_thread_value"] = round(u1 / t1 / 1e6, 3)
        out["single_thread_sample"] = f"smallest cases of the same workload, {u1} cell updates in {t1:.1f} s on 1 thread"
    except Exception as e:  # the single-thread figure is informative only
        out["single_thread_value"] = None
        out["single_thread_error"] = str(e)[:200]
    return out


def bench3d(args, P, W):
    """D3Q19 / D3Q27 periodic box (box3d = 512^3 D3Q19, box3d_q27 = 512^3
    D3Q27, box3d_256 = 256^3 D3Q19; flap3d = 256^3 D3Q19 with a pitching and
    plunging IBM ellipsoid of chord 48 and 2400 markers in a uniform stream):
    MLUPS and the bandwidth of the whole step (for flap3d including the
    forcing loop's launches) from HIP events on the stream it runs on."""
    import torch
    n = 256 if args.workload in ("box3d_256", "flap3d") else 512
    q = 27 if args.workload == "box3d_q27" else 19
    if args.workload == "flap3d":
        wl = W.flapping_ellipsoid3(n, chord=48.0, n_markers=2400, U=0.05, tau=0.6)
        name = f"d3q19_box_{n}^3_flapping_ellipsoid_chord48_2400_markers"
    else:
        wl = W.tgv3(n, nz=n).replace(lattice=q)
        name = f"d3q{q}_box_{n}^3_periodic_vortex"
    sim = P.Sim3(wl, args.storage)
    sim.step(args.warmup)
    sim.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    sim.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ups = sim.updates_per_step()
    s = P.STORAGE_BYTES[P.STORAGE[args.storage]]
    launch_ms = e0.elapsed_time(e1) / args.steps
    algo = ups * 2 * q * s
    gbs = algo / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": f"MLUPS & HBM GB/s fraction (D3Q{q} periodic box)",
        "value": round(ups * args.steps / dt / 1e6, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": name, "storage": args.storage,
                   "updates_per_step": ups, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic_3d(args.storage) if (n, q) == (512, 19) else None,
                     "kernel": f"step3_kernel (fused D3Q{q} pull stream + collide)" + (
                         " + the forcing loop's kernels (stream time per step)" if args.workload == "flap3d" else ""),
                     "bytes_per_update": 2 * q * s, "algorithmic_bytes_per_launch": algo,
                     "avg_launch_us": round(launch_ms * 1e3, 2)},
    }
    if args.storage != "f64" and not args.no_err:
        # the same run in FP64 (same steps), compared on three sampled planes
        total = args.warmup + args.steps
        ref = P.Sim3(wl, "f64")
        ref.step(total)
        ref.synchronize()
        num = den = 0.0
        for z in (0, wl.nz // 2, wl.nz - 1):
            a, b = sim.fields(z, z + 1), ref.fields(z, z + 1)
            num += sum(float(((a[k] - b[k]) ** 2).sum()) for k in (1, 2, 3))
            den += sum(float((b[k] ** 2).sum()) for k in (1, 2, 3))
        ref.close()
        out["rel_l2_u_vs_f64"] = float(f"{(num / den) ** 0.5:.3e}")
        out["error_sample"] = f"planes z = 0, {wl.nz // 2}, {wl.nz - 1} after {total} steps, against the FP64 run"
    if not args.no_cpu and args.workload != "flap3d":
        import oracle
        m = 64
        o = oracle.Oracle3Sim(W.tgv3(m, nz=m).replace(lattice=q))
        k, t_used = 0, 0.0
        while t_used < args.cpu_budget:
            t1 = time.perf_counter()
            o.step(1)
            t_used += time.perf_counter() - t1
            k += 1
        out["cpu_baseline"] = dict(value=round(m ** 3 * k / t_used / 1e6, 3), unit="MLUPS",
                                   cores=oracle.num_threads(), kind="oracle",
                                   sample=f"{m}^3 box of the same vortex, {k} steps in {t_used:.1f} s, FP64, OpenMP")
    print(json.dumps(out), flush=True)


def bench_forest3d(args, P, W):
    """The 3D block forest (forest3d = 256^3 D3Q19 level 0 with nested level-1
    and level-2 boxes over the central half and quarter of each axis;
    forest3d_q27 the same with D3Q27): MLUPS over the cell updates of a
    coarse step (owned cells of level l counted 2^l times) and the bandwidth
    of the step's launches from HIP events on the stream they run on."""
    import numpy as np
    import torch
    q = 27 if args.workload == "forest3d_q27" else 19
    wl = W.forest3d_bench(lattice=q)
    sim = P.Sim3F(wl, args.storage)
    sim.step(args.warmup)
    sim.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    sim.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ups = sim.updates_per_step()
    s = P.STORAGE_BYTES[P.STORAGE[args.storage]]
    step_ms = e0.elapsed_time(e1) / args.steps
    algo = ups * 2 * q * s
    gbs = algo / (step_ms * 1e-3) / 1e9
    launches = 1 + sum(1 << l for l in range(1, wl.n_levels))
    out = {
        "metric": f"MLUPS & HBM GB/s fraction (D3Q{q} 3D block forest)",
        "value": round(ups * args.steps / dt / 1e6, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"d3q{q}_forest_256^3_levels3_nested_half_quarter", "storage": args.storage,
                   "updates_per_step": ups, "levels": wl.n_levels,
                   "owned_cells": [i[3] for i in sim.info], "halo_cells": [i[4] for i in sim.info],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic_forest(args.storage) if q == 19 else None,
                     "traffic_unit": "HBM bytes per coarse step (the 7 step launches)",
                     "kernel": f"forest3_kernel (D3Q{q} pull stream + coalescence + collide + explosion), "
                               f"{launches} launches per coarse step",
                     "bytes_per_update": 2 * q * s, "algorithmic_bytes_per_step": algo,
                     "step_launch_ms": round(step_ms, 4)},
    }
    if args.storage != "f64" and not args.no_err:
        total = args.warmup + args.steps
        sim_steps = total
        ref = P.Sim3F(wl, "f64")
        ref.step(sim_steps)
        ref.synchronize()
        num = den = 0.0
        for l in range(wl.n_levels):
            x0, y0, z0, nx, ny, nz = sim.region_box(l)
            for z in (z0 + 1, z0 + nz // 2, z0 + nz - 2):
                a, b = sim.fields(l, (x0, y0, z, nx, ny, 1)), ref.fields(l, (x0, y0, z, nx, ny, 1))
                own = ~np.isnan(b[0])
                num += sum(float(((a[k] - b[k])[own] ** 2).sum()) for k in (1, 2, 3))
                den += sum(float((b[k][own] ** 2).sum()) for k in (1, 2, 3))
        ref.close()
        out["rel_l2_u_vs_f64"] = float(f"{(num / den) ** 0.5:.3e}")
        out["error_sample"] = f"three planes of every level after {total} coarse steps, against the FP64 run"
    if not args.no_cpu:
        import oracle
        small = W.forest3d_bench(n0=32, lattice=q)
        o = oracle.Oracle3FSim(small)
        ups_small = sum(int((o.kinds(l) == 1).sum()) << l for l in range(small.n_levels))
        k, t_used = 0, 0.0
        while t_used < args.cpu_budget:
            t1 = time.perf_counter()
            o.step(1)
            t_used += time.perf_counter() - t1
            k += 1
        out["cpu_baseline"] = dict(value=round(ups_small * k / t_used / 1e6, 3), unit="MLUPS",
                                   cores=oracle.num_threads(), kind="oracle",
                                   sample=f"the same forest at 32^3 level-0 cells ({ups_small} updates per "
                                          f"coarse step), {k} coarse steps in {t_used:.1f} s, FP64, OpenMP")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sweep")
    ap.add_argument("--storage", default="f16s")
    ap.add_argument("--forms", default="f64,f32,bf16s", help="other storage forms to time ('' = none)")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-err", action="store_true", help="3D workloads: skip the FP64 reference run")
    ap.add_argument("--tile", type=int, default=None)
    ap.add_argument("--persistent", action="store_true",
                    help="time the one-launch-per-step form (SBT_OPT_PERSISTENT) instead of the launch chain")
    ap.add_argument("--no-persistent-form", dest="persistent_form", action="store_false",
                    help="do not also time the one-launch-per-step form beside the launch chain")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="automatic blocks per workgroup instead of the autotuner's choice")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"],
                    help="collision model of the headline run")
    ap.add_argument("--no-mrt", dest="mrt", action="store_false",
                    help="skip the extra MRT-collision timing at the headline storage form")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; the batched sweep would shard by "
              "whole cases with no exchange between GPUs. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_calib:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        # the practical copy bandwidth of this GPU, for context
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        gbs = 10 * 2 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 13,
                          "copy_gbs": round(gbs, 1), "copy_frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}))
        return

    import paper_2402_04606_amd as P
    import workloads as W
    if args.workload.startswith("forest3d"):
        return bench_forest3d(args, P, W)
    if args.workload.startswith("box3d") or args.workload == "flap3d":
        return bench3d(args, P, W)
    wls, wname = workload_list(args.workload)
    if args.collision == "mrt":
        wls = [w.replace(collision=W.COLL_MRT) for w in wls]
        wname += "_mrt"
    V = max(w.n_levels for w in wls)

    # ---- headline form, timed with graphs --------------------------------------
    sim, dt, ups = time_form(P, wls, args.storage, args.steps, args.warmup, args.tile, args.autotune, args.persistent)
    mlups = ups * args.steps / dt / 1e6
    ms_per_step = dt * 1e3 / args.steps

    # ---- kernel bandwidth: HIP events around every launch, same stream ---------
    prof = sim.profile(args.profile_steps)
    sbytes = P.STORAGE_BYTES[P.STORAGE[args.storage]]
    fast_gbs = prof["fast_bytes"] / (prof["fast_ms"] * 1e-3) / 1e9 if prof["fast_ms"] > 0 else 0.0
    gen_ms = prof["level_ms"] - prof["fast_ms"]
    gen_bytes = prof["level_bytes"] - prof["fast_bytes"]
    roofline = {
        "bound": "hbm", "achieved": round(fast_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(fast_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload, args.storage),
        "kernel": "level_tile_kernel (LDS-staged stream+collide, all owned blocks)",
        "bytes_per_update": 2 * Q * sbytes,
        "algorithmic_bytes_per_launch": round(prof["fast_bytes"] / max(1, prof["fast_launches"])),
        "launches": prof["fast_launches"],
        "avg_launch_us": round(prof["fast_ms"] * 1e3 / max(1, prof["fast_launches"]), 2),
        "time_share": {
            "level_tile_kernel": round(prof["fast_ms"] / args.profile_steps, 4),
            "mdf_kernel": round(prof["mdf_ms"] / args.profile_steps, 4),
            "unit": "ms per step (eager, events)"},
        "mdf_avg_launch_us": round(prof["mdf_ms"] * 1e3 / max(1, prof["mdf_launches"]), 2),
    }

    # ---- other storage forms and their error against FP64 -----------------------
    forms = {}
    total_steps = args.warmup + args.steps
    want = [f for f in args.forms.split(",") if f]
    ref = None
    if want or args.storage != "f64":
        sims = {args.storage: sim}
        for st in want:
            if st == args.storage:
                continue
            s2, dt2, _ = time_form(P, wls, st, args.steps, args.warmup, args.tile, args.autotune)
            sims[st] = s2
            forms[st] = {"mlups": round(ups * args.steps / dt2 / 1e6, 1),
                         "ms_per_step": round(dt2 * 1e3 / args.steps, 3),
                         "bytes_per_update": 2 * Q * P.STORAGE_BYTES[P.STORAGE[st]]}
        forms[args.storage] = {"mlups": round(mlups, 1), "ms_per_step": round(ms_per_step, 3),
                               "bytes_per_update": 2 * Q * sbytes}
        if "f64" in sims:
            ref = sims["f64"]
            for st, s2 in sims.items():
                if st == "f64":
                    continue
                # the headline sim ran extra profile steps; compare at equal step counts
                if s2 is sim:
                    s2 = P.Sim(wls, st)
                    s2.step(total_steps)
                    s2.synchronize()
                e, worst = rel_l2_vs(ref, s2, wls)
                forms[st]["rel_l2_u_vs_f64"] = float(f"{e:.3e}")
                forms[st]["worst_case_rel_l2_u"] = float(f"{worst:.3e}")
                forms[st]["after_steps"] = total_steps

    # ---- the same step with the other collision model --------------------------
    if args.mrt:
        other = W.COLL_BGK if args.collision == "mrt" else W.COLL_MRT
        wo = [w.replace(collision=other) for w in wls]
        s3, dt3, _ = time_form(P, wo, args.storage, args.steps, args.warmup, args.tile, args.autotune)
        p3 = s3.profile(args.profile_steps)
        forms[("bgk" if other == W.COLL_BGK else "mrt") + "_" + args.storage] = {
            "mlups": round(ups * args.steps / dt3 / 1e6, 1), "ms_per_step": round(dt3 * 1e3 / args.steps, 3),
            "tile_gbs": round(p3["fast_bytes"] / (p3["fast_ms"] * 1e-3) / 1e9, 1) if p3["fast_ms"] > 0 else 0.0}
        del s3

    # ---- the same step as one persistent launch (SBT_OPT_PERSISTENT) -----------
    if not args.persistent and args.persistent_form:
        s4, dt4, _ = time_form(P, wls, args.storage, args.steps, args.warmup, args.tile, args.autotune, True)
        forms["persistent_" + args.storage] = {"mlups": round(ups * args.steps / dt4 / 1e6, 1),
                                               "ms_per_step": round(dt4 * 1e3 / args.steps, 3)}
        del s4

    out = {
        "metric": "MLUPS & HBM GB/s fraction; FP16/FP32-storage vs FP64 at stated L2 error",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": wname, "cases": len(wls), "levels": sorted({w.n_levels for w in wls}),
                   "storage": args.storage, "collision": args.collision, "updates_per_step": ups,
                   "block": "16x16",
                   "parallelism": "single GPU, all cases in one context"},
        "roofline": roofline,
        "forms": forms,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wls, args.cpu_budget, V, args.workload, args.collision == "mrt")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
