"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  FP64: bit for bit wherever both sides take the same
operations in the same order (fixed geometry, BGK); otherwise every velocity
component within 1e-12 of the level's largest |u| (MRT, whose two sides round
the moment transforms differently; bodies in prescribed motion, whose poses
use the device's sin and cos in 2D); force histories likewise, bit for bit or
within 1e-12 of their largest value.  Reduced-precision storage forms have
stated ceilings on the relative L2 norm of velocity."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2402_04606_amd as P
    P.lib()
    return P, oracle


def rel_l2(ug, vg, uo, vo):
    m = ~np.isnan(uo)
    assert m.sum() > 0
    assert not np.isnan(ug[m]).any(), "GPU field has NaN where the oracle has values"
    assert np.isnan(ug[~m]).all(), "GPU field defined where the oracle has no owned cell"
    num = np.sqrt(((ug[m] - uo[m]) ** 2 + (vg[m] - vo[m]) ** 2).sum())
    den = np.sqrt((uo[m] ** 2 + vo[m] ** 2).sum())
    # a level still at rest has |u| ~ roundoff; measure it against 1e-8 per cell
    return num / max(den, 1e-8 * np.sqrt(m.sum()))


def run_pair(env, wl, steps, storage="f64", **kw):
    P, O = env
    print(f"case {wl.name} storage {storage} steps {steps}", flush=True)
    g = P.Sim(wl, storage, **kw)
    o = O.OracleSim(wl)
    g.step(steps)
    g.synchronize()
    o.step(steps)
    return g, o


def compare_levels(g, o, wl, tol, c=0, exact=False, abs_u=0.0):
    """Per level, on every owned cell of the oracle (the GPU defines exactly
    those cells):
      exact: rho, ux, uy equal bit for bit;
      FP64 (tol <= 1e-11): every velocity component within tol * max|u| of
        the oracle's, or within abs_u on a level still near rest (abs_u > 0,
        where a relative bound measures rounding only), densities within
        10 tol;
      reduced storage: relative L2 norm of u within tol."""
    errs = []
    for l in range(wl.n_levels):
        rg, ug, vg = g.fields(c, l)
        ro, uo, vo = o.fields(l)
        e = rel_l2(ug, vg, uo, vo)
        m = ~np.isnan(ro)
        er = np.abs(rg[m] - ro[m]).max()
        ea = max(np.abs(ug[m] - uo[m]).max(), np.abs(vg[m] - vo[m]).max())
        umax = max(np.abs(uo[m]).max(), np.abs(vo[m]).max())
        print(f"  level {l}: rel L2 u {e:.3e}  max |du| {ea:.3e} (max |u| {umax:.3e})  max |drho| {er:.3e}",
              flush=True)
        errs.append(e)
        if exact:
            assert np.array_equal(rg, ro, equal_nan=True), (l, "rho", er)
            assert np.array_equal(ug, uo, equal_nan=True) and np.array_equal(vg, vo, equal_nan=True), (l, ea)
        elif tol <= 1e-11:
            assert ea <= tol * umax or ea <= abs_u, (l, ea, umax)
            assert er <= tol * 10, (l, er)
        else:
            assert e <= tol, (l, e)
    return errs


# Bodies in prescribed motion (2D): the poses use the device's sin and cos,
# which may differ from the host library's by an ulp; the flow amplifies that
# over hundreds of substeps, most in the body force (a sum of marker forces of
# both signs).  Their histories are held to this bound (fields to TOL64).
TOL_MOVING_HISTORY = 1e-10


def compare_history(g, o, c=0, exact=False, tol=TOL64):
    """The F_s history (per finest substep): bit for bit, or within tol of
    its largest value."""
    fxg, fyg = g.force_history(c)
    fxo, fyo = o.force_history()
    assert len(fxg) == len(fxo) > 0
    d = max(np.abs(fxg - fxo).max() / np.abs(fxo).max(), np.abs(fyg - fyo).max() / max(np.abs(fyo).max(), 1e-300))
    print(f"  force history: {len(fxo)} substeps, max rel diff {d:.3e}", flush=True)
    if exact:
        assert np.array_equal(fxg, fxo) and np.array_equal(fyg, fyo), d
    else:
        assert d <= tol, d
    return fxg, fyg


# ---- uniform grids ---------------------------------------------------------

def test_tgv_f64_matches_oracle(env):
    wl = W.tgv(64)
    g, o = run_pair(env, wl, 1000)
    compare_levels(g, o, wl, TOL64, exact=True)
    # and the closed-form decay (P7) holds on the GPU as well
    _, u, _ = g.fields(0, 0)
    _, ua, _ = wl.init(0, 64, 64)
    fac = math.exp(-2 * wl.meta["nu"] * wl.meta["k"] ** 2 * 1000)
    assert np.sqrt(((u - fac * ua) ** 2).sum() / ((fac * ua) ** 2).sum()) < 1e-2


def test_blocks_equal_monolithic_bitwise(env):
    """P10: 16x16 blocks reproduce the dense grid bit for bit (FP64)."""
    wl = W.tgv(48, tau=0.7)
    g, o = run_pair(env, wl, 200)
    rg, ug, vg = g.fields(0, 0)
    ro, uo, vo = o.fields(0)
    print("  max |du|", np.abs(ug - uo).max(), flush=True)
    assert np.array_equal(ug, uo) and np.array_equal(vg, vo) and np.array_equal(rg, ro)


def test_poiseuille_and_body_force(env):
    wl = W.poiseuille(nx=32, ny=32)
    g, o = run_pair(env, wl, 3000)
    compare_levels(g, o, wl, TOL64, exact=True)


def test_outflow_channel_both_ends(env):
    """The body-forced channel with zero-gradient outflow at W and E: bit for
    bit the oracle's, and bit for bit the periodic channel's (the flow does
    not vary along x)."""
    P, O = env
    base = W.poiseuille(nx=32, ny=32, tau=0.8, g=2e-6)
    wl = base.replace(bc=(W.OUTFLOW, W.OUTFLOW, W.WALL, W.WALL))
    g, o = run_pair(env, wl, 1500)
    compare_levels(g, o, wl, TOL64, exact=True)
    p = P.Sim(base, "f64")
    p.step(1500)
    p.synchronize()
    assert all(np.array_equal(a, b) for a, b in zip(g.fields(0, 0), p.fields(0, 0)))


def test_couette_moving_wall(env):
    wl = W.Workload(name="couette", nx0=32, ny0=48, tau0=0.9, bc=(0, 0, W.WALL, W.WALL),
                    bc_u=((0, 0), (0, 0), (0, 0), (0.01, 0.0)), init=W.uniform_init(1.0, 0, 0))
    g, o = run_pair(env, wl, 2000)
    compare_levels(g, o, wl, TOL64, exact=True)


def test_open_boundaries_and_corners(env):
    """Inflow, outflow, symmetry edges with a disturbance crossing them."""
    wl = W.Workload(name="open", nx0=64, ny0=48, tau0=0.62,
                    bc=(W.INFLOW, W.OUTFLOW, W.SYMMETRY, W.SYMMETRY),
                    bc_u=((0.04, 0.0),) + ((0.0, 0.0),) * 3, init=W.tgv_init(64, 0.02, 1.0))
    g, o = run_pair(env, wl, 400)
    compare_levels(g, o, wl, TOL64, exact=True)


def test_cavity_walls_uniform(env):
    wl = W.Workload(name="cavity_uniform", nx0=64, ny0=64, tau0=0.6, bc=(W.WALL,) * 4,
                    bc_u=((0, 0), (0, 0), (0, 0), (0.1, 0.0)), init=W.uniform_init(1.0, 0, 0))
    g, o = run_pair(env, wl, 500)
    compare_levels(g, o, wl, TOL64, exact=True)


def test_cylinder_small_ibm(env):
    wl = W.small_cylinder()
    g, o = run_pair(env, wl, 300)
    compare_levels(g, o, wl, TOL64, exact=True)
    fxg, _ = compare_history(g, o, exact=True)
    assert len(fxg) == 300
    mg, mo = g.marker_forces(), o.marker_forces()
    assert np.array_equal(mg[0], mo[0]) and np.array_equal(mg[1], mo[1])


def test_cylinder_full_size_short_horizon(env):
    """Workload C2 (1024x512, D 40, 126 markers) at a short horizon."""
    wl = W.cylinder()
    g, o = run_pair(env, wl, 60)
    compare_levels(g, o, wl, TOL64, exact=True)
    compare_history(g, o, exact=True)


# ---- refinement ------------------------------------------------------------

@pytest.mark.parametrize("m,cf", [(2, 0), (3, 0), (2, 1), (3, 1)])
def test_refined_patch_tgv(env, m, cf):
    wl = W.tgv_patch(m=m, cf_mode=cf)
    g, o = run_pair(env, wl, 40)
    compare_levels(g, o, wl, TOL64, exact=True)
    dg, do = g.diagnostics(), o.diagnostics()
    assert abs(dg[0] - do[0]) <= 1e-12 * do[0]


def test_refined_band_mass(env):
    wl = W.tgv_band()
    g, o = run_pair(env, wl, 60)
    compare_levels(g, o, wl, TOL64, exact=True)


def test_uniform_flow_refined_stays_uniform(env):
    wl = W.uniform_refined()
    g, o = run_pair(env, wl, 10)
    compare_levels(g, o, wl, TOL64, exact=True)


def test_cavity_three_levels_ibm(env):
    """Workload C3 at full size: 3 levels, lid, rescaled interfaces, fixed
    cylinder D 128 finest, 50 coarse steps (200 finest substeps): bit for
    bit."""
    wl = W.cavity()
    g, o = run_pair(env, wl, 50)
    compare_levels(g, o, wl, TOL64, exact=True)
    fxg, _ = compare_history(g, o, exact=True)
    assert len(fxg) == 200


def test_moving_body_refined(env):
    wl = W.small_refined_flap()
    g, o = run_pair(env, wl, 8)
    compare_levels(g, o, wl, TOL64)
    compare_history(g, o, tol=TOL_MOVING_HISTORY)


@pytest.mark.parametrize("make,steps", [(W.small_pitch_up, 16), (W.small_pitching_airfoil, 30)])
def test_pitching_laws_refined(env, make, steps):
    """Sec. 3.5 ramp (plate pitched about its leading edge) and Sec. 3.6
    smoothed triangular law (over a full period, every breakpoint) on a
    3-level forest: fields and force history against the oracle."""
    wl = make()
    g, o = run_pair(env, wl, steps)
    compare_levels(g, o, wl, TOL64)
    compare_history(g, o, tol=TOL_MOVING_HISTORY)


def test_force_stats_and_convergence_on_device(env):
    """Eq. (21) statistics reduced on the device against the oracle's reading
    of the same history, and against the oracle run's own history; the
    Sec. 3.2 measure E against the oracle's fields; a refreshed snapshot
    reads E = 0."""
    import oracle
    wl = W.small_pitching_airfoil()
    P, O = env
    g = P.Sim(wl, "f64")
    o = O.OracleSim(wl)
    g.step(10)
    o.step(10)
    snap = g.snapshot()
    then = o.velocity()
    g.step(20)
    o.step(20)
    g.synchronize()
    U, L = wl.meta["U"], wl.meta["chord"]
    fxg, fyg = g.force_history()
    sd = g.force_stats(U=U, L=L)
    so = oracle.force_stats(fxg, fyg, U, L)
    sr = oracle.force_stats(*o.force_history(), U, L)
    print("  device", sd, "\n  oracle", sr, flush=True)
    assert sd["samples"] == so["samples"] == len(fxg) == sr["samples"]
    assert sd["crossings"] == so["crossings"] == sr["crossings"] >= 2
    for key in ("CD_mean", "CL_mean", "CD_rms", "CL_rms", "St"):
        assert abs(sd[key] - so[key]) <= 1e-12 * abs(so[key]), key
        assert abs(sd[key] - sr[key]) <= 1e-9 * abs(sr[key]), key
    # the last 50 substeps only
    sd50 = g.force_stats(n_last=50, U=U, L=L)
    so50 = oracle.force_stats(fxg[-50:], fyg[-50:], U, L)
    assert sd50["samples"] == 50 and abs(sd50["CL_rms"] - so50["CL_rms"]) <= 1e-12 * so50["CL_rms"]
    Eg = g.convergence(snap, update=True)
    Eo = oracle.velocity_change(o.velocity(), then)
    print(f"  E device {Eg[2]:.15e} oracle {Eo[2]:.15e}", flush=True)
    assert Eg[2] > 0.0
    for a, b in zip(Eg, Eo):
        assert abs(a - b) <= 1e-10 * abs(b)
    assert g.convergence(snap)[0] == 0.0


# ---- solid cells with interpolated bounce-back ------------------------------

@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", 1e-5), ("f16s", 3e-3)])
def test_ibb_channel(env, storage, tol):
    """Walls at link fractions 0.3 and 0.7 (both Bouzidi branches) in a
    body-forced periodic channel, 300 steps."""
    wl = W.ibb_channel(q_bottom=0.3, q_top=0.7, tau=0.8, g=1e-5)
    g, o = run_pair(env, wl, 300, storage)
    compare_levels(g, o, wl, tol, exact=storage == "f64")


@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", 1e-4)])
def test_ibb_cylinder(env, storage, tol):
    """A solid circle (every link fraction in (0, 1)) in the inflow / outflow
    / symmetry channel, 200 steps; the convergence measure E with solid
    cells left out agrees with the oracle's."""
    import oracle
    wl = W.ibb_cylinder()
    P, O = env
    g = P.Sim(wl, storage)
    o = O.OracleSim(wl)
    g.step(100)
    o.step(100)
    snap = g.snapshot()
    then = o.velocity()
    g.step(100)
    o.step(100)
    g.synchronize()
    compare_levels(g, o, wl, tol, exact=storage == "f64")
    Eg = g.convergence(snap)
    Eo = oracle.velocity_change(o.velocity(), then)
    assert abs(Eg[2] - Eo[2]) <= max(tol, 1e-10) * Eo[2]
    assert np.isnan(g.fields(0, 0)[1][wl.solids[0][1] == 1]).all()


def test_ibb_cavity_three_levels(env):
    """The Sec. 3.2 comparison case: the cavity's cylinder as solid cells on
    the finest of 3 levels (RESCALE interface, moving lid), FP64, 50 steps:
    bit for bit."""
    wl = W.cavity_ibb()
    g, o = run_pair(env, wl, 50)
    compare_levels(g, o, wl, TOL64, exact=True)


# ---- MRT collision --------------------------------------------------------

@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", 2e-5), ("f16s", 3e-3), ("bf16s", 3e-2)])
def test_mrt_tgv(env, storage, tol):
    """MRT collision (Sec. 2.1 option) on the 64^2 Taylor-Green vortex,
    500 steps, every storage form against the FP64 oracle."""
    wl = W.tgv(64).replace(collision=W.COLL_MRT)
    g, o = run_pair(env, wl, 500, storage)
    compare_levels(g, o, wl, tol)


def test_mrt_refined_moving_body(env):
    """MRT on a 3-level forest with a flapping body: interface, IBM forcing
    in moment space and force history against the oracle (FP64)."""
    wl = W.small_refined_flap().replace(collision=W.COLL_MRT)
    g, o = run_pair(env, wl, 8)
    compare_levels(g, o, wl, TOL64)
    compare_history(g, o, tol=TOL_MOVING_HISTORY)


def test_mrt_cavity_rescale(env):
    """MRT with the RESCALE interface and moving-wall edges (C3, 3 levels,
    FP64, 10 steps).  The MRT forms round differently on the two sides (the
    oracle multiplies by the moment matrices, the kernel uses their closed
    forms), so the inner levels, still at rest to ~1e-8 after 10 steps, are
    held to an absolute 1e-14 on u (a few ulps of the populations)."""
    wl = W.cavity().replace(collision=W.COLL_MRT)
    g, o = run_pair(env, wl, 10)
    compare_levels(g, o, wl, TOL64, abs_u=1e-14)


@pytest.mark.parametrize("make,steps", [(lambda: W.flapping_ellipse(Re=10000.0), 500),
                                        (lambda: W.pitch_up_plate(Re=5000.0), 1600)])
def test_mrt_stays_stable_where_bgk_fails(env, make, steps):
    """Sec. 2.1 names MRT for low viscosity: the C4 flapping ellipse at
    Re 10 000 (tau0 = 0.50012) and the Sec. 3.5 plate at Re 5000 lose a
    finite density under BGK within the run (the library reports it), and
    stay finite under MRT (F32 storage)."""
    P, _ = env

    def survives(wl):
        g = P.Sim(wl, "f32")
        try:
            for _ in range(steps // 100):
                g.step(100)
                g.synchronize()
            return True
        except P.SbtError as e:
            assert e.code == -6, e          # SBT_ERR_NONFINITE
            return False
        finally:
            g.close()

    wl = make()
    assert not survives(wl)
    assert survives(wl.replace(collision=W.COLL_MRT))


def test_flapping_ellipse_four_levels(env):
    """Workload C4 at full size (4 levels, 200 moving markers), 50 coarse
    steps = 400 finest substeps, fields and force history."""
    wl = W.flapping_ellipse()
    g, o = run_pair(env, wl, 50)
    compare_levels(g, o, wl, TOL64)
    fxg, _ = compare_history(g, o, tol=TOL_MOVING_HISTORY)
    assert len(fxg) == 400


# ---- batch -------------------------------------------------------------------

def test_batch_matches_cases_run_alone(env):
    """Cases of 1, 2 and 3 levels in one context: each equals its own oracle
    run over 2^(V-m) of its coarse steps per batch step."""
    P, O = env
    cases = [W.tgv_patch(m=3), W.tgv_patch(m=2, cf_mode=1), W.tgv(32, tau=0.7), W.small_cylinder()]
    g = P.Sim(cases, "f64")
    steps = 3
    g.step(steps)
    g.synchronize()
    V = max(c.n_levels for c in cases)
    for k, wl in enumerate(cases):
        o = O.OracleSim(wl)
        o.step(steps * 2 ** (V - wl.n_levels))
        print(f"batch case {k} {wl.name}", flush=True)
        compare_levels(g, o, wl, TOL64, c=k, exact=True)


# ---- precision forms ---------------------------------------------------------

@pytest.mark.parametrize("storage,ceiling", [("f32", 2e-5), ("f16s", 3e-3), ("bf16s", 3e-2)])
def test_reduced_precision_error_ceiling(env, storage, ceiling):
    wl = W.tgv(64)
    g, o = run_pair(env, wl, 500, storage)
    compare_levels(g, o, wl, ceiling)


@pytest.mark.parametrize("storage,ceiling", [("f32", 1e-4), ("f16s", 2e-2)])
def test_reduced_precision_refined_ibm(env, storage, ceiling):
    wl = W.cavity()
    g, o = run_pair(env, wl, 30, storage)
    compare_levels(g, o, wl, ceiling)


# ---- engine behaviour ----------------------------------------------------------

def test_determinism_graph_eager_and_tiles(env):
    P, _ = env
    wl = W.small_refined_flap()
    outs = []
    for graph, tile in ((1, 0), (1, 0), (0, 0), (1, 1), (1, 2)):
        g = P.Sim(wl, "f64")
        g.set_option(P.OPT_GRAPH, graph)
        g.set_option(P.OPT_TILE, tile)
        g.step(3)
        g.synchronize()
        outs.append([g.fields(0, l) for l in range(wl.n_levels)] + [g.force_history()])
        g.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            for x, y in zip(a, b):
                assert np.array_equal(x, y, equal_nan=True)


def test_multi_step_graphs_match_eager(env):
    """Calls of n steps replay captured graphs of 4, 2 and 1 steps; any mix
    of call sizes gives the eager launch list's result bit for bit."""
    P, _ = env
    wl = W.small_refined_flap()
    outs = []
    for graph, calls in ((0, (15,)), (1, (7, 1, 1, 5, 1)), (1, (4, 4, 4, 3))):
        g = P.Sim(wl, "f64")
        g.set_option(P.OPT_GRAPH, graph)
        for n in calls:
            g.step(n)
        g.synchronize()
        outs.append([g.fields(0, l) for l in range(wl.n_levels)] + [g.force_history()])
        g.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            for x, y in zip(a, b):
                assert np.array_equal(x, y, equal_nan=True)


@pytest.mark.parametrize("storage", ["f64", "f16s"])
def test_persistent_step_matches_launch_chain(env, storage):
    """One persistent launch per step (SBT_OPT_PERSISTENT: plan builder,
    forcing loops and level substeps as phases behind grid barriers) against
    the launch chain: the 64-case batch, 4 and then 3 global steps (both
    level-0 parities of the phase tables), a refined patch without bodies
    (no plan or forcing phases), and the walled cavity with solid cells in
    MRT (solid blocks, domain edges, the MRT variant).  FP64 bit for bit.
    In the deviation
    forms the persistent step's per-cell path rounds differently from the
    tile kernel in FP32 arithmetic (last-bit differences on refined levels
    after one step), so the 2-byte form is held to a relative L2 of velocity
    of 1e-3, well inside its 5e-3 ceiling against FP64."""
    P, _ = env
    for wls in (W.batch_sweep(), [W.tgv_patch(m=3)], [W.cavity_ibb().replace(collision=W.COLL_MRT)]):
        outs = []
        for persistent in (1, 0):
            print(f"{len(wls)} cases {storage} persistent {persistent}", flush=True)
            g = P.Sim(wls, storage)
            g.set_option(P.OPT_PERSISTENT, persistent)
            g.step(4)
            g.step(3)
            g.synchronize()
            outs.append([[g.fields_blocks(c, l) for l in range(wl.n_levels)]
                         + ([g.force_history(c)[0]] if wl.body is not None else [])
                         for c, wl in enumerate(wls)])
            g.close()
        if storage == "f64":
            for c in range(len(wls)):
                for x, y in zip(outs[0][c], outs[1][c]):
                    assert np.array_equal(x, y, equal_nan=True), c
            continue
        num = den = 0.0
        for c, wl in enumerate(wls):
            for l in range(wl.n_levels):
                a, b = outs[1][c][l], outs[0][c][l]
                m = ~np.isnan(a[:, 0])
                assert (np.isnan(b[:, 0]) == ~m).all(), (c, l)
                for k in (1, 2):
                    num += float(((b[:, k][m] - a[:, k][m]) ** 2).sum())
                    den += float((a[:, k][m] ** 2).sum())
        e = math.sqrt(num / den)
        print(f"  persistent vs chain rel L2 u: {e:.3e}", flush=True)
        assert e <= 1e-3


def test_persistent_barrier_time_out_is_reported(env):
    """A grid barrier of the persistent step that gives up (forced from the
    host: one poll per wait) ends the launch normally and makes synchronize
    report SBT_ERR_DEVICE; the launch's last workgroup resets the barrier
    state, so after re-initialising, the same context steps exactly like a
    fresh one."""
    P, _ = env
    wl = W.small_refined_flap()
    g = P.Sim(wl, "f64")
    g.set_option(P.OPT_PERSISTENT, 1)
    g.step(1)
    g.synchronize()
    g.set_option(P.OPT_BARRIER_SPINS, 1)
    g.step(1)
    with pytest.raises(P.SbtError) as e:
        g.synchronize()
    assert e.value.code == -3
    g.set_option(P.OPT_BARRIER_SPINS, 0)
    ref = P.Sim(wl, "f64")
    ref.set_option(P.OPT_PERSISTENT, 1)
    for s in (g, ref):
        s.init_uniform(0, 1.0, 0.05, 0.0)
        s.step(3)
        s.synchronize()
    for l in range(wl.n_levels):
        for a, b in zip(g.fields(0, l), ref.fields(0, l)):
            assert np.array_equal(a, b, equal_nan=True), l
    assert np.array_equal(g.force_history()[0], ref.force_history()[0])


def test_checkpoint_resume_bitwise(env):
    P, _ = env
    wl = W.small_refined_flap()
    a = P.Sim(wl, "f32")
    a.step(2)
    st = a.read_state()
    a.step(3)
    ref = [a.fields(0, l) for l in range(wl.n_levels)] + [a.force_history()]
    b = P.Sim(wl, "f32")
    b.write_state(st)
    b.step(3)
    got = [b.fields(0, l) for l in range(wl.n_levels)] + [b.force_history()]
    for x, y in zip(ref, got):
        for p, q in zip(x, y):
            assert np.array_equal(p, q, equal_nan=True)


def test_nonfinite_detected(env):
    P, _ = env
    wl = W.tgv(32)
    g = P.Sim(wl, "f64")
    rho, u, v = wl.init(0, 32, 32)
    rho = rho.copy()
    rho[5, 7] = np.nan
    g.init_fields(0, 0, rho, u, v)
    g.step(1)
    with pytest.raises(P.SbtError) as e:
        g.synchronize()
    assert e.value.code == -6


def test_marker_outside_finest_level(env):
    P, _ = env
    wl = W.small_refined_flap()
    b = wl.body
    params = list(b.params)
    params[0] = 4.0        # pivot next to the domain edge, far outside the finest level
    bad = wl.replace(body=W.Body(b.kind, b.xb, b.yb, b.ds, params))
    g = P.Sim(bad, "f64")
    g.step(1)
    with pytest.raises(P.SbtError) as e:
        g.synchronize()
    assert e.value.code == -7


def test_diagnostics_match_oracle(env):
    wl = W.tgv_patch(m=3)
    g, o = run_pair(env, wl, 20)
    dg, do = g.diagnostics(), o.diagnostics()
    assert abs(dg[0] - do[0]) <= 1e-12 * do[0]
    assert np.abs(dg[1:] - do[1:]).max() <= 1e-12 * do[0]


# ---- full-size batch (the benchmark workload, in its launch configuration) ------

def _dense_cells(wl):
    return sum(wl.nx0 * wl.ny0 * 4 ** l for l in range(wl.n_levels))


SWEEP_STEPS = 8


@pytest.fixture(scope="module")
def sweep_f64(env):
    P, _ = env
    wls = W.batch_sweep()
    print(f"batch sweep: {len(wls)} cases, f64, graph, {SWEEP_STEPS} global steps", flush=True)
    g = P.Sim(wls, "f64")
    g.step(SWEEP_STEPS)
    g.synchronize()
    return wls, g


def test_sweep_cases_match_oracle(env, sweep_f64):
    """The 64-case batch in FP64 through the graph-replayed launch chain the
    benchmark times, 8 global steps (64 finest substeps of every case),
    against the oracle run of a case alone (8 global steps = 8 * 2^(4-m)
    coarse steps of a case with m levels): the smallest 2- and 3-level
    cases, and the smallest, the median and the largest 4-level case."""
    P, O = env
    wls, g = sweep_f64
    V = max(w.n_levels for w in wls)
    order = sorted(range(len(wls)), key=lambda c: _dense_cells(wls[c]))
    picked = []
    for m in (2, 3):
        picked += [c for c in order if wls[c].n_levels == m][:1]
    four = [c for c in order if wls[c].n_levels == 4]
    picked += [four[0], four[len(four) // 2], four[-1]]
    for c in picked:
        wl = wls[c]
        o = O.OracleSim(wl)
        o.step(SWEEP_STEPS * 2 ** (V - wl.n_levels))
        print(f"sweep case {c} ({wl.nx0}x{wl.ny0}, {wl.n_levels} levels)", flush=True)
        compare_levels(g, o, wl, TOL64, c=c)
        fg, _ = compare_history(g, o, c=c, tol=TOL_MOVING_HISTORY)
        assert len(fg) == SWEEP_STEPS * 2 ** (V - 1)


def test_sweep_batch_equals_cases_alone(env, sweep_f64):
    """Any size: every case of the batch equals, bit for bit, the same case
    run in a context of its own (batching changes no arithmetic)."""
    P, _ = env
    wls, g = sweep_f64
    V = max(w.n_levels for w in wls)
    for c, wl in enumerate(wls):
        a = P.Sim(wl, "f64")
        a.step(SWEEP_STEPS * 2 ** (V - wl.n_levels))
        a.synchronize()
        for l in range(wl.n_levels):
            x, y = g.fields_blocks(c, l), a.fields_blocks(0, l)
            assert np.array_equal(x, y, equal_nan=True), (c, l)
        assert np.array_equal(g.force_history(c)[0], a.force_history()[0]), c
        a.close()


def test_sweep_f16s_error_ceiling(env, sweep_f64):
    """The benchmark's storage form on the full batch: relative L2 of
    velocity against the FP64 batch after the same 8 global steps."""
    P, _ = env
    wls, g = sweep_f64
    h = P.Sim(wls, "f16s")
    h.step(SWEEP_STEPS)
    h.synchronize()
    num = den = 0.0
    for c, wl in enumerate(wls):
        for l in range(wl.n_levels):
            a, b = g.fields_blocks(c, l), h.fields_blocks(c, l)     # [block][rho, ux, uy][cell]
            m = ~np.isnan(a[:, 0])
            for k in (1, 2):
                num += float(((b[:, k][m] - a[:, k][m]) ** 2).sum())
                den += float((a[:, k][m] ** 2).sum())
    e = math.sqrt(num / den)
    print(f"  f16s vs f64 rel L2 u: {e:.3e}", flush=True)
    assert e <= 5e-3


# ---- physics against the paper's printed values ------------------------------------

def test_cylinder_table1_full_size(env):
    """Configuration C2 (1024x512, D 40, 126 markers, Re 100) run to a
    periodic wake: mean drag, rms lift and Strouhal number against Sec. 3.3,
    Table 1 (tests/golden/cylinder_table1.json).  C2's channel is 512 cells
    high with symmetry edges (blockage D/H = 0.078), which raises drag and
    shedding frequency above the paper's values, so C_D may sit up to 15 %
    and St up to 10 % above them (measured: C_D 1.469, St 0.169, C_L' 0.294);
    a lost factor 2, a wrong sign or a missing ds moves them far more."""
    import json
    import os
    P, _ = env
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cylinder_table1.json")))["Re100"]
    wl = W.cylinder()
    g = P.Sim(wl, "f64")
    n, chunk = 100000, 10000
    for done in range(0, n, chunk):
        g.step(chunk)
        g.synchronize()
        print(f"  cylinder steps {done + chunk}", flush=True)
    fx, fy = g.force_history()
    U, D = wl.meta["U"], wl.meta["D"]
    cd, cl = fx / (0.5 * U * U * D), fy / (0.5 * U * U * D)
    tail = slice(len(cl) - 30000, len(cl))
    c = cl[tail] - cl[tail].mean()
    up = np.nonzero((c[:-1] < 0) & (c[1:] >= 0))[0]
    assert len(up) >= 4, "no periodic shedding"
    st = D / (np.diff(up).mean() * U)
    print(f"  C_D {cd[tail].mean():.4f}  C_L' {c.std():.4f}  St {st:.4f}", flush=True)
    p = gold["present"]
    assert p["St"] * 0.97 <= st <= p["St"] * 1.10, st
    assert p["CD_mean"] * 0.97 <= cd[tail].mean() <= p["CD_mean"] * 1.15, cd[tail].mean()
    lo, hi = gold["literature_range"]["CL_rms"]
    assert lo <= c.std() <= 1.2 * hi, c.std()


def test_pitch_up_plate_first_lift_peak(env):
    """Sec. 3.5 workload (flat plate of 2.3 % thickness, chord 64 finest
    cells, Re 1000, 70c x 40c channel, 3 levels) run to t* = 1.6: the lift
    history has its first peak near the printed C_L = 2.6 at t* = 1.2
    (tests/golden/pitch_up_plate.json), after which lift keeps rising as the
    leading-edge vortex grows.  Measured here: 3.11 at t* = 1.04 (the ramp
    accelerates at t1 = 1, and this resolution responds earlier than the
    paper's, which it reports as delayed against other solvers), so the
    peak is held to 0.75-1.35 x 2.6 within t* 0.95-1.35; a wrong pitch
    direction, a lost factor 2 or a missing ds fails it."""
    import json
    import os
    P, _ = env
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pitch_up_plate.json")))
    pk = gold["first_lift_peak"]
    wl = W.pitch_up_plate()
    g = P.Sim(wl, "f64")
    U, c = wl.meta["U"], wl.meta["chord"]
    per_t = c / U
    g.step(int(round(1.6 * per_t / 4)))
    g.synchronize()
    fx, fy = g.force_history()
    cl = fy / (0.5 * U * U * c)
    t = (np.arange(len(cl)) + 1) / per_t
    w = (t > 0.9) & (t < 1.4)
    i = int(np.argmax(np.where(w, cl, -np.inf)))
    print(f"  first lift peak C_L {cl[i]:.3f} at t* {t[i]:.3f}; C_L(1.6) {cl[-1]:.3f}", flush=True)
    assert 0.75 * pk["CL"] <= cl[i] <= 1.35 * pk["CL"], cl[i]
    assert 0.95 <= t[i] <= 1.35, t[i]
    assert np.abs(cl[t < 0.8]).max() < 0.3          # no lift before the ramp starts
    assert cl[-1] > 0.6 * cl[i]


@pytest.mark.parametrize("vary_ds", [False, True])
def test_host_markers_match_oracle(env, vary_ds):
    """sbt_set_markers on the graph path against the oracle's caller-placed
    body: the markers of a flapping motion (positions r(t_k), desired
    velocity r(t_k+1) - r(t_k), and with vary_ds arc-length weights that
    change every step) are set before every step.  The GPU's step n runs the
    forcing loop of substep n (it collides one substep ahead; step 1 also
    runs substep 0), so the oracle is fed substep 0 with the markers of
    substep 1 and substep k >= 1 with those of k; both must agree bit for
    bit."""
    P, O = env
    U, chord = 0.05, 24.0
    xb, yb, ds = W.ellipse_markers(chord / 2, chord / 16, 60)
    flap = W.Body(W.BODY_FLAP, xb, yb, ds, W.flap_params(64.0, 64.0, chord, 30.0, 2.5 * np.pi, U))
    wl = W.Workload(name="flap1", nx0=128, ny0=128, tau0=0.56, bc=(W.INFLOW, W.OUTFLOW, W.SYMMETRY, W.SYMMETRY),
                    bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3, body=flap, init=W.uniform_init(1.0, U, 0.0))

    def markers(k):
        X, Y = O.body_positions(wl, k)
        X1, Y1 = O.body_positions(wl, k + 1)
        w = np.asarray(ds) * (1.0 + 0.05 * np.sin(0.7 * k)) if vary_ds else None
        return X, Y, X1 - X, Y1 - Y, w

    n = 40
    X0, Y0 = markers(0)[:2]
    host = wl.replace(body=W.Body(W.BODY_HOST, X0, Y0, ds, [0.0] * 16))
    o = O.OracleSim(host)
    for k in range(n):
        o.set_markers(*markers(max(k, 1)))
        o.step(1)
    g = P.Sim(host, "f64")
    for k in range(1, n + 1):
        g.set_markers(0, *markers(k))
        g.step(1)
    g.synchronize()
    for a, b in zip(g.fields(0, 0), o.fields(0)):
        assert np.array_equal(a, b, equal_nan=True)
    fg, fo = g.force_history()[0], o.force_history()[0]
    assert len(fg) == len(fo) == 40 and np.array_equal(fg, fo)


def test_autotune_keeps_state_and_results(env, tmp_path):
    """sbt_autotune times block-run lengths on the live context and restores
    its state: stepping after tuning gives the same bits as an untuned run."""
    P, _ = env
    wl = W.small_refined_flap()
    a = P.Sim(wl, "f32")
    a.step(2)
    a.autotune(steps=1, cache_path=str(tmp_path / "tune.json"))
    a.step(3)
    b = P.Sim(wl, "f32")
    b.step(5)
    for l in range(wl.n_levels):
        assert np.array_equal(a.fields_blocks(0, l), b.fields_blocks(0, l), equal_nan=True)
    assert np.array_equal(a.force_history()[0], b.force_history()[0])
    c = P.Sim(wl, "f32")              # the cached choice is read back, no trials
    c.autotune(steps=1, cache_path=str(tmp_path / "tune.json"))
    c.step(5)
    for l in range(wl.n_levels):
        assert np.array_equal(c.fields_blocks(0, l), b.fields_blocks(0, l), equal_nan=True)


def test_single_marker_body(env):
    """Degenerate body: one marker (one lane of the forcing workgroup, one
    4x4 stencil) in a uniform stream, against the oracle."""
    U = 0.05
    body = W.Body(W.BODY_FIXED, np.array([0.0]), np.array([0.0]), np.array([1.0]), [40.3, 31.7] + [0.0] * 14)
    wl = W.Workload(name="one_marker", nx0=96, ny0=64, tau0=0.6, bc=(W.INFLOW, W.OUTFLOW, W.SYMMETRY, W.SYMMETRY),
                    bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3, body=body, init=W.uniform_init(1.0, U, 0.0))
    g, o = run_pair(env, wl, 50)
    compare_levels(g, o, wl, TOL64, exact=True)
    fg, _ = compare_history(g, o, exact=True)
    assert fg[-1] > 0          # the marker drags the stream


def test_set_markers_rejects_other_bodies(env):
    P, _ = env
    wl = W.small_cylinder()
    g = P.Sim(wl, "f64")
    n = len(wl.body.xb)
    with pytest.raises(P.SbtError) as e:
        g.set_markers(0, np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n))
    assert e.value.code == -1


# ---- three dimensions: D3Q19 on one periodic level ---------------------------

def rel_l2_3(g, o):
    _, u, v, w = g
    _, uo, vo, wo = o
    num = np.sqrt(((u - uo) ** 2 + (v - vo) ** 2 + (w - wo) ** 2).sum())
    return num / np.sqrt((uo ** 2 + vo ** 2 + wo ** 2).sum())


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("make", [lambda: W.shear_wave3(32, nz=32).replace(fext=(2e-6, -1e-6, 3e-6)),
                                  lambda: W.tgv3(32, nz=16, tau=0.6)])
def test_3d_fp64_matches_oracle(env, make, q):
    """D3Q19 and D3Q27, FP64, against the oracle after 60 steps (forced shear
    wave, z-extended vortex): every field within 1e-12, in practice
    bit-exact."""
    P, O = env
    wl = make().replace(lattice=q)
    print(f"case {wl.name} f64", flush=True)
    g = P.Sim3(wl, "f64")
    o = O.Oracle3Sim(wl)
    g.step(60)
    g.synchronize()
    o.step(60)
    fg, fo = g.fields(), o.fields()
    e = rel_l2_3(fg, fo)
    dr = np.abs(fg[0] - fo[0]).max()
    print(f"  rel L2 u {e:.3e}  max |drho| {dr:.3e}", flush=True)
    assert e <= TOL64 and dr <= 1e-14


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f32", 2e-5), ("f16s", 3e-3), ("bf16s", 3e-2)])
def test_3d_storage_forms(env, storage, tol, q):
    """The reduced storage forms on a 32x32x8 vortex, 300 steps, against the
    FP64 oracle (the 2D ceilings)."""
    P, O = env
    wl = W.tgv3(32, nz=8).replace(lattice=q)
    print(f"case {wl.name} {storage}", flush=True)
    g = P.Sim3(wl, storage)
    o = O.Oracle3Sim(wl)
    g.step(300)
    g.synchronize()
    o.step(300)
    e = rel_l2_3(g.fields(), o.fields())
    print(f"  rel L2 u {e:.3e}", flush=True)
    assert e <= tol


@pytest.mark.parametrize("storage,tol,q", [("f64", 0.0, 19), ("f16s", 3e-3, 19), ("f32", 2e-5, 27)])
def test_3d_full_size_periodic_tiling(env, storage, tol, q):
    """512^3 (the size the 3D benchmark times) started from one 32x32 plane
    of the vortex tiled across x, y and z: by translation invariance every
    cell must equal the oracle's 32x32x2 run at (x mod 32, y mod 32); checked
    on sampled planes after 20 steps.  FP64 bit-exact; F16S within its
    ceiling."""
    P, O = env
    small = W.tgv3(32, nz=2, period=32).replace(lattice=q)
    cell = small.init(32, 32, 2, 0, 1)        # one plane, tiled exactly (no re-rounded cosines)

    def tiled(nx, ny, nz, z0=0, z1=None):
        z1 = nz if z1 is None else z1
        return tuple(np.tile(a, (z1 - z0, ny // 32, nx // 32)) for a in cell)

    big = W.tgv3(512, nz=512, period=32).replace(init=tiled, lattice=q)
    print(f"case tgv3 512^3 period 32 D3Q{q} {storage}", flush=True)
    g = P.Sim3(big, storage)
    o = O.Oracle3Sim(small)
    g.step(20)
    g.synchronize()
    o.step(20)
    ref = [np.tile(a[:1], (1, 16, 16)) for a in o.fields()]
    for z in (0, 255, 511):
        fg = g.fields(z, z + 1)
        e = rel_l2_3(fg, ref)
        print(f"  plane {z}: rel L2 u {e:.3e}", flush=True)
        assert e <= tol
        if storage == "f64":
            assert all(np.array_equal(a, b) for a, b in zip(fg, ref))


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", 2e-5), ("f16s", 3e-3)])
def test_3d_walls_channel(env, storage, tol, q):
    """Walls across z with a moving top wall and a body force (Couette plus
    Poiseuille), 400 steps from rest, against the oracle."""
    P, O = env
    wl = W.channel3(n=16, nz=24, tau=0.8, g=2e-6, lid=0.02, lattice=q)
    print(f"case {wl.name} D3Q{q} {storage}", flush=True)
    g = P.Sim3(wl, storage)
    o = O.Oracle3Sim(wl)
    g.step(400)
    g.synchronize()
    o.step(400)
    fg, fo = g.fields(), o.fields()
    e = rel_l2_3(fg, fo)
    print(f"  rel L2 u {e:.3e}", flush=True)
    assert e <= tol
    if storage == "f64":
        assert all(np.array_equal(a, b) for a, b in zip(fg, fo))


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("make,steps,storage,tol", [
    (lambda q: W.solid_channel3(n=16, nz=24, tau=0.8, g=1e-5, q_bottom=0.3, q_top=0.7, lattice=q), 300, "f64", TOL64),
    (lambda q: W.sphere3(32, r=5.0, g=2e-5, lattice=q), 200, "f64", TOL64),
    (lambda q: W.sphere3(32, r=5.0, g=2e-5, lattice=q), 200, "f32", 2e-5),
    (lambda q: W.sphere3(32, r=5.0, g=2e-5, lattice=q), 200, "f16s", 5e-3)])
def test_3d_solid_cells(env, make, steps, storage, tol, q):
    """3D solid cells with interpolated bounce-back: a channel with walls at
    link fractions 0.3 / 0.7 (both Bouzidi branches) and a solid sphere in a
    forced periodic box (every fraction in (0, 1)), against the oracle; FP64
    bit-exact, solid cells read NaN on both sides."""
    P, O = env
    wl = make(q)
    print(f"case {wl.name} D3Q{q} {storage}", flush=True)
    g = P.Sim3(wl, storage)
    o = O.Oracle3Sim(wl)
    g.step(steps)
    g.synchronize()
    o.step(steps)
    fg, fo = g.fields(), o.fields()
    m = ~np.isnan(fo[1])
    assert np.array_equal(m, ~np.isnan(fg[1]))
    fgm, fom = [a[m] for a in fg], [a[m] for a in fo]
    e = rel_l2_3(fgm, fom)
    print(f"  rel L2 u {e:.3e}", flush=True)
    assert e <= tol
    if storage == "f64":
        assert all(np.array_equal(a, b) for a, b in zip(fgm, fom))


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", 2e-5), ("f16s", 3e-3), ("bf16s", 3e-2)])
def test_3d_immersed_sphere(env, storage, tol, q):
    """A fixed IBM sphere (402 markers, N_F = 3) in a forced periodic box:
    fields and body force against the oracle after 150 steps; FP64
    bit-exact."""
    P, O = env
    wl = W.ibm_sphere3(24, r=4.0, tau=1.0, g=1e-5, lattice=q)
    print(f"case {wl.name} D3Q{q} {storage}", flush=True)
    g = P.Sim3(wl, storage)
    o = O.Oracle3Sim(wl)
    g.step(150)
    g.synchronize()
    o.step(150)
    e = rel_l2_3(g.fields(), o.fields())
    fg, fo = g.body_force(), o.body_force()
    ef = np.abs(fg - fo).max() / np.abs(fo).max()
    print(f"  rel L2 u {e:.3e}  body force {fg}  rel err {ef:.3e}", flush=True)
    assert e <= tol and ef <= max(tol, 1e-12) * 10
    if storage == "f64":
        assert all(np.array_equal(a, b) for a, b in zip(g.fields(), o.fields()))
        assert np.array_equal(fg, fo)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", 2e-5), ("f16s", 3e-3), ("bf16s", 3e-2)])
def test_3d_flapping_ellipsoid(env, storage, tol, q):
    """An IBM ellipsoid pitching about y and plunging along z in a uniform
    stream (400 markers, N_F = 3, 240-step period): the forcing loop
    rebuilds the markers, desired velocities, taps and box every step.
    Fields and body force against the oracle over half a period; FP64
    bit-exact."""
    P, O = env
    wl = W.flapping_ellipsoid3(32, lattice=q)
    print(f"case {wl.name} D3Q{q} {storage}", flush=True)
    g = P.Sim3(wl, storage)
    o = O.Oracle3Sim(wl)
    for _ in range(3):
        g.step(40)
        g.synchronize()
        o.step(40)
        e = rel_l2_3(g.fields(), o.fields())
        fg, fo = g.body_force(), o.body_force()
        ef = np.abs(fg - fo).max() / np.abs(fo).max()
        print(f"  rel L2 u {e:.3e}  body force {fg}  rel err {ef:.3e}", flush=True)
        assert e <= tol and ef <= max(tol, 1e-12) * 10
        if storage == "f64":  # the pose comes from the same C library sin / cos as the oracle's
            assert all(np.array_equal(a, b) for a, b in zip(g.fields(), o.fields()))
            assert np.array_equal(fg, fo)
    g.close()


@pytest.mark.parametrize("storage,tol", [("f64", TOL64), ("f32", 2e-5)])
def test_3d_flapping_ellipsoid_many_markers(env, storage, tol):
    """2400 markers (three staging blocks of the spread kernel and three
    chunks of the ordered body-force sum), N_F = 3, chord 24 in a 48^3 box:
    fields and body force against the oracle over 20 steps; FP64 bit for
    bit."""
    P, O = env
    wl = W.flapping_ellipsoid3(48, chord=24.0, n_markers=2400)
    print(f"case {wl.name} 2400 markers {storage}", flush=True)
    g = P.Sim3(wl, storage)
    o = O.Oracle3Sim(wl)
    for _ in range(2):
        g.step(10)
        g.synchronize()
        o.step(10)
        e = rel_l2_3(g.fields(), o.fields())
        fg, fo = g.body_force(), o.body_force()
        ef = np.abs(fg - fo).max() / np.abs(fo).max()
        print(f"  rel L2 u {e:.3e}  body force rel err {ef:.3e}", flush=True)
        assert e <= tol and ef <= max(tol, 1e-12) * 10
        if storage == "f64":
            assert all(np.array_equal(a, b) for a, b in zip(g.fields(), o.fields()))
            assert np.array_equal(fg, fo)
    g.close()


def test_3d_moving_body_box_overflow(env):
    """A moving body whose stencil box outgrows the capacity the caller gave
    (the t = 0 box exactly): the forcing loop skips the force and the next
    synchronisation reports SBT_ERR_MARKER_OUTSIDE."""
    P, _ = env
    wl = W.flapping_ellipsoid3(32)
    X, Y, Z, dA, it = wl.body
    p = wl.motion[1]
    ca, sa = math.cos(p[3] - p[4] * math.sin(p[7])), math.sin(p[3] - p[4] * math.sin(p[7]))
    zc = p[2] + 0.5 * p[5]
    pos = (p[0] + X * ca + Z * sa, p[1] + Y, zc - X * sa + Z * ca)
    cells = int(np.prod([np.floor(v - 1.5).max() - np.floor(v - 1.5).min() + 4 for v in pos]))
    g = P.Sim3(wl, "f32", box_cells=cells)
    g.step(60)
    with pytest.raises(P.SbtError, match="ibm_box_cells"):
        g.body_force()             # the force of a step without the body's forcing is no result
    with pytest.raises(P.SbtError, match="ibm_box_cells"):
        g.synchronize()
    g.close()
