"""GPU parity of the 3D block forest (``sbt3f_*``) against the FP64 oracle's
forest on the same seeded inputs: FP64 bit for bit (both sides take the same
operations in the same order), the reduced storage forms within the ceilings
of the 2D and single-level 3D paths on the relative L2 norm of velocity.  At
the benchmark's size the oracle cannot hold the finest level densely, so the
full-size checks use properties that hold at any size: a forest tiled from
copies of a small one equals the small oracle run in every tile, and a
uniform stream stays uniform."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 6
TOLS = {"f32": 2e-5, "f16s": 3e-3, "bf16s": 3e-2}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2402_04606_amd as P
    P.lib()
    return P, oracle


def _rel_l2(g, o):
    own = ~np.isnan(o[0])
    num = sum(((g[k] - o[k])[own] ** 2).sum() for k in (1, 2, 3))
    den = sum((o[k][own] ** 2).sum() for k in (1, 2, 3))
    return math.sqrt(num / max(den, 1e-16 * own.sum()))


def _compare(g, o, wl, storage, check_every_level=True):
    worst = 0.0
    for l in range(wl.n_levels):
        fg, fo = g.fields(l), o.fields(l)
        own = ~np.isnan(fo[0])
        assert own.sum() > 0
        assert (np.isnan(fg[0]) == ~own).all(), f"level {l}: owned cells differ"
        if storage == "f64":
            for k in range(4):
                assert np.array_equal(fg[k][own], fo[k][own]), (l, k, np.abs(fg[k] - fo[k])[own].max())
        else:
            e = _rel_l2(fg, fo)
            worst = max(worst, e)
            print(f"  level {l}: rel L2 u {e:.3e}", flush=True)
            assert e <= TOLS[storage], (l, e)
    return worst


CASES = {
    "uniform_nested": lambda q, cf: W.uniform3f(u=(0.04, 0.02, -0.03), n0=16, m=3, lattice=q, cf_mode=cf,
                                                boxes=((1, 1, 1, 1, 3, 3, 3), (2, 3, 3, 3, 5, 5, 5))),
    "slab_xz": lambda q, cf: W.tgv3f(n0=32, m=2, boxes=((1, 0, 0, 2, 8, 2, 6),), plane="xz", lattice=q, cf_mode=cf,
                                     n_third=8),
    "vortex_patch": lambda q, cf: W.vortex3f(n0=16, m=2, boxes=((1, 1, 0, 1, 3, 2, 4),), lattice=q, cf_mode=cf),
    "vortex_nested": lambda q, cf: W.vortex3f(n0=16, m=3, boxes=((1, 1, 1, 1, 3, 3, 3), (2, 3, 3, 3, 5, 5, 5)),
                                              lattice=q, cf_mode=cf, tau0=0.7),
}


@pytest.mark.parametrize("cf", [W.CF_HOMOGENEOUS, W.CF_RESCALE])
@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("case", sorted(CASES))
def test_forest3d_fp64_bitwise(env, case, q, cf):
    """Every owned cell of every level, bit for bit, after the prologue's
    collision and after 1 and STEPS coarse steps; the owned cells of the two
    sides are the same."""
    P, O = env
    wl = CASES[case](q, cf)
    print(f"case {case} D3Q{q} cf {cf} f64", flush=True)
    g = P.Sim3F(wl, "f64")
    o = O.Oracle3FSim(wl)
    _compare(g, o, wl, "f64")
    for n in (1, STEPS - 1):
        g.step(n)
        g.synchronize()
        o.step(n)
        _compare(g, o, wl, "f64")
    dg, do = g.diagnostics(), o.diagnostics()
    assert abs(dg[0] - do[0]) <= 1e-12 * do[0]
    assert np.abs(dg[1:] - do[1:]).max() <= 1e-12 * do[0]


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s"])
@pytest.mark.parametrize("q", [19, 27])
def test_forest3d_storage_forms(env, storage, q):
    """The deviation storage forms on the nested vortex (3 levels, both
    interface operators) after 40 coarse steps."""
    P, O = env
    for cf in (W.CF_HOMOGENEOUS, W.CF_RESCALE):
        wl = CASES["vortex_nested"](q, cf)
        print(f"case vortex_nested D3Q{q} cf {cf} {storage}", flush=True)
        g = P.Sim3F(wl, storage)
        o = O.Oracle3FSim(wl)
        g.step(40)
        g.synchronize()
        o.step(40)
        _compare(g, o, wl, storage)


def test_forest3d_force_and_tiny_domain(env):
    """A body force on a forest whose level 0 is a single block (every
    neighbour of a block is the block itself): bit for bit."""
    P, O = env
    wl = W.vortex3f(n0=8, m=2, boxes=((1, 0, 0, 0, 2, 2, 1),)).replace(fext=(2e-6, -1e-6, 3e-6))
    g = P.Sim3F(wl, "f64")
    o = O.Oracle3FSim(wl)
    g.step(10)
    g.synchronize()
    o.step(10)
    _compare(g, o, wl, "f64")


def test_forest3d_reinit_after_steps(env):
    """Initialising again after steps restarts from the new state: the run
    repeats bit for bit."""
    P, O = env
    wl = CASES["vortex_patch"](19, W.CF_HOMOGENEOUS)
    g = P.Sim3F(wl, "f64")
    g.step(3)
    g.synchronize()
    first = [g.fields(l) for l in range(2)]
    for l in range(2):
        for box in g.init_boxes(l):
            g.init_box(l, box, *wl.init(l, *box))
    g.step(3)
    g.synchronize()
    for l in range(2):
        for a, b in zip(first[l], g.fields(l)):
            assert np.array_equal(a, b, equal_nan=True)


# ---- full size -------------------------------------------------------------------

TILE = 32          # level-0 cells of one tile
TILE_BOXES = ((1, 2, 2, 2, 6, 6, 6), (2, 6, 6, 6, 10, 10, 10))


def _tiled(reps, lattice=19, cf=W.CF_HOMOGENEOUS):
    """reps^3 copies of a 32^3 forest with a nested 3-level patch and a
    periodic vortex of period 32."""
    base = W.vortex3f(n0=TILE, m=3, boxes=TILE_BOXES, lattice=lattice, cf_mode=cf)
    boxes = []
    for (l, *b) in TILE_BOXES:
        per = (TILE >> 3) << l          # blocks per tile on level l
        for k in range(reps):
            for j in range(reps):
                for i in range(reps):
                    o = (i * per, j * per, k * per)
                    boxes.append((l, *(b[a] + o[a] for a in range(3)), *(b[3 + a] + o[a] for a in range(3))))
    init0 = base.init

    def init(level, x0, y0, z0, nx, ny, nz):
        p = TILE << level                # the vortex repeats every p level cells
        cell = init0(level, 0, 0, 0, p, p, p)
        idx = [np.arange(o, o + n) % p for o, n in ((z0, nz), (y0, ny), (x0, nx))]
        return tuple(np.broadcast_to(a, (p, p, p))[np.ix_(*idx)] for a in cell)

    big = base.replace(nx0=TILE * reps, ny0=TILE * reps, nz0=TILE * reps, boxes=tuple(boxes), init=init,
                       name=f"tiled{reps}")
    return base, big


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_forest3d_full_size_tiling(env, storage):
    """256^3 level-0 cells made of 8^3 copies of the 32^3 three-level forest
    (the size the 3D forest benchmark times): by translation invariance
    every tile equals the oracle's run of one copy; checked on sampled
    planes of every level after 4 coarse steps."""
    P, O = env
    reps = 8
    base, big = _tiled(reps)
    print(f"case tiled forest {reps}^3 x 32^3 {storage}", flush=True)
    g = P.Sim3F(big, storage)
    o = O.Oracle3FSim(base)
    g.step(4)
    g.synchronize()
    o.step(4)
    for l in range(3):
        p = TILE << l
        fo = o.fields(l)
        for z in (3, p * reps // 2 + 5, p * reps - 2):
            for y0 in (0, p * (reps - 1)):
                box = (0, y0, z, p * reps, p, 1)
                fg = g.fields(l, box)
                ref = [np.tile(a[z % p][None], (1, 1, reps)) for a in fo]
                own = ~np.isnan(ref[0])
                assert (np.isnan(fg[0]) == ~own).all()
                if not own.any():
                    continue
                if storage == "f64":
                    for k in range(4):
                        assert np.array_equal(fg[k][own], ref[k][own]), (l, z, y0, k)
                else:
                    e = _rel_l2(fg, ref)
                    assert e <= TOLS[storage], (l, z, e)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
def test_forest3d_bench_case_uniform_stream(env, storage):
    """The benchmark's forest (256^3 level-0 cells, nested level-1 and
    level-2 boxes) carrying a uniform stream: both interface operators map
    equilibrium to itself, so every owned cell keeps the stream (to the
    storage form's rounding) after 4 coarse steps; sampled planes."""
    P, O = env
    wl = W.forest3d_bench().replace(init=W.uniform3f(u=(0.04, 0.02, -0.03)).init)
    print(f"case forest3d bench uniform {storage}", flush=True)
    g = P.Sim3F(wl, storage)
    g.step(4)
    g.synchronize()
    tol = {"f64": 1e-13, "f32": 2e-6, "f16s": 2e-3, "bf16s": 2e-2}[storage]
    for l in range(wl.n_levels):
        x0, y0, z0, nx, ny, nz = g.region_box(l)
        for z in (z0, z0 + nz // 2, z0 + nz - 1):
            r, u, v, w = g.fields(l, (x0, y0, z, nx, ny, 1))
            own = ~np.isnan(r)
            assert own.any()
            assert np.abs(r[own] - 1.0).max() <= tol * 10
            for a, ua in ((u, 0.04), (v, 0.02), (w, -0.03)):
                assert np.abs(a[own] - ua).max() <= tol * 0.05, (l, z, np.abs(a[own] - ua).max())
