"""Pins for the oracle's 3D block forest: the refinement of Sec. 2.3 and the
coarse-fine interface of Sec. 2.4 in three dimensions (D3Q19 and D3Q27,
periodic).

What fixes the 3D forest from outside itself:
  * a flow that is invariant along one axis, on a forest that is invariant
    along it too, sums (over the velocity component on that axis) to the 2D
    D2Q9 forest: both 3D lattices project exactly onto D2Q9 (their weights
    summed over a column are D2Q9's, the equilibrium and Guo's term only see
    the in-plane velocity), and so do collision, streaming, explosion and the
    8-child mean -- so every plane reproduces the separately pinned 2D
    oracle to rounding;
  * a single level is the uniform 3D solver;
  * a uniform stream is a fixed point of both interface operators;
  * a corner-free slab under the homogeneous operators conserves mass;
  * the lattices are invariant under permutations of the axes, so a forest
    and a flow permuted together give the permuted result;
  * a refined 3D patch leaves the Taylor-Green decay close to the exact one,
    with an interface error that falls with resolution.
The planted-slip tests build copies of oracle.c with a plausible mistake and
check that one of these pins rejects each."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

PLANES = {"xy": (0, 1), "xz": (0, 2), "yz": (1, 2)}


def _pair(m, plane, lattice, cf, boxes2, n0=32, tau0=0.8):
    """(2D workload, matching 3D workload invariant along the third axis)."""
    a_ax, b_ax = PLANES[plane]
    boxes3 = []
    for (l, x0, y0, x1, y1) in boxes2:
        lo, hi = [0, 0, 0], [max(1, (4 << l) // 8)] * 3
        lo[a_ax], hi[a_ax], lo[b_ax], hi[b_ax] = x0, x1, y0, y1
        boxes3.append((l, *lo, *hi))
    w2 = W.tgv(n0, tau=tau0, u0=0.02, n_levels=m, boxes=list(boxes2)).replace(block_n=8, cf_mode=cf)
    w3 = W.tgv3f(n0=n0, m=m, boxes=tuple(boxes3), tau0=tau0, lattice=lattice, cf_mode=cf, plane=plane,
                 n_third=4)
    return w2, w3


def _plane_view(a, plane):
    """A dense 3D array [nz, ny, nx] as [third, b, a] -- the 2D layout [y, x]
    with the invariant axis first."""
    if plane == "xy":
        return a
    if plane == "xz":
        return a.transpose(1, 0, 2)
    return a.transpose(2, 0, 1)


def _projection_gap(orc, m, plane, lattice, cf, boxes2, steps, so=None):
    w2, w3 = _pair(m, plane, lattice, cf, boxes2)
    s2, s3 = orc.OracleSim(w2), orc.Oracle3FSim(w3, so=so)
    s2.step(steps)
    s3.step(steps)
    a_ax, b_ax = PLANES[plane]
    gap = 0.0
    for l in range(m):
        k3 = _plane_view(s3.kinds(l), plane)
        if not (k3 == s2.kinds(l)[None]).all():
            return math.inf
        r2, u2, v2 = s2.fields(l)
        f3 = s3.fields(l)
        r3, ua, ub = (_plane_view(f3[i], plane) for i in (0, 1 + a_ax, 1 + b_ax))
        third = _plane_view(f3[1 + 3 - a_ax - b_ax], plane)
        own = s2.kinds(l) == 1
        for x3, x2 in ((r3, r2), (ua, u2), (ub, v2)):
            d = np.abs(x3[:, own] - x2[None, own])
            gap = max(gap, float(np.nan_to_num(d, nan=math.inf).max()))
        gap = max(gap, float(np.nan_to_num(np.abs(third[:, own]), nan=math.inf).max()))
    return gap


BOXES2 = {2: [(1, 2, 2, 6, 6)], 3: [(1, 1, 1, 7, 7), (2, 5, 5, 9, 9)]}


@pytest.mark.parametrize("lattice", [19, 27])
@pytest.mark.parametrize("plane", sorted(PLANES))
@pytest.mark.parametrize("cf", [W.CF_HOMOGENEOUS, W.CF_RESCALE])
def test_invariant_forest_reproduces_the_2d_forest(orc, lattice, plane, cf):
    """A Taylor-Green vortex in one coordinate plane on a forest invariant
    along the third axis: every level's rho and in-plane velocity equal the
    2D oracle's to rounding, the third velocity component stays zero, and
    the kinds of the cells (own, halo, hidden) are the 2D ones, for two and
    three levels."""
    for m in (2, 3):
        assert _projection_gap(orc, m, plane, lattice, cf, BOXES2[m], 6) < 1e-14


def test_single_level_forest_is_the_uniform_3d_solver(orc):
    """m = 1: the forest's collision and streaming are those of the uniform
    periodic solver (orc3_*), whose own pins fix them."""
    for lattice in (19, 27):
        wf = W.tgv3f(n0=32, m=1, boxes=(), lattice=lattice)
        wu = W.tgv3(32, nz=8, tau=0.8, u0=0.02).replace(lattice=lattice)
        a, b = orc.Oracle3FSim(wf), orc.Oracle3Sim(wu)
        a.step(20)
        b.step(20)
        for x, y in zip(a.fields(0), b.fields()):
            assert np.abs(x - y).max() < 1e-15


@pytest.mark.parametrize("lattice", [19, 27])
@pytest.mark.parametrize("cf", [W.CF_HOMOGENEOUS, W.CF_RESCALE])
def test_uniform_stream_on_a_3d_forest(orc, lattice, cf):
    """f_neq = 0 everywhere, so explosion and coalescence are identities: a
    uniform stream across a nested two-box forest (edges and corners in all
    three directions) stays uniform to rounding on every level."""
    wl = W.uniform3f(u=(0.04, 0.02, -0.03), n0=16, m=3,
                     boxes=((1, 1, 1, 1, 3, 3, 3), (2, 3, 3, 3, 5, 5, 5)), lattice=lattice, cf_mode=cf)
    s = orc.Oracle3FSim(wl)
    s.step(6)
    for l in range(3):
        r, u, v, w = s.fields(l)
        own = s.kinds(l) == 1
        assert own.sum() > 0
        assert np.abs(r[own] - 1).max() < 1e-13
        assert np.abs(u[own] - 0.04).max() < 1e-14 and np.abs(v[own] - 0.02).max() < 1e-14
        assert np.abs(w[own] + 0.03).max() < 1e-14


@pytest.mark.parametrize("lattice", [19, 27])
def test_refined_slab_conserves_mass(orc, lattice):
    """A refined slab spanning the periodic x and y axes (interfaces normal
    to z, no edges or corners) under the homogeneous operators: what one
    coarse cell hands the fine halo comes back through the 8-child mean, so
    the volume-weighted mass is conserved to rounding while a vortex in the
    x-z plane drives flow across both interfaces."""
    wl = W.tgv3f(n0=32, m=2, boxes=((1, 0, 0, 2, 8, 2, 6),), plane="xz", lattice=lattice, n_third=8)
    s = orc.Oracle3FSim(wl)
    m0 = s.diagnostics()[0]
    s.step(20)
    assert abs(s.diagnostics()[0] - m0) < 1e-12 * m0


def _permuted(wl, perm):
    """The workload with axes permuted: new axis d is old axis perm[d]."""
    n = (wl.nx0, wl.ny0, wl.nz0)
    boxes = tuple((b[0], *(b[1 + p] for p in perm), *(b[4 + p] for p in perm)) for b in wl.boxes)
    init0 = wl.init

    def init(level, x0, y0, z0, nx, ny, nz):
        size, org = [0, 0, 0], [0, 0, 0]
        for d, p in enumerate(perm):
            size[p], org[p] = (nx, ny, nz)[d], (x0, y0, z0)[d]
        rho, *u = (np.broadcast_to(v, (size[2], size[1], size[0])) for v in init0(level, *org, *size))
        # arrays are [z, y, x]: reverse the axis order to permute, then reverse back
        order = [2 - perm[2 - d] for d in range(3)]
        return (rho.transpose(order), *(u[p].transpose(order) for p in perm))
    return wl.replace(nx0=n[perm[0]], ny0=n[perm[1]], nz0=n[perm[2]], boxes=boxes, init=init)


def test_axis_permutation_equivariance(orc):
    """D3Q19 and D3Q27 are invariant under permutations of the axes: a
    genuinely 3D flow on a box-shaped patch, forest and flow permuted
    together, gives the permuted fields (to rounding) on every level."""
    wl = W.vortex3f(n0=16, m=2, boxes=((1, 1, 1, 1, 3, 3, 3),))
    wl = wl.replace(boxes=((1, 1, 0, 1, 3, 2, 4),))
    base = orc.Oracle3FSim(wl)
    base.step(5)
    for perm in ((1, 2, 0), (2, 0, 1), (1, 0, 2)):
        p = orc.Oracle3FSim(_permuted(wl, perm))
        p.step(5)
        order = [2 - perm[2 - d] for d in range(3)]
        for l in range(2):
            fb, fp = base.fields(l), p.fields(l)
            assert (p.kinds(l) == base.kinds(l).transpose(order)).all()
            pairs = [(fb[0], fp[0])] + [(fb[1 + perm[d]], fp[1 + d]) for d in range(3)]
            for x, y in pairs:
                assert np.nanmax(np.abs(x.transpose(order) - y)) < 1e-15


def _tgv3_error(orc, wl, steps):
    """Relative L2 velocity error against the exact decay, volume-weighted
    over the owned cells of every level."""
    s = orc.Oracle3FSim(wl)
    s.step(steps)
    u0, k, nu = wl.meta["u0"], wl.meta["k"], wl.meta["nu"]
    dec = math.exp(-2 * nu * k * k * steps)
    num = den = 0.0
    for l in range(wl.n_levels):
        x, y, _ = W._centres3(l, *s.level_size(l))
        _, u, v, w = s.fields(l)
        own = s.kinds(l) == 1
        ue, ve = -u0 * np.cos(k * x) * np.sin(k * y) * dec, u0 * np.sin(k * x) * np.cos(k * y) * dec
        num += 8.0 ** -l * ((u - ue) ** 2 + (v - ve) ** 2 + w ** 2)[own].sum()
        den += 8.0 ** -l * (ue ** 2 + ve ** 2)[own].sum()
    return math.sqrt(num / den)


def test_refined_3d_patch_tgv_error_falls_with_resolution(orc):
    """A patch confined in all three directions (so the interface has faces,
    edges and corners) under the homogeneous operators: the Taylor-Green
    error at a fixed physical time stays small and falls by at least 1.6
    when the resolution doubles (the interface is first order)."""
    errs = []
    for n0 in (16, 32):
        b = n0 // 8 * 2                       # level-1 blocks per axis
        wl = W.tgv3f(n0=n0, m=2, boxes=((1, b // 4, b // 4, b // 4, 3 * b // 4, 3 * b // 4, 3 * b // 4),),
                     n_third=n0, u0=0.02 * 16 / n0)
        steps = 25 * (n0 // 16) ** 2          # same diffusive time
        errs.append(_tgv3_error(orc, wl, steps))
    assert errs[0] < 0.05 and errs[1] < errs[0] / 1.6, errs


# ---- planted slips --------------------------------------------------------------

_SLIPS = {
    # the z offset of the children dropped in the 8-child mean
    "child_z": [("sum += F->f[c3(F, 2 * x + cx, 2 * y + cy, 2 * z + cz) * Q3 + i];",
                 "sum += F->f[c3(F, 2 * x + cx, 2 * y + cy, 2 * z) * Q3 + i];")],
    # explosion from the parent's pre-collision populations
    "explode_pre": [("const double *src = C->fs + p * Q3;", "const double *src = C->f + p * Q3;")],
    # the halo's second fine substep streams stale sources
    "no_second_halo": [("else halo_second3f(s, l);", "else {}")],
    # hidden-source test on the cell itself rather than its source
    "hidden_self": [("int sx = x - C3X[i], sy = y - C3Y[i], sz = z - C3Z[i];\n            wrap3(C, &sx, &sy, &sz);\n"
                     "            hid[i]", "int sx = x, sy = y, sz = z;\n            wrap3(C, &sx, &sy, &sz);\n"
                     "            hid[i]")],
    # streaming pulls the z component from the wrong side
    "stream_z_sign": [("int sx = x - C3X[i], sy = y - C3Y[i], sz = z - C3Z[i];\n            wrap3(L, &sx, &sy, &sz);",
                       "int sx = x - C3X[i], sy = y - C3Y[i], sz = z + C3Z[i];\n            wrap3(L, &sx, &sy, &sz);")],
    # a halo layer of one cell instead of two
    "halo_one": [("for (int dz = -2; dz <= 2; ++dz)\n                        for (int dy = -2; dy <= 2; ++dy)\n"
                  "                            for (int dx = -2; dx <= 2; ++dx) {",
                  "for (int dz = -1; dz <= 1; ++dz)\n                        for (int dy = -1; dy <= 1; ++dy)\n"
                  "                            for (int dx = -1; dx <= 1; ++dx) {")],
}


@pytest.mark.parametrize("slip", sorted(_SLIPS))
def test_forest3d_pins_catch_planted_slips(orc, tmp_path, slip):
    from oracle import build as B
    so = orc.load_variant(B.build_variant(_SLIPS[slip], str(tmp_path), "orc3f_" + slip))
    caught = []
    for plane in ("xz", "yz", "xy"):
        for cf in (W.CF_HOMOGENEOUS, W.CF_RESCALE):
            caught.append(_projection_gap(orc, 2, plane, 19, cf, BOXES2[2], 4, so=so) > 1e-12)
    assert any(caught), slip
