"""Host side of the 3D block forest (no GPU): the library's planner builds
the same cells as the oracle's forest -- owned, halo and hidden, level by
level -- and both reject the same invalid topologies."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def pkg():
    import paper_2402_04606_amd as P
    try:
        P.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return P


TOPOLOGIES = {
    "nested3": W.uniform3f(n0=16, m=3, boxes=((1, 1, 1, 1, 3, 3, 3), (2, 3, 3, 3, 5, 5, 5))),
    "slab_z": W.tgv3f(n0=32, m=2, boxes=((1, 0, 0, 2, 8, 2, 6),), plane="xz", n_third=8),
    "wrapping_patch": W.vortex3f(n0=16, m=2, boxes=((1, 1, 0, 1, 3, 2, 4),)),
    "two_boxes_touching": W.uniform3f(n0=32, m=2, boxes=((1, 1, 1, 1, 3, 3, 3), (1, 3, 1, 1, 5, 2, 2))),
    "single_block_level0": W.vortex3f(n0=8, m=2, boxes=((1, 0, 0, 0, 2, 2, 1),)),
    "four_levels": W.uniform3f(n0=8, m=4, boxes=((1, 0, 0, 0, 2, 2, 2), (2, 1, 1, 1, 3, 3, 3),
                                                  (3, 3, 3, 3, 5, 5, 5))),
}


@pytest.mark.parametrize("name", sorted(TOPOLOGIES))
def test_planner_cells_match_the_oracle(pkg, orc, name):
    wl = TOPOLOGIES[name]
    o = orc.Oracle3FSim(wl)
    for l in range(wl.n_levels):
        ko = o.kinds(l)
        kg = pkg.level_kinds3f(wl, l)
        assert (kg == ko).all(), (name, l)
        info = pkg.level_info3f(wl, l)
        assert info[:3] == o.level_size(l)
        assert info[3:] == tuple(int((ko == k).sum()) for k in (1, 2, 3))


BAD = {
    # a level-2 box outside the level-1 region
    "not_nested": ((1, 1, 1, 1, 3, 3, 3), (2, 0, 0, 0, 2, 2, 2)),
    # a level-2 box flush with the level-1 boundary: its halo has no owned parent
    "no_clearance": ((1, 1, 1, 1, 3, 3, 3), (2, 2, 2, 2, 4, 4, 4)),
}


@pytest.mark.parametrize("name", sorted(BAD))
def test_invalid_topologies_rejected_by_both(pkg, orc, name):
    wl = W.uniform3f(n0=16, m=3, boxes=BAD[name])
    with pytest.raises(RuntimeError):
        orc.Oracle3FSim(wl)
    with pytest.raises(pkg.SbtError) as e:
        pkg.level_info3f(wl, 0)
    assert e.value.code == -2


def test_planner_argument_errors(pkg):
    import ctypes as C
    ok = W.uniform3f(n0=16, m=2, boxes=((1, 1, 1, 1, 3, 3, 3),))
    for bad in (ok.replace(boxes=((1, 1, 1, 1, 9, 3, 3),)),       # outside the level-1 grid
                ok.replace(boxes=((2, 1, 1, 1, 3, 3, 3),)),       # level beyond n_levels - 1
                ok.replace(nx0=12),                               # not a multiple of 8
                ok.replace(lattice=15),
                ok.replace(tau0=0.5),
                ok.replace(cf_mode=W.CF_RESCALE, tau0=1.0),       # RESCALE with tau_0 = 1
                ok.replace(n_levels=7)):
        d, keep = pkg.desc3f(bad)
        n = C.c_size_t()
        assert pkg.lib().sbt3f_plan(C.byref(d), C.byref(n)) == -1
    d, keep = pkg.desc3f(ok)
    n = C.c_size_t()
    assert pkg.lib().sbt3f_plan(C.byref(d), C.byref(n)) == 0 and n.value > 0


def test_plan_size_scales_with_storage(pkg):
    import ctypes as C
    wl = TOPOLOGIES["nested3"]
    sizes = {}
    for st in (pkg.F64, pkg.F32, pkg.F16S):
        d, keep = pkg.desc3f(wl, st)
        n = C.c_size_t()
        assert pkg.lib().sbt3f_plan(C.byref(d), C.byref(n)) == 0
        sizes[st] = n.value
    assert sizes[pkg.F64] > sizes[pkg.F32] > sizes[pkg.F16S]
