"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side forest builder validates descriptors (no GPU call)."""
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pkg():
    import paper_2402_04606_amd as P
    P.lib()
    return P


def declared_symbols():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(sbt(?:3f?)?_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_and_binding_agree(pkg):
    assert declared_symbols() == sorted(pkg.ABI_SYMBOLS)


def test_library_exports_every_symbol(pkg):
    L = pkg.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_plan_sizes(pkg):
    small = pkg.plan([W.tgv(64)], pkg.F64)
    assert small > 2 * 9 * 64 * 64 * 8
    assert pkg.plan([W.tgv(64)], pkg.F16S) < small
    big = pkg.plan(W.batch_sweep(), pkg.F16S)
    assert big > 256 * 2 ** 20          # larger than the 256 MB Infinity Cache


@pytest.mark.parametrize("bad,code", [
    (dict(boxes=[(1, 0, 0, 4, 4)], n_levels=2, body=None), -2),       # touches a wall
    (dict(boxes=[(1, 12, 12, 20, 20), (2, 22, 22, 42, 42)]), -2),     # level 2 not nested
    (dict(boxes=[(1, 12, 12, 20, 20), (2, 24, 24, 40, 40)]), -2),     # no 2:1 margin
    (dict(boxes=[(3, 1, 1, 2, 2)]), -2),                              # level beyond n_levels
    (dict(tau0=0.5), -1),
    (dict(nx0=250), -1),
    (dict(bc=(0, 1, 1, 1)), -1),                                      # unpaired periodic edge
])
def test_plan_rejects_invalid(pkg, bad, code):
    wl = W.cavity().replace(**bad)
    with pytest.raises(pkg.SbtError) as e:
        pkg.plan([wl])
    assert e.value.code == code


def test_plan_rejects_mixed_storage(pkg):
    import ctypes as C
    arr = (pkg.CaseDesc * 2)()
    d0, k0 = pkg.make_desc(W.tgv(32), pkg.F64)
    d1, k1 = pkg.make_desc(W.tgv(32), pkg.F32)
    arr[0], arr[1] = d0, d1
    n = C.c_size_t()
    assert pkg.lib().sbt_plan(arr, 2, C.byref(n)) == -1


def test_plan_rejects_mixed_collision_and_bad_mrt_rates(pkg):
    import ctypes as C
    arr = (pkg.CaseDesc * 2)()
    d0, k0 = pkg.make_desc(W.tgv(32), pkg.F32)
    d1, k1 = pkg.make_desc(W.tgv(32).replace(collision=W.COLL_MRT), pkg.F32)
    arr[0], arr[1] = d0, d1
    n = C.c_size_t()
    assert pkg.lib().sbt_plan(arr, 2, C.byref(n)) == -1
    assert pkg.plan([W.tgv(32).replace(collision=W.COLL_MRT)]) > 0
    for bad in ((0.0, 1.5, 1.5), (1.5, 2.0, 1.5), (1.5, 1.5, -1.0)):
        with pytest.raises(pkg.SbtError):
            pkg.plan([W.tgv(32).replace(collision=W.COLL_MRT, mrt_rates=bad)])


def test_plan_rejects_bad_solids(pkg):
    import numpy as np
    ok = W.ibb_cylinder()
    assert pkg.plan([ok]) > 0
    mask, q = W.solid_circle(128, 64, 2.0, 32.0, 5.0)          # touches the inflow edge
    with pytest.raises(pkg.SbtError):
        pkg.plan([ok.replace(solids=[(0, mask, q)])])
    mask, q = W.solid_circle(128, 64, 40.0, 32.0, 6.0)
    with pytest.raises(pkg.SbtError):
        pkg.plan([ok.replace(solids=[(0, mask, np.zeros_like(q))])])   # q must lie in (0, 1]
    cav = W.cavity_ibb()
    lvl, mask, q = cav.solids[0]
    with pytest.raises(pkg.SbtError):                          # level 1 is covered there
        pkg.plan([cav.replace(solids=[(1, mask[::2, ::2][:512, :512], None)])])
    assert pkg.plan([cav]) > 0


def test_3d_plan_and_validation(pkg):
    import ctypes as C
    d = pkg.Desc3()
    d.nx, d.ny, d.nz, d.tau, d.rho0, d.storage, d.lattice = 64, 32, 16, 0.8, 1.0, pkg.F32, 19
    n = C.c_size_t()
    assert pkg.lib().sbt3_plan(C.byref(d), C.byref(n)) == 0
    assert n.value >= 2 * 19 * 64 * 32 * 16 * 4
    d.lattice = 27
    assert pkg.lib().sbt3_plan(C.byref(d), C.byref(n)) == 0 and n.value >= 2 * 27 * 64 * 32 * 16 * 4
    for field, bad in (("tau", 0.5), ("nx", 0), ("storage", 7), ("rho0", 0.0), ("lattice", 15)):
        e = pkg.Desc3.from_buffer_copy(d)
        setattr(e, field, bad)
        assert pkg.lib().sbt3_plan(C.byref(e), C.byref(n)) == -1, field


def test_3d_body_and_solid_validation(pkg):
    """sbt3_plan rejects an immersed body whose stencils wrap across a face,
    a body in a walled or solid box, and wall fractions outside (0, 1]."""
    import ctypes as C
    import numpy as np

    def plan(wl):
        d = pkg.Desc3()
        d.nx, d.ny, d.nz, d.tau, d.rho0, d.storage, d.lattice = wl.nx, wl.ny, wl.nz, wl.tau, 1.0, pkg.F32, wl.lattice
        d.walls_z = 1 if wl.walls_z else 0
        keep = []
        if wl.body is not None:
            X, Y, Z, dA, it = wl.body
            xyz = np.ascontiguousarray(np.concatenate([X, Y, Z]))
            da = np.ascontiguousarray(dA)
            keep += [xyz, da]
            d.n_markers, d.mdf_iters = len(X), it
            d.ibm_box_cells = wl.nx * wl.ny * wl.nz
            d.marker_xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
            d.marker_dA = da.ctypes.data_as(C.POINTER(C.c_double))
        if wl.solid is not None:
            m, q = (np.ascontiguousarray(a) for a in wl.solid)
            keep += [m, q]
            d.solid_mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
            d.solid_q = q.ctypes.data_as(C.POINTER(C.c_double))
        n = C.c_size_t()
        return pkg.lib().sbt3_plan(C.byref(d), C.byref(n)), n.value

    ok = W.ibm_sphere3(24, r=4.0)
    rc, n = plan(ok)
    assert rc == 0 and n > 2 * 19 * 24 ** 3 * 4
    X, Y, Z, dA, it = ok.body
    assert plan(ok.replace(body=(X - 10.5, Y, Z, dA, it)))[0] == -1       # stencils wrap across x = 0
    assert plan(ok.replace(walls_z=True))[0] == -1
    assert plan(W.sphere3(16, r=3.0))[0] == 0
    m, q = W.sphere3(16, r=3.0).solid
    assert plan(W.sphere3(16, r=3.0).replace(solid=(m, np.zeros_like(q))))[0] == -1


def test_3d_moving_body_validation(pkg):
    """sbt3_plan rejects a moving body with an unknown motion, a zero period
    or chord, a box capacity below 64 cells or below the stencil box, and
    a pose at t = 0 whose stencils wrap; the binding sizes the box from the
    body's reach over its motion."""
    import ctypes as C
    import numpy as np

    wl = W.flapping_ellipsoid3(32)

    def plan(kind=1, params=None, cap=None, shift=0.0):
        X, Y, Z, dA, it = wl.body
        kind_, p = wl.motion
        p = list(p if params is None else params)
        p[0] += shift
        d = pkg.Desc3()
        d.nx, d.ny, d.nz, d.tau, d.rho0, d.storage, d.lattice = wl.nx, wl.ny, wl.nz, wl.tau, 1.0, pkg.F32, 19
        xyz = np.ascontiguousarray(np.concatenate([X, Y, Z]))
        da = np.ascontiguousarray(dA)
        d.n_markers, d.mdf_iters = len(X), it
        d.marker_xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
        d.marker_dA = da.ctypes.data_as(C.POINTER(C.c_double))
        d.ibm_box_cells = wl.nx * wl.ny * wl.nz if cap is None else cap
        d.body_motion = kind
        for i, v in enumerate(p):
            d.motion_p[i] = v
        n = C.c_size_t()
        return pkg.lib().sbt3_plan(C.byref(d), C.byref(n))

    assert plan() == 0
    assert plan(kind=2) == -1
    p = list(wl.motion[1])
    assert plan(params=p[:6] + [0.0] + p[7:]) == -1          # period T = 0
    assert plan(params=p[:9] + [0.0]) == -1                   # chord = 0
    assert plan(cap=32) == -1
    assert plan(cap=100) == -1                                # below the stencil box
    assert plan(shift=-12.0) == -1                            # stencils wrap across x = 0


def test_rescale_rejects_unit_tau(pkg):
    wl = W.tgv_patch(m=2, tau=1.0, cf_mode=W.CF_RESCALE)
    with pytest.raises(pkg.SbtError):
        pkg.plan([wl])


def test_valid_configs_plan(pkg):
    for wl in (W.cylinder(), W.cavity(), W.flapping_ellipse(), W.tgv_band(), W.tgv_patch(m=3),
               W.small_refined_flap(), W.uniform_refined()):
        assert pkg.plan([wl], pkg.F32) > 0
