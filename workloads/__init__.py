"""Seeded, synthetic workload descriptions shared by the GPU path and the oracle.

This module only *describes* inputs: domain sizes, refinement boxes, relaxation
time, edge kinds, initial fields, marker geometry and kinematic parameters.  It
holds none of the method's arithmetic (no collision, streaming, interpolation,
kinematics or interface operator), so both sides can consume it without sharing
any of the computation.

Shapes follow the benchmarks of arXiv 2402.04606, Sec. 3, scaled to the five
workloads this package is measured on:
  tgv(...)            Sec. 3.1 Taylor-Green vortex (periodic, closed form)
  cylinder(...)       Sec. 3.3 stationary cylinder, uniform 1024x512 grid
  cavity(...)         Sec. 3.2 lid-driven cavity with a central cylinder,
                      3 levels of 16x16-cell blocks
  flapping_ellipse()  Sec. 3.5/3.6 pitching and plunging wing, 4 levels
  pitch_up_plate()    Sec. 3.5 pitch-up ramp of a thin flat plate, 3 levels
  pitching_airfoil()  Sec. 3.6 smoothed triangular pitching of a 18 %-thick
                      symmetric section, 3 levels
  batch_sweep()       64 uneven flapping cases drawn from a fixed seed
Plus small cases used as pins (Poiseuille channel, uniform flow on a refined
forest, refined periodic band).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

# Edge kinds, order of edges W, E, S, N.
PERIODIC, WALL, INFLOW, OUTFLOW, SYMMETRY = 0, 1, 2, 3, 4
W, E, S, N = 0, 1, 2, 3
CF_HOMOGENEOUS, CF_RESCALE = 0, 1
COLL_BGK, COLL_MRT = 0, 1
# MRT rates of the non-hydrodynamic moments (e, eps, q), Lallemand and Luo's values
MRT_RATES = (1.64, 1.54, 1.9)
BODY_FIXED, BODY_FLAP, BODY_HOST, BODY_RAMP, BODY_TRI = 0, 1, 2, 3, 4


@dataclasses.dataclass
class Body:
    kind: int                      # BODY_FIXED, BODY_FLAP or BODY_HOST (xb, yb absolute)
    xb: np.ndarray                 # body-frame marker x (finest cells)
    yb: np.ndarray
    ds: np.ndarray                 # arc length per marker (finest cells)
    params: list                   # 16 kinematic parameters
    # FIXED: params[0:2] = (x0, y0)
    # FLAP : (x0, y0, alpha0, A_pitch, A0, beta, T, phi, U_ref, chord)
    # RAMP : (x0, y0, A, a_s, K, t1, -, -, U_ref, chord), pivot (x0, y0)
    # TRI  : (x0, y0, alpha0, xi, T, ta/T, -, -, U_ref, chord), pivot (x0, y0)


@dataclasses.dataclass
class Workload:
    name: str
    nx0: int
    ny0: int
    n_levels: int = 1
    block_n: int = 16
    boxes: list = dataclasses.field(default_factory=list)   # (level, bx0, by0, bx1, by1)
    tau0: float = 0.8
    rho0: float = 1.0
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    bc_u: tuple = ((0.0, 0.0),) * 4
    fext: tuple = (0.0, 0.0)
    cf_mode: int = CF_HOMOGENEOUS
    mdf_iters: int = 3
    collision: int = COLL_BGK
    mrt_rates: tuple = MRT_RATES
    body: Optional[Body] = None
    # solid cells with interpolated bounce-back: (level, mask [ny, nx] uint8,
    # q [ny, nx, 9] wall fraction of link i toward a solid neighbour, or None)
    solids: list = dataclasses.field(default_factory=list)
    init: Optional[Callable] = None   # init(level, nx, ny) -> (rho, ux, uy) dense [ny, nx]
    meta: dict = dataclasses.field(default_factory=dict)

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def _cell_centres(level, nx, ny):
    h = 1.0 / (2 ** level)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    return np.meshgrid(x, y)            # level-0 units, arrays [ny, nx]


def uniform_init(rho0, ux, uy, perturb=None):
    """Uniform flow; optional perturbation (x0, y0, size, duy) in level-0 cells."""
    def init(level, nx, ny):
        rho = np.full((ny, nx), rho0)
        u = np.full((ny, nx), float(ux))
        v = np.full((ny, nx), float(uy))
        if perturb is not None:
            x0, y0, size, duy = perturb
            X, Y = _cell_centres(level, nx, ny)
            m = (X >= x0) & (X < x0 + size) & (Y >= y0) & (Y < y0 + size)
            v[m] += duy
        return rho, u, v
    if perturb is None:
        init.uniform_state = (rho0, ux, uy)    # lets a consumer skip dense arrays
    return init


def tgv_init(nx0, u0, rho0):
    """Taylor-Green initial state (Sec. 3.1; pressure written with cos terms)."""
    k = 2.0 * math.pi / nx0

    def init(level, nx, ny):
        X, Y = _cell_centres(level, nx, ny)
        u = -u0 * np.cos(k * X) * np.sin(k * Y)
        v = u0 * np.sin(k * X) * np.cos(k * Y)
        p = -(rho0 * u0 * u0 / 4.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
        return rho0 + 3.0 * p, u, v
    return init


def tgv(n=64, tau=0.8, u0=0.02, rho0=1.0, n_levels=1, boxes=(), name=None):
    return Workload(name=name or f"tgv{n}", nx0=n, ny0=n, n_levels=n_levels, boxes=list(boxes),
                    tau0=tau, rho0=rho0, init=tgv_init(n, u0, rho0),
                    meta=dict(u0=u0, k=2 * math.pi / n, nu=(tau - 0.5) / 3.0))


def tgv_ladder(n):
    """Resolution ladder of Sec. 3.1: nu = 1/6, Re = U0 N / nu = 7.68, t* = 0.25."""
    nu = 1.0 / 6.0
    u0 = 7.68 * nu / n
    wl = tgv(n, tau=3 * nu + 0.5, u0=u0)
    wl.meta["steps"] = int(round(0.25 * n / u0))
    return wl


def poiseuille(nx=16, ny=16, tau=0.5 + math.sqrt(3) / 4, g=1e-6):
    return Workload(name="poiseuille", nx0=nx, ny0=ny, tau0=tau,
                    bc=(PERIODIC, PERIODIC, WALL, WALL), fext=(g, 0.0),
                    init=uniform_init(1.0, 0.0, 0.0), meta=dict(g=g, nu=(tau - 0.5) / 3.0))


def circle_markers(radius, n):
    th = 2.0 * math.pi * np.arange(n) / n
    ds = np.full(n, 2.0 * math.pi * radius / n)
    return radius * np.cos(th), radius * np.sin(th), ds


def ellipse_markers(a, b, n, samples=200000):
    """n markers at equal arc-length spacing on x = a cos s, y = b sin s."""
    s = np.linspace(0.0, 2.0 * math.pi, samples + 1)
    x, y = a * np.cos(s), b * np.sin(s)
    seg = np.hypot(np.diff(x), np.diff(y))
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    per = arc[-1]
    target = per * np.arange(n) / n
    sj = np.interp(target, arc, s)
    return a * np.cos(sj), b * np.sin(sj), np.full(n, per / n)


def cylinder(nx=1024, ny=512, D=40.0, centre=(256.0, 256.0), n_markers=126, U=0.05, Re=100.0,
             mdf_iters=3, perturb=True):
    nu = U * D / Re
    xb, yb, ds = circle_markers(D / 2.0, n_markers)
    body = Body(BODY_FIXED, xb, yb, ds, [centre[0], centre[1]] + [0.0] * 14)
    pert = (centre[0] + D / 2 + 2.0, centre[1], 4.0, 1e-3 * U) if perturb else None
    return Workload(name=f"cylinder{nx}x{ny}", nx0=nx, ny0=ny, tau0=3 * nu + 0.5,
                    bc=(INFLOW, OUTFLOW, SYMMETRY, SYMMETRY), bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3,
                    mdf_iters=mdf_iters, body=body, init=uniform_init(1.0, U, 0.0, pert),
                    meta=dict(U=U, D=D, Re=Re))


def cavity(cf_mode=CF_RESCALE, U=0.1, Re=1000.0):
    """256^2 base, 3 levels; L1 over base [96,160)^2, L2 over base [104,152)^2;
    cylinder D = 32 base cells (128 finest) at the centre."""
    n0 = 256
    nu0 = U * n0 / Re
    n_m = int(round(math.pi * 128))
    xb, yb, ds = circle_markers(64.0, n_m)
    body = Body(BODY_FIXED, xb, yb, ds, [512.0, 512.0] + [0.0] * 14)
    return Workload(name="cavity256_3lvl", nx0=n0, ny0=n0, n_levels=3,
                    boxes=[(1, 12, 12, 20, 20), (2, 26, 26, 38, 38)], tau0=3 * nu0 + 0.5,
                    bc=(WALL, WALL, WALL, WALL), bc_u=((0, 0), (0, 0), (0, 0), (U, 0.0)),
                    cf_mode=cf_mode, body=body, init=uniform_init(1.0, 0.0, 0.0),
                    meta=dict(U=U, Re=Re, D_finest=128))


def flap_params(x0, y0, chord, amp_deg, T, U, A0_over_c=2.5, beta_deg=90.0, alpha0=0.0, phi=0.0):
    return [x0, y0, alpha0, math.radians(amp_deg), A0_over_c * chord, math.radians(beta_deg), T,
            phi, U, chord] + [0.0] * 6


def flapping_ellipse(Re=100.0, U=0.05, n_markers=200, chord=64.0, amp_deg=64.0,
                     T=2.5 * math.pi):
    """Coarse 512x256, 4 levels, chord 64 finest cells, thickness 0.125."""
    m = 4
    nu_f = U * chord / Re
    tau0 = 0.5 + (3 * nu_f) / 2 ** (m - 1)
    xb, yb, ds = ellipse_markers(chord / 2, chord / 16, n_markers)
    body = Body(BODY_FLAP, xb, yb, ds, flap_params(1024.0, 1024.0, chord, amp_deg, T, U))
    boxes = [(1, 13, 11, 19, 21), (2, 29, 26, 35, 38), (3, 61, 56, 67, 72)]
    return Workload(name=f"flap_ellipse_re{int(Re)}", nx0=512, ny0=256, n_levels=m, boxes=boxes,
                    tau0=tau0, bc=(INFLOW, OUTFLOW, SYMMETRY, SYMMETRY),
                    bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3, body=body,
                    init=uniform_init(1.0, U, 0.0), meta=dict(U=U, Re=Re, chord=chord))


def _nested_boxes(bbox_f, m, B, nx0, ny0):
    """Block-aligned boxes for levels 1..m-1 around a finest-level bounding box
    (x0, y0, x1, y1), each level containing the finer one plus a 1-cell margin.
    Returns None if a refined level would come within one block of an edge."""
    boxes = []
    x0, y0, x1, y1 = bbox_f
    bx0, by0 = math.floor(x0 / B), math.floor(y0 / B)
    bx1, by1 = math.ceil(x1 / B), math.ceil(y1 / B)
    for l in range(m - 1, 0, -1):
        boxes.append((l, bx0, by0, bx1, by1))
        # extent on level l-1 in cells, plus one cell, rounded out to blocks
        cx0, cy0 = bx0 * B // 2 - 1, by0 * B // 2 - 1
        cx1, cy1 = bx1 * B // 2 + 1, by1 * B // 2 + 1
        bx0, by0 = math.floor(cx0 / B), math.floor(cy0 / B)
        bx1, by1 = math.ceil(cx1 / B), math.ceil(cy1 / B)
    # (bx0..bx1) is now the level-0 block box that must contain level 1
    if bx0 < 1 or by0 < 1 or bx1 > nx0 // B - 1 or by1 > ny0 // B - 1:
        return None
    return sorted(boxes)


def flapping_case(nx0, m, amp_deg, Re, n_markers, T, U=0.05, ds_target=0.65, name="flap"):
    B = 16
    per_over_c = 2.0453          # perimeter / chord of a 0.125-thick ellipse
    chord = 2.0 * round(n_markers * ds_target / per_over_c / 2.0)
    ny0 = nx0 // 2
    f = 2 ** (m - 1)
    xc, yc = nx0 / 4.0 * f, ny0 / 2.0 * f
    half_x = 0.5 * chord + 6.0
    half_y = 1.25 * chord + 0.5 * chord * math.sin(math.radians(amp_deg)) + chord / 16 + 6.0
    bbox = (xc - half_x, yc - half_y, xc + half_x, yc + half_y)
    boxes = _nested_boxes(bbox, m, B, nx0, ny0)
    if boxes is None:
        return None
    nu_f = U * chord / Re
    tau0 = 0.5 + 3 * nu_f / f
    xb, yb, ds = ellipse_markers(chord / 2, chord / 16, n_markers)
    body = Body(BODY_FLAP, xb, yb, ds, flap_params(xc, yc, chord, amp_deg, T, U))
    return Workload(name=name, nx0=nx0, ny0=ny0, n_levels=m, boxes=boxes, tau0=tau0,
                    bc=(INFLOW, OUTFLOW, SYMMETRY, SYMMETRY), bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3,
                    body=body, init=uniform_init(1.0, U, 0.0),
                    meta=dict(U=U, Re=Re, chord=chord, amp_deg=amp_deg, T=T))


def batch_sweep(n_cases=64, seed=4606):
    """64 flapping cases of uneven size; a draw whose refined region would not
    fit its domain is drawn again (same generator, so the list is fixed)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n_cases:
        nx0 = int(rng.integers(256 // 32, 1024 // 32 + 1)) * 32    # ny0 = nx0/2 stays a block multiple
        m = int(rng.integers(2, 5))
        amp = float(rng.uniform(10.0, 64.0))
        Re = float(math.exp(rng.uniform(math.log(100.0), math.log(1000.0))))
        nm = int(rng.integers(100, 301))
        T = float(rng.uniform(2 * math.pi, 3 * math.pi))
        wl = flapping_case(nx0, m, amp, Re, nm, T, name=f"sweep{len(out):02d}")
        if wl is not None:
            out.append(wl)
    return out


def uniform_refined(u=(0.05, 0.02), n0=64, boxes=((1, 2, 2, 6, 6), (2, 6, 6, 10, 10)), m=3,
                    cf_mode=CF_RESCALE, tau0=0.6):
    return Workload(name="uniform_refined", nx0=n0, ny0=n0, n_levels=m, boxes=list(boxes), tau0=tau0,
                    cf_mode=cf_mode, init=uniform_init(1.0, u[0], u[1]))


def tgv_band(n=64, u0=0.02, tau=0.8):
    """Refined band spanning the periodic x axis (no corners)."""
    wl = tgv(n, tau=tau, u0=u0, n_levels=2, boxes=[(1, 0, 3, 2 * n // 16, 5)], name="tgv_band")
    return wl


def tgv_patch(n=64, u0=0.02, tau=0.8, m=2, cf_mode=CF_HOMOGENEOUS):
    boxes = [(1, 2, 2, 6, 6)] if m == 2 else [(1, 2, 2, 6, 6), (2, 6, 6, 10, 10)]
    wl = tgv(n, tau=tau, u0=u0, n_levels=m, boxes=boxes, name=f"tgv_patch{m}")
    wl.cf_mode = cf_mode
    return wl


def small_cylinder(nx=128, ny=64, D=12.0, n_markers=38, U=0.05, Re=40.0):
    return cylinder(nx, ny, D=D, centre=(40.0, 32.0), n_markers=n_markers, U=U, Re=Re)


def small_refined_flap(Re=100.0, m=3):
    """A small moving-body case on a refined forest (parity-test size)."""
    wl = flapping_case(256, m, 40.0, Re, 60, 2.5 * math.pi, name=f"small_flap{m}")
    assert wl is not None
    return wl


# ---- pitch-up ramp (Sec. 3.5) and triangular pitching (Sec. 3.6) ------------

def ramp_params(x0, y0, chord, U, A=math.pi / 2, a_s=11.0, K=0.2, t1=1.0):
    """Sec. 3.5 ramp: amplitude A (rad), smoothing a_s, pitch rate K, start t1 (t* units)."""
    return [x0, y0, A, a_s, K, t1, 0.0, 0.0, U, chord] + [0.0] * 6


def tri_params(x0, y0, chord, U, alpha0_deg, k_red, xi=0.5, ta_frac=0.15):
    """Sec. 3.6 triangular law: amplitude alpha0, reduced frequency k = pi f c / U
    (period pi / k in t* = t U / c), asymmetry xi, blend time ta = ta_frac T."""
    return [x0, y0, math.radians(alpha0_deg), xi, math.pi / k_red, ta_frac, 0.0, 0.0, U, chord] + [0.0] * 6


def _resample_closed(x, y, n):
    """n points at equal arc length along the closed polyline (x, y)."""
    xs, ys = np.append(x, x[0]), np.append(y, y[0])
    seg = np.hypot(np.diff(xs), np.diff(ys))
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    target = arc[-1] * np.arange(n) / n
    return np.interp(target, arc, xs), np.interp(target, arc, ys), np.full(n, arc[-1] / n)


def plate_markers(chord, thickness, n):
    """Outline of the rectangle [0, chord] x [-t/2, t/2] (leading edge at the
    body-frame origin, the pivot of the ramp), n markers at equal spacing."""
    h = 0.5 * thickness
    x = np.array([0.0, chord, chord, 0.0])
    y = np.array([-h, -h, h, h])
    return _resample_closed(x, y, n)


def naca_symmetric_markers(chord, t, n, pivot=0.25, samples=20000):
    """Symmetric NACA four-digit section of thickness t (fraction of chord),
    half-thickness 5 t c (0.2969 sqrt(s) - 0.1260 s - 0.3516 s^2 + 0.2843 s^3
    - 0.1015 s^4), s = x / c, closed at the trailing edge; the body-frame
    origin (pivot) sits at x = pivot * chord on the chord line."""
    b = 0.5 * (1.0 - np.cos(np.linspace(0.0, math.pi, samples)))   # dense near both ends
    yt = 5.0 * t * chord * (0.2969 * np.sqrt(b) - 0.1260 * b - 0.3516 * b ** 2 + 0.2843 * b ** 3
                            - 0.1015 * b ** 4)
    yt[-1] = 0.0
    x = np.concatenate([b[::-1], b[1:-1]]) * chord - pivot * chord
    y = np.concatenate([-yt[::-1], yt[1:-1]])
    return _resample_closed(x, y, n)


def _pitching_case(name, body_of, sweep_box, chord, m, Re, U, nx_c, ny_c, x_c, ds_target=0.65,
                   perimeter=None):
    """Inflow / outflow / symmetry channel nx_c x ny_c chords (level-0 cells =
    chords * chord / 2^(m-1)); pivot at x_c chords from the inlet, mid-height;
    refined boxes nest around the region the body sweeps (sweep_box, relative
    to the pivot, finest cells)."""
    B = 16
    f = 2 ** (m - 1)
    c0 = chord / f
    nx0 = int(math.ceil(nx_c * c0 / B)) * B
    ny0 = int(math.ceil(ny_c * c0 / B)) * B
    xp, yp = x_c * chord, 0.5 * ny0 * f
    sx0, sy0, sx1, sy1 = sweep_box
    boxes = _nested_boxes((xp + sx0 - 6.0, yp + sy0 - 6.0, xp + sx1 + 6.0, yp + sy1 + 6.0), m, B, nx0, ny0)
    assert boxes is not None, "refined region does not fit the channel"
    n = int(round(perimeter / ds_target))
    body = body_of(xp, yp, n)
    nu_f = U * chord / Re
    return Workload(name=name, nx0=nx0, ny0=ny0, n_levels=m, boxes=boxes, tau0=0.5 + 3 * nu_f / f,
                    bc=(INFLOW, OUTFLOW, SYMMETRY, SYMMETRY), bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3,
                    body=body, init=uniform_init(1.0, U, 0.0),
                    meta=dict(U=U, Re=Re, chord=chord, D=chord))


def pitch_up_plate(chord=64.0, m=3, Re=1000.0, U=0.05, nx_c=70.0, ny_c=40.0, x_c=20.0,
                   thickness=0.023, A=math.pi / 2, a_s=11.0, K=0.2, t1=1.0, name=None):
    """Sec. 3.5: flat plate of 2.3 % thickness pitched up about its leading
    edge from 0 to A by the smoothed ramp, Re = U c / nu, in a 70c x 40c
    channel with 3 levels (streamwise length read as the longer side)."""
    t = thickness * chord

    def body_of(xp, yp, n):
        xb, yb, ds = plate_markers(chord, t, n)
        return Body(BODY_RAMP, xb, yb, ds, ramp_params(xp, yp, chord, U, A, a_s, K, t1))

    reach = chord + t
    return _pitching_case(name or f"pitch_up_plate_c{int(chord)}", body_of, (-reach, -reach, reach, t),
                          chord, m, Re, U, nx_c, ny_c, x_c, perimeter=2.0 * (chord + t))


def pitching_airfoil(chord=64.0, m=3, Re=1000.0, U=0.05, alpha0_deg=64.0, k_red=0.22, xi=0.5,
                     ta_frac=0.15, thickness=0.18, pivot=0.25, nx_c=70.0, ny_c=40.0, x_c=20.0,
                     name=None):
    """Sec. 3.6: a symmetric 18 %-thick section pitching about its quarter
    chord by the smoothed triangular law (alpha0, k, xi), same channel and
    levels as the pitch-up plate."""
    def body_of(xp, yp, n):
        xb, yb, ds = naca_symmetric_markers(chord, thickness, n, pivot)
        return Body(BODY_TRI, xb, yb, ds, tri_params(xp, yp, chord, U, alpha0_deg, k_red, xi, ta_frac))

    reach = (1.0 - pivot) * chord + 1.0
    return _pitching_case(name or f"pitching_airfoil_c{int(chord)}", body_of, (-reach, -reach, reach, reach),
                          chord, m, Re, U, nx_c, ny_c, x_c, perimeter=2.04 * chord)


def small_pitch_up(m=3, Re=100.0):
    """Parity-test size of the ramp case: chord 32 finest cells, 16c x 12c
    channel, ramp centred near the start (t1 = 0, K = 0.5) so that a short
    run turns the plate at a trailing-edge speed near U."""
    return pitch_up_plate(chord=32.0, m=m, Re=Re, nx_c=16.0, ny_c=12.0, x_c=5.0, t1=0.0, K=0.5,
                          name=f"small_pitch_up{m}")


def small_pitching_airfoil(m=3, Re=100.0):
    """Parity-test size of the triangular case: alpha0 = 4 deg at k = 20 (a
    period of about 100 finest substeps), so that a run of 30 coarse steps
    crosses every breakpoint of the law."""
    return pitching_airfoil(chord=32.0, m=m, Re=Re, alpha0_deg=4.0, k_red=20.0, nx_c=16.0, ny_c=12.0,
                            x_c=5.0, name=f"small_pitching_airfoil{m}")


# ---- solid cells for the interpolated bounce-back (Sec. 2.1, Sec. 3.2) -----

_CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
_CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)


def solid_circle(nx, ny, cx, cy, r):
    """Cells whose centres lie inside the circle (centre (cx, cy), radius r,
    level cells) are solid; for a fluid cell x and a direction i with
    x + c_i solid, q is the fraction of the link from the centre of x along
    c_i at which it meets the circle."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    px, py = xx + 0.5, yy + 0.5
    mask = ((px - cx) ** 2 + (py - cy) ** 2 < r * r).astype(np.uint8)
    q = np.full((ny, nx, 9), 0.5)
    for i in range(1, 9):
        dx, dy = _CX[i], _CY[i]
        a = dx * dx + dy * dy
        b = 2 * (dx * (px - cx) + dy * (py - cy))
        c = (px - cx) ** 2 + (py - cy) ** 2 - r * r
        disc = np.sqrt(np.maximum(b * b - 4 * a * c, 0.0))
        t = (-b - disc) / (2 * a)
        nb = np.roll(np.roll(mask, -dy, axis=0), -dx, axis=1)
        hit = (mask == 0) & (nb == 1)
        q[..., i] = np.where(hit, np.clip(t, 1e-6, 1.0), 0.5)
    return mask, q


def solid_channel(nx, ny, q_bottom=0.5, q_top=0.5):
    """Periodic channel whose rows 0 and 1 are solid: fluid rows 2 .. ny-1
    see a wall q_bottom below the centre of row 2 and q_top above the
    centre of row ny-1 (through the periodic wrap)."""
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[0:2] = 1
    q = np.full((ny, nx, 9), 0.5)
    for i in range(1, 9):
        if _CY[i] < 0:
            q[2, :, i] = q_bottom
        if _CY[i] > 0:
            q[ny - 1, :, i] = q_top
    return mask, q


def ibb_channel(nx=16, ny=32, tau=0.5 + math.sqrt(3) / 4, g=1e-6, q_bottom=0.5, q_top=0.5):
    """Body-forced flow between the walls of solid_channel (fully periodic
    domain); wall positions y_b = 2.5 - q_bottom, y_t = ny - 0.5 + q_top."""
    mask, q = solid_channel(nx, ny, q_bottom, q_top)
    return Workload(name=f"ibb_channel_q{q_bottom}_{q_top}", nx0=nx, ny0=ny, tau0=tau, fext=(g, 0.0),
                    solids=[(0, mask, q)], init=uniform_init(1.0, 0.0, 0.0),
                    meta=dict(g=g, nu=(tau - 0.5) / 3.0, y_b=2.5 - q_bottom, y_t=ny - 0.5 + q_top))


def ibb_cylinder(nx=128, ny=64, D=12.0, centre=(40.0, 32.0), U=0.05, Re=40.0):
    """Stationary cylinder as solid cells with interpolated bounce-back in the
    channel of small_cylinder (inflow, outflow, symmetry edges)."""
    nu = U * D / Re
    mask, q = solid_circle(nx, ny, centre[0], centre[1], D / 2.0)
    return Workload(name=f"ibb_cylinder{nx}x{ny}", nx0=nx, ny0=ny, tau0=3 * nu + 0.5,
                    bc=(INFLOW, OUTFLOW, SYMMETRY, SYMMETRY), bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3,
                    solids=[(0, mask, q)], init=uniform_init(1.0, U, 0.0), meta=dict(U=U, D=D, Re=Re))


def cavity_ibb(cf_mode=CF_RESCALE, U=0.1, Re=1000.0):
    """The 3-level cavity of cavity() with its cylinder (D = 128 finest cells at
    the centre) as solid cells with interpolated bounce-back instead of IBM
    markers -- the comparison of Sec. 3.2."""
    wl = cavity(cf_mode, U, Re)
    n2 = wl.nx0 * 4
    mask, q = solid_circle(n2, n2, 512.0, 512.0, 64.0)
    return wl.replace(name="cavity256_3lvl_ibb", body=None, solids=[(2, mask, q)])


# ---- three dimensions: D3Q19 on one periodic level ----------------------------

@dataclasses.dataclass
class Workload3:
    name: str
    nx: int
    ny: int
    nz: int
    tau: float = 0.8
    rho0: float = 1.0
    fext: tuple = (0.0, 0.0, 0.0)
    lattice: int = 19                 # D3Q19 or D3Q27
    walls_z: bool = False             # half-way bounce-back walls across z instead of periodic
    wall_u: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))   # bottom, top wall velocities
    # solid cells with interpolated bounce-back: (mask [nz, ny, nx] uint8,
    # q [nz, ny, nx, lattice] wall fraction of link i toward a solid neighbour, or None)
    solid: Optional[tuple] = None
    # immersed body: (X, Y, Z, dA, N_F), marker positions in cells
    body: Optional[tuple] = None
    # its motion: (0, None) fixed (markers absolute) or (1, 10 parameters) pitch
    # about y + plunge along z with markers in the body frame
    motion: tuple = (0, None)
    init: Optional[Callable] = None   # init(nx, ny, nz, z0=0, z1=nz) -> (rho, ux, uy, uz), each [z1 - z0, ny, nx]
    meta: dict = dataclasses.field(default_factory=dict)

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def shear_wave3(n=32, nz=None, tau=0.8, u0=0.01, period=None):
    """u_x = u0 sin(2 pi (z + 1/2) / period), a pure shear wave: an exact
    Navier-Stokes solution decaying as exp(-nu k^2 t)."""
    nz = nz or n
    period = period or nz
    k = 2 * math.pi / period

    def init(nx, ny, nz_, z0=0, z1=None):
        z1 = nz_ if z1 is None else z1
        z = np.arange(z0, z1) + 0.5
        m = z1 - z0
        ux = np.broadcast_to((u0 * np.sin(k * z))[:, None, None], (m, ny, nx)).copy()
        zero = np.zeros((m, ny, nx))
        return np.ones((m, ny, nx)), ux, zero, zero.copy()

    return Workload3(name=f"shear_wave3_{n}x{n}x{nz}", nx=n, ny=n, nz=nz, tau=tau, init=init,
                     meta=dict(u0=u0, k=k, nu=(tau - 0.5) / 3.0))


def tgv3(n=32, nz=8, tau=0.8, u0=0.02, period=None):
    """The Sec. 3.1 Taylor-Green vortex in the x-y plane, uniform along z
    (an exact 3D solution with the 2D decay exp(-2 nu k^2 t)); the pressure
    term of Sec. 3.1 sets rho."""
    period = period or n
    k = 2 * math.pi / period

    def init(nx, ny, nz_, z0=0, z1=None):
        z1 = nz_ if z1 is None else z1
        x = np.arange(nx) + 0.5
        y = np.arange(ny) + 0.5
        X, Y = np.meshgrid(x, y)
        u = -u0 * np.cos(k * X) * np.sin(k * Y)
        v = u0 * np.sin(k * X) * np.cos(k * Y)
        p = -(u0 * u0 / 4) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
        r = 1.0 + 3.0 * p
        m = z1 - z0
        rep = lambda a: np.broadcast_to(a[None], (m, ny, nx)).copy()
        return rep(r), rep(u), rep(v), np.zeros((m, ny, nx))

    return Workload3(name=f"tgv3_{n}x{n}x{nz}", nx=n, ny=n, nz=nz, tau=tau, init=init,
                     meta=dict(u0=u0, k=k, nu=(tau - 0.5) / 3.0))


def channel3(n=8, nz=16, tau=0.5 + math.sqrt(3) / 4, g=1e-6, lid=0.0, lattice=19):
    """Flow between walls across z (periodic in x and y): body force g along
    x (Poiseuille) and/or a top wall moving at lid along x (Couette)."""
    def init(nx, ny, nz_, z0=0, z1=None):
        z1 = nz_ if z1 is None else z1
        m = z1 - z0
        zero = np.zeros((m, ny, nx))
        return np.ones((m, ny, nx)), zero, zero.copy(), zero.copy()

    return Workload3(name=f"channel3_{n}x{n}x{nz}", nx=n, ny=n, nz=nz, tau=tau, fext=(g, 0.0, 0.0),
                     lattice=lattice, walls_z=True, wall_u=((0.0, 0.0, 0.0), (lid, 0.0, 0.0)), init=init,
                     meta=dict(g=g, lid=lid, nu=(tau - 0.5) / 3.0))


_C3X = (0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1)
_C3Y = (0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1)
_C3Z = (0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1)


def solid_sphere3(nx, ny, nz, centre, r, lattice=19):
    """Cells whose centres lie inside the sphere are solid; q is the fraction
    of the link from a fluid cell centre along c_i at which it meets the
    sphere (3D counterpart of solid_circle)."""
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx]
    px, py, pz = xx + 0.5 - centre[0], yy + 0.5 - centre[1], zz + 0.5 - centre[2]
    mask = (px * px + py * py + pz * pz < r * r).astype(np.uint8)
    q = np.full((nz, ny, nx, lattice), 0.5)
    for i in range(1, lattice):
        dx, dy, dz = _C3X[i], _C3Y[i], _C3Z[i]
        a = dx * dx + dy * dy + dz * dz
        b = 2 * (dx * px + dy * py + dz * pz)
        c = px * px + py * py + pz * pz - r * r
        t = (-b - np.sqrt(np.maximum(b * b - 4 * a * c, 0.0))) / (2 * a)
        nb = np.roll(mask, (-dz, -dy, -dx), axis=(0, 1, 2))
        hit = (mask == 0) & (nb == 1)
        q[..., i] = np.where(hit, np.clip(t, 1e-6, 1.0), 0.5)
    return mask, q


def solid_channel3(n=4, nz=20, tau=0.5 + math.sqrt(3) / 4, g=1e-6, q_bottom=0.5, q_top=0.5, lattice=19):
    """Periodic box whose planes z = 0 and 1 are solid: body-forced flow
    between walls at q_bottom below the centre of plane 2 and q_top above the
    centre of plane nz - 1 (3D counterpart of ibb_channel)."""
    mask = np.zeros((nz, n, n), dtype=np.uint8)
    mask[0:2] = 1
    q = np.full((nz, n, n, lattice), 0.5)
    for i in range(1, lattice):
        if _C3Z[i] < 0:
            q[2, :, :, i] = q_bottom
        if _C3Z[i] > 0:
            q[nz - 1, :, :, i] = q_top

    def init(nx, ny, nz_, z0=0, z1=None):
        z1 = nz_ if z1 is None else z1
        m = z1 - z0
        zero = np.zeros((m, ny, nx))
        return np.ones((m, ny, nx)), zero, zero.copy(), zero.copy()

    return Workload3(name=f"solid_channel3_q{q_bottom}_{q_top}", nx=n, ny=n, nz=nz, tau=tau, fext=(g, 0.0, 0.0),
                     lattice=lattice, solid=(mask, q), init=init,
                     meta=dict(g=g, nu=(tau - 0.5) / 3.0, z_b=2.5 - q_bottom, z_t=nz - 0.5 + q_top))


def sphere3(n=32, r=5.0, tau=0.8, g=2e-6, lattice=19):
    """A solid sphere at the centre of a periodic box driven by a body force
    along x (a periodic array of spheres)."""
    mask, q = solid_sphere3(n, n, n, (n / 2, n / 2, n / 2), r, lattice)

    def init(nx, ny, nz_, z0=0, z1=None):
        z1 = nz_ if z1 is None else z1
        m = z1 - z0
        zero = np.zeros((m, ny, nx))
        return np.ones((m, ny, nx)), zero, zero.copy(), zero.copy()

    return Workload3(name=f"sphere3_{n}_r{r}", nx=n, ny=n, nz=n, tau=tau, fext=(g, 0.0, 0.0), lattice=lattice,
                     solid=(mask, q), init=init, meta=dict(g=g, r=r))


def sphere_markers(centre, r, n):
    """n markers spread evenly over a sphere (golden-angle spiral), each
    carrying the surface element 4 pi r^2 / n."""
    k = np.arange(n) + 0.5
    zc = 1.0 - 2.0 * k / n
    rho = np.sqrt(1.0 - zc * zc)
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    X = centre[0] + r * rho * np.cos(phi)
    Y = centre[1] + r * rho * np.sin(phi)
    Z = centre[2] + r * zc
    return X, Y, Z, np.full(n, 4.0 * math.pi * r * r / n)


def ibm_sphere3(n=24, r=4.0, tau=0.8, g=1e-5, n_markers=None, mdf_iters=3, lattice=19):
    """A fixed IBM sphere (markers about 0.7 cells apart) at the centre of a
    periodic box driven by a body force along x: a periodic array of
    spheres (Sec. 2.2 in 3D)."""
    nm = n_markers or int(round(4 * math.pi * r * r / 0.5))
    X, Y, Z, dA = sphere_markers((n / 2, n / 2, n / 2), r, nm)

    def init(nx, ny, nz_, z0=0, z1=None):
        z1 = nz_ if z1 is None else z1
        m = z1 - z0
        zero = np.zeros((m, ny, nx))
        return np.ones((m, ny, nx)), zero, zero.copy(), zero.copy()

    return Workload3(name=f"ibm_sphere3_{n}_r{r}", nx=n, ny=n, nz=n, tau=tau, fext=(g, 0.0, 0.0), lattice=lattice,
                     body=(X, Y, Z, dA, mdf_iters), init=init, meta=dict(g=g, r=r, n_markers=nm))


def flapping_ellipsoid3(n=32, chord=12.0, amp_deg=30.0, T=1.0, U=0.05, tau=0.8, A0_over_c=0.5, n_markers=None,
                        mdf_iters=3, lattice=19):
    """A thin ellipsoid (semi-axes c/2, c/4 along y, c/8 along z) pitching
    about the y axis and plunging along z (the Sec. 3.6 law in the x-z
    plane) in a periodic box with a uniform stream U along x."""
    a, b, cz = chord / 2, chord / 4, chord / 8
    nm = n_markers or 400
    k = np.arange(nm) + 0.5
    zc = 1.0 - 2.0 * k / nm
    rr = np.sqrt(1.0 - zc * zc)
    ph = k * math.pi * (3.0 - math.sqrt(5.0))
    xb, yb, zb = a * rr * np.cos(ph), b * rr * np.sin(ph), cz * zc
    # surface element: the ellipsoid's area (Knud Thomsen's approximation) shared evenly
    pp = 1.6075
    area = 4 * math.pi * (((a * b) ** pp + (a * cz) ** pp + (b * cz) ** pp) / 3) ** (1 / pp)
    dA = np.full(nm, area / nm)
    params = [n / 2, n / 2, n / 2, 0.0, math.radians(amp_deg), A0_over_c * chord, T, 0.0, U, chord]

    def init(nx, ny, nz_, z0=0, z1=None):
        z1 = nz_ if z1 is None else z1
        m = z1 - z0
        zero = np.zeros((m, ny, nx))
        return np.ones((m, ny, nx)), np.full((m, ny, nx), U), zero, zero.copy()

    return Workload3(name=f"flapping_ellipsoid3_{n}", nx=n, ny=n, nz=n, tau=tau, lattice=lattice,
                     body=(xb, yb, zb, dA, mdf_iters), motion=(1, params), init=init,
                     meta=dict(U=U, chord=chord, n_markers=nm))


# ---- three dimensions on a block forest ------------------------------------------

@dataclasses.dataclass
class Workload3F:
    """A periodic 3D case on a block forest (Sec. 2.3-2.4 in three dimensions).

    Level l has (nx0, ny0, nz0) * 2**l cells; a box (level, bx0, by0, bz0,
    bx1, by1, bz1) covers the half-open range of level-l blocks of block_n^3
    cells.  tau_l = 1/2 + 2**l (tau0 - 1/2) and F_l = F_0 / 2**l (Eq. (9))."""
    name: str
    nx0: int
    ny0: int
    nz0: int
    n_levels: int = 1
    boxes: tuple = ()
    block_n: int = 8
    tau0: float = 0.8
    rho0: float = 1.0
    fext: tuple = (0.0, 0.0, 0.0)
    lattice: int = 19
    cf_mode: int = CF_HOMOGENEOUS
    # init(level, x0, y0, z0, nx, ny, nz) -> (rho, ux, uy, uz) on the level's
    # cells [x0, x0 + nx) x [y0, ...) x [z0, ...), each [nz, ny, nx] or a scalar
    init: Optional[Callable] = None
    meta: dict = dataclasses.field(default_factory=dict)

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def _centres3(level, nx, ny, nz, x0=0, y0=0, z0=0):
    """Centres of level-l cells [x0, x0 + nx) x ... in level-0 units, each [nz, ny, nx]."""
    h = 1.0 / (1 << level)
    z, y, x = np.meshgrid((z0 + np.arange(nz) + 0.5) * h, (y0 + np.arange(ny) + 0.5) * h,
                          (x0 + np.arange(nx) + 0.5) * h, indexing="ij")
    return x, y, z


def uniform3f(u=(0.04, 0.02, -0.01), n0=32, m=2, boxes=((1, 1, 1, 1, 3, 3, 3),), tau0=0.8, lattice=19,
              cf_mode=CF_HOMOGENEOUS, rho0=1.0, name="uniform3f"):
    """A uniform stream on a refined forest: every scheme that is consistent
    across the interface keeps it uniform exactly (up to rounding)."""
    def init(level, x0, y0, z0, nx, ny, nz):
        return rho0, u[0], u[1], u[2]
    return Workload3F(name, n0, n0, n0, m, tuple(boxes), 8, tau0, rho0, (0.0, 0.0, 0.0), lattice, cf_mode, init)


def tgv3f(n0=32, m=2, boxes=((1, 2, 2, 0, 6, 6, 1),), tau0=0.8, u0=0.02, lattice=19, cf_mode=CF_HOMOGENEOUS,
          rho0=1.0, plane="xy", n_third=None, name="tgv3f"):
    """The Taylor-Green vortex of Sec. 3.1 in one coordinate plane ("xy",
    "xz" or "yz"), uniform along the third axis (n_third level-0 cells,
    default n0 / 4), on a 3D forest: the exact solution decays as
    exp(-2 nu k^2 t) on every level."""
    n_third = n_third or n0 // 4
    k = 2.0 * math.pi / n0
    a_ax, b_ax = {"xy": (0, 1), "xz": (0, 2), "yz": (1, 2)}[plane]
    size = [n_third] * 3
    size[a_ax] = size[b_ax] = n0

    def init(level, x0, y0, z0, nx, ny, nz):
        c = _centres3(level, nx, ny, nz, x0, y0, z0)
        a, b = c[a_ax], c[b_ax]
        u = [np.zeros_like(a) for _ in range(3)]
        u[a_ax] = -u0 * np.cos(k * a) * np.sin(k * b)
        u[b_ax] = u0 * np.sin(k * a) * np.cos(k * b)
        p = -0.25 * rho0 * u0 * u0 * (np.cos(2 * k * a) + np.cos(2 * k * b))
        return rho0 + 3.0 * p, u[0], u[1], u[2]
    return Workload3F(name, size[0], size[1], size[2], m, tuple(boxes), 8, tau0, rho0, (0.0, 0.0, 0.0), lattice,
                      cf_mode, init, {"u0": u0, "k": k, "nu": (tau0 - 0.5) / 3.0, "axes": (a_ax, b_ax)})


def vortex3f(n0=32, m=2, boxes=((1, 2, 2, 2, 6, 6, 6),), tau0=0.8, u0=0.02, lattice=19, cf_mode=CF_HOMOGENEOUS,
             rho0=1.0, seed=4606, name="vortex3f"):
    """A genuinely 3D periodic flow: a sum of a few divergence-free Fourier
    modes with seeded amplitudes and phases, velocities of order u0."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(4):
        kv = rng.integers(-2, 3, size=3)
        while not kv.any():
            kv = rng.integers(-2, 3, size=3)
        a = rng.normal(size=3)
        a -= kv * (a @ kv) / (kv @ kv)              # amplitude normal to the wave vector
        modes.append((kv.astype(float), a * u0 / np.linalg.norm(a) / 2.0, rng.uniform(0, 2 * math.pi)))
    k = 2.0 * math.pi / n0

    def init(level, x0, y0, z0, nx, ny, nz):
        x, y, z = _centres3(level, nx, ny, nz, x0, y0, z0)
        u = [np.zeros_like(x) for _ in range(3)]
        for kv, a, ph in modes:
            s = np.sin(k * (kv[0] * x + kv[1] * y + kv[2] * z) + ph)
            for d in range(3):
                u[d] += a[d] * s
        return np.full_like(x, rho0), u[0], u[1], u[2]
    return Workload3F(name, n0, n0, n0, m, tuple(boxes), 8, tau0, rho0, (0.0, 0.0, 0.0), lattice, cf_mode, init,
                      {"u0": u0})


def forest3d_bench(n0=256, lattice=19, cf_mode=CF_HOMOGENEOUS, tau0=0.6, u0=0.02):
    """The 3D forest the benchmark times: a 256^3 periodic level 0 with a
    nested level 1 over the central half of each axis and a level 2 over the
    central quarter (a body-centred refinement of the shape Sec. 2.3
    describes), carrying the seeded 3D vortex of period n0 / 4."""
    b1 = n0 // 8 * 2                      # level-1 blocks per axis
    b2 = n0 // 8 * 4
    boxes = ((1, b1 // 4, b1 // 4, b1 // 4, 3 * b1 // 4, 3 * b1 // 4, 3 * b1 // 4),
             (2, 3 * b2 // 8, 3 * b2 // 8, 3 * b2 // 8, 5 * b2 // 8, 5 * b2 // 8, 5 * b2 // 8))
    wl = vortex3f(n0=n0 // 4, m=3, boxes=boxes, tau0=tau0, u0=u0, lattice=lattice, cf_mode=cf_mode,
                  name="forest3d_bench")
    return wl.replace(nx0=n0, ny0=n0, nz0=n0)
