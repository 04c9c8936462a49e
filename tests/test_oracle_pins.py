"""Pins for the FP64 oracle: each check is a property fixed by the paper or by
the mathematics (an identity, a closed form, an invariant), never a re-typing
of the oracle's own formula, and each is chosen so that a plausible slip in
the oracle (a dropped term, a flipped sign, a transposed index) fails it."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---- Sec. 2.1, Eq. (1): velocity set -------------------------------------

def test_velocity_set_isotropy(orc):
    cx, cy, w = orc.velocity_set()
    assert list(cx) == [0, 1, 0, -1, 0, 1, -1, -1, 1]
    assert list(cy) == [0, 0, 1, 0, -1, 1, 1, -1, -1]
    assert abs(w.sum() - 1.0) < 1e-15
    # lattice isotropy up to 4th order with c_s^2 = 1/3
    assert abs((w * cx * cx).sum() - 1 / 3) < 1e-15
    assert abs((w * cx * cy).sum()) < 1e-15
    assert abs((w * cx ** 4).sum() - 3 * (1 / 3) ** 2) < 1e-15
    assert abs((w * cx ** 2 * cy ** 2).sum() - (1 / 3) ** 2) < 1e-15


# ---- Eq. (7): equilibrium moments (P2) -----------------------------------

def test_equilibrium_moments(orc):
    cx, cy, _ = orc.velocity_set()
    rng = np.random.default_rng(1)
    for _ in range(50):
        rho = rng.uniform(0.5, 1.5)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        f = orc.feq(rho, ux, uy)
        assert abs(f.sum() - rho) < 1e-14
        assert abs((cx * f).sum() - rho * ux) < 1e-15
        assert abs((cy * f).sum() - rho * uy) < 1e-15
        assert abs((cx * cx * f).sum() - (rho / 3 + rho * ux * ux)) < 1e-14
        assert abs((cx * cy * f).sum() - rho * ux * uy) < 1e-14
        assert abs((cy * cy * f).sum() - (rho / 3 + rho * uy * uy)) < 1e-14


# ---- Eqs. (3)-(5): Guo forcing moments (P1) ------------------------------

def test_guo_moments(orc):
    cx, cy, _ = orc.velocity_set()
    rng = np.random.default_rng(2)
    for _ in range(50):
        tau = rng.uniform(0.51, 2.0)
        ux, uy, Fx, Fy = rng.uniform(-0.1, 0.1, 4)
        Fi = orc.guo(tau, ux, uy, Fx, Fy)
        pre = 1 - 1 / (2 * tau)
        assert abs(Fi.sum()) < 1e-15                                   # Eq. (4)
        assert abs((cx * Fi).sum() - pre * Fx) < 1e-15                 # Eq. (5)
        assert abs((cy * Fi).sum() - pre * Fy) < 1e-15
        # second moment of Guo's term: (1 - 1/2tau)(uF + Fu)
        assert abs((cx * cx * Fi).sum() - pre * 2 * ux * Fx) < 1e-15
        assert abs((cx * cy * Fi).sum() - pre * (ux * Fy + uy * Fx)) < 1e-15


def test_collision_conserves_mass_and_adds_force(orc):
    """Eqs. (6), (8): a collision keeps rho and raises sum c f by exactly F."""
    cx, cy, _ = orc.velocity_set()
    rng = np.random.default_rng(3)
    for _ in range(50):
        tau = rng.uniform(0.51, 2.0)
        f = orc.feq(1.0, 0.03, -0.02) + rng.uniform(-1e-3, 1e-3, 9)
        Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
        fs = orc.collide_cell(tau, f, Fx, Fy)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert abs((cx * fs).sum() - (cx * f).sum() - Fx) < 1e-16
        assert abs((cy * fs).sum() - (cy * f).sum() - Fy) < 1e-16
        # relaxation of the stress: sum c c (f* - f^eq) = (1 - 1/tau) sum c c (f - f^eq) + guo part
        rho = f.sum()
        u = ((cx * f).sum() + Fx / 2) / rho
        v = ((cy * f).sum() + Fy / 2) / rho
        fe = orc.feq(rho, u, v)
        lhs = (cx * cy * (fs - fe)).sum()
        rhs = (1 - 1 / tau) * (cx * cy * (f - fe)).sum() + (1 - 1 / (2 * tau)) * (u * Fy + v * Fx)
        assert abs(lhs - rhs) < 1e-16


# ---- Eq. (14): Peskin kernel (P3) ----------------------------------------

# ---- MRT collision (Sec. 2.1 option) ---------------------------------------

def test_mrt_basis_and_equilibrium_moments(orc):
    """The moment basis is orthogonal with row norms (9, 36, 36, 6, 12, 6, 12,
    4, 4), its inverse inverts it, and the moments of the Eq. (7)
    equilibrium are the textbook D2Q9 ones: rho, rho(-2 + 3u^2),
    rho(1 - 3u^2), rho ux, -rho ux, rho uy, -rho uy, rho(ux^2 - uy^2),
    rho ux uy."""
    M, Mi = orc.mrt_matrices()
    G = M @ M.T
    assert np.allclose(G, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]), atol=1e-14, rtol=0)
    assert np.abs(Mi @ M - np.eye(9)).max() < 1e-15
    rho, ux, uy = 1.03, 0.07, -0.04
    u2 = ux * ux + uy * uy
    want = [rho, rho * (-2 + 3 * u2), rho * (1 - 3 * u2), rho * ux, -rho * ux, rho * uy, -rho * uy,
            rho * (ux * ux - uy * uy), rho * ux * uy]
    assert np.abs(M @ orc.feq(rho, ux, uy) - want).max() < 1e-15


def test_mrt_forcing_moments(orc):
    """Moments of Guo's forcing term without its prefactor: (0, 6 u.F, -6 u.F,
    Fx, -Fx, Fy, -Fy, 2(ux Fx - uy Fy), ux Fy + uy Fx)."""
    M, _ = orc.mrt_matrices()
    ux, uy, Fx, Fy = 0.06, -0.03, 2e-4, -5e-5
    fbar = orc.guo(1e300, ux, uy, Fx, Fy)          # prefactor 1 - 1/(2 tau) -> 1
    uF = ux * Fx + uy * Fy
    want = [0, 6 * uF, -6 * uF, Fx, -Fx, Fy, -Fy, 2 * (ux * Fx - uy * Fy), ux * Fy + uy * Fx]
    assert np.abs(M @ fbar - want).max() < 1e-18


def test_mrt_with_equal_rates_is_bgk(orc):
    """All rates 1/tau: the MRT step is Eqs. (2)-(3) (BGK with Guo forcing)."""
    rng = np.random.default_rng(11)
    tau = 0.63
    f = orc.feq(1.02, 0.05, -0.02) * (1 + 0.01 * rng.normal(size=9))
    for F in ((0.0, 0.0), (3e-4, -1e-4)):
        a = orc.collide_cell_mrt(tau, [1 / tau] * 3, f, *F)
        b = orc.collide_cell(tau, f, *F)
        assert np.abs(a - b).max() < 1e-15


def test_mrt_relaxes_each_moment_at_its_rate(orc):
    """From equilibrium plus eps times one basis moment (no force), the
    collision leaves (1 - s_k) eps in that moment and nothing in the others;
    density and momentum are conserved, and a force adds exactly F to the
    momentum."""
    M, Mi = orc.mrt_matrices()
    tau, rates = 0.57, (1.64, 1.54, 1.9)
    S = [1.0, rates[0], rates[1], 1.0, rates[2], 1.0, rates[2], 1 / tau, 1 / tau]
    feq = orc.feq(0.98, 0.04, 0.03)
    for k in (1, 2, 4, 6, 7, 8):
        e = np.zeros(9)
        e[k] = 1e-3
        out = orc.collide_cell_mrt(tau, rates, feq + Mi @ e)
        d = M @ (out - feq)
        want = np.zeros(9)
        want[k] = (1 - S[k]) * 1e-3
        assert np.abs(d - want).max() < 1e-15, k
    rng = np.random.default_rng(5)
    f = feq * (1 + 0.02 * rng.normal(size=9))
    F = (2e-4, 1e-4)
    out = orc.collide_cell_mrt(tau, rates, f, *F)
    cx, cy, _ = orc.velocity_set()
    assert abs(out.sum() - f.sum()) < 1e-15
    assert abs((cx * out).sum() - (cx * f).sum() - F[0]) < 1e-16
    assert abs((cy * out).sum() - (cy * f).sum() - F[1]) < 1e-16


def test_mrt_tgv_decays_at_the_shear_viscosity(orc):
    """A Taylor-Green vortex under MRT decays at nu = (tau - 1/2) / 3: the
    shear rate is 1/tau; the other rates only damp non-hydrodynamic modes."""
    wl = W.tgv(64).replace(collision=W.COLL_MRT)
    err, _ = _tgv_error(orc, wl, 1000)
    assert err < 1e-2
    bgk = orc.OracleSim(W.tgv(64))
    mrt = orc.OracleSim(wl)
    bgk.step(20)
    mrt.step(20)
    assert np.abs(bgk.fields(0)[1] - mrt.fields(0)[1]).max() > 1e-12      # the MRT path ran


def test_peskin_kernel_moments(orc):
    rng = np.random.default_rng(4)
    assert orc.phi(2.0) == 0.0 and orc.phi(-2.5) == 0.0 and orc.phi(7.0) == 0.0
    assert abs(orc.phi(1.0) - 0.25) < 1e-16 and abs(orc.phi(1.0 - 1e-12) - 0.25) < 1e-11
    assert abs(orc.phi(0.0) - 0.5) < 1e-16
    for X in rng.uniform(-3, 3, 200):
        i = np.arange(math.floor(X) - 3, math.floor(X) + 4)
        r = i + 0.5 - X
        p = np.array([orc.phi(v) for v in r])
        assert (p > 0).sum() <= 4
        assert abs(p.sum() - 1.0) < 1e-14                  # partition of unity
        assert abs((r * p).sum()) < 1e-14                  # first moment
        assert abs((p * p).sum() - 3.0 / 8.0) < 1e-14      # sum phi^2
        assert abs(p[i % 2 == 0].sum() - 0.5) < 1e-14      # even/odd sums
        assert abs(p[i % 2 == 1].sum() - 0.5) < 1e-14


# ---- Eqs. (12), (15), (16): interpolation and spreading (P4) -------------

def test_interpolation_exact_for_linear_fields(orc):
    ny, nx = 32, 40
    yy, xx = np.mgrid[0:ny, 0:nx] + 0.5
    u = 0.3 + 0.01 * xx - 0.02 * yy
    v = -0.1 + 0.005 * xx + 0.007 * yy
    rng = np.random.default_rng(5)
    X, Y = rng.uniform(8, nx - 8, 30), rng.uniform(8, ny - 8, 30)
    U, V = orc.interpolate(u, v, X, Y)
    assert np.abs(U - (0.3 + 0.01 * X - 0.02 * Y)).max() < 1e-14
    assert np.abs(V - (-0.1 + 0.005 * X + 0.007 * Y)).max() < 1e-14


def test_spread_total_equals_marker_total(orc):
    rng = np.random.default_rng(6)
    X, Y = rng.uniform(5, 45, 40), rng.uniform(5, 35, 40)
    Fjx, Fjy, ds = rng.normal(size=40), rng.normal(size=40), rng.uniform(0.5, 1.5, 40)
    Fx, Fy = orc.spread((40, 50), X, Y, Fjx, Fjy, ds)
    assert abs(Fx.sum() - (Fjx * ds).sum()) < 1e-12
    assert abs(Fy.sum() - (Fjy * ds).sum()) < 1e-12
    # first moment of the spread force sits at the markers
    yy, xx = np.mgrid[0:40, 0:50] + 0.5
    assert abs((Fx * xx).sum() - (Fjx * ds * X).sum()) < 1e-10


# ---- MDF closed form for one marker (P5) ---------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_mdf_single_marker_closed_form(orc, k):
    ny, nx = 24, 24
    rho = np.ones((ny, nx))
    u0 = np.zeros((ny, nx))
    X, Y = np.array([11.37]), np.array([12.81])
    ux, uy, Fx, Fy, ftx, fty = orc.mdf(rho, u0, u0, X, Y, np.array([1.0]), np.array([0.0]),
                                       np.array([1.0]), k)
    U, V = orc.interpolate(ux, uy, X, Y)
    r = 55.0 / 64.0                        # 1 - ds (sum phi^2)^2 = 1 - 9/64
    assert abs((1.0 - U[0]) - r ** k) < 1e-14
    assert abs(V[0]) < 1e-15
    assert abs(ftx[0] - 2.0 * sum(r ** i for i in range(k))) < 1e-13
    assert abs(Fx.sum() - ftx[0]) < 1e-13   # Eq. (16) with ds = 1


def test_mdf_slip_decreases_on_a_circle(orc):
    """Reading 1: the iterated loop must reduce the boundary slip."""
    ny, nx = 48, 48
    rho = np.ones((ny, nx))
    u = np.full((ny, nx), 0.05)
    v = np.zeros((ny, nx))
    xb, yb, ds = W.circle_markers(8.0, 50)
    X, Y = 24.3 + xb, 23.9 + yb
    slips = []
    for k in (1, 2, 3, 4):
        ux, uy, *_ = orc.mdf(rho, u, v, X, Y, np.zeros(50), np.zeros(50), ds, k)
        U, V = orc.interpolate(ux, uy, X, Y)
        slips.append(np.sqrt((U ** 2 + V ** 2).mean()))
    assert all(slips[i + 1] < slips[i] for i in range(3))
    assert slips[-1] < 0.2 * 0.05


# ---- Kinematics (Sec. 3.6 law) -------------------------------------------

def test_flap_kinematics_is_rigid_and_periodic(orc):
    wl = W.flapping_ellipse()
    X0, Y0 = orc.body_positions(wl, 0)
    d0 = np.hypot(X0[:, None] - X0[None], Y0[:, None] - Y0[None])
    p = wl.body.params
    period_steps = p[6] * p[9] / p[8]
    for k in (17, 333, 1234.5, period_steps / 4):
        X, Y = orc.body_positions(wl, k)
        d = np.hypot(X[:, None] - X[None], Y[:, None] - Y[None])
        assert np.abs(d - d0).max() < 1e-10
    X, Y = orc.body_positions(wl, period_steps)
    assert np.abs(X - X0).max() < 1e-9 and np.abs(Y - Y0).max() < 1e-9
    # at t = 0: pitch angle alpha0 - A sin(phi) = 0, heave at +A0/2 along beta = 90 deg
    assert abs(Y0.mean() - (p[1] + p[4] / 2)) < 1e-9 and abs(X0.mean() - p[0]) < 1e-9
    # a quarter period later the pitch angle is -A (nose down by A)
    Xq, Yq = orc.body_positions(wl, period_steps / 4)
    j = int(np.argmin(wl.body.xb))                      # leading-edge marker (xb = -c/2)
    ang = math.atan2(Yq[j] - Yq.mean(), -(Xq[j] - Xq.mean()))
    assert abs(ang + p[3]) < 1e-9      # positive alpha is nose-up


def test_flap_with_zero_amplitudes_is_fixed(orc):
    wl = W.flapping_ellipse()
    b = wl.body
    params = list(b.params)
    params[3] = 0.0
    params[4] = 0.0
    moving = wl.replace(body=W.Body(W.BODY_FLAP, b.xb, b.yb, b.ds, params))
    fixed = wl.replace(body=W.Body(W.BODY_FIXED, b.xb, b.yb, b.ds, params))
    for k in (0, 10, 999):
        Xm, Ym = orc.body_positions(moving, k)
        Xf, Yf = orc.body_positions(fixed, k)
        assert np.abs(Xm - Xf).max() < 1e-12 and np.abs(Ym - Yf).max() < 1e-12


def _ramp(orc, **kw):
    p = W.ramp_params(100.0, 50.0, 32.0, 0.05, **kw)
    return p, (lambda t: orc.ramp_alpha(p, t))


@pytest.mark.parametrize("A,a_s,K,t1", [(math.pi / 2, 11.0, 0.2, 1.0), (0.7, 4.0, 0.05, 0.3)])
def test_ramp_law_closed_forms(orc, A, a_s, K, t1):
    """Sec. 3.5 ramp.  G is 0 long before t1 and 2 a_s (t2 - t1) long after t2
    (t2 = t1 + A / (2K)), so alpha runs from 0 to A; it is point-symmetric about
    the mid-ramp, alpha(t) + alpha(t1 + t2 - t) = A; G(t1) = log 2 up to
    exp(-2 a_s (t2 - t1)); and the mid-ramp rate is dalpha/dt* = 2K, the
    definition of the pitch rate K = alpha_dot c / (2 U)."""
    p, al = _ramp(orc, A=A, a_s=a_s, K=K, t1=t1)
    t2 = t1 + A / (2 * K)
    span = 2 * a_s * (t2 - t1)
    assert abs(al(t1 - 40.0 / a_s)) < 1e-12 * A
    assert abs(al(t2 + 40.0 / a_s) - A) < 1e-12 * A
    assert abs(al(t2 + 2000.0) - A) < 1e-12 * A          # no overflow far past the ramp
    for t in (t1 - 1.0, t1, 0.5 * (t1 + t2) + 0.3 * (t2 - t1), t2 + 0.1):
        assert abs(al(t) + al(t1 + t2 - t) - A) < 1e-12 * A
    tail = math.exp(-2 * a_s * (t2 - t1))
    assert abs(al(t1) - A * math.log(2.0) / span) < 1e-12 * A + 2 * A * tail
    assert abs(al(0.5 * (t1 + t2)) - 0.5 * A) < 1e-13 * A
    h, tm = 1e-4, 0.5 * (t1 + t2)
    rate = (al(tm + h) - al(tm - h)) / (2 * h)
    assert abs(rate - 2 * K) < 1e-7 * 2 * K + 4 * a_s * A * tail
    ts = np.linspace(t1 - 2, t2 + 2, 2001)
    a = np.array([al(t) for t in ts])
    assert np.all(np.diff(a) >= -1e-15)                   # monotone ramp, no overshoot
    assert a.max() <= A * (1 + 1e-14)


def test_ramp_angle_at_the_printed_lift_peak(orc):
    """Sec. 3.5 prints a pitch angle of about 5 deg at t* = 1.2, when lift
    peaks first (tests/golden/pitch_up_plate.json).  With the printed
    A, a_s, K, t1 the law gives 4.6 deg there, while reading t2 = t1 + A / K
    gives 1.2 deg.  (Normalising G by its value at t2 instead of its
    supremum changes alpha by only log 2 / (2 a_s (t2 - t1)) ~ 0.8 %.)"""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pitch_up_plate.json")))
    st, pk = gold["setup"], gold["first_lift_peak"]
    p = W.ramp_params(0.0, 0.0, 64.0, st["U0"], A=st["A_rad"], a_s=st["a_s"], K=st["K"], t1=st["t1_star"])
    a = math.degrees(orc.ramp_alpha(p, pk["t_star"]))
    assert abs(a - pk["alpha_deg"]) < 1.0, a


@pytest.mark.parametrize("xi", [0.5, 0.35, 0.6])
def test_triangular_law_closed_forms(orc, xi):
    """Sec. 3.6 smoothed triangular law: alpha(0) = 0; extremes +alpha0 at
    xi T / 2 and -alpha0 at T (1 - xi / 2) and nowhere beyond them; straight
    ramps of the printed rates 2 alpha0 / (xi T - ta) and -2 alpha0 /
    ((1 - xi) T - ta); alpha and its rate continuous at all six breakpoints
    (this is what fixes the quartic denominators to ta); period T; and for
    xi = 1/2 the second half-period mirrors the first."""
    a0, T, taf = math.radians(64.0), math.pi / 0.22, 0.15
    p = W.tri_params(0.0, 0.0, 64.0, 0.05, 64.0, 0.22, xi=xi, ta_frac=taf)
    al = lambda t: orc.tri_alpha(p, t)
    ta = taf * T
    r1, r2 = 2 * a0 / (xi * T - ta), -2 * a0 / ((1 - xi) * T - ta)
    te, tm = 0.5 * xi * T, T * (1 - 0.5 * xi)
    assert al(0.0) == 0.0
    assert abs(al(te) - a0) < 1e-14 and abs(al(tm) + a0) < 1e-14
    h = 1e-6 * T
    for t in (0.3 * (te - ta), te + ta + 0.5 * (tm - te - 2 * ta), tm + ta + 0.5 * (T - tm - ta)):
        r = (al(t + h) - al(t - h)) / (2 * h)
        want = r2 if te + ta < t < tm - ta else r1
        assert abs(r - want) < 1e-7 * abs(want)
    eps = 1e-9 * T
    for b in (te - ta, te, te + ta, tm - ta, tm, tm + ta):
        assert abs(al(b + eps) - al(b - eps)) < 1e-12 + 2 * eps * max(abs(r1), abs(r2))
        left = (al(b - eps) - al(b - eps - h)) / h
        right = (al(b + eps + h) - al(b + eps)) / h
        assert abs(left - right) < 1e-4 * max(abs(r1), abs(r2)), (b, left, right)
    ts = np.linspace(0.0, T, 4001)
    a = np.array([al(t) for t in ts])
    assert a.max() <= a0 * (1 + 1e-14) and a.min() >= -a0 * (1 + 1e-14)
    for t in (0.1 * T, 0.55 * T, 0.93 * T):
        assert abs(al(t + T) - al(t)) < 1e-12 and abs(al(t + 7 * T) - al(t)) < 1e-11
    if xi == 0.5:
        for t in ts[::97]:
            assert abs(al(t + 0.5 * T) + al(t)) < 1e-12


@pytest.mark.parametrize("make", [W.small_pitch_up, W.small_pitching_airfoil])
def test_pitching_bodies_rotate_rigidly_about_the_pivot(orc, make):
    """RAMP and TRI bodies: every marker keeps its distance to the pivot
    (x0, y0) and to every other marker, and the chord line turns by exactly
    the law's alpha (positive alpha: trailing edge down, nose up)."""
    wl = make()
    p = wl.body.params
    law = orc.ramp_alpha if wl.body.kind == W.BODY_RAMP else orc.tri_alpha
    xb, yb = np.asarray(wl.body.xb), np.asarray(wl.body.yb)
    r0 = np.hypot(xb, yb)
    j = int(np.argmax(xb))                                  # trailing-edge marker
    for k in (0.0, 7.0, 40.5, 123.0, 1000.0):
        X, Y = orc.body_positions(wl, k)
        assert np.abs(np.hypot(X - p[0], Y - p[1]) - r0).max() < 1e-10
        alpha = law(p, k * p[8] / p[9])
        th0 = math.atan2(yb[j], xb[j])
        th = math.atan2(Y[j] - p[1], X[j] - p[0])
        assert abs(math.remainder(th0 - th - alpha, 2 * math.pi)) < 1e-10


# ---- Solid cells with interpolated bounce-back (Sec. 2.1, Sec. 3.2) --------

def _ibb_profile_error(orc, ny, qb, qt, tau, steps):
    wl = W.ibb_channel(nx=4, ny=ny, tau=tau, q_bottom=qb, q_top=qt)
    s = orc.OracleSim(wl)
    s.step(steps)
    _, u, v = s.fields(0)
    g, nu = wl.meta["g"], wl.meta["nu"]
    y = np.arange(ny) + 0.5
    ua = g / (2 * nu) * (y - wl.meta["y_b"]) * (wl.meta["y_t"] - y)
    m = ~np.isnan(u[:, 0])
    assert m.sum() == ny - 2 and np.isnan(u[:2]).all()          # the solid rows read NaN
    assert np.abs(v[m]).max() < 1e-13
    return np.abs(u[m, 0] - ua[m]).max() / ua[m].max()


def test_ibb_half_way_walls_give_the_exact_channel(orc):
    """q = 1/2 is half-way bounce-back: at tau = 1/2 + sqrt(3)/4 the body-
    forced channel between solid rows is the exact parabola with walls half
    a cell beyond the last fluid rows (as P8 for domain walls)."""
    assert _ibb_profile_error(orc, 20, 0.5, 0.5, 0.5 + math.sqrt(3) / 4, 30000) < 1e-9


def test_ibb_off_grid_walls_converge_at_second_order(orc):
    """Walls at fractions 0.3 and 0.7 of the wall links: the steady profile
    approaches the parabola between the interpolated wall positions, the
    error falling about fourfold per doubling of the channel (second order
    in space)."""
    errs = [_ibb_profile_error(orc, ny, 0.3, 0.7, 0.8, int(3 * ny * ny / 0.1)) for ny in (12, 22, 42)]
    assert errs[2] < 1e-3
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_ibb_short_link_without_fluid_behind_is_half_way(orc):
    """A one-row fluid gap between solid rows: no fluid cell lies behind any
    short link, so q = 0.3 acts as q = 1/2 (the rule of the solid-cell
    interface), bit for bit."""
    runs = []
    for qb in (0.3, 0.5):
        s = orc.OracleSim(W.ibb_channel(nx=4, ny=3, tau=0.8, q_bottom=qb, q_top=qb))
        s.step(50)
        runs.append(s.populations(0))
    assert np.array_equal(runs[0], runs[1], equal_nan=True)


def test_ibb_cylinder_flow_is_mirror_symmetric(orc):
    """A solid circle on the centre line of a symmetric channel: u even and v
    odd about the centre line (a wrong link fraction or direction in the
    bounce-back breaks the mirror symmetry)."""
    wl = W.ibb_cylinder()
    s = orc.OracleSim(wl)
    s.step(300)
    _, u, v = s.fields(0)
    m = ~np.isnan(u)
    assert np.array_equal(m, m[::-1])
    su = np.abs(np.nan_to_num(u - u[::-1])).max()
    sv = np.abs(np.nan_to_num(v + v[::-1])).max()
    assert su < 1e-12 * np.nanmax(np.abs(u)) and sv < 1e-12 * np.nanmax(np.abs(u)), (su, sv)
    assert np.nanmax(np.abs(v)) > 1e-4                                # the body deflects the flow


# ---- Run statistics (Sec. 3.2 criterion E, Sec. 3.3 Eq. (21)) ------------

def test_force_stats_of_a_sampled_sinusoid(orc):
    """Lift A sin(2 pi t / P + phi) + b over whole periods of P samples: mean
    b and rms A / sqrt(2) exactly (sums of sampled sines over whole periods
    vanish); St = L / (P U) from the crossings; drag constant -> rms 0."""
    U, L, P, periods, A, b, cd = 0.05, 20.0, 100, 30, 0.7, 0.2, 1.4
    t = np.arange(P * periods)
    scale = 0.5 * U * U * L
    fy = (A * np.sin(2 * np.pi * t / P + 0.3) + b) * scale
    fx = np.full(len(t), cd * scale)
    r = orc.force_stats(fx, fy, U, L)
    assert abs(r["CL_mean"] - b) < 1e-13 and abs(r["CL_rms"] - A / math.sqrt(2)) < 1e-13
    assert abs(r["CD_mean"] - cd) < 1e-13 and r["CD_rms"] < 1e-13
    assert r["crossings"] in (periods - 1, periods) and r["samples"] == len(t)
    assert abs(r["St"] - L / (P * U)) < 1e-6 * L / (P * U)


def test_force_stats_against_numpy_on_noise(orc):
    """Means and rms deviations against numpy's mean and std; the crossing
    count and the first and last crossing against a brute-force scan."""
    rng = np.random.default_rng(7)
    n, U, L = 5001, 0.05, 12.0
    fx, fy = rng.normal(1.0, 0.3, n), np.cumsum(rng.normal(0.0, 1.0, n))
    r = orc.force_stats(fx, fy, U, L)
    s = 1.0 / (0.5 * U * U * L)
    cd, cl = fx * s, fy * s
    assert abs(r["CD_mean"] - cd.mean()) < 1e-12 * abs(cd.mean())
    assert abs(r["CD_rms"] - cd.std()) < 1e-11 * cd.std()
    assert abs(r["CL_rms"] - cl.std()) < 1e-11 * cl.std()
    c = cl - r["CL_mean"]
    up = np.nonzero((c[:-1] < 0) & (c[1:] >= 0))[0]
    assert r["crossings"] == len(up) and len(up) >= 3
    t0 = up[0] + c[up[0]] / (c[up[0]] - c[up[0] + 1])
    t1 = up[-1] + c[up[-1]] / (c[up[-1]] - c[up[-1] + 1])
    assert abs(r["St"] - (len(up) - 1) / (t1 - t0) * L / U) < 1e-12 * r["St"]


def test_velocity_change_measure(orc):
    """E = 0 between a state and itself; E = eps / (1 + eps) when every
    velocity grows by the factor 1 + eps; a level-1 cell weighs 1/4 of a
    level-0 cell; NaN (non-leaf) cells are left out."""
    rng = np.random.default_rng(3)
    u0 = [(rng.normal(size=(8, 8)), rng.normal(size=(8, 8))), (rng.normal(size=(16, 16)), rng.normal(size=(16, 16)))]
    for l in range(2):
        u0[l][0][:2, :2] = np.nan
        u0[l][1][:2, :2] = np.nan
    assert orc.velocity_change(u0, u0)[0] == 0.0
    eps = 0.125
    u1 = [(ux * (1 + eps), uy * (1 + eps)) for ux, uy in u0]
    assert abs(orc.velocity_change(u1, u0)[2] - eps / (1 + eps)) < 1e-14
    z = [(np.zeros((8, 8)), np.zeros((8, 8))), (np.zeros((16, 16)), np.zeros((16, 16)))]
    one = [(np.ones((8, 8)), np.zeros((8, 8))), (np.ones((16, 16)), np.zeros((16, 16)))]
    one[1][0][0, 0] = np.nan
    num, den, _ = orc.velocity_change(one, z)
    assert num == den == 64 + 255 / 4


def test_velocity_change_of_decaying_tgv(orc):
    """Taylor-Green decay: u(t + dt) = u(t) exp(-2 nu k^2 dt), so
    E = 1 - exp(-2 nu k^2 dt) up to the scheme's error (Sec. 3.1 flow, Sec. 3.2
    criterion with dt = 200 steps instead of 1000)."""
    wl = W.tgv(32, tau=0.8, u0=0.02)
    s = orc.OracleSim(wl)
    s.step(50)
    then = s.velocity()
    s.step(200)
    E = orc.velocity_change(s.velocity(), then)[2]
    k, nu = wl.meta["k"], wl.meta["nu"]
    want = math.exp(2 * nu * k * k * 200) - 1.0      # |u(t) - u(t+dt)| / |u(t+dt)|
    assert abs(E - want) < 0.01 * want, (E, want)


# ---- Whole-step invariants and closed forms ------------------------------

def test_periodic_conservation_with_body_force(orc):
    """P6: mass constant; total momentum grows by exactly N F per step."""
    g = (2e-6, -1e-6)
    wl = W.tgv(32).replace(fext=g)
    s = orc.OracleSim(wl)
    d0 = s.diagnostics()
    s.step(50)
    d1 = s.diagnostics()
    n = 32 * 32
    assert abs(d1[0] - d0[0]) < 1e-11 * n
    assert abs((d1[1] - d0[1]) - 50 * n * g[0]) < 1e-12
    assert abs((d1[2] - d0[2]) - 50 * n * g[1]) < 1e-12


def _tgv_error(orc, wl, steps):
    s = orc.OracleSim(wl)
    s.step(steps)
    fac = math.exp(-2 * wl.meta["nu"] * wl.meta["k"] ** 2 * steps)
    num = den = 0.0
    for l in range(wl.n_levels):
        nx, ny = s.level_size(l)
        _, u, _ = s.fields(l)
        _, ua, _ = wl.init(l, nx, ny)
        m = ~np.isnan(u)
        num += ((u[m] - fac * ua[m]) ** 2).sum() / 4 ** l
        den += ((fac * ua[m]) ** 2).sum() / 4 ** l
    return math.sqrt(num / den), fac


def test_tgv_closed_form_decay(orc):
    """P7: 64x64, tau 0.8, u0 0.02, 1000 steps: u(t) = u(0) exp(-2 nu k^2 t)."""
    err, fac = _tgv_error(orc, W.tgv(64), 1000)
    assert abs(fac - 0.14549) < 1e-5
    assert err < 1e-2


def test_tgv_second_order_convergence(orc):
    """Sec. 3.1: nu = 1/6, Re = 7.68, t* = 0.25; error falls as N^-2."""
    ns = [32, 64, 96, 128]
    errs = []
    for n in ns:
        wl = W.tgv_ladder(n)
        errs.append(_tgv_error(orc, wl, wl.meta["steps"])[0])
    order = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert 1.8 < order < 2.3, (errs, order)


def test_poiseuille_exact_profile(orc):
    """P8: BGK + Guo + half-way bounce-back: parabolic profile, walls exactly
    half-way at tau = 1/2 + sqrt(3)/4; constant 2nd difference -g/nu at any tau."""
    for tau, exact in ((0.5 + math.sqrt(3) / 4, True), (0.8, False), (1.3, False)):
        wl = W.poiseuille(nx=4, ny=16, tau=tau)
        s = orc.OracleSim(wl)
        s.step(30000 if tau < 1 else 12000)
        _, u, v = s.fields(0)
        g, nu = wl.meta["g"], wl.meta["nu"]
        prof = u[:, 0]
        d2 = prof[2:] - 2 * prof[1:-1] + prof[:-2]
        assert np.abs(d2 * nu / g + 1.0).max() < 1e-6
        assert np.abs(v).max() < 1e-13
        if exact:
            y = np.arange(16) + 0.5
            ua = g / (2 * nu) * y * (16 - y)
            assert np.abs(prof - ua).max() < 1e-9 * ua.max()


def test_couette_linear_profile(orc):
    """Moving-wall bounce-back: steady linear profile, walls half-way."""
    U = 0.01
    wl = W.Workload(name="couette", nx0=4, ny0=12, tau0=0.9, bc=(0, 0, W.WALL, W.WALL),
                    bc_u=((0, 0), (0, 0), (0, 0), (U, 0.0)), init=W.uniform_init(1.0, 0, 0))
    s = orc.OracleSim(wl)
    s.step(20000)
    _, u, _ = s.fields(0)
    y = np.arange(12) + 0.5
    assert np.abs(u[:, 0] - U * y / 12).max() < 1e-9 * U


def test_closed_box_conserves_mass(orc):
    wl = W.tgv(32).replace(bc=(W.WALL,) * 4)
    s = orc.OracleSim(wl)
    m0 = s.diagnostics()[0]
    s.step(300)
    assert abs(s.diagnostics()[0] - m0) < 1e-12 * m0


def test_uniform_stream_is_fixed_point_of_open_boundaries(orc):
    """Equilibrium inflow, zero-gradient outflow and symmetry edges keep a
    uniform equilibrium stream exactly uniform; free-slip on all four edges
    keeps a uniform x-stream uniform too."""
    for bc in ((W.INFLOW, W.OUTFLOW, W.SYMMETRY, W.SYMMETRY),
               (W.SYMMETRY, W.SYMMETRY, W.PERIODIC, W.PERIODIC)):
        U = 0.05 if bc[0] == W.INFLOW else 0.0
        V = 0.0 if bc[0] == W.INFLOW else 0.04
        wl = W.Workload(name="stream", nx0=32, ny0=16, tau0=0.7, bc=bc,
                        bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3, init=W.uniform_init(1.0, U, V))
        s = orc.OracleSim(wl)
        s.step(100)
        r, u, v = s.fields(0)
        assert np.abs(r - 1).max() < 1e-14 and np.abs(u - U).max() < 1e-15
        assert np.abs(v - V).max() < 1e-15


def test_uniform_flow_on_refined_forest(orc):
    """P9: f_neq = 0, so both interface operators are identities."""
    for cf in (W.CF_HOMOGENEOUS, W.CF_RESCALE):
        s = orc.OracleSim(W.uniform_refined(cf_mode=cf))
        s.step(15)
        for l in range(3):
            r, u, v = s.fields(l)
            m = ~np.isnan(r)
            assert m.sum() > 0
            assert np.abs(r[m] - 1).max() < 1e-13
            assert np.abs(u[m] - 0.05).max() < 1e-14 and np.abs(v[m] - 0.02).max() < 1e-14


def test_refined_band_conserves_mass(orc):
    """P11: straight coarse-fine interfaces without corners, HOMOGENEOUS
    operators: volume-weighted mass is conserved to roundoff."""
    s = orc.OracleSim(W.tgv_band())
    m0 = s.diagnostics()[0]
    s.step(200)
    assert abs(s.diagnostics()[0] - m0) < 1e-12 * m0


def test_refined_patch_tgv_stays_close(orc):
    """P12: a refined patch does not degrade TGV beyond an interface error
    that shrinks with resolution."""
    e_uni, _ = _tgv_error(orc, W.tgv(64), 500)
    e_p2, _ = _tgv_error(orc, W.tgv_patch(m=2), 500)
    e_p3, _ = _tgv_error(orc, W.tgv_patch(m=3), 500)
    assert e_p2 < 1e-2 and e_p3 < 1e-2
    wl128 = W.tgv(128, u0=0.01).replace(n_levels=2, boxes=[(1, 4, 4, 12, 12)])
    e128, _ = _tgv_error(orc, wl128, 2000)
    assert e128 < 0.5 * e_p2


def test_symmetric_body_symmetric_flow(orc):
    """P13: symmetric body in a symmetric channel: u_y odd about the centre line."""
    wl = W.cylinder(128, 64, D=12.0, centre=(40.0, 32.0), n_markers=38, Re=40.0, perturb=False)
    s = orc.OracleSim(wl)
    s.step(300)
    _, u, v = s.fields(0)
    assert np.abs(v + v[::-1]).max() < 1e-12 * 0.05
    assert np.abs(u - u[::-1]).max() < 1e-12 * 0.05
    fx, fy = s.force_history()
    assert len(fx) == 300 and np.abs(fy).max() < 1e-12


def test_cylinder_drag_in_sane_range(orc):
    """Sanity: steady drag of a cylinder at Re 40 in a channel is O(1)-O(few)."""
    wl = W.cylinder(160, 80, D=16.0, centre=(48.0, 40.0), n_markers=50, Re=40.0, perturb=False)
    s = orc.OracleSim(wl)
    s.step(3000)
    fx, _ = s.force_history()
    cd = fx[-1] / (0.5 * 0.05 ** 2 * 16.0)      # Eq. (16): force on the body
    assert 1.0 < cd < 4.0


def test_marker_outside_finest_level_is_rejected(orc):
    wl = W.small_cylinder()
    b = wl.body
    bad = wl.replace(body=W.Body(b.kind, b.xb, b.yb, b.ds, [2.0, 32.0] + [0.0] * 14))
    s = orc.OracleSim(bad)
    with pytest.raises(RuntimeError):
        s.step(1)


def test_invalid_topology_rejected(orc):
    # level-1 box touching a non-periodic edge
    wl = W.cavity().replace(boxes=[(1, 0, 0, 4, 4)], n_levels=2, body=None)
    with pytest.raises(RuntimeError):
        orc.OracleSim(wl)


def test_cylinder_shedding_matches_table1(orc):
    """Sec. 3.3, Table 1 (tests/golden/cylinder_table1.json): at Re 100 the
    shed wake of a fixed cylinder has St = 0.16 and C_L' = 0.24.  Here the
    cylinder is coarse (D = 10 cells, 31 markers) and the channel narrow
    (D/H = 0.1), both of which raise the drag of a diffuse-interface IBM, so
    C_D is held to [0.9, 1.25] x the paper's 1.33 while St and C_L' must sit
    near the printed values.  A wrong force sign, a dropped factor 2 in the
    boundary force, or a missing ds would move these by far more."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cylinder_table1.json")))["Re100"]
    D, nx, ny, steps, U = 10.0, 200, 100, 24000, 0.05
    wl = W.cylinder(nx, ny, D=D, centre=(nx / 4.0, ny / 2.0), n_markers=31, U=U, Re=100.0)
    s = orc.OracleSim(wl)
    s.step(steps)
    fx, fy = s.force_history()
    cd = fx / (0.5 * U * U * D)
    cl = fy / (0.5 * U * U * D)
    tail = slice(steps - 8000, steps)              # about six shedding periods
    c = cl[tail] - cl[tail].mean()
    up = np.nonzero((c[:-1] < 0) & (c[1:] >= 0))[0]
    assert len(up) >= 4, "no periodic shedding"
    st = D / (np.diff(up).mean() * U)
    p = gold["present"]
    assert abs(st - p["St"]) <= 0.1 * p["St"], st
    lo, hi = gold["literature_range"]["CL_rms"]
    assert lo <= c.std() <= hi, c.std()
    assert 0.9 * p["CD_mean"] <= cd[tail].mean() <= 1.25 * p["CD_mean"], cd[tail].mean()


def _flap_single_level():
    """A flapping ellipse on one uniform level (one finest substep per step)."""
    U, chord = 0.05, 24.0
    xb, yb, ds = W.ellipse_markers(chord / 2, chord / 16, 60)
    body = W.Body(W.BODY_FLAP, xb, yb, ds, W.flap_params(64.0, 64.0, chord, 30.0, 2.5 * np.pi, U))
    return W.Workload(name="flap1", nx0=128, ny0=128, tau0=0.56, bc=(W.INFLOW, W.OUTFLOW, W.SYMMETRY, W.SYMMETRY),
                      bc_u=((U, 0.0),) + ((0.0, 0.0),) * 3, body=body, init=W.uniform_init(1.0, U, 0.0))


def host_driven(wl, orc_sim, steps, positions):
    """Drive a HOST body with the positions of wl's prescribed body: before
    each step, markers at r(t_k) and desired velocity r(t_k+1) - r(t_k)."""
    for k in range(steps):
        X, Y = positions(k)
        X1, Y1 = positions(k + 1)
        orc_sim.set_markers(X, Y, X1 - X, Y1 - Y)
        orc_sim.step(1)


def test_host_markers_reproduce_prescribed_motion(orc):
    """Sec. 2.2 takes marker positions and desired velocities as given: a
    caller-placed body fed the positions of a prescribed flapping body, one
    substep at a time, reproduces that body's run bit for bit."""
    wl = _flap_single_level()
    ref = orc.OracleSim(wl)
    ref.step(40)
    b = wl.body
    host = wl.replace(body=W.Body(W.BODY_HOST, np.zeros(len(b.xb)), np.zeros(len(b.xb)), b.ds, [0.0] * 16))
    h = orc.OracleSim(host)
    pos = lambda k: orc.body_positions(wl, k)
    host_driven(wl, h, 40, pos)
    for l in range(wl.n_levels):
        for a, c in zip(ref.fields(l), h.fields(l)):
            assert np.array_equal(a, c, equal_nan=True)
    assert np.array_equal(ref.force_history()[0], h.force_history()[0])


def test_host_markers_replace_arc_lengths(orc):
    """The arc-length weights ds_j of Eqs. (15)-(16) given with the markers
    replace the body's: a HOST body created with twice the weights and fed
    the prescribed body's positions and weights every step reproduces the
    prescribed run bit for bit (and a run that keeps the doubled weights
    does not)."""
    wl = _flap_single_level()
    ref = orc.OracleSim(wl)
    ref.step(20)
    b = wl.body
    runs = []
    for give_ds in (True, False):
        host = wl.replace(body=W.Body(W.BODY_HOST, np.zeros(len(b.xb)), np.zeros(len(b.xb)), 2.0 * np.asarray(b.ds),
                                      [0.0] * 16))
        h = orc.OracleSim(host)
        for k in range(20):
            X, Y = orc.body_positions(wl, k)
            X1, Y1 = orc.body_positions(wl, k + 1)
            h.set_markers(X, Y, X1 - X, Y1 - Y, b.ds if give_ds else None)
            h.step(1)
        runs.append(h.force_history()[0])
    assert np.array_equal(ref.force_history()[0], runs[0])
    assert not np.allclose(ref.force_history()[0], runs[1], rtol=1e-3)


# ---- three dimensions: D3Q19 ---------------------------------------------------

@pytest.mark.parametrize("q", [19, 27])
def test_d3q19_isotropy_and_equilibrium_moments(orc, q):
    """D3Q19 and D3Q27: weights sum to 1; odd moments vanish; sum w c_a c_b = delta_ab / 3 and
    sum w c_a c_b c_c c_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9; the
    equilibrium carries rho, rho u and rho (u u + I/3)."""
    cx, cy, cz, w = orc.velocity_set3(q)
    c = np.stack([cx, cy, cz]).astype(float)
    assert len({(a, b, e) for a, b, e in zip(cx, cy, cz)}) == q
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(c @ w).max() < 1e-15
    d = np.eye(3)
    assert np.abs(np.einsum("i,ai,bi->ab", w, c, c) - d / 3).max() < 1e-15
    m4 = np.einsum("i,ai,bi,ci,di->abcd", w, c, c, c, c)
    want = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.abs(m4 - want).max() < 1e-15
    assert np.abs(np.einsum("i,ai,bi,ci->abc", w, c, c, c)).max() < 1e-15
    rho, u = 1.04, np.array([0.03, -0.02, 0.05])
    f = orc.feq3(rho, *u, q=q)
    assert abs(f.sum() - rho) < 1e-15 and np.abs(c @ f - rho * u).max() < 1e-15
    assert np.abs(np.einsum("i,ai,bi->ab", f, c, c) - rho * (np.outer(u, u) + d / 3)).max() < 1e-15


@pytest.mark.parametrize("axis,q", [("shear", 19), ("tgv", 19), ("shear", 27), ("tgv", 27)])
def test_d3q19_decay_converges_to_closed_form(orc, axis, q):
    """A shear wave u_x(z) and the Sec. 3.1 vortex extended along z are exact
    solutions decaying as exp(-nu k^2 t) and exp(-2 nu k^2 t); at fixed
    diffusive time the error falls about fourfold per doubling of n."""
    errs = []
    for n in (16, 32, 64):
        t = int(round(0.5 * (n / 16) ** 2 * 100))
        if axis == "shear":
            wl = W.shear_wave3(4, nz=n, tau=0.8).replace(lattice=q)
            fac = math.exp(-wl.meta["nu"] * wl.meta["k"] ** 2 * t)
        else:
            wl = W.tgv3(n, nz=2, tau=0.8).replace(lattice=q)
            fac = math.exp(-2 * wl.meta["nu"] * wl.meta["k"] ** 2 * t)
        s = orc.Oracle3Sim(wl)
        s.step(t)
        _, u, v, w = s.fields()
        _, ua, va, _ = wl.init(wl.nx, wl.ny, wl.nz)
        num = np.sqrt(((u - fac * ua) ** 2 + (v - fac * va) ** 2 + w ** 2).sum())
        errs.append(num / np.sqrt(((fac * ua) ** 2 + (fac * va) ** 2).sum()))
    assert errs[2] < 2e-3 and errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3, errs


@pytest.mark.parametrize("q", [19, 27])
def test_d3q19_conservation_and_translation(orc, q):
    """D3Q19 and D3Q27: mass is constant and momentum grows by N F per step under a uniform
    force; an initial state shifted by one cell along each axis gives the
    shifted result (periodic streaming indexes)."""
    F = (2e-6, -1e-6, 3e-6)
    wl = W.tgv3(16, nz=8, tau=0.7).replace(fext=F, lattice=q)
    s = orc.Oracle3Sim(wl)
    r0 = s.fields()[0].sum()
    s.step(20)
    r, u, v, w = s.fields()
    n = 16 * 16 * 8
    assert abs(r.sum() - r0) < 1e-11 * n
    for comp, Fk in zip((u, v, w), F):
        # momentum = sum(rho u) - N F / 2 (half-force velocity); initial momentum 0 in every direction
        assert abs((r * comp).sum() - n * Fk / 2 - 20 * n * Fk) < 1e-13 * n
    base = W.tgv3(16, nz=8, tau=0.7).replace(lattice=q)
    init0 = base.init

    def shifted(nx, ny, nz):
        return tuple(np.roll(a, (1, 1, 1), axis=(0, 1, 2)) for a in init0(nx, ny, nz))

    a, b = orc.Oracle3Sim(base), orc.Oracle3Sim(base.replace(init=shifted))
    a.step(7)
    b.step(7)
    for fa, fb in zip(a.fields(), b.fields()):
        assert np.array_equal(np.roll(fa, (1, 1, 1), axis=(0, 1, 2)), fb)


@pytest.mark.parametrize("q", [19, 27])
def test_3d_walls_give_exact_channel_flows(orc, q):
    """Half-way bounce-back walls across z: body-forced flow is the exact
    parabola at tau = 1/2 + sqrt(3)/4 with the walls half a cell beyond the
    last rows, and a moving top wall gives the exact linear profile (as the
    2D walls)."""
    nz = 16
    z = np.arange(nz) + 0.5
    wl = W.channel3(nz=nz, lattice=q)
    s = orc.Oracle3Sim(wl)
    s.step(30000)
    _, u, v, w = s.fields()
    g, nu = wl.meta["g"], wl.meta["nu"]
    ua = g / (2 * nu) * z * (nz - z)
    assert np.abs(u[:, 0, 0] - ua).max() < 1e-9 * ua.max()
    assert np.abs(u - u[:, :1, :1]).max() < 1e-18 and np.abs(w).max() < 1e-13
    wl = W.channel3(nz=nz, g=0.0, lid=0.01, tau=0.8, lattice=q)
    s = orc.Oracle3Sim(wl)
    s.step(8000)
    _, u, _, _ = s.fields()
    assert np.abs(u[:, 0, 0] - 0.01 * z / nz).max() < 1e-9


@pytest.mark.parametrize("q", [19, 27])
def test_3d_solid_cells_channel_and_sphere(orc, q):
    """3D solid cells with interpolated bounce-back: half-way links give the
    exact channel at the magic tau; walls at fractions 0.3 / 0.7 converge to
    the parabola at second order; a centred sphere in a box driven along x
    keeps the flow mirror-symmetric in y and z, and reads NaN inside."""
    def err(nz, qb, qt, tau):
        wl = W.solid_channel3(nz=nz, q_bottom=qb, q_top=qt, tau=tau, lattice=q)
        s = orc.Oracle3Sim(wl)
        s.step(int(3 * nz * nz / wl.meta["nu"]))
        _, u, _, w = s.fields()
        z = np.arange(nz) + 0.5
        ua = wl.meta["g"] / (2 * wl.meta["nu"]) * (z - wl.meta["z_b"]) * (wl.meta["z_t"] - z)
        m = ~np.isnan(u[:, 0, 0])
        assert m.sum() == nz - 2 and np.abs(w[m]).max() < 1e-13
        return np.abs(u[m, 0, 0] - ua[m]).max() / ua[m].max()

    assert err(20, 0.5, 0.5, 0.5 + math.sqrt(3) / 4) < 1e-9
    e = [err(nz, 0.3, 0.7, 0.8) for nz in (12, 22, 42)]
    assert e[2] < 1e-3 and e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e
    wl = W.sphere3(24, r=4.0, lattice=q)
    s = orc.Oracle3Sim(wl)
    s.step(150)
    _, u, v, w = s.fields()
    assert np.isnan(u[12, 12, 12]) and np.nanmax(np.abs(v)) > 1e-7
    # mirror about the centre plane y = 12 (cell y <-> 23 - y), and z likewise
    for a, b, sgn in ((u, u[:, ::-1, :], 1), (v, v[:, ::-1, :], -1), (u, u[::-1], 1), (w, w[::-1], -1)):
        assert np.nanmax(np.abs(a - sgn * b)) < 1e-12 * np.nanmax(np.abs(u))


def test_3d_ibm_sphere_momentum_balance_and_stokes_drag(orc):
    """Sec. 2.2 in 3D: a fixed IBM sphere (r = 4) in a periodic box forced
    along x.  At steady state the body force F_s balances the force on all
    the fluid, g n^3, exactly (momentum balance; the cross components
    vanish); the drag factor F / (6 pi mu r U) sits above Hasimoto's
    periodic-array value K(c) (1.83 here) by the diffuse interface's larger
    effective radius, within [1.0, 1.6] x K."""
    n, g, r = 24, 1e-5, 4.0
    wl = W.ibm_sphere3(n, r=r, tau=1.0, g=g)
    s = orc.Oracle3Sim(wl)
    s.step(4000)
    F = s.body_force()
    assert abs(F[0] / (g * n ** 3) - 1.0) < 5e-3, F
    assert abs(F[1]) < 1e-4 * F[0] and abs(F[2]) < 1e-4 * F[0]
    _, u, _, _ = s.fields()
    c = 4.0 / 3.0 * math.pi * r ** 3 / n ** 3
    K = 1.0 / (1 - 1.7601 * c ** (1 / 3) + c - 1.5593 * c ** 2 + 3.9799 * c ** (7 / 3) - 3.0734 * c ** (8 / 3))
    k = F[0] / (6 * math.pi * (0.5 / 3) * r * u.mean())
    assert 1.0 * K <= k <= 1.6 * K, (k, K)


def test_3d_moving_body_with_zero_amplitudes_is_fixed(orc):
    """The 3D pitch/plunge law with zero amplitudes is the fixed body at the
    pivot: same run, bit for bit (markers in the body frame shifted by the
    pivot against markers given absolute)."""
    wl = W.flapping_ellipsoid3(24, chord=8.0)
    xb, yb, zb, dA, it = wl.body
    p = list(wl.motion[1])
    p[4] = p[5] = 0.0
    moving = wl.replace(motion=(1, p))
    fixed = wl.replace(body=(p[0] + xb, p[1] + yb, p[2] + zb, dA, it), motion=(0, None))
    a, b = orc.Oracle3Sim(moving), orc.Oracle3Sim(fixed)
    a.step(20)
    b.step(20)
    assert np.array_equal(a.body_force(), b.body_force())
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
