"""FP64 CPU oracle for the SBoTFlow LBM-IBM time step (arXiv 2402.04606).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2402_04606_amd``); both sides consume the
same seeded inputs from ``workloads``.

This module is argument marshalling around ``liborc.so`` (built from
``oracle.c`` by ``oracle/build.py``); all arithmetic lives in the C file.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc.so")

ORC_BODY_NONE, ORC_BODY_FIXED, ORC_BODY_FLAP, ORC_BODY_HOST = -1, 0, 1, 2


class _Case(C.Structure):
    _fields_ = [
        ("nx0", C.c_int32), ("ny0", C.c_int32), ("block_n", C.c_int32), ("n_levels", C.c_int32),
        ("n_boxes", C.c_int32), ("boxes", C.POINTER(C.c_int32)),
        ("tau0", C.c_double), ("rho0", C.c_double),
        ("bc", C.c_int32 * 4), ("bc_u", C.c_double * 8), ("fext", C.c_double * 2),
        ("cf_mode", C.c_int32), ("mdf_iters", C.c_int32), ("body_kind", C.c_int32),
        ("n_markers", C.c_int32),
        ("xb", C.POINTER(C.c_double)), ("yb", C.POINTER(C.c_double)), ("ds", C.POINTER(C.c_double)),
        ("bp", C.c_double * 16),
        ("collision", C.c_int32), ("mrt", C.c_double * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _configure(C.CDLL(LIB_PATH))
    return _lib


def load_variant(path):
    """A separately built copy of oracle.c (for tests that plant a mistake in
    the oracle and check that a pin catches it), with the same signatures."""
    return _configure(C.CDLL(path))


def _configure(L):
    """Argument and result types of every entry point of a build of oracle.c."""
    d = C.POINTER(C.c_double)
    L.orc_create.argtypes = [C.POINTER(_Case), C.POINTER(C.c_void_p)]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_destroy.restype = None
    L.orc_level_size.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.orc_level_kinds.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint8)]
    L.orc_init_fields.argtypes = [C.c_void_p, C.c_int, d, d, d]
    L.orc_step.argtypes = [C.c_void_p, C.c_int32]
    L.orc_init_populations.argtypes = [C.c_void_p, C.c_int, d]
    L.orc_interface_factors.argtypes = [C.c_double, C.c_double, d]
    L.orc_interface_factors.restype = None
    L.orc_read_fields.argtypes = [C.c_void_p, C.c_int, d, d, d]
    L.orc_read_populations.argtypes = [C.c_void_p, C.c_int, d]
    L.orc_marker_forces.argtypes = [C.c_void_p, d, d]
    L.orc_set_markers.argtypes = [C.c_void_p, C.c_int32, d, d, d, d, d]
    L.orc_force_history.argtypes = [C.c_void_p, C.c_int32, d, d, C.POINTER(C.c_int32)]
    L.orc_diagnostics.argtypes = [C.c_void_p, d]
    L.orc_substeps.argtypes = [C.c_void_p]
    L.orc_substeps.restype = C.c_int64
    L.orc_velocity_set.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), d]
    L.orc_velocity_set.restype = None
    L.orc_feq.argtypes = [C.c_double] * 3 + [d]
    L.orc_feq.restype = None
    L.orc_guo.argtypes = [C.c_double] * 5 + [d]
    L.orc_guo.restype = None
    L.orc_collide_cell.argtypes = [C.c_double, d, C.c_double, C.c_double, d]
    L.orc_collide_cell.restype = None
    L.orc_mrt_matrices.argtypes = [d, d]
    L.orc_mrt_matrices.restype = None
    L.orc_collide_cell_mrt.argtypes = [C.c_double, d, d, C.c_double, C.c_double, d]
    L.orc_collide_cell_mrt.restype = None
    L.orc_phi.argtypes = [C.c_double]
    L.orc_phi.restype = C.c_double
    L.orc_body_positions.argtypes = [C.POINTER(_Case), C.c_double, d, d]
    for f in (L.orc_ramp_alpha, L.orc_tri_alpha):
        f.argtypes = [d, C.c_double]
        f.restype = C.c_double
    L.orc_mdf.argtypes = [C.c_int32, C.c_int32, d, d, d, d, d, C.c_int32, d, d, d, d, d,
                             C.c_int32, d, d]
    L.orc_interpolate.argtypes = [C.c_int32, C.c_int32, d, d, C.c_int32, d, d, d, d]
    L.orc_spread.argtypes = [C.c_int32, C.c_int32, C.c_int32, d, d, d, d, d, d, d]
    L.orc_force_stats.argtypes = [d, d, C.c_int32, C.c_double, C.c_double, d]
    L.orc_set_solid.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint8), d]
    L.orc3_velocity_set.argtypes = [C.c_int32] + [C.POINTER(C.c_int32)] * 3 + [d]
    L.orc3_velocity_set.restype = None
    L.orc3_feq.argtypes = [C.c_int32] + [C.c_double] * 4 + [d]
    L.orc3_feq.restype = None
    L.orc3_create.argtypes = [C.c_int32] * 4 + [C.c_double, d, C.POINTER(C.c_void_p)]
    L.orc3_destroy.argtypes = [C.c_void_p]
    L.orc3_destroy.restype = None
    L.orc3_init_fields.argtypes = [C.c_void_p, d, d, d, d]
    L.orc3_step.argtypes = [C.c_void_p, C.c_int32]
    L.orc3_read_fields.argtypes = [C.c_void_p, d, d, d, d]
    L.orc3_set_walls.argtypes = [C.c_void_p, C.c_double, d, d]
    L.orc3_set_solid.argtypes = [C.c_void_p, C.POINTER(C.c_uint8), d]
    L.orc3_set_body.argtypes = [C.c_void_p, C.c_int32, d, d, d, d, C.c_int32]
    L.orc3_body_force.argtypes = [C.c_void_p, d]
    L.orc3_set_motion.argtypes = [C.c_void_p, C.c_int32, d]
    L.orc3f_create.argtypes = [C.POINTER(_Case3F), C.POINTER(C.c_void_p)]
    L.orc3f_destroy.argtypes = [C.c_void_p]
    L.orc3f_destroy.restype = None
    L.orc3f_level_size.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int32)]
    L.orc3f_level_kinds.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint8)]
    L.orc3f_init_fields.argtypes = [C.c_void_p, C.c_int, d, d, d, d]
    L.orc3f_step.argtypes = [C.c_void_p, C.c_int32]
    L.orc3f_read_fields.argtypes = [C.c_void_p, C.c_int, d, d, d, d]
    L.orc3f_diagnostics.argtypes = [C.c_void_p, d]
    L.orc_num_threads.argtypes = []
    L.orc3_marker_positions.argtypes = [C.c_void_p, C.c_double, d, d, d]
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_case(wl):
    """Marshal a ``workloads.Workload`` into the oracle's C struct.

    Returns (struct, keepalive) -- keepalive holds the numpy buffers."""
    c = _Case()
    c.nx0, c.ny0, c.block_n, c.n_levels = wl.nx0, wl.ny0, wl.block_n, wl.n_levels
    boxes = np.ascontiguousarray(np.array(wl.boxes, dtype=np.int32).reshape(-1, 5))
    c.n_boxes = boxes.shape[0]
    c.boxes = boxes.ctypes.data_as(C.POINTER(C.c_int32))
    c.tau0, c.rho0 = wl.tau0, wl.rho0
    for e in range(4):
        c.bc[e] = wl.bc[e]
        c.bc_u[2 * e], c.bc_u[2 * e + 1] = wl.bc_u[e]
    c.fext[0], c.fext[1] = wl.fext
    c.cf_mode, c.mdf_iters = wl.cf_mode, wl.mdf_iters
    c.collision = wl.collision
    for k in range(3):
        c.mrt[k] = wl.mrt_rates[k]
    keep = [boxes]
    if wl.body is None:
        c.body_kind, c.n_markers = ORC_BODY_NONE, 0
    else:
        b = wl.body
        xb, yb, ds = _f64(b.xb), _f64(b.yb), _f64(b.ds)
        keep += [xb, yb, ds]
        c.body_kind, c.n_markers = b.kind, len(xb)
        c.xb, c.yb, c.ds = _dp(xb), _dp(yb), _dp(ds)
        for i, v in enumerate(b.params):
            c.bp[i] = v
    return c, keep


class OracleSim:
    """One case on the oracle.  Fields are dense per-level arrays [ny, nx]."""

    def __init__(self, wl, so=None):
        self.wl = wl
        self._L = so if so is not None else lib()
        self._case, self._keep = make_case(wl)
        h = C.c_void_p()
        rc = self._L.orc_create(C.byref(self._case), C.byref(h))
        if rc != 0:
            raise RuntimeError(f"orc_create failed: {rc}")
        self._h = h
        self.n_levels = wl.n_levels
        for level, mask, q in getattr(wl, "solids", ()):
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            qq = None if q is None else _f64(q)
            rc = self._L.orc_set_solid(h, level, m.ctypes.data_as(C.POINTER(C.c_uint8)),
                                     None if qq is None else _dp(qq))
            if rc != 0:
                raise RuntimeError(f"orc_set_solid failed: {rc}")
        if wl.init is not None:
            for l in range(wl.n_levels):
                nx, ny = self.level_size(l)
                rho, ux, uy = wl.init(l, nx, ny)
                self.init_fields(l, rho, ux, uy)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._L.orc_destroy(h)
            self._h = None

    def level_size(self, l):
        nx, ny = C.c_int32(), C.c_int32()
        self._L.orc_level_size(self._h, l, C.byref(nx), C.byref(ny))
        return nx.value, ny.value

    def kinds(self, l):
        nx, ny = self.level_size(l)
        k = np.zeros((ny, nx), dtype=np.uint8)
        self._L.orc_level_kinds(self._h, l, k.ctypes.data_as(C.POINTER(C.c_uint8)))
        return k

    def init_fields(self, l, rho, ux, uy):
        nx, ny = self.level_size(l)
        rho = _f64(np.broadcast_to(rho, (ny, nx)))
        ux = _f64(np.broadcast_to(ux, (ny, nx)))
        uy = _f64(np.broadcast_to(uy, (ny, nx)))
        rc = self._L.orc_init_fields(self._h, l, _dp(rho), _dp(ux), _dp(uy))
        if rc:
            raise RuntimeError(rc)

    def init_populations(self, l, f):
        """Pre-collision populations of the owned cells of level l, [ny, nx, 9]."""
        nx, ny = self.level_size(l)
        f = _f64(np.broadcast_to(f, (ny, nx, 9)))
        rc = self._L.orc_init_populations(self._h, l, _dp(f))
        if rc:
            raise RuntimeError(rc)

    def step(self, n=1):
        rc = self._L.orc_step(self._h, int(n))
        if rc:
            raise RuntimeError(f"orc_step failed: {rc}")

    def fields(self, l):
        nx, ny = self.level_size(l)
        r, u, v = (np.empty((ny, nx)) for _ in range(3))
        self._L.orc_read_fields(self._h, l, _dp(r), _dp(u), _dp(v))
        return r, u, v

    def populations(self, l):
        nx, ny = self.level_size(l)
        f = np.empty((ny, nx, 9))
        self._L.orc_read_populations(self._h, l, _dp(f))
        return f

    def marker_forces(self):
        n = 0 if self.wl.body is None else len(self.wl.body.xb)
        fx, fy = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._L.orc_marker_forces(self._h, _dp(fx), _dp(fy))
        return fx[:n], fy[:n]

    def set_markers(self, X, Y, udx, udy, ds=None):
        """Caller-placed markers (body kind HOST) for the next steps; ds
        (optional) replaces their arc-length weights."""
        X, Y, udx, udy = (_f64(a) for a in (X, Y, udx, udy))
        w = None if ds is None else _f64(ds)
        rc = self._L.orc_set_markers(self._h, len(X), _dp(X), _dp(Y), _dp(udx), _dp(udy),
                                     None if w is None else _dp(w))
        if rc:
            raise RuntimeError(f"orc_set_markers failed: {rc}")

    def force_history(self, cap=1 << 20):
        fx, fy = np.empty(cap), np.empty(cap)
        n = C.c_int32()
        self._L.orc_force_history(self._h, cap, _dp(fx), _dp(fy), C.byref(n))
        return fx[: n.value].copy(), fy[: n.value].copy()

    def velocity(self):
        """[(ux, uy)] per level, NaN off the leaf cells."""
        out = []
        for l in range(self.wl.n_levels):
            _, ux, uy = self.fields(l)
            out.append((ux, uy))
        return out

    def diagnostics(self):
        out = np.zeros(3)
        self._L.orc_diagnostics(self._h, _dp(out))
        return out

    def substeps(self):
        return int(self._L.orc_substeps(self._h))


# ---- building blocks ------------------------------------------------------

def interface_factors(tau_c, tau_f):
    """(s_cf, s_fc) the RESCALE interface applies between levels of these taus."""
    out = np.zeros(2)
    lib().orc_interface_factors(tau_c, tau_f, _dp(out))
    return float(out[0]), float(out[1])


def velocity_set():
    cx, cy = (C.c_int32 * 9)(), (C.c_int32 * 9)()
    w = np.zeros(9)
    lib().orc_velocity_set(cx, cy, _dp(w))
    return np.array(cx[:]), np.array(cy[:]), w


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_feq(rho, ux, uy, _dp(out))
    return out


def guo(tau, ux, uy, Fx, Fy):
    out = np.zeros(9)
    lib().orc_guo(tau, ux, uy, Fx, Fy, _dp(out))
    return out


def collide_cell(tau, f, Fx=0.0, Fy=0.0):
    f = _f64(f)
    out = np.zeros(9)
    lib().orc_collide_cell(tau, _dp(f), Fx, Fy, _dp(out))
    return out


def mrt_matrices():
    """The MRT moment basis M (9 x 9, rows rho, e, eps, jx, qx, jy, qy, pxx, pxy) and its inverse."""
    M, Mi = np.zeros(81), np.zeros(81)
    lib().orc_mrt_matrices(_dp(M), _dp(Mi))
    return M.reshape(9, 9), Mi.reshape(9, 9)


def collide_cell_mrt(tau, rates, f, Fx=0.0, Fy=0.0):
    f = _f64(f)
    r = _f64(np.asarray(rates, dtype=np.float64))
    out = np.zeros(9)
    lib().orc_collide_cell_mrt(float(tau), _dp(r), _dp(f), float(Fx), float(Fy), _dp(out))
    return out


def phi(r):
    return lib().orc_phi(float(r))


def body_positions(wl, k):
    c, keep = make_case(wl)
    n = len(wl.body.xb)
    X, Y = np.zeros(n), np.zeros(n)
    rc = lib().orc_body_positions(C.byref(c), float(k), _dp(X), _dp(Y))
    if rc:
        raise RuntimeError(rc)
    return X, Y


def ramp_alpha(p, tstar):
    """Pitch angle of the Sec. 3.5 ramp law at t* (p: the body's 16 parameters)."""
    p = _f64(np.asarray(p, dtype=np.float64))
    return lib().orc_ramp_alpha(_dp(p), float(tstar))


def tri_alpha(p, tstar):
    """Pitch angle of the Sec. 3.6 smoothed triangular law at t*."""
    p = _f64(np.asarray(p, dtype=np.float64))
    return lib().orc_tri_alpha(_dp(p), float(tstar))


def force_stats(fx, fy, U, L, rho0=1.0):
    """Sec. 3.3, Eq. (21) statistics of a force history: dict with CD_mean,
    CL_mean, CD_rms, CL_rms, St, crossings, samples."""
    fx, fy = _f64(fx), _f64(fy)
    out = np.zeros(7)
    rc = lib().orc_force_stats(_dp(fx), _dp(fy), len(fx), 1.0 / (0.5 * rho0 * U * U * L), L / U, _dp(out))
    if rc:
        raise RuntimeError(rc)
    keys = ("CD_mean", "CL_mean", "CD_rms", "CL_rms", "St", "crossings", "samples")
    return dict(zip(keys, out.tolist()))


def velocity_change(now, then):
    """Sec. 3.2 convergence measure between two velocity states, each a list
    over levels l of (ux, uy) dense arrays that are NaN off the level's leaf
    cells (owned, not covered by level l+1), as OracleSim.velocity() gives:
    returns (sum |u - u0|, sum |u|, E = ratio), every cell weighted by its
    area 4^-l, |.| the Euclidean norm."""
    num = den = 0.0
    for l, ((ux, uy), (vx, vy)) in enumerate(zip(now, then)):
        m = ~np.isnan(ux)
        w = 0.25 ** l
        num += w * np.sum(np.hypot(ux[m] - vx[m], uy[m] - vy[m]))
        den += w * np.sum(np.hypot(ux[m], uy[m]))
    return num, den, num / den


def mdf(rho, ux, uy, X, Y, udx, udy, ds, iters):
    """Run the MDF loop on a dense periodic grid; returns (ux, uy, Fx, Fy, ftx, fty)."""
    ny, nx = rho.shape
    rho = _f64(rho)
    ux, uy = _f64(ux).copy(), _f64(uy).copy()
    Fx, Fy = np.zeros((ny, nx)), np.zeros((ny, nx))
    X, Y, udx, udy, ds = (_f64(a) for a in (X, Y, udx, udy, ds))
    n = len(X)
    ftx, fty = np.zeros(n), np.zeros(n)
    lib().orc_mdf(nx, ny, _dp(rho), _dp(ux), _dp(uy), _dp(Fx), _dp(Fy), n, _dp(X), _dp(Y),
                  _dp(udx), _dp(udy), _dp(ds), iters, _dp(ftx), _dp(fty))
    return ux, uy, Fx, Fy, ftx, fty


def interpolate(ux, uy, X, Y):
    ny, nx = ux.shape
    ux, uy, X, Y = (_f64(a) for a in (ux, uy, X, Y))
    U, V = np.zeros(len(X)), np.zeros(len(X))
    lib().orc_interpolate(nx, ny, _dp(ux), _dp(uy), len(X), _dp(X), _dp(Y), _dp(U), _dp(V))
    return U, V


def spread(shape, X, Y, Fjx, Fjy, ds):
    ny, nx = shape
    X, Y, Fjx, Fjy, ds = (_f64(a) for a in (X, Y, Fjx, Fjy, ds))
    Fx, Fy = np.zeros((ny, nx)), np.zeros((ny, nx))
    lib().orc_spread(nx, ny, len(X), _dp(X), _dp(Y), _dp(Fjx), _dp(Fjy), _dp(ds), _dp(Fx), _dp(Fy))
    return Fx, Fy


def num_threads():
    return int(lib().orc_num_threads())


# ---- three dimensions ----------------------------------------------------------

def velocity_set3(q=19):
    cx, cy, cz = (np.zeros(q, dtype=np.int32) for _ in range(3))
    w = np.zeros(q)
    p32 = C.POINTER(C.c_int32)
    lib().orc3_velocity_set(q, cx.ctypes.data_as(p32), cy.ctypes.data_as(p32), cz.ctypes.data_as(p32), _dp(w))
    return cx, cy, cz, w


def feq3(rho, ux, uy, uz, q=19):
    out = np.zeros(q)
    lib().orc3_feq(q, float(rho), float(ux), float(uy), float(uz), _dp(out))
    return out


class _Case3F(C.Structure):
    _fields_ = [
        ("nx0", C.c_int32), ("ny0", C.c_int32), ("nz0", C.c_int32), ("block_n", C.c_int32),
        ("n_levels", C.c_int32), ("q", C.c_int32), ("n_boxes", C.c_int32), ("boxes", C.POINTER(C.c_int32)),
        ("tau0", C.c_double), ("rho0", C.c_double), ("fext", C.c_double * 3), ("cf_mode", C.c_int32),
    ]


class Oracle3FSim:
    """A periodic 3D block forest (a ``workloads.Workload3F``); fields are dense
    per-level arrays [nz, ny, nx], NaN where the level owns no cell."""

    def __init__(self, wl, so=None):
        self.wl = wl
        self._L = so if so is not None else lib()
        c = _Case3F()
        c.nx0, c.ny0, c.nz0, c.block_n = wl.nx0, wl.ny0, wl.nz0, wl.block_n
        c.n_levels, c.q = wl.n_levels, wl.lattice
        self._boxes = np.ascontiguousarray(np.array(wl.boxes, dtype=np.int32).reshape(-1, 7))
        c.n_boxes = self._boxes.shape[0]
        c.boxes = self._boxes.ctypes.data_as(C.POINTER(C.c_int32))
        c.tau0, c.rho0 = wl.tau0, wl.rho0
        for k in range(3):
            c.fext[k] = wl.fext[k]
        c.cf_mode = wl.cf_mode
        self._case = c
        h = C.c_void_p()
        rc = self._L.orc3f_create(C.byref(c), C.byref(h))
        if rc:
            raise RuntimeError(f"orc3f_create failed: {rc}")
        self._h = h
        self.n_levels = wl.n_levels
        if wl.init is not None:
            for l in range(wl.n_levels):
                self.init_fields(l, *wl.init(l, 0, 0, 0, *self.level_size(l)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._L.orc3f_destroy(h)
            self._h = None

    def level_size(self, l):
        out = (C.c_int32 * 3)()
        self._L.orc3f_level_size(self._h, l, out)
        return out[0], out[1], out[2]

    def kinds(self, l):
        nx, ny, nz = self.level_size(l)
        k = np.zeros((nz, ny, nx), dtype=np.uint8)
        self._L.orc3f_level_kinds(self._h, l, k.ctypes.data_as(C.POINTER(C.c_uint8)))
        return k

    def init_fields(self, l, rho, ux, uy, uz):
        nx, ny, nz = self.level_size(l)
        a = [_f64(np.broadcast_to(v, (nz, ny, nx))) for v in (rho, ux, uy, uz)]
        rc = self._L.orc3f_init_fields(self._h, l, *[_dp(v) for v in a])
        if rc:
            raise RuntimeError(rc)

    def step(self, n=1):
        rc = self._L.orc3f_step(self._h, int(n))
        if rc:
            raise RuntimeError(f"orc3f_step failed: {rc}")

    def fields(self, l):
        nx, ny, nz = self.level_size(l)
        out = [np.empty((nz, ny, nx)) for _ in range(4)]
        self._L.orc3f_read_fields(self._h, l, *[_dp(v) for v in out])
        return out

    def diagnostics(self):
        """(mass, momentum x, y, z) over owned cells, each level weighted by 8^-l."""
        out = np.zeros(4)
        self._L.orc3f_diagnostics(self._h, _dp(out))
        return out


class Oracle3Sim:
    """D3Q19 / D3Q27 BGK + Guo forcing on one periodic level (a ``workloads.Workload3``)."""

    def __init__(self, wl, so=None):
        self.wl = wl
        self._L = so if so is not None else lib()
        F = _f64(np.asarray(wl.fext, dtype=np.float64))
        h = C.c_void_p()
        rc = self._L.orc3_create(wl.nx, wl.ny, wl.nz, wl.lattice, wl.tau, _dp(F), C.byref(h))
        if rc:
            raise RuntimeError(f"orc3_create failed: {rc}")
        self._h = h
        if getattr(wl, "walls_z", False):
            ub, ut = (_f64(np.asarray(a, dtype=np.float64)) for a in wl.wall_u)
            self._L.orc3_set_walls(h, float(wl.rho0), _dp(ub), _dp(ut))
        if getattr(wl, "solid", None) is not None:
            mask, q = wl.solid
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            qq = None if q is None else _f64(q)
            rc = self._L.orc3_set_solid(h, m.ctypes.data_as(C.POINTER(C.c_uint8)), None if qq is None else _dp(qq))
            if rc:
                raise RuntimeError(f"orc3_set_solid failed: {rc}")
        if getattr(wl, "body", None) is not None:
            X, Y, Z, dA, iters = wl.body
            X, Y, Z, dA = (_f64(a) for a in (X, Y, Z, dA))
            self._body = (X, Y, Z, dA)
            rc = self._L.orc3_set_body(h, len(X), _dp(X), _dp(Y), _dp(Z), _dp(dA), int(iters))
            if rc:
                raise RuntimeError(f"orc3_set_body failed: {rc}")
            kind, params = getattr(wl, "motion", (0, None))
            pm = _f64(np.asarray(params if params is not None else [0.0] * 10, dtype=np.float64))
            self._L.orc3_set_motion(h, int(kind), _dp(pm))
        r, u, v, w = (_f64(a) for a in wl.init(wl.nx, wl.ny, wl.nz))
        self._L.orc3_init_fields(h, _dp(r), _dp(u), _dp(v), _dp(w))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._L.orc3_destroy(h)

    def step(self, n=1):
        self._L.orc3_step(self._h, int(n))

    def marker_positions(self, t):
        """Marker positions of the body at step t (the motion law's pose)."""
        n = len(self._body[0])
        X, Y, Z = np.zeros(n), np.zeros(n), np.zeros(n)
        self._L.orc3_marker_positions(self._h, float(t), _dp(X), _dp(Y), _dp(Z))
        return X, Y, Z

    def body_force(self):
        """F_s = -sum_j F_j dA_j of the last step (3 components)."""
        out = np.zeros(3)
        self._L.orc3_body_force(self._h, _dp(out))
        return out

    def fields(self):
        shape = (self.wl.nz, self.wl.ny, self.wl.nx)
        out = [np.empty(shape) for _ in range(4)]
        self._L.orc3_read_fields(self._h, *[_dp(a) for a in out])
        return out
