"""MI355X (gfx950) hot path of SBoTFlow's LBM-IBM method (arXiv 2402.04606).

Thin ctypes binding over ``libsbt.so`` (C ABI declared in ``include/sbt.h``).
This module only marshals arguments: every step of the time step runs in the
HIP kernels.  PyTorch provides the device buffer and the stream.  If the
library is not built, every entry point raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsbt.so")

F64, F32, F16S, BF16S = 0, 1, 2, 3
STORAGE = {"f64": F64, "f32": F32, "f16s": F16S, "bf16s": BF16S}
STORAGE_BYTES = {F64: 8, F32: 4, F16S: 2, BF16S: 2}
OPT_GRAPH, OPT_TILE, OPT_XCD_REMAP, OPT_PERSISTENT, OPT_BARRIER_SPINS = 0, 1, 2, 3, 4

ERRORS = {-1: "ARG", -2: "TOPOLOGY", -3: "DEVICE", -4: "NOMEM", -5: "STATE", -6: "NONFINITE",
          -7: "MARKER_OUTSIDE", -8: "BUFSIZE"}

# Every function include/sbt.h declares.
ABI_SYMBOLS = [
    "sbt_plan", "sbt_create", "sbt_create_static", "sbt_destroy", "sbt_level_blocks", "sbt_level_info", "sbt_init_fields",
    "sbt_init_uniform", "sbt_set_body", "sbt_set_markers", "sbt_step", "sbt_synchronize", "sbt_read_fields",
    "sbt_read_fields_blocks", "sbt_read_marker_forces",
    "sbt_read_force_history", "sbt_diagnostics", "sbt_force_stats", "sbt_snapshot_bytes",
    "sbt_convergence", "sbt_state_bytes", "sbt_read_state",
    "sbt_write_state", "sbt_set_option", "sbt_autotune", "sbt_profile", "sbt_updates_per_step",
    "sbt_last_error",
    "sbt3_plan", "sbt3_create", "sbt3_destroy", "sbt3_init_slab", "sbt3_step", "sbt3_synchronize",
    "sbt3_read_slab", "sbt3_body_force",
    "sbt3f_plan", "sbt3f_create", "sbt3f_destroy", "sbt3f_level_kinds", "sbt3f_init_box", "sbt3f_step",
    "sbt3f_synchronize", "sbt3f_read_box", "sbt3f_diagnostics",
]


class SbtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sbt error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class Box(C.Structure):
    _fields_ = [("level", C.c_int32), ("bx0", C.c_int32), ("by0", C.c_int32), ("bx1", C.c_int32),
                ("by1", C.c_int32)]


class Solid(C.Structure):
    _fields_ = [("level", C.c_int32), ("mask", C.POINTER(C.c_uint8)), ("q", C.POINTER(C.c_double))]


class Desc3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("tau", C.c_double),
                ("rho0", C.c_double), ("fext", C.c_double * 3), ("storage", C.c_int32),
                ("lattice", C.c_int32), ("walls_z", C.c_int32), ("wall_u", (C.c_double * 3) * 2),
                ("solid_mask", C.POINTER(C.c_uint8)), ("solid_q", C.POINTER(C.c_double)),
                ("n_markers", C.c_int32), ("marker_xyz", C.POINTER(C.c_double)),
                ("marker_dA", C.POINTER(C.c_double)), ("mdf_iters", C.c_int32),
                ("ibm_box_cells", C.c_int64), ("body_motion", C.c_int32), ("motion_p", C.c_double * 10)]


class Desc3F(C.Structure):
    _fields_ = [("nx0", C.c_int32), ("ny0", C.c_int32), ("nz0", C.c_int32), ("n_levels", C.c_int32),
                ("n_boxes", C.c_int32), ("boxes", C.POINTER(C.c_int32)), ("tau0", C.c_double),
                ("rho0", C.c_double), ("fext", C.c_double * 3), ("storage", C.c_int32), ("lattice", C.c_int32),
                ("cf_mode", C.c_int32)]


class CaseDesc(C.Structure):
    _fields_ = [
        ("nx0", C.c_int32), ("ny0", C.c_int32), ("block_n", C.c_int32), ("n_levels", C.c_int32),
        ("refine", C.POINTER(Box)), ("n_refine", C.c_int32),
        ("tau0", C.c_double), ("rho0", C.c_double),
        ("bc", C.c_int32 * 4), ("bc_u", (C.c_double * 2) * 4), ("fext", C.c_double * 2),
        ("storage", C.c_int32), ("cf_mode", C.c_int32), ("mdf_iters", C.c_int32),
        ("max_markers", C.c_int32), ("history_cap", C.c_int32),
        ("collision", C.c_int32), ("mrt_rates", C.c_double * 3),
        ("solids", C.POINTER(Solid)), ("n_solids", C.c_int32),
    ]


class Body(C.Structure):
    _fields_ = [("n", C.c_int32), ("xb", C.POINTER(C.c_double)), ("yb", C.POINTER(C.c_double)),
                ("ds", C.POINTER(C.c_double)), ("kind", C.c_int32), ("p", C.c_double * 16)]


_lib = None


def lib():
    """Load libsbt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        d, i32, i64, vp = C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_void_p
        sig = {
            "sbt_plan": [C.POINTER(CaseDesc), i32, C.POINTER(C.c_size_t)],
            "sbt_create": [C.POINTER(CaseDesc), i32, vp, C.c_size_t, vp, C.POINTER(vp)],
            "sbt_create_static": [C.POINTER(CaseDesc), i32, vp, C.POINTER(vp)],
            "sbt_destroy": [vp],
            "sbt_level_blocks": [vp, i32, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
            "sbt_level_info": [vp, i32, i32, C.POINTER(i64)],
            "sbt_init_fields": [vp, i32, i32, d, d, d],
            "sbt_init_uniform": [vp, i32, C.c_double, C.c_double, C.c_double],
            "sbt_read_fields_blocks": [vp, i32, i32, d],
            "sbt_set_body": [vp, i32, C.POINTER(Body)],
            "sbt_set_markers": [vp, i32, i32, d, d, d, d, d],
            "sbt_step": [vp, i32],
            "sbt_synchronize": [vp],
            "sbt_read_fields": [vp, i32, i32, d, d, d],
            "sbt_read_marker_forces": [vp, i32, d, d],
            "sbt_read_force_history": [vp, i32, i32, d, d, C.POINTER(i32)],
            "sbt_diagnostics": [vp, i32, d],
            "sbt_force_stats": [vp, i32, i32, C.c_double, C.c_double, d],
            "sbt_snapshot_bytes": [vp, i32, C.POINTER(C.c_size_t)],
            "sbt_convergence": [vp, i32, vp, C.c_size_t, i32, d],
            "sbt_state_bytes": [vp, C.POINTER(C.c_size_t)],
            "sbt_read_state": [vp, vp, C.c_size_t],
            "sbt_write_state": [vp, vp, C.c_size_t],
            "sbt_set_option": [vp, i32, i32],
            "sbt_autotune": [vp, i32, C.c_char_p],
            "sbt_profile": [vp, i32, d],
            "sbt_updates_per_step": [vp, C.POINTER(i64)],
            "sbt3_plan": [C.POINTER(Desc3), C.POINTER(C.c_size_t)],
            "sbt3_create": [C.POINTER(Desc3), vp, C.c_size_t, vp, C.POINTER(vp)],
            "sbt3_destroy": [vp],
            "sbt3_init_slab": [vp, i32, i32, d, d, d, d],
            "sbt3_step": [vp, i32],
            "sbt3_synchronize": [vp],
            "sbt3_read_slab": [vp, i32, i32, d, d, d, d],
            "sbt3_body_force": [vp, d],
            "sbt3f_plan": [C.POINTER(Desc3F), C.POINTER(C.c_size_t)],
            "sbt3f_create": [C.POINTER(Desc3F), vp, C.c_size_t, vp, C.POINTER(vp)],
            "sbt3f_destroy": [vp],
            "sbt3f_level_kinds": [C.POINTER(Desc3F), i32, C.POINTER(i32), C.POINTER(C.c_uint8), C.POINTER(i64)],
            "sbt3f_init_box": [vp, i32, C.POINTER(i32), d, d, d, d],
            "sbt3f_step": [vp, i32],
            "sbt3f_synchronize": [vp],
            "sbt3f_read_box": [vp, i32, C.POINTER(i32), d, d, d, d],
            "sbt3f_diagnostics": [vp, d],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int32
        L.sbt_last_error.argtypes = []
        L.sbt_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SbtError(rc, lib().sbt_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_desc(wl, storage=F64, history_cap=1 << 16, max_markers=None):
    """Marshal a ``workloads.Workload`` into an sbt_case_desc (+ keepalive)."""
    d = CaseDesc()
    d.nx0, d.ny0, d.block_n, d.n_levels = wl.nx0, wl.ny0, wl.block_n, wl.n_levels
    boxes = (Box * max(1, len(wl.boxes)))()
    for k, b in enumerate(wl.boxes):
        boxes[k].level, boxes[k].bx0, boxes[k].by0, boxes[k].bx1, boxes[k].by1 = b
    d.refine = C.cast(boxes, C.POINTER(Box))
    d.n_refine = len(wl.boxes)
    d.tau0, d.rho0 = wl.tau0, wl.rho0
    for e in range(4):
        d.bc[e] = wl.bc[e]
        d.bc_u[e][0], d.bc_u[e][1] = wl.bc_u[e]
    d.fext[0], d.fext[1] = wl.fext
    d.storage = storage
    d.cf_mode = wl.cf_mode
    d.mdf_iters = wl.mdf_iters
    nm = 0 if wl.body is None else len(wl.body.xb)
    d.max_markers = nm if max_markers is None else max_markers
    d.history_cap = history_cap
    d.collision = getattr(wl, "collision", 0)
    for k, v in enumerate(getattr(wl, "mrt_rates", (0.0, 0.0, 0.0))):
        d.mrt_rates[k] = v
    keep = [boxes]
    solids = list(getattr(wl, "solids", ()))
    if solids:
        arr = (Solid * len(solids))()
        for k, (level, mask, q) in enumerate(solids):
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            keep.append(m)
            arr[k].level = level
            arr[k].mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
            if q is not None:
                qq = np.ascontiguousarray(q, dtype=np.float64)
                keep.append(qq)
                arr[k].q = _dp(qq)
        keep.append(arr)
        d.solids = C.cast(arr, C.POINTER(Solid))
        d.n_solids = len(solids)
    return d, keep


def plan(workloads, storage=F64):
    descs, keep = _descs(workloads, storage)
    n = C.c_size_t()
    _check(lib().sbt_plan(descs, len(workloads), C.byref(n)))
    return n.value


def _descs(workloads, storage, history_cap=1 << 16):
    arr = (CaseDesc * len(workloads))()
    keep = []
    for k, wl in enumerate(workloads):
        d, b = make_desc(wl, storage, history_cap)
        arr[k] = d
        keep.append(b)
    return arr, keep


class Sim:
    """One context on cuda:0 holding one or more cases (a batch).

    Device memory is a torch uint8 buffer; the stream is torch's current
    stream unless one is given.  static_memory=True creates the context
    with sbt_create_static instead: its memory is the library's static
    device array and no buffer is allocated here."""

    def __init__(self, workloads, storage="f64", stream=None, history_cap=1 << 16, init=True,
                 static_memory=False):
        import torch
        if not isinstance(workloads, (list, tuple)):
            workloads = [workloads]
        self.workloads = list(workloads)
        self.storage = STORAGE[storage] if isinstance(storage, str) else storage
        L = lib()
        self._descs, self._keep = _descs(self.workloads, self.storage, history_cap)
        n = C.c_size_t()
        _check(L.sbt_plan(self._descs, len(self.workloads), C.byref(n)))
        self.device_bytes = n.value
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        if static_memory:
            self._buf = None
            _check(L.sbt_create_static(self._descs, len(self.workloads), C.c_void_p(self._stream.cuda_stream),
                                       C.byref(h)))
        else:
            self._buf = torch.empty(self.device_bytes + 256, dtype=torch.uint8, device="cuda")
            ptr = self._buf.data_ptr()
            ptr = (ptr + 255) // 256 * 256
            _check(L.sbt_create(self._descs, len(self.workloads), C.c_void_p(ptr), self.device_bytes,
                                C.c_void_p(self._stream.cuda_stream), C.byref(h)))
        self._h = h
        if init:
            for c, wl in enumerate(self.workloads):
                uni = getattr(wl.init, "uniform_state", None)
                if uni is not None:
                    self.init_uniform(c, *uni)
                elif wl.init is not None:
                    for l in range(wl.n_levels):
                        nx, ny = self.level_size(c, l)
                        r, u, v = wl.init(l, nx, ny)
                        self.init_fields(c, l, r, u, v)
                if wl.body is not None:
                    self.set_body(c, wl.body)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().sbt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- geometry ---------------------------------------------------------
    def level_size(self, c, l):
        wl = self.workloads[c]
        return wl.nx0 << l, wl.ny0 << l

    def level_blocks(self, c, l):
        n = C.c_int32()
        _check(lib().sbt_level_blocks(self._h, c, l, C.byref(n), None, None))
        ox, oy = np.zeros(n.value, np.int32), np.zeros(n.value, np.int32)
        _check(lib().sbt_level_blocks(self._h, c, l, C.byref(n),
                                      ox.ctypes.data_as(C.POINTER(C.c_int32)),
                                      oy.ctypes.data_as(C.POINTER(C.c_int32))))
        return ox, oy

    def level_info(self, c, l):
        out = (C.c_int64 * 4)()
        _check(lib().sbt_level_info(self._h, c, l, out))
        return dict(owned_cells=out[0], blocks=out[1], halo_blocks=out[2], substeps=out[3])

    def updates_per_step(self):
        u = C.c_int64()
        _check(lib().sbt_updates_per_step(self._h, C.byref(u)))
        return u.value

    # ---- state ------------------------------------------------------------
    def init_fields(self, c, l, rho, ux, uy):
        nx, ny = self.level_size(c, l)
        r = np.ascontiguousarray(np.broadcast_to(rho, (ny, nx)), dtype=np.float64)
        u = np.ascontiguousarray(np.broadcast_to(ux, (ny, nx)), dtype=np.float64)
        v = np.ascontiguousarray(np.broadcast_to(uy, (ny, nx)), dtype=np.float64)
        _check(lib().sbt_init_fields(self._h, c, l, _dp(r), _dp(u), _dp(v)))

    def init_uniform(self, c, rho, ux, uy):
        _check(lib().sbt_init_uniform(self._h, c, float(rho), float(ux), float(uy)))

    def set_body(self, c, body):
        xb, yb, ds = (np.ascontiguousarray(a, dtype=np.float64) for a in (body.xb, body.yb, body.ds))
        b = Body()
        b.n = len(xb)
        b.xb, b.yb, b.ds = _dp(xb), _dp(yb), _dp(ds)
        b.kind = body.kind
        for k, v in enumerate(body.params):
            b.p[k] = v
        _check(lib().sbt_set_body(self._h, c, C.byref(b)))

    def set_markers(self, c, x, y, udx, udy, ds=None):
        """Caller-placed markers (body kind HOST): positions, desired
        velocities and (optionally) arc-length weights for every finest
        substep from the next step on."""
        x, y, udx, udy = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, udx, udy))
        w = None if ds is None else np.ascontiguousarray(ds, dtype=np.float64)
        _check(lib().sbt_set_markers(self._h, c, len(x), _dp(x), _dp(y), _dp(udx), _dp(udy),
                                     None if w is None else _dp(w)))

    def step(self, n=1):
        _check(lib().sbt_step(self._h, int(n)))

    def synchronize(self):
        _check(lib().sbt_synchronize(self._h))

    # ---- outputs ----------------------------------------------------------
    def fields(self, c, l):
        nx, ny = self.level_size(c, l)
        r, u, v = (np.empty((ny, nx)) for _ in range(3))
        _check(lib().sbt_read_fields(self._h, c, l, _dp(r), _dp(u), _dp(v)))
        return r, u, v

    def fields_blocks(self, c, l):
        """Fields in block order [n_blocks, 3, 16, 16] (rho, ux, uy)."""
        n = self.level_info(c, l)["blocks"]
        out = np.empty((n, 3, 16, 16))
        _check(lib().sbt_read_fields_blocks(self._h, c, l, _dp(out)))
        return out

    def marker_forces(self, c=0):
        n = len(self.workloads[c].body.xb)
        fx, fy = np.empty(n), np.empty(n)
        _check(lib().sbt_read_marker_forces(self._h, c, _dp(fx), _dp(fy)))
        return fx, fy

    def force_history(self, c=0, cap=1 << 16):
        fx, fy = np.empty(cap), np.empty(cap)
        n = C.c_int32()
        _check(lib().sbt_read_force_history(self._h, c, cap, _dp(fx), _dp(fy), C.byref(n)))
        return fx[: n.value].copy(), fy[: n.value].copy()

    def diagnostics(self, c=0):
        out = np.zeros(3)
        _check(lib().sbt_diagnostics(self._h, c, _dp(out)))
        return out

    def force_stats(self, c=0, n_last=1 << 30, U=None, L=None):
        """Eq. (21) statistics of the last n_last finest substeps (device
        reduction): dict with CD_mean, CL_mean, CD_rms, CL_rms, St, crossings,
        samples.  U, L default to the workload's meta U and D (or chord)."""
        meta = self.workloads[c].meta or {}
        U = meta["U"] if U is None else U
        L = (meta.get("D") or meta.get("chord")) if L is None else L
        out = np.zeros(7)
        _check(lib().sbt_force_stats(self._h, c, int(min(n_last, 2 ** 31 - 1)), float(U), float(L), _dp(out)))
        keys = ("CD_mean", "CL_mean", "CD_rms", "CL_rms", "St", "crossings", "samples")
        return dict(zip(keys, out.tolist()))

    def snapshot(self, c=0):
        """A device buffer holding the velocity of every leaf cell now (for
        convergence())."""
        import torch
        n = C.c_size_t()
        _check(lib().sbt_snapshot_bytes(self._h, c, C.byref(n)))
        buf = torch.empty(max(1, n.value // 8), dtype=torch.float64, device="cuda")
        _check(lib().sbt_convergence(self._h, c, C.c_void_p(buf.data_ptr()), n.value, 1, None))
        return buf

    def convergence(self, snap, c=0, update=False):
        """Sec. 3.2 criterion E of the current velocity against a snapshot
        (sum |u - u0|, sum |u|, E); update=True also refreshes the snapshot."""
        out = np.zeros(3)
        _check(lib().sbt_convergence(self._h, c, C.c_void_p(snap.data_ptr()), snap.numel() * 8,
                                     3 if update else 2, _dp(out)))
        return out

    def state_bytes(self):
        n = C.c_size_t()
        _check(lib().sbt_state_bytes(self._h, C.byref(n)))
        return n.value

    def read_state(self):
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        _check(lib().sbt_read_state(self._h, buf.ctypes.data_as(C.c_void_p), buf.nbytes))
        return buf

    def write_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().sbt_write_state(self._h, buf.ctypes.data_as(C.c_void_p), buf.nbytes))

    # ---- tuning / measurement ------------------------------------------------
    def set_option(self, opt, value):
        _check(lib().sbt_set_option(self._h, opt, int(value)))

    def autotune(self, steps=3, cache_path=None):
        _check(lib().sbt_autotune(self._h, steps, cache_path.encode() if cache_path else None))

    def profile(self, n):
        out = np.zeros(9)
        _check(lib().sbt_profile(self._h, n, _dp(out)))
        return dict(level_ms=out[0], level_launches=int(out[1]), mdf_ms=out[2],
                    mdf_launches=int(out[3]), level_bytes=out[4], updates=out[5],
                    fast_ms=out[6], fast_launches=int(out[7]), fast_bytes=out[8])


class Sim3:
    """A D3Q19/D3Q27 box (``workloads.Workload3``) on cuda:0: torch device
    buffer, torch's current stream.  ``box_cells`` overrides the capacity of
    an immersed body's stencil box (default: the body's reach over its
    motion plus the stencil, capped at the lattice)."""

    def __init__(self, wl, storage="f64", stream=None, slab=None, box_cells=None):
        import torch
        self.wl = wl
        self.storage = STORAGE[storage] if isinstance(storage, str) else storage
        d = Desc3()
        d.nx, d.ny, d.nz, d.tau, d.rho0 = wl.nx, wl.ny, wl.nz, wl.tau, wl.rho0
        for k in range(3):
            d.fext[k] = wl.fext[k]
        d.storage = self.storage
        d.lattice = getattr(wl, "lattice", 19)
        d.walls_z = 1 if getattr(wl, "walls_z", False) else 0
        self._solid_keep = []
        if getattr(wl, "solid", None) is not None:
            mask, q = wl.solid
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            self._solid_keep.append(m)
            d.solid_mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
            if q is not None:
                qq = np.ascontiguousarray(q, dtype=np.float64)
                self._solid_keep.append(qq)
                d.solid_q = _dp(qq)
        if getattr(wl, "body", None) is not None:
            X, Y, Z, dA, iters = wl.body
            xyz = np.ascontiguousarray(np.concatenate([X, Y, Z]), dtype=np.float64)
            da = np.ascontiguousarray(dA, dtype=np.float64)
            self._solid_keep += [xyz, da]
            d.n_markers = len(X)
            d.marker_xyz = _dp(xyz)
            d.marker_dA = _dp(da)
            d.mdf_iters = int(iters)
            kind, params = getattr(wl, "motion", (0, None))
            d.ibm_box_cells = int(box_cells or 0)       # 0: sized by the library
            d.body_motion = int(kind)
            for i, v in enumerate(params or ()):
                d.motion_p[i] = float(v)
        for a, u in enumerate(getattr(wl, "wall_u", ((0.0,) * 3,) * 2)):
            for k in range(3):
                d.wall_u[a][k] = u[k]
        self._desc = d
        n = C.c_size_t()
        _check(lib().sbt3_plan(C.byref(d), C.byref(n)))
        self.device_bytes = n.value
        self._buf = torch.empty(n.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (self._buf.data_ptr() + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().sbt3_create(C.byref(d), C.c_void_p(ptr), n.value, C.c_void_p(self._stream.cuda_stream),
                                 C.byref(h)))
        self._h = h
        # initial state, a few planes at a time
        self.slab = slab or max(1, min(wl.nz, (1 << 24) // (wl.nx * wl.ny)))
        for z0 in range(0, wl.nz, self.slab):
            z1 = min(wl.nz, z0 + self.slab)
            r, u, v, w = (np.ascontiguousarray(a, dtype=np.float64) for a in wl.init(wl.nx, wl.ny, wl.nz, z0, z1))
            _check(lib().sbt3_init_slab(h, z0, z1 - z0, _dp(r), _dp(u), _dp(v), _dp(w)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().sbt3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().sbt3_step(self._h, int(n)))

    def synchronize(self):
        _check(lib().sbt3_synchronize(self._h))

    def fields(self, z0=0, z1=None):
        """(rho, ux, uy, uz), each [z1 - z0, ny, nx] FP64."""
        z1 = self.wl.nz if z1 is None else z1
        shape = (z1 - z0, self.wl.ny, self.wl.nx)
        out = [np.empty(shape) for _ in range(4)]
        _check(lib().sbt3_read_slab(self._h, z0, z1 - z0, *[_dp(a) for a in out]))
        return out

    def body_force(self):
        """F_s of the last step (3 components)."""
        out = np.zeros(3)
        _check(lib().sbt3_body_force(self._h, _dp(out)))
        return out

    def updates_per_step(self):
        return self.wl.nx * self.wl.ny * self.wl.nz


def desc3f(wl, storage=F64):
    """A ``workloads.Workload3F`` as the C descriptor; returns (desc, keepalive)."""
    d = Desc3F()
    d.nx0, d.ny0, d.nz0, d.n_levels = wl.nx0, wl.ny0, wl.nz0, wl.n_levels
    boxes = np.ascontiguousarray(np.array(wl.boxes, dtype=np.int32).reshape(-1, 7))
    d.n_boxes = boxes.shape[0]
    d.boxes = boxes.ctypes.data_as(C.POINTER(C.c_int32))
    d.tau0, d.rho0 = wl.tau0, wl.rho0
    for k in range(3):
        d.fext[k] = wl.fext[k]
    d.storage = STORAGE[storage] if isinstance(storage, str) else storage
    d.lattice, d.cf_mode = wl.lattice, wl.cf_mode
    return d, boxes


def _box(box):
    return (C.c_int32 * 6)(*[int(v) for v in box])


def level_info3f(wl, level):
    """(nx, ny, nz, owned, halo, hidden) of a level of the forest (host only)."""
    d, keep = desc3f(wl)
    info = (C.c_int64 * 6)()
    _check(lib().sbt3f_level_kinds(C.byref(d), level, None, None, info))
    return tuple(info)


def level_kinds3f(wl, level, box=None):
    """Kinds [nz, ny, nx] (0 none, 1 owned, 2 halo, 3 hidden) of a level's cells
    inside box (x0, y0, z0, nx, ny, nz; default: the whole level), host only."""
    info = level_info3f(wl, level)
    box = box or (0, 0, 0, info[0], info[1], info[2])
    d, keep = desc3f(wl)
    k = np.zeros((box[5], box[4], box[3]), dtype=np.uint8)
    _check(lib().sbt3f_level_kinds(C.byref(d), level, _box(box), k.ctypes.data_as(C.POINTER(C.c_uint8)), None))
    return k


class Sim3F:
    """A periodic 3D block forest (``workloads.Workload3F``) on cuda:0: torch
    device buffer, torch's current stream.  Each level is initialised over
    the bounding box of its region (level 0: the whole grid)."""

    def __init__(self, wl, storage="f64", stream=None):
        import torch
        self.wl = wl
        self.storage = STORAGE[storage] if isinstance(storage, str) else storage
        self._desc, self._keep = desc3f(wl, self.storage)
        n = C.c_size_t()
        _check(lib().sbt3f_plan(C.byref(self._desc), C.byref(n)))
        self.device_bytes = n.value
        self._buf = torch.empty(n.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (self._buf.data_ptr() + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().sbt3f_create(C.byref(self._desc), C.c_void_p(ptr), n.value,
                                  C.c_void_p(self._stream.cuda_stream), C.byref(h)))
        self._h = h
        self.n_levels = wl.n_levels
        self.info = [level_info3f(wl, l) for l in range(wl.n_levels)]
        if wl.init is not None:
            for l in range(wl.n_levels):
                for box in self.init_boxes(l):
                    self.init_box(l, box, *wl.init(l, *box))

    def level_size(self, l):
        return self.info[l][:3]

    def region_box(self, l):
        """Bounding box (x0, y0, z0, nx, ny, nz) of level l's boxes, level cells."""
        nx, ny, nz = self.level_size(l)
        if l == 0:
            return (0, 0, 0, nx, ny, nz)
        b = np.array([q for q in self.wl.boxes if q[0] == l]).reshape(-1, 7)
        lo, hi = b[:, 1:4].min(0) * 8, b[:, 4:7].max(0) * 8
        return (int(lo[0]), int(lo[1]), int(lo[2]), int(hi[0] - lo[0]), int(hi[1] - lo[1]), int(hi[2] - lo[2]))

    def init_boxes(self, l, max_cells=1 << 24):
        """The level's region box cut into z-slabs of at most max_cells cells."""
        x0, y0, z0, nx, ny, nz = self.region_box(l)
        dz = max(1, min(nz, max_cells // (nx * ny)))
        return [(x0, y0, z, nx, ny, min(dz, z0 + nz - z)) for z in range(z0, z0 + nz, dz)]

    def init_box(self, l, box, rho, ux, uy, uz):
        shape = (box[5], box[4], box[3])
        a = [np.ascontiguousarray(np.broadcast_to(v, shape), dtype=np.float64) for v in (rho, ux, uy, uz)]
        _check(lib().sbt3f_init_box(self._h, l, _box(box), *[_dp(v) for v in a]))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().sbt3f_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().sbt3f_step(self._h, int(n)))

    def synchronize(self):
        _check(lib().sbt3f_synchronize(self._h))

    def fields(self, l, box=None):
        """(rho, ux, uy, uz) of level l inside box (default: the whole level),
        each [nz, ny, nx] FP64, NaN where the level owns no cell."""
        box = box or (0, 0, 0, *self.level_size(l))
        out = [np.empty((box[5], box[4], box[3])) for _ in range(4)]
        _check(lib().sbt3f_read_box(self._h, l, _box(box), *[_dp(a) for a in out]))
        return out

    def diagnostics(self):
        out = np.zeros(4)
        _check(lib().sbt3f_diagnostics(self._h, _dp(out)))
        return out

    def updates_per_step(self):
        """Cell updates of one coarse step: owned cells of level l times 2^l."""
        return sum(self.info[l][3] << l for l in range(self.n_levels))
