"""Python binding of libhsgn.so (include/hsgn.h): argument marshalling only.

Every step of the time step runs in the library's HIP kernels.  Arrays are
numpy (host, on_device=0) or torch CUDA tensors (device, on_device=1); the
library copies them and never keeps the pointers.  If the library has not
been built, importing works but every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import types

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsgn.so")

HSGN_OK, HSGN_EINVAL, HSGN_ENOMEM, HSGN_ECFL, HSGN_ENONHYP, HSGN_ENAN, HSGN_ERANGE, \
    HSGN_EDEVICE, HSGN_ENOTSUP, HSGN_ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
BC_PERIODIC, BC_WALL, BC_EXTRAP = 0, 1, 2

EXPORTS = ("hsgn_create", "hsgn_add_grid", "hsgn_finalize", "hsgn_set_bathymetry",
           "hsgn_set_state", "hsgn_get_state", "hsgn_get_mask", "hsgn_set_mask",
           "hsgn_set_gauges", "hsgn_read_gauges", "hsgn_advance", "hsgn_diagnostics",
           "hsgn_get_clock", "hsgn_set_clock", "hsgn_work_items", "hsgn_set_timing",
           "hsgn_get_timing", "hsgn_autotune", "hsgn_regrid", "hsgn_num_patches",
           "hsgn_patch_info", "hsgn_set_mapping", "hsgn_set_sponge", "hsgn_advance_static",
           "hsgn_destroy", "hsgn_strerror", "hsgn_last_error")


class hsgn_params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("precision", ctypes.c_int),
                ("g", ctypes.c_double), ("alpha", ctypes.c_double), ("eta0", ctypes.c_double),
                ("h_star", ctypes.c_double), ("dry_tol", ctypes.c_double),
                ("xi0", ctypes.c_double), ("xi1", ctypes.c_double), ("cfl", ctypes.c_double),
                ("cfl_max", ctypes.c_double), ("kappa", ctypes.c_double),
                ("nbr_n", ctypes.c_int), ("limiter", ctypes.c_int),
                ("transverse", ctypes.c_int), ("splitting", ctypes.c_int),
                ("tile_rows", ctypes.c_int), ("c2", ctypes.c_double)]


class hsgn_regrid_params(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("nbuf", ctypes.c_int), ("tol", ctypes.c_double),
                ("cutoff", ctypes.c_double), ("max_side", ctypes.c_int)]


class hsgn_diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("clipped_mass", ctypes.c_double),
                ("max_courant", ctypes.c_double), ("last_courant", ctypes.c_double),
                ("steps", ctypes.c_longlong), ("rejected", ctypes.c_longlong),
                ("cell_updates", ctypes.c_longlong), ("n_swe_cells", ctypes.c_longlong),
                ("n_breaking", ctypes.c_longlong)]


class HsgnError(RuntimeError):
    def __init__(self, code, where, msg=""):
        super().__init__("%s failed: %d (%s) %s" % (where, code, _strerror(code), msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhsgn.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
        L.hsgn_create.argtypes = [ctypes.POINTER(hsgn_params), vp, ctypes.POINTER(vp)]
        L.hsgn_add_grid.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ip, ip]
        L.hsgn_finalize.argtypes = [vp]
        for n in ("hsgn_set_bathymetry", "hsgn_set_state", "hsgn_get_state", "hsgn_get_mask",
                  "hsgn_set_mask"):
            getattr(L, n).argtypes = [vp, ctypes.c_int, dp, ctypes.c_int]
        L.hsgn_set_gauges.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp]
        L.hsgn_read_gauges.argtypes = [vp, ctypes.c_int, dp, dp, ctypes.c_int, ip]
        L.hsgn_advance.argtypes = [vp, ctypes.c_double, ctypes.c_int]
        L.hsgn_autotune.argtypes = [vp, ctypes.c_int, ip]
        L.hsgn_diagnostics.argtypes = [vp, ctypes.c_int, ctypes.POINTER(hsgn_diag)]
        L.hsgn_get_clock.argtypes = [vp, ctypes.c_int, dp, dp, dp]
        L.hsgn_set_clock.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_longlong]
        L.hsgn_work_items.argtypes = [vp, ip]
        L.hsgn_set_timing.argtypes = [vp, ctypes.c_int]
        L.hsgn_get_timing.argtypes = [vp, dp, dp]
        L.hsgn_regrid.argtypes = [vp, ctypes.c_int, ctypes.POINTER(hsgn_regrid_params), ip]
        L.hsgn_set_sponge.argtypes = [vp, ctypes.c_int, dp, ctypes.c_double]
        L.hsgn_set_mapping.argtypes = [vp, ctypes.c_int, vp, vp]
        L.hsgn_num_patches.argtypes = [vp, ip]
        L.hsgn_patch_info.argtypes = [vp, ctypes.c_int, ip, ip, ip, ip, dp, dp, dp, dp]
        L.hsgn_advance_static.argtypes = [ctypes.POINTER(hsgn_params), vp, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_int), vp, vp, ctypes.c_double,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
        L.hsgn_destroy.argtypes = [vp]
        L.hsgn_strerror.argtypes = [ctypes.c_int]
        L.hsgn_strerror.restype = ctypes.c_char_p
        L.hsgn_last_error.argtypes = [vp]
        L.hsgn_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().hsgn_strerror(code).decode()
    except Exception:
        return "?"


def make_params(p, tile_rows=0, precision=0) -> hsgn_params:
    """hsgn_params from a workloads.Params."""
    return hsgn_params(getattr(p, "model", 0), precision, p.g, p.alpha, p.eta0, p.h_star,
                       p.dry_tol, p.xi0, p.xi1,
                       p.cfl, p.cfl_max, p.kappa, p.nbr_n, p.limiter, p.transverse,
                       p.splitting, tile_rows, getattr(p, "c2", 0.0))


def _ptr(a):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return ctypes.c_void_p(a.ctypes.data), 0
    if hasattr(a, "data_ptr"):
        assert a.is_contiguous()
        return ctypes.c_void_p(a.data_ptr()), 1 if a.is_cuda else 0
    raise TypeError("numpy array or torch tensor expected")


class Context:
    """One hsgn_ctx: patches grouped into scenarios, advanced together."""

    def __init__(self, params, tile_rows=0, stream=None, precision=0):
        L = lib()
        self._prm = make_params(params, tile_rows, precision)
        h = ctypes.c_void_p()
        s = ctypes.c_void_p(stream) if stream is not None else None
        self._check(L.hsgn_create(ctypes.byref(self._prm), s, ctypes.byref(h)), "hsgn_create", None)
        self.h = h
        self.grids = []
        self.ngauge = {}

    def _check(self, rc, where, h="self"):
        if rc != HSGN_OK:
            msg = ""
            hh = self.h if h == "self" else None
            if hh:
                msg = lib().hsgn_last_error(hh).decode()
            raise HsgnError(rc, where, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().hsgn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_grid(self, scenario, grid, level=0):
        pid = ctypes.c_int(-1)
        bc = (ctypes.c_int * 4)(*grid.bc)
        self._check(lib().hsgn_add_grid(self.h, scenario, level, grid.nx, grid.ny, grid.x0,
                                        grid.y0, grid.dx, grid.dy, bc, ctypes.byref(pid)),
                    "hsgn_add_grid")
        self.grids.append(grid)
        return pid.value

    def finalize(self):
        self._check(lib().hsgn_finalize(self.h), "hsgn_finalize")

    def set_bathymetry(self, patch, b):
        if isinstance(b, np.ndarray):
            b = np.ascontiguousarray(b, dtype=np.float64)
        p, dev = _ptr(b)
        self._check(lib().hsgn_set_bathymetry(self.h, patch, p, dev), "hsgn_set_bathymetry")

    def set_state(self, patch, q):
        if isinstance(q, np.ndarray):
            q = np.ascontiguousarray(q, dtype=np.float64)
        p, dev = _ptr(q)
        self._check(lib().hsgn_set_state(self.h, patch, p, dev), "hsgn_set_state")

    def get_state(self, patch, out=None):
        g = self.grids[patch]
        if out is None:
            out = np.empty((7, g.ny, g.nx))
        p, dev = _ptr(out)
        self._check(lib().hsgn_get_state(self.h, patch, p, dev), "hsgn_get_state")
        return out

    def get_mask(self, patch):
        g = self.grids[patch]
        out = np.empty((g.ny, g.nx), dtype=np.uint8)
        p, dev = _ptr(out)
        self._check(lib().hsgn_get_mask(self.h, patch, p, dev), "hsgn_get_mask")
        return out

    def set_mask(self, patch, m):
        m = np.ascontiguousarray(m, dtype=np.uint8)
        p, dev = _ptr(m)
        self._check(lib().hsgn_set_mask(self.h, patch, p, dev), "hsgn_set_mask")

    def set_mapping(self, patch, xn, yn):
        """mapped grid or patch-set patch: node coordinates [ny + 5][nx + 5]
        of nodes (i, j), i = -2..nx+2, j = -2..ny+2 (two ghost layers
        included)"""
        xn = np.ascontiguousarray(xn, dtype=np.float64)
        yn = np.ascontiguousarray(yn, dtype=np.float64)
        nx, ny = ctypes.c_int(0), ctypes.c_int(0)
        self._check(lib().hsgn_patch_info(self.h, int(patch), None, None, ctypes.byref(nx),
                                          ctypes.byref(ny), None, None, None, None),
                    "hsgn_patch_info")
        if xn.shape != (ny.value + 5, nx.value + 5) or yn.shape != xn.shape:
            raise ValueError("node arrays of shape [ny + 5][nx + 5] = (%d, %d) expected, got %s, %s"
                             % (ny.value + 5, nx.value + 5, xn.shape, yn.shape))
        self._check(lib().hsgn_set_mapping(self.h, int(patch), ctypes.c_void_p(xn.ctypes.data),
                                           ctypes.c_void_p(yn.ctypes.data)), "hsgn_set_mapping")

    def set_sponge(self, scenario, width, rate):
        """sponge widths (m) from the x-low, x-high, y-low, y-high sides of
        the scenario's domain and peak rate (1/s); rate 0 removes it"""
        w = np.ascontiguousarray(width, dtype=np.float64)
        if w.shape != (4,):
            raise ValueError("four widths")
        self._check(lib().hsgn_set_sponge(self.h, int(scenario), ctypes.c_void_p(w.ctypes.data),
                                          float(rate)), "hsgn_set_sponge")

    def set_gauges(self, scenario, xy):
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        self.ngauge[scenario] = xy.shape[0]
        self._check(lib().hsgn_set_gauges(self.h, scenario, xy.shape[0],
                                          ctypes.c_void_p(xy.ctypes.data)), "hsgn_set_gauges")

    def read_gauges(self, scenario, max_records=1 << 20):
        ng = max(self.ngauge.get(scenario, 0), 1)
        t = np.empty(max_records)
        e = np.empty((max_records, ng))
        n = ctypes.c_int(0)
        self._check(lib().hsgn_read_gauges(self.h, scenario, ctypes.c_void_p(t.ctypes.data),
                                           ctypes.c_void_p(e.ctypes.data), max_records,
                                           ctypes.byref(n)), "hsgn_read_gauges")
        return t[:n.value].copy(), e[:n.value, :self.ngauge.get(scenario, 0)].copy()

    def advance(self, dt, n):
        self._check(lib().hsgn_advance(self.h, float(dt), int(n)), "hsgn_advance")

    def advance_status(self, dt, n):
        """hsgn_advance returning the status code instead of raising."""
        return lib().hsgn_advance(self.h, float(dt), int(n))

    def diagnostics(self, scenario=0):
        d = hsgn_diag()
        self._check(lib().hsgn_diagnostics(self.h, scenario, ctypes.byref(d)), "hsgn_diagnostics")
        return {f: getattr(d, f) for f, _ in hsgn_diag._fields_}

    def clock(self, scenario=0):
        t, d, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        self._check(lib().hsgn_get_clock(self.h, scenario, ctypes.byref(t), ctypes.byref(d),
                                         ctypes.byref(s)), "hsgn_get_clock")
        return t.value, d.value, s.value

    def set_clock(self, scenario, t, dt_next, steps):
        self._check(lib().hsgn_set_clock(self.h, scenario, t, dt_next, steps), "hsgn_set_clock")

    def set_timing(self, on):
        self._check(lib().hsgn_set_timing(self.h, 1 if on else 0), "hsgn_set_timing")

    def get_timing(self):
        """(summed step-kernel milliseconds, launches) since the last call."""
        ms, n = ctypes.c_double(), ctypes.c_longlong()
        self._check(lib().hsgn_get_timing(self.h, ctypes.byref(ms), ctypes.byref(n)),
                    "hsgn_get_timing")
        return ms.value, n.value

    def autotune(self, trials=3):
        """time the candidate tile heights per refinement level on the
        current state (which does not advance); returns the chosen heights"""
        rows = (ctypes.c_int * 8)()
        self._check(lib().hsgn_autotune(self.h, int(trials), rows), "hsgn_autotune")
        return [rows[k] for k in range(8) if rows[k] > 0]

    def regrid(self, scenario, level, tol, nbuf=2, cutoff=0.7, max_side=32):
        """rebuild level+1 of a patch-set scenario from the surface-jump
        flags on `level` (deeper levels are dropped); patch ids change:
        returns the new patch list (self.patches())"""
        r = hsgn_regrid_params(int(level), int(nbuf), float(tol), float(cutoff), int(max_side))
        n = ctypes.c_int(0)
        self._check(lib().hsgn_regrid(self.h, int(scenario), ctypes.byref(r), ctypes.byref(n)),
                    "hsgn_regrid")
        plist = self.patches()
        self.grids = [types.SimpleNamespace(nx=p["nx"], ny=p["ny"], x0=p["x0"], y0=p["y0"],
                                            dx=p["dx"], dy=p["dy"]) for p in plist]
        return plist

    def patches(self):
        """[{scenario, level, nx, ny, x0, y0, dx, dy}] by patch id"""
        n = ctypes.c_int(0)
        self._check(lib().hsgn_num_patches(self.h, ctypes.byref(n)), "hsgn_num_patches")
        out = []
        for pid in range(n.value):
            s, l, nx, ny = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            x0, y0, dx, dy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            self._check(lib().hsgn_patch_info(self.h, pid, ctypes.byref(s), ctypes.byref(l),
                                              ctypes.byref(nx), ctypes.byref(ny),
                                              ctypes.byref(x0), ctypes.byref(y0),
                                              ctypes.byref(dx), ctypes.byref(dy)),
                        "hsgn_patch_info")
            out.append(dict(scenario=s.value, level=l.value, nx=nx.value, ny=ny.value,
                            x0=x0.value, y0=y0.value, dx=dx.value, dy=dy.value))
        return out

    def work_items(self):
        n = ctypes.c_int()
        self._check(lib().hsgn_work_items(self.h, ctypes.byref(n)), "hsgn_work_items")
        return n.value


def advance_static(params, grid, b, q, dt, n_steps, stream=None, tile_rows=0):
    """hsgn_advance_static: one FP64 grid (workloads.Grid) advanced in place
    by n_steps fixed steps with no allocation; b [ny][nx] and q [7][ny][nx]
    are float64 CUDA tensors.  Returns the accepted steps."""
    for a in (b, q):
        if not (hasattr(a, "is_cuda") and a.is_cuda and a.is_contiguous()):
            raise TypeError("contiguous CUDA tensors expected")
    prm = make_params(params, tile_rows, 0)
    bc = (ctypes.c_int * 4)(*grid.bc)
    done = ctypes.c_longlong(0)
    s = ctypes.c_void_p(stream) if stream is not None else None
    rc = lib().hsgn_advance_static(ctypes.byref(prm), s, grid.nx, grid.ny, grid.dx, grid.dy, bc,
                                   ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                   float(dt), int(n_steps), ctypes.byref(done))
    if rc != HSGN_OK:
        raise HsgnError(rc, "hsgn_advance_static")
    return done.value


def from_amr_workloads(workloads, tile_rows=0, stream=None, gauges=True, precision=0,
                       nodes=None):
    """A finalized context with one patch-set scenario per AMR workload
    (patches added in workload order), bathymetry, state, gauges and the
    fixed level-0 step (scenario clock) set; nodes: per workload, None or the
    (xn, yn) node coordinates of each of its patches (a mapped patch set).
    Returns (context, patch ids)."""
    ws = list(workloads)
    for w in ws[1:]:
        if w.params != ws[0].params:
            raise ValueError("workloads of one context must share their parameters")
    ctx = Context(ws[0].params, tile_rows=tile_rows, stream=stream, precision=precision)
    ids = []
    for s, w in enumerate(ws):
        ids.append([])
        for p in w.patches:
            d = 4.0 ** p.level
            g = types.SimpleNamespace(nx=p.nx, ny=p.ny, x0=p.x0, y0=p.y0, dx=w.dx0 / d,
                                      dy=w.dy0 / d, bc=tuple(w.bc))
            ids[s].append(ctx.add_grid(s, g, level=p.level))
    ctx.finalize()
    for s, w in enumerate(ws):
        for pid, p in zip(ids[s], w.patches):
            ctx.set_bathymetry(pid, p.b)
        for pid, p in zip(ids[s], w.patches):
            ctx.set_state(pid, p.q)
        if gauges and w.gauges is not None and len(w.gauges):
            ctx.set_gauges(s, w.gauges)
        ctx.set_clock(s, 0.0, w.dt, 0)
        if nodes is not None and nodes[s] is not None:
            for pid, (xn, yn) in zip(ids[s], nodes[s]):
                ctx.set_mapping(pid, xn, yn)
    return ctx, ids


def from_workloads(workloads, tile_rows=0, stream=None, gauges=True, precision=0):
    """A finalized context with one scenario per workload (one patch each),
    bathymetry, state and gauges set; precision 0 is FP64, 1 mixed."""
    ws = list(workloads)
    for w in ws[1:]:
        if w.params != ws[0].params:
            raise ValueError("workloads of one context must share their parameters")
    ctx = Context(ws[0].params, tile_rows=tile_rows, stream=stream, precision=precision)
    for s, w in enumerate(ws):
        ctx.add_grid(s, w.grid)
    ctx.finalize()
    for s, w in enumerate(ws):
        ctx.set_bathymetry(s, w.b)
        ctx.set_state(s, w.q)
        if gauges and w.gauges is not None and len(w.gauges):
            ctx.set_gauges(s, w.gauges)
    return ctx
