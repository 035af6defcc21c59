"""ctypes binding of the plain FP64 CPU oracle (oracle/hsgn_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HSGN_ORACLE_LIB", os.path.join(HERE, "libhsgn_oracle.so"))
# the same source in x87 extended precision (measurement of the FP64
# oracle's own rounding error on a case; never a parity reference)
LIB_PATH_EXT = os.path.join(HERE, "libhsgn_oracle_ext.so")
SRC_PATH = os.path.join(HERE, "hsgn_oracle.c")

OK, EINVAL, ENOMEM, ECFL, ENONHYP, ENAN, ERANGE = 0, -1, -2, -3, -4, -5, -6


def build(openmp: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, no fast-math;
    once in FP64 and once in extended precision."""
    for path, extra in ((LIB_PATH, []), (LIB_PATH_EXT, ["-DORC_LONG_DOUBLE"])):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
               "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas"] + extra + \
              ["-o", path, SRC_PATH, "-lm"]
        if openmp:
            cmd.insert(1, "-fopenmp")
        subprocess.run(cmd, check=True)
    return LIB_PATH


class OrcParams(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("alpha", ctypes.c_double),
                ("eta0", ctypes.c_double), ("h_star", ctypes.c_double),
                ("dry_tol", ctypes.c_double), ("xi0", ctypes.c_double),
                ("xi1", ctypes.c_double), ("cfl", ctypes.c_double),
                ("cfl_max", ctypes.c_double), ("kappa", ctypes.c_double),
                ("nbr_n", ctypes.c_int), ("limiter", ctypes.c_int),
                ("transverse", ctypes.c_int), ("splitting", ctypes.c_int),
                ("model", ctypes.c_int), ("c2", ctypes.c_double)]


def _params(p) -> OrcParams:
    return OrcParams(p.g, p.alpha, p.eta0, p.h_star, p.dry_tol, p.xi0, p.xi1,
                     p.cfl, p.cfl_max, p.kappa, p.nbr_n, p.limiter,
                     p.transverse, p.splitting, getattr(p, "model", 0),
                     getattr(p, "c2", 0.0))


_lib = None
_lib_ext = None


def lib(extended: bool = False):
    """the FP64 oracle, or (extended=True) its extended-precision build"""
    global _lib, _lib_ext
    if extended:
        if _lib_ext is None:
            if not os.path.exists(LIB_PATH_EXT):
                build()
            _lib_ext = _bind(ctypes.CDLL(LIB_PATH_EXT))
        return _lib_ext
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _bind(L):
    """argument and result types of the oracle's C interface"""
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_create.restype = ctypes.c_void_p
    L.orc_create.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_int, ctypes.c_int,
                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    for name in ("orc_set_bathymetry", "orc_set_state", "orc_get_state"):
        getattr(L, name).argtypes = [ctypes.c_void_p, dp]
    L.orc_get_mask.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    L.orc_set_mask.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_double, dp]
    L.orc_advance.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
    L.orc_initial_dt.argtypes = [ctypes.c_void_p, dp]
    L.orc_get_clock.argtypes = [ctypes.c_void_p, dp, dp,
                                ctypes.POINTER(ctypes.c_longlong),
                                ctypes.POINTER(ctypes.c_longlong)]
    L.orc_set_clock.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                ctypes.c_longlong]
    L.orc_set_gauges.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    L.orc_read_gauges.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int)]
    L.orc_mass.restype = ctypes.c_double
    L.orc_mass.argtypes = [ctypes.c_void_p]
    L.orc_clipped_mass.restype = ctypes.c_double
    L.orc_clipped_mass.argtypes = [ctypes.c_void_p]
    L.orc_riemann_x.argtypes = [ctypes.POINTER(OrcParams), dp, dp, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int)]
    L.orc_source_cell.argtypes = [dp, ctypes.c_double, ctypes.c_double]
    L.orc_source_cell_mb.argtypes = [dp, ctypes.c_double, ctypes.c_double]
    ucp = ctypes.POINTER(ctypes.c_ubyte)
    L.orc_framed.argtypes = [ctypes.c_void_p, ctypes.POINTER(dp), ctypes.POINTER(dp),
                             ctypes.POINTER(ucp), ctypes.POINTER(ucp), ctypes.POINTER(ucp),
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.orc_set_external_ghosts.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_set_sponge.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_longlong,
                                 ctypes.c_longlong, ctypes.c_longlong, ctypes.c_longlong]
    L.orc_update_phi_framed.argtypes = [ctypes.c_void_p]
    L.orc_set_mapping.argtypes = [ctypes.c_void_p, dp, dp]
    L.orc_metric.argtypes = [ctypes.c_void_p, dp]
    L.orc_edge_dflux_mapped_n.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_int, ctypes.c_int,
                                          dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.orc_boundary_flux.argtypes = [ctypes.c_void_p, dp]
    L.orc_edge_dflux.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_int, dp, dp,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, dp]
    L.orc_set_radial.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_source_cells.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int]
    L.orc_edge_dflux_n.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_int, ctypes.c_int, dp, dp,
                                   dp, dp, dp, dp, dp]
    L.orc_limiter_phi.restype = ctypes.c_double
    L.orc_limiter_phi.argtypes = [ctypes.c_int, ctypes.c_double]
    L.orc_gauge_eta.restype = ctypes.c_double
    L.orc_gauge_eta.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__("oracle %s failed with status %d" % (where, code))
        self.code = code


def _check(rc, where):
    if rc != OK:
        raise OracleError(rc, where)


class OracleGrid:
    """One grid patch advanced by the oracle."""

    def __init__(self, params, grid, extended=False):
        L = self.L = lib(extended)
        self.params = params
        self.grid = grid
        self._p = _params(params)
        bc = (ctypes.c_int * 4)(*grid.bc)
        self.h = L.orc_create(ctypes.byref(self._p), grid.nx, grid.ny, grid.x0, grid.y0,
                              grid.dx, grid.dy, bc)
        if not self.h:
            raise OracleError(EINVAL, "create")
        self.ngauge = 0

    def close(self):
        if self.h:
            self.L.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_bathymetry(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        assert b.shape == (self.grid.ny, self.grid.nx)
        _check(self.L.orc_set_bathymetry(self.h, _dp(b)), "set_bathymetry")

    def set_state(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == (7, self.grid.ny, self.grid.nx)
        _check(self.L.orc_set_state(self.h, _dp(q)), "set_state")

    def get_state(self):
        q = np.empty((7, self.grid.ny, self.grid.nx))
        _check(self.L.orc_get_state(self.h, _dp(q)), "get_state")
        return q

    def get_mask(self):
        m = np.empty((self.grid.ny, self.grid.nx), dtype=np.uint8)
        _check(self.L.orc_get_mask(self.h, m.ctypes.data_as(ctypes.c_char_p)), "get_mask")
        return m

    def set_mask(self, m):
        m = np.ascontiguousarray(m, dtype=np.uint8)
        _check(self.L.orc_set_mask(self.h, m.ctypes.data_as(ctypes.c_char_p)), "set_mask")

    def step(self, dt):
        c = ctypes.c_double(0.0)
        _check(self.L.orc_step(self.h, dt, ctypes.byref(c)), "step")
        return c.value

    def advance(self, dt, n):
        _check(self.L.orc_advance(self.h, float(dt), int(n)), "advance")

    def initial_dt(self):
        d = ctypes.c_double(0.0)
        _check(self.L.orc_initial_dt(self.h, ctypes.byref(d)), "initial_dt")
        return d.value

    def clock(self):
        t, d = ctypes.c_double(), ctypes.c_double()
        s, r = ctypes.c_longlong(), ctypes.c_longlong()
        _check(self.L.orc_get_clock(self.h, ctypes.byref(t), ctypes.byref(d),
                                   ctypes.byref(s), ctypes.byref(r)), "get_clock")
        return t.value, d.value, s.value, r.value

    def set_clock(self, t, dt_next, steps):
        _check(self.L.orc_set_clock(self.h, t, dt_next, steps), "set_clock")

    def set_gauges(self, xy):
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        self.ngauge = xy.shape[0]
        _check(self.L.orc_set_gauges(self.h, self.ngauge, _dp(xy)), "set_gauges")

    def read_gauges(self, max_records=1 << 20):
        t = np.empty(max_records)
        e = np.empty((max_records, max(self.ngauge, 1)))
        n = ctypes.c_int(0)
        _check(self.L.orc_read_gauges(self.h, _dp(t), _dp(e), max_records,
                                     ctypes.byref(n)), "read_gauges")
        return t[:n.value].copy(), e[:n.value, :self.ngauge].copy()

    def mass(self):
        return self.L.orc_mass(self.h)

    # --- patch sets: framed arrays shared with the C grid (no copies) ---
    def framed(self):
        """numpy views (q[7][sy][sx], b, phi, brk, iface [sy][sx]) of the
        grid's own arrays; interior cell (i, j) sits at [j + 2, i + 2]."""
        dp = ctypes.POINTER(ctypes.c_double)
        ucp = ctypes.POINTER(ctypes.c_ubyte)
        q, b = dp(), dp()
        phi, brk, ifc = ucp(), ucp(), ucp()
        sx, sy = ctypes.c_int(), ctypes.c_int()
        _check(self.L.orc_framed(self.h, ctypes.byref(q), ctypes.byref(b), ctypes.byref(phi),
                                ctypes.byref(brk), ctypes.byref(ifc), ctypes.byref(sx),
                                ctypes.byref(sy)), "framed")
        n = sx.value * sy.value
        shp = (sy.value, sx.value)
        return (np.ctypeslib.as_array(q, shape=(7 * n,)).reshape((7,) + shp),
                np.ctypeslib.as_array(b, shape=(n,)).reshape(shp),
                np.ctypeslib.as_array(phi, shape=(n,)).reshape(shp),
                np.ctypeslib.as_array(brk, shape=(n,)).reshape(shp),
                np.ctypeslib.as_array(ifc, shape=(n,)).reshape(shp))

    def set_sponge(self, width, rate, offset=(0, 0), domain=None):
        """sponge widths (m) from the x-low, x-high, y-low, y-high sides of
        the domain and peak rate (1/s); offset: global index of cell (0, 0);
        domain: the domain in cells of this spacing (default: this grid)"""
        w = np.ascontiguousarray(width, dtype=np.float64)
        assert w.shape == (4,)
        nxd, nyd = domain if domain is not None else (self.grid.nx, self.grid.ny)
        _check(self.L.orc_set_sponge(self.h, _dp(w), float(rate), int(offset[0]), int(offset[1]),
                                    int(nxd), int(nyd)), "set_sponge")

    def set_mapping(self, xn, yn):
        """mapped grid: node coordinates [ny + 5][nx + 5] of nodes (i, j),
        i = -2..nx+2, j = -2..ny+2 (two ghost layers included); the grid's
        dx, dy become the computational spacings"""
        g = self.grid
        xn = np.ascontiguousarray(xn, dtype=np.float64)
        yn = np.ascontiguousarray(yn, dtype=np.float64)
        assert xn.shape == (g.ny + 5, g.nx + 5) and yn.shape == xn.shape
        self._nodes = (xn, yn)
        _check(self.L.orc_set_mapping(self.h, _dp(xn), _dp(yn)), "set_mapping")

    def metric(self):
        """the mapped grid's metric planes [7][ny + 4][nx + 4] (frame
        indices): capacity; unit normal (x, y) and length ratio of each
        cell's left edge; the same for its bottom edge"""
        g = self.grid
        out = np.empty((7, g.ny + 4, g.nx + 4))
        _check(self.L.orc_metric(self.h, _dp(out)), "metric")
        return out

    def set_radial(self, on=True):
        """radially symmetric solutions (Appendix D): x is the radius and
        every step adds the geometric source terms"""
        _check(self.L.orc_set_radial(self.h, 1 if on else 0), "set_radial")

    def set_external_ghosts(self, on=True):
        self.L.orc_set_external_ghosts(self.h, 1 if on else 0)

    def update_phi_framed(self):
        _check(self.L.orc_update_phi_framed(self.h), "update_phi_framed")

    def boundary_flux(self):
        nx, ny = self.grid.nx, self.grid.ny
        K = np.empty((2 * ny + 2 * nx, 7))
        _check(self.L.orc_boundary_flux(self.h, _dp(K)), "boundary_flux")
        return K

    def gauge_eta(self, x, y):
        return self.L.orc_gauge_eta(self.h, float(x), float(y))

    def clipped_mass(self):
        return self.L.orc_clipped_mass(self.h)


def from_workload(w, extended=False) -> OracleGrid:
    g = OracleGrid(w.params, w.grid, extended=extended)
    g.set_bathymetry(w.b)
    g.set_state(w.q)
    if w.gauges is not None and len(w.gauges):
        g.set_gauges(w.gauges)
    return g


def riemann_x(params, qL, qR, bL, bR, c2L, c2R):
    """One x-edge f-wave solve: returns (waves[7,7], speeds[7], amdq, apdq,
    kind)."""
    p = _params(params)
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    waves = np.zeros((7, 7)); speeds = np.zeros(7)
    amdq = np.zeros(7); apdq = np.zeros(7)
    kind = ctypes.c_int(0)
    rc = lib().orc_riemann_x(ctypes.byref(p), _dp(qL), _dp(qR), bL, bR, c2L, c2R,
                             _dp(waves), _dp(speeds), _dp(amdq), _dp(apdq),
                             ctypes.byref(kind))
    _check(rc, "riemann_x")
    return waves, speeds, amdq, apdq, kind.value


def edge_dflux(params, direction, qL, qR, bL, bR, c2L, c2R):
    """A-dQ + A+dQ of one edge (direction 0: x, 1: y)."""
    p = _params(params)
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    df = np.zeros(7)
    rc = lib().orc_edge_dflux(ctypes.byref(p), int(direction), _dp(qL), _dp(qR), float(bL),
                              float(bR), float(c2L), float(c2R), _dp(df))
    _check(rc, "edge_dflux")
    return df


def source_cell(q, c2, tau, model=0):
    q = np.array(q, dtype=np.float64)
    (lib().orc_source_cell_mb if model == 1 else lib().orc_source_cell)(_dp(q), c2, tau)
    return q


def limiter_phi(lim, theta):
    """the oracle's limiter function phi(theta)"""
    return lib().orc_limiter_phi(int(lim), float(theta))


def source_cells(q, c2, tau, model=0):
    """source_cell over cells: q[n][7] (a copy is returned), c2[n]"""
    q = np.array(q, dtype=np.float64, order="C")
    c2 = np.ascontiguousarray(c2, dtype=np.float64)
    lib().orc_source_cells(int(q.shape[0]), _dp(q), _dp(c2), float(tau), int(model))
    return q


def edge_dflux_n(params, direction, qL, qR, bL, bR, c2L, c2R):
    """edge_dflux over edges: qL, qR [n][7], the rest [n]; returns [n][7]"""
    p = _params(params)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (qL, qR, bL, bR, c2L, c2R)]
    df = np.zeros((a[0].shape[0], 7))
    rc = lib().orc_edge_dflux_n(ctypes.byref(p), int(direction), int(a[0].shape[0]),
                                *[_dp(x) for x in a], _dp(df))
    _check(rc, "edge_dflux_n")
    return df


def edge_dflux_mapped_n(params, direction, qL, qR, bL, bR, c2L, c2R, nx, ny, gm):
    """edge_dflux over mapped edges of unit normals (nx, ny) and length
    ratios gm (direction 0: left edges, 1: bottom edges), in the global
    frame; returns [n][7]"""
    p = _params(params)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (qL, qR, bL, bR, c2L, c2R, nx, ny, gm)]
    df = np.zeros((a[0].shape[0], 7))
    rc = lib().orc_edge_dflux_mapped_n(ctypes.byref(p), int(direction), int(a[0].shape[0]),
                                       *[_dp(x) for x in a], _dp(df))
    _check(rc, "edge_dflux_mapped_n")
    return df
