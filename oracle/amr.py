"""Static AMR patch sets advanced by the FP64 oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests and the smoke check.  The
GPU library never imports it.

The paper's solver runs the wave-propagation scheme on block-structured
adaptive grids (Sec. 4, which cites the wave-propagation AMR of Berger and
LeVeque and GeoClaw).  The paper gives no detail of the AMR rules; this file
states the rules the library implements, in the plainest form, on top of the
single-patch oracle step:

* Levels l = 0..L-1 with refinement ratio 4 in space and in time.  Level-0
  patches tile the domain; a level-l patch is aligned to level-(l-1) cells,
  has sides that are multiples of 4, lies at least one level-(l-1) cell away
  from the domain boundary and inside the union of level-(l-1) patches with
  one level-(l-1) cell to spare (proper nesting).
* Ghost cells (2 layers) of a level-l patch come, in this order of
  preference, from (a) the level-l patch covering the ghost cell (copy),
  (b) for level 0, the domain boundary condition applied to the domain cell
  it maps onto (periodic, wall with the normal momentum negated,
  extrapolation), (c) the level-(l-1) solution: time-interpolated linearly
  between the coarse old and new states, then linear in space with
  minmod-limited slopes of (eta', hu, hv, hw, h sigma, hp, h p_b), where
  eta' = h + b - eta0; slopes are zero in a direction with a missing
  neighbour and in all directions when a stencil cell is dry.  The ghost's
  bathymetry is the coarse cell's, its depth (eta' + eta0 - b)^+, its mask
  bits the coarse cell's current ones.
* One level-l step of size dt_l: fill ghosts, step every patch, then (if a
  finer level exists) 4 recursive level-(l+1) steps at time fractions
  s/4, s = 0..3, then refluxing and averaging down.
* Refluxing.  A coarse cell C next to a finer patch drops, in its own step,
  everything that reaches it through that edge (normal fluctuation,
  limited correction and transverse correction).  The finer patch records,
  per boundary edge and substep, the flux through the edge minus the flux
  function of C's state: its own boundary contribution (orc_boundary_flux)
  plus the total fluctuation between C* and the ghost g* (both after the
  first source half step of their own level), orc_edge_dflux(C*, g*) on the
  low sides and -orc_edge_dflux(g*, C*) on the high sides.  After the
  substeps C receives -/+ dt_l/dx_l times the mean of the 4 x 4 fine
  records over its edge, then the cell fix-ups (clipping with mass
  bookkeeping, dry cells, SWE auxiliaries).  This keeps the mass exact.
* Averaging down: a covered coarse cell takes the mean of its 4 x 4 fine
  cells, all seven variables (plane 0 being h); the coarse bathymetry of
  covered cells is the mean of the fine bathymetry (set once).
* Gauges record after each level-0 step from the finest patch containing
  the point; the mass is the level-0 sum.

Mapped patch sets (Sec. 4, mapped grids, on block-structured grids).  Every
patch carries the node coordinates of its frame; a finer patch's nodes are
the bilinear refinement of the coarser level's (so that its cells tile each
coarse cell exactly, with straight edges: the fine areas sum to the coarse
area, and the fine edges along a coarse edge to its length, with its
normal).  Each patch steps as a mapped grid.  On top of the rules above:
* ghost interpolation stays in computational (index) space; the momenta
  are in the physical frame;
* a level-0 wall ghost mirrors the momentum about the wall edge's unit
  normal n (m - 2 (m . n) n), the edge being the domain edge of the
  interior cell's row (x walls) or column (y walls), as on a single grid;
* the boundary-flux records take the fine step's mapped contributions
  (global frame, scaled by the edge's length ratio) and the total
  fluctuation between C* and g* solved in the fine edge's frame and scaled
  by its length ratio;
* refluxing divides by the coarse cell's capacity (dt/dx over kap), the
  clipped mass counts kap dx dy;
* averaging down weighs the 4 x 4 fine cells by their capacities:
  sum(kap q) / sum(kap), both sums in row order; the bathymetry likewise;
* the mass is the level-0 sum of kap h dx dy.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

RATIO = 4


def _map_index(i, n, lo, hi):
    """index of a ghost cell after the domain boundary condition; flip = 1
    when the normal momentum changes sign (wall)"""
    if i < 0:
        if lo == 0:
            return i + n, 0
        if lo == 1:
            return -1 - i, 1
        return 0, 0
    if i >= n:
        if hi == 0:
            return i - n, 0
        if hi == 1:
            return 2 * n - 1 - i, 1
        return n - 1, 0
    return i, 0


def _minmod(a, b):
    if a > 0.0 and b > 0.0:
        return a if a <= b else b
    if a < 0.0 and b < 0.0:
        return a if a >= b else b
    return 0.0


def _minmod_arrays(a, b):
    """_minmod element by element"""
    return np.where((a > 0.0) & (b > 0.0), np.where(a <= b, a, b),
                    np.where((a < 0.0) & (b < 0.0), np.where(a >= b, a, b), 0.0))


class _Patch:
    def __init__(self, pid, level, nx, ny, x0, y0, dx, dy, I0, J0, grid):
        self.pid, self.level, self.nx, self.ny = pid, level, nx, ny
        self.x0, self.y0, self.dx, self.dy = x0, y0, dx, dy
        self.I0, self.J0 = I0, J0
        self.g = grid
        self.q, self.b, self.phi, self.brk, self.iface = grid.framed()
        self.b_raw = None          # bathymetry as set, before averaging down
        self.met = None            # metric planes [7][ny + 4][nx + 4] (mapped)

    def contains(self, I, J):
        return self.I0 <= I < self.I0 + self.nx and self.J0 <= J < self.J0 + self.ny


class _GridSpec:
    def __init__(self, nx, ny, x0, y0, dx, dy, bc):
        self.nx, self.ny, self.x0, self.y0, self.dx, self.dy, self.bc = nx, ny, x0, y0, dx, dy, bc


class AmrOracle:
    """One scenario: a static patch set advanced with fixed level-0 steps."""

    def __init__(self, params, dx0, dy0, bc, patches, reflux=True, capacity=True):
        """patches: sequence of (level, nx, ny, x0, y0).  reflux=False leaves
        the refluxing out, capacity=False the capacities out of refluxing and
        averaging down on mapped patch sets (deliberately wrong variants for
        the tests that show the conservation check notices them)."""
        self.P = params
        self.do_reflux = reflux
        self.use_capacity = capacity
        self.bc = list(bc)
        self.dx0, self.dy0 = dx0, dy0
        self.levels = []
        self.patches = []
        lv0 = [p for p in patches if p[0] == 0]
        X0 = min(p[3] for p in lv0)
        Y0 = min(p[4] for p in lv0)
        self.X0, self.Y0 = X0, Y0
        for pid, (lev, nx, ny, x0, y0) in enumerate(patches):
            dx, dy = dx0 / RATIO ** lev, dy0 / RATIO ** lev
            I0 = int(round((x0 - X0) / dx))
            J0 = int(round((y0 - Y0) / dy))
            g = O.OracleGrid(params, _GridSpec(nx, ny, x0, y0, dx, dy, self.bc))
            g.set_external_ghosts(True)
            p = _Patch(pid, lev, nx, ny, x0, y0, dx, dy, I0, J0, g)
            self.patches.append(p)
            while len(self.levels) <= lev:
                self.levels.append([])
            self.levels[lev].append(p)
        self.NX = max(p.I0 + p.nx for p in self.levels[0])
        self.NY = max(p.J0 + p.ny for p in self.levels[0])
        self.t = 0.0
        self.steps = 0
        self.gauges = np.zeros((0, 2))
        self.records_t, self.records = [], []
        self.clip = 0.0
        self.prepared = False
        self.old = {}

    def set_sponge(self, width, rate):
        """sponge widths (m) from the x-low, x-high, y-low, y-high sides of
        the level-0 domain and peak rate (1/s), on every patch (its place in
        the domain of its level)"""
        for p in self.patches:
            r = RATIO ** p.level
            p.g.set_sponge(width, rate, offset=(p.I0, p.J0), domain=(self.NX * r, self.NY * r))

    # -------------------------------------------------------------- lookup
    _BUCKET = 16

    def find(self, level, I, J):
        """the patch of `level` containing level cell (I, J), or None; the
        patches are looked up through 16 x 16-cell buckets of the level's
        index space (each bucket lists the patches that overlap it, in
        patch order)"""
        idx = self.__dict__.setdefault("_index", {})
        lp = self.levels[level]
        ent = idx.get(level)
        if ent is None or ent[0] != len(lp):
            B = self._BUCKET
            table = {}
            for p in lp:
                for bj in range(p.J0 // B, (p.J0 + p.ny - 1) // B + 1):
                    for bi in range(p.I0 // B, (p.I0 + p.nx - 1) // B + 1):
                        table.setdefault((bi, bj), []).append(p)
            ent = idx[level] = (len(lp), table)
        for p in ent[1].get((I // self._BUCKET, J // self._BUCKET), ()):
            if p.contains(I, J):
                return p
        return None

    # ------------------------------------------------------------ data in/out
    def set_bathymetry(self, pid, b):
        p = self.patches[pid]
        p.b_raw = np.array(b, dtype=np.float64).reshape(p.ny, p.nx)
        p.b[2:-2, 2:-2] = p.b_raw
        self.prepared = False

    def set_state(self, pid, q):
        p = self.patches[pid]
        p.q[:, 2:-2, 2:-2] = np.asarray(q, dtype=np.float64)

    def get_state(self, pid):
        return self.patches[pid].q[:, 2:-2, 2:-2].copy()

    def get_mask(self, pid):
        p = self.patches[pid]
        return (p.phi[2:-2, 2:-2] | (p.brk[2:-2, 2:-2] << 1)).astype(np.uint8)

    def set_gauges(self, xy):
        self.gauges = np.asarray(xy, dtype=np.float64).reshape(-1, 2)

    def set_mapping(self, pid, xn, yn):
        """node coordinates [ny + 5][nx + 5] of patch pid (nodes i = -2..nx+2,
        j = -2..ny+2, the ghost frame included); every patch of the set is
        mapped before the first step, or none"""
        p = self.patches[pid]
        p.g.set_mapping(xn, yn)
        p.met = p.g.metric()
        self.prepared = False

    @property
    def mapped(self):
        return any(p.met is not None for p in self.patches)

    # --------------------------------------------------------------- set-up
    def prepare(self):
        """bathymetry of covered coarse cells, ghost bathymetry, phi_T and
        the interface flags"""
        if self.mapped and any(p.met is None for p in self.patches):
            raise ValueError("a patch set is mapped in every patch or in none")
        # coarse bathymetry of covered cells := mean of the fine bathymetry,
        # finest level first
        for lev in range(len(self.levels) - 1, 0, -1):
            for f in self.levels[lev]:
                self._average_down_patch(f, bath_only=True)
        for lev in range(len(self.levels)):
            for p in self.levels[lev]:
                self._fill_ghost_bathymetry(p)
        for p in self.patches:
            p.g.update_phi_framed()
        # interface flags of uncovered cells next to a finer patch: a
        # level-lev cell (I, J) is covered when the finer cell (4 I, 4 J)
        # lies in a level-(lev+1) patch; the coverage of each patch and a
        # one-cell rim is painted from the finer patches
        for lev in range(len(self.levels) - 1):
            for p in self.levels[lev]:
                p.iface[:] = 0
                cov = np.zeros((p.ny + 2, p.nx + 2), dtype=bool)    # cells I0-1 .. I0+nx
                for f in self.levels[lev + 1]:
                    # I covered by f iff f.I0 <= 4 I < f.I0 + f.nx
                    i0 = max(-(-f.I0 // RATIO), p.I0 - 1)
                    i1 = min(-(-(f.I0 + f.nx) // RATIO), p.I0 + p.nx + 1)
                    j0 = max(-(-f.J0 // RATIO), p.J0 - 1)
                    j1 = min(-(-(f.J0 + f.ny) // RATIO), p.J0 + p.ny + 1)
                    if i0 < i1 and j0 < j1:
                        cov[j0 - p.J0 + 1:j1 - p.J0 + 1, i0 - p.I0 + 1:i1 - p.I0 + 1] = True
                c = cov[1:-1, 1:-1]
                bits = (cov[1:-1, :-2] * 1) | (cov[1:-1, 2:] * 2) | (cov[:-2, 1:-1] * 4) | (cov[2:, 1:-1] * 8)
                p.iface[2:-2, 2:-2] = np.where(c, 0, bits).astype(np.uint8)
        self.prepared = True

    def _ghost_cells(self, p):
        for j in range(-2, p.ny + 2):
            for i in range(-2, p.nx + 2):
                if 0 <= i < p.nx and 0 <= j < p.ny:
                    continue
                yield i, j

    def _source_of(self, p, i, j):
        """('copy', src patch, si, sj, flip_u, flip_v, wi, wj) or ('coarse',
        I, J, ox, oy); wi (wj) is the source-local column (row) of the cell
        whose left (bottom) edge is the domain wall of an x (y) flip"""
        I, J = p.I0 + i, p.J0 + j
        if p.level == 0:
            mi, fx = _map_index(I, self.NX, self.bc[0], self.bc[1])
            mj, fy = _map_index(J, self.NY, self.bc[2], self.bc[3])
            s = self.find(0, mi, mj)
            wi = (0 if I < 0 else self.NX) - s.I0
            wj = (0 if J < 0 else self.NY) - s.J0
            return ("copy", s, mi - s.I0, mj - s.J0, fx, fy, wi, wj)
        s = self.find(p.level, I, J)
        if s is not None:
            return ("copy", s, I - s.I0, J - s.J0, 0, 0, 0, 0)
        Ic, Jc = I // RATIO, J // RATIO
        ox = ((I - RATIO * Ic) + 0.5) / RATIO - 0.5
        oy = ((J - RATIO * Jc) + 0.5) / RATIO - 0.5
        return ("coarse", Ic, Jc, ox, oy)

    def _ghost_tables(self, p):
        """the ghost sources of patch p (static for the patch set), as
        arrays in frame indices: copies grouped by source patch
        (dj, di, sj, si, fx, fy, wi, wj), and the coarse ghosts (dj, di, ox, oy)
        with, for the coarse centre and its left, right, lower and upper
        neighbours, the coarse patch id (-1: none) and frame indices"""
        tabs = self.__dict__.setdefault("_gtab", {})
        if p.pid in tabs:
            return tabs[p.pid]
        copies = {}
        co = {"dj": [], "di": [], "ox": [], "oy": [], "pid": [[] for _ in range(5)],
              "cj": [[] for _ in range(5)], "ci": [[] for _ in range(5)]}
        for i, j in self._ghost_cells(p):
            src = self._source_of(p, i, j)
            if src[0] == "copy":
                _, sp, si, sj, fx, fy, wi, wj = src
                c = copies.setdefault(sp.pid, ([], [], [], [], [], [], [], []))
                for lst, v in zip(c, (j + 2, i + 2, sj + 2, si + 2, fx, fy, wi + 2, wj + 2)):
                    lst.append(v)
                continue
            _, Ic, Jc, ox, oy = src
            co["dj"].append(j + 2)
            co["di"].append(i + 2)
            co["ox"].append(ox)
            co["oy"].append(oy)
            for k, (di, dj) in enumerate(((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))):
                c = self.find(p.level - 1, Ic + di, Jc + dj)
                co["pid"][k].append(c.pid if c is not None else -1)
                co["cj"][k].append(Jc + dj - c.J0 + 2 if c is not None else 0)
                co["ci"][k].append(Ic + di - c.I0 + 2 if c is not None else 0)
        ct = {sp: tuple(np.array(a, dtype=np.int64) for a in c[:4]) +
              tuple(np.array(a, dtype=bool) for a in c[4:6]) +
              tuple(np.array(a, dtype=np.int64) for a in c[6:]) for sp, c in copies.items()}
        cc = {"dj": np.array(co["dj"], dtype=np.int64), "di": np.array(co["di"], dtype=np.int64),
              "ox": np.array(co["ox"], dtype=np.float64), "oy": np.array(co["oy"], dtype=np.float64),
              "pid": [np.array(a, dtype=np.int64) for a in co["pid"]],
              "cj": [np.array(a, dtype=np.int64) for a in co["cj"]],
              "ci": [np.array(a, dtype=np.int64) for a in co["ci"]]}
        tabs[p.pid] = (ct, cc)
        return tabs[p.pid]

    def _gather(self, arrays, pid, j, i):
        """values of arrays[pid][..., j, i] for every entry (pid >= 0; the
        others stay 0)"""
        lead = next(iter(arrays.values())).shape[:-2]
        out = np.zeros(lead + pid.shape)
        for u in np.unique(pid[pid >= 0]):
            k = pid == u
            out[..., k] = arrays[int(u)][..., j[k], i[k]]
        return out

    def _fill_ghost_bathymetry(self, p):
        ct, cc = self._ghost_tables(p)
        for sp, (dj, di, sj, si, _, _, _, _) in ct.items():
            p.b[dj, di] = self.patches[sp].b[sj, si]
        if len(cc["dj"]):
            bs = {c.pid: c.b for c in self.levels[p.level - 1]}
            p.b[cc["dj"], cc["di"]] = self._gather(bs, cc["pid"][0], cc["cj"][0], cc["ci"][0])

    # ---------------------------------------------------------------- ghosts
    def fill_ghosts(self, lev, theta):
        """every ghost cell of the level's patches by the rules above (the
        same arithmetic per cell, evaluated over arrays of ghost cells)"""
        eta0, dtol = self.P.eta0, self.P.dry_tol
        coarse = self.levels[lev - 1] if lev > 0 else []
        old = {c.pid: self.old[c.pid] for c in coarse}
        new = {c.pid: c.q for c in coarse}
        bath = {c.pid: c.b for c in coarse}
        phi = {c.pid: c.phi for c in coarse}
        brk = {c.pid: c.brk for c in coarse}
        for p in self.levels[lev]:
            ct, cc = self._ghost_tables(p)
            for sp, (dj, di, sj, si, fx, fy, wi, wj) in ct.items():
                s = self.patches[sp]
                p.q[:, dj, di] = s.q[:, sj, si]
                if s.met is None:
                    p.q[1, dj[fx], di[fx]] = -p.q[1, dj[fx], di[fx]]
                    p.q[2, dj[fy], di[fy]] = -p.q[2, dj[fy], di[fy]]
                else:
                    # mirrored about the wall edge: x walls first, then y
                    for flip, (a, b), (mj, mi) in ((fx, (1, 2), (sj, wi)), (fy, (4, 5), (wj, si))):
                        if not flip.any():
                            continue
                        k = (dj[flip], di[flip])
                        nx_ = s.met[a][mj[flip], mi[flip]]
                        ny_ = s.met[b][mj[flip], mi[flip]]
                        hu, hv = p.q[1][k], p.q[2][k]
                        d = hu * nx_ + hv * ny_
                        p.q[1][k] = hu - 2.0 * d * nx_
                        p.q[2][k] = hv - 2.0 * d * ny_
                p.phi[dj, di] = s.phi[sj, si]
                p.brk[dj, di] = s.brk[sj, si]
            if not len(cc["dj"]):
                continue
            vals, dry, have = [], [], []
            for k in range(5):
                pid, cj, ci = cc["pid"][k], cc["cj"][k], cc["ci"][k]
                qo, qn = self._gather(old, pid, cj, ci), self._gather(new, pid, cj, ci)
                b = self._gather(bath, pid, cj, ci)
                vo, vn = qo.copy(), qn.copy()
                vo[0] = (qo[0] + b) - eta0
                vn[0] = (qn[0] + b) - eta0
                vals.append((1.0 - theta) * vo + theta * vn)
                dry.append(~(qo[0] > dtol) | ~(qn[0] > dtol))
                have.append(pid >= 0)
            v = vals[0]
            any_dry = dry[0].copy()
            for k in range(1, 5):
                any_dry |= have[k] & dry[k]
            sx = np.where(~any_dry & have[1] & have[2], _minmod_arrays(vals[2] - v, v - vals[1]), 0.0)
            sy = np.where(~any_dry & have[3] & have[4], _minmod_arrays(vals[4] - v, v - vals[3]), 0.0)
            out = (v + cc["ox"] * sx) + cc["oy"] * sy
            bg = p.b[cc["dj"], cc["di"]]
            h = (out[0] + eta0) - bg
            out[0] = np.where(h > 0.0, h, 0.0)
            p.q[:, cc["dj"], cc["di"]] = out
            p.phi[cc["dj"], cc["di"]] = self._gather(phi, cc["pid"][0], cc["cj"][0], cc["ci"][0])
            p.brk[cc["dj"], cc["di"]] = self._gather(brk, cc["pid"][0], cc["cj"][0], cc["ci"][0])

    # ------------------------------------------------------------ stepping
    def _flux_records(self, f):
        """boundary edges of fine patch f whose outside cell comes from the
        coarse level: (entry, direction, low_side, ghost (i, j))"""
        out = []
        for j in range(f.ny):
            out.append((j, 0, True, (-1, j)))
            out.append((f.ny + j, 0, False, (f.nx, j)))
        for i in range(f.nx):
            out.append((2 * f.ny + i, 1, True, (i, -1)))
            out.append((2 * f.ny + f.nx + i, 1, False, (i, f.ny)))
        return [r for r in out if self._source_of(f, *r[3])[0] == "coarse"]

    def _flux_table(self, f):
        """the flux records of fine patch f as arrays (static): entry,
        direction, low side, the ghost's frame indices, and the coarse cell
        C's patch and frame indices"""
        tabs = self.__dict__.setdefault("_ftab", {})
        if f.pid not in tabs:
            rows = []
            for e, direction, low, (gi, gj) in self._flux_records(f):
                _, Ic, Jc, _, _ = self._source_of(f, gi, gj)
                c = self.find(f.level - 1, Ic, Jc)
                rows.append((e, direction, int(low), gj + 2, gi + 2, c.pid, Jc - c.J0 + 2,
                             Ic - c.I0 + 2))
            tabs[f.pid] = np.array(rows, dtype=np.int64).reshape(-1, 8)
        return tabs[f.pid]

    def _pre_source_cells(self, q, b, phi, brk, tau):
        """_pre_source over cells: q[7][n], b, phi, brk [n]"""
        q = np.array(q, dtype=np.float64)
        swe = (phi == 0) | (brk != 0)
        wet = q[0] > self.P.dry_tol
        if self.P.splitting:
            src = wet & ~swe
            if src.any():
                q[:, src] = O.source_cells(q[:, src].T, self._c2_cells(b[src], phi[src], brk[src]),
                                           tau, getattr(self.P, "model", 0)).T
            q[3:, ~src] = 0.0
        else:
            q[3:, ~wet | swe] = 0.0
        return q

    def _c2_cells(self, b, phi, brk):
        """_c2 over cells"""
        swe = (phi == 0) | (brk != 0)
        if getattr(self.P, "c2", 0.0) > 0.0:
            return np.where(swe, 0.0, self.P.c2)
        H = self.P.eta0 - b
        H = np.where(H > 0.0, H, 0.0)
        return np.where(swe, 0.0, self.P.alpha * self.P.alpha * self.P.g * H)

    def _accumulate_fluxes(self, lev, dt_f, dt_c):
        """after a level-lev substep: R += K + (+/-) dflux(C*, g*)"""
        for f in self.levels[lev]:
            T = self._flux_table(f)
            if not len(T):
                continue
            K = f.g.boundary_flux()
            e, direction, low = T[:, 0], T[:, 1], T[:, 2] == 1
            gj, gi = T[:, 3], T[:, 4]
            cp, cj, ci = T[:, 5], T[:, 6], T[:, 7]
            qo = self._gather(self.old, cp, cj, ci)
            bC = self._gather({c.pid: c.b for c in self.levels[lev - 1]}, cp, cj, ci)
            phC = self._gather(self.old_phi, cp, cj, ci)
            bkC = self._gather(self.old_brk, cp, cj, ci)
            qC = self._pre_source_cells(qo, bC, phC, bkC, 0.5 * dt_c)
            c2C = self._c2_cells(bC, phC, bkC)
            qg_raw = self.old[f.pid][:, gj, gi]
            bg = f.b[gj, gi]
            pg, kg = self.old_phi[f.pid][gj, gi], self.old_brk[f.pid][gj, gi]
            qg = self._pre_source_cells(qg_raw, bg, pg, kg, 0.5 * dt_f)
            c2g = self._c2_cells(bg, pg, kg)
            D = np.zeros((len(T), 7))
            for d in (0, 1):
                for lo in (True, False):
                    k = (direction == d) & (low == lo)
                    if not k.any():
                        continue
                    a, b = (qC[:, k].T, qg[:, k].T) if lo else (qg[:, k].T, qC[:, k].T)
                    ba, bb = (bC[k], bg[k]) if lo else (bg[k], bC[k])
                    ca, cb = (c2C[k], c2g[k]) if lo else (c2g[k], c2C[k])
                    if f.met is None:
                        df = O.edge_dflux_n(self.P, d, a, b, ba, bb, ca, cb)
                    else:
                        # the fine edge: the left (bottom) edge of the cell
                        # right of (above) the ghost on a low side, of the
                        # ghost itself on a high side
                        ej = gj[k] + (1 if (lo and d == 1) else 0)
                        ei = gi[k] + (1 if (lo and d == 0) else 0)
                        pl = (1, 2, 3) if d == 0 else (4, 5, 6)
                        df = O.edge_dflux_mapped_n(self.P, d, a, b, ba, bb, ca, cb,
                                                   f.met[pl[0]][ej, ei], f.met[pl[1]][ej, ei],
                                                   f.met[pl[2]][ej, ei])
                    D[k] = df if lo else -df
            R = self.R[f.pid]
            R[e] = R[e] + (K[e] + D)

    def _reflux(self, lev, dt_c):
        for p in self.levels[lev]:
            dtdx, dtdy = dt_c / p.dx, dt_c / p.dy
            for j in range(p.ny):
                for i in range(p.nx):
                    fl = int(p.iface[j + 2, i + 2])
                    if not fl:
                        continue
                    I, J = p.I0 + i, p.J0 + j
                    v = p.q[:, j + 2, i + 2].copy()
                    # mapped: the records are fluxes times length ratios, the
                    # update divides them by the cell's capacity
                    kap = p.met[0, j + 2, i + 2] if (p.met is not None and self.use_capacity) \
                        else None
                    for bit in range(4):
                        if not fl & (1 << bit):
                            continue
                        if bit == 0:     # finer patch on the left: its right side
                            f = self.find(lev + 1, RATIO * I - 1, RATIO * J)
                            e0, sgn, dtd = f.ny + (RATIO * J - f.J0), 1.0, dtdx
                        elif bit == 1:   # on the right: its left side
                            f = self.find(lev + 1, RATIO * I + RATIO, RATIO * J)
                            e0, sgn, dtd = RATIO * J - f.J0, -1.0, dtdx
                        elif bit == 2:   # below: its top side
                            f = self.find(lev + 1, RATIO * I, RATIO * J - 1)
                            e0, sgn, dtd = 2 * f.ny + f.nx + (RATIO * I - f.I0), 1.0, dtdy
                        else:            # above: its bottom side
                            f = self.find(lev + 1, RATIO * I, RATIO * J + RATIO)
                            e0, sgn, dtd = 2 * f.ny + (RATIO * I - f.I0), -1.0, dtdy
                        Rf = self.R[f.pid]
                        S = ((Rf[e0] + Rf[e0 + 1]) + Rf[e0 + 2]) + Rf[e0 + 3]
                        if kap is not None:
                            dtd = dtd / kap
                        corr = dtd * (S * 0.0625)
                        v = v + corr if sgn > 0 else v - corr
                    # cell fix-ups
                    if v[0] < 0.0:
                        if kap is not None:
                            self.clip += -v[0] * kap * p.dx * p.dy
                        else:
                            self.clip += -v[0] * p.dx * p.dy
                        v[0] = 0.0
                    if v[0] <= self.P.dry_tol:
                        v[1:] = 0.0
                    if (not p.phi[j + 2, i + 2]) or p.brk[j + 2, i + 2] or v[0] <= self.P.dry_tol:
                        v[3:] = 0.0
                    p.q[:, j + 2, i + 2] = v

    def _average_down_patch(self, f, bath_only=False):
        """covered coarse cells take the mean of their 4 x 4 fine cells: the
        16 values summed in row order (a fine row, then the next), times
        1/16; on a mapped patch set sum(kap q) / sum(kap) over the same
        cells in the same order; the bathymetry alone with bath_only"""
        lev = f.level
        nbx, nby = f.nx // RATIO, f.ny // RATIO
        src = f.b[None] if bath_only else f.q
        s = np.zeros((src.shape[0], nby, nbx))
        weighted = f.met is not None and self.use_capacity
        w = np.zeros((nby, nbx))
        for a in range(RATIO):
            for bb in range(RATIO):
                sl = (slice(2 + a, 2 + a + RATIO * nby, RATIO), slice(2 + bb, 2 + bb + RATIO * nbx, RATIO))
                if weighted:
                    k = f.met[0][sl]
                    s = s + k * src[(slice(None),) + sl]
                    w = w + k
                else:
                    s = s + src[(slice(None),) + sl]
        mean = s / w if weighted else s * 0.0625
        Ic0, Jc0 = f.I0 // RATIO, f.J0 // RATIO
        for c in self.levels[lev - 1]:
            i0, i1 = max(Ic0, c.I0), min(Ic0 + nbx, c.I0 + c.nx)
            j0, j1 = max(Jc0, c.J0), min(Jc0 + nby, c.J0 + c.ny)
            if i0 >= i1 or j0 >= j1:
                continue
            blk = mean[:, j0 - Jc0:j1 - Jc0, i0 - Ic0:i1 - Ic0]
            if bath_only:
                c.b[j0 - c.J0 + 2:j1 - c.J0 + 2, i0 - c.I0 + 2:i1 - c.I0 + 2] = blk[0]
            else:
                c.q[:, j0 - c.J0 + 2:j1 - c.J0 + 2, i0 - c.I0 + 2:i1 - c.I0 + 2] = blk

    def _step_level(self, lev, dt, theta):
        self.fill_ghosts(lev, theta)
        for p in self.levels[lev]:
            self.old[p.pid] = p.q.copy()
            self.old_phi[p.pid] = p.phi.copy()
            self.old_brk[p.pid] = p.brk.copy()
        clip0 = [p.g.clipped_mass() for p in self.levels[lev]]
        for p in self.levels[lev]:
            courant = p.g.step(dt)
            if courant > self.P.cfl_max:
                raise O.OracleError(O.ECFL, "amr step (level %d)" % lev)
        self.clip += sum(p.g.clipped_mass() - c0 for p, c0 in zip(self.levels[lev], clip0))
        if lev + 1 < len(self.levels):
            dt_f = dt / RATIO
            for f in self.levels[lev + 1]:
                self.R[f.pid] = np.zeros((2 * f.ny + 2 * f.nx, 7))
            for s in range(RATIO):
                self._step_level(lev + 1, dt_f, s / RATIO)
                self._accumulate_fluxes(lev + 1, dt_f, dt)
            if self.do_reflux:
                self._reflux(lev, dt)
            for f in self.levels[lev + 1]:
                self._average_down_patch(f)

    def step(self, dt):
        """one level-0 step of size dt (with all finer substeps)"""
        if not self.prepared:
            self.prepare()
        self.old_phi, self.old_brk, self.R = {}, {}, {}
        self._step_level(0, dt, 0.0)
        self.t += dt
        self.steps += 1
        if len(self.gauges):
            self.records_t.append(self.t)
            self.records.append([self.gauge_eta(x, y) for x, y in self.gauges])

    def advance(self, dt, n):
        for _ in range(n):
            self.step(dt)

    def gauge_eta(self, x, y):
        for lev in range(len(self.levels) - 1, -1, -1):
            for p in self.levels[lev]:
                if p.x0 <= x <= p.x0 + p.nx * p.dx and p.y0 <= y <= p.y0 + p.ny * p.dy:
                    return p.g.gauge_eta(x, y)
        raise ValueError("gauge outside the domain")

    def read_gauges(self):
        t = np.array(self.records_t)
        e = np.array(self.records).reshape(len(self.records_t), len(self.gauges))
        self.records_t, self.records = [], []
        return t, e

    def mass(self):
        """level-0 sum of h dx dy (kap h dx dy on a mapped patch set)"""
        if self.mapped:
            return sum(float((p.met[0, 2:-2, 2:-2] * p.q[0, 2:-2, 2:-2]).sum()) * p.dx * p.dy
                       for p in self.levels[0])
        return sum(float(p.q[0, 2:-2, 2:-2].sum()) * p.dx * p.dy for p in self.levels[0])


def from_workload(w, reflux=True, capacity=True, nodes=None) -> AmrOracle:
    """an AmrOracle from an AMR workload (paper_2606_12162_amd.workloads);
    nodes: per patch (xn, yn) of a mapped patch set"""
    o = AmrOracle(w.params, w.dx0, w.dy0, w.bc, [(p.level, p.nx, p.ny, p.x0, p.y0)
                                                  for p in w.patches], reflux=reflux,
                  capacity=capacity)
    if nodes is not None:
        for pid, (xn, yn) in enumerate(nodes):
            o.set_mapping(pid, xn, yn)
    for pid, p in enumerate(w.patches):
        o.set_bathymetry(pid, p.b)
        o.set_state(pid, p.q)
    if w.gauges is not None and len(w.gauges):
        o.set_gauges(w.gauges)
    return o
