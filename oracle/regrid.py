"""Regridding of a patch set by the oracle (adaptive refinement, Sec. 4).

TEST INFRASTRUCTURE ONLY: imported by the tests.  The GPU library never
imports it.

The paper runs the Berger-Oliger-Colella algorithm (Sec. 4): cells are
flagged by a surface-jump criterion (as in the solitary-wave test of Sec. 5:
the surface differs between neighbouring cells by more than a tolerance),
flagged cells are clustered into rectangles (Berger-Rigoutsos), and the
rectangles become the patches of the next finer level.  The paper gives no
further detail; these are the rules the library implements, in plain form.
One call rebuilds level l+1 from flags on level l; deeper levels are
dropped (the caller regrids them next, level by level).

  1. Flags (level-l patch, interior cells).  With eta' = (h + b) - eta0, a
     pair of face neighbours inside the patch, both wet (h > dry_tol),
     whose eta' differ by more than tol flags both cells.
  2. Buffer: a cell within nbuf cells (max norm, inside the patch) of a
     flagged cell is flagged.
  3. Clusters, per level-l patch (Berger-Rigoutsos).  A box is shrunk to
     the bounding box of its flags.  If its flagged fraction is at least
     `cutoff` it is accepted, after halving its longer side (x on ties)
     until both sides are at most `max_side` cells.  Otherwise it is split:
     (a) at an empty column or row of the flag signatures, the one nearest
     the middle of its side (ties: x first, then the lower index), the box
     going to [lo, k) and [k, hi); else (b) at the strongest sign change of
     the signature's second difference L_k = S_(k-1) - 2 S_k + S_(k+1),
     between k and k+1, strength |L_(k+1) - L_k| (ties: nearest the middle,
     x first, lower index), sides of at least 4 cells only; else (c) at the
     middle of the longer side (x on ties).  Halves are processed low first.
  4. Nesting: a box is clipped to its patch less one cell on every side and
     dropped if empty; the new level-(l+1) patch is the box refined by 4.
  5. Bathymetry of a new patch: the bilinear interpolant of the level-0
     bathymetry as set (before averaging down), at the cell centre in
     level-0 index coordinates fx = (I + 1/2) / 4^l - 1/2 (exact in binary),
     i = floor(fx) clamped to [0, NX - 2], t = fx - i clamped to [0, 1];
     b = (b00 (1 - t) + b10 t) (1 - s) + (b01 (1 - t) + b11 t) s.  Patches
     kept from before keep the bathymetry they were given.  Covered coarse
     cells then take the mean of their fine cells, as for static sets.
  6. State.  Kept patches (levels <= l) keep their state; where a cell's
     bathymetry changed (covered or uncovered anew), a wet cell keeps its
     surface, h = max(h + (b_old - b_new), 0), and a dry cell keeps h.  A new
     level-(l+1) cell takes the ghost rule's spatial interpolation from its
     coarse cell (minmod-linear in eta', hu, ..., h p_b; zero slopes when a
     stencil cell is dry; h = max(eta' + eta0 - b, 0) with its own b) and its
     coarse cell's breaking latch; where an old level-(l+1) patch covered
     the cell, its old state and latch are copied instead (with the same
     depth rule if b changed).
  7. Clock, gauges (recorded series included) and clipped mass carry over.
"""
from __future__ import annotations

import math

import numpy as np

from . import amr as A

RATIO = A.RATIO


def flag_patch(o, p, tol):
    """step 1 on patch p: boolean flags [ny, nx]"""
    q, b = p.q[:, 2:-2, 2:-2], p.b[2:-2, 2:-2]
    h = q[0]
    eta = (h + b) - o.P.eta0
    wet = h > o.P.dry_tol
    F = np.zeros((p.ny, p.nx), dtype=bool)
    hx = wet[:, :-1] & wet[:, 1:] & (np.abs(eta[:, 1:] - eta[:, :-1]) > tol)
    F[:, :-1] |= hx
    F[:, 1:] |= hx
    vy = wet[:-1, :] & wet[1:, :] & (np.abs(eta[1:, :] - eta[:-1, :]) > tol)
    F[:-1, :] |= vy
    F[1:, :] |= vy
    return F


def buffer_flags(F, nbuf):
    """step 2: dilation by nbuf cells (max norm) inside the patch"""
    ny, nx = F.shape
    out = F.copy()
    for dj in range(-nbuf, nbuf + 1):
        for di in range(-nbuf, nbuf + 1):
            src = F[max(0, -dj):ny - max(0, dj), max(0, -di):nx - max(0, di)]
            out[max(0, dj):ny - max(0, -dj), max(0, di):nx - max(0, -di)] |= src
    return out


def cluster(F, cutoff, max_side):
    """step 3: boxes (i0, i1, j0, j1), half-open, in patch cells"""
    out = []

    def rec(i0, i1, j0, j1):
        sub = F[j0:j1, i0:i1]
        if not sub.any():
            return
        cols = np.nonzero(sub.any(axis=0))[0]
        rows = np.nonzero(sub.any(axis=1))[0]
        i0, i1 = i0 + int(cols[0]), i0 + int(cols[-1]) + 1
        j0, j1 = j0 + int(rows[0]), j0 + int(rows[-1]) + 1
        sub = F[j0:j1, i0:i1]
        nx, ny = i1 - i0, j1 - j0
        n = int(sub.sum())
        cut = None
        if n >= cutoff * (nx * ny):
            if nx <= max_side and ny <= max_side:
                out.append((i0, i1, j0, j1))
                return
            cut = (0, nx // 2) if nx >= ny else (1, ny // 2)
        else:
            S = (sub.sum(axis=0).astype(np.int64), sub.sum(axis=1).astype(np.int64))
            Ls = (nx, ny)
            best = None
            for dim in (0, 1):
                for k in range(1, Ls[dim] - 1):
                    if S[dim][k] == 0:
                        key = (abs(2 * k - (Ls[dim] - 1)), dim, k)
                        if best is None or key < best:
                            best, cut = key, (dim, k)
            if cut is None:
                best = None
                for dim in (0, 1):
                    Ld, Sd = Ls[dim], S[dim]
                    if Ld < 4:
                        continue
                    lap = [int(Sd[k - 1] - 2 * Sd[k] + Sd[k + 1]) for k in range(1, Ld - 1)]
                    for k in range(1, Ld - 2):
                        a, b = lap[k - 1], lap[k]          # L_k and L_(k+1)
                        if a * b < 0:
                            key = (-abs(b - a), abs(2 * (k + 1) - Ld), dim, k)
                            if best is None or key < best:
                                best, cut = key, (dim, k + 1)
            if cut is None:
                cut = (0, nx // 2) if nx >= ny else (1, ny // 2)
        dim, k = cut
        if dim == 0:
            rec(i0, i0 + k, j0, j1)
            rec(i0 + k, i1, j0, j1)
        else:
            rec(i0, i1, j0, j0 + k)
            rec(i0, i1, j0 + k, j1)

    rec(0, F.shape[1], 0, F.shape[0])
    return out


def new_boxes(o, level, tol, nbuf, cutoff, max_side):
    """steps 1-4: the new level-(level+1) patches as (nx, ny, I0, J0) in
    level-(level+1) cells, in the order of the level-l patches and of
    their clusters"""
    boxes = []
    for p in o.levels[level]:
        F = buffer_flags(flag_patch(o, p, tol), nbuf)
        for i0, i1, j0, j1 in cluster(F, cutoff, max_side):
            i0, i1 = max(i0, 1), min(i1, p.nx - 1)
            j0, j1 = max(j0, 1), min(j1, p.ny - 1)
            if i1 <= i0 or j1 <= j0:
                continue
            boxes.append((RATIO * (i1 - i0), RATIO * (j1 - j0),
                          RATIO * (p.I0 + i0), RATIO * (p.J0 + j0)))
    return boxes


def topo_level0(o):
    """the level-0 bathymetry as set, as one [NY, NX] array"""
    B = np.empty((o.NY, o.NX))
    for p in o.levels[0]:
        B[p.J0:p.J0 + p.ny, p.I0:p.I0 + p.nx] = p.b_raw
    return B


def topo_bilinear(B, level, nx, ny, I0, J0):
    """step 5 for a level-`level` box"""
    NY, NX = B.shape
    out = np.empty((ny, nx))
    sc = float(RATIO ** level)
    for j in range(ny):
        fy = (J0 + j + 0.5) / sc - 0.5
        jj = min(max(int(math.floor(fy)), 0), NY - 2)
        s = min(max(fy - jj, 0.0), 1.0)
        for i in range(nx):
            fx = (I0 + i + 0.5) / sc - 0.5
            ii = min(max(int(math.floor(fx)), 0), NX - 2)
            t = min(max(fx - ii, 0.0), 1.0)
            out[j, i] = ((B[jj, ii] * (1.0 - t) + B[jj, ii + 1] * t) * (1.0 - s)
                         + (B[jj + 1, ii] * (1.0 - t) + B[jj + 1, ii + 1] * t) * s)
    return out


def _depth_rule(h, b_old, b_new, dry_tol):
    if b_old == b_new or not h > dry_tol:
        return h
    v = h + (b_old - b_new)
    return v if v > 0.0 else 0.0


def regrid(o, level, tol, nbuf=2, cutoff=0.7, max_side=32):
    """a new AmrOracle whose levels <= level are those of o and whose level
    level+1 is rebuilt from the flags; o is left unchanged"""
    if not o.prepared:
        o.prepare()
    if level + 1 > len(o.levels) or level < 0:
        raise ValueError("no level %d to regrid from" % level)
    boxes = new_boxes(o, level, tol, nbuf, cutoff, max_side)
    kept = [p for p in o.patches if p.level <= level]
    specs = [(p.level, p.nx, p.ny, p.x0, p.y0) for p in kept]
    dxf, dyf = o.dx0 / RATIO ** (level + 1), o.dy0 / RATIO ** (level + 1)
    for nx, ny, I0, J0 in boxes:
        specs.append((level + 1, nx, ny, o.X0 + I0 * dxf, o.Y0 + J0 * dyf))
    n = A.AmrOracle(o.P, o.dx0, o.dy0, o.bc, specs, reflux=o.do_reflux)
    B = topo_level0(o)
    for pid, p in enumerate(kept):
        n.set_bathymetry(pid, p.b_raw)
    for k, (nx, ny, I0, J0) in enumerate(boxes):
        n.set_bathymetry(len(kept) + k, topo_bilinear(B, level + 1, nx, ny, I0, J0))
    n.prepare()
    dry_tol = o.P.dry_tol
    # kept patches: state and latch, depth rule where b changed
    for pid, p in enumerate(kept):
        np_ = n.patches[pid]
        q = p.q[:, 2:-2, 2:-2].copy()
        bo, bn = p.b[2:-2, 2:-2], np_.b[2:-2, 2:-2]
        for j in range(p.ny):
            for i in range(p.nx):
                q[0, j, i] = _depth_rule(q[0, j, i], bo[j, i], bn[j, i], dry_tol)
        np_.q[:, 2:-2, 2:-2] = q
        np_.brk[2:-2, 2:-2] = p.brk[2:-2, 2:-2]
    # new patches: interpolation from the coarse level, then old copies
    eta0 = o.P.eta0
    for k in range(len(boxes)):
        f = n.patches[len(kept) + k]
        for j in range(f.ny):
            for i in range(f.nx):
                I, J = f.I0 + i, f.J0 + j
                Ic, Jc = I // RATIO, J // RATIO
                c = n.find(level, Ic, Jc)
                ci, cj = Ic - c.I0 + 2, Jc - c.J0 + 2
                old = o.find(level + 1, I, J) if level + 1 < len(o.levels) else None
                if old is not None:
                    oi, oj = I - old.I0 + 2, J - old.J0 + 2
                    v = old.q[:, oj, oi].copy()
                    v[0] = _depth_rule(v[0], old.b[oj, oi], f.b[j + 2, i + 2], dry_tol)
                    f.q[:, j + 2, i + 2] = v
                    f.brk[j + 2, i + 2] = old.brk[oj, oi]
                    continue

                def val(a, bb):
                    qq, b_ = c.q[:, bb, a], c.b[bb, a]
                    v = qq.copy()
                    v[0] = (qq[0] + b_) - eta0
                    return v, not qq[0] > dry_tol

                v, dry = val(ci, cj)
                nb = [val(ci - 1, cj), val(ci + 1, cj), val(ci, cj - 1), val(ci, cj + 1)]
                any_dry = dry or any(x[1] for x in nb)
                ox = ((I - RATIO * Ic) + 0.5) / RATIO - 0.5
                oy = ((J - RATIO * Jc) + 0.5) / RATIO - 0.5
                out = np.empty(7)
                for m in range(7):
                    sx = sy = 0.0
                    if not any_dry:
                        sx = A._minmod(nb[1][0][m] - v[m], v[m] - nb[0][0][m])
                        sy = A._minmod(nb[3][0][m] - v[m], v[m] - nb[2][0][m])
                    out[m] = (v[m] + ox * sx) + oy * sy
                h = (out[0] + eta0) - f.b[j + 2, i + 2]
                out[0] = h if h > 0.0 else 0.0
                f.q[:, j + 2, i + 2] = out
                f.brk[j + 2, i + 2] = c.brk[cj, ci]
    n.t, n.steps, n.clip = o.t, o.steps, o.clip
    n.gauges = o.gauges.copy()
    n.records_t, n.records = list(o.records_t), [list(r) for r in o.records]
    return n
