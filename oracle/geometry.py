"""Precompute from the indicator field lambda (done once per lambda).

Follows the paper's Sec. "Mask fields construction" (cell groups), Sec.
"Calculation of y+ at the immersed boundary" (eqs. for y+, y_perp and the
auxiliary sigma and n) and Sec. "Calculation of imposed fields" (interpolation
along the surface normal through two free-stream points and the surface point).

Readings where the paper is silent (each listed in the design notes):
* cell neighbours are the Moore neighbours (cells sharing at least a vertex);
* grad(lambda) uses central differences, one-sided at domain edges; when
  |grad lambda| h < 1e-12 the normal falls back to the normalised sum of
  (P - N) over in-solid Moore neighbours N;
* the in-solid neighbour N minimises -n_P.(P - N); values within 1e-12 h are
  ties, broken by the smaller |P - N|; y_perp is the mean over neighbours that
  are still tied (a choice that keeps mirror-symmetric geometry symmetric);
* y_perp is clamped to >= yperp_min_frac * h;
* interpolation points P1 = P + m h n_P and P2 = P + (m+1) h n_P with m = 1,
  moved outward (m = 2, 3) while P1 or P2 is unusable (outside the domain, or
  its multilinear stencil gives weight > 1e-9 to an in-solid cell); failing
  that a linear profile through S and the first usable P1, failing that the
  solid velocity itself;
* SST wall distance: distance to the point set {S-points of cut cells} U
  {face midpoints between lambda = 0 and lambda = 1 face neighbours}, and to
  no-slip domain walls.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from .grid import Grid

FC, BC, IC = 0, 1, 2
W_TOUCH = 1e-9
TIE_TOL = 1e-12


def moore_offsets(dim):
    offs = []
    rng = (-1, 0, 1)
    for o in itertools.product(rng, rng, rng if dim == 3 else (0,)):
        if o != (0, 0, 0):
            offs.append(o)  # (ox, oy, oz)
    return offs


def shift_offset(a, off, fill):
    """b[P] = a[P + off] (off in physical (x, y, z) order), ``fill`` outside."""
    b = np.full_like(a, fill)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    for d in range(3):
        o = off[d]
        A = 2 - d
        n = a.shape[A]
        if o > 0:
            src[A] = slice(o, n)
            dst[A] = slice(0, n - o)
        elif o < 0:
            src[A] = slice(0, n + o)
            dst[A] = slice(-o, n)
    b[tuple(dst)] = a[tuple(src)]
    return b


def classify(lam, g: Grid):
    """Cell groups (paper, Sec. Mask fields construction):
    in-solid if lambda >= 0.5; boundary if 0 < lambda < 0.5, or lambda = 0 with an
    in-solid neighbour; free-stream otherwise."""
    ic = lam >= 0.5
    nb_ic = np.zeros_like(ic)
    for off in moore_offsets(g.dim):
        nb_ic |= shift_offset(ic, off, False)
    bc = ((lam > 0.0) & (lam < 0.5)) | ((lam == 0.0) & nb_ic)
    tag = np.full(lam.shape, FC, dtype=np.int8)
    tag[bc] = BC
    tag[ic] = IC
    return tag


def grad_lambda(lam, g: Grid):
    """central differences, one-sided at the domain edges"""
    out = []
    for d in range(3):
        gd = np.zeros(lam.shape)
        if d in g.axes and g.n[d] > 1:
            A = 2 - d
            D = g.delta[d]
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            mid = [slice(None)] * 3
            lo[A], hi[A], mid[A] = slice(0, -2), slice(2, None), slice(1, -1)
            gd[tuple(mid)] = (lam[tuple(hi)] - lam[tuple(lo)]) / (2.0 * D)
            first = [slice(None)] * 3
            second = [slice(None)] * 3
            first[A], second[A] = 0, 1
            gd[tuple(first)] = (lam[tuple(second)] - lam[tuple(first)]) / D
            last = [slice(None)] * 3
            before = [slice(None)] * 3
            last[A], before[A] = -1, -2
            gd[tuple(last)] = (lam[tuple(last)] - lam[tuple(before)]) / D
        out.append(gd)
    return out


@dataclass
class Geometry:
    tag: np.ndarray
    lam: np.ndarray
    sigma: np.ndarray
    bc_cells: np.ndarray          # linear indices, increasing
    ic_cells: np.ndarray          # linear indices, increasing
    normal: np.ndarray            # (n_bc, 3) outward unit normal n_P at boundary cells
    yperp: np.ndarray             # (n_bc,)
    yeff: np.ndarray              # (n_bc,)
    mode: np.ndarray              # (n_bc,) 3 quadratic, 2 linear, 1 constant
    L: np.ndarray                 # (n_bc, 3) Lagrange weights of (S, P1, P2) at s = y_perp
    st1_idx: np.ndarray           # (n_bc, 8) stencil cells of P1 (weight 0 padding -> own cell)
    st1_w: np.ndarray
    st2_idx: np.ndarray
    st2_w: np.ndarray
    nstar: np.ndarray             # (n_bc,) chosen in-solid neighbour (-1 if not searched)
    wall_cells: np.ndarray = None  # free-stream cells next to a no-slip domain face
    wall_y: np.ndarray = None      # their wall distance (half the cell width)
    wall_n: np.ndarray = None      # (n_wall, 3) unit normal pointing away from the wall
    dw: np.ndarray = None         # wall distance (SST)
    extra: dict = field(default_factory=dict)


def _lin(g, i, j, k):
    return i + g.nx * (j + g.ny * k)


def _unlin(g, c):
    return c % g.nx, (c // g.nx) % g.ny, c // (g.nx * g.ny)


def _center(g, i, j, k):
    return np.array([g.o[0] + (i + 0.5) * g.dx, g.o[1] + (j + 0.5) * g.dy,
                     g.o[2] + (k + 0.5) * g.dz if g.dim == 3 else 0.0])


def cell_normal(g, lam, tag, gl, i, j, k):
    """n = -grad(lambda)/|grad(lambda)| (eq. for sigma and n), with the fallback
    to the normalised sum of (P - N) over in-solid Moore neighbours."""
    gv = np.array([gl[0][k, j, i], gl[1][k, j, i], gl[2][k, j, i]])
    nrm = np.sqrt(gv @ gv)
    if nrm * g.h >= 1e-12:
        return -gv / nrm
    acc = np.zeros(3)
    for (ox, oy, oz) in moore_offsets(g.dim):
        ii, jj, kk = i + ox, j + oy, k + oz
        if 0 <= ii < g.nx and 0 <= jj < g.ny and 0 <= kk < g.nz and tag[kk, jj, ii] == IC:
            acc -= np.array([ox * g.dx, oy * g.dy, oz * g.dz])
    a = np.sqrt(acc @ acc)
    return acc / a if a > 0.0 else acc


def multilinear_stencil(g, X):
    """cells and weights of multilinear interpolation at point X from the
    surrounding 2^d cell centres (indices clamped to the grid)"""
    per_axis = []
    for d in range(3):
        if d not in g.axes:
            per_axis.append([(0, 1.0)])
            continue
        t = (X[d] - g.o[d]) / g.delta[d] - 0.5
        i0 = int(np.floor(t))
        i0 = min(max(i0, 0), g.n[d] - 2)
        f = t - i0
        f = min(max(f, 0.0), 1.0)
        per_axis.append([(i0, 1.0 - f), (i0 + 1, f)])
    cells, ws = [], []
    for (ix, wx) in per_axis[0]:
        for (iy, wy) in per_axis[1]:
            for (iz, wz) in per_axis[2]:
                cells.append(_lin(g, ix, iy, iz))
                ws.append(wx * wy * wz)
    return cells, ws


def _inside_domain(g, X):
    for d in g.axes:
        if not (g.o[d] <= X[d] <= g.o[d] + g.n[d] * g.delta[d]):
            return False
    return True


def _usable(g, tag_flat, X):
    """an interpolation point is usable when it lies inside the domain and its
    stencil gives no weight > 1e-9 to an in-solid cell"""
    if not _inside_domain(g, X):
        return None
    cells, ws = multilinear_stencil(g, X)
    if any(w > W_TOUCH and tag_flat[c] == IC for c, w in zip(cells, ws)):
        return None
    return cells, ws


def _lagrange3(s, s1, s2):
    """weights of the quadratic through nodes 0, s1, s2 evaluated at s"""
    L0 = (s - s1) * (s - s2) / (s1 * s2)
    L1 = s * (s - s2) / (s1 * (s1 - s2))
    L2 = s * (s - s1) / (s2 * (s2 - s1))
    return L0, L1, L2


def _pad8(cells, ws, own):
    cells = list(cells) + [own] * (8 - len(cells))
    ws = list(ws) + [0.0] * (8 - len(ws))
    return cells, ws


def _yperp_via(g, lam_flat, sig_flat, lam, tag, gl, P, i, j, k, ii, jj, kk):
    """y_perp of boundary cell P (lambda_P = 0) through its in-solid neighbour N"""
    cn = _lin(g, ii, jj, kk)
    N = _center(g, ii, jj, kk)
    if lam_flat[cn] < 1.0:
        # second case: distance from P to the plane through N + |sigma_N| n_N
        nN = cell_normal(g, lam, tag, gl, ii, jj, kk)
        return float(nN @ (P - (N + abs(sig_flat[cn]) * nN)))
    # third case: distance to the mean of the vertices shared by P and N
    vp = {(i + a, j + bb, k + cc) for a in (0, 1) for bb in (0, 1) for cc in ((0, 1) if g.dim == 3 else (0,))}
    vn = {(ii + a, jj + bb, kk + cc) for a in (0, 1) for bb in (0, 1) for cc in ((0, 1) if g.dim == 3 else (0,))}
    shared = np.array(sorted(vp & vn), dtype=np.float64)
    m = shared.mean(axis=0)
    vmean = np.array([g.o[0] + m[0] * g.dx, g.o[1] + m[1] * g.dy, g.o[2] + m[2] * g.dz if g.dim == 3 else 0.0])
    return float(np.sqrt((P - vmean) @ (P - vmean)))


def precompute(spec, with_wall_distance=None):
    g = Grid(spec)
    lam = np.asarray(spec.lam, dtype=np.float64)
    C = spec.constants
    tag = classify(lam, g)
    tag_flat = tag.ravel()
    lam_flat = lam.ravel()
    sigma = np.full(lam.shape, np.nan)
    cut = (lam > 0.0) & (lam < 1.0)
    sigma[cut] = g.h * np.arctanh(1.0 - 2.0 * lam[cut])  # eq. for sigma_perp
    sig_flat = sigma.ravel()
    gl = grad_lambda(lam, g)
    bc_cells = np.flatnonzero(tag_flat == BC)
    ic_cells = np.flatnonzero(tag_flat == IC)
    nb = len(bc_cells)
    normal = np.zeros((nb, 3))
    yperp = np.zeros(nb)
    nstar = np.full(nb, -1, dtype=np.int64)
    mode = np.zeros(nb, dtype=np.int8)
    Lw = np.zeros((nb, 3))
    st1_idx = np.zeros((nb, 8), dtype=np.int64)
    st2_idx = np.zeros((nb, 8), dtype=np.int64)
    st1_w = np.zeros((nb, 8))
    st2_w = np.zeros((nb, 8))
    h = g.h
    for b, c in enumerate(bc_cells):
        i, j, k = _unlin(g, c)
        P = _center(g, i, j, k)
        nP = cell_normal(g, lam, tag, gl, i, j, k)
        normal[b] = nP
        lp = lam_flat[c]
        if 0.0 < lp < 0.5:
            yp = abs(sig_flat[c])  # eq. for y_perp, first case
        else:
            # in-solid neighbour minimising -n_P.(P - N); among equal values the
            # nearer one; y_perp is averaged over neighbours that remain tied
            best = None
            ysum, ycnt = 0.0, 0
            for (ox, oy, oz) in moore_offsets(g.dim):
                ii, jj, kk = i + ox, j + oy, k + oz
                if not (0 <= ii < g.nx and 0 <= jj < g.ny and 0 <= kk < g.nz):
                    continue
                cn = _lin(g, ii, jj, kk)
                if tag_flat[cn] != IC:
                    continue
                PN = P - _center(g, ii, jj, kk)
                v = -float(nP @ PN)
                dist = float(np.sqrt(PN @ PN))
                if best is None or v < best[0] - TIE_TOL * h or (
                        abs(v - best[0]) <= TIE_TOL * h and dist < best[1] - TIE_TOL * h):
                    best = (v, dist, cn)
                    ysum, ycnt = _yperp_via(g, lam_flat, sig_flat, lam, tag, gl, P, i, j, k, ii, jj, kk), 1
                elif abs(v - best[0]) <= TIE_TOL * h and abs(dist - best[1]) <= TIE_TOL * h:
                    ysum += _yperp_via(g, lam_flat, sig_flat, lam, tag, gl, P, i, j, k, ii, jj, kk)
                    ycnt += 1
            nstar[b] = best[2]
            yp = ysum / ycnt
        yp = max(yp, C["yperp_min_frac"] * h)
        yperp[b] = yp
        # interpolation points along n_P
        done = False
        for m in (1, 2, 3):
            q1 = _usable(g, tag_flat, P + m * h * nP)
            q2 = _usable(g, tag_flat, P + (m + 1) * h * nP)
            if q1 is not None and q2 is not None:
                mode[b] = 3
                Lw[b] = _lagrange3(yp, yp + m * h, yp + (m + 1) * h)
                st1_idx[b], st1_w[b] = _pad8(q1[0], q1[1], c)
                st2_idx[b], st2_w[b] = _pad8(q2[0], q2[1], c)
                done = True
                break
        if not done:
            for m in (1, 2, 3):
                q1 = _usable(g, tag_flat, P + m * h * nP)
                if q1 is not None:
                    c1, w1 = q1
                    s1 = yp + m * h
                    mode[b] = 2
                    Lw[b] = (1.0 - yp / s1, yp / s1, 0.0)
                    st1_idx[b], st1_w[b] = _pad8(c1, w1, c)
                    st2_idx[b], st2_w[b] = _pad8([], [], c)
                    done = True
                    break
        if not done:
            mode[b] = 1
            Lw[b] = (1.0, 0.0, 0.0)
            st1_idx[b], st1_w[b] = _pad8([], [], c)
            st2_idx[b], st2_w[b] = _pad8([], [], c)
    if getattr(spec, "yplus_dist", "eff") == "perp":
        yeff = yperp.copy()  # appendix variant: y+ from the perpendicular distance alone
    else:
        yeff = 0.5 * (yperp + 0.5 * h)  # eq. for y_eff
    geo = Geometry(tag=tag, lam=lam, sigma=sigma, bc_cells=bc_cells, ic_cells=ic_cells,
                   normal=normal, yperp=yperp, yeff=yeff, mode=mode, L=Lw,
                   st1_idx=st1_idx, st1_w=st1_w, st2_idx=st2_idx, st2_w=st2_w, nstar=nstar)
    # free-stream cells touching a no-slip domain face (owner lambda = 0): the wall
    # functions of the domain walls act there; the first face in the order
    # xmin, xmax, ymin, ymax, zmin, zmax with the smallest half width is used
    wall_y = np.full(g.shape, np.inf)
    wall_n = np.zeros(g.shape + (3,))
    for d in g.axes:
        for s_ in (-1, 1):
            if g.face_kind(d, s_) != "noslip":
                continue
            sel = np.zeros(g.shape, dtype=bool)
            sel[g.bnd(d, s_)] = True
            sel &= (lam == 0.0) & (tag == FC)
            y = 0.5 * g.delta[d]
            better = sel & (y < wall_y)
            wall_y[better] = y
            nv = np.zeros(3)
            nv[d] = -float(s_)
            wall_n[better] = nv
    wall_cells = np.flatnonzero(np.isfinite(wall_y).ravel())
    geo.wall_cells = wall_cells
    geo.wall_y = wall_y.ravel()[wall_cells]
    geo.wall_n = wall_n.reshape(-1, 3)[wall_cells]
    if with_wall_distance is None:
        with_wall_distance = spec.model == "sst"
    if with_wall_distance:
        geo.dw = wall_distance(g, lam, tag, gl, sigma)
    return geo


def interface_points(g, lam, tag, gl, sigma):
    """S-points of cut cells and face midpoints between lambda=0 / lambda=1 pairs"""
    pts = []
    cutc = np.flatnonzero(((lam > 0.0) & (lam < 1.0)).ravel())
    sig_flat = sigma.ravel()
    for c in cutc:
        i, j, k = _unlin(g, c)
        nP = cell_normal(g, lam, tag, gl, i, j, k)
        pts.append(_center(g, i, j, k) - sig_flat[c] * nP)
    for d in g.axes:
        lo = lam[g.interior_lo(d)]
        hi = lam[g.interior_hi(d)]
        pair = ((lo == 0.0) & (hi == 1.0)) | ((lo == 1.0) & (hi == 0.0))
        kk, jj, ii = np.nonzero(pair)
        for (i, j, k) in zip(ii, jj, kk):
            P = _center(g, i, j, k)
            P[d] += 0.5 * g.delta[d]
            pts.append(P)
    return np.array(pts).reshape(-1, 3)


def wall_distance(g, lam, tag, gl, sigma):
    from scipy.spatial import cKDTree
    X = np.stack([g.centers[0], g.centers[1],
                  g.centers[2] if g.dim == 3 else np.zeros(g.shape)], axis=-1).reshape(-1, 3)
    dw = np.full(g.N, 1e30)
    pts = interface_points(g, lam, tag, gl, sigma)
    if len(pts):
        dist, _ = cKDTree(pts).query(X)
        dw = np.minimum(dw, dist)
    for d in g.axes:
        for s in (-1, 1):
            if g.face_kind(d, s) == "noslip":
                wall = g.o[d] + (0.0 if s < 0 else g.n[d] * g.delta[d])
                dw = np.minimum(dw, np.abs(X[:, d] - wall))
    return dw.reshape(g.shape)
