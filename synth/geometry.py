"""Signed-distance descriptions of the synthetic bodies and their projection to lambda.

Sign convention (Sec. "Mask fields construction", eq. for lambda): the signed
distance is positive in the fluid and negative in the solid.

Projection rule used to build the input field lambda (the paper leaves open how
"intersected" cells are detected; this is input preparation, not solver work):

* a cell is *cut* when the signed distance changes sign strictly among its
  2^d vertices (min < 0 < max);
* a cut cell receives lambda = 1/2 [1 - tanh(sigma_c / h)], with sigma_c the
  signed distance at the cell centre and h the cell length scale
  ((dx dy dz)^(1/3) in 3D, (dx dy)^(1/2) in 2D);
* any other cell is solid (lambda = 1) when its largest vertex distance is
  <= 0, and fluid (lambda = 0) otherwise.

Grid-aligned bodies therefore give lambda in {0, 1} exactly.
"""

from __future__ import annotations

import numpy as np


def _vertex_coords(n, o, d):
    return o + d * np.arange(n + 1, dtype=np.float64)


def _center_coords(n, o, d):
    return o + d * (np.arange(n, dtype=np.float64) + 0.5)


def lambda_from_sdf(sdf, grid, chunk_z=16):
    """Project a signed-distance function onto the cell-centred grid.

    ``sdf(x, y, z)`` takes broadcastable float64 arrays and returns the signed
    distance (positive in fluid).  ``grid`` is a :class:`synth.cases.CaseSpec`
    (or any object with nx, ny, nz, dim, x0, y0, z0, dx, dy, dz).
    Returns lambda with shape (nz, ny, nx), x fastest.
    """
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    h = (grid.dx * grid.dy) ** 0.5 if grid.dim == 2 else (grid.dx * grid.dy * grid.dz) ** (1.0 / 3.0)
    xc = _center_coords(nx, grid.x0, grid.dx)
    yc = _center_coords(ny, grid.y0, grid.dy)
    xv = _vertex_coords(nx, grid.x0, grid.dx)
    yv = _vertex_coords(ny, grid.y0, grid.dy)
    lam = np.empty((nz, ny, nx), dtype=np.float64)
    if grid.dim == 2:
        zc = np.array([grid.z0 + 0.5 * grid.dz])
        Yc, Xc = np.meshgrid(yc, xc, indexing="ij")
        sc = sdf(Xc, Yc, np.full_like(Xc, zc[0]))
        Yv, Xv = np.meshgrid(yv, xv, indexing="ij")
        sv = sdf(Xv, Yv, np.full_like(Xv, zc[0]))
        vmin = np.minimum.reduce([sv[:-1, :-1], sv[:-1, 1:], sv[1:, :-1], sv[1:, 1:]])
        vmax = np.maximum.reduce([sv[:-1, :-1], sv[:-1, 1:], sv[1:, :-1], sv[1:, 1:]])
        lam[0] = _project(sc, vmin, vmax, h)
        return lam
    zc = _center_coords(nz, grid.z0, grid.dz)
    zv = _vertex_coords(nz, grid.z0, grid.dz)
    for k0 in range(0, nz, chunk_z):
        k1 = min(nz, k0 + chunk_z)
        Zc, Yc, Xc = np.meshgrid(zc[k0:k1], yc, xc, indexing="ij")
        sc = sdf(Xc, Yc, Zc)
        Zv, Yv, Xv = np.meshgrid(zv[k0:k1 + 1], yv, xv, indexing="ij")
        sv = sdf(Xv, Yv, Zv)
        corners = [sv[a:a + (k1 - k0), b:b + ny, c:c + nx]
                   for a in (0, 1) for b in (0, 1) for c in (0, 1)]
        vmin = np.minimum.reduce(corners)
        vmax = np.maximum.reduce(corners)
        lam[k0:k1] = _project(sc, vmin, vmax, h)
    return lam


def _project(sc, vmin, vmax, h):
    cut = (vmin < 0.0) & (vmax > 0.0)
    out = np.where(vmax <= 0.0, 1.0, 0.0)
    out = np.where(cut, 0.5 * (1.0 - np.tanh(sc / h)), out)
    return out


# ---------------------------------------------------------------------------
# signed distance functions (positive outside the body = in the fluid)
# ---------------------------------------------------------------------------

def sdf_box(lo, hi):
    """Axis-aligned box [lo, hi] (3 components; use +-inf for unbounded axes).

    Exact inside; outside the max-of-planes value (exact on faces, a lower bound
    near edges), which is all the projection rule needs.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)

    def f(x, y, z):
        d = None
        for c, a, b in ((x, lo[0], hi[0]), (y, lo[1], hi[1]), (z, lo[2], hi[2])):
            if np.isfinite(a):
                t = a - c
                d = t if d is None else np.maximum(d, t)
            if np.isfinite(b):
                t = c - b
                d = t if d is None else np.maximum(d, t)
        return d
    return f


def sdf_halfspace(point, normal):
    """Solid on the side opposite to ``normal``: distance = (x - point).normal."""
    p = np.asarray(point, dtype=np.float64)
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)

    def f(x, y, z):
        return (x - p[0]) * n[0] + (y - p[1]) * n[1] + (z - p[2]) * n[2]
    return f


def sdf_sphere(center, radius):
    c = np.asarray(center, dtype=np.float64)

    def f(x, y, z):
        return np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - radius
    return f


def _rounded_rect_2d(a, b, ca, cb, ha, hb, r):
    """2D rounded rectangle centred at (ca, cb) with half sizes (ha, hb), radius r."""
    qa = np.abs(a - ca) - (ha - r)
    qb = np.abs(b - cb) - (hb - r)
    outside = np.sqrt(np.maximum(qa, 0.0) ** 2 + np.maximum(qb, 0.0) ** 2)
    inside = np.minimum(np.maximum(qa, qb), 0.0)
    return outside + inside - r


def sdf_ahmed_like(x_front=0.0, length=1.044, width=0.389, height=0.288,
                   clearance=0.05, y_center=0.0, radius=0.1,
                   slant_deg=25.0, slant_len=0.222):
    """Ahmed-like bluff body: a box whose four front edges are rounded with
    ``radius`` and whose rear top edge is cut by a slant of ``slant_deg`` degrees
    over ``slant_len`` (measured along the slanted face).  The body stands
    ``clearance`` above the ground plane z = 0.

    Built as the intersection of (i) a rectangle rounded in the x-z plane,
    (ii) a rectangle rounded in the x-y plane (both extended far downstream so
    that only their front corners are rounded), (iii) the rear plane and
    (iv) the slant plane.  Interior distances are exact; exterior distances are
    lower bounds near edges.
    """
    zb = clearance
    zt = clearance + height
    zc = 0.5 * (zb + zt)
    L = length
    ext = 2.0 * L  # far downstream extension of the rounded profiles
    th = np.deg2rad(slant_deg)
    ax = x_front + L - slant_len * np.cos(th)
    az = zt
    nsx, nsz = np.sin(th), np.cos(th)

    def f(x, y, z):
        d_xz = _rounded_rect_2d(x, z, x_front + ext, zc, ext, 0.5 * height, radius)
        d_xy = _rounded_rect_2d(x, y, x_front + ext, y_center, ext, 0.5 * width, radius)
        d_rear = x - (x_front + L)
        d_slant = (x - ax) * nsx + (z - az) * nsz
        return np.maximum(np.maximum(d_xz, d_xy), np.maximum(d_rear, d_slant))
    return f


def naca4_half_thickness(x, t):
    """Half thickness of a symmetric NACA four-digit section of relative
    thickness t at chord fraction x in [0, 1] (the standard polynomial)."""
    return 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2 + 0.2843 * x ** 3 - 0.1015 * x ** 4)


def sdf_naca_symmetric(t=0.12, chord=1.0, gamma_deg=0.0, pivot=(0.25, 0.0), npts=4000):
    """Signed distance (positive in fluid) to a symmetric NACA section with its
    leading edge at the origin and the chord along +x, pitched nose-up by the
    angle of attack gamma (the section is rotated by -gamma about the pivot, so
    a flow along +x meets it at incidence gamma).  The magnitude is the
    distance to a dense cosine-spaced polyline of the surface (npts points per
    side), the sign comes from the exact thickness function."""
    from scipy.spatial import cKDTree
    beta = np.linspace(0.0, np.pi, npts)
    xs = 0.5 * (1.0 - np.cos(beta))
    ys = naca4_half_thickness(xs, t)
    pts = np.concatenate([np.stack([xs, ys], 1), np.stack([xs[::-1], -ys[::-1]], 1)]) * chord
    # densify along each segment so the point distance approximates the polyline distance
    seg = np.diff(pts, axis=0)
    dense = [pts[:-1] + seg * f for f in np.linspace(0.0, 1.0, 8, endpoint=False)]
    tree = cKDTree(np.concatenate(dense + [pts[-1:]]))
    g = np.deg2rad(gamma_deg)
    cg, sg = np.cos(g), np.sin(g)
    px, py = pivot

    def f(x, y, z):
        # world -> section frame: undo the rotation by -gamma about the pivot
        X = np.asarray(x, dtype=np.float64) - px
        Y = np.asarray(y, dtype=np.float64) - py
        xa = cg * X - sg * Y + px
        ya = sg * X + cg * Y + py
        shape = np.broadcast(xa, ya).shape
        xa = np.broadcast_to(xa, shape)
        ya = np.broadcast_to(ya, shape)
        xr, yr = xa.ravel(), ya.ravel()
        # exact distances only near the section (far points are fluid and never
        # part of a cut cell: any positive value serves)
        near = (xr > -0.2 * chord) & (xr < 1.2 * chord) & (np.abs(yr) < 0.3 * chord)
        dist = np.full(xr.shape, chord)
        if near.any():
            dist[near], _ = tree.query(np.stack([xr[near], yr[near]], 1))
        xc = xr / chord
        inside = (xc > 0.0) & (xc < 1.0) & (np.abs(yr) < chord * naca4_half_thickness(np.clip(xc, 0.0, 1.0), t))
        return np.where(inside, -dist, dist).reshape(shape)
    return f


def sdf_lbend(y_in=(0.65, 0.9), x_end=1.85, x_leg=(1.6, 1.85)):
    """Fluid inside an L-shaped duct: a horizontal leg x < x_end, y_in[0] < y <
    y_in[1] joined to a vertical leg x_leg[0] < x < x_leg[1], y < y_in[1] (the
    solid is everything else).  Union of two rectangles: the signed distance is
    the larger of the two inside distances (positive in the fluid)."""
    h = sdf_box((-np.inf, y_in[0], -np.inf), (x_end, y_in[1], np.inf))
    v = sdf_box((x_leg[0], -np.inf, -np.inf), (x_leg[1], y_in[1], np.inf))

    def f(x, y, z):
        return np.maximum(-h(x, y, z), -v(x, y, z))
    return f
