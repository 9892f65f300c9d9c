"""Pins of the oracle's per-lambda precompute against closed forms of the
paper's geometry (eq. for lambda and its inverse for sigma; the three cases of
y_perp; y_eff) and brute-force classification of hand-made patterns."""

import numpy as np
import pytest

import synth
from synth import geometry as G
from oracle.geometry import precompute, classify, FC, BC, IC, multilinear_stencil
from oracle.grid import Grid


def _spec(nx, ny, nz, dim, lam, d=1.0, model="laminar", bc=None):
    if bc is None:
        bc = ("inlet", "outlet", "slip", "slip") + (("slip", "slip") if dim == 3 else ("empty", "empty"))
    s = synth.CaseSpec(name="t", dim=dim, nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=d,
                       bc=bc, u_in=(1.0, 0.0, 0.0), k_in=1e-3, eps_in=1e-4, omega_in=1.0, nu=1e-3, model=model)
    s.lam = np.asarray(lam, dtype=np.float64).reshape(s.shape)
    return s.validate()


def test_sigma_inverts_lambda_on_a_cut_plane():
    # a plane z-normal... here y-normal in 2D at an offset inside a cell row: lambda of the
    # cut cells is 1/2(1 - tanh(sigma/h)); the oracle's sigma must return the exact
    # signed distance of the cell centre to the plane
    for off in (0.13, 0.37, 0.5, 0.71):
        s = synth.CaseSpec(name="plane", dim=2, nx=8, ny=8, nz=1, x0=0.0, y0=0.0, z0=0.0, dx=1.0, dy=1.0,
                           dz=1.0, bc=("inlet", "outlet", "slip", "slip", "empty", "empty"), u_in=(1, 0, 0),
                           k_in=1e-3, eps_in=1e-4, omega_in=1.0, nu=1e-3, model="laminar")
        wall = 3.0 + off
        s.lam = G.lambda_from_sdf(G.sdf_halfspace((0.0, wall, 0.0), (0.0, 1.0, 0.0)), s)
        s.validate()
        geo = precompute(s)
        yc = 0.5 + np.arange(8)
        cut = (s.lam[0, :, 0] > 0) & (s.lam[0, :, 0] < 1)
        np.testing.assert_allclose(geo.sigma[0, cut, 0], yc[cut] - wall, rtol=0, atol=1e-13)
        # boundary cells cut by the plane: y_perp = |sigma| (first case), normal = +y
        for b, c in enumerate(geo.bc_cells):
            j = (c // 8) % 8
            lam = s.lam.ravel()[c]
            if 0 < lam < 0.5:
                assert abs(geo.yperp[b] - abs(yc[j] - wall)) < 1e-13
                np.testing.assert_allclose(geo.normal[b], [0.0, 1.0, 0.0], atol=1e-14)


def test_classification_hand_pattern_2d():
    lam = np.zeros((6, 6))
    lam[2, 2] = 1.0    # in-solid
    lam[2, 3] = 0.6    # in-solid (>= 0.5)
    lam[4, 4] = 0.3    # cut, < 0.5: boundary
    tag = classify(lam[None], Grid(_spec(6, 6, 1, 2, lam)))[0]
    expect = np.full((6, 6), FC)
    for (j, i) in [(1, 1), (1, 2), (1, 3), (1, 4), (2, 1), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4), (4, 4)]:
        expect[j, i] = BC
    expect[2, 2] = IC
    expect[2, 3] = IC
    np.testing.assert_array_equal(tag, expect)


def test_classification_brute_force_random_3d():
    rng = np.random.default_rng(3)
    lam = rng.choice([0.0, 0.0, 0.0, 0.2, 0.5, 0.7, 1.0], size=(5, 6, 7))
    s = _spec(7, 6, 5, 3, lam)
    tag = classify(s.lam, Grid(s))
    for k in range(5):
        for j in range(6):
            for i in range(7):
                l = lam[k, j, i]
                nb = False
                for dk in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            kk, jj, ii = k + dk, j + dj, i + di
                            if (dk, dj, di) != (0, 0, 0) and 0 <= kk < 5 and 0 <= jj < 6 and 0 <= ii < 7:
                                nb |= lam[kk, jj, ii] >= 0.5
                if l >= 0.5:
                    e = IC
                elif (0 < l < 0.5) or (l == 0 and nb):
                    e = BC
                else:
                    e = FC
                assert tag[k, j, i] == e


@pytest.mark.parametrize("dim", [2, 3])
def test_yperp_grid_aligned_special_cases(dim):
    # one in-solid cell (lambda = 1) in the middle: its Moore neighbours are boundary
    # cells whose y_perp is the distance to the mean of the shared vertices:
    # face h/2, edge h/sqrt(2), corner h sqrt(3)/2 (third case of the y_perp equation)
    n = 5
    h = 0.5
    shape = (n, n, n) if dim == 3 else (1, n, n)
    lam = np.zeros(shape)
    if dim == 3:
        lam[2, 2, 2] = 1.0
    else:
        lam[0, 2, 2] = 1.0
    s = _spec(n, n, n if dim == 3 else 1, dim, lam, d=h)
    geo = precompute(s)
    assert len(geo.bc_cells) == (26 if dim == 3 else 8)
    for b, c in enumerate(geo.bc_cells):
        i, j, k = c % n, (c // n) % n, c // (n * n)
        off = np.abs([i - 2, j - 2, (k - 2) if dim == 3 else 0]).sum()
        expect = {1: h / 2, 2: h / np.sqrt(2), 3: h * np.sqrt(3) / 2}[off]
        assert abs(geo.yperp[b] - expect) < 1e-14
        assert abs(geo.yeff[b] - 0.5 * (expect + 0.5 * h)) < 1e-14
        # the normal points from the solid cell to P
        v = np.array([i - 2, j - 2, (k - 2) if dim == 3 else 0], dtype=float)
        np.testing.assert_allclose(geo.normal[b], v / np.linalg.norm(v), atol=1e-14)


def test_yperp_second_case_plane_through_insolid_neighbour():
    # a wall plane at y = 2.8 (cells of height 1): the cell row j = 2 (centre 2.5) is
    # cut with lambda > 0.5 (in-solid), row j = 3 (centre 3.5) has lambda = 0 and is a
    # boundary cell whose y_perp is the distance to the plane through N + |sigma_N| n_N
    s = synth.CaseSpec(name="plane2", dim=2, nx=6, ny=8, nz=1, x0=0.0, y0=0.0, z0=0.0, dx=1.0, dy=1.0, dz=1.0,
                       bc=("inlet", "outlet", "slip", "slip", "empty", "empty"), u_in=(1, 0, 0),
                       k_in=1e-3, eps_in=1e-4, omega_in=1.0, nu=1e-3, model="laminar")
    s.lam = G.lambda_from_sdf(G.sdf_halfspace((0.0, 2.8, 0.0), (0.0, 1.0, 0.0)), s)
    s.validate()
    assert np.all(s.lam[0, 2, :] > 0.5) and np.all(s.lam[0, 3, :] == 0.0)
    geo = precompute(s)
    row3 = [b for b, c in enumerate(geo.bc_cells) if (c // 6) % 8 == 3]
    assert len(row3) == 6
    for b in row3:
        assert abs(geo.yperp[b] - (3.5 - 2.8)) < 1e-13


def test_quadratic_interpolation_reproduces_wall_parabola():
    # grid-aligned channel wall: the quadratic through (0, 0), P1, P2 along the normal
    # reproduces any profile u = a y + b y^2 measured from the wall exactly
    s = synth.case_channel_ib(nx=12, n_fluid=8, n_solid=2)
    geo = precompute(s)
    g = Grid(s)
    y = g.centers[1]  # wall at y = 0 and y = 1
    for (a, bq) in [(1.0, 0.0), (2.0, -3.0), (0.3, 5.0)]:
        ywall = np.where(y < 0.5, y, 1.0 - y)
        f = (a * ywall + bq * ywall ** 2).ravel()
        v1 = (geo.st1_w * f[geo.st1_idx]).sum(axis=1)
        v2 = (geo.st2_w * f[geo.st2_idx]).sum(axis=1)
        val = geo.L[:, 1] * v1 + geo.L[:, 2] * v2
        np.testing.assert_allclose(val, f[geo.bc_cells], rtol=0, atol=1e-13)
        assert np.all(geo.mode == 3)


def test_multilinear_stencil_partition_of_unity_and_linear_exactness():
    s = synth.case_small_body3d()
    g = Grid(s)
    rng = np.random.default_rng(5)
    for _ in range(50):
        X = np.array([rng.uniform(0.1, 1.9), rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.9)])
        cells, ws = multilinear_stencil(g, X)
        assert abs(sum(ws) - 1.0) < 1e-14
        cx = g.centers[0].ravel()[cells]
        cy = g.centers[1].ravel()[cells]
        assert abs(np.dot(ws, cx) - X[0]) < 1e-13 and abs(np.dot(ws, cy) - X[1]) < 1e-13


def test_wall_distance_flat_wall():
    # face-midpoint interface points of a flat grid-aligned wall: the distance of a
    # cell m rows above the wall is (m + 1/2) h exactly
    s = synth.case_small_body3d(model="sst", shape="box")
    h = s.dx  # 1/12: the box below lies on cell faces
    s.lam = G.lambda_from_sdf(G.sdf_box((0.5, 0.25, 0.25), (0.75, 0.75, 0.5)), s)
    assert set(np.unique(s.lam)) <= {0.0, 1.0}
    geo = precompute(s)
    i, j = 7, 6  # cell column above the middle of the top face z = 0.5 = 6 h
    for m in range(0, 3):
        k = 6 + m
        assert abs(geo.dw[k, j, i] - (m + 0.5) * h) < 1e-13
