"""Pins of the oracle's SIMPLE iteration against closed forms and invariants:
discrete plane-Poiseuille solutions (body-fitted and grid-aligned immersed walls),
the pressure system (symmetry, definiteness, mass conservation), mirror
symmetry, the explicit transpose stress term, red-black Gauss-Seidel against a
direct solve, and decaying homogeneous turbulence against its ODE solution."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from synth import geometry as G
from oracle.solver import Simple
from oracle.grid import Grid


def _converge(sim, tol=1e-13, maxit=4000):
    for _ in range(maxit):
        r = sim.step()
        if max(r.values()) < tol:
            return r
    return r


def _developed(sim, i):
    g = sim.g
    p = sim.p[0]
    jm = p.shape[0] // 2  # a fluid row (solid rows hold no pressure information)
    G_ = -(p[jm, i + 1] - p[jm, i - 1]) / (2 * g.dx)
    return G_, sim.u[0][0][:, i], g.centers[1][0, :, 0]


def test_bodyfitted_poiseuille_exact():
    # no-slip walls at y = 0, H with half-cell wall distance: the discrete solution is
    # u_j = G/(2 nu) y_j (H - y_j) + G D^2/(8 nu) and G = 12 nu U / (H^2 + 2 D^2)
    s = synth.case_channel_bodyfitted(nx=64, n_fluid=8, nu=0.1, U=1.0)
    sim = Simple(s)
    _converge(sim)
    H, D, nu = 1.0, 1.0 / 8, 0.1
    G_, u, y = _developed(sim, 40)
    Gx = 12 * nu * 1.0 / (H ** 2 + 2 * D ** 2)
    assert abs(G_ / Gx - 1.0) < 1e-8
    np.testing.assert_allclose(u, Gx / (2 * nu) * y * (H - y) + Gx * D ** 2 / (8 * nu), rtol=1e-9)


def test_immersed_channel_developed_profile_and_pressure_drop():
    # grid-aligned immersed walls (lambda in {0,1}, laminar: every boundary cell forced):
    # the quadratic interpolation reproduces the parabola through 0 at the wall, so
    # u_j = G/(2 nu) y_j (H - y_j) exactly, and the flux Q through a cross-section is the
    # midpoint sum of that profile: G = 12 nu (Q/H) / (H^2 + D^2/2)
    s = synth.case_channel_ib(nx=96, n_fluid=8, n_solid=2, nu=0.1, U=1.0)
    sim = Simple(s)
    _converge(sim)
    H, D, nu = 1.0, 1.0 / 8, 0.1
    i = 56
    G_, u, y = _developed(sim, i)
    fl = (y > 0) & (y < H)
    np.testing.assert_allclose(u[fl], G_ / (2 * nu) * y[fl] * (H - y[fl]), rtol=1e-9, atol=1e-12)
    Q = sim.phi[0][0][:, i].sum()
    assert abs(G_ / (12 * nu * (Q / H) / (H ** 2 + D ** 2 / 2)) - 1.0) < 1e-9
    # solid rows carry no velocity and no flux
    assert np.all(u[~fl] == 0.0)
    assert np.all(sim.phi[0][0][~fl, :] == 0.0)


def test_immersed_vs_bodyfitted_offset():
    # at equal pressure gradient the two discrete solutions differ by G D^2 / (8 nu)
    nu = 0.1
    bf = Simple(synth.case_channel_bodyfitted(nx=64, n_fluid=8, nu=nu))
    ib = Simple(synth.case_channel_ib(nx=96, n_fluid=8, n_solid=2, nu=nu))
    _converge(bf)
    _converge(ib)
    Gb, ub, yb = _developed(bf, 40)
    Gi, ui, yi = _developed(ib, 56)
    ui_f = ui[(yi > 0) & (yi < 1)]
    D = 1.0 / 8
    # (the measured gradients carry ~1e-9 relative convergence error; the offset is a
    # difference of two O(10) profiles, hence the looser bound)
    np.testing.assert_allclose(ub / Gb - ui_f / Gi, D ** 2 / (8 * nu), rtol=1e-6)


def _pressure_setup(spec):
    sim = Simple(spec)
    sim.step()
    rAU = sim.last["rAU"]
    return sim, sim.pressure_matrix(rAU)


@pytest.mark.parametrize("mk", [lambda: synth.case_cavity_block(nx=12, ny=8),
                                lambda: synth.case_small_body3d(nx=10, ny=6, nz=6)])
def test_pressure_matrix_symmetric_positive_definite(mk):
    sim, A = _pressure_setup(mk())
    Ad = A.toarray()
    np.testing.assert_array_equal(Ad, Ad.T)
    ev = np.linalg.eigvalsh(Ad)
    assert ev.min() > 0.0
    kappa = ev.max() / ev.min()  # condition number of the pressure system
    assert np.isfinite(kappa) and kappa > 1.0
    # off-diagonals are <= 0 and rows of coupled cells are weakly diagonally dominant
    off = Ad - np.diag(np.diag(Ad))
    assert np.all(off <= 0.0)
    assert np.all(np.diag(Ad) + off.sum(axis=1) >= -1e-12 * np.diag(Ad))


@pytest.mark.parametrize("continuity", ["literal", "weighted"])
def test_mass_conservation_after_pressure_solve(continuity):
    # after the (direct) pressure solve the corrected fluxes satisfy the lambda-masked
    # continuity equation: zero net outflow in every cell with lambda = 0 (both
    # readings) and, for the literal reading, in every cell with lambda < 1 that is
    # coupled to the pressure field
    # turbulent with a small viscosity, so that some cut boundary cells are on the
    # logarithmic branch (not forced) and take part in the pressure coupling
    s = synth.case_small_body3d(nx=16, ny=8, nz=8, model="keps", nu=1e-5)
    sim = Simple(s, continuity=continuity)
    for _ in range(3):
        sim.step()
    g = sim.g
    div = sum(g.outward_flux(sim.phi, d, s_) for (d, s_) in sim.dirs)
    scale = np.abs(sim.phi[0]).sum() + np.abs(sim.phi[1]).sum() + np.abs(sim.phi[2]).sum()
    fluid = s.lam == 0.0
    assert np.abs(div[fluid]).max() < 1e-12 * scale
    if continuity == "literal":
        cut = (s.lam > 0) & (s.lam < 1) & (sim.last["rAU"] > 0)
        assert np.abs(div[cut]).max() < 1e-12 * scale


def test_mirror_symmetry():
    # a sphere centred in a duct with slip walls on both y faces and an odd number of
    # cells across: mirror-symmetric lambda and boundary data give mirror-symmetric fields
    s = synth.CaseSpec(name="sym", dim=3, nx=16, ny=9, nz=8, x0=0.0, y0=0.0, z0=0.0, dx=1 / 9, dy=1 / 9,
                       dz=1 / 9, bc=("inlet", "outlet", "slip", "slip", "noslip", "slip"), u_in=(1.0, 0.0, 0.0),
                       k_in=1e-3, eps_in=1e-4, omega_in=1.0, nu=1e-2, model="keps")
    lam = G.lambda_from_sdf(G.sdf_sphere((0.7, 0.5, 0.45), 0.22), s)
    s.lam = 0.5 * (lam + lam[:, ::-1, :])  # exact mirror symmetry of the input
    s.validate()
    np.testing.assert_array_equal(s.lam, s.lam[:, ::-1, :])
    sim = Simple(s)
    for _ in range(8):
        sim.step()
    for f, sign in ((sim.u[0], 1), (sim.u[1], -1), (sim.u[2], 1), (sim.p, 1), (sim.k, 1), (sim.nut, 1)):
        scale = np.abs(f).max() + 1e-300
        assert np.abs(f - sign * f[:, ::-1, :]).max() < 1e-11 * scale


def test_transpose_stress_term_closed_form():
    # div(nu (grad u)^T) for u = (x^2, 0, 0) and constant nu is (2 nu, 0, 0) in the
    # interior (Gauss gradients with linear interpolation are exact for quadratics)
    s = synth.case_small_body3d(nx=10, ny=6, nz=6)
    s.lam[...] = 0.0
    sim = Simple(s)
    g = sim.g
    x = g.centers[0]
    u = [x ** 2, np.zeros(g.shape), np.zeros(g.shape)]
    nu = np.full(g.shape, 0.37)
    T = sim.transpose_term(nu, sim.grad_u(u))
    inner = (slice(2, -2), slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(T[0][inner], 2 * 0.37 * g.V, rtol=1e-10)
    assert np.abs(T[1][inner]).max() < 1e-14 and np.abs(T[2][inner]).max() < 1e-14


def test_red_black_gauss_seidel_converges_to_direct_solve():
    # the sweeps use exactly the assembled coefficients: many sweeps reproduce the
    # direct solution of the same (diagonally dominant) system
    s = synth.case_cavity_block(nx=12, ny=8)
    sim = Simple(s)
    sim.step()
    g = sim.g
    nuEff = s.nu + sim.nut
    anb = sim.neighbor_coeffs(nuEff, sim.phi)
    aPr = (sum(anb.values()) + 0.3) / 0.7
    rhs = np.random.default_rng(0).standard_normal(g.shape)
    x = sim.rbgs(aPr, anb, rhs, np.zeros(g.shape), 3000)
    lin = np.arange(g.N).reshape(g.shape)
    rows, cols, vals = [lin.ravel()], [lin.ravel()], [aPr.ravel()]
    for (d, s_), a in anb.items():
        nb = g.neighbor(lin.astype(float), d, s_, fill=-1).astype(int).ravel()
        m = nb >= 0
        rows.append(lin.ravel()[m])
        cols.append(nb[m])
        vals.append(-a.ravel()[m])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(g.N, g.N))
    xd = spla.spsolve(A.tocsc(), rhs.ravel())
    np.testing.assert_allclose(x.ravel(), xd, rtol=1e-10, atol=1e-12)


@pytest.mark.slow
def test_decaying_turbulence_first_order_convergence():
    # uniform inflow without shear: production vanishes and the k-eps pair decays as
    # U dk/dx = -eps, U deps/dx = -C2 eps^2/k, i.e. k = k0 (1 + x/(U tau))^-n with
    # n = 1/(C2 - 1), tau = n k0/eps0.  Upwind convection converges at first order.
    errs = []
    for nx in (32, 64):
        s = synth.case_uniform_duct(nx=nx, ny=4)
        sim = Simple(s)
        _converge(sim, tol=1e-11, maxit=3000)
        C2 = s.constants["C2"]
        n = 1.0 / (C2 - 1.0)
        tau = n * s.k_in / s.eps_in
        x = sim.g.centers[0][0, 0, :]
        kx = s.k_in * (1.0 + x / tau) ** (-n)
        errs.append(np.abs(sim.k[0, 1, :] - kx).max() / s.k_in)
    assert errs[1] < 0.05
    assert 1.6 < errs[0] / errs[1] < 2.6


def test_decaying_turbulence_komega_first_order_convergence():
    # the paper's k-omega form without shear: U dk/dx = -beta* k omega and
    # U domega/dx = -C_beta1 omega^2, i.e. omega = omega0 / (1 + C_beta1 omega0 x / U)
    # and k = k0 (1 + C_beta1 omega0 x / U)^(-beta*/C_beta1); upwind converges at
    # first order
    errs = []
    for nx in (32, 64):
        s = synth.case_uniform_duct(nx=nx, ny=4, model="komega")
        sim = Simple(s)
        _converge(sim, tol=1e-11, maxit=3000)
        C = s.constants
        x = sim.g.centers[0][0, 0, :]
        t = 1.0 + C["beta_kw"] * s.omega_in * x / 1.0
        wx = s.omega_in / t
        kx = s.k_in * t ** (-C["Cmu"] / C["beta_kw"])
        errs.append(max(np.abs(sim.k[0, 1, :] - kx).max() / s.k_in, np.abs(sim.w[0, 1, :] - wx).max() / s.omega_in))
        # nu_t = k / omega exactly
        np.testing.assert_allclose(sim.nut, sim.k / sim.w, rtol=1e-14)
    assert errs[1] < 0.05
    assert 1.6 < errs[0] / errs[1] < 2.6


@pytest.mark.slow
@pytest.mark.parametrize("model", ["sst", "keps"])
def test_backward_facing_step_stays_bounded(model):
    # boundary cells above the step leave the forced group once y+ crosses
    # y+_lam; the in-solid cells behind them then join the pressure solve.  Their
    # pressure must be consistent with the fluid at that moment (identity rows
    # carry the mean of their coupled neighbours): with a stale value the
    # under-relaxed update produced a pressure jump and |u| grew past 100 U within
    # ten iterations for every turbulence model
    s = synth.case_bfs(model=model)
    sim = Simple(s)
    peak = 0.0
    for _ in range(120):
        sim.step()
        peak = max(peak, np.abs(sim.u[0]).max(), np.abs(sim.u[1]).max())
    assert np.isfinite(peak) and peak < 2.5, peak


def test_identity_pressure_rows_change_no_flux():
    # identity pressure rows (forced cells all of whose face neighbours are forced)
    # are decoupled from the solve; taking the mean pressure of their coupled
    # neighbours after the solve changes only their own pressure: one step from the
    # same state with and without it gives identical fluxes, velocities and
    # coupled-cell pressures
    import copy
    sim = Simple(synth.case_bfs(nx=80, ny=20, model="keps"))
    for _ in range(4):
        sim.step()
    other = copy.deepcopy(sim)
    other.identity_mean = False
    sim.step()
    other.step()
    g = sim.g
    alpha = sim.last["alpha"]
    iso = alpha.copy()
    for (d, s) in sim.dirs:
        iso &= ~g.has_neighbor(d, s) | g.neighbor(alpha, d, s, fill=False)
    assert iso.sum() > 20
    for d in range(2):
        np.testing.assert_array_equal(sim.phi[d], other.phi[d])
        np.testing.assert_array_equal(sim.u[d], other.u[d])
    np.testing.assert_array_equal(sim.p[~iso], other.p[~iso])
    np.testing.assert_array_equal(sim.k, other.k)
    # ... and the identity rows next to coupled cells do take a different value
    assert np.abs(sim.p[iso] - other.p[iso]).max() > 0.0
