"""Pins of the oracle's wall treatment in converged turbulent channels (no GPU).

A plane channel of height H = 1 between no-slip domain walls (body-fitted) or
between grid-aligned immersed solid bands (lambda in {0, 1}), uniform inflow,
Re_H = 5e4, 16 cells across: the first cells sit at y+ ~ 75, on the logarithmic
branch of the wall functions.  In the developed part of the converged flow:

* the log law u+ = ln(E y+) / kappa holds at the wall-function cells with
  u_tau = C_mu^(1/4) sqrt(k) (eq. for the friction velocity): the k equation at
  those cells balances the imposed production (eq. for P_ib) against the imposed
  dissipation, which is the equilibrium of the log layer;
* the wall shear of the momentum equation (from the developed pressure gradient,
  tau_w = -H/2 dp/dx) equals u_tau^2 (the momentum side of the wall function);
* the log-law friction velocity of the velocity (the FP64 Newton diagnostic)
  equals the k-based one;
* the immersed and the body-fitted channel give the same y+.

Tolerances are those of a sanity check (~10 %): the channel is only ~20 H long
and the discrete profile is not exactly logarithmic.  Planted mistakes in the
wall treatment (the cell-centred velocity gradient in P_ib; no wall-function
coupling of the immersed wall in the momentum rows; a wrong log-branch omega)
fail these pins."""

import numpy as np
import pytest

import synth
from oracle import wallfn
from oracle.solver import Simple

C = synth.DEFAULT_CONSTANTS
NU = 2e-5


def _channel(kind, model):
    if kind == "ib":
        s = synth.case_channel_ib(nx=320, n_fluid=16, n_solid=2, nu=NU, model=model)
    else:
        s = synth.case_channel_bodyfitted(nx=320, n_fluid=16, nu=NU, model=model)
    # inlet turbulence: I = 5 %, length scale 0.07 H
    s.k_in, s.eps_in, s.omega_in = None, None, None
    s.inlet_I, s.inlet_l = 0.05, 0.07
    return s


def _converge(sim, tol=1e-9, maxit=3000):
    for _ in range(maxit):
        r = sim.step()
        if max(r.values()) < tol:
            return True
    return False


def channel_metrics(kind, model, patch=None):
    """(u+ / (ln(E y+)/kappa) min and max, tau_w / u_tau^2, y+ mean) over the
    wall-function cells of the developed region 0.6 L .. 0.95 L"""
    s = _channel(kind, model)
    sim = Simple(s)
    if patch:
        patch(sim)
    assert _converge(sim)
    g = sim.g
    if kind == "ib":
        cells = sim.bc_cells
        yp, ut = sim.last["yp"], sim.last["utau"]
        lg = yp > C["ylam"]
        utU = sim.last["utau_U"]
    else:
        cells = sim.geo.wall_cells
        ut = wallfn.u_tau_from_k(sim.k.ravel()[cells], C)
        yp = wallfn.y_plus(sim.geo.wall_y, ut, s.nu)
        lg = yp > C["ylam"]
        utU = None
    i = cells % s.nx
    sel = lg & (i > 0.6 * s.nx) & (i < 0.95 * s.nx)
    assert sel.sum() > 100
    up = sim.u[0].ravel()[cells][sel] / ut[sel]
    ratio = up / (np.log(C["E"] * yp[sel]) / C["kappa"])
    p = sim.p[0]
    jm = p.shape[0] // 2
    i0, i1 = int(0.7 * s.nx), int(0.9 * s.nx)
    tau_w = -(p[jm, i1] - p[jm, i0]) / ((i1 - i0) * g.dx) * 1.0 / 2.0
    out = dict(lo=float(ratio.min()), hi=float(ratio.max()), tau=float(tau_w / np.mean(ut[sel] ** 2)),
               yp=float(np.mean(yp[sel])))
    if utU is not None:
        out["utauU"] = float(np.abs(utU[sel] / ut[sel] - 1.0).max())
    return out


@pytest.mark.parametrize("kind, model", [("ib", "keps"), ("bf", "keps"), ("ib", "sst")])
def test_log_law_at_wall_function_cells(kind, model):
    m = channel_metrics(kind, model)
    assert 0.9 < m["lo"] and m["hi"] < 1.1, m
    assert 0.9 < m["tau"] < 1.1, m
    if kind == "ib":
        assert m["utauU"] < 0.05, m
        # the body-fitted channel of the same Reynolds number has y+ = 73.8 at its
        # first cells (same wall distance d/2)
        assert 70.0 < m["yp"] < 80.0, m


def _cell_gradient_production(sim):
    # planted: |n . grad u| from the cell-centred Gauss gradient
    def shear(u, cells, normal, y, us=None):
        Gu = sim.grad_u(u)
        ng = np.zeros((len(cells), 3))
        for j in range(3):
            for i in range(3):
                ng[:, j] += normal[:, i] * Gu[i][j].ravel()[cells]
        return (ng * ng).sum(axis=1)
    sim.wall_shear_rate_sq = shear


def _no_wall_coupling(sim):
    # planted: the immersed wall coupled through the face-mean diffusivity only
    sim.ib_wall_coupling = lambda cells, normal, y, yp, nuEff: np.zeros(len(cells))


@pytest.mark.parametrize("patch, check", [
    (_cell_gradient_production, lambda m: m["hi"] > 1.5),
    (_no_wall_coupling, lambda m: m["tau"] < 0.6),
])
def test_planted_wall_treatment_mistakes_fail(patch, check):
    m = channel_metrics("ib", "keps", patch)
    assert check(m), m


def test_planted_log_branch_omega_mistake_fails(monkeypatch):
    # planted: C_mu^(1/4) instead of sqrt(C_mu) in the logarithmic omega branch
    good = wallfn.omega_ib

    def bad(yp, yeff, utau, nu, C_):
        C2 = dict(C_)
        C2["Cmu"] = C_["Cmu"] ** 0.5  # sqrt(C2["Cmu"]) = C_mu^(1/4)
        return np.where(yp <= C_["ylam"], good(yp, yeff, utau, nu, C_), good(yp, yeff, utau, nu, C2))
    monkeypatch.setattr(wallfn, "omega_ib", bad)
    m = channel_metrics("ib", "keps")
    assert not (0.9 < m["lo"] and m["hi"] < 1.1), m
