"""Pins of the oracle's frozen-turbulence discrete adjoint (no GPU), on a 64 x 32
version of the bend-duct workload (k-epsilon, Re = 2000, a seeded design
field of intermediate lambda in the bend):

* the residual R(x; lambda) vanishes at the fixed point of the oracle's own
  SIMPLE iteration with the turbulence held (it is that fixed point, written
  as equations), and Newton's method with the assembled Jacobian converges from
  there in one step to rounding;
* the assembled Jacobian (complex steps over colour groups) equals central
  finite differences of R along random directions of the velocity and
  pressure;
* the adjoint gradient dJ/dlambda of the inlet mean pressure equals central
  finite differences (step 1e-6, the primal re-solved to 1e-13) on 20 seeded
  cells with intermediate lambda, to 1e-5 relative;
* planted mistakes (the Jacobian instead of its transpose in the adjoint
  solve; the imposed velocity's lambda dependence dropped) fail that pin.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import adjoint


@pytest.fixture(scope="module")
def bend():
    spec = synth.case_bend2d(64, 32, seed=12356)
    F = adjoint.frozen_from(spec, rans_iters=300)
    x0 = F.state()
    R0 = np.real(F.residual(x0, F.sim.geo, spec.lam))
    x, hist = F.newton(x0, spec.lam)
    J = F.jacobian_x(x, F.sim.geo, spec.lam)
    lu = spla.splu(J.tocsc())
    lam = spec.lam.ravel()
    cand = np.flatnonzero(((lam >= 0.05) & (lam <= 0.45)) | ((lam >= 0.55) & (lam <= 0.95)))
    grad, psi = F.adjoint_gradient(x, spec.lam, cand, lu=lu)
    ok = cand[~np.isnan(grad)]
    pick = np.sort(ok[np.random.default_rng(7).choice(len(ok), 20, replace=False)])
    fd = {}
    for c in pick:
        vals = []
        for sg in (1.0, -1.0):
            l2 = spec.lam.copy()
            l2.ravel()[c] += sg * 1e-6
            xs, hs = F.newton(x, l2, lu=lu)
            assert hs[-1] <= 1e-13
            vals.append(F.cost(xs))
        fd[c] = (vals[0] - vals[1]) / 2e-6
    return dict(spec=spec, F=F, x0=x0, R0=R0, x=x, hist=hist, J=J, lu=lu, cand=cand, grad=grad, pick=pick, fd=fd)


def test_residual_vanishes_at_the_simple_fixed_point(bend):
    # the frozen SIMPLE iteration was run to normalised residuals of 1e-11
    assert np.abs(bend["R0"]).max() < 1e-10
    assert bend["hist"][-1] <= 1e-13 and len(bend["hist"]) <= 3


def test_jacobian_matches_finite_differences(bend):
    F, x, J, spec = bend["F"], bend["x"], bend["J"], bend["spec"]
    o = F.offsets
    na = len(F.g.axes)
    rng = np.random.default_rng(3)
    for b in range(na + 1):  # velocity components and pressure
        v = np.zeros(x.size)
        v[o[b]:o[b + 1]] = rng.standard_normal(o[b + 1] - o[b])
        fd = (np.real(F.residual(x + 1e-6 * v, F.sim.geo, spec.lam))
              - np.real(F.residual(x - 1e-6 * v, F.sim.geo, spec.lam))) / 2e-6
        assert np.abs(J @ v - fd).max() <= 1e-7 * np.abs(fd).max(), b


def _errors(grad, cand, fd):
    out = []
    for c, f in fd.items():
        g = grad[np.flatnonzero(cand == c)[0]]
        out.append(abs(g - f) / abs(f))
    return np.array(out)


def test_adjoint_gradient_matches_central_differences(bend):
    err = _errors(bend["grad"], bend["cand"], bend["fd"])
    assert np.all(np.isfinite(err)) and len(err) == 20
    assert err.max() <= 1e-5, err.max()
    # the gradient is not trivially small
    assert np.abs(list(bend["fd"].values())).max() > 1e-2


def test_planted_adjoint_mistakes_fail(bend, monkeypatch):
    F, x, spec, cand = bend["F"], bend["x"], bend["spec"], bend["cand"]
    # the Jacobian itself instead of its transpose
    psi = bend["lu"].solve(F.cost_grad_x())
    Rl, ok = F.jacobian_lambda(x, spec.lam, cand)
    bad = -(psi @ Rl)
    bad[~ok] = np.nan
    assert np.nanmax(_errors(bad, cand, bend["fd"])) > 1e-2
    # the imposed velocity without its lambda dependence (the interpolation
    # weights and distances frozen at the base lambda)
    base = F.sim.geo
    orig = F.residual

    def frozen_weights(xx, geo, lam):
        return orig(xx, base, lam)
    monkeypatch.setattr(F, "residual", frozen_weights)
    bad, _ = F.adjoint_gradient(x, spec.lam, cand, lu=bend["lu"])
    assert np.nanmax(_errors(bad, cand, bend["fd"])) > 1e-2
