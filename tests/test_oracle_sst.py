"""Pins of the oracle's turbulence closures in flows with known answers (no GPU):

* homogeneous shear (a frozen velocity field with uniform strain, convected at a
  uniform speed, so that each cell row is the same initial-value problem along
  x):
  - the production of k is nu_t (du/dy)^2 in every cell (2 S:S for simple shear);
  - standard k-epsilon: P/eps tends to (C2 - 1)/(C1 - 1), the equilibrium of the
    time-scale equation of the model in homogeneous shear (the steady upwind
    march reaches it exactly, since at geometric growth both equations give the
    same growth factor);
  - SST near a wall (F1 = F2 = 1): the shear-stress limiter is active and gives
    Bradshaw's relation nu_t |S| = a1 k exactly, and omega tends to the fixed
    point of its equation, gamma_1 a1 |S| / beta_1 (set 1 constants);
  - SST far from walls (F1 = F2 = 0): the production limiter holds P_k at
    10 beta* k omega where nu_t S^2 exceeds it, and omega tends to
    |S| sqrt(gamma_2 / beta_2) (set 2 constants; the cross-diffusion term vanishes
    at that fixed point);
* decaying turbulence in a uniform stream: SST with F1 = 1 follows the closed
  form of its inner set (the cross-diffusion term is switched off by 1 - F1);
  with F1 = 0 it follows the integral of U dk/dx = -beta* k omega,
  U domega/dx = -beta_2 omega^2 + 2 sigma_w2 (dk/dx)(domega/dx)/omega;
* the blending functions at their published limits and at hand-picked states.

Each pin is also run with a planted mistake in the closure (a swapped blend, a
wrong exponent, a dropped factor, |S|^2 for |S|, a misplaced source term), which
must make it fail."""

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synth
from oracle import closure
from oracle.solver import Simple

C = synth.DEFAULT_CONSTANTS


def _duct(nx, L, model, k_in, eps_in, om_in, nu=1e-8, ny=3):
    d = L / nx
    s = synth.CaseSpec(name="shear", dim=2, nx=nx, ny=ny, nz=1, x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=1.0,
                       bc=("inlet", "outlet", "slip", "slip", "empty", "empty"), u_in=(1.0, 0.0, 0.0),
                       k_in=k_in, eps_in=eps_in, omega_in=om_in, nu=nu, model=model)
    s.lam = np.zeros(s.shape)
    return s.validate()


def _frozen_shear(spec, S, dw=None, maxit=4000, tol=1e-11):
    """Iterates the oracle's turbulence stage alone on the frozen field
    u = (U0, S x): uniform convection along x (face fluxes of (U0, 0)) and a
    uniform strain dv/dx = S (boundary values of the linear field, so that the
    Gauss gradients are exact everywhere).  dw overrides the SST wall distance."""
    sim = Simple(spec)
    g = sim.g
    U0 = spec.u_in[0]
    x = g.centers[0]
    u = [np.full(g.shape, U0), S * x, np.zeros(g.shape)]
    xb = {-1: g.o[0], 1: g.o[0] + g.nx * g.dx}

    def face_value(c):
        def bv(d, s, uP):
            if c == 0:
                return np.full_like(uP, U0)
            if c == 1:
                return np.full_like(uP, S * xb[s]) if d == 0 else S * x[g.bnd(d, s)]
            return np.zeros_like(uP)
        return bv
    sim.u_face_value = face_value
    phi = g.zero_faces()
    phi[0][...] = U0 * g.area[0]
    if dw is not None:
        sim.geo.dw = np.full(g.shape, dw)
    n0 = np.zeros(0)
    alpha = np.zeros(g.shape, dtype=bool)
    first = None
    for it in range(maxit):
        res = {}
        sim.turbulence(u, phi, sim.k.copy(), sim.w.copy(), sim.nut.copy(), alpha, np.zeros(0, bool), n0, n0, n0,
                       n0, res)
        if first is None:
            first = {k: np.array(v, copy=True) for k, v in sim.last.items() if isinstance(v, np.ndarray)}
        if max(res.values()) < tol:
            break
    sim.first = first
    sim.converged = max(res.values()) < tol
    return sim


# ---------------------------------------------------------------- metrics
def keps_shear_metrics():
    """(max relative error of G = nu_t S^2 on the first pass, |P/eps - (C2-1)/(C1-1)|
    at the outlet, relative)"""
    S, kin, tau0 = 1.0, 1e-6, 2.5
    sim = _frozen_shear(_duct(128, 36.0, "keps", kin, kin / tau0, 1.0), S)
    assert sim.converged
    f = sim.first
    # initial nu_t = C_mu k^2 / eps = C_mu k tau0; simple shear: 2 S:S = S^2
    g_err = float(np.abs(f["G"] / (C["Cmu"] * kin * tau0 * S * S) - 1.0).max())
    r = sim.last["G"][0, 1, -1] / sim.w[0, 1, -1]
    target = (C["C2"] - 1.0) / (C["C1"] - 1.0)
    return g_err, abs(r / target - 1.0)


def sst_near_wall_metrics():
    """(max |nu_t S / (a1 k) - 1|, |omega_out / (gamma_1 a1 S / beta_1) - 1|)"""
    S = 5.0
    sim = _frozen_shear(_duct(128, 12.0, "sst", 1e-6, 1.0, S), S, dw=1e-12)
    assert sim.converged
    brad = float(np.abs(sim.nut * S / (C["a1"] * sim.k) - 1.0).max())
    w_star = C["gamma_1"] * C["a1"] * S / C["beta_1"]
    return brad, abs(sim.w[0, 1, -1] / w_star - 1.0)


def sst_far_field_metrics():
    """(max relative error of P_k against 10 beta* k omega where G exceeds it on the
    first pass, |omega_out / (S sqrt(gamma_2/beta_2)) - 1|)"""
    S = 5.0
    # first pass from omega = S/2: nu_t = k/omega, G = k S^2/omega = 10 k S > 0.9 k omega
    sim = _frozen_shear(_duct(64, 4.0, "sst", 1e-6, 1.0, 0.5 * S), S, maxit=1)
    f = sim.first
    lim = 10.0 * C["Cmu"] * 1e-6 * 0.5 * S
    assert np.all(f["G"] > lim)
    p_err = float(np.abs(f["Pk"] / lim - 1.0).max())
    sim = _frozen_shear(_duct(128, 6.0, "sst", 1e-6, 1.0, 2.0 * S), S)
    assert sim.converged
    w_star = S * np.sqrt(C["gamma_2"] / C["beta_2"])
    return p_err, abs(sim.w[0, 1, -1] / w_star - 1.0)


def sst_decay_errors(inner):
    """first-order convergence of decaying SST turbulence in a uniform stream:
    (error at nx = 32, error at nx = 64), errors relative to the inlet values.
    inner: F1 = 1 (tiny wall distance; closed form of set 1), else F1 = 0 (no
    wall; the ODE pair with the cross-diffusion term)"""
    errs = []
    for nx in (32, 64):
        s = synth.case_uniform_duct(nx=nx, ny=4, model="sst")
        s.omega_in = 50.0  # beta omega0 L / U = O(4): a strong decay
        sim = Simple(s)
        if inner:
            sim.geo.dw = np.full(sim.g.shape, 1e-12)
        for _ in range(3000):
            r = sim.step()
            if max(r["k"], r["omega"]) < 1e-11:
                break
        assert max(r["k"], r["omega"]) < 1e-11
        x = sim.g.centers[0][0, 0, :]
        k0, w0, U = s.k_in, s.omega_in, 1.0
        bs = C["Cmu"]
        if inner:
            t = 1.0 + C["beta_1"] * w0 * x / U
            wx, kx = w0 / t, k0 * t ** (-bs / C["beta_1"])
        else:
            def rhs(xx, y):
                k, w = y
                dk = -bs * k * w / U
                # U w' = -beta2 w^2 + 2 sigma_w2 k' w' / w, solved for w'
                dw_ = -C["beta_2"] * w * w / (U - 2.0 * C["sigma_w2"] * dk / w)
                return [dk, dw_]
            sol = solve_ivp(rhs, (0.0, x[-1]), [k0, w0], t_eval=x, rtol=1e-12, atol=1e-16)
            kx, wx = sol.y
        errs.append(max(np.abs(sim.k[0, 1, :] - kx).max() / k0, np.abs(sim.w[0, 1, :] - wx).max() / w0))
    return errs


def sst_inner_vs_komega():
    """max relative difference between SST with F1 = 1 (tiny wall distance) and the
    k-omega model given the constants of SST's inner set (Menter's inner layer is
    Wilcox's k-omega model: no cross-diffusion, set-1 coefficients), on decaying
    turbulence with k0 / U^2 = O(1), where a cross-diffusion term would show"""
    out = {}
    for model in ("sst", "komega"):
        s = synth.case_uniform_duct(nx=32, ny=4, model=model)
        s.k_in, s.omega_in = 1.0, 50.0
        s.constants.update(alpha_kw=C["gamma_1"], beta_kw=C["beta_1"], sigma_k_kw=1.0 / C["sigma_k1"],
                           sigma_w_kw=1.0 / C["sigma_w1"])
        sim = Simple(s)
        sim.geo.dw = np.full(sim.g.shape, 1e-12)
        for _ in range(40):
            sim.step()
        out[model] = sim
    a, b = out["sst"], out["komega"]
    return max(float(np.abs(a.k - b.k).max() / np.abs(b.k).max()), float(np.abs(a.w - b.w).max() / np.abs(b.w).max()))


def blend_metrics():
    """max deviation of the blending functions from their published values at
    hand-picked states (each state makes one term of arg1 / arg2 decide)"""
    nu = 1e-5
    dev = 0.0
    # inner and outer limits: F1 -> 1 as d -> 0, F1 -> 0 as d -> inf; the blended
    # constants are set 1 at F1 = 1 and set 2 at F1 = 0
    k, w = np.array([1e-2]), np.array([10.0])
    cd = np.array([1e-10])
    dev = max(dev, abs(closure.sst_f1(k, w, np.array([1e-9]), cd, nu, C)[0] - 1.0))
    dev = max(dev, abs(closure.sst_f1(k, w, np.array([1e9]), cd, nu, C)[0]))
    for a, b in (("sigma_k1", "sigma_k2"), ("sigma_w1", "sigma_w2"), ("beta_1", "beta_2"), ("gamma_1", "gamma_2")):
        dev = max(dev, abs(closure.sst_blend(np.array([1.0]), C, a, b)[0] - C[a]))
        dev = max(dev, abs(closure.sst_blend(np.array([0.0]), C, a, b)[0] - C[b]))
    # arg1 = sqrt(k)/(beta* omega d) = 0.8 (the viscous and cross-diffusion terms
    # do not decide): F1 = tanh(0.8^4)
    k, w = np.array([0.01]), np.array([1.0])
    d = np.sqrt(0.01) / (0.09 * 1.0 * 0.8)
    big_cd = np.array([1e-12])  # 4 sigma k/(CD d^2) huge: the min keeps the max term
    f1 = closure.sst_f1(k, w, np.array([d]), big_cd, 1e-9, C)[0]
    dev = max(dev, abs(f1 - np.tanh(0.8 ** 4)))
    # the cross-diffusion term decides: 4 sigma_w2 k / (CD d^2) = 0.5
    cdv = 4.0 * C["sigma_w2"] * 0.01 / (0.5 * d * d)
    f1 = closure.sst_f1(k, w, np.array([d]), np.array([cdv]), 1e-9, C)[0]
    dev = max(dev, abs(f1 - np.tanh(0.5 ** 4)))
    # F2: arg2 = 2 sqrt(k)/(beta* omega d) = 1.6 at the same state
    f2 = closure.sst_f2(k, w, np.array([d]), 1e-9, C)[0]
    dev = max(dev, abs(f2 - np.tanh(1.6 ** 2)))
    # the viscous term decides: 500 nu/(d^2 omega) = 1.2
    nu2 = 1.2 * d * d * 1.0 / 500.0
    f1 = closure.sst_f1(np.array([1e-12]), w, np.array([d]), big_cd, nu2, C)[0]
    dev = max(dev, abs(f1 - np.tanh(1.2 ** 4)))
    return dev


# ---------------------------------------------------------------- pins
def test_keps_homogeneous_shear_production_and_equilibrium():
    g_err, r_err = keps_shear_metrics()
    assert g_err < 1e-12
    assert r_err < 2e-4


def test_sst_near_wall_bradshaw_limiter_and_omega_fixed_point():
    brad, w_err = sst_near_wall_metrics()
    assert brad < 1e-12
    assert w_err < 1e-3


def test_sst_far_field_production_limiter_and_omega_fixed_point():
    p_err, w_err = sst_far_field_metrics()
    assert p_err < 1e-12
    assert w_err < 1e-3


@pytest.mark.parametrize("inner", [True, False])
def test_sst_decay_first_order_convergence(inner):
    e32, e64 = sst_decay_errors(inner)
    assert e64 < 0.05
    assert 1.6 < e32 / e64 < 2.6


def test_sst_inner_set_is_the_komega_model():
    assert sst_inner_vs_komega() < 1e-12


def test_sst_blending_functions():
    assert blend_metrics() < 1e-14


def test_sst_wall_distance_zero_gives_inner_limits():
    # in-solid cells have d = 0: every term of arg1 and arg2 is +inf, F1 = F2 = 1,
    # without a floating-point warning
    k, w = np.array([1e-3, 2.0]), np.array([5.0, 0.1])
    with np.errstate(all="raise"):
        assert np.all(closure.sst_f1(k, w, np.zeros(2), np.array([1e-10, 1e-3]), 1e-5, C) == 1.0)
        assert np.all(closure.sst_f2(k, w, np.zeros(2), 1e-5, C) == 1.0)


# ---------------------------------------------------------------- planted mistakes
def _swap_blend(F1, C_, inner, outer):
    return F1 * C_[outer] + (1.0 - F1) * C_[inner]


def _f1_square(k, w, dw, CDkw, nu, C_):
    bs = C_["Cmu"]
    with np.errstate(divide="ignore"):
        arg1 = np.minimum(np.maximum(np.sqrt(k) / (bs * w * dw), 500.0 * nu / (dw * dw * w)),
                          4.0 * C_["sigma_w2"] * k / (CDkw * dw * dw))
    return np.tanh(arg1 ** 2)


def _cd_no_blend(F1, kw, w, C_):
    return 2.0 * C_["sigma_w2"] * kw / w


def _nut_s2(k, w, S2, F2, C_):
    return C_["a1"] * k / np.maximum(C_["a1"] * w, S2 * F2)


def _production_half(nut, S2):
    return 0.5 * nut * S2


def _no_limit(G, k, w, C_):
    return G


MISTAKES = {
    "swapped_blend": ("sst_blend", _swap_blend, lambda: max(sst_near_wall_metrics()[1],
                                                             sst_far_field_metrics()[1]) > 1e-2),
    "tanh_arg1_squared": ("sst_f1", _f1_square, lambda: blend_metrics() > 1e-3),
    "cross_diffusion_without_1_minus_F1": ("sst_cd_term", _cd_no_blend, lambda: sst_inner_vs_komega() > 1e-3),
    "S2_for_sqrt_S2_in_limiter": ("sst_nut", _nut_s2, lambda: sst_near_wall_metrics()[0] > 1e-2),
    "production_S_colon_S": ("production", _production_half, lambda: keps_shear_metrics()[0] > 0.1),
    "no_production_limiter": ("sst_production_limit", _no_limit, lambda: sst_far_field_metrics()[0] > 0.1),
}


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_planted_closure_mistake_fails_a_pin(name, monkeypatch):
    fn, bad, fails = MISTAKES[name]
    monkeypatch.setattr(closure, fn, bad)
    assert fails()


@pytest.mark.parametrize("c1, c2", [(1.92, 1.44), (1.0, 1.92)])
def test_planted_keps_constant_mistake_fails_the_equilibrium(c1, c2):
    # C1 and C2 swapped, or the eps source without its C1: P/eps no longer tends to
    # the model's equilibrium (computed with the published constants)
    S, kin, tau0 = 1.0, 1e-6, 2.5
    spec = _duct(128, 36.0, "keps", kin, kin / tau0, 1.0)
    spec.constants["C1"], spec.constants["C2"] = c1, c2
    sim = _frozen_shear(spec, S, maxit=3000)
    r = sim.last["G"][0, 1, -1] / sim.w[0, 1, -1]
    assert abs(r / ((1.92 - 1.0) / (1.44 - 1.0)) - 1.0) > 0.05
