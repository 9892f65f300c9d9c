"""Closure relations of the two-equation models, one function per relation.

TEST INFRASTRUCTURE: part of the CPU oracle (see the package docstring); only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

The paper lists its four closures in Sec. "Governing equations" (k-epsilon,
the k-omega model in its printed form, Menter's k-omega SST, realizable
k-epsilon) and gives the IB-specific terms; the model relations themselves are
the published ones:

* production of k from the mean strain rate, P = nu_t 2 S:S with
  S = (grad u + grad u^T)/2 (the Boussinesq production of every model here);
* Menter's SST (Menter 1992/1994): the blending function
  F1 = tanh(arg1^4), arg1 = min(max(sqrt(k)/(beta* omega d), 500 nu/(d^2 omega)),
  4 sigma_w2 k/(CD_kw d^2)), CD_kw = max(2 sigma_w2 grad k . grad omega / omega,
  floor); each coefficient phi = F1 phi_1 + (1 - F1) phi_2 (set 1 is the inner,
  near-wall k-omega set); the production limiter P_k = min(P, c_lim beta* k omega);
  the second blending function F2 = tanh(arg2^2),
  arg2 = max(2 sqrt(k)/(beta* omega d), 500 nu/(d^2 omega)); and the
  shear-stress limiter nu_t = a1 k / max(a1 omega, |S| F2), |S| = sqrt(2 S:S),
  which makes nu_t |S| = a1 k (Bradshaw's relation) where |S| F2 > a1 omega.

The wall distance d is 0 in the in-solid group (no fluid distance there).  At
d = 0 every term of arg1 and arg2 is +inf in IEEE arithmetic, so F1 = F2 = 1,
their limits at a wall; the divisions are done with the divide warning
silenced for that reason.  Those cells carry nu_t = 0 and a fixed omega row in
the solver, so the value only has to be finite.
"""

from __future__ import annotations

import numpy as np


def strain_rate_sq(Gu):
    """2 S:S from the gradient tensor Gu[i][j] = d u_j / d x_i"""
    S2 = np.zeros_like(Gu[0][0])
    for i in range(3):
        for j in range(3):
            sij = 0.5 * (Gu[i][j] + Gu[j][i])
            S2 = S2 + 2.0 * sij * sij
    return S2


def production(nut, S2):
    """Boussinesq production of k: nu_t 2 S:S"""
    return nut * S2


def sst_cross_diffusion(gk, gw, w, C):
    """CD_kw = max(2 sigma_w2 grad k . grad omega / omega, floor), and the dot
    product grad k . grad omega itself"""
    kw = gk[0] * gw[0] + gk[1] * gw[1] + gk[2] * gw[2]
    return np.maximum(2.0 * C["sigma_w2"] / w * kw, C["cd_floor"]), kw


def sst_cd_term(F1, kw, w, C):
    """cross-diffusion term of the omega equation, (1 - F1) 2 sigma_w2
    grad k . grad omega / omega (active in the outer, k-epsilon-like region)"""
    return (1.0 - F1) * 2.0 * C["sigma_w2"] * kw / w


def sst_f1(k, w, dw, CDkw, nu, C):
    """first blending function (1 near walls, 0 far from them)"""
    bs = C["Cmu"]
    with np.errstate(divide="ignore"):
        arg1 = np.minimum(np.maximum(np.sqrt(k) / (bs * w * dw), 500.0 * nu / (dw * dw * w)),
                          4.0 * C["sigma_w2"] * k / (CDkw * dw * dw))
    return np.tanh(arg1 ** 4)


def sst_blend(F1, C, inner, outer):
    """F1 phi_inner + (1 - F1) phi_outer for the named constants"""
    return F1 * C[inner] + (1.0 - F1) * C[outer]


def sst_production_limit(G, k, w, C):
    """P_k = min(G, c_lim beta* k omega)"""
    return np.minimum(G, C["c_lim"] * C["Cmu"] * k * w)


def sst_f2(k, w, dw, nu, C):
    """second blending function (for the shear-stress limiter)"""
    bs = C["Cmu"]
    with np.errstate(divide="ignore"):
        arg2 = np.maximum(2.0 * np.sqrt(k) / (bs * w * dw), 500.0 * nu / (dw * dw * w))
    return np.tanh(arg2 * arg2)


def sst_nut(k, w, S2, F2, C):
    """nu_t = a1 k / max(a1 omega, |S| F2), |S| = sqrt(2 S:S)"""
    return C["a1"] * k / np.maximum(C["a1"] * w, np.sqrt(S2) * F2)
