"""Realizable k-epsilon closure: the fourth turbulence model the paper lists
beside k-epsilon, k-omega and k-omega SST (Sec. "Governing equations", which
cites Shih et al. 1995 for it without restating its equations).

Test infrastructure: the CPU oracle the HIP library is checked against.  Only
the tests, the smoke check and the bench's CPU baseline use it.

The model as published by Shih et al. (1995):
  nu_t = C_mu k^2 / eps,  C_mu = 1 / (A0 + A_s U* k / eps),
  U* = sqrt(S_ij S_ij + Omega_ij Omega_ij),  A_s = sqrt(6) cos(phi),
  phi = arccos(sqrt(6) W) / 3,  W = S_ij S_jk S_ki / (S_ij S_ij)^(3/2);
  the eps equation gains the source C1 S eps with S = sqrt(2 S_ij S_ij),
  C1 = max(0.43, eta / (eta + 5)), eta = S k / eps, and the sink
  C2 eps^2 / (k + sqrt(nu eps)); the k equation is that of k-epsilon.

Readings (the paper is silent; each is listed in the design notes):
* S_ij is the deviatoric part of the strain rate of the discrete velocity
  gradient: the model is defined for solenoidal fields, whose strain rate is
  traceless, and only then does |sqrt(6) W| <= 1 hold;
* sqrt(6) W is clipped to [-1, 1] against rounding, and W = 0 where S_ij = 0
  (near sqrt(6) W = -1, axisymmetric compression, A_s has a square-root
  sensitivity to rounding: a change delta of W moves C_mu by ~sqrt(delta));
* the IB and wall treatment is that of k-epsilon (the paper implements all
  models alike), so eps_ib = Cmu k omega_ib keeps the constant Cmu = 0.09;
* the initial nu_t is that of k-epsilon (Cmu k^2 / eps); the variable C_mu
  acts from the first turbulence update on.
"""

from __future__ import annotations

import numpy as np


def strain_invariants(Gu):
    """Gu[i][j] = d u_j / d x_i (the solver's velocity gradient; the three
    invariants are the same for the transposed tensor).  Returns (S_ij S_ij,
    Omega_ij Omega_ij, S_ij S_jk S_ki) of the deviatoric strain rate S and the
    rotation rate Omega."""
    tr = Gu[0][0] + Gu[1][1] + Gu[2][2]
    S = [[0.5 * (Gu[i][j] + Gu[j][i]) - (tr / 3.0 if i == j else 0.0) for j in range(3)] for i in range(3)]
    Om = [[0.5 * (Gu[i][j] - Gu[j][i]) for j in range(3)] for i in range(3)]
    SS = sum(S[i][j] * S[i][j] for i in range(3) for j in range(3))
    OO = sum(Om[i][j] * Om[i][j] for i in range(3) for j in range(3))
    S3 = sum(S[i][j] * S[j][l] * S[l][i] for i in range(3) for j in range(3) for l in range(3))
    return SS, OO, S3


def c_mu(Gu, k, eps, C):
    """Variable C_mu = 1 / (A0 + A_s U* k / eps)."""
    SS, OO, S3 = strain_invariants(Gu)
    pos = SS > 0.0
    W = np.where(pos, S3 / np.where(pos, SS, 1.0) ** 1.5, 0.0)
    phi = np.arccos(np.clip(np.sqrt(6.0) * W, -1.0, 1.0)) / 3.0
    As = np.sqrt(6.0) * np.cos(phi)
    Ustar = np.sqrt(SS + OO)
    return 1.0 / (C["A0_rke"] + As * Ustar * k / eps)


def eps_terms(Gu, k, eps, nu, C):
    """Per-volume eps-equation terms: the explicit source C1 S eps and the
    coefficient C2 eps / (k + sqrt(nu eps)) of the sink, which multiplies eps."""
    SS, _, _ = strain_invariants(Gu)
    S = np.sqrt(2.0 * SS)
    eta = S * k / eps
    C1 = np.maximum(0.43, eta / (eta + 5.0))
    return C1 * S * eps, C["C2_rke"] * eps / (k + np.sqrt(nu * eps))
