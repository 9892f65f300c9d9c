"""Frozen-turbulence discrete adjoint of the converged momentum-continuity
system, with respect to the indicator field lambda (test infrastructure: part
of the CPU oracle).

The paper motivates the method by shape and topology optimisation with an
immersed boundary (Introduction and Conclusion); the adjoint gives the
gradient of a cost J (here the area-mean pressure on the inlet face, i.e. the
pressure drop to the outlet at p = 0) with respect to every lambda_i.

Frozen turbulence: nu_t, k and eps/omega of a RANS state are held, and with
them y+, the forcing masks alpha_u and every discrete decision of the
geometry (cell groups, the in-solid neighbour of each boundary cell, the
interpolation mode).  What remains is the fixed point of the SIMPLE iteration
(steps 3.1-3.4 of the solver) written as a residual R(x; lambda) = 0 in the
state x = (u, p, phi):

* momentum rows of cells that are not forced: the unrelaxed discrete momentum
  equation a_P u_P - sum_N a_N u_N - b_P + V (grad p)_P, with the upwind
  coefficients of the fluxes phi (at a fixed point the relaxation terms cancel);
* momentum rows of forced cells: u_P - u_ib,P(u; lambda) (the correction
  u <- u + alpha_u (u_ib - u) at its fixed point), with u_ib from the frozen
  interpolation stencils and the lambda-dependent normals, distances, weights;
* flux rows: phi_f minus the corrected flux phi*_f - c_f (p_N - p_P) of the
  pressure corrector, phi* the face interpolation of HbyA (eq. of the flux
  predictor), c_f = mean(rAU)|S|/d;
* pressure rows: the continuity sum of the fluxes on coupled cells with
  lambda < 1 (the literal reading of the lambda-masked continuity equation),
  the pressure-equation row on coupled cells with lambda = 1, and on the
  identity rows the mean of the coupled face neighbours (or the frozen value
  where there is none).

dR/dx is assembled exactly by complex-step differentiation (each column of a
structured colouring of the grid at once; the residual is written so that its
complex extension is analytic away from the upwind switch of zero fluxes);
dR/dlambda by central differences of R over colour groups of lambda, with the
geometry recomputed and every discrete decision checked unchanged.  The
adjoint solve (dR/dx)^T psi = dJ/dx is a direct sparse solve; the gradient is
dJ/dlambda = -psi^T dR/dlambda (J does not depend on lambda explicitly).
Pinned against central finite differences of J with the primal re-solved by
Newton's method (tests/test_oracle_adjoint.py).
"""

from __future__ import annotations

import copy

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import wallfn as wf
from .geometry import precompute


class FrozenFlow:
    """The frozen-turbulence momentum-continuity problem of a converged (or
    iterated) oracle state ``sim`` (a solver.Simple with upwind convection)."""

    def __init__(self, sim):
        if getattr(sim.spec, "conv_scheme", "upwind") != "upwind":
            raise ValueError("the adjoint is written for upwind momentum convection")
        self.sim = sim
        self.spec = sim.spec
        self.g = sim.g
        self.C = sim.C
        g = self.g
        self.nut = sim.nut.copy()
        self.k = sim.k.copy()
        self.alpha = sim.last["alpha"].copy()
        self.alpha_bc = self.alpha.ravel()[sim.bc_cells]
        self.yp = sim.last["yp"].copy()
        self.turb = sim.spec.model != "laminar"
        iso = self.alpha.copy()
        for (d, s) in sim.dirs:
            iso &= ~g.has_neighbor(d, s) | g.neighbor(self.alpha, d, s, fill=False)
        self.iso = iso
        cnt = np.zeros(g.shape)
        for (d, s) in sim.dirs:
            cnt += g.has_neighbor(d, s) & g.neighbor(~iso, d, s, fill=False)
        self.iso_cnt = cnt
        self.p_frozen = sim.p.copy()
        # layout of x: u_c for c in axes, p, phi_d for d in axes
        self.sizes = [g.N] * len(g.axes) + [g.N] + [sim.phi[d].size for d in g.axes]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])
        # inlet-face cells of the cost (fluid owners of the inlet face)
        self.cost_w = self._cost_weights()

    # ------------------------------------------------------------ packing
    def pack(self, u, p, phi):
        g = self.g
        parts = [u[c].ravel() for c in g.axes] + [p.ravel()] + [phi[d].ravel() for d in g.axes]
        return np.concatenate(parts)

    def unpack(self, x):
        g = self.g
        o = self.offsets
        na = len(g.axes)
        u = [np.zeros(g.shape, dtype=x.dtype) for _ in range(3)]
        for i, c in enumerate(g.axes):
            u[c] = x[o[i]:o[i + 1]].reshape(g.shape)
        p = x[o[na]:o[na + 1]].reshape(g.shape)
        phi = [np.zeros(a.shape, dtype=x.dtype) for a in self.sim.phi]
        for i, d in enumerate(g.axes):
            phi[d] = x[o[na + 1 + i]:o[na + 2 + i]].reshape(self.sim.phi[d].shape)
        return u, p, phi

    def state(self):
        s = self.sim
        return self.pack(s.u, s.p, s.phi)

    # ------------------------------------------------------------ pieces
    def _flux_of(self, vec):
        """face interpolation of a cell vector (the flux predictor's phi*),
        boundary faces as in the solver; keeps the element type"""
        g, sim = self.g, self.sim
        dt = vec[g.axes[0]].dtype
        phi = [np.zeros(a.shape, dtype=dt) for a in sim.phi]
        for d in g.axes:
            A = g.area[d]
            inner = [slice(None)] * 3
            inner[2 - d] = slice(1, -1)
            phi[d][tuple(inner)] = 0.5 * (vec[d][g.interior_lo(d)] + vec[d][g.interior_hi(d)]) * A
            for s in (-1, 1):
                face = [slice(None)] * 3
                face[2 - d] = 0 if s < 0 else -1
                kind = g.face_kind(d, s)
                owner = vec[d][g.bnd(d, s)]
                if kind == "inlet":
                    val = np.full_like(owner, self.spec.u_in[d] * A)
                elif kind == "outlet":
                    val = owner * A
                else:
                    val = np.zeros_like(owner)
                phi[d][tuple(face)] = np.where(sim.solid_owner(d, s), 0.0, val)
        return phi

    def _wall_gamma(self, d, s):
        g, sp_, C = self.g, self.spec, self.C
        nuEff = sp_.nu + self.nut
        if g.face_kind(d, s) != "noslip":
            return nuEff[g.bnd(d, s)]
        if not self.turb:
            return np.full(nuEff[g.bnd(d, s)].shape, sp_.nu)
        ypf = wf.y_plus(0.5 * g.delta[d], wf.u_tau_from_k(self.k[g.bnd(d, s)], C), sp_.nu)
        return sp_.nu + wf.nut_wall(ypf, sp_.nu, C)

    def _cost_weights(self):
        """J = area-mean pressure over the inlet face (fluid owners): weights on p"""
        g, sim = self.g, self.sim
        w = np.zeros(g.shape)
        for (d, s) in sim.dirs:
            if g.face_kind(d, s) != "inlet":
                continue
            m = np.zeros(g.shape, dtype=bool)
            m[g.bnd(d, s)] = True
            m &= self.spec.lam == 0.0
            w[m] += g.area[d]
        tot = w.sum()
        return (w / tot).ravel()

    def cost(self, x):
        u, p, phi = self.unpack(x)
        return float(np.real(self.cost_w @ p.ravel()))

    def cost_grad_x(self):
        gx = np.zeros(self.offsets[-1])
        na = len(self.g.axes)
        gx[self.offsets[na]:self.offsets[na + 1]] = self.cost_w
        return gx

    # ------------------------------------------------------------ residual
    def residual(self, x, geo, lam):
        """R(x; lambda) for the frozen problem (complex-safe in x); geo is the
        precompute of lam (with the frozen decisions)"""
        g, sim, sp_, C = self.g, self.sim, self.spec, self.C
        u, p, phi = self.unpack(x)
        V = g.V
        alpha = self.alpha
        af = alpha.astype(np.float64)
        bcc = sim.bc_cells
        nuEff = sp_.nu + self.nut
        # imposed velocity (frozen stencils, lambda-dependent weights)
        uib = [sim.us[c].astype(x.dtype) for c in range(3)]
        for c in g.axes:
            uf = u[c].ravel()
            v1 = (geo.st1_w * uf[geo.st1_idx]).sum(axis=1)
            v2 = (geo.st2_w * uf[geo.st2_idx]).sum(axis=1)
            val = geo.L[:, 0] * sim.us[c].ravel()[bcc] + geo.L[:, 1] * v1 + geo.L[:, 2] * v2
            f = uib[c].ravel().copy()
            f[bcc] = np.where(self.alpha_bc, val, f[bcc])
            uib[c] = f.reshape(g.shape)
        # momentum coefficients
        anb = sim.neighbor_coeffs(nuEff, phi)
        aP = sum(anb.values())
        bsrc = [np.zeros(g.shape, dtype=x.dtype) for _ in range(3)]
        for (d, s, kind, a) in sim.dirichlet_faces(nuEff, phi, ("inlet", "noslip"), gam_face=self._wall_gamma):
            aP[g.bnd(d, s)] += a
            for c in g.axes:
                ub = sp_.u_in[c] if kind == "inlet" else 0.0
                bsrc[c][g.bnd(d, s)] += a * ub
        lg_cells = bcc[~self.alpha_bc]
        if self.turb and len(lg_cells):
            dD = sim.ib_wall_coupling(lg_cells, geo.normal[~self.alpha_bc], geo.yeff[~self.alpha_bc],
                                      self.yp[~self.alpha_bc], nuEff)
            af_ = aP.ravel().copy()
            af_[lg_cells] += dD
            aP = af_.reshape(g.shape)
            for c in g.axes:
                bf_ = bsrc[c].ravel().copy()
                bf_[lg_cells] += dD * sim.us[c].ravel()[lg_cells]
                bsrc[c] = bf_.reshape(g.shape)
        Gu = sim.grad_u(u)
        T = sim.transpose_term(nuEff, Gu)
        gP = sim.pressure_gradient_V(p)
        urf = sp_.urf_u
        aPr = aP / urf
        Rm, HbyA = [], [np.zeros(g.shape, dtype=x.dtype) for _ in range(3)]
        for c in g.axes:
            b0 = T[c] + bsrc[c]
            ut = np.where(alpha, uib[c], u[c])
            forced = aP * ut - sim.nbsum(anb, ut)
            RHS = (1.0 - af) * (b0 - gP[c]) + af * forced + (1.0 - urf) / urf * aP * u[c]
            nb = sim.nbsum(anb, u[c])
            Rm.append(np.where(alpha, u[c] - uib[c], aPr * u[c] - nb - RHS).ravel())
            H = np.where(alpha, nb + RHS, nb + RHS + gP[c])
            HbyA[c] = H / aPr
        # corrected fluxes
        phis = self._flux_of(HbyA)
        rAU = np.where(alpha, 0.0, V / aPr)
        cint, cout = sim.pressure_coeffs(rAU)
        phin = [a.copy() for a in phis]
        for d in g.axes:
            inner = [slice(None)] * 3
            inner[2 - d] = slice(1, -1)
            phin[d][tuple(inner)] = phin[d][tuple(inner)] - cint[d] * (p[g.interior_hi(d)] - p[g.interior_lo(d)])
        for (d, s, cc) in cout:
            face = [slice(None)] * 3
            face[2 - d] = 0 if s < 0 else -1
            phin[d][tuple(face)] = phin[d][tuple(face)] + s * cc * p[g.bnd(d, s)]
        Rf = [(phi[d] - phin[d]).ravel() for d in g.axes]
        # pressure rows
        div = sum(g.outward_flux(phi, d, s) for (d, s) in sim.dirs)
        # (A p)_P = sum_f c_f (p_P - p_N) + sum_outlet c_b p_P (the pressure-equation row)
        Ap = np.zeros(g.shape, dtype=x.dtype)
        for d in g.axes:
            dp = cint[d] * (p[g.interior_lo(d)] - p[g.interior_hi(d)])
            Ap[g.interior_lo(d)] = Ap[g.interior_lo(d)] + dp
            Ap[g.interior_hi(d)] = Ap[g.interior_hi(d)] - dp
        for (d, s, cc) in cout:
            Ap[g.bnd(d, s)] = Ap[g.bnd(d, s)] + cc * p[g.bnd(d, s)]
        acc = np.zeros(g.shape, dtype=x.dtype)
        for (d, s) in sim.dirs:
            has = g.has_neighbor(d, s) & g.neighbor(~self.iso, d, s, fill=False)
            acc = acc + np.where(has, g.neighbor(p, d, s, fill=0.0), 0.0)
        idrow = np.where(self.iso_cnt > 0, p - acc / np.maximum(self.iso_cnt, 1), p - self.p_frozen)
        Rp = np.where(self.iso, idrow, np.where(lam < 1.0, div, Ap))
        return np.concatenate(Rm + [Rp.ravel()] + Rf)

    # ------------------------------------------------------------ derivatives
    def _colour_groups(self, block, K):
        """column indices of variable block `block`, grouped by a structured
        colouring with spacing K in every grid direction"""
        g = self.g
        o = self.offsets
        n = self.sizes[block]
        na = len(g.axes)
        if block <= na:  # cell variable
            shape = g.shape
        else:
            shape = self.sim.phi[g.axes[block - na - 1]].shape
        idx = np.arange(n).reshape(shape)
        k, j, i = np.meshgrid(*[np.arange(m) for m in shape], indexing="ij")
        col = (i % K) + K * (j % K) + K * K * (k % K)
        return [o[block] + idx[col == q] for q in np.unique(col)]

    def jacobian_x(self, x, geo, lam, K_u=17, K_other=9, h=1e-30):
        """dR/dx (sparse CSR) by complex steps over colour groups.  A velocity
        column reaches rows up to 8 cells away (the interpolation stencils of a
        forced cell's neighbours enter its HbyA, whose flux rows follow), a
        pressure or flux column up to 4: the colour spacings K_u, K_other keep
        every row within reach of one column of a group"""
        g = self.g
        na = len(g.axes)
        rows, cols, vals = [], [], []
        pos = self._positions()
        for b in range(len(self.sizes)):
            Kb = K_u if b < na else K_other
            for grp in self._colour_groups(b, Kb):
                xc = x.astype(np.complex128)
                xc[grp] += 1j * h
                d = np.imag(self.residual(xc, geo, lam)) / h
                nz = np.flatnonzero(d)
                if len(nz) == 0:
                    continue
                owner = self._nearest(pos[nz], pos[grp])
                rows.append(nz)
                cols.append(grp[owner])
                vals.append(d[nz])
        n = self.offsets[-1]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    def _positions(self):
        """(i, j, k) grid position of each unknown (face positions on the face
        lattice: face index i of a d-face sits between cells i-1 and i)"""
        g = self.g
        out = []
        na = len(g.axes)
        for b in range(len(self.sizes)):
            if b <= na:
                shape = g.shape
            else:
                shape = self.sim.phi[g.axes[b - na - 1]].shape
            k, j, i = np.meshgrid(*[np.arange(m) for m in shape], indexing="ij")
            out.append(np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1))
        return np.concatenate(out)

    @staticmethod
    def _nearest(rpos, cpos):
        """index into cpos of the column whose periodic-colour cell is nearest
        to each row (the colouring guarantees exactly one within reach)"""
        from scipy.spatial import cKDTree
        tree = cKDTree(cpos)
        _, ix = tree.query(rpos, k=1, p=np.inf)
        return ix

    def jacobian_lambda(self, x, lam, cells, K=9, h=1e-6):
        """dR/dlambda for the listed cells (dense columns, n x len(cells)) by
        central differences over colour groups of spacing K; the geometry is
        recomputed at lambda +- h and its discrete decisions checked unchanged.
        Returns the matrix and a mask of the columns whose decisions held."""
        g = self.g
        n = self.offsets[-1]
        out = np.zeros((n, len(cells)))
        ok = np.ones(len(cells), dtype=bool)
        base = self.sim.geo
        i, j, k = (np.asarray(a).ravel()[cells] for a in g.idx3)
        col = (i % K) + K * (j % K) + K * K * (k % K)
        pos = self._positions()
        cpos_all = np.stack([i, j, k], axis=1)
        for q in np.unique(col):
            sel = np.flatnonzero(col == q)
            res = []
            good = True
            for sgn in (1.0, -1.0):
                spec = copy.copy(self.spec)
                lam2 = np.array(lam, dtype=np.float64, copy=True)
                lam2.ravel()[cells[sel]] += sgn * h
                spec.lam = lam2
                geo = precompute(spec, with_wall_distance=False)
                if not self._same_decisions(base, geo):
                    good = False
                    break
                res.append(np.real(self.residual(x, geo, lam2)))
            if not good:
                ok[sel] = False
                continue
            d = (res[0] - res[1]) / (2.0 * h)
            nz = np.flatnonzero(np.abs(d) > 0.0)
            if len(nz) == 0:
                continue
            owner = self._nearest(pos[nz], cpos_all[sel])
            out[nz, sel[owner]] = d[nz]
        return out, ok

    @staticmethod
    def _same_decisions(a, b):
        return (np.array_equal(a.tag, b.tag) and np.array_equal(a.nstar, b.nstar)
                and np.array_equal(a.mode, b.mode) and np.array_equal(a.st1_idx, b.st1_idx)
                and np.array_equal(a.st2_idx, b.st2_idx))

    # ------------------------------------------------------------ solves
    def geometry(self, lam):
        """precompute of lam; raises when a discrete decision changes"""
        spec = copy.copy(self.spec)
        spec.lam = lam
        geo = precompute(spec, with_wall_distance=False)
        if not self._same_decisions(self.sim.geo, geo):
            raise ValueError("lambda changes a discrete decision of the geometry")
        return geo

    def newton(self, x, lam, tol=1e-13, maxit=40, lu=None):
        """solves R(x; lambda) = 0: Newton's method with the exact Jacobian, or
        (lu given: a factorisation of dR/dx at a nearby state) the chord
        iteration with that fixed factorisation; returns x and the history of
        max |R|"""
        geo = self.geometry(lam)
        hist = []
        for _ in range(maxit):
            R = np.real(self.residual(x, geo, lam))
            hist.append(float(np.abs(R).max()))
            if hist[-1] <= tol:
                break
            if lu is None:
                J = self.jacobian_x(x, geo, lam)
                x = x - spla.splu(J.tocsc()).solve(R)
            else:
                x = x - lu.solve(R)
        return x, hist

    def adjoint_gradient(self, x, lam, cells, lu=None):
        """dJ/dlambda on the listed cells (nan where a perturbation changes a
        discrete decision) and the adjoint state psi: (dR/dx)^T psi = dJ/dx,
        dJ/dlambda = -psi^T dR/dlambda.  lu: a SuperLU factorisation of dR/dx
        at x (computed when not given)"""
        if lu is None:
            lu = spla.splu(self.jacobian_x(x, self.sim.geo, lam).tocsc())
        psi = lu.solve(self.cost_grad_x(), trans="T")
        Rl, ok = self.jacobian_lambda(x, lam, cells)
        grad = -(psi @ Rl)
        grad[~ok] = np.nan
        return grad, psi


def frozen_from(spec, rans_iters, simple_iters=4000, tol=1e-11, p_rtol=1e-12):
    """a frozen-turbulence problem: the RANS iteration for rans_iters
    iterations, then the momentum-continuity iteration with the turbulence
    held until its residuals are below tol"""
    from .solver import Simple
    sim = Simple(spec, p_solver="direct", p_rtol=p_rtol)
    for _ in range(rans_iters):
        sim.step()
    sim.frozen_turbulence = True
    for _ in range(simple_iters):
        r = sim.step()
        rr = [v for k, v in r.items() if k in ("Ux", "Uy", "Uz", "p")]
        if max(rr) <= tol:
            break
    return FrozenFlow(sim)
