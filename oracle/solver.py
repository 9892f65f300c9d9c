"""The IB-aware steady SIMPLE iteration, one plain step at a time (FP64).

Follows the paper's solver loop (figure of the SIMPLE algorithm with the
additional immersed-boundary steps, and the paragraph describing it):

  1. set alpha_u, compute u_ib (from k and u of the previous iteration);
  2. momentum predictor of the RANS equation with the IB source f_ib;
  3. correction u <- u + alpha_u (u_ib - u);
  4. pressure corrector from the lambda-masked continuity equation;
  5. velocity (and flux) update;
  6. turbulence: alpha_omega, omega_ib (eps_ib) and P_ib; P_k <- P_ib; the
     omega (eps) equation with omega_ib enforced by fixing the rows of the
     alpha_omega cells; solve; k_ib; the k equation with S_ib; solve;
     k <- k + alpha_k (k_ib - k); turbulent viscosity.

Discretisation (upwind convection, Sec. "Numerical schemes"; central diffusion
with arithmetic-mean face diffusivity; Gauss gradients with linear face
interpolation; implicit under-relaxation).  Readings of the points the paper
leaves open are stated where they are used and collected in the design notes.

The linear systems are solved exactly as the iteration prescribes:
* momentum, k and eps/omega: ``n_sweeps`` red-black Gauss-Seidel sweeps
  (red = (i+j+k) even, updated first) from the previous values;
* pressure: a direct sparse solve (SuperLU) -- or, for grids too large for a
  direct factorisation, SciPy's conjugate gradients to a stated tolerance.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import Grid
from .geometry import precompute, IC, BC
from . import wallfn as wf
from . import realizable
from . import closure

DIRS = None  # filled per grid: list of (d, s)


class Simple:
    def __init__(self, spec, geo=None, solid_vel=None, p_solver="direct", p_rtol=1e-12, recorrect=True,
                 continuity="literal", identity_mean=True):
        self.spec = spec
        self.g = Grid(spec)
        self.C = dict(spec.constants)
        self.geo = geo if geo is not None else precompute(spec)
        self.lam = np.asarray(spec.lam, dtype=np.float64)
        g = self.g
        self.dirs = [(d, s) for d in g.axes for s in (-1, 1)]
        self.us = [np.zeros(g.shape) for _ in range(3)] if solid_vel is None else [np.asarray(a, float) for a in solid_vel]
        self.p_solver = p_solver
        self.p_rtol = p_rtol
        self.recorrect = recorrect
        self.continuity = continuity
        # identity pressure rows take the mean solved pressure of their coupled
        # face neighbours after each solve (off: they keep their value)
        self.identity_mean = identity_mean
        self.frozen_turbulence = False
        self.ic = self.geo.tag == IC
        self.bcm = self.geo.tag == BC
        self.bc_cells = self.geo.bc_cells
        self.ic_cells = self.geo.ic_cells
        self.k_in, self.eps_in, self.omega_in = wf.inlet_from_spec(spec, self.C)
        self.it = 0
        self.last = {}
        self.initial_conditions()

    # ------------------------------------------------------------ boundary data
    def solid_owner(self, d, s):
        """domain faces whose owner cell has lambda > 0 are walls inside the solid:
        zero gradient for every variable and no flux (paper, boundary-condition
        paragraph)"""
        return self.lam[self.g.bnd(d, s)] > 0.0

    def u_face_value(self, c):
        """boundary values of velocity component c for Gauss gradients"""
        u_in = self.spec.u_in

        def bv(d, s, uP):
            kind = self.g.face_kind(d, s)
            solid = self.solid_owner(d, s)
            if kind == "inlet":
                v = np.full_like(uP, u_in[c])
            elif kind == "noslip":
                v = np.zeros_like(uP)
            elif kind == "slip":
                v = np.zeros_like(uP) if c == d else uP.copy()
            else:  # outlet
                v = uP.copy()
            return np.where(solid, uP, v)
        return bv

    def p_face_value(self, d, s, pP):
        if self.g.face_kind(d, s) == "outlet":
            return np.where(self.solid_owner(d, s), pP, 0.0)
        return pP.copy()

    def scalar_face_value(self, inlet_value):
        def bv(d, s, psiP):
            if self.g.face_kind(d, s) == "inlet":
                return np.where(self.solid_owner(d, s), psiP, inlet_value)
            return psiP.copy()
        return bv

    # ------------------------------------------------------------ O2: start
    def initial_conditions(self):
        g, sp_ = self.g, self.spec
        self.u = [np.where(self.lam < 0.5, sp_.u_in[c], self.us[c]) for c in range(3)]
        if g.dim == 2:
            self.u[2] = np.zeros(g.shape)
        self.p = np.zeros(g.shape)
        if sp_.model in ("keps", "rkeps"):
            self.k = np.full(g.shape, self.k_in)
            self.w = np.full(g.shape, self.eps_in)
            self.nut = np.full(g.shape, self.C["Cmu"] * self.k_in ** 2 / self.eps_in)
        elif sp_.model in ("sst", "komega"):
            self.k = np.full(g.shape, self.k_in)
            self.w = np.full(g.shape, self.omega_in)
            self.nut = np.full(g.shape, self.k_in / self.omega_in)
        else:
            self.k = np.zeros(g.shape)
            self.w = np.zeros(g.shape)
            self.nut = np.zeros(g.shape)
        self.phi = self.interpolated_flux(self.u)

    def interpolated_flux(self, vec):
        """face fluxes from linear interpolation of a cell vector field; boundary
        faces: inlet u_in.S, outlet owner value, walls/slip/solid-owner 0"""
        g = self.g
        phi = g.zero_faces()
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
                phi[d][tuple(face)] = np.where(self.solid_owner(d, s), 0.0, val)
        return phi

    # ------------------------------------------------------------ operators
    def neighbor_coeffs(self, Gam, phi):
        """a_nb = D_f + max(-F_f, 0), D_f = mean(Gam) |S_f| / d_f (upwind convection
        in the bounded form a_P = sum a_nb); zero across boundary faces"""
        g = self.g
        anb = {}
        for (d, s) in self.dirs:
            F = g.outward_flux(phi, d, s)
            Gn = g.neighbor(Gam, d, s, fill=0.0)
            a = 0.5 * (Gam + Gn) * g.area[d] / g.delta[d] + np.maximum(-F, 0.0)
            a[~g.has_neighbor(d, s)] = 0.0
            anb[(d, s)] = a
        return anb

    def dirichlet_faces(self, Gam, phi, kinds, gam_face=None):
        """boundary coefficients a_b = Gam_b |S|/(d/2) + max(-F_b, 0) on the domain
        faces of the given kinds (owner lambda = 0 only); Gam_b is the owner value
        unless ``gam_face(d, s)`` supplies a face value; list of (d, s, kind, a_b)"""
        g = self.g
        out = []
        for (d, s) in self.dirs:
            kind = g.face_kind(d, s)
            if kind not in kinds:
                continue
            F = g.outward_flux(phi, d, s)[g.bnd(d, s)]
            Gb = Gam[g.bnd(d, s)] if gam_face is None else gam_face(d, s)
            a = Gb * g.area[d] / (0.5 * g.delta[d]) + np.maximum(-F, 0.0)
            a = np.where(self.solid_owner(d, s), 0.0, a)
            out.append((d, s, kind, a))
        return out

    def nbsum(self, anb, x):
        """sum_nb a_nb x_nb, faces taken in the order W, E, S, N, B, T"""
        g = self.g
        acc = np.zeros(g.shape)
        for (d, s) in self.dirs:
            acc = acc + anb[(d, s)] * g.neighbor(x, d, s)
        return acc

    def rbgs(self, aPr, anb, rhs, x, nsweeps, fixed=None):
        """red-black Gauss-Seidel: red cells ((i+j+k) even) first, then black"""
        g = self.g
        x = x.copy()
        free = np.ones(g.shape, dtype=bool) if fixed is None else ~fixed
        for _ in range(nsweeps):
            for color in (0, 1):
                upd = (rhs + self.nbsum(anb, x)) / aPr
                m = (g.color == color) & free
                x = np.where(m, upd, x)
        return x

    def norm_residual(self, aPr, anb, rhs, x, skip=None):
        """normalised residual sum|b - Ax| / (sum|Ax - A xbar| + sum|b - A xbar|),
        xbar = mean of x over all cells; the sums run over the rows that are
        actually solved (rows of forced or fixed cells, ``skip``, are left out)"""
        nb = self.nbsum(anb, x)
        one = self.nbsum(anb, np.ones(self.g.shape))
        Ax = aPr * x - nb
        xbar = x.mean()
        Axb = (aPr - one) * xbar
        keep = np.ones(self.g.shape, dtype=bool) if skip is None else ~skip
        num = np.abs(rhs - Ax)[keep].sum()
        den = np.abs(Ax - Axb)[keep].sum() + np.abs(rhs - Axb)[keep].sum()
        return float(num / (den + 1e-300))

    def grad_u(self, u):
        """gradient tensor G[i][j] = d u_j / d x_i (Gauss, linear interpolation)"""
        gr = [self.g.gauss_grad(u[c], self.u_face_value(c)) for c in range(3)]
        return [[gr[j][i] for j in range(3)] for i in range(3)]

    def transpose_term(self, nuEff, G):
        """explicit div(nuEff (grad u)^T), volume integrated:
        component c = sum_f nuEff_f (d u_n / d x_c)_f |S_f| (sign of the face normal n);
        face gradient = mean of the two cell gradients (owner value on domain faces)"""
        g = self.g
        T = [np.zeros(g.shape) for _ in range(3)]
        for c in g.axes:
            for (d, s) in self.dirs:
                if g.face_kind(d, s) == "empty":
                    continue
                Gc = G[c][d]
                has = g.has_neighbor(d, s)
                nu_f = np.where(has, 0.5 * (nuEff + g.neighbor(nuEff, d, s)), nuEff)
                gf = np.where(has, 0.5 * (Gc + g.neighbor(Gc, d, s)), Gc)
                T[c] = T[c] + s * g.area[d] * nu_f * gf
        return T

    def convection_correction(self, phi, u, G, scheme):
        """Higher-order momentum convection (the schemes of the paper's appendix on
        divergence schemes) as a deferred correction of the upwind matrix,
        evaluated from the previous iterate: per cell
        -sum over interior faces of F_out (u_f - u_C), with C the upwind and D the
        downwind cell of the face and u_f the scheme's face value:
          linear upwind: u_f = u_C + (x_f - x_C) . grad u_C;
          van Leer:      u_f = u_C + psi(r) (u_D - u_C) / 2,
                         psi(r) = (r + |r|) / (1 + |r|),
                         r = 2 (x_D - x_C) . grad u_C / (u_D - u_C) - 1 (r = 0 where
                         u_D = u_C; the face value is u_C there either way).
        grad u_C is the cell's Gauss gradient G[d][c] = d u_c / d x_d.  At the
        fixed point u = u_old the upwind terms cancel and the discretisation is
        the higher-order one.  One array per velocity component."""
        g = self.g
        out = [np.zeros(g.shape) for _ in range(3)]
        for c in g.axes:
            for (d, s) in self.dirs:
                has = g.has_neighbor(d, s)
                F = g.outward_flux(phi, d, s)
                up = F > 0.0  # this cell is upwind of the face
                uC = np.where(up, u[c], g.neighbor(u[c], d, s))
                uD = np.where(up, g.neighbor(u[c], d, s), u[c])
                gC = np.where(up, G[d][c], g.neighbor(G[d][c], d, s))
                dxC = np.where(up, s, -s) * 0.5 * g.delta[d]  # x_f - x_C along axis d
                if scheme == "linear_upwind":
                    uf = uC + dxC * gC
                elif scheme == "vanleer":
                    dCD = uD - uC
                    nz = dCD != 0.0
                    r = np.where(nz, 2.0 * (2.0 * dxC * gC) / np.where(nz, dCD, 1.0) - 1.0, 0.0)
                    psi = (r + np.abs(r)) / (1.0 + np.abs(r))
                    uf = uC + 0.5 * psi * dCD
                else:
                    raise ValueError(scheme)
                out[c] = out[c] - np.where(has, F * (uf - uC), 0.0)
        return out

    def ib_wall_coupling(self, cells, normal, y, yp, nuEff):
        """Change of the momentum diagonal of boundary cells on the logarithmic
        branch (the reading of the paper's high-Reynolds-number treatment, where
        the boundary velocity follows from the turbulent viscosity instead of the
        interpolation): each face shared with an in-solid neighbour couples the
        cell to the solid through D_w = (nu + nu_w) |n . e_f| A_f / y, the
        wall-function viscosity nu_w = nu (kappa y+ / ln(E y+) - 1) over the wall
        distance y with the projected face area, instead of the face-mean
        diffusivity over the centre distance, D_f = mean(nu_eff) A_f / d_f.
        Returns sum_f (D_w - D_f) per listed cell; the solid velocity of the cell
        goes to the right-hand side with the same coefficient, so that the face
        coupling is exact once the in-solid neighbour holds u_s.  Under the log law
        the momentum flux to the wall is then u_tau^2 per unit wall area."""
        g, C, nu = self.g, self.C, self.spec.nu
        nuw = nu + wf.nut_wall(yp, nu, C)
        ic = self.ic.ravel()
        ne = nuEff.ravel()
        idx = [np.asarray(a).ravel()[cells] for a in g.idx3]
        n_ = (g.nx, g.ny, g.nz)
        dD = np.zeros(len(cells))
        for (d, s) in self.dirs:
            q = idx[d] + s
            inside = (q >= 0) & (q < n_[d])
            nb = cells + s * (1 if d == 0 else (g.nx if d == 1 else g.nx * g.ny))
            nb = np.where(inside, nb, cells)
            wall = inside & ic[nb]
            Df = 0.5 * (ne[cells] + ne[nb]) * g.area[d] / g.delta[d]
            Dw = nuw * g.area[d] * np.abs(normal[:, d]) / y
            dD = dD + np.where(wall, Dw - Df, 0.0)
        return dD

    def wall_shear_rate_sq(self, u, cells, normal, y, us=None):
        """(|u_t,P - u_s,t| / y)^2 on the listed cells: the tangential part (to the
        unit normal) of the velocity relative to the wall velocity (0 for domain
        walls), over the wall distance y"""
        ur = np.stack([u[c].ravel()[cells] - (0.0 if us is None else us[c].ravel()[cells]) for c in range(3)],
                      axis=1)
        un = (ur * normal).sum(axis=1)
        tang = ur - un[:, None] * normal
        return (tang * tang).sum(axis=1) / (y * y)

    def pressure_gradient_V(self, p):
        """V (grad p)_P (Gauss; outlet faces p = 0, other faces zero gradient)"""
        gp = self.g.gauss_grad(p, self.p_face_value)
        return [self.g.V * gp[c] for c in range(3)]

    def pressure_coeffs(self, rAU):
        """c_f = mean(rAU) |S|/d on interior faces; c_b = rAU_P |S|/(d/2) on outlet faces"""
        g = self.g
        cint = {}
        for d in g.axes:
            cint[d] = 0.5 * (rAU[g.interior_lo(d)] + rAU[g.interior_hi(d)]) * g.area[d] / g.delta[d]
        cout = []
        for (d, s) in self.dirs:
            if g.face_kind(d, s) == "outlet":
                c = rAU[g.bnd(d, s)] * g.area[d] / (0.5 * g.delta[d])
                cout.append((d, s, np.where(self.solid_owner(d, s), 0.0, c)))
        return cint, cout

    def pressure_matrix(self, rAU):
        """SPD matrix of sum_f c_f (p_P - p_nb) + sum_outlet c_b p_P"""
        g = self.g
        cint, cout = self.pressure_coeffs(rAU)
        lin = np.arange(g.N).reshape(g.shape)
        rows, cols, vals = [], [], []
        diag = np.zeros(g.shape)
        for d in g.axes:
            L = lin[g.interior_lo(d)].ravel()
            R = lin[g.interior_hi(d)].ravel()
            c = cint[d].ravel()
            rows += [L, R]
            cols += [R, L]
            vals += [-c, -c]
            diag[g.interior_lo(d)] += cint[d]
            diag[g.interior_hi(d)] += cint[d]
        for (d, s, c) in cout:
            diag[g.bnd(d, s)] += c
        # rows without any coupling (forced cells surrounded by forced cells) are
        # identity rows; their right-hand side keeps p unchanged
        diag = np.where(diag == 0.0, 1.0, diag)
        rows.append(lin.ravel())
        cols.append(lin.ravel())
        vals.append(diag.ravel())
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(g.N, g.N))
        return A

    def solve_pressure(self, A, b, x0, coupled=None):
        if self.p_solver == "direct":
            return spla.splu(A.tocsc()).solve(b)
        dinv = 1.0 / A.diagonal()
        M = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
        # the relative tolerance refers to |b| over the coupled rows
        bn = np.linalg.norm(b if coupled is None else b[coupled])
        x, info = spla.cg(A, b, x0=x0, rtol=0.0, atol=self.p_rtol * bn, M=M, maxiter=100000)
        return x

    # ------------------------------------------------------------ O3: iteration
    def step(self):
        g, C, sp_ = self.g, self.C, self.spec
        geo = self.geo
        V = g.V
        u_old = [a.copy() for a in self.u]
        p_old = self.p.copy()
        k_old = self.k.copy()
        w_old = self.w.copy()
        nut_old = self.nut.copy()
        phi_old = [a.copy() for a in self.phi]
        res = {}
        turb = sp_.model != "laminar"
        bcc = self.bc_cells

        # ---- 3.1 IB-pre: u_tau, y+ from k_old; masks; u_ib ------------------
        if turb:
            utau = wf.u_tau_from_k(k_old.ravel()[bcc], C)
            yp = wf.y_plus(geo.yeff, utau, sp_.nu)
        else:
            utau = np.zeros(len(bcc))
            yp = np.zeros(len(bcc))
        alpha_bc = yp <= C["ylam"]
        wc = geo.wall_cells
        if turb:
            utau_w = wf.u_tau_from_k(k_old.ravel()[wc], C)
            yp_w = wf.y_plus(geo.wall_y, utau_w, sp_.nu)
        else:
            utau_w = np.zeros(len(wc))
            yp_w = np.zeros(len(wc))
        alpha = self.ic.copy().ravel()
        alpha[bcc[alpha_bc]] = True
        alpha = alpha.reshape(g.shape)
        uib = [self.us[c].copy() for c in range(3)]
        for c in g.axes:
            uflat = u_old[c].ravel()
            v1 = (geo.st1_w * uflat[geo.st1_idx]).sum(axis=1)
            v2 = (geo.st2_w * uflat[geo.st2_idx]).sum(axis=1)
            usS = self.us[c].ravel()[bcc]
            val = geo.L[:, 0] * usS + geo.L[:, 1] * v1 + geo.L[:, 2] * v2
            f = uib[c].ravel()
            f[bcc] = np.where(alpha_bc, val, f[bcc])
            uib[c] = f.reshape(g.shape)

        # ---- 3.2 momentum assembly ---------------------------------------
        nuEff = sp_.nu + nut_old
        anb = self.neighbor_coeffs(nuEff, phi_old)
        aP = sum(anb.values())

        def wall_gamma(d, s):
            # no-slip domain faces: nu plus the log-law wall viscosity from the
            # owner's y+ at half a cell width (laminar: nu)
            kind = g.face_kind(d, s)
            if kind != "noslip":
                return nuEff[g.bnd(d, s)]
            if not turb:
                return np.full(nuEff[g.bnd(d, s)].shape, sp_.nu)
            ypf = wf.y_plus(0.5 * g.delta[d], wf.u_tau_from_k(k_old[g.bnd(d, s)], C), sp_.nu)
            return sp_.nu + wf.nut_wall(ypf, sp_.nu, C)
        bnd = self.dirichlet_faces(nuEff, phi_old, ("inlet", "noslip"), gam_face=wall_gamma)
        bsrc = [np.zeros(g.shape) for _ in range(3)]
        for (d, s, kind, a) in bnd:
            aP[g.bnd(d, s)] += a
            for c in g.axes:
                ub = sp_.u_in[c] if kind == "inlet" else 0.0
                bsrc[c][g.bnd(d, s)] += a * ub
        # boundary cells on the logarithmic branch (not forced): their faces to
        # in-solid neighbours carry the wall shear of the wall function
        lg_cells = bcc[~alpha_bc]
        if turb and len(lg_cells):
            dD = self.ib_wall_coupling(lg_cells, geo.normal[~alpha_bc], geo.yeff[~alpha_bc], yp[~alpha_bc], nuEff)
            af_ = aP.ravel()
            af_[lg_cells] += dD
            aP = af_.reshape(g.shape)
            for c in g.axes:
                bf_ = bsrc[c].ravel()
                bf_[lg_cells] += dD * self.us[c].ravel()[lg_cells]
                bsrc[c] = bf_.reshape(g.shape)
        self.last["wall_dD"] = np.zeros(0) if not (turb and len(lg_cells)) else dD
        Gu = self.grad_u(u_old)
        T = self.transpose_term(nuEff, Gu)
        scheme = getattr(sp_, "conv_scheme", "upwind")
        if scheme != "upwind":
            Cc = self.convection_correction(phi_old, u_old, Gu, scheme)
            T = [T[c] + Cc[c] for c in range(3)]
        gP = self.pressure_gradient_V(p_old)
        urf = sp_.urf_u
        aPr = aP / urf
        af = alpha.astype(np.float64)
        RHS = [None] * 3
        for c in g.axes:
            b0 = T[c] + bsrc[c]
            ut = np.where(alpha, uib[c], u_old[c])
            forced = aP * ut - self.nbsum(anb, ut)
            RHS[c] = (1.0 - af) * (b0 - gP[c]) + af * forced + (1.0 - urf) / urf * aP * u_old[c]
            res["U" + "xyz"[c]] = self.norm_residual(aPr, anb, RHS[c], u_old[c], skip=alpha)

        # ---- 3.3 momentum solve + correction --------------------------------
        u = [np.zeros(g.shape) for _ in range(3)]
        for c in g.axes:
            uc = self.rbgs(aPr, anb, RHS[c], u_old[c], sp_.n_sweeps)
            u[c] = np.where(alpha, uc + 1.0 * (uib[c] - uc), uc)

        # ---- 3.4 pressure corrector ----------------------------------------
        # Forced cells carry no pressure gradient in their momentum row (f_ib
        # contains +grad p), so their velocity does not respond to pressure:
        # rAU = 0 there and H has no pressure term.
        rAU = np.where(alpha, 0.0, V / aPr)
        HbyA = [np.zeros(g.shape) for _ in range(3)]
        for c in g.axes:
            H = np.where(alpha, self.nbsum(anb, u[c]) + RHS[c], self.nbsum(anb, u[c]) + RHS[c] + gP[c])
            HbyA[c] = H / aPr
        phis = self.interpolated_flux(HbyA)
        div_star = sum(g.outward_flux(phis, d, s) for (d, s) in self.dirs)
        # (1 - lambda) div u = 0.  "literal": div u = 0 wherever 1 - lambda != 0 and
        # no condition where lambda = 1 (the Laplacian row keeps p harmonic there);
        # "weighted": the predictor divergence scaled by (1 - lambda) in every cell
        if self.continuity == "literal":
            bp = np.where(self.lam < 1.0, -div_star, 0.0)
        else:
            bp = -(1.0 - self.lam) * div_star
        A = self.pressure_matrix(rAU)
        iso = np.ones(g.shape, dtype=bool) & alpha
        for (d, s) in self.dirs:
            iso &= ~g.has_neighbor(d, s) | g.neighbor(alpha, d, s, fill=False)
        bp = np.where(iso, p_old, bp)  # identity rows: p unchanged
        bflat = bp.ravel()
        pflat_old = p_old.ravel()
        Ax = A @ pflat_old
        xb = pflat_old.mean()
        Axb = A @ np.full(g.N, xb)
        # normalised residual over the coupled rows (identity rows, whose right-hand
        # side is a pressure value, are left out like the forced rows of u and k)
        cp = ~iso.ravel()
        res["p"] = float(np.abs(bflat - Ax)[cp].sum()
                         / (np.abs(Ax - Axb)[cp].sum() + np.abs(bflat - Axb)[cp].sum() + 1e-300))
        p_sol = self.solve_pressure(A, bflat, pflat_old, coupled=cp).reshape(g.shape)
        # identity rows next to coupled cells take the mean solved pressure of their
        # coupled face neighbours (deeper identity rows keep p).  Without it their p
        # stays at a stale value; when a neighbour leaves the forced group (y+
        # crossing y+_lam) the cell joins the solve and its under-relaxed pressure
        # starts from that stale value, a jump that drove the backward-facing step
        # to divergence with every turbulence model.
        acc = np.zeros(g.shape)
        cnt = np.zeros(g.shape)
        for (d, s) in self.dirs:
            has = g.has_neighbor(d, s) & g.neighbor(~iso, d, s, fill=False)
            acc += np.where(has, g.neighbor(p_sol, d, s, fill=0.0), 0.0)
            cnt += has
        if self.identity_mean:
            p_sol = np.where(iso & (cnt > 0), acc / np.maximum(cnt, 1), p_sol)
        cint, cout = self.pressure_coeffs(rAU)
        phi = [a.copy() for a in phis]
        for d in g.axes:
            inner = [slice(None)] * 3
            inner[2 - d] = slice(1, -1)
            phi[d][tuple(inner)] -= cint[d] * (p_sol[g.interior_hi(d)] - p_sol[g.interior_lo(d)])
        for (d, s, c) in cout:
            face = [slice(None)] * 3
            face[2 - d] = 0 if s < 0 else -1
            phi[d][tuple(face)] += s * c * p_sol[g.bnd(d, s)]
        p = p_old + sp_.urf_p * (p_sol - p_old)
        gPn = self.pressure_gradient_V(p)
        for c in g.axes:
            u[c] = np.where(alpha, HbyA[c], HbyA[c] - gPn[c] / aPr)
            if self.recorrect:
                u[c] = np.where(alpha, u[c] + 1.0 * (uib[c] - u[c]), u[c])
        self.u, self.p, self.phi = u, p, phi
        self.last.update(dict(alpha=alpha, uib=uib, yp=yp, utau=utau, aP=aP, rAU=rAU,
                              HbyA=HbyA, phistar=phis, rhs_p=bp, p_sol=p_sol, RHS=RHS))

        # ---- 3.5 turbulence -------------------------------------------------
        # (frozen_turbulence: k, eps/omega and nu_t are held, so y+ and the masks
        # stay as well: the momentum-continuity system of the frozen-turbulence
        # adjoint)
        if turb and not self.frozen_turbulence:
            self.turbulence(u, phi, k_old, w_old, nut_old, alpha, alpha_bc, utau, yp, utau_w, yp_w, res)
            # velocity-based friction velocity from the log law (diagnostic)
            lg = yp > C["ylam"]
            ut = np.zeros(len(bcc))
            if lg.any():
                nrm = geo.normal
                ur = np.stack([u[c].ravel()[bcc] - self.us[c].ravel()[bcc] for c in range(3)], axis=1)
                un = (ur * nrm).sum(axis=1)
                tang = ur - un[:, None] * nrm
                mag = np.sqrt((tang * tang).sum(axis=1))
                ut[lg] = wf.loglaw_utau(mag[lg], geo.yeff[lg], sp_.nu, utau[lg], C)
            self.last["utau_U"] = ut
        self.it += 1
        self.last["res"] = res
        return res

    def turbulence(self, u, phi, k_old, w_old, nut_old, alpha, alpha_bc, utau, yp, utau_w, yp_w, res):
        g, C, sp_, geo = self.g, self.C, self.spec, self.geo
        V = g.V
        nu = sp_.nu
        bcc, icc = self.bc_cells, self.ic_cells
        rke = sp_.model == "rkeps"
        keps = sp_.model == "keps" or rke  # eps-based: inlet eps, eps_ib = Cmu k omega_ib, eps/k sink of k
        sst = sp_.model == "sst"
        urf = sp_.urf_t
        Gu = self.grad_u(u)
        S2 = closure.strain_rate_sq(Gu)  # 2 S:S
        G = closure.production(nut_old, S2)
        wc = geo.wall_cells
        alpha_w = (self.ic | self.bcm).ravel()
        alpha_w[wc] = True
        alpha_w = alpha_w.reshape(g.shape)
        kin = self.k_in
        win = self.eps_in if keps else self.omega_in
        if sst:
            # Menter's SST from the previous iterate: F1 (d_w = 0 in the in-solid
            # group gives F1 = 1 there, see oracle.closure), blended coefficients,
            # production limiter
            gk = g.gauss_grad(k_old, self.scalar_face_value(kin))
            gw = g.gauss_grad(w_old, self.scalar_face_value(win))
            CDkw, kw = closure.sst_cross_diffusion(gk, gw, w_old, C)
            F1 = closure.sst_f1(k_old, w_old, geo.dw, CDkw, nu, C)
            sig_k = closure.sst_blend(F1, C, "sigma_k1", "sigma_k2")
            sig_w = closure.sst_blend(F1, C, "sigma_w1", "sigma_w2")
            beta = closure.sst_blend(F1, C, "beta_1", "beta_2")
            gamma = closure.sst_blend(F1, C, "gamma_1", "gamma_2")
            Pk = closure.sst_production_limit(G, k_old, w_old, C)
        else:
            Pk = G.copy()

        # imposed omega (eps) and production
        yeff = geo.yeff
        om_bc = wf.omega_ib(yp, yeff, utau, nu, C)
        if keps:
            w_bc = C["Cmu"] * k_old.ravel()[bcc] * om_bc  # eps_ib = Cmu k_P omega_ib
        else:
            w_bc = om_bc
        nonic = ~self.ic
        w_ic = w_old[nonic].max() if nonic.any() else win  # max over boundary and free-stream cells
        # |n . grad u| of the logarithmic-branch production: the wall-normal
        # difference of the tangential velocity relative to the solid over the
        # wall distance, |u_t,P - u_s,t| / y (the wall-face normal gradient of the
        # wall-function form the paper adopts; it makes P_ib the equilibrium
        # production u_tau^3 / (kappa y) under the log law)
        P_bc = wf.production_ib(yp, Pk.ravel()[bcc],
                                self.wall_shear_rate_sq(u, bcc, geo.normal, yeff, self.us), nu, C)
        # first cells at no-slip domain walls: the same wall functions with y = d/2
        om_w = wf.omega_ib(yp_w, geo.wall_y, utau_w, nu, C)
        w_w = C["Cmu"] * k_old.ravel()[wc] * om_w if keps else om_w
        P_w = wf.production_ib(yp_w, Pk.ravel()[wc], self.wall_shear_rate_sq(u, wc, geo.wall_n, geo.wall_y), nu, C)
        wib = np.zeros(g.N)
        wib[icc] = w_ic
        wib[bcc] = w_bc
        wib[wc] = w_w
        wib = wib.reshape(g.shape)
        Pf = Pk.ravel().copy()
        Pf[icc] = 0.0
        Pf[bcc] = P_bc
        Pf[wc] = P_w
        Pk = Pf.reshape(g.shape)  # P_k <- P_ib on alpha_omega cells

        # omega (eps) equation, rows of alpha_omega cells fixed at the imposed value
        if rke:
            Gam = nu + nut_old / C["sigma_eps_rke"]
        elif keps:
            Gam = nu + nut_old / C["sigma_eps"]
        elif sst:
            Gam = nu + sig_w * nut_old
        else:  # k-omega in the paper's form
            Gam = nu + nut_old / C["sigma_w_kw"]
        anb = self.neighbor_coeffs(Gam, phi)
        aP = sum(anb.values())
        b0 = np.zeros(g.shape)
        for (d, s, kind, a) in self.dirichlet_faces(Gam, phi, ("inlet",)):
            aP[g.bnd(d, s)] += a
            b0[g.bnd(d, s)] += a * win
        if rke:
            # C1 S eps explicit, C2 eps^2 / (k + sqrt(nu eps)) linearised in eps
            src, sink = realizable.eps_terms(Gu, k_old, w_old, nu, C)
            aP = aP + sink * V
            b0 = b0 + src * V
        elif keps:
            aP = aP + C["C2"] * w_old / k_old * V
            b0 = b0 + C["C1"] * Pk * w_old / k_old * V
        elif not sst:
            # C_alpha1 (omega/k) P_k - C_beta1 omega^2, the sink linearised in omega
            aP = aP + C["beta_kw"] * w_old * V
            b0 = b0 + C["alpha_kw"] * (w_old / k_old) * Pk * V
        else:
            aP = aP + beta * w_old * V
            b0 = b0 + gamma * (w_old / k_old) * Pk * V
            CD = closure.sst_cd_term(F1, kw, w_old, C)
            b0 = b0 + np.where(CD > 0.0, CD * V, 0.0)
            aP = aP + np.where(CD < 0.0, -CD / w_old * V, 0.0)
        aPr = aP / urf
        rhs = b0 + (1.0 - urf) / urf * aP * w_old
        w0 = np.where(alpha_w, wib, w_old)
        rhs = np.where(alpha_w, aPr * wib, rhs)
        res["eps" if keps else "omega"] = self.norm_residual(aPr, anb, rhs, w0, skip=alpha_w)
        w = self.rbgs(aPr, anb, rhs, w0, sp_.n_sweeps, fixed=alpha_w)
        w = np.maximum(w, C["bound_frac"] * win)

        # k_ib: 0 in solid, quadratic with the wall-function surface value in boundary cells
        kib = np.zeros(g.N)
        kflat = k_old.ravel()
        v1 = (geo.st1_w * kflat[geo.st1_idx]).sum(axis=1)
        v2 = (geo.st2_w * kflat[geo.st2_idx]).sum(axis=1)
        kS = wf.k_vis(yp, C) * utau ** 2
        kib[bcc] = np.where(alpha_bc, geo.L[:, 0] * kS + geo.L[:, 1] * v1 + geo.L[:, 2] * v2, 0.0)
        kib = kib.reshape(g.shape)

        # k equation with S_ib
        if rke:
            Gam = nu + nut_old / C["sigma_k_rke"]
        elif keps:
            Gam = nu + nut_old / C["sigma_k"]
        elif sst:
            Gam = nu + sig_k * nut_old
        else:
            Gam = nu + nut_old / C["sigma_k_kw"]
        anb = self.neighbor_coeffs(Gam, phi)
        aP = sum(anb.values())
        b0 = np.zeros(g.shape)
        for (d, s, kind, a) in self.dirichlet_faces(Gam, phi, ("inlet",)):
            aP[g.bnd(d, s)] += a
            b0[g.bnd(d, s)] += a * kin
        if keps:
            aP = aP + w / k_old * V
        else:
            aP = aP + C["Cmu"] * w * V
        b0 = b0 + Pk * V
        af = alpha.astype(np.float64)
        kt = np.where(alpha, kib, k_old)
        forced = aP * kt - self.nbsum(anb, kt)
        aPr = aP / urf
        rhs = (1.0 - af) * b0 + af * forced + (1.0 - urf) / urf * aP * k_old
        res["k"] = self.norm_residual(aPr, anb, rhs, k_old, skip=alpha)
        k = self.rbgs(aPr, anb, rhs, k_old, sp_.n_sweeps)
        k = np.where(alpha, k + 1.0 * (kib - k), k)
        k = np.maximum(k, C["bound_frac"] * kin)

        # turbulent viscosity
        if rke:
            nut = realizable.c_mu(Gu, k, w, C) * k * k / w
        elif keps:
            nut = C["Cmu"] * k * k / w
        elif not sst:
            nut = k / w
        else:
            # (d_w = 0 in the in-solid group gives F2 = 1 there; those cells get
            # nu_t = 0 below)
            F2 = closure.sst_f2(k, w, geo.dw, nu, C)
            nut = closure.sst_nut(k, w, S2, F2, C)
        nf = nut.ravel().copy()
        lg = yp > C["ylam"]
        nf[bcc] = np.where(lg, wf.nut_wall(yp, nu, C), nf[bcc])
        nf[icc] = 0.0
        self.k, self.w, self.nut = k, w, nf.reshape(g.shape)
        self.last.update(dict(G=G, Pk=Pk, wib=wib, kib=kib, S2=S2, alpha_w=alpha_w))
        if sst:
            self.last["F1"] = F1

    def run(self, n, tol=0.0, callback=None):
        hist = []
        for _ in range(n):
            r = self.step()
            hist.append(r)
            if callback:
                callback(self)
            if tol > 0.0 and max(r.values()) <= tol:
                break
        return hist

    def fields(self):
        return dict(ux=self.u[0], uy=self.u[1], uz=self.u[2], p=self.p, k=self.k,
                    w=self.w, nut=self.nut, phix=self.phi[0], phiy=self.phi[1], phiz=self.phi[2])
