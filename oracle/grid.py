"""Uniform Cartesian finite-volume grid (cell centred, collocated).

Arrays are indexed a[k, j, i] (x fastest).  Physical axis d in {0: x, 1: y,
2: z} lives on array axis 2 - d.  In 2D the grid is one cell thick (nz = 1) and
the z faces are "empty": no flux and no diffusion cross them, and the cell
length scale is h = (dx dy)^(1/2) (the paper's V^(1/3) is read this way for
one-cell-thick 2D meshes).

Face flux arrays phi[d] hold the volumetric flux in the +d direction through the
n_d + 1 faces normal to d.
"""

from __future__ import annotations

import numpy as np

FACE_NAMES = ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax")


def ax(d):
    """array axis of physical axis d"""
    return 2 - d


def sl(d, s):
    """index tuple selecting slice ``s`` on physical axis d"""
    idx = [slice(None)] * 3
    idx[ax(d)] = s
    return tuple(idx)


class Grid:
    def __init__(self, spec):
        self.dim = spec.dim
        self.nx, self.ny, self.nz = spec.nx, spec.ny, spec.nz
        self.n = (spec.nx, spec.ny, spec.nz)
        self.o = (spec.x0, spec.y0, spec.z0)
        self.dx, self.dy, self.dz = spec.dx, spec.dy, spec.dz
        self.delta = (spec.dx, spec.dy, spec.dz)
        self.shape = (spec.nz, spec.ny, spec.nx)
        self.N = spec.nx * spec.ny * spec.nz
        self.axes = tuple(range(spec.dim))
        self.area = (spec.dy * spec.dz, spec.dx * spec.dz, spec.dx * spec.dy)
        self.V = spec.dx * spec.dy * spec.dz
        if spec.dim == 2:
            self.h = (spec.dx * spec.dy) ** 0.5
        else:
            self.h = self.V ** (1.0 / 3.0)
        self.bc = tuple(spec.bc)
        k, j, i = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        self.idx3 = (i, j, k)  # integer cell coordinates per physical axis
        self.centers = tuple(self.o[d] + (self.idx3[d] + 0.5) * self.delta[d] for d in range(3))
        self.color = (i + j + k) % 2  # red = 0 (updated first), black = 1

    # ---------------------------------------------------------------- faces
    def face_kind(self, d, s):
        """boundary kind of the domain face normal to d on side s (-1 low, +1 high)"""
        return self.bc[2 * d + (0 if s < 0 else 1)]

    def bnd(self, d, s):
        """index tuple of the boundary cells adjacent to the domain face (d, s)"""
        return sl(d, 0 if s < 0 else -1)

    def interior_lo(self, d):
        """cells on the low side of interior faces normal to d"""
        return sl(d, slice(0, -1))

    def interior_hi(self, d):
        """cells on the high side of interior faces normal to d"""
        return sl(d, slice(1, None))

    def neighbor(self, a, d, s, fill=0.0):
        """b[P] = a[P + s e_d]; ``fill`` where P + s e_d is outside the domain"""
        b = np.full_like(a, fill)
        if s > 0:
            b[self.interior_lo(d)] = a[self.interior_hi(d)]
        else:
            b[self.interior_hi(d)] = a[self.interior_lo(d)]
        return b

    def has_neighbor(self, d, s):
        m = np.zeros(self.shape, dtype=bool)
        m[self.interior_lo(d) if s > 0 else self.interior_hi(d)] = True
        return m

    def outward_flux(self, phi, d, s):
        """per cell: flux leaving the cell through its face (d, s)"""
        if s > 0:
            return phi[d][sl(d, slice(1, None))]
        return -phi[d][sl(d, slice(0, -1))]

    def zero_faces(self):
        return [np.zeros(tuple(self.shape[i] + (1 if i == ax(d) else 0) for i in range(3)))
                for d in range(3)]

    # ---------------------------------------------------------------- gradient
    def gauss_grad(self, psi, bvalue):
        """Gauss gradient with linear face interpolation:
        (grad psi)_P = (1/V) sum_f psi_f S_f, i.e. (psi_+ - psi_-)/delta_d per axis.

        ``bvalue(d, s, psiP)`` returns the boundary-face values on face (d, s)
        given the owner values psiP.  Returns a list of 3 arrays (z = 0 in 2D).
        """
        dt = np.result_type(psi.dtype, np.float64)  # (complex states of the adjoint's complex steps)
        g = [np.zeros(self.shape, dtype=dt) for _ in range(3)]
        for d in self.axes:
            fp = np.empty(self.shape, dtype=dt)
            fm = np.empty(self.shape, dtype=dt)
            fp[self.interior_lo(d)] = 0.5 * (psi[self.interior_lo(d)] + psi[self.interior_hi(d)])
            fm[self.interior_hi(d)] = fp[self.interior_lo(d)]
            fp[self.bnd(d, +1)] = bvalue(d, +1, psi[self.bnd(d, +1)])
            fm[self.bnd(d, -1)] = bvalue(d, -1, psi[self.bnd(d, -1)])
            g[d] = (fp - fm) / self.delta[d]
        return g
