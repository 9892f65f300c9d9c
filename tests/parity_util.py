"""Helpers shared by the GPU parity tests: run the oracle and the HIP library on
the same seeded case and compare fields."""

from __future__ import annotations

import numpy as np

FIELDS = ("ux", "uy", "uz", "p", "k", "w", "nut", "phix", "phiy", "phiz")


def oracle_fields(sim):
    f = sim.fields()
    return {k: np.asarray(v).ravel() for k, v in f.items()}


def gpu_fields(solver):
    return {k: solver.get_field(k).cpu().numpy() for k in FIELDS}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.linalg.norm(b)
    num = np.linalg.norm(a - b)
    if den == 0.0:
        return num
    return num / den


# a field whose oracle values are all below ZERO_FIELD times the velocity scale
# (zero up to rounding, e.g. the cross-stream velocity of a uniform flow) is
# compared in absolute terms, scaled by that velocity scale
ZERO_FIELD = 1e-12


def compare(sim, solver, fields=FIELDS, dim=3, model="keps"):
    of = oracle_fields(sim)
    gf = gpu_fields(solver)
    scale = max(np.abs(of["ux"]).max(), np.abs(of["uy"]).max(), np.abs(of["uz"]).max(), 1e-300)
    out = {}
    for k in fields:
        if dim == 2 and k in ("uz", "phiz"):
            continue
        if model == "laminar" and k in ("k", "w", "nut"):
            continue
        if np.abs(of[k]).max() <= ZERO_FIELD * scale:
            out[k] = np.abs(gf[k] - of[k]).max() / scale
        else:
            out[k] = rel_l2(gf[k], of[k])
    return out


CELL_FIELDS = ("ux", "uy", "uz", "p", "k", "w", "nut")


def compare_at(sim, solver, cells, dim=3, model="keps"):
    """Largest error over the given cells (e.g. the immersed-boundary cells, a
    small fraction of the grid that whole-field norms dilute), relative to the
    largest magnitude of the field over the whole grid (the velocity scale for
    the velocity components)."""
    cells = np.asarray(cells, dtype=np.int64).ravel()
    of = oracle_fields(sim)
    gf = {k: solver.get_field(k).cpu().numpy() for k in CELL_FIELDS}
    vscale = max(np.abs(of["ux"]).max(), np.abs(of["uy"]).max(), np.abs(of["uz"]).max(), 1e-300)
    out = {}
    for k in CELL_FIELDS:
        if dim == 2 and k == "uz":
            continue
        if model == "laminar" and k in ("k", "w", "nut"):
            continue
        scale = vscale if k in ("ux", "uy", "uz") else max(np.abs(of[k]).max(), 1e-300)
        out[k] = float(np.abs(gf[k][cells] - of[k][cells]).max()) / scale if cells.size else 0.0
    return out
