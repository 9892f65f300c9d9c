"""hfdib_forces_noalloc (the entry point for callers that cannot allocate)
against hfdib_forces through the C ABI, on two calls in a row, the second on a
smaller grid: the eight force values agree to 1e-13 relative (the partials are
summed in another order) and the call leaves no host wait behind (the output is
a device tensor read afterwards)."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _solver(spec, gpu):
    import torch
    from paper_2606_06135_amd import Solver
    s = Solver.from_spec(spec, device=gpu, p_rtol=1e-6, p_maxit=200)
    s.set_indicator(torch.from_numpy(spec.lam.ravel()))
    return s


def test_forces_noalloc_matches_forces(gpu):
    cases = [synth.case_naca(6.0, 512, 256), synth.case_small_body3d(model="keps", nu=1e-4)]
    assert cases[0].ncells > cases[1].ncells
    for spec in cases:
        s = _solver(spec, gpu)
        s.iterate(8)
        dev = s.forces_noalloc().cpu().numpy()
        f = s.forces()
        host = np.array(f["pressure"] + f["viscous"] + [f["area"], f["bc_area"]])
        scale = np.abs(host).max()
        assert scale > 0
        assert np.abs(dev - host).max() <= 1e-13 * scale, (spec.name, dev, host)
        assert abs(host[6]) > 0 and abs(host[7]) > 0
