"""Body forces, tile shapes and batched graph execution through the C ABI.

Forces are compared with the oracle's force integral on the same iterated
states; tile widths and batching must not change the iteration (parity with
the oracle, and bitwise equality between batched and isolated contexts)."""

import sys

import numpy as np
import pytest

import synth
from oracle.forces import body_force
from oracle.solver import Simple
from parity_util import compare

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solver(spec, gpu, stream=None, **kw):
    import torch
    from paper_2606_06135_amd import Solver
    kw.setdefault("p_rtol", 1e-13)
    kw.setdefault("p_maxit", 300)
    s = Solver.from_spec(spec, device=gpu, stream=stream, **kw)
    s.set_indicator(torch.from_numpy(spec.lam.ravel()))
    return s


FORCE_CASES = {
    "naca_128x64_sst": (lambda: synth.case_naca(6.0, 128, 64), 30),
    "sphere3d_keps": (lambda: synth.case_small_body3d(model="keps", nu=1e-4), 20),
    "channel_ib_laminar": (lambda: synth.case_channel_ib(nx=32, n_fluid=8), 30),
}


@pytest.mark.parametrize("name", list(FORCE_CASES))
def test_forces_match_oracle(gpu, name):
    mk, iters = FORCE_CASES[name]
    spec = mk()
    _say("forces", name, spec.ncells)
    sim = Simple(spec)
    for _ in range(iters):
        sim.step()
    s = _solver(spec, gpu)
    s.iterate(iters)
    F = body_force(sim)
    G = s.forces()
    # the net force is a sum of terms of either sign that can cancel (a symmetric
    # channel): tolerances scale with the size of the terms, max|p| or the largest
    # viscous component, times the surface area, and with the net value
    pscale = np.abs(sim.p).max() * F["area"]
    for key in ("pressure", "viscous"):
        a, b = np.asarray(F[key]), np.asarray(G[key])
        scale = max(np.abs(a).max(), pscale if key == "pressure" else 0.0, 1e-300)
        _say(f"  {key}: oracle {a}, gpu {b}")
        assert np.abs(a - b).max() <= 1e-8 * scale + 1e-15, (key, a, b)
    assert abs(F["area"] - G["area"]) <= 1e-12 * F["area"]
    assert abs(F["bc_area"] - G["bc_area"]) <= 1e-12 * max(F["bc_area"], 1e-300)


def test_naca_sweep_forces_match_oracle_fixture(gpu):
    # one instance of the batched sweep on each of its grids (256 x 128, 512 x 256,
    # 1024 x 512) at its own inlet turbulence: drag, lift and the force components
    # after 10 iterations against the stored oracle values
    # (tests/golden/make_naca_forces.py)
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "naca_sweep_forces_it10.json")
    with open(path) as fh:
        fx = json.load(fh)
    specs = synth.naca_sweep_specs(64)
    for rec in fx["instances"]:
        sp = specs[rec["index"]]
        assert sp.lambda_sha256() == rec["lambda_sha256"]
        s = _solver(sp, gpu, p_maxit=400)
        s.iterate(fx["iterations"])
        G = s.forces()
        cd, cl = s.coefficients(ref_area=1.0)
        scale = max(np.abs(rec["pressure"]).max(), np.abs(rec["viscous"]).max())
        dev = max(np.abs(np.array(G["pressure"]) - rec["pressure"]).max(),
                  np.abs(np.array(G["viscous"]) - rec["viscous"]).max()) / scale
        _say(f"  {sp.name}: cd {cd:.6e} (oracle {rec['cd']:.6e}), cl {cl:.6e} (oracle {rec['cl']:.6e}), "
             f"force deviation {dev:.1e}")
        assert dev <= 1e-9, (sp.name, dev)
        assert abs(cd - rec["cd"]) <= 1e-9 * max(abs(rec["cd"]), abs(rec["cl"]))
        assert abs(cl - rec["cl"]) <= 1e-9 * max(abs(rec["cd"]), abs(rec["cl"]))
        assert abs(G["area"] - rec["area"]) <= 1e-12 * rec["area"]


@pytest.mark.parametrize("width", [32, 64, 128, 256])
def test_tile_widths_keep_parity(gpu, width):
    # odd extents: partial tiles in x and y for every width
    spec = synth.case_small_body3d(nx=37, ny=13, nz=11, model="sst", nu=1e-4)
    sim = Simple(spec)
    for _ in range(15):
        sim.step()
    s = _solver(spec, gpu)
    s.set_tile_width(width)
    s.iterate(15)
    c = compare(sim, s, dim=spec.dim, model=spec.model)
    _say(f"width {width}:", {k: f"{v:.1e}" for k, v in c.items()})
    for k, v in c.items():
        assert v <= 1e-9, (width, k, v)


@pytest.mark.parametrize("width, depth, zfirst", [(64, 2, 0), (32, 4, 0), (128, 2, 1), (256, 1, 1)])
def test_tile_depths_keep_parity(gpu, width, depth, zfirst):
    # tiles spanning several planes (nz = 12 divisible by the depth), odd x and y extents
    spec = synth.case_small_body3d(nx=37, ny=13, nz=12, model="sst", nu=1e-4)
    spec.conv_scheme = "linear_upwind"
    sim = Simple(spec)
    for _ in range(15):
        sim.step()
    s = _solver(spec, gpu)
    s.set_tile_order(zfirst)
    s.set_tile_depth(depth)
    s.set_tile_width(width)
    s.iterate(15)
    c = compare(sim, s, dim=spec.dim, model=spec.model)
    _say(f"width {width} depth {depth} z-first {zfirst}:", {k: f"{v:.1e}" for k, v in c.items()})
    for k, v in c.items():
        assert v <= 1e-9, (width, depth, zfirst, k, v)


def test_invalid_tile_depth_rejected(gpu):
    from paper_2606_06135_amd.binding import HfdibError
    spec = synth.case_small_body3d(nx=24, ny=12, nz=10, model="laminar")
    s = _solver(spec, gpu)
    with pytest.raises(HfdibError):
        s.set_tile_depth(4)  # does not divide nz = 10
    with pytest.raises(HfdibError):
        s.set_tile_depth(3)
    s.set_tile_depth(2)
    with pytest.raises(HfdibError):
        s.set_tile_width(256)  # 256 x 2 > 256 cells
    s.iterate(2)
    assert np.isfinite(s.get_field("ux").cpu().numpy()).all()


def test_sampled_kernel_timing(gpu):
    # recording every 3rd of 7 iterations times iterations 0, 3 and 6 only: one
    # momentum assembly and one iteration span each; the timed launches leave
    # the results as they are
    spec = synth.case_small_body3d(model="sst", nu=1e-4)
    a = _solver(spec, gpu, p_rtol=1e-2, p_maxit=100)
    b = _solver(spec, gpu, p_rtol=1e-2, p_maxit=100)
    a.timing(True, 3)
    a.iterate(7)
    for name in ("mom_assemble", "mom_explicit", "iteration", "p_solve"):
        ms, cnt = a.timing_query(name)
        assert cnt == 3 and ms > 0.0, (name, cnt, ms)
    ms, cnt = a.timing_query("mom_sweep")
    assert cnt == 3 * 2 * spec.n_sweeps
    a.timing(False)
    b.iterate(7)
    for k in ("ux", "p", "k", "w"):
        np.testing.assert_array_equal(a.get_field(k).cpu().numpy(), b.get_field(k).cpu().numpy())


def test_autotune_leaves_the_state_alone(gpu):
    spec = synth.case_small_body3d(model="sst", nu=1e-4)
    s = _solver(spec, gpu)
    s.iterate(5)
    keys = ("ux", "uy", "uz", "p", "k", "w", "nut", "phix")
    before = {k: s.get_field(k).cpu().numpy() for k in keys}
    width, ms = s.autotune_tiles(reps=2)
    _say("autotune", width, ms)
    assert width in (32, 64, 128, 256) and all(v > 0 for v in ms.values())
    for k in keys:
        np.testing.assert_array_equal(s.get_field(k).cpu().numpy(), before[k])


def _batch_specs():
    return [synth.case_naca(3.0, 64, 32), synth.case_naca(-5.0, 128, 64),
            synth.case_small_body3d(model="keps", nu=1e-4)]


def _batched(gpu, specs, iters, pcg_iters, tol=1e-8):
    import torch
    from paper_2606_06135_amd import Batch
    solvers = [_solver(sp, gpu, stream=torch.cuda.Stream(gpu), p_rtol=1e-2, p_maxit=100) for sp in specs]
    b = Batch(solvers, pcg_iters=pcg_iters, tol=tol)
    b.run(iters)
    st = b.status()
    fields = [{k: s.get_field(k).cpu().numpy() for k in ("ux", "uy", "p", "k", "w", "nut")} for s in solvers]
    b.close()
    return st, fields, solvers


def test_batched_contexts_match_isolated_ones_bitwise(gpu):
    specs = _batch_specs()
    st, together, _ = _batched(gpu, specs, 10, 4)
    assert st["iters_done"] == [10, 10, 10] and not st["diverged"]
    for q, sp in enumerate(specs):
        st1, alone, _ = _batched(gpu, [sp], 10, 4)
        for k in together[q]:
            np.testing.assert_array_equal(together[q][k], alone[0][k])


def test_batch_with_converged_pressure_matches_oracle(gpu):
    spec = synth.case_naca(3.0, 64, 32)
    sim = Simple(spec)
    for _ in range(10):
        sim.step()
    st, fields, solvers = _batched(gpu, [spec], 10, 60)
    c = compare(sim, solvers[0], dim=spec.dim, model=spec.model)
    _say("batched vs oracle", {k: f"{v:.1e}" for k, v in c.items()})
    for k, v in c.items():
        assert v <= 1e-9, (k, v)


def test_batch_device_convergence_flag(gpu):
    spec = synth.case_small_body3d(model="sst", shape="box", nu=1e-5)
    st, _, solvers = _batched(gpu, [spec], 400, 8, tol=1e-6)
    _say("convergence flag", st)
    assert 0 < st["conv_iter"][0] < 400
    assert st["iters_done"][0] == 400
    assert max(st["residuals"][0]) <= 1e-6


def test_batch_arguments_and_shared_streams(gpu):
    # contexts may share a stream (each gets its own capture stream); a context
    # listed twice or the batch stream used by a context is rejected
    import ctypes as C
    import torch
    from paper_2606_06135_amd import Batch, HfdibError, lib
    st = torch.cuda.Stream(gpu)
    specs = [synth.case_naca(0.0, 64, 32), synth.case_naca(2.0, 64, 32)]
    a = _solver(specs[0], gpu, stream=st, p_rtol=1e-2, p_maxit=100)
    b = _solver(specs[1], gpu, stream=st, p_rtol=1e-2, p_maxit=100)
    bt = Batch([a, b], pcg_iters=3)
    bt.run(6)
    assert bt.status()["iters_done"] == [6, 6]
    bt.close()
    st2, alone, _ = _batched(gpu, [specs[1]], 6, 3)
    np.testing.assert_array_equal(b.get_field("ux").cpu().numpy(), alone[0]["ux"])
    with pytest.raises(HfdibError) as e:
        Batch([a, a], pcg_iters=2)
    assert e.value.status == -1
    with pytest.raises(HfdibError) as e:
        Batch([a], pcg_iters=2, stream=st)
    assert e.value.status == -1
