"""Writes the full-size oracle fixture of the Ahmed-like workload
(256 x 96 x 96 cells, k-omega SST, FP64): the state after N SIMPLE iterations
from the initial conditions, with the pressure solved to a relative residual
of 1e-13 (SciPy's Jacobi-preconditioned CG), sampled at every boundary and
in-solid cell and at a seeded sample of the other cells.

Only the oracle and the seeded input generator are used.  The GPU test
``test_full_size_iterated_state_matches_oracle_fixture`` runs the HIP path for
the same N iterations with the same pressure tolerance and compares the sampled
values (relative L2 <= 1e-9 per field).

    python tests/golden/make_ahmed_fixture.py [N]      (about 2 minutes per iteration)
"""

import os
import sys
import time
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.geometry import precompute  # noqa: E402
from oracle.solver import Simple  # noqa: E402

FIELDS = ("ux", "uy", "uz", "p", "k", "w", "nut")
N_SAMPLE = 6000
SEED = 20260


def main(n_iter=10):
    warnings.simplefilter("ignore")
    spec = synth.case_ahmed(scale=1)
    t0 = time.time()
    geo = precompute(spec)
    sim = Simple(spec, geo=geo, p_solver="cg", p_rtol=1e-13)
    print(f"precompute {time.time() - t0:.1f}s", flush=True)
    hist = []
    for it in range(n_iter):
        t1 = time.time()
        r = sim.step()
        hist.append([r[k] for k in ("Ux", "Uy", "Uz", "p", "k", "omega")])
        print(f"iteration {it + 1}: {time.time() - t1:.1f}s residuals {np.round(hist[-1], 6).tolist()}", flush=True)
    rng = np.random.default_rng(SEED)
    others = np.setdiff1d(np.arange(spec.ncells), np.concatenate([geo.bc_cells, geo.ic_cells]))
    sample = np.sort(np.concatenate([geo.bc_cells, geo.ic_cells, rng.choice(others, N_SAMPLE, replace=False)]))
    f = sim.fields()
    out = {k: np.asarray(f[k]).ravel()[sample] for k in FIELDS}
    path = os.path.join(HERE, f"ahmed_256x96x96_sst_it{n_iter}.npz")
    np.savez_compressed(path, cells=sample.astype(np.int64), iterations=np.int64(n_iter), p_rtol=1e-13,
                        lambda_sha256=np.array(spec.lambda_sha256()), residuals=np.array(hist), **out)
    print("wrote", path, f"{os.path.getsize(path) / 1024:.0f} KiB", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 10)
