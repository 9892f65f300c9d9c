"""Writes the oracle's drag and lift of three instances of the batched NACA 0012
sweep, one on each of its grids (256 x 128, 512 x 256, 1024 x 512: sweep
instances 30, 31 and 29, angles 4.29, 4.76 and 3.81 degrees, the sweep's own
inlet turbulence), after N SIMPLE iterations from the initial conditions with a
direct pressure solve.  Only the oracle and the seeded input generator are
used.  The GPU test ``test_naca_sweep_forces_match_oracle_fixture`` iterates the
same instances with a pressure tolerance of 1e-13 and compares.

    python tests/golden/make_naca_forces.py [N]
"""

import json
import os
import sys
import time
import warnings

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.forces import body_force, coefficients  # noqa: E402
from oracle.solver import Simple  # noqa: E402

INSTANCES = (30, 31, 29)


def main(n_iter=10):
    warnings.simplefilter("ignore")
    specs = synth.naca_sweep_specs(64)
    out = {"iterations": n_iter, "instances": []}
    for j in INSTANCES:
        sp = specs[j]
        t0 = time.time()
        sim = Simple(sp)
        for _ in range(n_iter):
            sim.step()
        F = body_force(sim)
        cd, cl = coefficients(F, ref_area=1.0)
        rec = {"index": j, "name": sp.name, "grid": [sp.nx, sp.ny], "pressure": list(map(float, F["pressure"])),
               "viscous": list(map(float, F["viscous"])), "area": float(F["area"]), "bc_area": float(F["bc_area"]),
               "cd": float(cd), "cl": float(cl), "lambda_sha256": sp.lambda_sha256()}
        out["instances"].append(rec)
        print(sp.name, f"cd {cd:.6e} cl {cl:.6e}", f"{time.time() - t0:.0f}s", flush=True)
    path = os.path.join(HERE, f"naca_sweep_forces_it{n_iter}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 10)
