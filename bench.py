#!/usr/bin/env python3
"""Benchmark of the IB-aware steady SIMPLE iteration on one MI355X.

A step is one SIMPLE iteration of the whole hot path (IB pre-step, momentum
predictor and sweeps, IB correction, pressure-correction PCG-GMG solve, flux and
velocity update, SST transport with the imposed omega/P_k, k_ib and k correction,
turbulent viscosity, residuals).  Workload: the Ahmed-like bluff body in a
256 x 96 x 96 channel (2 359 296 cells), k-omega SST, FP64, synthetic lambda.

Besides the throughput line it measures the mixed-precision policy against
FP64 at equal residual: both runs start from identical initial conditions on
the 512 x 192 x 192 Ahmed-like workload (18.9 M cells) and iterate until the
maximum normalised residual reaches 1e-8; the wall time of each, the speedup
and the relative L2 difference of the converged fields are reported.

It also runs the batched angle-of-attack sweep: 64 NACA 0012 instances
(-10..+20 degrees, grids of 256 x 128, 512 x 256 and 1024 x 512 cells) iterated
together by one HIP graph (two SIMPLE iterations of every instance per launch,
fixed PCG count, device-side convergence flags), with tile widths chosen per
grid size by the autotuner, reporting instance-iterations per second and each
instance's drag and lift coefficients.

The same 256 x 96 x 96 workload is also timed under the other closures
(k-epsilon, k-omega, realizable k-epsilon), with y+ from y_perp alone, and with
the linear-upwind and van Leer momentum convection ("variants").

Prints one JSON line (see the fields below).  --gpus N > 1 is refused: the
library runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

# Algorithmic bytes per cell and launch of the timed kernel classes (every FP64
# array streamed once per pass at the granularity the pass needs, neighbours
# reused on chip; per-pass figures of the byte model of one SIMPLE iteration):
#   k / omega sweeps: 2 x 144 B/cell for n_s = 2 -> 36 per one-colour launch
#   momentum sweeps: 224 B/cell for n_s = 2 -> 56 per one-colour launch
#   momentum assembly: u,v,w,p,phi(3),nu_t, the explicit terms (3) (+flags) in,
#     b(3), a_P out: 121
#   explicit momentum terms (transpose viscous term; deferred convection
#     correction under the higher-order schemes) and the iteration means:
#     u,v,w,nu_t,p,k in, 3 terms out: 72
#   omega and k assembly: 2 x 80 -> 80 per launch
#   pressure operator apply: x, rAU (+flags) in, y out: 25
#   V-cycle half sweep (one colour): r and D^-1 of that colour (8), rAU (8),
#     flags (1), z of the other colour in and of this colour out (8): 25
#   V-cycle pre-smoothing pass from zero: r, D^-1, rAU (+flags) in, z and the
#     colour-split copy of r out: 41
#   restriction of the red rows' residuals: r of the red cells (4), z, rAU
#     (+flags) in, the coarse residual (1/8 of a cell) out: 22
#   apply with the direction update: z, d_old, rAU (+flags) in, d_new, q out: 41
#   CG vector update: x, d, r, q in, x, r out: 48
# (reduction finalize launches and the coarse levels of the V-cycle are bound by
# launch latency, not by bytes: they are timed but have no byte model)
ALGO_BYTES = {"scalar_sweep": 36.0, "mom_sweep": 56.0, "mom_assemble": 121.0, "mom_explicit": 72.0,
              "scalar_assemble": 80.0,
              "p_apply": 25.0, "p_smooth": 25.0, "p_presmooth": 41.0, "p_restrict": 22.0, "p_apply_dir": 41.0,
              "p_axpy": 48.0}
KERNEL = {"scalar_sweep": "k_scalar_sweep", "mom_sweep": "k_mom_sweep", "mom_assemble": "k_mom_assemble",
          "mom_explicit": "k_mom_explicit_z",
          "scalar_assemble": "k_scalar_assemble", "p_apply": "k_fine_apply", "p_smooth": "k_fine_smooth",
          "p_presmooth": "k_fine_presmooth", "p_restrict": "k_restrict_fine_res", "p_apply_dir": "k_fine_apply_dir",
          "p_axpy": "k_axpy2"}
PRESSURE_CLASSES = ("p_apply", "p_smooth", "p_presmooth", "p_restrict", "p_apply_dir", "p_axpy")
# the mixed policy's sweeps are one-colour launches of their own kernels; its
# V-cycle moves FP32 arrays
ALGO_BYTES_MIXED = dict(ALGO_BYTES, p_smooth=13.0, p_presmooth=21.0, p_restrict=12.0, p_apply_dir=37.0, p_axpy=52.0)
KERNEL_MIXED = dict(KERNEL, scalar_sweep="k_scalar_sweep32", mom_sweep="k_mom_sweep32")
KERNEL_SOURCES = {"k_scalar_sweep": "turbulence.hip", "k_scalar_sweep32": "turbulence.hip",
                  "k_scalar_assemble": "turbulence.hip", "k_mom_sweep": "simple.hip",
                  "k_mom_sweep32": "simple.hip", "k_mom_assemble": "simple.hip", "k_mom_explicit_z": "simple.hip"}
for _k in ("k_fine_apply", "k_fine_smooth", "k_fine_presmooth", "k_restrict_fine_res", "k_fine_apply_dir", "k_axpy2"):
    KERNEL_SOURCES[_k] = "pressure.hip"


def kernel_source_hash(kernel):
    """SHA-256 of the sources a kernel is built from (its file and the shared
    device headers): a stored traffic measurement is valid only while equal."""
    import hashlib
    csrc = os.path.join(HERE, "paper_2606_06135_amd", "csrc")
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES[kernel], "device_common.h", "hfdib_internal.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel, workload):
    """HBM-side traffic per launch (bytes) from the committed counter summary of
    this kernel and workload, or None when absent or taken on other sources."""
    path = os.path.join(HERE, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return float(vals["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", default="64x1x0",
                    help="tile shape of the full-grid kernels, WIDTHxDEPTHxZFIRST (default: the library's "
                         "64 x 4 x 1, x-first), or auto (the autotuner's choice from timed rounds of the "
                         "gradient, assembly and pressure operator); on the 2.36 M-cell case whole "
                         "iterations take the same time for every shape within 1 %")
    ap.add_argument("--case", default="ahmed", choices=["ahmed", "bfs", "ahmed2"])
    ap.add_argument("--p-rtol", type=float, default=1e-2)
    ap.add_argument("--p-sweeps", type=int, default=2,
                    help="red-black sweeps before and after the coarse correction on the fine pressure level")
    ap.add_argument("--p-sweeps-coarse", type=int, default=2,
                    help="the same on the coarse levels of the pressure V-cycle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true")
    ap.add_argument("--timing-every", type=int, default=10,
                    help="HIP-event kernel timing records every n-th iteration of the timed region (a recorded "
                         "iteration takes about 0.5 ms longer: the timestamps end the overlap of consecutive "
                         "launches)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--mixed-case", default="ahmed2", choices=["ahmed", "ahmed2", "none"])
    ap.add_argument("--mixed-tol", type=float, default=1e-8)
    ap.add_argument("--mixed-maxit", type=int, default=5000)
    ap.add_argument("--variant-steps", type=int, default=30,
                    help="timed iterations of each closure / scheme variant (0: skip)")
    ap.add_argument("--variant-warmup", type=int, default=10)
    ap.add_argument("--sweep-iters", type=int, default=600, help="iterations of the batched NACA sweep (0: skip)")
    ap.add_argument("--sweep-pcg", type=int, default=4, help="PCG iterations per pressure solve in the sweep")
    ap.add_argument("--sweep-p-sweeps", type=int, default=1,
                    help="red-black sweeps per side of the V-cycle in the sweep's pressure solves (with a fixed "
                         "PCG count, one sweep: 1.49x the instance rate of two, the same instances converge)")
    ap.add_argument("--sweep-warmup", type=int, default=20,
                    help="iterations of each sweep instance on its own (adaptive PCG) before the batch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2606_06135_amd import Solver

    log("building case", args.case)
    t0 = time.time()
    if args.case == "ahmed":
        spec = synth.case_ahmed(scale=1)
    elif args.case == "ahmed2":
        spec = synth.case_ahmed(scale=2)
    else:
        spec = synth.case_bfs()
    N = spec.ncells
    log(f"lambda ready in {time.time() - t0:.1f}s; cells {N}")
    dev = torch.device("cuda:0")
    solver = Solver.from_spec(spec, device=dev, p_rtol=args.p_rtol, p_maxit=100, precision=args.precision,
                              p_sweeps=args.p_sweeps, p_sweeps_coarse=args.p_sweeps_coarse)
    lam = torch.from_numpy(spec.lam.ravel()).to(dev)
    t0 = time.time()
    solver.set_indicator(lam)
    torch.cuda.synchronize()
    counts = solver.counts()
    log(f"set_indicator {time.time() - t0:.2f}s counts {counts}")

    # tile shape (set-up, outside the timed region): the given one, or (--tile auto)
    # for each tile order and each depth that divides nz the autotuner's fastest
    # width, the fastest of those kept
    if args.tile != "auto":
        w, d, z = (int(v) for v in args.tile.split("x"))
        solver.set_tile_order(z)
        solver.set_tile_width(64)
        solver.set_tile_depth(d)
        solver.set_tile_width(w)
        tile = {"width": w, "depth": d, "zfirst": z}
    else:
        best = None
        for zfirst in (0, 1):
            for depth in (1, 2, 4):
                if spec.dim != 3 or spec.nz % depth:
                    continue
                solver.set_tile_order(zfirst)
                solver.set_tile_width(64)
                solver.set_tile_depth(depth)
                w, ms = solver.autotune_tiles(reps=3)
                log(f"tile order z-first {zfirst} depth {depth}: ms per round by width {ms}")
                if best is None or ms[w] < best[0]:
                    best = (ms[w], w, depth, zfirst)
        solver.set_tile_order(best[3])
        solver.set_tile_width(64)
        solver.set_tile_depth(best[2])
        solver.set_tile_width(best[1])
        tile = {"width": best[1], "depth": best[2], "zfirst": best[3]}
    log(f"tile {tile}")

    done, res = solver.iterate(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {done} iterations, residuals {np.round(res, 5).tolist()}")

    if not args.no_timing:
        # kernel timing on a sample of the timed iterations (every n-th): recording
        # costs a few microseconds per timed launch
        solver.timing(True, args.timing_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, res = solver.iterate(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = solver.stats()
    log(f"timed {done} iterations in {elapsed:.3f}s; residuals {np.round(res, 6).tolist()}; "
        f"PCG iterations {stats[0]:.0f} (max {stats[2]:.0f})")
    finite = all(np.isfinite(res))

    roof = None
    roof_all = []
    kern = {}
    psolve_hbm = None
    if not args.no_timing:
        for name in ("p_apply", "mom_sweep", "mom_assemble", "mom_explicit", "scalar_sweep", "scalar_assemble",
                     "p_solve", "iteration", "p_smooth", "p_presmooth", "p_restrict", "p_apply_dir", "p_axpy",
                     "p_coarse",
                     "finalize"):
            ms, cnt = solver.timing_query(name)
            kern[name] = (ms, cnt)
        solver.timing(False)
        log("kernel timing (ms total, launches): " + ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in kern.items()))
        algo, knames = (ALGO_BYTES, KERNEL) if args.precision == "fp64" else (ALGO_BYTES_MIXED, KERNEL_MIXED)
        cand = {k: kern[k] for k in algo if kern[k][1] > 0}
        workload = spec.name + "_" + spec.model + "_" + args.precision
        it_ms = max(kern["iteration"][0], 1e-12)

        def roofline_of(cls):
            ms, cnt = cand[cls]
            avg_s = ms / 1e3 / cnt
            achieved = algo[cls] * N / avg_s / 1e9
            kname = knames[cls]
            traffic = stored_traffic(kname, workload) if args.precision == "fp64" else None
            return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(achieved / PEAK_HBM_GBS, 4),
                    "traffic": None if traffic is None else round(traffic),
                    "kernel": kname, "avg_launch_us": round(avg_s * 1e6, 2),
                    "algorithmic_bytes_per_cell": algo[cls], "timed_every_nth_iteration": args.timing_every,
                    "share_of_iteration": round(ms / it_ms, 4)}
        if cand:
            # the dominant kernel: the largest total time in the timed iterations
            dom = max(cand, key=lambda k: cand[k][0])
            roof = roofline_of(dom)
            roof_all = [roofline_of(k) for k in sorted(cand, key=lambda k: -cand[k][0])]
        # the pressure solve as a whole: algorithmic bytes of the fine-level
        # kernels it ran (coarse levels and reductions not counted) over its time,
        # and the per-CG-iteration byte model of the minimal design (190 B/cell)
        ps_ms, ps_cnt = kern["p_solve"]
        if ps_cnt > 0:
            nbytes = sum(algo[k] * N * kern[k][1] for k in PRESSURE_CLASSES if k in algo)
            ach = nbytes / (ps_ms / 1e3) / 1e9
            n_cg_timed = kern["p_apply_dir"][1] + kern["p_apply"][1]
            ach190 = 190.0 * N * n_cg_timed / (ps_ms / 1e3) / 1e9
            share = {k: round(kern[k][0] / ps_ms, 4) for k in
                     ("p_smooth", "p_presmooth", "p_restrict", "p_apply", "p_apply_dir", "p_axpy", "p_coarse")}
            psolve_hbm = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": round(ach / PEAK_HBM_GBS, 4),
                          "bytes_per_cell_per_cg_iteration": round(nbytes / max(n_cg_timed, 1) / N, 1),
                          "achieved_at_190_B_per_cell_per_cg_iteration": round(ach190, 1),
                          "frac_at_190": round(ach190 / PEAK_HBM_GBS, 4),
                          "ms_per_solve": round(ps_ms / ps_cnt, 4), "cg_iterations_timed": n_cg_timed,
                          "share_of_solve": share,
                          "finalize_ms_per_iteration": round(kern["finalize"][0] / max(kern["iteration"][1], 1), 4),
                          "p_sweeps": [args.p_sweeps, args.p_sweeps_coarse]}

    # whole-iteration %HBM peak with the per-iteration byte model of the minimal
    # fused design (3-D SST, FP64): 1178 B/cell for everything but the pressure
    # solve, 190 B/cell per CG iteration (N_cg measured over the timed region)
    n_cg = stats[0] / max(done, 1)
    bpc = 1178.0 + 190.0 * n_cg
    ach = bpc * N * done / elapsed / 1e9
    iteration_hbm = {"bytes_per_cell": round(bpc, 1), "cg_iters_per_step": round(n_cg, 3),
                     "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(ach / PEAK_HBM_GBS, 4)}
    value = N * done / elapsed
    del solver
    torch.cuda.empty_cache()
    mixed = None
    if args.mixed_case != "none":
        mixed = mixed_vs_fp64(args)
    var = None
    if args.variant_steps > 0 and args.case == "ahmed":
        var = variants(args)
    sweep = None
    if args.sweep_iters > 0:
        sweep = naca_sweep(args)
    hbm_ref = hbm_reference()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, args.p_rtol)

    out = {
        "metric": "SIMPLE cell-iters/s at 2.4M cells, %HBM peak; mixed-vs-FP64 at equal residual",
        "value": value,
        "unit": "cell-iters/s",
        "n_gpus": 1,
        "steps": done,
        "warmup": args.warmup,
        "ms_per_step": elapsed / done * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": spec.name + "_" + spec.model, "cells": N, "model": "k-omega SST" if spec.model == "sst"
                   else spec.model, "precision": args.precision, "p_rtol": args.p_rtol, "n_sweeps": spec.n_sweeps,
                   "boundary_cells": counts["bc"], "insolid_cells": counts["ic"], "tile": tile,
                   # the momentum assembly's own launch shape (3-D, nz a multiple of 4)
                   "assembly_tile": ("32x2x4 z-first" if spec.dim == 3 and spec.nz % 4 == 0 else "as tile"),
                   "pcg_iters_per_step": round(stats[0] / max(done, 1), 2), "finite": bool(finite),
                   "final_residuals": [float(x) for x in res]},
        "roofline": roof,
        "roofline_kernels": roof_all,
        "pressure_solve_hbm": psolve_hbm,
        "hbm_reference": hbm_ref,
        "iteration_hbm": iteration_hbm,
        "cpu_baseline": cpu,
        "mixed_vs_fp64": mixed,
        "naca_sweep": sweep,
        "variants": var,
    }
    print(json.dumps(out), flush=True)


def mixed_vs_fp64(args):
    """Time to the residual target in FP64 and under the mixed policy from the
    same initial conditions, and the difference of the converged fields."""
    import numpy as np
    import torch
    import synth
    from paper_2606_06135_amd import Solver
    spec = synth.case_ahmed(scale=2 if args.mixed_case == "ahmed2" else 1)
    dev = torch.device("cuda:0")
    lam = torch.from_numpy(spec.lam.ravel()).to(dev)
    runs, fields = {}, {}
    for prec in ("fp64", "mixed"):
        s = Solver.from_spec(spec, device=dev, p_rtol=args.p_rtol, p_maxit=100, precision=prec)
        s.set_indicator(lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, res = s.iterate(args.mixed_maxit, args.mixed_tol, 25)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        runs[prec] = {"iterations": done, "seconds": round(dt, 3), "max_residual": max(res),
                      "ms_per_iteration": round(dt / done * 1e3, 3),
                      "cell_iters_per_s": spec.ncells * done / dt, "converged": max(res) <= args.mixed_tol}
        log(f"{spec.name} {prec}: {done} iterations to {max(res):.2e} in {dt:.2f}s")
        fields[prec] = {k: s.get_field(k).cpu().numpy() for k in ("ux", "uy", "uz", "p", "k", "w")}
        del s
        torch.cuda.empty_cache()
    err = {}
    for k, a in fields["fp64"].items():
        b = fields["mixed"][k]
        err[k] = float(np.linalg.norm(b - a) / max(np.linalg.norm(a), 1e-300))
    return {"workload": spec.name + "_" + spec.model, "cells": spec.ncells, "target_residual": args.mixed_tol,
            "fp64": runs["fp64"], "mixed": runs["mixed"],
            "speedup": round(runs["fp64"]["seconds"] / runs["mixed"]["seconds"], 4),
            "rel_l2_mixed_vs_fp64": err}


VARIANTS = (("sst", "upwind", "eff"), ("keps", "upwind", "eff"), ("komega", "upwind", "eff"),
            ("rkeps", "upwind", "eff"),
            ("sst", "upwind", "perp"), ("sst", "linear_upwind", "eff"), ("sst", "vanleer", "eff"))


def variants(args):
    """The same workload under the other closures, the y_perp variant of y+ and
    the higher-order convection schemes, and for comparison the SST / upwind /
    y_eff configuration of the headline run over the same early iterations:
    time per iteration and the momentum / scalar assembly kernel averages over
    a short timed run each."""
    import torch
    import synth
    from paper_2606_06135_amd import Solver
    dev = torch.device("cuda:0")
    out = []
    for model, conv, ydist in VARIANTS:
        spec = synth.case_ahmed(scale=1, model=model)
        spec.conv_scheme = conv
        spec.yplus_dist = ydist
        s = Solver.from_spec(spec, device=dev, p_rtol=args.p_rtol, p_maxit=200)
        s.set_indicator(torch.from_numpy(spec.lam.ravel()).to(dev))
        s.iterate(args.variant_warmup)
        torch.cuda.synchronize()
        s.timing(True, args.timing_every)
        t0 = time.perf_counter()
        done, res = s.iterate(args.variant_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"model": model, "convection": conv, "yplus_distance": ydist, "iterations": done,
               "ms_per_iteration": round(dt / done * 1e3, 4),
               "pcg_iters_per_step": round(s.stats()[0] / max(done, 1), 2),
               "finite": bool(all(math.isfinite(x) for x in res))}
        for cls in ("mom_assemble", "scalar_assemble"):
            ms, cnt = s.timing_query(cls)
            rec[cls + "_avg_us"] = round(ms / cnt * 1e3, 2) if cnt else None
        s.timing(False)
        log(f"variant {model}/{conv}/{ydist}: {rec['ms_per_iteration']} ms per iteration")
        out.append(rec)
        del s
        torch.cuda.empty_cache()
    return {"workload": "ahmed_256x96x96", "warmup": args.variant_warmup, "steps": args.variant_steps, "runs": out}


def naca_sweep(args):
    """The batched angle-of-attack sweep (one graph for all instances)."""
    import numpy as np
    import torch
    import synth
    from paper_2606_06135_amd import Solver, Batch
    dev = torch.device("cuda:0")
    t0 = time.time()
    specs = synth.naca_sweep_specs(64)
    log(f"naca sweep: indicators of {len(specs)} instances in {time.time() - t0:.1f}s")
    solvers = []
    for sp in specs:
        s = Solver.from_spec(sp, device=dev, stream=torch.cuda.Stream(dev), p_rtol=args.p_rtol, p_maxit=100,
                             p_sweeps=args.sweep_p_sweeps, p_sweeps_coarse=args.sweep_p_sweeps)
        s.set_indicator(torch.from_numpy(sp.lam.ravel()))
        solvers.append(s)
    # the first iterations (large pressure corrections) on each instance's own
    # stream with the adaptive PCG tolerance, then the fixed-count graph
    for s in solvers:
        s.iterate(args.sweep_warmup)
    widths = {}
    for s, sp in zip(solvers, specs):
        key = f"{sp.nx}x{sp.ny}"
        if key not in widths:
            widths[key] = s.autotune_tiles(reps=3)[0]
        else:
            s.set_tile_width(widths[key])
    torch.cuda.synchronize()
    b = Batch(solvers, pcg_iters=args.sweep_pcg, tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(args.sweep_iters)
    st = b.status()
    dt = time.perf_counter() - t0
    b.close()
    cells = sum(sp.ncells for sp in specs)
    iters = st["iters_done"][0]
    inst = []
    for j, (s, sp) in enumerate(zip(solvers, specs)):
        cd, cl = s.coefficients(ref_area=1.0)
        g = -10.0 + 30.0 * j / (len(specs) - 1)
        inst.append({"gamma_deg": round(g, 3), "grid": f"{sp.nx}x{sp.ny}", "cd": round(cd, 5), "cl": round(cl, 5),
                     "thin_airfoil_cl": round(2 * np.pi * np.deg2rad(g), 5), "converged_at": st["conv_iter"][j],
                     "max_residual": max(st["residuals"][j])})
    log(f"naca sweep: {iters} iterations of {len(specs)} instances in {dt:.2f}s")
    return {"workload": "naca0012_sweep_64", "instances": len(specs), "cells": cells, "iterations": iters,
            "inlet_turbulence_intensity": specs[0].inlet_I,
            "launch_design": "one HIP graph holding every instance (a branch per context), two SIMPLE iterations "
                             "per graph launch with a fixed PCG iteration count, relaunched ceil(iterations / 2) "
                             "times with no host synchronisation between launches; not a persistent kernel",
            "warmup_iterations_each": args.sweep_warmup, "pcg_iters": args.sweep_pcg,
            "p_sweeps": args.sweep_p_sweeps, "seconds": round(dt, 3),
            "instance_iterations_per_s": round(len(specs) * iters / dt, 1),
            "instances_per_s": round(len(specs) / dt, 4), "cell_iters_per_s": cells * iters / dt,
            "tile_widths": widths, "converged_1e-6": sum(1 for x in st["conv_iter"] if x > 0),
            "diverged": st["diverged"], "per_instance": inst}


def hbm_reference():
    """Achievable HBM bandwidth on this GPU for the same element type: a copy
    (b = a) and a STREAM triad (a = b + s c) of FP64 arrays of 18.9 M elements
    (151 MB each, beyond the last-level cache), with torch's element-wise
    kernels, best of 10 timed repetitions.  A reference for the kernels'
    achieved bandwidth beside the nominal 8 TB/s."""
    import torch
    n = 18874368
    dev = torch.device("cuda:0")
    a = torch.rand(n, dtype=torch.float64, device=dev)
    b = torch.rand(n, dtype=torch.float64, device=dev)
    c = torch.rand(n, dtype=torch.float64, device=dev)
    out = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 16 * n),
                             ("triad", lambda: torch.add(b, c, alpha=1.5, out=a), 24 * n)):
        for _ in range(3):
            fn()
        best = None
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[name + "_GBs"] = round(nbytes / (best / 1e3) / 1e9, 1)
    del a, b, c
    torch.cuda.empty_cache()
    out["elements"] = n
    return out


def cpu_baseline(spec, p_rtol):
    """The oracle (plain NumPy, FP64) on the host: two SIMPLE iterations of the
    same workload after its precompute, once limited to one thread and once with
    every host thread allowed; rate in cell-iters/s, with the core count and the
    CPU model."""
    import warnings
    warnings.simplefilter("ignore")
    from oracle.solver import Simple
    log("cpu baseline: oracle precompute ...")
    t0 = time.time()
    sim = Simple(spec, p_solver="cg", p_rtol=p_rtol)
    log(f"cpu baseline: precompute {time.time() - t0:.1f}s; timing {2} iterations on one thread, then on all")
    import copy
    import platform
    from threadpoolctl import threadpool_limits
    nproc = os.cpu_count()
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n_it = 2
    rates = {}
    for label, limit in (("one", 1), ("all", None)):
        s = copy.deepcopy(sim)
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            for _ in range(n_it):
                s.step()
            dt = time.perf_counter() - t0
        rates[label] = (spec.ncells * n_it / dt, dt)
        del s
    return {"value": rates["one"][0], "unit": "cell-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_it} SIMPLE iterations of the same {spec.ncells}-cell workload from the initial "
                      f"conditions, pressure by SciPy CG (rtol {p_rtol}), {rates['one'][1]:.1f}s wall on one thread",
            "all_cores": {"value": rates["all"][0], "threads_available": nproc, "seconds": round(rates["all"][1], 2),
                          "note": "the NumPy/SciPy oracle is element-wise and sparse code: it uses one core "
                                  "whatever the thread limit (only dense BLAS calls would use more)"},
            "nproc": nproc, "cpu_model": model}


if __name__ == "__main__":
    main()
