"""ctypes binding of ``libhfdib.so`` (the C ABI declared in include/hfdib.h).

Argument marshalling only: every step of the SIMPLE iteration runs in the HIP
kernels of the library.  PyTorch supplies device memory (one workspace tensor per
solver) and the HIP stream.  There is no CPU fallback: loading fails with an
error when the compiled library is absent.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhfdib.so")

ABI_VERSION = 4

BC = {"inlet": 0, "outlet": 1, "noslip": 2, "slip": 3, "empty": 4}
MODEL = {"laminar": 0, "keps": 1, "sst": 2, "komega": 3, "rkeps": 4}
YPLUS_DIST = {"eff": 0, "perp": 1}
CONV_SCHEME = {"upwind": 0, "linear_upwind": 1, "vanleer": 2}
FIELD = {"ux": 0, "uy": 1, "uz": 2, "p": 3, "k": 4, "w": 5, "nut": 6,
         "phix": 7, "phiy": 8, "phiz": 9, "lambda": 10, "class": 11, "alpha_u": 12, "walldist": 13,
         "uib_x": 14, "uib_y": 15, "uib_z": 16, "kib": 17, "wib": 18, "pk": 19, "yplus": 20}
IB = {"bc_cells": 0, "ic_cells": 1, "wall_cells": 2, "normal": 3, "yperp": 4, "yeff": 5, "mode": 6,
      "lagrange": 7, "st1_idx": 8, "st1_w": 9, "st2_idx": 10, "st2_w": 11, "yplus": 12,
      "utau_loglaw": 13, "wall_y": 14, "utau": 15, "wall_yplus": 16, "wall_utau": 17}
TIMER = {"p_apply": 0, "mom_sweep": 1, "mom_assemble": 2, "p_solve": 3, "iteration": 4, "scalar_sweep": 5,
         "scalar_assemble": 6, "p_smooth": 7, "p_presmooth": 8, "p_restrict": 9, "p_apply_dir": 10, "p_axpy": 11,
         "p_coarse": 12, "finalize": 13, "mom_explicit": 14}
STATUS = {0: "ok", -1: "invalid argument", -2: "workspace too small", -3: "HIP runtime error",
          -4: "diverged", -5: "call out of order"}


class GridDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("bc", C.c_int * 6), ("u_in", C.c_double * 3),
                ("k_in", C.c_double), ("eps_in", C.c_double), ("omega_in", C.c_double),
                ("turb_intensity", C.c_double), ("turb_length", C.c_double)]


_CONST_NAMES = ["Cmu", "kappa", "E", "beta1_wf", "Ceps2_wf", "C_wf", "ylam",
                "C1", "C2", "sigma_k", "sigma_eps",
                "sigma_k1", "sigma_w1", "beta_1", "gamma_1", "sigma_k2", "sigma_w2", "beta_2", "gamma_2",
                "a1", "c_lim", "sigma_k_kw", "sigma_w_kw", "alpha_kw", "beta_kw",
                "A0_rke", "C2_rke", "sigma_k_rke", "sigma_eps_rke",
                "bound_frac", "yperp_min_frac", "cd_floor"]


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_int), ("model", C.c_int), ("precision", C.c_int), ("n_sweeps", C.c_int),
                ("nu", C.c_double), ("urf_u", C.c_double), ("urf_p", C.c_double), ("urf_t", C.c_double),
                ("p_rtol", C.c_double), ("p_maxit", C.c_int), ("recorrect", C.c_int),
                ("bc_capacity", C.c_int), ("continuity", C.c_int), ("yplus_dist", C.c_int),
                ("conv_scheme", C.c_int)] + [(n, C.c_double) for n in _CONST_NAMES] + [
                    ("keep_state", C.c_int), ("div_factor", C.c_double), ("p_sweeps", C.c_int), ("p_sweeps_coarse", C.c_int)]


class HfdibError(RuntimeError):
    def __init__(self, fn, status, detail=""):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({status}) {detail}".strip())
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_06135_amd.build` "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    L.hfdib_abi_version.restype = i
    L.hfdib_default_config.argtypes = [C.POINTER(Config)]
    L.hfdib_default_config.restype = None
    L.hfdib_workspace_bytes.argtypes = [C.POINTER(GridDesc), C.POINTER(Config), C.POINTER(sz)]
    L.hfdib_init_grid.argtypes = [C.POINTER(GridDesc), C.POINTER(Config), vp, sz, vp, C.POINTER(vp)]
    L.hfdib_set_indicator.argtypes = [vp, vp, vp]
    L.hfdib_simple_iterate.argtypes = [vp, i, d, i, C.POINTER(i), C.POINTER(d)]
    L.hfdib_get_field.argtypes = [vp, i, vp]
    L.hfdib_set_field.argtypes = [vp, i, vp]
    L.hfdib_get_counts.argtypes = [vp, C.POINTER(i)]
    L.hfdib_get_ib_array.argtypes = [vp, i, vp]
    L.hfdib_pressure_solve.argtypes = [vp, vp, vp, vp, d, i, C.POINTER(i), C.POINTER(d)]
    L.hfdib_last_stats.argtypes = [vp, C.POINTER(d)]
    L.hfdib_timing_enable.argtypes = [vp, i]
    L.hfdib_timing_query.argtypes = [vp, i, C.POINTER(d), C.POINTER(C.c_longlong)]
    L.hfdib_destroy.argtypes = [vp]
    L.hfdib_destroy.restype = None
    L.hfdib_status_string.argtypes = [i]
    L.hfdib_status_string.restype = C.c_char_p
    L.hfdib_last_error.argtypes = [vp]
    L.hfdib_last_error.restype = C.c_char_p
    L.hfdib_forces.argtypes = [vp, C.POINTER(d)]
    L.hfdib_forces_noalloc.argtypes = [vp, vp]
    L.hfdib_force_coefficients.argtypes = [vp, d, d, C.POINTER(d), C.POINTER(d), C.POINTER(d)]
    L.hfdib_autotune_tiles.argtypes = [vp, i, C.POINTER(i), C.POINTER(d)]
    L.hfdib_set_tile_width.argtypes = [vp, i]
    L.hfdib_set_tile_depth.argtypes = [vp, i]
    L.hfdib_set_tile_order.argtypes = [vp, i]
    L.hfdib_batch_create.argtypes = [C.POINTER(vp), i, i, d, vp, C.POINTER(vp)]
    L.hfdib_batch_run.argtypes = [vp, i]
    L.hfdib_batch_status.argtypes = [vp, C.POINTER(i), C.POINTER(i), C.POINTER(d)]
    L.hfdib_batch_last_error.argtypes = [vp]
    L.hfdib_batch_last_error.restype = C.c_char_p
    L.hfdib_batch_destroy.argtypes = [vp]
    L.hfdib_batch_destroy.restype = None
    for fn in ("hfdib_workspace_bytes", "hfdib_init_grid", "hfdib_set_indicator", "hfdib_simple_iterate",
               "hfdib_get_field", "hfdib_set_field", "hfdib_get_counts", "hfdib_get_ib_array",
               "hfdib_pressure_solve", "hfdib_last_stats", "hfdib_timing_enable", "hfdib_timing_query",
               "hfdib_forces", "hfdib_forces_noalloc", "hfdib_force_coefficients", "hfdib_batch_create",
               "hfdib_batch_run", "hfdib_batch_status",
               "hfdib_autotune_tiles", "hfdib_set_tile_width", "hfdib_set_tile_depth",
               "hfdib_set_tile_order"):
        getattr(L, fn).restype = i
    if L.hfdib_abi_version() != ABI_VERSION:
        raise ImportError("libhfdib ABI version mismatch")
    _lib = L
    return L


EXPORTED = ["hfdib_abi_version", "hfdib_default_config", "hfdib_workspace_bytes", "hfdib_init_grid",
            "hfdib_set_indicator", "hfdib_simple_iterate", "hfdib_get_field", "hfdib_set_field",
            "hfdib_get_counts", "hfdib_get_ib_array", "hfdib_pressure_solve", "hfdib_last_stats",
            "hfdib_timing_enable", "hfdib_timing_query", "hfdib_destroy", "hfdib_status_string",
            "hfdib_last_error", "hfdib_forces", "hfdib_forces_noalloc", "hfdib_force_coefficients",
            "hfdib_batch_create", "hfdib_batch_run", "hfdib_batch_status",
            "hfdib_batch_last_error", "hfdib_batch_destroy", "hfdib_autotune_tiles", "hfdib_set_tile_width",
            "hfdib_set_tile_depth", "hfdib_set_tile_order"]


def default_config():
    cfg = Config()
    lib().hfdib_default_config(C.byref(cfg))
    return cfg


def make_desc_config(spec, p_rtol=1e-2, p_maxit=200, recorrect=True, bc_capacity=0, continuity="literal",
                     precision="fp64", keep_state=False, div_factor=None, p_sweeps=None, p_sweeps_coarse=None):
    """Grid descriptor and configuration from a case description (any object with
    the attributes of synth.CaseSpec)."""
    d = GridDesc()
    d.dim, d.nx, d.ny, d.nz = spec.dim, spec.nx, spec.ny, spec.nz
    d.x0, d.y0, d.z0 = spec.x0, spec.y0, spec.z0
    d.dx, d.dy, d.dz = spec.dx, spec.dy, spec.dz
    for f in range(6):
        d.bc[f] = BC[spec.bc[f]]
    for q in range(3):
        d.u_in[q] = spec.u_in[q]
    d.k_in, d.eps_in, d.omega_in = (0.0 if v is None else v for v in (spec.k_in, spec.eps_in, spec.omega_in))
    d.turb_intensity = getattr(spec, "inlet_I", 0.0) or 0.0
    d.turb_length = getattr(spec, "inlet_l", 0.0) or 0.0
    c = default_config()
    c.model = MODEL[spec.model]
    c.n_sweeps = spec.n_sweeps
    c.nu = spec.nu
    c.urf_u, c.urf_p, c.urf_t = spec.urf_u, spec.urf_p, spec.urf_t
    c.p_rtol = p_rtol
    c.p_maxit = p_maxit
    c.recorrect = 1 if recorrect else 0
    c.bc_capacity = bc_capacity
    c.continuity = {"literal": 0, "weighted": 1}[continuity]
    c.yplus_dist = YPLUS_DIST[getattr(spec, "yplus_dist", "eff")]
    c.conv_scheme = CONV_SCHEME[getattr(spec, "conv_scheme", "upwind")]
    c.precision = {"fp64": 0, "mixed": 1}[precision]
    c.keep_state = 1 if keep_state else 0
    if div_factor is not None:
        c.div_factor = float(div_factor)
    if p_sweeps is not None:
        c.p_sweeps = int(p_sweeps)
    if p_sweeps_coarse is not None:
        c.p_sweeps_coarse = int(p_sweeps_coarse)
    for n in _CONST_NAMES:
        if n in spec.constants:
            setattr(c, n, float(spec.constants[n]))
    return d, c


def _check(fn, st, ctx=None):
    if st != 0:
        detail = ""
        if ctx is not None:
            msg = lib().hfdib_last_error(ctx)
            detail = msg.decode() if msg else ""
        raise HfdibError(fn, st, detail)


class Solver:
    """One HFDIB SIMPLE context on a CUDA/HIP device.

    Tensors passed in must be float64 and contiguous on the solver's device.
    """

    def __init__(self, desc, cfg, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.desc, self.cfg = desc, cfg
        L = lib()
        nbytes = C.c_size_t(0)
        _check("hfdib_workspace_bytes", L.hfdib_workspace_bytes(C.byref(desc), C.byref(cfg), C.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        _check("hfdib_init_grid", L.hfdib_init_grid(C.byref(desc), C.byref(cfg), C.c_void_p(aligned),
                                                    self.ws_bytes, C.c_void_p(self.stream.cuda_stream),
                                                    C.byref(ctx)))
        self.ctx = ctx
        self.N = desc.nx * desc.ny * desc.nz

    @classmethod
    def from_spec(cls, spec, device="cuda:0", stream=None, **kw):
        d, c = make_desc_config(spec, **kw)
        return cls(d, c, device=device, stream=stream)

    # stream ordering between torch's current stream and the solver's stream
    def _sync_in(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _sync_out(self, *tensors):
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)
            for t in tensors:
                t.record_stream(self.stream)

    def close(self):
        if getattr(self, "ctx", None):
            lib().hfdib_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, a, dtype=None):
        t = self.torch
        dtype = dtype or t.float64
        if not isinstance(a, t.Tensor):
            a = t.as_tensor(a)
        return a.to(device=self.device, dtype=dtype).contiguous()

    def set_indicator(self, lam, solid_vel=None):
        self._lam = self._t(lam).reshape(-1)
        self._us = None if solid_vel is None else self._t(solid_vel).reshape(-1)
        self._sync_in()
        st = lib().hfdib_set_indicator(self.ctx, C.c_void_p(self._lam.data_ptr()),
                                       C.c_void_p(self._us.data_ptr()) if self._us is not None else None)
        _check("hfdib_set_indicator", st, self.ctx)

    def iterate(self, n, tol=0.0, check_every=0):
        done = C.c_int(0)
        res = (C.c_double * 6)()
        st = lib().hfdib_simple_iterate(self.ctx, int(n), float(tol), int(check_every), C.byref(done), res)
        _check("hfdib_simple_iterate", st, self.ctx)
        return done.value, list(res)

    def field_size(self, name):
        d = self.desc
        if name == "phix":
            return (d.nx + 1) * d.ny * d.nz
        if name == "phiy":
            return d.nx * (d.ny + 1) * d.nz
        if name == "phiz":
            return d.nx * d.ny * (d.nz + 1)
        return self.N

    def get_field(self, name):
        out = self.torch.empty(self.field_size(name), dtype=self.torch.float64, device=self.device)
        self._sync_in()
        _check("hfdib_get_field", lib().hfdib_get_field(self.ctx, FIELD[name], C.c_void_p(out.data_ptr())), self.ctx)
        self._sync_out(out)
        return out

    def set_field(self, name, values):
        v = self._t(values).reshape(-1)
        assert v.numel() == self.field_size(name)
        self._sync_in()
        _check("hfdib_set_field", lib().hfdib_set_field(self.ctx, FIELD[name], C.c_void_p(v.data_ptr())), self.ctx)
        self.stream.synchronize()

    def counts(self):
        a = (C.c_int * 3)()
        _check("hfdib_get_counts", lib().hfdib_get_counts(self.ctx, a), self.ctx)
        return {"bc": a[0], "ic": a[1], "wall": a[2]}

    def ib_array(self, name):
        n = self.counts()
        t = self.torch
        sizes = {"bc_cells": (n["bc"], t.int32), "ic_cells": (n["ic"], t.int32), "wall_cells": (n["wall"], t.int32),
                 "normal": (3 * n["bc"], t.float64), "yperp": (n["bc"], t.float64), "yeff": (n["bc"], t.float64),
                 "mode": (n["bc"], t.int32), "lagrange": (3 * n["bc"], t.float64),
                 "st1_idx": (8 * n["bc"], t.int32), "st1_w": (8 * n["bc"], t.float64),
                 "st2_idx": (8 * n["bc"], t.int32), "st2_w": (8 * n["bc"], t.float64),
                 "yplus": (n["bc"], t.float64), "utau_loglaw": (n["bc"], t.float64),
                 "wall_y": (n["wall"], t.float64), "utau": (n["bc"], t.float64),
                 "wall_yplus": (n["wall"], t.float64), "wall_utau": (n["wall"], t.float64)}
        cnt, dt = sizes[name]
        out = t.empty(max(cnt, 1), dtype=dt, device=self.device)
        self._sync_in()
        _check("hfdib_get_ib_array", lib().hfdib_get_ib_array(self.ctx, IB[name], C.c_void_p(out.data_ptr())),
               self.ctx)
        self._sync_out(out)
        return out[:cnt]

    def pressure_solve(self, rAU, rhs, p0, rtol=1e-12, maxit=200):
        rAU, rhs = self._t(rAU).reshape(-1), self._t(rhs).reshape(-1)
        p = self._t(p0).reshape(-1).clone()
        it = C.c_int(0)
        rr = C.c_double(0.0)
        self._sync_in()
        st = lib().hfdib_pressure_solve(self.ctx, C.c_void_p(rAU.data_ptr()), C.c_void_p(rhs.data_ptr()),
                                        C.c_void_p(p.data_ptr()), float(rtol), int(maxit), C.byref(it),
                                        C.byref(rr))
        _check("hfdib_pressure_solve", st, self.ctx)
        self._sync_out(p)
        return p, it.value, rr.value

    def autotune_tiles(self, reps=5):
        """Times the tile widths on the current state, keeps the fastest;
        returns (width, {width: ms per round})."""
        best = C.c_int(0)
        ms = (C.c_double * 4)()
        _check("hfdib_autotune_tiles", lib().hfdib_autotune_tiles(self.ctx, int(reps), C.byref(best), ms), self.ctx)
        return best.value, {32 << q: ms[q] for q in range(4)}

    def set_tile_width(self, width):
        _check("hfdib_set_tile_width", lib().hfdib_set_tile_width(self.ctx, int(width)), self.ctx)

    def set_tile_depth(self, depth):
        _check("hfdib_set_tile_depth", lib().hfdib_set_tile_depth(self.ctx, int(depth)), self.ctx)

    def set_tile_order(self, zfirst):
        _check("hfdib_set_tile_order", lib().hfdib_set_tile_order(self.ctx, 1 if zfirst else 0), self.ctx)

    def forces(self):
        """Force on the body per unit density: pressure part, viscous part,
        interface area and its boundary-cell part (see hfdib_forces)."""
        a = (C.c_double * 8)()
        _check("hfdib_forces", lib().hfdib_forces(self.ctx, a), self.ctx)
        return {"pressure": [a[0], a[1], a[2]], "viscous": [a[3], a[4], a[5]], "area": a[6], "bc_area": a[7]}

    def forces_noalloc(self, out=None):
        """hfdib_forces_noalloc into a device tensor of 8 doubles (no host wait)."""
        if out is None:
            out = self.torch.empty(8, dtype=self.torch.float64, device=self.device)
        self._sync_in()
        _check("hfdib_forces_noalloc", lib().hfdib_forces_noalloc(self.ctx, C.c_void_p(out.data_ptr())), self.ctx)
        self._sync_out(out)
        return out

    def coefficients(self, ref_area, u_ref=1.0, drag_dir=(1.0, 0.0, 0.0), lift_dir=(0.0, 1.0, 0.0)):
        """Drag and lift coefficients of the current state (hfdib_force_coefficients)."""
        out = (C.c_double * 2)()
        dd = (C.c_double * 3)(*drag_dir)
        ld = (C.c_double * 3)(*lift_dir)
        _check("hfdib_force_coefficients",
               lib().hfdib_force_coefficients(self.ctx, float(ref_area), float(u_ref), dd, ld, out), self.ctx)
        return out[0], out[1]

    def stats(self):
        a = (C.c_double * 8)()
        _check("hfdib_last_stats", lib().hfdib_last_stats(self.ctx, a), self.ctx)
        return list(a)

    def timing(self, enable, every=1):
        """Kernel timing on (recording every `every`-th SIMPLE iteration) or off."""
        _check("hfdib_timing_enable", lib().hfdib_timing_enable(self.ctx, int(every) if enable else 0), self.ctx)

    def timing_query(self, name):
        ms = C.c_double(0.0)
        cnt = C.c_longlong(0)
        _check("hfdib_timing_query", lib().hfdib_timing_query(self.ctx, TIMER[name], C.byref(ms), C.byref(cnt)),
               self.ctx)
        return ms.value, cnt.value


class Batch:
    """Independent solvers (each with its own stream) iterated together by one
    HIP graph launch per two SIMPLE iterations (see hfdib_batch_create)."""

    def __init__(self, solvers, pcg_iters=4, tol=1e-8, stream=None):
        import torch
        self.torch = torch
        self.solvers = list(solvers)  # keeps the workspaces alive
        self.stream = stream  # None: the batch creates and owns its launch stream
        arr = (C.c_void_p * len(self.solvers))(*[s.ctx for s in self.solvers])
        b = C.c_void_p()
        sp = None if stream is None else C.c_void_p(stream.cuda_stream)
        st = lib().hfdib_batch_create(arr, len(self.solvers), int(pcg_iters), float(tol), sp, C.byref(b))
        if st != 0:
            raise HfdibError("hfdib_batch_create", st, "")
        self.b = b

    def run(self, iters):
        st = lib().hfdib_batch_run(self.b, int(iters))
        if st != 0:
            raise HfdibError("hfdib_batch_run", st, lib().hfdib_batch_last_error(self.b).decode())

    def status(self):
        n = len(self.solvers)
        conv = (C.c_int * n)()
        done = (C.c_int * n)()
        res = (C.c_double * (6 * n))()
        st = lib().hfdib_batch_status(self.b, conv, done, res)
        if st not in (0, -4):
            raise HfdibError("hfdib_batch_status", st, lib().hfdib_batch_last_error(self.b).decode())
        return {"diverged": st == -4, "conv_iter": list(conv), "iters_done": list(done),
                "residuals": [list(res[6 * i:6 * i + 6]) for i in range(n)]}

    def close(self):
        if getattr(self, "b", None):
            lib().hfdib_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
