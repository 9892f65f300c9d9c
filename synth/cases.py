"""Workload descriptions: grid, boundary kinds, fluid/model parameters and lambda.

Every number here is an *input* of the solver.  The shapes follow the paper's
test cases (backward-facing step, Ahmed body, channel flows) as synthetic
stand-ins: none of the paper's meshes or data is used.
"""

from __future__ import annotations

import dataclasses
import hashlib
from typing import Dict, Optional, Tuple

import numpy as np

from . import geometry as G

FACES = ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax")
BC_KINDS = ("inlet", "outlet", "noslip", "slip", "empty")
MODELS = ("laminar", "keps", "sst", "komega", "rkeps")
YPLUS_DIST = ("eff", "perp")
CONV_SCHEMES = ("upwind", "linear_upwind", "vanleer")

# Model constants.  The paper defers their values to the turbulence-model
# literature; these are the standard published values and both implementations
# receive them from here as inputs.
DEFAULT_CONSTANTS: Dict[str, float] = {
    # wall treatment (eqs. for k_vis, u_tau, omega_ib, P_ib, alpha masks)
    "Cmu": 0.09, "kappa": 0.41, "E": 9.8, "beta1_wf": 0.075, "Ceps2_wf": 1.9,
    "C_wf": 11.0, "ylam": 11.0,
    # standard k-epsilon
    "C1": 1.44, "C2": 1.92, "sigma_k": 1.0, "sigma_eps": 1.3,
    # Menter SST (multiplicative diffusion coefficients)
    "sigma_k1": 0.85, "sigma_w1": 0.5, "beta_1": 0.075, "gamma_1": 0.5532,
    "sigma_k2": 1.0, "sigma_w2": 0.856, "beta_2": 0.0828, "gamma_2": 0.4404,
    "a1": 0.31, "c_lim": 10.0,
    # standard k-omega in the paper's form: nu + nu_t / sigma diffusion,
    # C_alpha1 (omega/k) P_k - C_beta1 omega^2 (Wilcox's 2006 values; beta* = Cmu)
    "sigma_k_kw": 1.0 / 0.6, "sigma_w_kw": 2.0, "alpha_kw": 0.52, "beta_kw": 0.0708,
    # realizable k-epsilon (Shih et al. 1995): A0, C2 of the eps sink, sigma_k, sigma_eps
    "A0_rke": 4.0, "C2_rke": 1.9, "sigma_k_rke": 1.0, "sigma_eps_rke": 1.2,
    # numerical safeguards
    "bound_frac": 1e-10,      # k >= bound_frac*k_in, eps/omega >= bound_frac*inlet value
    "yperp_min_frac": 1e-6,   # y_perp >= yperp_min_frac*h
    "cd_floor": 1e-10,        # SST cross-diffusion floor
}


@dataclasses.dataclass
class CaseSpec:
    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    x0: float
    y0: float
    z0: float
    dx: float
    dy: float
    dz: float
    bc: Tuple[str, str, str, str, str, str]  # kinds of xmin,xmax,ymin,ymax,zmin,zmax
    u_in: Tuple[float, float, float]
    # inlet turbulence, either given directly (k_in, eps_in, omega_in) or, when
    # inlet_I > 0, as a turbulence intensity with a length scale inlet_l (or, with
    # inlet_l = 0, with omega_in given); each solver converts them itself
    k_in: Optional[float]
    eps_in: Optional[float]
    omega_in: Optional[float]
    nu: float
    model: str
    urf_u: float = 0.7
    urf_p: float = 0.3
    urf_t: float = 0.85
    n_sweeps: int = 2
    # distance in y+ of boundary cells: "eff" = y_eff of the paper's y+ definition,
    # "perp" = the perpendicular distance alone (the variant of the appendix on
    # effective vs perpendicular distance)
    yplus_dist: str = "eff"
    # momentum convection: upwind (the paper's setting), or the higher-order schemes
    # of its appendix on divergence schemes (linear upwind, van Leer)
    conv_scheme: str = "upwind"
    constants: Dict[str, float] = dataclasses.field(default_factory=lambda: dict(DEFAULT_CONSTANTS))
    lam: np.ndarray = None
    seed: int = 0
    inlet_I: float = 0.0
    inlet_l: float = 0.0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncells(self):
        return self.nx * self.ny * self.nz

    def lambda_sha256(self):
        return hashlib.sha256(np.ascontiguousarray(self.lam, dtype=np.float64).tobytes()).hexdigest()

    def validate(self):
        assert self.dim in (2, 3)
        if self.dim == 2:
            assert self.nz == 1 and self.bc[4] == "empty" and self.bc[5] == "empty"
        for b in self.bc:
            assert b in BC_KINDS
        assert self.model in MODELS
        assert self.yplus_dist in YPLUS_DIST
        assert self.conv_scheme in CONV_SCHEMES
        assert self.lam is not None and self.lam.shape == self.shape
        return self


def _spec(**kw):
    return CaseSpec(**kw)


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def case_bfs(nx=160, ny=40, h=1.0, model="keps"):
    """2D backward-facing step as an immersed 1h x 3h block at the inlet bottom of
    a 20h x 5h domain; Re_h = 5000 (nu = 2e-4), inlet U = 1, I = 5 %,
    mixing length 0.07 h.  The block lies on cell faces, so lambda is 0/1."""
    dx = 20.0 * h / nx
    dy = 5.0 * h / ny
    s = _spec(name=f"bfs_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1,
              x0=0.0, y0=0.0, z0=0.0, dx=dx, dy=dy, dz=1.0,
              bc=("inlet", "outlet", "noslip", "slip", "empty", "empty"),
              u_in=(1.0, 0.0, 0.0), k_in=None, eps_in=None, omega_in=None,
              nu=2e-4, model=model, inlet_I=0.05, inlet_l=0.07 * h)
    s.lam = G.lambda_from_sdf(G.sdf_box((-np.inf, -np.inf, -np.inf), (3.0 * h, 1.0 * h, np.inf)), s)
    return s.validate()


def case_ahmed(scale=1, model="sst"):
    """Ahmed-like body (1.044 x 0.389 x 0.288, front radius 0.1, 25 deg slant,
    ground clearance 0.05) in a channel x in [-2, 5.68], y in [-1.44, 1.44],
    z in [0, 2.88].  scale=1 gives 256 x 96 x 96 cells (dx = 0.03), scale=2 gives
    512 x 192 x 192 (dx = 0.015).  Re = 7.7e5 on the body length, U = 1,
    inlet I = 2 %, length scale a tenth of the body height."""
    d = 0.03 / scale
    nx, ny, nz = 256 * scale, 96 * scale, 96 * scale
    s = _spec(name=f"ahmed_{nx}x{ny}x{nz}", dim=3, nx=nx, ny=ny, nz=nz,
              x0=-2.0, y0=-1.44, z0=0.0, dx=d, dy=d, dz=d,
              bc=("inlet", "outlet", "slip", "slip", "noslip", "slip"),
              u_in=(1.0, 0.0, 0.0), k_in=None, eps_in=None, omega_in=None,
              nu=1.044 / 7.7e5, model=model, inlet_I=0.02, inlet_l=0.1 * 0.288)
    s.lam = G.lambda_from_sdf(G.sdf_ahmed_like(), s)
    return s.validate()


def case_ahmed_small(model="sst", nx=48, ny=16, nz=16, d=0.06):
    """Reduced Ahmed-like case for oracle-speed parity tests: the same body in a
    tighter box x in [-0.5, -0.5 + nx d], y centred, z from the ground."""
    s = _spec(name=f"ahmed_small_{nx}x{ny}x{nz}", dim=3, nx=nx, ny=ny, nz=nz,
              x0=-0.5, y0=-0.5 * ny * d, z0=0.0, dx=d, dy=d, dz=d,
              bc=("inlet", "outlet", "slip", "slip", "noslip", "slip"),
              u_in=(1.0, 0.0, 0.0), k_in=None, eps_in=None, omega_in=None,
              nu=1.044 / 7.7e5, model=model, inlet_I=0.02, inlet_l=0.1 * 0.288)
    s.lam = G.lambda_from_sdf(G.sdf_ahmed_like(), s)
    return s.validate()


def case_channel_ib(nx=48, n_fluid=8, n_solid=2, H=1.0, nu=0.1, U=1.0,
                    model="laminar", urf_u=0.7, urf_p=0.3):
    """2D channel whose walls are immersed solid bands on cell faces:
    n_solid solid rows below and above n_fluid fluid rows of height H.
    Uniform inlet U; outlet at x max.  Domain faces adjacent to the solid bands
    are handled as walls inside the solid."""
    d = H / n_fluid
    ny = n_fluid + 2 * n_solid
    y0 = -n_solid * d
    s = _spec(name=f"channel_ib_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1,
              x0=0.0, y0=y0, z0=0.0, dx=d, dy=d, dz=1.0,
              bc=("inlet", "outlet", "slip", "slip", "empty", "empty"),
              u_in=(U, 0.0, 0.0), k_in=1e-4, eps_in=1e-5, omega_in=1.0,
              nu=nu, model=model, urf_u=urf_u, urf_p=urf_p)
    lo_band = G.sdf_box((-np.inf, -np.inf, -np.inf), (np.inf, 0.0, np.inf))
    hi_band = G.sdf_box((-np.inf, H, -np.inf), (np.inf, np.inf, np.inf))
    s.lam = G.lambda_from_sdf(lambda x, y, z: np.minimum(lo_band(x, y, z), hi_band(x, y, z)), s)
    return s.validate()


def case_channel_bodyfitted(nx=48, n_fluid=8, H=1.0, nu=0.1, U=1.0,
                            model="laminar", urf_u=0.7, urf_p=0.3):
    """2D channel with no-slip domain walls at y = 0 and y = H (no solid)."""
    d = H / n_fluid
    s = _spec(name=f"channel_bf_{nx}x{n_fluid}", dim=2, nx=nx, ny=n_fluid, nz=1,
              x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=1.0,
              bc=("inlet", "outlet", "noslip", "noslip", "empty", "empty"),
              u_in=(U, 0.0, 0.0), k_in=1e-4, eps_in=1e-5, omega_in=1.0,
              nu=nu, model=model, urf_u=urf_u, urf_p=urf_p)
    s.lam = np.zeros(s.shape)
    return s.validate()


def case_cavity_block(nx=24, ny=12, model="laminar"):
    """Small 2D inflow/outflow box with a grid-aligned block in the middle."""
    d = 1.0 / ny
    s = _spec(name=f"block2d_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1,
              x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=1.0,
              bc=("inlet", "outlet", "noslip", "slip", "empty", "empty"),
              u_in=(1.0, 0.0, 0.0), k_in=1e-3, eps_in=1e-4, omega_in=1.0,
              nu=1e-2, model=model)
    s.lam = G.lambda_from_sdf(G.sdf_box((0.5, 0.25, -np.inf), (0.75, 0.5, np.inf)), s)
    return s.validate()


def case_small_body3d(nx=24, ny=12, nz=12, model="laminar", shape="sphere", nu=1e-2):
    """Small 3D duct with a sphere (cut cells) or a grid-aligned box."""
    d = 1.0 / ny
    s = _spec(name=f"{shape}3d_{nx}x{ny}x{nz}", dim=3, nx=nx, ny=ny, nz=nz,
              x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=d,
              bc=("inlet", "outlet", "slip", "slip", "noslip", "slip"),
              u_in=(1.0, 0.0, 0.0), k_in=None, eps_in=None, omega_in=None,
              nu=nu, model=model, inlet_I=0.05, inlet_l=0.07)
    if shape == "sphere":
        f = G.sdf_sphere((0.6, 0.5, 0.5), 0.2)
    else:
        f = G.sdf_box((0.5, 0.375, 0.375), (0.75, 0.625, 0.625))
    s.lam = G.lambda_from_sdf(f, s)
    return s.validate()


def case_uniform_duct(nx=64, ny=4, model="keps", U=1.0, L=1.0):
    """2D slip-walled duct without solid: uniform inflow carrying decaying
    turbulence (no shear, so production vanishes)."""
    d = L / nx
    s = _spec(name=f"duct_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1,
              x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=1.0,
              bc=("inlet", "outlet", "slip", "slip", "empty", "empty"),
              u_in=(U, 0.0, 0.0), k_in=1e-2, eps_in=1e-2, omega_in=100.0 / 9.0,
              nu=1e-5, model=model)
    s.lam = np.zeros(s.shape)
    return s.validate()


def case_naca(gamma_deg=4.0, nx=256, ny=128, model="sst", intensity=0.001):
    """2D NACA 0012 section (chord 1, leading edge at the origin) pitched to the
    angle of attack gamma about the quarter chord, in x in [-2, 6],
    y in [-2, 2] (square cells: 256 x 128, 512 x 256 or 1024 x 512).
    Re = 1e6 on the chord (nu = 1e-6, U = 1 along +x), inlet turbulence
    intensity I (default 0.1 %) with omega_in = 5 U / c; inlet at
    x = -2, outlet at x = 6, slip far-field top and bottom.  Lift is along +y,
    drag along +x."""
    dx = 8.0 / nx
    dy = 4.0 / ny
    s = _spec(name=f"naca0012_a{gamma_deg:+.2f}_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1,
              x0=-2.0, y0=-2.0, z0=0.0, dx=dx, dy=dy, dz=1.0,
              bc=("inlet", "outlet", "slip", "slip", "empty", "empty"),
              u_in=(1.0, 0.0, 0.0), k_in=None, eps_in=None, omega_in=5.0,
              nu=1e-6, model=model, inlet_I=intensity)
    s.lam = G.lambda_from_sdf(G.sdf_naca_symmetric(0.12, 1.0, gamma_deg), s)
    return s.validate()


def naca_sweep_specs(n=64, gamma_min=-10.0, gamma_max=20.0, sizes=((256, 128), (512, 256), (1024, 512))):
    """The batched sweep: n angles of attack uniformly spaced over
    [gamma_min, gamma_max], instance j on grid sizes[j % len(sizes)]."""
    out = []
    for j in range(n):
        g = gamma_min + (gamma_max - gamma_min) * j / max(n - 1, 1)
        nx, ny = sizes[j % len(sizes)]
        out.append(case_naca(g, nx, ny))
    return out


def case_bend2d(nx=384, ny=192, seed=12345, model="keps", design=True):
    """The adjoint workload: a 2D 90-degree bend duct of width 0.25 in
    [0, 2] x [0, 1] (square cells; 384 x 192 by default), inlet at x = 0 for
    0.65 < y < 0.9, outlet at y = 0 for 1.6 < x < 1.85; Re = 2000 on the width
    (U = 1, nu = 1.25e-4), k-epsilon, inlet I = 5 % with length scale 0.07 of the
    width.  Lambda: the duct's projection, and inside the design box
    [1.35, 1.85] x [0.4, 0.9] the larger of it and clip((g - 1)/0.5, 0, 1) with g
    white noise of the given seed, Gaussian-smoothed over 3 cells and scaled to
    unit standard deviation; the seed is advanced until the cells with
    lambda < 0.5 connect the inlet to the outlet."""
    from scipy import ndimage
    d = 2.0 / nx
    s = _spec(name=f"bend2d_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1,
              x0=0.0, y0=0.0, z0=0.0, dx=d, dy=1.0 / ny, dz=1.0,
              bc=("inlet", "slip", "outlet", "slip", "empty", "empty"),
              u_in=(1.0, 0.0, 0.0), k_in=None, eps_in=None, omega_in=None,
              nu=1.25e-4, model=model, inlet_I=0.05, inlet_l=0.07 * 0.25)
    geom = G.lambda_from_sdf(G.sdf_lbend(), s)
    if not design:
        s.lam = geom
        return s.validate()
    xc = (np.arange(nx) + 0.5) * d
    yc = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xc, yc)
    box = (X > 1.35) & (X < 1.85) & (Y > 0.4) & (Y < 0.9)
    inlet = (X < d) & (Y > 0.65) & (Y < 0.9)
    outlet = (Y < 1.0 / ny) & (X > 1.6) & (X < 1.85)
    sd = seed
    while True:
        g = ndimage.gaussian_filter(np.random.default_rng(sd).standard_normal((ny, nx)), 3.0)
        g = g / g.std()
        lam = geom[0].copy()
        lam[box] = np.maximum(lam[box], np.clip((g[box] - 1.0) / 0.5, 0.0, 1.0))
        lab, _ = ndimage.label(lam < 0.5)
        ins = set(np.unique(lab[inlet & (lab > 0)]))
        outs = set(np.unique(lab[outlet & (lab > 0)]))
        if ins & outs:
            break
        sd += 1
    s.lam = lam[None]
    s.seed = sd
    return s.validate()
