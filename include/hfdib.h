/*
 * hfdib.h -- C ABI of the MI355X library for the IB-aware steady SIMPLE
 * iteration of the hybrid fictitious domain-immersed boundary (HFDIB) RANS
 * method (Kubickova & Isoz, "Extending the hybrid fictitious domain-immersed
 * boundary method for Reynolds-averaged turbulence modeling").
 *
 * Problem statement followed by the entry points:
 *   - a fluid/solid domain on a uniform Cartesian grid, the solid given by the
 *     cell indicator lambda in [0,1] (Sec. "Mask fields construction", eq. for
 *     lambda);
 *   - the steady RANS equations with IB source f_ib and the lambda-masked
 *     continuity equation (eq. of the governing equations), closed by a
 *     two-equation model with S_ib in the k equation (Sec. "Governing
 *     equations", "Immersed boundary-induced source terms");
 *   - inlet/outlet/wall conditions and inlet turbulence (boundary-condition
 *     paragraph of the pipe-flow section), upwind convection and implicit
 *     under-relaxation (paragraph "Numerical schemes");
 *   - the SIMPLE loop extended by the IB steps (figure of the SIMPLE algorithm
 *     and the paragraph "SIMPLE-based solution strategy").
 *
 * Memory: every heavy buffer is caller-owned device memory.  The caller
 * allocates one workspace of hfdib_workspace_bytes() bytes on the device and
 * keeps it alive for the lifetime of the context; the library never calls
 * hipMalloc.  Arrays are FP64, structure-of-arrays, cell index
 * c = i + nx*(j + ny*k) (x fastest).  Face-flux arrays phi_x, phi_y, phi_z hold
 * (nx+1)*ny*nz, nx*(ny+1)*nz and nx*ny*(nz+1) values (flux in the +axis
 * direction), face index f = i + (nx+1)*(j + ny*k) etc.
 *
 * Streams: all device work of a context is enqueued on the hipStream_t given to
 * hfdib_init_grid (NULL = default stream).  Pointers passed in are consumed in
 * stream order.  Host synchronisation happens only where documented.
 *
 * Errors: every int-returning call returns an hfdib_status; no exception
 * crosses the ABI.  On HFDIB_EDEVICE the HIP error string is kept and returned
 * by hfdib_last_error().  A context is not thread safe; separate contexts are
 * independent.
 */
#ifndef HFDIB_H
#define HFDIB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HFDIB_ABI_VERSION 4

typedef enum {
  HFDIB_OK = 0,
  HFDIB_EINVAL = -1,    /* invalid argument, lambda NaN or outside [0,1], capacity exceeded */
  HFDIB_ENOMEM = -2,    /* workspace smaller than hfdib_workspace_bytes() */
  HFDIB_EDEVICE = -3,   /* a HIP runtime error; message in hfdib_last_error() */
  HFDIB_EDIVERGED = -4, /* NaN/Inf in the state or residual blow-up */
  HFDIB_ESTATE = -5     /* call out of order (e.g. iterate before set_indicator) */
} hfdib_status;

typedef enum {
  HFDIB_BC_INLET = 0,  /* Dirichlet u = u_in, k, eps/omega; zero-gradient p */
  HFDIB_BC_OUTLET = 1, /* p = 0; zero-gradient u, k, eps/omega */
  HFDIB_BC_NOSLIP = 2, /* u = 0 with log-law wall viscosity; wall functions for eps/omega */
  HFDIB_BC_SLIP = 3,   /* no flux; zero-gradient u (normal part 0 in gradients) and scalars */
  HFDIB_BC_EMPTY = 4   /* z faces of a 2D grid */
} hfdib_bc_kind;

/* KOMEGA: the k-omega equations in the paper's form (diffusion nu + nu_t / sigma,
 * omega sources C_alpha1 (omega/k) P_k - C_beta1 omega^2, sink beta* k omega with
 * beta* = Cmu, nu_t = k / omega), wall treatment as for SST.
 * RKEPS: the realizable k-epsilon model the paper lists beside the others (Sec.
 * "Governing equations", after Shih et al. 1995): nu_t = C_mu k^2 / eps with
 * C_mu = 1 / (A0 + A_s U* k / eps) from the deviatoric strain rate S and the
 * rotation rate of the velocity gradient (U* = sqrt(S:S + Omega:Omega),
 * A_s = sqrt(6) cos(arccos(sqrt(6) W) / 3), W = S_ij S_jk S_ki / (S:S)^1.5);
 * eps source C1 |S| eps with |S| = sqrt(2 S:S), C1 = max(0.43, eta / (eta + 5)),
 * eta = |S| k / eps, and sink C2 eps^2 / (k + sqrt(nu eps)); k equation, IB and
 * wall treatment as for KEPS. */
typedef enum {
  HFDIB_LAMINAR = 0,
  HFDIB_KEPS = 1,
  HFDIB_KOMEGA_SST = 2,
  HFDIB_KOMEGA = 3,
  HFDIB_RKEPS = 4
} hfdib_model;
/* Distance in y+ of boundary cells (Sec. "Calculation of y+ at the immersed
 * boundary"): EFF the effective distance y_eff = (y_perp + h/2) / 2 of the paper's
 * definition; PERP the perpendicular distance y_perp alone (the appendix comparing
 * effective and perpendicular distance).  The chosen distance replaces y_eff in
 * every wall function: y+, u_tau of the log law, omega_ib and the wall shear. */
typedef enum { HFDIB_YPLUS_EFF = 0, HFDIB_YPLUS_PERP = 1 } hfdib_yplus_dist;
/* Convection scheme of the momentum equation (the paper's appendix on divergence
 * schemes; upwind is the setting of its main results).  LINEAR_UPWIND and VANLEER
 * enter as a deferred correction of the upwind rows from the previous iterate,
 * -sum_f F_out (u_f - u_C) over interior faces (C upwind, D downwind cell):
 * linear upwind u_f = u_C + (x_f - x_C).grad u_C; van Leer
 * u_f = u_C + psi(r) (u_D - u_C)/2, psi(r) = (r + |r|)/(1 + |r|),
 * r = 2 (x_D - x_C).grad u_C / (u_D - u_C) - 1, with grad u_C the Gauss cell
 * gradient.  At a fixed point the discretisation is the higher-order one.  k and
 * eps/omega stay upwind. */
typedef enum { HFDIB_CONV_UPWIND = 0, HFDIB_CONV_LINEAR_UPWIND = 1, HFDIB_CONV_VANLEER = 2 } hfdib_conv_scheme;
typedef enum { HFDIB_FP64 = 0, HFDIB_MIXED = 1 } hfdib_precision;

/* Grid and boundary data.  dim = 2 requires nz = 1 and EMPTY z faces.
 * bc[] order: xmin, xmax, ymin, ymax, zmin, zmax.
 * Inlet turbulence: with turb_intensity = I > 0 the library derives the inlet
 * values from the intensity as in the paper's inlet condition (boundary-condition
 * paragraph of the pipe-flow section, eq. bcspkoein): k_in = 3/2 |u_in|^2 I^2 and,
 * with turb_length = l_t > 0, eps_in = C_nu k_in^(3/2) / l_t and
 * omega_in = eps_in / (C_nu k_in) (C_nu = hfdib_config.Cmu); with turb_length <= 0
 * omega_in is taken as given and eps_in = C_nu k_in omega_in.  The k_in, eps_in
 * (and, with l_t > 0, omega_in) fields are then ignored.  With turb_intensity <= 0
 * k_in, eps_in and omega_in are used as given. */
typedef struct {
  int dim;
  int nx, ny, nz;
  double x0, y0, z0;
  double dx, dy, dz;
  int bc[6];
  double u_in[3];
  double k_in, eps_in, omega_in;
  double turb_intensity, turb_length;
} hfdib_grid_desc;

/* Solver configuration.  hfdib_default_config() fills every field. */
typedef struct {
  int abi_version;      /* must equal HFDIB_ABI_VERSION */
  int model;            /* hfdib_model */
  int precision;        /* hfdib_precision.  FP64: every step in FP64.  MIXED: the state, every
                           assembly, defect, residual norm, reduction, the PCG vectors and dots and
                           the log-law Newton stay FP64; the momentum and k, eps/omega red-black
                           sweeps solve for an FP32 correction of the FP64 defect (coefficients
                           from FP32 mirrors, x <- x + d in FP64) and the multigrid preconditioner
                           (smoothing, transfers, coarse operators) runs in FP32.  The workspace
                           size depends on this field. */
  int n_sweeps;         /* red-black Gauss-Seidel sweeps per transport solve (>= 1) */
  double nu;            /* kinematic viscosity (> 0) */
  double urf_u, urf_p, urf_t; /* under-relaxation of momentum, pressure, turbulence, in (0,1] */
  double p_rtol;        /* relative residual target of the pressure PCG solve (|r| <= p_rtol |b|, |b|
                           over the coupled rows; see hfdib_pressure_solve) */
  int p_maxit;          /* PCG iteration cap per pressure solve */
  int recorrect;        /* 1: re-impose u_ib on forced cells after the velocity update */
  int bc_capacity;      /* max boundary (and in-solid, wall) cells; 0 = automatic */
  int continuity;       /* lambda-masked continuity: 0 = div u = 0 wherever lambda < 1 (pressure
                           rhs sum_f phi*_f there, 0 in lambda = 1 cells); 1 = rhs scaled by
                           (1 - lambda) in every cell */
  int yplus_dist;       /* hfdib_yplus_dist */
  int conv_scheme;      /* hfdib_conv_scheme */
  /* wall treatment */
  double Cmu, kappa, E, beta1_wf, Ceps2_wf, C_wf, ylam;
  /* standard k-epsilon */
  double C1, C2, sigma_k, sigma_eps;
  /* Menter SST */
  double sigma_k1, sigma_w1, beta_1, gamma_1, sigma_k2, sigma_w2, beta_2, gamma_2, a1, c_lim;
  /* standard k-omega (divisors sigma of nu_t, C_alpha1, C_beta1) */
  double sigma_k_kw, sigma_w_kw, alpha_kw, beta_kw;
  /* realizable k-epsilon (A0 of C_mu, C2 of the eps sink, divisors sigma of nu_t) */
  double A0_rke, C2_rke, sigma_k_rke, sigma_eps_rke;
  /* safeguards */
  double bound_frac, yperp_min_frac, cd_floor;
  /* 1: hfdib_set_indicator keeps the current state (velocity, pressure, fluxes,
     k, eps/omega, nu_t) instead of resetting it to the initial conditions, e.g. to
     restart from a converged state after a small change of lambda */
  int keep_state;
  /* residual blow-up guard of hfdib_simple_iterate: HFDIB_EDIVERGED when the sum of
     the absolute momentum residuals sum |b - A u| at a residual check exceeds
     div_factor times its value at the first check of the call (<= 0: off) */
  double div_factor;
  /* red-black Gauss-Seidel sweeps before and after the coarse correction in the
     pressure preconditioner's V-cycle, on the fine level (p_sweeps) and on every
     coarse level (p_sweeps_coarse), each 1..4; the V-cycle stays symmetric
     (red-black sweeps before, black-red after) */
  int p_sweeps, p_sweeps_coarse;
} hfdib_config;

typedef struct hfdib_ctx hfdib_ctx;

/* Field identifiers for hfdib_get_field / hfdib_set_field (FP64 device arrays). */
enum {
  HFDIB_FIELD_UX = 0, HFDIB_FIELD_UY, HFDIB_FIELD_UZ, HFDIB_FIELD_P,
  HFDIB_FIELD_K, HFDIB_FIELD_EPS_OR_OMEGA, HFDIB_FIELD_NUT,
  HFDIB_FIELD_PHI_X, HFDIB_FIELD_PHI_Y, HFDIB_FIELD_PHI_Z,
  HFDIB_FIELD_LAMBDA,   /* get only */
  HFDIB_FIELD_CLASS,    /* get only: 0 free-stream, 1 boundary, 2 in-solid */
  HFDIB_FIELD_ALPHA_U,  /* get only: alpha_u of the last iteration */
  HFDIB_FIELD_WALLDIST, /* get only: SST wall distance */
  /* get only, values of the last iteration (eq. of the imposed fields, eqs. for
     k_vis, omega_ib and P_ib): the imposed velocity on forced cells (in-solid cells
     and boundary cells with alpha_u = 1; other cells undefined), the imposed k on
     the same cells, the imposed eps/omega on in-solid, boundary and domain-wall
     cells (alpha_omega = 1; other cells undefined), the production of k with P_ib
     on those cells, and y+ (boundary and domain-wall cells, 0 elsewhere) */
  HFDIB_FIELD_UIB_X, HFDIB_FIELD_UIB_Y, HFDIB_FIELD_UIB_Z, HFDIB_FIELD_KIB, HFDIB_FIELD_WIB,
  HFDIB_FIELD_PK, HFDIB_FIELD_YPLUS,
  HFDIB_FIELD_COUNT
};

/* Per-boundary-cell records for hfdib_get_ib_array (device destination). */
enum {
  HFDIB_IB_BC_CELLS = 0, /* int32[n_bc], increasing cell index */
  HFDIB_IB_IC_CELLS,     /* int32[n_ic] */
  HFDIB_IB_WALL_CELLS,   /* int32[n_wall]: free-stream cells next to no-slip domain faces */
  HFDIB_IB_NORMAL,       /* double[3*n_bc], (nx,ny,nz) per cell */
  HFDIB_IB_YPERP,        /* double[n_bc] */
  HFDIB_IB_YEFF,         /* double[n_bc] */
  HFDIB_IB_MODE,         /* int32[n_bc]: 3 quadratic, 2 linear, 1 constant */
  HFDIB_IB_LAGRANGE,     /* double[3*n_bc] weights of (S, P1, P2) */
  HFDIB_IB_ST1_IDX,      /* int32[8*n_bc] */
  HFDIB_IB_ST1_W,        /* double[8*n_bc] */
  HFDIB_IB_ST2_IDX,      /* int32[8*n_bc] */
  HFDIB_IB_ST2_W,        /* double[8*n_bc] */
  HFDIB_IB_YPLUS,        /* double[n_bc]: y+ of the last iteration */
  HFDIB_IB_UTAU_LOGLAW,  /* double[n_bc]: log-law u_tau of the last iteration (0 off branch) */
  HFDIB_IB_WALL_Y,       /* double[n_wall] */
  HFDIB_IB_UTAU,         /* double[n_bc]: u_tau = C_mu^(1/4) sqrt(k) of the last iteration */
  HFDIB_IB_WALL_YPLUS,   /* double[n_wall]: y+ of the last iteration */
  HFDIB_IB_WALL_UTAU,    /* double[n_wall]: u_tau of the last iteration */
  HFDIB_IB_COUNT
};

/* Returns HFDIB_ABI_VERSION. */
int hfdib_abi_version(void);

/* Fills *cfg with the defaults (standard model constants, URF 0.7/0.3/0.85,
 * n_sweeps 2, p_rtol 1e-2, p_maxit 200, recorrect 1, continuity 0, keep_state 0,
 * div_factor 1e6, p_sweeps 2, p_sweeps_coarse 2). */
void hfdib_default_config(hfdib_config* cfg);

/* Bytes of device workspace a context needs for this grid and configuration. */
int hfdib_workspace_bytes(const hfdib_grid_desc* d, const hfdib_config* c, size_t* bytes);

/* Creates a context.  Copies d and c, lays out the caller's workspace (device
 * pointer, >= hfdib_workspace_bytes, 256-byte aligned) and records the stream
 * (a hipStream_t, NULL for the default stream).  No device work is enqueued
 * and no HIP call is made.  Errors: EINVAL for a bad descriptor or workspace
 * pointer, ENOMEM for a workspace below hfdib_workspace_bytes. */
int hfdib_init_grid(const hfdib_grid_desc* d, const hfdib_config* c, void* workspace,
                    size_t bytes, void* hip_stream, hfdib_ctx** out);

/* Sets the indicator field (Sec. "Mask fields construction") and runs the
 * per-lambda precompute: cell groups, normals, sigma, y_perp, y_eff,
 * interpolation stencils, wall-function cells and (SST) the wall distance; then
 * resets the state to the initial conditions (unless cfg.keep_state).
 * lambda_dev: N doubles in [0,1]
 * (device).  solid_vel_dev: 3*N doubles (ux block, uy block, uz block) with the
 * solid velocity, or NULL for a resting solid.  Both are copied.  Synchronises
 * the stream once (to validate lambda and read list sizes).
 * Errors: EINVAL for NaN/out-of-range lambda or list capacity exceeded. */
int hfdib_set_indicator(hfdib_ctx* ctx, const double* lambda_dev, const double* solid_vel_dev);

/* Runs up to max_iters SIMPLE iterations (the paper's extended loop).  Stops
 * early when tol > 0 and the largest normalised residual <= tol (checked every
 * check_every iterations and after the last one, with a host synchronisation).
 * tol <= 0 runs exactly max_iters.  The pressure solve of every iteration also
 * synchronises once per PCG iteration (see hfdib_pressure_solve).
 * *iters_done (nullable) receives the count; res_out (nullable, host, 6 doubles)
 * the residuals of Ux, Uy, Uz, p, k, eps/omega of the last iteration.  Returns
 * EDIVERGED on a NaN/Inf residual or on a residual blow-up (see
 * hfdib_config.div_factor), with the state left as of the failing iteration. */
int hfdib_simple_iterate(hfdib_ctx* ctx, int max_iters, double tol, int check_every,
                         int* iters_done, double* res_out);

/* Copies a field to / from caller device memory (stream ordered). */
int hfdib_get_field(hfdib_ctx* ctx, int field_id, double* dst_dev);
int hfdib_set_field(hfdib_ctx* ctx, int field_id, const double* src_dev);

/* Sizes of the precomputed lists: counts[0] = n_bc, [1] = n_ic, [2] = n_wall. */
int hfdib_get_counts(hfdib_ctx* ctx, int* counts);

/* Force on the immersed body per unit density (kinematic) from the current
 * state, for the drag and lift coefficients (Sec. "Flow over a cylinder", eq. of
 * the drag coefficient; eq. of the lift coefficient).  The surface element of a
 * cell is |grad lambda| V (central differences, one-sided at domain edges), its
 * outward normal -grad lambda / |grad lambda|.  out8 (host, 8 doubles):
 * [0..2] pressure force sum_cells p grad(lambda) V; [3..5] viscous force: the
 * |grad lambda| V-weighted mean over boundary cells of tau_w t (t: direction of
 * the tangential velocity relative to the solid; tau_w = u_tau^2 of the log-law
 * Newton solve on logarithmic-branch cells, nu |u_t| / y_eff on viscous-branch
 * cells) times the interface area; [6] interface area sum_cells |grad lambda| V;
 * [7] the part of it on boundary cells.  C = 2 F.v / (|u_in|^2 A_ref).
 * Synchronises the stream.  HFDIB_ESTATE before hfdib_set_indicator. */
int hfdib_forces(hfdib_ctx* ctx, double* out8);

/* Drag and lift coefficients of the current state (the drag-coefficient equation
 * of the cylinder section and the lift-coefficient equation of the airfoil
 * section): C = 2 F.e / (u_ref^2 A_ref) for the total force F of hfdib_forces
 * (pressure plus viscous part) along the unit directions drag_dir and lift_dir
 * (host, 3 doubles each).  out2 (host): [0] C_d, [1] C_l.  Synchronises the
 * stream.  HFDIB_EINVAL for ref_area <= 0 or u_ref = 0, HFDIB_ESTATE before
 * hfdib_set_indicator. */
int hfdib_force_coefficients(hfdib_ctx* ctx, double ref_area, double u_ref, const double* drag_dir,
                             const double* lift_dir, double* out2);

/* For callers that cannot allocate or wait on the host (code under HIP graph
 * capture, tight serving loops): the same eight values as hfdib_forces, written
 * to out8_dev (8 doubles of caller device memory) in stream order, with no host
 * synchronisation and no allocation of any kind.  The block partial sums live in
 * a fixed 4 MiB device array of the library (one per GPU, kept until the process
 * ends), which limits the grid to about 33 M cells (4 doubles per 256-cell tile
 * plus 4 per 256 boundary cells); larger grids get HFDIB_EINVAL with the sizes in
 * hfdib_last_error.  Every call on a GPU shares that array: calls that overlap on
 * one GPU (different streams or contexts) race and must be ordered by the caller.
 * The sums may differ from hfdib_forces in the last bits (another summation
 * order of the partials).  HFDIB_ESTATE before hfdib_set_indicator. */
int hfdib_forces_noalloc(hfdib_ctx* ctx, double* out8_dev);

/* Tile shape of the full-grid kernels: 256-thread tiles of width 32, 64 (the
 * default), 128 or 256 cells along x.  hfdib_autotune_tiles times, for each
 * width, reps rounds of the momentum assembly and the pressure operator on
 * the current state (neither changes the state),
 * keeps the fastest width and returns it in *best_width (nullable) with the
 * average milliseconds per round of widths 32, 64, 128, 256 in ms4 (host,
 * nullable).  The width changes only the order of partial sums in reductions.
 * A batch captures the width in force when it is created.  HFDIB_EINVAL for
 * other widths or reps < 1, HFDIB_ESTATE before hfdib_set_indicator. */
int hfdib_autotune_tiles(hfdib_ctx* ctx, int reps, int* best_width, double* ms4);
int hfdib_set_tile_width(hfdib_ctx* ctx, int width);
/* Tile depth of the full-grid kernels: 1 (the default), 2 or 4 planes per
 * 256-thread tile (the tile then spans 256 / (width * depth) rows), so the
 * z-neighbour planes a stencil reads are shared by more cells of one tile.
 * The depth must divide nz (3-D grids only) and width * depth must not exceed
 * 256; otherwise HFDIB_EINVAL and the depth is unchanged.  Results are
 * unchanged up to the order of partial sums in reductions.  hfdib_autotune_tiles
 * times the widths at the current depth (ms4 entry -1 for a width too wide). */
int hfdib_set_tile_depth(hfdib_ctx* ctx, int depth);
/* Order in which the tiles of the full-grid kernels are handed to each XCD
 * (each XCD takes a contiguous run of tiles): zfirst = 0 (the default) x
 * fastest, then y, then z; zfirst = 1 z fastest, so vertically adjacent tiles run
 * together and share their z-neighbour planes in that XCD's L2.  Results are
 * unchanged up to the order of partial sums in reductions.  HFDIB_EINVAL for
 * other values. */
int hfdib_set_tile_order(hfdib_ctx* ctx, int zfirst);

/* Copies one per-boundary-cell record array (HFDIB_IB_*) to dst_dev. */
int hfdib_get_ib_array(hfdib_ctx* ctx, int array_id, void* dst_dev);

/* Solves the pressure-correction system alone: sum_f c_f (p_P - p_nb) +
 * sum_outlet c_b p_P = rhs with c_f = mean(rAU)|S_f|/d_f and
 * c_b = rAU_P|S|/(d/2) on outlet faces of cells with lambda = 0 (requires
 * set_indicator).  rAU_dev, rhs_dev: N doubles; p_dev: initial guess in,
 * solution out.  Conjugate gradients preconditioned by one geometric-multigrid
 * V-cycle; stops at |r| <= rtol |b| or after maxit iterations, where |b| is taken
 * over the coupled rows (an uncoupled row, all of whose coefficients are zero,
 * is the identity p = rhs and its right-hand side does not enter |b|).
 * *iters and *relres (host, nullable) report the outcome.  Waits on the host
 * once per PCG iteration: the device writes the convergence scalars and then a
 * sequence number to a 208-byte pinned, host-coherent buffer that the context
 * allocates on its first solve (EDEVICE if that fails) and frees in
 * hfdib_destroy; the host polls the sequence number (and the stream, for
 * errors).  Returns after the last iteration's scalars have arrived; the
 * solution is complete in stream order (the standalone call also synchronises
 * the stream before returning). */
int hfdib_pressure_solve(hfdib_ctx* ctx, const double* rAU_dev, const double* rhs_dev,
                         double* p_dev, double rtol, int maxit, int* iters, double* relres);

/* Statistics of the last hfdib_simple_iterate call (host, 8 doubles):
 * [0] total PCG iterations, [1] iterations done, [2] max PCG iterations in one
 * solve, [3] last pressure relative residual. */
int hfdib_last_stats(hfdib_ctx* ctx, double* out8);

/* Per-kernel timing with HIP events on the context stream.  enable > 0 starts
 * recording in every enable-th SIMPLE iteration (1: every iteration; calls
 * outside hfdib_simple_iterate are always recorded): the kernel's own start and
 * end are stamped on every launch of the named kernel class, or on the first
 * and last of the 2 n_sweeps consecutive launches of a red-black solve, which
 * count as that many launches (see hfdib_timing_query).  0 stops.  Recording
 * adds a few microseconds per timed launch; off by default.  EINVAL for
 * enable < 0. */
int hfdib_timing_enable(hfdib_ctx* ctx, int enable);
/* kernel_class: 0 pressure operator apply (fine level), 1 momentum sweep,
 * 2 momentum assembly, 3 whole pressure solve, 4 whole SIMPLE iteration,
 * 5 k / eps-omega sweep (one colour), 6 turbulence scalar assembly,
 * 7 fine-level V-cycle half sweep (one colour), 8 fine-level pre-smoothing pass
 * from zero, 9 restriction of the fine residual, 10 operator apply with the
 * direction update, 11 CG vector update (x, r), 12 coarse levels of one V-cycle
 * (one span from the first coarse-level launch to the last, counted as one),
 * 13 reduction finalize launches (every reduction of the iteration),
 * 14 momentum explicit-term pass (transpose viscous term, deferred convection
 * correction).
 * Returns accumulated milliseconds and the launch count (host pointers).
 * Synchronises the stream. */
int hfdib_timing_query(hfdib_ctx* ctx, int kernel_class, double* total_ms, long long* count);

void hfdib_destroy(hfdib_ctx* ctx);

/* ---------------------------------------------------------------- batches
 * Independent contexts (for instance one section at many angles of attack, on
 * grids of different sizes) iterated together by one HIP graph launch.  The
 * batch stream (nullable: the batch then creates and owns one) must differ
 * from every context's stream; contexts may share streams.  hfdib_batch_create captures two SIMPLE iterations of every context,
 * each on a capture stream of its own (created for the capture, released after
 * it) between a fork and a join of the batch stream, with exactly
 * pcg_iters PCG iterations per pressure solve and no host read; a device record
 * per context counts iterations, keeps the first iteration whose maximum
 * normalised residual is <= tol, and flags non-finite residuals.  It finishes
 * the contexts' pending work; the graph references their workspaces, which
 * must stay alive until hfdib_batch_destroy, and the contexts must not be
 * iterated otherwise while a batch run is in flight.  HFDIB_EINVAL: bad
 * arguments, a context listed twice, the batch stream used by a context;
 * HFDIB_ESTATE: a context without set_indicator; HFDIB_EDEVICE: capture or
 * instantiation failed (hfdib_batch_last_error). */
typedef struct hfdib_batch hfdib_batch;
int hfdib_batch_create(hfdib_ctx* const* ctxs, int n, int pcg_iters, double tol, void* hip_stream,
                       hfdib_batch** out);
/* Launches the graph ceil(iters / 2) times on the batch stream (every context
 * advances by two iterations per launch).  Returns after queueing; no host
 * synchronisation with the device.  Work queued on the contexts' own streams
 * before the call is waited for. */
int hfdib_batch_run(hfdib_batch* b, int iters);
/* Waits for the batch stream and copies, per context i (host arrays of n):
 * iters_done[i], conv_iter[i] (first converged iteration counted from
 * hfdib_batch_create, -1 if none) and res[6 i .. 6 i + 5] (last normalised
 * residuals, as hfdib_simple_iterate).  Any array may be null.  Returns
 * HFDIB_EDIVERGED if a context produced a non-finite residual. */
int hfdib_batch_status(hfdib_batch* b, int* conv_iter, int* iters_done, double* res);
const char* hfdib_batch_last_error(const hfdib_batch* b);
void hfdib_batch_destroy(hfdib_batch* b);
const char* hfdib_status_string(int status);
const char* hfdib_last_error(const hfdib_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HFDIB_H */
