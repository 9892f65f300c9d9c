// Internal declarations of the HFDIB SIMPLE library (gfx950, HIP).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/hfdib.h"

namespace hfdib {

// cell flag bits (uint8 per cell)
enum : uint8_t {
  F_IC = 1u,       // in-solid cell (lambda >= 0.5)
  F_BC = 2u,       // boundary cell
  F_SOLID = 4u,    // lambda > 0 (domain faces of such cells are walls inside the solid)
  F_ALPHA_U = 8u,  // alpha_u = alpha_k of the current iteration
  F_ALPHA_W = 16u, // alpha_omega (in-solid, boundary and domain-wall cells)
  F_WALL = 32u,    // free-stream cell next to a no-slip domain face
  F_RED = 64u      // (i+j+k) even
};

constexpr int NTHREADS = 256;
constexpr int MAX_PARTIAL_BLOCKS = 2048;  // per reduction slot
constexpr int NRED = 24;                  // reduction slots per pass
constexpr int MAX_LEVELS = 12;
constexpr int FIN2_STRIDE = 1024;         // second-stage partials per reduction row
constexpr int TILE_LOG2_MIN = 5, TILE_LOG2_MAX = 8;  // tile widths 32 .. 256 cells

// Plain-old-data parameters passed by value to every kernel.
struct Params {
  int dim, nx, ny, nz;
  long long N;
  // colour-split storage of per-row arrays of the red-black solves: colour
  // (i+j+k)&1 first, then (k, j, i/2); nxh = (nx+1)/2 slots per row and colour,
  // nrb = nz ny nxh slots per colour
  int nxh;
  long long nrb;
  double x0, y0, z0, dx, dy, dz;
  double area[3], delta[3], V, h;
  int bc[6];
  double u_in[3], k_in, w_in;  // w_in: eps_in (k-eps) or omega_in (SST)
  int model;
  int n_sweeps;
  double nu, urf_u, urf_p, urf_t;
  double Cmu, kappa, E, beta1_wf, Ceps2_wf, C_wf, ylam;
  double C1, C2, sigma_k, sigma_eps;
  double sigma_k1, sigma_w1, beta_1, gamma_1, sigma_k2, sigma_w2, beta_2, gamma_2, a1, c_lim;
  double alpha_kw, beta_kw, isig_k_kw, isig_w_kw;  // standard k-omega (1/sigma host-computed)
  double A0_rke, C2_rke, isig_k_rke, isig_eps_rke; // realizable k-epsilon
  int yplus_perp;                                  // 1: y+ from y_perp alone
  int conv;                                        // momentum convection (hfdib_conv_scheme)
  double bound_frac, yperp_min_frac, cd_floor;
  double Cmu25, sqrtCmu;  // Cmu^(1/4), sqrt(Cmu) (host-computed)
  // host-computed reciprocals (kernels multiply instead of dividing): |S_d|/d_d,
  // |S_d|/(d_d/2) for boundary faces, 1/d_d, 1/sigma_k and 1/sigma_eps
  double AoD[3], Ab[3], idelta[3], isig_k, isig_eps;
  // boundary face values as affine maps of the owner value (cells with
  // lambda = 0): velocity component cc on face f = 2d + (s > 0) is
  // ubA[f][cc] u_P + ubB[f][cc]; scalars take their inlet value where
  // sc_inlet[f] != 0; the pressure is 0 where p_outlet[f] != 0
  double ubA[6][3], ubB[6][3];
  int sc_inlet[6], p_outlet[6];
  int recorrect;
  int continuity;
  int precision;  // HFDIB_FP64 or HFDIB_MIXED
  int tx_log2;    // tile width of the full-grid kernels: 2^tx_log2 cells (5..8), 256 threads per tile
  int tz_log2;    // tile depth: 2^tz_log2 planes (0..2; 2^tz_log2 divides nz, tx_log2 + tz_log2 <= 8)
  int tile_zfirst;  // 1: tiles ordered z fastest within each XCD's run (else x, then y, then z)
  int p_nu;         // red-black sweeps before and after the coarse correction on the fine pressure level
  int p_nu_c;       // the same on the coarse levels
};

// Coarse multigrid level (level 0 is the fine grid, matrix free from rAU).
// FP64 storage under the FP64 policy, FP32 storage under the mixed policy (the
// other set of pointers is null).
struct Level {
  int nx, ny, nz;
  long long N;
  double* r;
  double* z;
  double* cx;    // (nx+1)*ny*nz face coefficients
  double* cy;    // nx*(ny+1)*nz
  double* cz;    // nx*ny*(nz+1)
  double* diag;  // N
  float *r32, *z32, *cx32, *cy32, *cz32, *diag32;
};

struct Timers;

}  // namespace hfdib

struct hfdib_ctx {
  hfdib_grid_desc desc;
  hfdib_config cfg;
  hfdib::Params P;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  int ready;  // set_indicator done
  int ncu;    // compute units of the device (launch shapes)
  std::string err;

  // --- cell arrays (N)
  double *u[3], *p, *k, *w, *nut, *lam, *dw;
  double *rhs[3], *aPr, *hbya[3], *rAU, *F1;
  double *uib[3], *kib, *wib, *Pk, *us[3];
  double *t0, *t1, *t2;  // scratch (turbulence rhs / diagonal)
  double* wallD;  // immersed-wall coupling of boundary cells on the logarithmic branch
  // 2 S:S of the current velocity (written by the first turbulence pass of an
  // iteration, read by the production terms)
  double* S2;
  // explicit momentum terms of the previous iterate (transpose viscous term and
  // deferred convection correction), written before each assembly
  double* ex[3];
  double *rhs_p, *px, *pr, *pz, *pd, *pq, *pnew;
  double* pd2;  // second PCG search-direction buffer (the direction update writes the other one)
  double* invD;  // inverse diagonal of the fine pressure operator (FP64 policy), colour-split
  double *pzs, *prs;  // colour-split z and r of the V-cycle's fine level (FP64 policy)
  double* usp[3];     // colour-split copy of u for the momentum sweeps (FP64 policy)
  double* xsp;        // colour-split copy of k or eps/omega for the scalar sweeps (FP64 policy)
  uint8_t* flags;
  // --- face arrays
  double* phi[3];
  // --- FP32 arrays of the mixed policy (null under FP64): defects and
  // corrections of the stencil solves, mirrors of the sweep coefficients
  // (relaxed diagonal, face fluxes, nu_t, SST blending), pressure smoother
  // inputs (rAU) and the preconditioner residual / output
  float *r32[3], *d32[3], *a32, *phi32[3], *nut32;  // (r32, d32, a32 colour-split)
  float *rAU32, *pr32, *pz32, *invD32;
  float *pzs32, *prs32;  // colour-split z and r of the V-cycle's fine level (mixed policy)
  float* gam32;  // FP32 diffusivity of the scalar being solved (mixed policy)
  // --- lists
  int cap;  // capacity of each list
  int *bc_cells, *ic_cells, *wall_cells;
  double *bc_n, *bc_yperp, *bc_yeff, *bc_L, *bc_w1, *bc_w2, *bc_yplus, *bc_utau, *bc_utauU;
  int *bc_mode, *bc_s1, *bc_s2;
  double *wall_y, *wall_n, *wall_yplus, *wall_utau;
  int n_bc, n_ic, n_wall;
  // --- interface points for the SST wall distance
  double* ipts;  // 3*cap
  int n_ipts;
  // --- reductions
  double* partials;  // 16 rows of pstride partial sums
  long long pstride;
  double* partials2; // 16 rows of FIN2_STRIDE second-stage partials
  double* scal;      // 512 scalars
  int* iscal;        // 64 ints
  // pinned, host-coherent mirror of the first NMIR PCG scalars and, after
  // them, the sequence number of the CG step that wrote them (the host waits
  // for it instead of synchronising the stream)
  double* hmir;
  double* hmir_dev;    // its device address
  long long mir_seq;   // sequence number of the last CG step enqueued
  int pcg_prev_iters;  // CG steps of the previous adaptive solve (0: none yet)
  // --- multigrid
  int nlev;
  hfdib::Level lev[hfdib::MAX_LEVELS];
  // --- graph mode (batched replay): fixed PCG iteration count, no host reads
  int graph_mode, graph_pcg;
  // --- stats
  double stats[8];
  double last_pres[3];
  // --- timing
  hfdib::Timers* timers;
};

namespace hfdib {

// launch helpers
// Full-grid kernels run 256-thread tiles of 2^tx_log2 x 2^(8 - tx_log2 - tz_log2)
// cells (the width chosen by hfdib_autotune_tiles; 64 x 4 x 1 by default)
// and 2^tz_log2 planes (a depth that divides nz: no tile reaches past the grid
// in z, so the kernels only bound i and j)
inline dim3 grid3(const Params& P) {
  const int TX = 1 << P.tx_log2, TY = 256 >> (P.tx_log2 + P.tz_log2);
  return dim3((unsigned)(((P.nx + TX - 1) / TX) * ((P.ny + TY - 1) / TY) * (P.nz >> P.tz_log2)), 1, 1);
}
inline dim3 block3(const Params& P) {
  return dim3(1u << P.tx_log2, 256u >> (P.tx_log2 + P.tz_log2), 1u << P.tz_log2);
}
// grid of the red-black half sweeps (half the x extent, see tile_ijk_rb)
inline dim3 grid3_rb(const Params& P) {
  const int TX = 1 << P.tx_log2, TY = 256 >> (P.tx_log2 + P.tz_log2);
  return dim3((unsigned)((((P.nx + 1) / 2 + TX - 1) / TX) * ((P.ny + TY - 1) / TY) * (P.nz >> P.tz_log2)), 1, 1);
}
// Launch shape of the stencil kernels that read many arrays at their
// z-neighbours (the momentum assembly, HbyA, the velocity gradient): 32 x 2 x 4
// tiles in z-first order wherever the grid allows (3-D, nz a multiple of 4),
// since tiles over four planes re-read fewer planes (the momentum assembly:
// 157 -> 146 us at 2.36 M cells); elsewhere, and for every other kernel, the
// configured tiles
// plane_limited: only on planes of at most 32768 cells (HbyA and the velocity
// gradient run faster on these tiles with 256 x 96 planes and slower with
// 512 x 192 planes; our reading: the z-first runs of tiles come back to their y-halo rows
// after these have left the L2)
inline Params deep_tile_params(const Params& P, bool plane_limited = false) {
  Params A = P;
  if (P.dim == 3 && P.nz % 4 == 0 && (!plane_limited || (long long)P.nx * P.ny <= 32768)) {
    A.tx_log2 = 5;
    A.tz_log2 = 2;
    A.tile_zfirst = 1;
  }
  return A;
}
// blocks of the stored multigrid levels (3-D grids of 64 x 4 tiles)
inline dim3 block_lv() { return dim3(64, 4, 1); }
inline int nblocks1(long long n) {
  long long b = (n + NTHREADS - 1) / NTHREADS;
  return (int)(b < 1 ? 1 : b);
}
// blocks of the streaming sums (each thread adds SUM_PER cells)
constexpr int SUM_PER = 8;
inline int nblocks_sum(long long n) { return nblocks1((n + SUM_PER - 1) / SUM_PER); }

// error plumbing
int set_hip_error(hfdib_ctx* c, hipError_t e, const char* where);
#define HFDIB_CHECK_LAUNCH(ctx, where)                                  \
  do {                                                                  \
    hipError_t _e = hipGetLastError();                                  \
    if (_e != hipSuccess) return hfdib::set_hip_error(ctx, _e, where);  \
  } while (0)
#define HFDIB_CHECK(ctx, call, where)                                  \
  do {                                                                 \
    hipError_t _e = (call);                                            \
    if (_e != hipSuccess) return hfdib::set_hip_error(ctx, _e, where); \
  } while (0)

// timing classes
enum { T_PAPPLY = 0, T_MOMSWEEP = 1, T_MOMASM = 2, T_PSOLVE = 3, T_ITER = 4, T_SCALSWEEP = 5, T_SCALASM = 6,
       T_PSMOOTH = 7, T_PPRESMOOTH = 8, T_PRESTRICT = 9, T_PAPPLYDIR = 10, T_PAXPY = 11, T_PCOARSE = 12,
       T_FINALIZE = 13, T_MOMEXPL = 14, T_NCLASS = 15 };
void timer_begin(hfdib_ctx* c, int cls);
// brackets one SIMPLE iteration (begin = true at its start, false at its end):
// with a recording period n > 1 only every n-th iteration is recorded
void timer_iteration(hfdib_ctx* c, bool begin);
// closes the open span of class cls, which covered `launches` consecutive
// launches of that class (its per-launch average divides by them)
void timer_end(hfdib_ctx* c, int cls, int launches = 1);
// events of one kernel launch in a timed span of class cls, for
// hipExtLaunchKernelGGL (the runtime stamps them with the kernel's own start
// and end, no marker packets): `start` when the launch opens the span, `stop`
// when it closes a span of `launches` consecutive launches; null when timing is
// off or for launches inside the span
struct LaunchEv {
  hipEvent_t start, stop;
};
LaunchEv timer_launch(hfdib_ctx* c, int cls, bool first, bool last, int launches = 1);
// launch with the span events of timer_launch (a plain launch when it has none,
// e.g. with timing off or under graph capture)
template <typename K, typename... A>
inline void launch_ev(K kernel, dim3 grid, dim3 block, hipStream_t stream, LaunchEv ev, A... args) {
  if (ev.start || ev.stop)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, ev.start, ev.stop, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, stream, args...);
}

// stages (each returns an hfdib_status)
int geometry_precompute(hfdib_ctx* c);
int init_state(hfdib_ctx* c);
int simple_step(hfdib_ctx* c, int it, double* res6_dev_slot);
int pressure_solve(hfdib_ctx* c, const double* rAU, const double* rhs, double* x, double rtol,
                   int maxit, int* iters, double* relres, const double* xmean_dev);
int refresh_mirrors(hfdib_ctx* c);

// deterministic reduction of `nval` rows of per-block partial sums into
// ctx->scal[SCAL_PCG + out + v]; op selects a PCG scalar update (pressure.hip)
// (hmir: after the update, copy scal[SCAL_PCG .. SCAL_PCG + NMIR) to that host
// mirror, then write seq to hmir[NMIR])
void launch_finalize(hfdib_ctx* c, int nblk, int nval, int out, int op, double divisor = 1.0, int row0 = 0,
                     double* hmir = nullptr, double seq = 0.0);
int turbulence_stage(hfdib_ctx* c);
int body_forces(hfdib_ctx* c, double* out8);
int body_forces_noalloc(hfdib_ctx* c, double* out8_dev);
int tile_bench_round(hfdib_ctx* c);
void pressure_apply_bench(hfdib_ctx* c);
// offsets (relative to SCAL_PCG) of device scalars
enum {
  SC_MEANS = 100,    // means of u, v, w, p, k (5) and of omega/eps after fixing (1)
  SC_RESSUM = 120,   // residual sums: U 9, omega/eps 3, k 3
  SC_RES = 150,      // normalised residuals Ux, Uy, Uz, p, k, eps/omega
  SC_WMAX = 160,     // max of omega/eps over boundary and free-stream cells
  SC_FORCE = 170,    // body-force sums (8)
  SC_CONV = 180      // batched runs: iterations done, first converged iteration (-1), non-finite flag
};
constexpr int SCAL_PCG = 64;
constexpr int NMIR = 25;  // PCG scalars mirrored to the host (S_RR, S_BB, the residual sums)

}  // namespace hfdib
