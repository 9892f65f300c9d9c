// Momentum predictor, IB forcing/correction, pressure-corrector right-hand side
// and velocity/flux update of the extended SIMPLE loop (figure of the SIMPLE
// algorithm; eqs. of the governing equations, of f_ib and of the correction).
#include "device_common.h"

namespace hfdib {

struct Mom {
  const double* u[3];
  const double* p;
  const double* phi[3];
  const double* nut;
  const double* k;  // (wall functions of no-slip domain faces)
  const uint8_t* flags;
  const double* uib[3];
  const double* us[3];   // solid velocity
  const double* wallD;   // immersed-wall coupling of boundary cells on the logarithmic branch (k_ib_pre)
  const double* ex[3];   // explicit terms of the previous iterate (k_mom_explicit)
};

// FP32 outputs of the momentum assembly under the mixed policy (all null under
// FP64): the defect b - A u_old of each component and the relaxed diagonal used
// by the FP32 sweeps (colour-split)
struct MixOut {
  float* r[3];
  float* a;
  double* us[3];  // FP64 policy: the colour-split copy of u the sweeps work on (else null)
};

// FP32 coefficient mirrors read by the FP32 sweeps
struct Mir32 {
  const float* phi[3];
  const float* nut;
};

__device__ __forceinline__ double nut_wall(const Params& P, double yp) {
  if (!(yp > P.ylam)) return 0.0;
  double v = P.kappa * yp / log(P.E * yp) - 1.0;
  return P.nu * (v > 0.0 ? v : 0.0);
}

// interior neighbour coefficient a_nb = D_f + max(-F_f, 0) (upwind, bounded form)
__device__ __forceinline__ double anb_coef(const Params& P, double gP, double gN, int d, double F) {
  double mf = -F;
  return 0.5 * (gP + gN) * P.AoD[d] + (mf > 0.0 ? mf : 0.0);
}

__device__ __forceinline__ double p_bface(const Params& P, int d, int s, bool solid, double pP) {
  const bool outl = P.p_outlet[2 * d + (s > 0 ? 1 : 0)] != 0;
  return (outl && !solid) ? 0.0 : pP;
}

// V (grad p)_c, Gauss with linear interpolation, from preloaded values: pP = p_c,
// pn[q] = p at the (clamped) face neighbour q of N
__device__ __forceinline__ double gradp_V_nb(const Params& P, bool solid, int cc, const Nbr& N, double pP,
                                             const double (&pn)[6]) {
  const double fp = sel(is_bnd(N, 2 * cc + 1), p_bface(P, cc, +1, solid, pP), 0.5 * (pP + pn[2 * cc + 1]));
  const double fm = sel(is_bnd(N, 2 * cc), p_bface(P, cc, -1, solid, pP), 0.5 * (pn[2 * cc] + pP));
  return P.V * ((fp - fm) * P.idelta[cc]);
}

// ---------------------------------------------------------------- state init
__global__ void k_init_cells(Params P, const double* lam, const double* us0, const double* us1, const double* us2,
                             double* u0, double* u1, double* u2, double* p, double* k, double* w, double* nut) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c >= P.N) return;
  bool fl = lam[c] < 0.5;
  u0[c] = fl ? P.u_in[0] : us0[c];
  u1[c] = fl ? P.u_in[1] : us1[c];
  u2[c] = P.dim == 2 ? 0.0 : (fl ? P.u_in[2] : us2[c]);
  p[c] = 0.0;
  if (P.model == HFDIB_KEPS || P.model == HFDIB_RKEPS) {
    // (realizable k-epsilon starts from the standard C_mu; its variable C_mu
    // acts from the first turbulence update on)
    k[c] = P.k_in;
    w[c] = P.w_in;
    nut[c] = P.Cmu * P.k_in * P.k_in / P.w_in;
  } else if (P.model == HFDIB_KOMEGA_SST || P.model == HFDIB_KOMEGA) {
    k[c] = P.k_in;
    w[c] = P.w_in;
    nut[c] = P.k_in / P.w_in;
  } else {
    k[c] = 0.0;
    w[c] = 0.0;
    nut[c] = 0.0;
  }
}

// face fluxes of a cell vector field: linear interpolation inside; inlet u_in.S,
// outlet owner value, walls / slip / solid-owner faces 0.  Each thread writes the
// high face of its cell and, on the low domain boundary, the low face.
__global__ void k_interp_flux(Params P, const double* v0, const double* v1, const double* v2, const uint8_t* flags,
                              double* phx, double* phy, double* phz) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, k);
  const double* v[3] = {v0, v1, v2};
  double* ph[3] = {phx, phy, phz};
  bool solid = flags[c] & F_SOLID;
  for (int d = 0; d < P.dim; ++d) {
    double A = P.area[d];
    long long f = fidx(P, d, i, j, k);
    long long fo = d == 0 ? 1LL : (d == 1 ? (long long)P.nx : (long long)P.nx * P.ny);
    for (int s = -1; s <= 1; s += 2) {
      if (!on_bnd(P, d, s, i, j, k)) {
        if (s > 0) ph[d][f + fo] = 0.5 * (v[d][c] + v[d][c + stride(P, d)]) * A;
        continue;
      }
      int kind = face_kind(P, d, s);
      double val;
      if (kind == HFDIB_BC_INLET) val = P.u_in[d] * A;
      else if (kind == HFDIB_BC_OUTLET) val = v[d][c] * A;
      else val = 0.0;
      if (solid) val = 0.0;
      ph[d][s > 0 ? f + fo : f] = val;
    }
  }
}

// ---------------------------------------------------------------- IB-pre
// boundary cells: u_tau = Cmu^(1/4) sqrt(k_P), y+ = y_eff u_tau / nu (eq. for
// y+ and u_tau), alpha_u = alpha_k = [y+ <= y+_lam] (eq. for alpha_u), and the
// imposed velocity from the quadratic along n_P through (0,u_s), P1, P2.
// Boundary cells on the logarithmic branch (not forced) get instead, in wallD,
// the change of their momentum diagonal that makes each face shared with an
// in-solid neighbour couple the cell to the solid through the wall function:
// sum over those faces of D_w - D_f, D_w = (nu + nu_w) |n . e_f| A_f / y (nu_w the
// log-law wall viscosity at the cell's y+, y its wall distance), D_f = the
// face-mean diffusivity over the centre distance that the row already holds.
// The momentum assembly adds it to a_P and, times the solid velocity, to the
// right-hand side (the paper's high-Reynolds-number treatment, in which the
// boundary velocity follows from the turbulent viscosity: under the log law the
// momentum flux to the wall is u_tau^2 per unit wall area).
__global__ void k_ib_pre(Params P, int nbc, const int* bc_cells, const double* bc_yeff, const double* bc_L,
                         const int* st1, const double* w1, const int* st2, const double* w2, const double* kold,
                         const double* u0, const double* u1, const double* u2, const double* us0, const double* us1,
                         const double* us2, uint8_t* flags, double* ub0, double* ub1, double* ub2, double* bc_utau,
                         double* bc_yplus, int nw, const int* wall_cells, const double* wall_y, double* wall_utau,
                         double* wall_yplus, const double* bc_n, const double* nut, double* wallD) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nbc + nw) return;
  if (b >= nbc) {
    // free-stream cells next to a no-slip domain face (same launch)
    b -= nbc;
    double ut = 0.0, yp = 0.0;
    if (P.model != HFDIB_LAMINAR) {
      double kk = kold[wall_cells[b]];
      ut = P.Cmu25 * sqrt(kk > 0.0 ? kk : 0.0);
      yp = wall_y[b] * ut / P.nu;
    }
    wall_utau[b] = ut;
    wall_yplus[b] = yp;
    return;
  }
  int c = bc_cells[b];
  double ut = 0.0, yp = 0.0;
  if (P.model != HFDIB_LAMINAR) {
    double kk = kold[c];
    ut = P.Cmu25 * sqrt(kk > 0.0 ? kk : 0.0);
    yp = bc_yeff[b] * ut / P.nu;
  }
  bc_utau[b] = ut;
  bc_yplus[b] = yp;
  bool a = yp <= P.ylam;
  uint8_t f = flags[c];
  flags[c] = a ? (uint8_t)(f | F_ALPHA_U) : (uint8_t)(f & ~F_ALPHA_U);
  if (!a) {
    // (only the in-solid bit of the neighbours' flags is read: it never changes)
    const int i = (int)(c % P.nx), j = (int)((c / P.nx) % P.ny), kz = (int)(c / ((long long)P.nx * P.ny));
    const int ii[3] = {i, j, kz}, nn[3] = {P.nx, P.ny, P.nz};
    const long long st[3] = {1, P.nx, (long long)P.nx * P.ny};
    const double y = bc_yeff[b];
    const double nuw = P.nu + nut_wall(P, yp);
    const double nuP = P.nu + nut[c];
    double dD = 0.0;
    for (int d = 0; d < P.dim; ++d)
      for (int s = -1; s <= 1; s += 2) {
        const int q = ii[d] + s;
        if (q < 0 || q >= nn[d]) continue;
        const long long n = c + s * st[d];
        if (!(flags[n] & F_IC)) continue;
        const double Df = 0.5 * (nuP + (P.nu + nut[n])) * P.area[d] / P.delta[d];
        const double Dw = nuw * P.area[d] * fabs(bc_n[3 * b + d]) / y;
        dD += Dw - Df;
      }
    wallD[c] = dD;
    return;
  }
  const double* uu[3] = {u0, u1, u2};
  const double* us[3] = {us0, us1, us2};
  double* ub[3] = {ub0, ub1, ub2};
  double L0 = bc_L[3 * b], L1 = bc_L[3 * b + 1], L2 = bc_L[3 * b + 2];
  for (int cc = 0; cc < P.dim; ++cc) {
    double v1 = 0.0, v2 = 0.0;
    for (int q = 0; q < 8; ++q) v1 += w1[8 * b + q] * uu[cc][st1[8 * b + q]];
    for (int q = 0; q < 8; ++q) v2 += w2[8 * b + q] * uu[cc][st2[8 * b + q]];
    ub[cc][c] = L0 * us[cc][c] + L1 * v1 + L2 * v2;
  }
}

// ---------------------------------------------------------------- momentum
// Neighbour coefficients of a momentum row: anb[q] for the faces q = 2d + (s>0)
// in the order W, E, S, N, B, T, 0 on domain faces and beyond dim (loads from
// clamped indices, no branches around them)
__device__ __forceinline__ void mom_anb(const Params& P, const Mom& M, double nuP, const Nbr& N, int i, int j, int k,
                                        double (&anb)[6]) {
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int sh = 0; sh < 2; ++sh) {
      const int s = sh ? 1 : -1, q = 2 * d + sh;
      // loads from clamped indices for every face (also beyond dim: the face-flux
      // arrays have their nz + 1 planes in 2-D as well), chosen with selects
      const double a = anb_coef(P, nuP, P.nu + M.nut[N.n[q]], d, outward_flux(P, M.phi, d, s, i, j, k));
      anb[q] = sel(d < P.dim && !is_bnd(N, q), a, 0.0);
    }
}

// Explicit terms of the momentum rows that depend on the previous iterate
// alone, one pass before the assembly: the transpose part of the viscous term,
// div(nuEff (grad u)^T) with face value nuEff_f (d u_d / d x_cc)_f, the face
// gradient being the mean of the two cell gradients; and under the
// higher-order convection schemes (CONV: 0 upwind, 1 linear upwind, 2 van Leer)
// their deferred correction of the upwind rows, -sum_f F_out (u_f - u_C), with C
// the upwind cell of the face, D the downwind one, and the face value
//   linear upwind  u_f = u_C + (x_f - x_C) . grad u_C
//   van Leer       u_f = u_C + psi(r) (u_D - u_C) / 2, psi(r) = (r + |r|) / (1 + |r|),
//                  r = 2 (x_D - x_C) . grad u_C / (u_D - u_C) - 1 (0 where u_D = u_C)
// (interior faces).  The cell gradients (Gauss, linear face interpolation, at
// the cell and at its face neighbours) are taken from u here, not stored: the
// extra u values (edge and second neighbours) come from cache lines the stencil
// already holds.  Out: ex[cc] = the sum of both terms of component cc, and per
// workgroup the sums of u, v, w, p, k over its cells (the iteration means).
template <int CONV, int DIM>
__global__ void __launch_bounds__(256)
k_mom_explicit(Params P, Mom M, double* ex0, double* ex1, double* ex2, double* part, long long pstride) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < P.nx && j < P.ny) {
  const long long c = cidx(P, i, j, k);
  const Nbr N = make_nbr(P, i, j, k, c);
  const bool solid = M.flags[c] & F_SOLID;
  const double nuP = P.nu + M.nut[c];
  double nuN[6], fo[6];
  bool sn[6];  // neighbours with lambda > 0 (domain-face values of their gradients)
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    nuN[q] = P.nu + M.nut[N.n[q]];
    fo[q] = CONV != 0 ? outward_flux(P, M.phi, q >> 1, (q & 1) ? 1 : -1, i, j, k) : 0.0;
    sn[q] = M.flags[N.n[q]] & F_SOLID;
  }
  double ex[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int cc = 0; cc < DIM; ++cc) {
    double T = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      // d u_d / d x_cc at the cell and at its two neighbours along d
      const double GP = gradu_bf(P, M.u[d], d, cc, c, is_bnd(N, 2 * cc), is_bnd(N, 2 * cc + 1), solid);
#pragma unroll
      for (int sh = 0; sh < 2; ++sh) {
        const int s = sh ? 1 : -1, q = 2 * d + sh;
        const bool fb = is_bnd(N, q);
        const double GN = gradu_nb(P, M.u[d], d, cc, N, q, i, j, k, sn[q]);
        const double nuf = sel(fb, nuP, 0.5 * (nuP + nuN[q]));
        const double gf = sel(fb, GP, 0.5 * (GP + GN));
        T += (double)s * P.area[d] * nuf * gf;
      }
    }
    if (CONV != 0) {
      const double uP = M.u[cc][c];
      double Cc = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        // d u_cc / d x_d at the cell and at its two neighbours along d
        const double gP = gradu_bf(P, M.u[cc], cc, d, c, is_bnd(N, 2 * d), is_bnd(N, 2 * d + 1), solid);
#pragma unroll
        for (int sh = 0; sh < 2; ++sh) {
          const int s = sh ? 1 : -1, q = 2 * d + sh;
          const double gN = gradu_nb(P, M.u[cc], cc, d, N, q, i, j, k, sn[q]);
          const double uN = M.u[cc][N.n[q]];
          const double F = fo[q];
          const bool up = F > 0.0;
          const double uC = sel(up, uP, uN), uD = sel(up, uN, uP);
          const double gC = sel(up, gP, gN);
          const double dxC = (double)s * 0.5 * P.delta[d] * sel(up, 1.0, -1.0);
          double uf;
          if (CONV == 1) {
            uf = uC + dxC * gC;
          } else {
            const double dCD = uD - uC;
            const double r = sel(dCD != 0.0, 2.0 * (2.0 * dxC * gC) / dCD - 1.0, 0.0);
            const double psi = (r + fabs(r)) / (1.0 + fabs(r));
            uf = uC + 0.5 * psi * dCD;
          }
          Cc = sel(is_bnd(N, q), Cc, Cc - F * (uf - uC));
        }
      }
      T = T + Cc;
    }
    ex[cc] = T;
  }
  ex0[c] = ex[0];
  ex1[c] = ex[1];
  if (DIM == 3) ex2[c] = ex[2];
  sums[0] = M.u[0][c];
  sums[1] = M.u[1][c];
  sums[2] = M.u[2][c];
  sums[3] = M.p[c];
  sums[4] = M.k[c];
  }
  block_sums_store<5>(sums, part, pstride, block_linear());
}

// The same explicit terms on 3-D grids, with the stencil staged through LDS.
// Computed in place from u, the cell gradients of a cell and its face
// neighbours touch about 60 values of u per cell (edge and second neighbours
// included).  Here a workgroup owns a 32 x 8 column of cells over exz
// consecutive planes and marches along z: a ring of three planes (k - 1, k,
// k + 1) of u, v, w and nu_t, each with a halo of two cells in x and y, sits in
// LDS, so each value is fetched from global memory about twice (halo and the
// plane re-reads at the column ends) and the stencil reads are LDS reads at
// fixed offsets; the values two planes away (d/dz of the z-neighbours'
// gradients) are loaded per cell.  The host chooses exz so that the workgroups
// fill the chip in few rounds.  Each workgroup also sums u, v, w, p and k over
// its cells (the iteration means).
// Domain faces cost no branches or selects in the gradients: a position one
// cell beyond a domain face (and inside the domain along the other axes) is
// staged as the ghost value 2 u_f - u_X of the face value u_f that the Gauss
// gradient of the cell X inside takes on that face, so the interior formula
// 0.5 (u_X + ghost) gives u_f (up to rounding).  Every other position outside
// the domain holds the nearest cell's value and enters only terms the selects
// on domain faces drop (face values of nu_t and of the gradient on a domain
// face are the cell's own, as in the global-memory form).
constexpr int EXTX = 32, EXTY = 8, EXW = EXTX + 4, EXH = EXTY + 4;
inline long long blocks_explicit_z(const Params& P, int exz) {
  return (long long)((P.nx + EXTX - 1) / EXTX) * ((P.ny + EXTY - 1) / EXTY) * ((P.nz + exz - 1) / exz);
}
// u, v, w and nu_t at a position as staged: the values themselves inside the
// domain; one cell beyond exactly one domain face the ghost 2 u_f - u of the
// inner neighbour (face value u_bface, the inner cell's in-solid bit); any
// other outside position, and nu_t at every outside position, the nearest
// cell's values
struct Staged {
  double u[3], nu;
};
// the ghost 2 u_f - u of component q beyond face f (2 d + high side) of a cell
// with value u (u_f the face value of u_bface; the owner's value on faces of
// in-solid cells)
__device__ __forceinline__ double ghost_value(const Params& P, int f, int q, bool solid, double u) {
  double A = 1.0, Bc = 0.0;
#pragma unroll
  for (int ff = 0; ff < 6; ++ff) {
    A = sel(f == ff, P.ubA[ff][q], A);
    Bc = sel(f == ff, P.ubB[ff][q], Bc);
  }
  const double uf = solid ? u : A * u + Bc;
  return 2.0 * uf - u;
}
// ghost face of an outside position (offsets ox, oy, oz beyond the domain):
// the face index when exactly one offset is nonzero and it is +-1, else -1
__device__ __forceinline__ int ghost_face(int ox, int oy, int oz) {
  const int nout = (ox != 0) + (oy != 0) + (oz != 0);
  if (nout != 1 || ox < -1 || ox > 1 || oy < -1 || oy > 1 || oz < -1 || oz > 1) return -1;
  return ox != 0 ? (ox > 0 ? 1 : 0) : (oy != 0 ? (oy > 0 ? 3 : 2) : (oz > 0 ? 5 : 4));
}
__device__ __forceinline__ Staged staged_value(const Params& P, const Mom& M, int gi, int gj, int gk) {
  const int ci = gi < 0 ? 0 : (gi >= P.nx ? P.nx - 1 : gi);
  const int cj = gj < 0 ? 0 : (gj >= P.ny ? P.ny - 1 : gj);
  const int ck = gk < 0 ? 0 : (gk >= P.nz ? P.nz - 1 : gk);
  const long long g = cidx(P, ci, cj, ck);
  Staged v;
#pragma unroll
  for (int q = 0; q < 3; ++q) v.u[q] = M.u[q][g];
  v.nu = M.nut[g];
  const int f = ghost_face(gi - ci, gj - cj, gk - ck);
  if (f >= 0) {  // (positions outside the domain only)
    const bool solid = M.flags[g] & F_SOLID;
#pragma unroll
    for (int q = 0; q < 3; ++q) v.u[q] = ghost_value(P, f, q, solid, v.u[q]);
  }
  return v;
}
// component q alone at (i, j, gk), as staged
__device__ __forceinline__ double staged_u(const Params& P, const Mom& M, int q, int i, int j, int gk) {
  const int ck = gk < 0 ? 0 : (gk >= P.nz ? P.nz - 1 : gk);
  const long long g = cidx(P, i, j, ck);
  double u = M.u[q][g];
  const int f = ghost_face(0, 0, gk - ck);
  if (f >= 0) u = ghost_value(P, f, q, M.flags[g] & F_SOLID, u);
  return u;
}
template <int CONV>
__global__ void __launch_bounds__(256)
k_mom_explicit_z(Params P, Mom M, double* ex0, double* ex1, double* ex2, int exz, double* part, long long pstride) {
  __shared__ double su[3][3][EXH][EXW];        // component, ring slot, y, x
  __shared__ double snu[3][EXH - 2][EXW - 2];  // (face neighbours only: halo of one)
  // workgroup -> (x, y, z-segment), the z-segments of a column contiguous on
  // one XCD (their shared planes stay in that XCD's L2)
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned qq = nb >> 3, rr = nb & 7u, xc = b & 7u, id = b >> 3;
  const unsigned L = xc < rr ? xc * (qq + 1) + id : rr * (qq + 1) + (xc - rr) * qq + id;
  const int bxn = (P.nx + EXTX - 1) / EXTX, bzn = (P.nz + exz - 1) / exz;
  const int tz = (int)(L % (unsigned)bzn), rest = (int)(L / (unsigned)bzn);
  const int i0 = (rest % bxn) * EXTX, j0 = (rest / bxn) * EXTY, k0 = tz * exz;
  const int k1 = k0 + exz < P.nz ? k0 + exz : P.nz;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + EXTX * ly;
  const int i = i0 + lx, j = j0 + ly;
  const bool act = i < P.nx && j < P.ny;
  // a plane is staged in two steps: fetch (global loads into registers, for the
  // thread's two positions of the 36 x 12 plane) and commit (registers to the
  // plane's ring slot); the fetch of plane k + 2 is in flight while plane k is
  // computed
  static_assert(EXW * EXH <= 512 && EXW * EXH > 256, "two staging positions per thread");
  const bool two = tid + 256 < EXW * EXH;
  Staged pf[2];
  auto fetch = [&](int kp) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = r == 0 ? tid : (two ? tid + 256 : tid);
      const int hx = e % EXW, hy = e / EXW;
      pf[r] = staged_value(P, M, i0 + hx - 2, j0 + hy - 2, kp);
    }
  };
  auto commit = [&](int kp) {
    const int sl = (kp + 3) % 3;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (r == 1 && !two) continue;
      const int e = tid + 256 * r;
      const int hx = e % EXW, hy = e / EXW;
      su[0][sl][hy][hx] = pf[r].u[0];
      su[1][sl][hy][hx] = pf[r].u[1];
      su[2][sl][hy][hx] = pf[r].u[2];
      if (hx >= 1 && hx <= EXW - 2 && hy >= 1 && hy <= EXH - 2) snu[sl][hy - 1][hx - 1] = pf[r].nu;
    }
  };
  double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // u, v, w, p, k over the workgroup's cells
  fetch(k0 - 1);
  commit(k0 - 1);
  fetch(k0);
  commit(k0);
  fetch(k0 + 1);
  for (int k = k0; k < k1; ++k) {
    commit(k + 1);
    __syncthreads();
    const int sm = (k + 2) % 3, s0 = k % 3, sp = (k + 1) % 3;
    // values two planes away at this column (the staged form: ghosts one plane
    // beyond a z face), issued before the next plane's fetch, which stays in
    // flight while this plane is computed
    double far[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    if (act) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (CONV == 0 && q != 2) continue;  // (upwind: d/dz of w only)
        far[q][0] = staged_u(P, M, q, i, j, k - 2);
        far[q][1] = staged_u(P, M, q, i, j, k + 2);
      }
    }
    fetch(k + 2);
    if (act) {
      const long long c = cidx(P, i, j, k);
      const Nbr N = make_nbr(P, i, j, k, c);
      // u_q at offset (ox, oy, oz) from the cell (|ox|, |oy| <= 2, |oz| <= 1,
      // or oz = +-2 with ox = oy = 0)
      auto V = [&](int q, int ox, int oy, int oz) -> double {
        if (oz == -2) return far[q][0];
        if (oz == 2) return far[q][1];
        const int sl = oz < 0 ? sm : (oz > 0 ? sp : s0);
        return su[q][sl][ly + 2 + oy][lx + 2 + ox];
      };
      // d u_jc / d x_b at offset o (Gauss gradient, linear face interpolation;
      // domain faces through the ghosts)
      auto grad = [&](int jc, int b, int ox, int oy, int oz) -> double {
        const int ex = b == 0, ey = b == 1, ez = b == 2;
        const double uP = V(jc, ox, oy, oz);
        const double fp = 0.5 * (uP + V(jc, ox + ex, oy + ey, oz + ez));
        const double fm = 0.5 * (V(jc, ox - ex, oy - ey, oz - ez) + uP);
        return (fp - fm) * P.idelta[b];
      };
      const double nuP = P.nu + snu[s0][ly + 1][lx + 1];
      double nuN[6], fo[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int a = q >> 1, s = (q & 1) ? 1 : -1;
        const int ox = a == 0 ? s : 0, oy = a == 1 ? s : 0, oz = a == 2 ? s : 0;
        const int sl = oz < 0 ? sm : (oz > 0 ? sp : s0);
        nuN[q] = P.nu + snu[sl][ly + 1 + oy][lx + 1 + ox];
        fo[q] = CONV != 0 ? outward_flux(P, M.phi, a, s, i, j, k) : 0.0;
      }
      double ex[3];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        double T = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          // d u_d / d x_cc at the cell and at its two neighbours along d
          const double GP = grad(d, cc, 0, 0, 0);
#pragma unroll
          for (int sh = 0; sh < 2; ++sh) {
            const int s = sh ? 1 : -1, q = 2 * d + sh;
            const bool fb = is_bnd(N, q);
            const double GN = grad(d, cc, d == 0 ? s : 0, d == 1 ? s : 0, d == 2 ? s : 0);
            const double nuf = sel(fb, nuP, 0.5 * (nuP + nuN[q]));
            const double gf = sel(fb, GP, 0.5 * (GP + GN));
            T += (double)s * P.area[d] * nuf * gf;
          }
        }
        if (CONV != 0) {
          const double uP = V(cc, 0, 0, 0);
          double Cc = 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            // d u_cc / d x_d at the cell and at its two neighbours along d
            const double gP = grad(cc, d, 0, 0, 0);
#pragma unroll
            for (int sh = 0; sh < 2; ++sh) {
              const int s = sh ? 1 : -1, q = 2 * d + sh;
              const int ox = d == 0 ? s : 0, oy = d == 1 ? s : 0, oz = d == 2 ? s : 0;
              const double gN = grad(cc, d, ox, oy, oz);
              const double uN = V(cc, ox, oy, oz);
              const double F = fo[q];
              const bool up = F > 0.0;
              const double uC = sel(up, uP, uN), uD = sel(up, uN, uP);
              const double gC = sel(up, gP, gN);
              const double dxC = (double)s * 0.5 * P.delta[d] * sel(up, 1.0, -1.0);
              double uf;
              if (CONV == 1) {
                uf = uC + dxC * gC;
              } else {
                const double dCD = uD - uC;
                const double r = sel(dCD != 0.0, 2.0 * (2.0 * dxC * gC) / dCD - 1.0, 0.0);
                const double psi = (r + fabs(r)) / (1.0 + fabs(r));
                uf = uC + 0.5 * psi * dCD;
              }
              Cc = sel(is_bnd(N, q), Cc, Cc - F * (uf - uC));
            }
          }
          T = T + Cc;
        }
        ex[cc] = T;
      }
      ex0[c] = ex[0];
      ex1[c] = ex[1];
      ex2[c] = ex[2];
#pragma unroll
      for (int q = 0; q < 3; ++q) sums[q] += V(q, 0, 0, 0);
      sums[3] += M.p[c];
      sums[4] += M.k[c];
    }
    __syncthreads();
  }
  block_sums_store<5>(sums, part, pstride, blockIdx.x);
}

// Assembly of the relaxed momentum rows with the explicit IB source
// (discrete f_ib = alpha [M(u~) + grad p]), plus the normalised-residual sums
// of the rows that are solved (alpha_u = 0); the explicit terms of the previous
// iterate come from k_mom_explicit (M.ex).
template <int DIM>
__global__ void __launch_bounds__(256)
k_mom_assemble(Params P, Mom M, MixOut X, double* rhs0, double* rhs1, double* rhs2, double* aPr_out,
               const double* means, double* part, long long pstride) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  bool act = i < P.nx && j < P.ny;
  double red[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (act) {
    long long c = cidx(P, i, j, k);
    Nbr N = make_nbr(P, i, j, k, c);
    // the stencil's loads first, with no store in between (a store could alias
    // a later load and would hold it back); conditional terms are selects
    const uint8_t fl = M.flags[c];
    const bool solid = fl & F_SOLID;
    const double nuP = P.nu + M.nut[c];
    double nuN[6], fo[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      nuN[q] = P.nu + M.nut[N.n[q]];
      fo[q] = outward_flux(P, M.phi, q >> 1, (q & 1) ? 1 : -1, i, j, k);
    }
    double uc[DIM], un[DIM][6];
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) {
      uc[cc] = M.u[cc][c];
#pragma unroll
      for (int q = 0; q < 6; ++q) un[cc][q] = M.u[cc][N.n[q]];
    }
    double anb[6];
#pragma unroll
    for (int q = 0; q < 6; ++q)
      anb[q] = sel((q >> 1) < DIM && !is_bnd(N, q), anb_coef(P, nuP, nuN[q], q >> 1, fo[q]), 0.0);
    double aP = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) aP += anb[q];
    // Dirichlet domain faces (inlet, no-slip) of cells with lambda = 0
    double bsrc[3] = {0.0, 0.0, 0.0};
    const double kc = P.model == HFDIB_LAMINAR ? 0.0 : M.k[c];
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int sh = 0; sh < 2; ++sh) {
        const int s = sh ? 1 : -1;
        int kind = face_kind(P, d, s);
        if (kind != HFDIB_BC_INLET && kind != HFDIB_BC_NOSLIP) continue;
        if (!is_bnd(N, 2 * d + sh) || solid) continue;
        double Gb = nuP;
        if (kind == HFDIB_BC_NOSLIP) {
          if (P.model == HFDIB_LAMINAR) {
            Gb = P.nu;
          } else {
            double ut = P.Cmu25 * sqrt(kc > 0.0 ? kc : 0.0);
            double ypf = 0.5 * P.delta[d] * ut / P.nu;
            Gb = P.nu + nut_wall(P, ypf);
          }
        }
        double mf = -fo[2 * d + sh];
        double a = Gb * P.Ab[d] + (mf > 0.0 ? mf : 0.0);
        aP += a;
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) {
          double ubv = kind == HFDIB_BC_INLET ? P.u_in[cc] : 0.0;
          bsrc[cc] += a * ubv;
        }
      }
    const bool alpha = fl & F_ALPHA_U;
    if ((fl & F_BC) && !alpha && P.model != HFDIB_LAMINAR) {
      // boundary cell on the logarithmic branch: immersed-wall coupling (k_ib_pre)
      const double dD = M.wallD[c];
      aP += dD;
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc) bsrc[cc] += dD * M.us[cc][c];
    }
    const double urf = P.urf_u;
    const double aPr = aP / urf;
    double rh[DIM], Ax[DIM];
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) {
      const double b0 = M.ex[cc][c] + bsrc[cc];
      // V (grad p)_c, Gauss with linear interpolation
      const double pP = M.p[c], pp = M.p[N.n[2 * cc + 1]], pm = M.p[N.n[2 * cc]];
      const double fp = sel(is_bnd(N, 2 * cc + 1), p_bface(P, cc, +1, solid, pP), 0.5 * (pP + pp));
      const double fm = sel(is_bnd(N, 2 * cc), p_bface(P, cc, -1, solid, pP), 0.5 * (pm + pP));
      const double g = P.V * ((fp - fm) * P.idelta[cc]);
      const double uo = uc[cc];
      const double r = (1.0 - urf) / urf * aP * uo;
      double nb = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) nb += anb[q] * un[cc][q];
      double rr;
      if (alpha) {
        const double* ub = M.uib[cc];
        double nbt = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          long long n = N.n[q];
          double ut = (M.flags[n] & F_ALPHA_U) ? ub[n] : un[cc][q];
          nbt += anb[q] * ut;
        }
        double ut = ub[c];
        rr = (aP * ut - nbt) + r;
      } else {
        rr = (b0 - g) + r;
      }
      rh[cc] = rr;
      Ax[cc] = aPr * uo - nb;
      if (!alpha) {
        double one = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) one += anb[q];
        double Axb = (aPr - one) * means[cc];
        red[3 * cc + 0] = fabs(rr - Ax[cc]);
        red[3 * cc + 1] = fabs(Ax[cc] - Axb);
        red[3 * cc + 2] = fabs(rr - Axb);
      }
    }
    // rhs and a'_P are stored colour-split; under the mixed policy also the FP64
    // defect of every row (all rows are swept) for the FP32 correction
    const long long sidx = rb_split(P, i, j, k);
    aPr_out[sidx] = aPr;
    double* rhs[3] = {rhs0, rhs1, rhs2};
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) rhs[cc][sidx] = rh[cc];
    if (X.a) {
      X.a[sidx] = (float)aPr;
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc) X.r[cc][sidx] = (float)(rh[cc] - Ax[cc]);
    }
    if (X.us[0] && ((i + j + k) & 1)) {
      // (only the black half: the first half sweep, red, reads the black
      // neighbours and writes the red half itself)
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc) X.us[cc][sidx] = uc[cc];
    }
  }
  block_sums_store<9>(red, part, pstride, block_linear());
}

// u <- u + alpha_u (u_ib - u) (alpha_u = 1) on a forced cell, the value v
// unchanged on the others; u_ib is read on forced cells only
__device__ __forceinline__ double ib_correct(bool forced, double v, const double* uib, long long c) {
  return forced ? v + 1.0 * (uib[c] - v) : v;
}

// one colour of a red-black Gauss-Seidel sweep over the three components, on
// the colour-split copy s of u that the assembly wrote (a one-colour pass reads
// only the other colour's half and writes only its own).  fin: the last half
// sweep (black), which writes u in the natural order instead, for both cells of
// its pair (the red partner is a face neighbour, its final value already
// loaded), with u <- u + alpha_u (u_ib - u) on the forced cells; the split copy
// is dead after it.
__global__ void k_mom_sweep(Params P, Mom M, const double* rhs0, const double* rhs1, const double* rhs2,
                            const double* aPr, double* s0, double* s1, double* s2, double* u0, double* u1, double* u2,
                            int color, int fin) {
  int i, j, k;
  tile_ijk_rb(P, color, i, j, k);
  if (j >= P.ny) return;
  double* uo[3] = {u0, u1, u2};
  if (i >= P.nx) {
    // only the partner of this pair lies in the grid (odd nx)
    const int io = i ^ 1;
    if (fin && io < P.nx) {
      const long long co = cidx(P, io, j, k), so = rb_split(P, io, j, k);
      const double* sv[3] = {s0, s1, s2};
      const bool forced = M.flags[co] & F_ALPHA_U;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        if (cc < P.dim) uo[cc][co] = ib_correct(forced, sv[cc][so], M.uib[cc], co);
    }
    return;
  }
  long long c = cidx(P, i, j, k);
  Nbr N = make_nbr(P, i, j, k, c);
  const long long sidx = rb_split(P, i, j, k);
  // every load of the three rows before the first store (the stores could
  // alias later loads otherwise, which would serialise the components)
  double un[3][6];
  double* s[3] = {s0, s1, s2};
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int q = 0; q < 6; ++q) un[cc][q] = s[cc][nb_split(P, N, i, j, k, q)];
  const double b0 = rhs0[sidx], b1 = rhs1[sidx], b2 = rhs2[sidx], a = aPr[sidx];
  double anb[6];
  mom_anb(P, M, P.nu + M.nut[c], N, i, j, k, anb);
  double nb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int q = 0; q < 6; ++q) nb[cc] += anb[q] * un[cc][q];
  const double v[3] = {(b0 + nb[0]) / a, (b1 + nb[1]) / a, (b2 + nb[2]) / a};
  if (!fin) {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      if (cc < P.dim) s[cc][sidx] = v[cc];
  } else {
    // the partner (i ^ 1) is the west (i odd) or east (i even) neighbour
    const int io = i ^ 1;
    const bool partner = io < P.nx, west = i & 1;
    const long long co = cidx(P, io < P.nx ? io : i, j, k);
    const bool fc = M.flags[c] & F_ALPHA_U, fp = M.flags[co] & F_ALPHA_U;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      if (cc >= P.dim) continue;
      uo[cc][c] = ib_correct(fc, v[cc], M.uib[cc], c);
      if (partner) uo[cc][co] = ib_correct(fp, sel(west, un[cc][0], un[cc][1]), M.uib[cc], co);
    }
  }
}

// Mixed policy: one colour of a red-black Gauss-Seidel sweep of the FP32
// correction d (A d = r, r the FP64 defect of the assembled rows, d = 0 before
// the first sweep), coefficients from the FP32 mirrors.  init: first sweep
// (cells of the other colour set to 0); fin: last sweep of this colour, which
// also writes u <- u_old + d in FP64, then u <- u + alpha_u (u_ib - u) on the
// forced cells.  Equal to the FP64 sweeps from u_old in exact arithmetic.
__global__ void k_mom_sweep32(Params P, Mir32 M, const float* r0, const float* r1, const float* r2, const float* a32,
                              float* d0, float* d1, float* d2, double* u0, double* u1, double* u2, int color, int init,
                              int fin, const uint8_t* flags, const double* ub0, const double* ub1, const double* ub2) {
  int i, j, k;
  tile_ijk_rb(P, color, i, j, k);
  if (j >= P.ny) return;
  bool three = P.dim == 3;
  if (init) {
    // the partner cell of the other colour in this pair starts from d = 0
    int io = i ^ 1;
    if (io < P.nx) {
      const long long so = rb_split(P, io, j, k);
      d0[so] = 0.0f;
      d1[so] = 0.0f;
      if (three) d2[so] = 0.0f;
    }
  }
  if (i >= P.nx) return;
  long long c = cidx(P, i, j, k);
  // defects, diagonal and the corrections d are colour-split (a one-colour pass
  // reads only the other colour's half of d)
  const long long sidx = rb_split(P, i, j, k);
  // loads first (clamped neighbours, selects), stores last
  const float a = a32[sidx], b0 = r0[sidx], b1 = r1[sidx], b2 = r2[sidx];
  float n0 = 0.0f, n1 = 0.0f, n2 = 0.0f;
  if (!init) {
    const Nbr N = make_nbr(P, i, j, k, c);
    const float nu = (float)P.nu;
    const float nuP = nu + M.nut[c];
    float nun[6], fo[6], z0[6], z1[6], z2[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int d = q >> 1, s = (q & 1) ? 1 : -1;
      const long long n = N.n[q];
      const long long f = fidx(P, d, i, j, k) + (s > 0 ? stride(P, d) : 0);
      const long long ns = nb_split(P, N, i, j, k, q);
      nun[q] = M.nut[n];
      fo[q] = M.phi[d][f];
      z0[q] = d0[ns];
      z1[q] = d1[ns];
      z2[q] = d2[ns];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int d = q >> 1;
      const float mf = (q & 1) ? -fo[q] : fo[q];
      float an = 0.5f * (nuP + (nu + nun[q])) * (float)P.AoD[d] + (mf > 0.0f ? mf : 0.0f);
      an = sel(d < P.dim && !is_bnd(N, q), an, 0.0f);
      n0 += an * z0[q];
      n1 += an * z1[q];
      n2 += an * z2[q];
    }
  }
  const float e0 = (b0 + n0) / a, e1 = (b1 + n1) / a, e2 = (b2 + n2) / a;
  double uo[3] = {0.0, 0.0, 0.0};
  bool forced = false;
  if (fin) {
    uo[0] = u0[c];
    uo[1] = u1[c];
    if (three) uo[2] = u2[c];
    forced = flags[c] & F_ALPHA_U;
  }
  d0[sidx] = e0;
  d1[sidx] = e1;
  if (fin) {
    u0[c] = ib_correct(forced, uo[0] + (double)e0, ub0, c);
    u1[c] = ib_correct(forced, uo[1] + (double)e1, ub1, c);
  }
  if (three) {
    d2[sidx] = e2;
    if (fin) u2[c] = ib_correct(forced, uo[2] + (double)e2, ub2, c);
  }
}

// HbyA = (sum a_nb u_nb + rhs + V grad p_old) / a'_P and rAU = V / a'_P
__global__ void k_hbya(Params P, Mom M, const double* rhs0, const double* rhs1, const double* rhs2,
                       const double* aPr, double* h0, double* h1, double* h2, double* rAU) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, k);
  Nbr N = make_nbr(P, i, j, k, c);
  const long long sidx = rb_split(P, i, j, k);
  // loads of the three rows first, stores last
  const uint8_t fl = M.flags[c];
  double un[3][6], pn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    un[0][q] = M.u[0][N.n[q]];
    un[1][q] = M.u[1][N.n[q]];
    un[2][q] = M.u[2][N.n[q]];
    pn[q] = M.p[N.n[q]];
  }
  const double pP = M.p[c], a = aPr[sidx];
  const double b[3] = {rhs0[sidx], rhs1[sidx], rhs2[sidx]};
  double anb[6];
  mom_anb(P, M, P.nu + M.nut[c], N, i, j, k, anb);
  // forced cells: no pressure term in the momentum row (f_ib contains +grad p),
  // hence no pressure-velocity coupling (rAU = 0)
  const bool forced = fl & F_ALPHA_U;
  const bool solid = fl & F_SOLID;
  double H[3];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    double nb = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) nb += anb[q] * un[cc][q];
    H[cc] = sel(forced, nb + b[cc], nb + b[cc] + gradp_V_nb(P, solid, cc, N, pP, pn));
  }
  h0[c] = H[0] / a;
  h1[c] = H[1] / a;
  h2[c] = P.dim == 3 ? H[2] / a : 0.0;
  rAU[c] = forced ? 0.0 : P.V / a;
}

// face flux predictor phi* from HbyA (overwrites phi) and the pressure
// right-hand side -(1 - lambda_P) sum_f phi*_out (lambda-masked continuity)
__global__ void k_flux_rhs(Params P, const double* h0, const double* h1, const double* h2, const double* lam,
                           const uint8_t* flags, const double* pold, double* phx, double* phy, double* phz,
                           double* rhs_p, double* px) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, k);
  const Nbr N = make_nbr(P, i, j, k, c);
  const double* hv[3] = {h0, h1, h2};
  double* ph[3] = {phx, phy, phz};
  // loads first (clamped neighbours), stores last
  const uint8_t fl = flags[c];
  const double l = lam[c], po = pold[c];
  double hc[3], hlo[3], hhi[3];
  uint8_t fn[6];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    hc[d] = hv[d][c];
    hlo[d] = hv[d][N.n[2 * d]];
    hhi[d] = hv[d][N.n[2 * d + 1]];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) fn[q] = flags[N.n[q]];
  const bool solid = fl & F_SOLID;
  double div = 0.0, vlo[3], vhi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double A = P.area[d];
    double vb[2];
#pragma unroll
    for (int sh = 0; sh < 2; ++sh) {
      const int kind = face_kind(P, d, sh ? 1 : -1);
      double v = kind == HFDIB_BC_INLET ? P.u_in[d] * A : (kind == HFDIB_BC_OUTLET ? hc[d] * A : 0.0);
      vb[sh] = solid ? 0.0 : v;
    }
    vlo[d] = sel(is_bnd(N, 2 * d), vb[0], 0.5 * (hlo[d] + hc[d]) * A);
    vhi[d] = sel(is_bnd(N, 2 * d + 1), vb[1], 0.5 * (hc[d] + hhi[d]) * A);
    if (d < P.dim) {
      div -= vlo[d];
      div += vhi[d];
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= P.dim) continue;
    const long long f = fidx(P, d, i, j, k);
    const long long fo = d == 0 ? 1LL : (d == 1 ? (long long)P.nx : (long long)P.nx * P.ny);
    ph[d][f + fo] = vhi[d];
    if (is_bnd(N, 2 * d)) ph[d][f] = vlo[d];
  }
  // lambda-masked continuity (1 - lambda) div u = 0: either div u = 0 wherever
  // lambda < 1, or the predictor divergence weighted by (1 - lambda)
  double rp = P.continuity == 0 ? (l < 1.0 ? -div : 0.0) : -(1.0 - l) * div;
  // a forced cell whose face neighbours are all forced has no pressure coupling:
  // identity row, p unchanged
  bool iso = (fl & F_ALPHA_U) != 0;
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if ((q >> 1) < P.dim && !is_bnd(N, q) && !(fn[q] & F_ALPHA_U)) iso = false;
  rhs_p[c] = iso ? po : rp;
  px[c] = po;  // the pressure solve starts from the current pressure
}

// Pressure of an identity row (a forced cell whose face neighbours are all
// forced): the mean solved pressure of its coupled face neighbours (forced cells
// with a free face neighbour), summed axis by axis, low side first; a row
// without such neighbours keeps its value.  The cell then enters the solve with a
// consistent value when a neighbour leaves the forced group.
__device__ __forceinline__ double decoupled_pressure(const Params& P, const uint8_t* flags, const double* psol, int i,
                                                     int j, int k, long long c) {
  for (int d = 0; d < P.dim; ++d)
    for (int s = -1; s <= 1; s += 2)
      if (!on_bnd(P, d, s, i, j, k) && !(flags[c + s * stride(P, d)] & F_ALPHA_U)) return psol[c];
  double acc = 0.0;
  int cnt = 0;
  for (int d = 0; d < P.dim; ++d)
    for (int s = -1; s <= 1; s += 2) {
      if (on_bnd(P, d, s, i, j, k)) continue;
      long long n = c + s * stride(P, d);
      const int qi = i + (d == 0 ? s : 0), qj = j + (d == 1 ? s : 0), qk = k + (d == 2 ? s : 0);
      bool coupled = false;
      for (int d2 = 0; d2 < P.dim; ++d2)
        for (int s2 = -1; s2 <= 1; s2 += 2)
          if (!on_bnd(P, d2, s2, qi, qj, qk) && !(flags[n + s2 * stride(P, d2)] & F_ALPHA_U)) coupled = true;
      if (coupled) {
        acc += psol[n];
        ++cnt;
      }
    }
  return cnt > 0 ? acc / (double)cnt : psol[c];
}

// flux correction with the solved pressure and relaxation of p (into pnew)
// (mixed policy: also the FP32 mirror of every face flux this cell owns)
struct Phi32Out {
  float* f[3];
};

__global__ void k_flux_correct(Params P, const double* rAU, const double* psol, const double* pold,
                               const uint8_t* flags, double* phx, double* phy, double* phz, double* pnew,
                               Phi32Out m32) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, k);
  const Nbr N = make_nbr(P, i, j, k, c);
  double* ph[3] = {phx, phy, phz};
  // loads first (clamped neighbours), stores last
  const uint8_t fl = flags[c];
  const double rc = rAU[c], psc = psol[c], po = pold[c];
  double rhi[3], phi_hi[3], phi_lo[3], pshi[3];
  long long f[3], fo[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    f[d] = fidx(P, d, i, j, k);
    fo[d] = d == 0 ? 1LL : (d == 1 ? (long long)P.nx : (long long)P.nx * P.ny);
    rhi[d] = rAU[N.n[2 * d + 1]];
    pshi[d] = psol[N.n[2 * d + 1]];
    phi_hi[d] = ph[d][f[d] + fo[d]];
    phi_lo[d] = ph[d][f[d]];
  }
  const bool solid = fl & F_SOLID;
  const double cbv = solid ? 0.0 : rc;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= P.dim) continue;
    const bool lo = is_bnd(N, 2 * d), hi = is_bnd(N, 2 * d + 1);
    const bool out_lo = lo && face_kind(P, d, -1) == HFDIB_BC_OUTLET;
    const bool out_hi = hi && face_kind(P, d, +1) == HFDIB_BC_OUTLET;
    const double cb = cbv * P.Ab[d];
    const double cf = 0.5 * (rc + rhi[d]) * P.AoD[d];
    const double v_in = phi_hi[d] - cf * (pshi[d] - psc);
    const double v_out = phi_hi[d] + cb * psc;
    const double vh = sel(hi, sel(out_hi, v_out, phi_hi[d]), v_in);
    const double vl = sel(out_lo, phi_lo[d] + (-1.0) * cb * psc, phi_lo[d]);
    if (!hi || out_hi) ph[d][f[d] + fo[d]] = vh;
    if (out_lo) ph[d][f[d]] = vl;
    if (m32.f[0]) {
      m32.f[d][f[d] + fo[d]] = (float)vh;
      if (lo) m32.f[d][f[d]] = (float)vl;
    }
  }
  double ps = (fl & F_ALPHA_U) ? decoupled_pressure(P, flags, psol, i, j, k, c) : psc;
  pnew[c] = po + P.urf_p * (ps - po);
}

// u = HbyA - rAU grad p (relaxed p), optional re-imposition of u_ib, copy p
__global__ void k_vel_update(Params P, const double* h0, const double* h1, const double* h2, const double* aPr,
                             const double* pnew, const uint8_t* flags, const double* ub0, const double* ub1,
                             const double* ub2, double* u0, double* u1, double* u2, double* p) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, k);
  const Nbr N = make_nbr(P, i, j, k, c);
  // loads first, stores last
  const uint8_t fl = flags[c];
  const double a = aPr[rb_split(P, i, j, k)], pP = pnew[c];
  const double h[3] = {h0[c], h1[c], h2[c]};
  double pn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) pn[q] = pnew[N.n[q]];
  const bool alpha = (fl & F_ALPHA_U) && P.recorrect;
  const bool forced = fl & F_ALPHA_U;
  const bool solid = fl & F_SOLID;
  double v[3];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) v[cc] = sel(forced, h[cc], h[cc] - gradp_V_nb(P, solid, cc, N, pP, pn) / a);
  if (alpha) {
    // (forced cells only: their u_ib is read there)
    const double ub[3] = {ub0[c], ub1[c], ub2[c]};
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) v[cc] = v[cc] + 1.0 * (ub[cc] - v[cc]);
  }
  u0[c] = v[0];
  u1[c] = v[1];
  if (P.dim == 3) u2[c] = v[2];
}

__global__ void k_copy(long long n, const double* src, double* dst) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c < n) dst[c] = src[c];
}

}  // namespace hfdib

// ====================================================================== host
namespace hfdib {

static Mom make_mom(hfdib_ctx* c) {
  Mom M;
  for (int q = 0; q < 3; ++q) {
    M.u[q] = c->u[q];
    M.phi[q] = c->phi[q];
    M.uib[q] = c->uib[q];
  }
  for (int q = 0; q < 3; ++q) M.us[q] = c->us[q];
  for (int q = 0; q < 3; ++q) M.ex[q] = c->ex[q];
  M.p = c->p;
  M.nut = c->nut;
  M.k = c->k;
  M.flags = c->flags;
  M.wallD = c->wallD;
  return M;
}

__global__ void k_init_ib(Params P, int nic, const int* ic_cells, const double* us0, const double* us1,
                          const double* us2, double* ub0, double* ub1, double* ub2, double* kib) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nic) return;
  int c = ic_cells[b];
  ub0[c] = us0[c];
  ub1[c] = us1[c];
  ub2[c] = us2[c];
  kib[c] = 0.0;
}

__global__ void k_fill(long long n, double* a, double v) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c < n) a[c] = v;
}

// initial conditions (u_in in cells with lambda < 0.5, the solid velocity in
// in-solid cells, p = 0, inlet turbulence) and the derived fluxes / gradients
int init_state(hfdib_ctx* c) {
  const Params& P = c->P;
  int nb = nblocks1(P.N);
  hipLaunchKernelGGL(k_init_cells, dim3(nb), dim3(NTHREADS), 0, c->stream, P, c->lam, c->us[0], c->us[1], c->us[2],
                     c->u[0], c->u[1], c->u[2], c->p, c->k, c->w, c->nut);
  hipLaunchKernelGGL(k_interp_flux, grid3(P), block3(P), 0, c->stream, P, c->u[0], c->u[1], c->u[2], c->flags,
                     c->phi[0], c->phi[1], c->phi[2]);
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(NTHREADS), 0, c->stream, P.N, c->kib, 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(NTHREADS), 0, c->stream, P.N, c->wib, 0.0);
  for (int q = 0; q < 3; ++q)
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(NTHREADS), 0, c->stream, P.N, c->uib[q], 0.0);
  if (c->n_ic > 0)
    hipLaunchKernelGGL(k_init_ib, dim3(nblocks1(c->n_ic)), dim3(NTHREADS), 0, c->stream, P, c->n_ic, c->ic_cells,
                       c->us[0], c->us[1], c->us[2], c->uib[0], c->uib[1], c->uib[2], c->kib);
  // the pressure solve's start vector (each iteration's flux pass sets it
  // again); a plain copy of N doubles, also the reference of known traffic for
  // memory-counter calibration
  hipLaunchKernelGGL(k_copy, dim3(nb), dim3(NTHREADS), 0, c->stream, P.N, (const double*)c->p, c->px);
  HFDIB_CHECK_LAUNCH(c, "init state");
  return refresh_mirrors(c);
}

__global__ void k_residuals(const double* S, int dim, int turb, double* out) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < 3; ++q) {
    const double* r = S + SC_RESSUM + 3 * q;
    out[q] = q < dim ? r[0] / (r[1] + r[2] + 1e-300) : 0.0;
  }
  const double* rp = S + 22;  // pressure residual sums written by the PCG set-up
  out[3] = rp[0] / (rp[1] + rp[2] + 1e-300);
  if (turb) {
    const double* rk = S + SC_RESSUM + 12;
    const double* rw = S + SC_RESSUM + 9;
    out[4] = rk[0] / (rk[1] + rk[2] + 1e-300);
    out[5] = rw[0] / (rw[1] + rw[2] + 1e-300);
  } else {
    out[4] = 0.0;
    out[5] = 0.0;
  }
  // sum of the absolute momentum residuals (blow-up guard of the iteration)
  out[6] = S[SC_RESSUM] + (dim > 1 ? S[SC_RESSUM + 3] : 0.0) + (dim > 2 ? S[SC_RESSUM + 6] : 0.0);
}

// the momentum assembly instance of the configured convection scheme
using MomAssembleFn = void (*)(Params, Mom, MixOut, double*, double*, double*, double*, const double*, double*,
                               long long);
static MomAssembleFn mom_assemble_kernel(const Params& P) {
  return P.dim == 2 ? k_mom_assemble<2> : k_mom_assemble<3>;
}
// the explicit-term pass of the configured convection scheme
using MomExplicitFn = void (*)(Params, Mom, double*, double*, double*, double*, long long);
static MomExplicitFn mom_explicit_kernel(const Params& P) {
  if (P.dim == 2) {
    if (P.conv == HFDIB_CONV_LINEAR_UPWIND) return k_mom_explicit<1, 2>;
    if (P.conv == HFDIB_CONV_VANLEER) return k_mom_explicit<2, 2>;
    return k_mom_explicit<0, 2>;
  }
  if (P.conv == HFDIB_CONV_LINEAR_UPWIND) return k_mom_explicit<1, 3>;
  if (P.conv == HFDIB_CONV_VANLEER) return k_mom_explicit<2, 3>;
  return k_mom_explicit<0, 3>;
}
// (returns the number of workgroups, whose partial sums of u, v, w, p, k are in
// c->partials)
static int launch_mom_explicit(hfdib_ctx* c, const Mom& M) {
  const Params& P = c->P;
  if (P.dim == 3) {
    auto kern = P.conv == HFDIB_CONV_LINEAR_UPWIND ? k_mom_explicit_z<1>
                : (P.conv == HFDIB_CONV_VANLEER ? k_mom_explicit_z<2> : k_mom_explicit_z<0>);
    // planes per workgroup: fewest rounds of resident workgroups (4 per CU for
    // the upwind instance, LDS-bound; 2 for the others, register-bound) times
    // the planes each one stages
    const long long slots = (long long)(P.conv == HFDIB_CONV_UPWIND ? 4 : 2) * c->ncu;
    int best = 8;
    long long bcost = -1;
    for (int z = 4; z <= 16; ++z) {
      // (a partial-sum row holds one entry per workgroup; it is sized for the
      // finest tile grid, which has at least as many tiles as any z here)
      if (blocks_explicit_z(P, z) > c->pstride) continue;
      const long long cost = (blocks_explicit_z(P, z) + slots - 1) / slots * (z + 2);
      if (bcost < 0 || cost < bcost) {
        bcost = cost;
        best = z;
      }
    }
    const int nb = (int)blocks_explicit_z(P, best);
    LaunchEv ev = timer_launch(c, T_MOMEXPL, true, true);
    launch_ev(kern, dim3((unsigned)nb), dim3(EXTX, EXTY, 1), c->stream, ev, P, M, c->ex[0], c->ex[1], c->ex[2], best,
              c->partials, c->pstride);
    return nb;
  }
  const Params PA = deep_tile_params(P);
  const dim3 g = grid3(PA);
  LaunchEv ev = timer_launch(c, T_MOMEXPL, true, true);
  launch_ev(mom_explicit_kernel(PA), g, block3(PA), c->stream, ev, PA, M, c->ex[0], c->ex[1], c->ex[2], c->partials,
            c->pstride);
  return (int)((long long)g.x * g.y * g.z);
}

// One round of the kernels the tile autotuner times: the explicit-term pass,
// the momentum assembly and the pressure operator.  None of them changes the
// state (the pass and assembly outputs are recomputed from the same state by the
// next iteration; the operator writes a PCG scratch vector).
int tile_bench_round(hfdib_ctx* c) {
  const Params& P = c->P;
  Mom M = make_mom(c);
  launch_mom_explicit(c, M);
  MixOut X{{nullptr, nullptr, nullptr}, nullptr};
  const Params PA = deep_tile_params(P);
  hipLaunchKernelGGL(mom_assemble_kernel(P), grid3(PA), block3(PA), 0, c->stream, PA, M, X, c->rhs[0], c->rhs[1],
                     c->rhs[2], c->aPr, c->scal + SCAL_PCG + SC_MEANS, c->partials, c->pstride);
  pressure_apply_bench(c);
  HFDIB_CHECK_LAUNCH(c, "tile bench");
  return HFDIB_OK;
}

__global__ void k_to_f32_n(long long n, const double* a, float* b) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c < n) b[c] = (float)a[c];
}

// mixed policy: FP32 mirrors of the sweep coefficients (face fluxes, nu_t, SST
// blending) from the FP64 state, after initialisation or after the state was
// set from outside; during iterations the producing kernels keep them current
int refresh_mirrors(hfdib_ctx* c) {
  const Params& P = c->P;
  if (P.precision != HFDIB_MIXED) return HFDIB_OK;
  long long nf[3] = {(long long)(P.nx + 1) * P.ny * P.nz, (long long)P.nx * (P.ny + 1) * P.nz,
                     (long long)P.nx * P.ny * (P.nz + 1)};
  for (int d = 0; d < 3; ++d)
    hipLaunchKernelGGL(k_to_f32_n, dim3(nblocks1(nf[d])), dim3(NTHREADS), 0, c->stream, nf[d], c->phi[d],
                       c->phi32[d]);
  hipLaunchKernelGGL(k_to_f32_n, dim3(nblocks1(P.N)), dim3(NTHREADS), 0, c->stream, P.N, c->nut, c->nut32);
  HFDIB_CHECK_LAUNCH(c, "mirrors");
  return HFDIB_OK;
}

int simple_step(hfdib_ctx* c, int it, double* res_host) {
  (void)it;
  const Params& P = c->P;
  const dim3 b = block3(P);
  double* S = c->scal + SCAL_PCG;
  int st;
  // the explicit momentum terms of the previous iterate, and its means (the
  // residual normalisation) from the same pass; opens the timing span of the
  // iteration
  timer_begin(c, T_ITER);
  Mom M = make_mom(c);
  const int nbx = launch_mom_explicit(c, M);
  launch_finalize(c, nbx, 5, SC_MEANS, 0, (double)P.N);
  // 1. IB-pre
  if (c->n_bc + c->n_wall > 0)
    hipLaunchKernelGGL(k_ib_pre, dim3(nblocks1(c->n_bc + c->n_wall)), dim3(NTHREADS), 0, c->stream, P, c->n_bc,
                       c->bc_cells, c->bc_yeff, c->bc_L, c->bc_s1, c->bc_w1, c->bc_s2, c->bc_w2, c->k, c->u[0],
                       c->u[1], c->u[2], c->us[0], c->us[1], c->us[2], c->flags, c->uib[0], c->uib[1], c->uib[2],
                       c->bc_utau, c->bc_yplus, c->n_wall, c->wall_cells, c->wall_y, c->wall_utau, c->wall_yplus,
                       c->bc_n, c->nut, c->wallD);
  // 2. momentum predictor
  bool mixed = P.precision == HFDIB_MIXED;
  MixOut X{{nullptr, nullptr, nullptr}, nullptr, {c->usp[0], c->usp[1], c->usp[2]}};
  if (mixed) X = MixOut{{c->r32[0], c->r32[1], c->r32[2]}, c->a32, {nullptr, nullptr, nullptr}};
  LaunchEv ev = timer_launch(c, T_MOMASM, true, true);
  const Params PA = deep_tile_params(P);
  const dim3 ga = grid3(PA);
  launch_ev(mom_assemble_kernel(P), ga, block3(PA), c->stream, ev, PA, M, X, c->rhs[0], c->rhs[1], c->rhs[2], c->aPr,
            S + SC_MEANS, c->partials, c->pstride);
  launch_finalize(c, (int)((long long)ga.x * ga.y * ga.z), 9, SC_RESSUM, 0);
  Mir32 M32{{c->phi32[0], c->phi32[1], c->phi32[2]}, c->nut32};
  // (one timing span over the 2 n_s consecutive launches)
  for (int s = 0; s < P.n_sweeps; ++s)
    for (int color = 0; color < 2; ++color) {
      const bool first = s == 0 && color == 0, last = s == P.n_sweeps - 1 && color == 1;
      ev = timer_launch(c, T_MOMSWEEP, first, last, 2 * P.n_sweeps);
      if (mixed)
        launch_ev(k_mom_sweep32, grid3_rb(P), b, c->stream, ev, P, M32, c->r32[0], c->r32[1], c->r32[2], c->a32,
                  c->d32[0], c->d32[1], c->d32[2], c->u[0], c->u[1], c->u[2], color, first ? 1 : 0,
                  s == P.n_sweeps - 1 ? 1 : 0, (const uint8_t*)c->flags, (const double*)c->uib[0],
                  (const double*)c->uib[1], (const double*)c->uib[2]);
      else
        launch_ev(k_mom_sweep, grid3_rb(P), b, c->stream, ev, P, M, c->rhs[0], c->rhs[1], c->rhs[2], c->aPr,
                  c->usp[0], c->usp[1], c->usp[2], c->u[0], c->u[1], c->u[2], color, last ? 1 : 0);
    }
  // 3. u <- u + alpha_u (u_ib - u): done by the last half sweep
  // 4. pressure corrector
  {
    const Params PH = deep_tile_params(P, true);
    hipLaunchKernelGGL(k_hbya, grid3(PH), block3(PH), 0, c->stream, PH, M, c->rhs[0], c->rhs[1], c->rhs[2], c->aPr,
                       c->hbya[0], c->hbya[1], c->hbya[2], c->rAU);
  }
  // the flux predictor, the flux correction and the velocity update on the
  // z-first tiles too (planes of at most 32768 cells, as HbyA): 48 -> 43 us
  // for the correction at 2.36 M cells
  const Params PF = deep_tile_params(P, true);
  const dim3 gf = grid3(PF), bf = block3(PF);
  hipLaunchKernelGGL(k_flux_rhs, gf, bf, 0, c->stream, PF, c->hbya[0], c->hbya[1], c->hbya[2], c->lam, c->flags,
                     c->p, c->phi[0], c->phi[1], c->phi[2], c->rhs_p, c->px);
  HFDIB_CHECK_LAUNCH(c, "momentum stage");
  int iters = 0;
  double relres = 0.0;
  st = pressure_solve(c, c->rAU, c->rhs_p, c->px, c->cfg.p_rtol, c->cfg.p_maxit, &iters, &relres, S + SC_MEANS + 3);
  if (st != HFDIB_OK) return st;
  c->stats[0] += iters;
  c->stats[2] = iters > c->stats[2] ? iters : c->stats[2];
  c->stats[3] = relres;
  // 5. flux and velocity update
  Phi32Out m32{{nullptr, nullptr, nullptr}};
  if (mixed) m32 = Phi32Out{{c->phi32[0], c->phi32[1], c->phi32[2]}};
  hipLaunchKernelGGL(k_flux_correct, gf, bf, 0, c->stream, PF, c->rAU, c->px, c->p, c->flags, c->phi[0], c->phi[1],
                     c->phi[2], c->pnew, m32);
  hipLaunchKernelGGL(k_vel_update, gf, bf, 0, c->stream, PF, c->hbya[0], c->hbya[1], c->hbya[2], c->aPr, c->pnew,
                     c->flags, c->uib[0], c->uib[1], c->uib[2], c->u[0], c->u[1], c->u[2], c->p);
  double* tmp = c->p;
  c->p = c->pnew;
  c->pnew = tmp;
  HFDIB_CHECK_LAUNCH(c, "velocity update");
  // 6. turbulence
  if (P.model != HFDIB_LAMINAR) {
    st = turbulence_stage(c);
    if (st != HFDIB_OK) return st;
  }
  ev = timer_launch(c, T_ITER, false, true);
  launch_ev(k_residuals, dim3(1), dim3(64), c->stream, ev, S, P.dim, P.model != HFDIB_LAMINAR ? 1 : 0, S + SC_RES);
  HFDIB_CHECK_LAUNCH(c, "residuals");
  if (res_host) {
    HFDIB_CHECK(c, hipMemcpyAsync(res_host, S + SC_RES, 7 * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                "residual copy");
    HFDIB_CHECK(c, hipStreamSynchronize(c->stream), "residual sync");
  }
  return HFDIB_OK;
}

}  // namespace hfdib
