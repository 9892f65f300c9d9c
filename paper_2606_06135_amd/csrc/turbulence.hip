// Turbulence stage of the extended SIMPLE loop: alpha_omega, imposed omega
// (eps) and production, the omega (eps) equation with fixed rows, k_ib, the k
// equation with S_ib, the k correction and the turbulent viscosity
// (Sec. "Treatment of production and dissipation of k", eqs. for the imposed
// values, k_vis, u_tau, omega_ib and P_ib; k-epsilon and Menter SST closures).
#include "device_common.h"

namespace hfdib {

// production of k by the closure (k-eps: nu_t 2S:S; SST: limited by
// c_lim beta* k omega), from the current velocity and the k, omega, nu_t
// entering the turbulence stage
__device__ __forceinline__ double model_production(const Params& P, double S2, double nut, double kk, double ww) {
  double Gp = nut * S2;
  if (P.model != HFDIB_KOMEGA_SST) return Gp;
  double lim = P.c_lim * P.Cmu * kk * ww;
  return Gp < lim ? Gp : lim;
}

__device__ __forceinline__ double omega_ib(const Params& P, double yp, double y, double ut) {
  if (yp <= P.ylam) return 6.0 * P.nu / (P.beta1_wf * (y * y));
  return ut / (P.kappa * P.sqrtCmu * y);
}
__device__ __forceinline__ double prod_ib(const Params& P, double yp, double Gk, double ng2) {
  if (yp <= P.ylam) return Gk;
  double lg = log(P.E * yp);
  return P.kappa * P.nu * yp * ng2 / (lg * lg);
}

// boundary cells (mode 0) and domain-wall cells (mode 1): imposed omega/eps and
// production; the omega field takes its fixed value on these rows
struct Vel {
  const double* u[3];
};

// Realizable k-epsilon (Shih et al. 1995): invariants S:S, Omega:Omega and
// S_ij S_jk S_ki of the deviatoric strain rate S and the rotation rate Omega of
// the velocity gradient G[a][b] = d u_b / d x_a of cell c with neighbours N
// (Gauss, from u; entries beyond dim are 0; the transposed tensor has the same
// invariants)
struct RkeInv {
  double SS, OO, S3;
};
__device__ __forceinline__ RkeInv rke_invariants(const Params& P, const Vel& U, bool solid, const Nbr& N,
                                                 long long c) {
  double G[3][3];
  gradu_all_bf(P, U.u, solid, N, c, G);
  const double tr = G[0][0] + G[1][1] + G[2][2];
  double S[3][3];
  RkeInv I{0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      S[a][b] = 0.5 * (G[a][b] + G[b][a]) - (a == b ? tr / 3.0 : 0.0);
      double o = 0.5 * (G[a][b] - G[b][a]);
      I.SS += S[a][b] * S[a][b];
      I.OO += o * o;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int e = 0; e < 3; ++e) I.S3 += S[a][b] * S[b][e] * S[e][a];
  return I;
}
// C_mu = 1 / (A0 + A_s U* k / eps), A_s = sqrt(6) cos(arccos(sqrt(6) W) / 3),
// W = S_ij S_jk S_ki / (S:S)^1.5 (0 without strain, sqrt(6) W clipped to [-1, 1])
__device__ __forceinline__ double rke_cmu(const Params& P, const RkeInv& I, double kk, double ee) {
  double W = I.SS > 0.0 ? I.S3 / pow(I.SS, 1.5) : 0.0;
  double x = sqrt(6.0) * W;
  x = x < -1.0 ? -1.0 : (x > 1.0 ? 1.0 : x);
  double As = sqrt(6.0) * cos(acos(x) / 3.0);
  double Us = sqrt(I.SS + I.OO);
  return 1.0 / (P.A0_rke + As * Us * kk / ee);
}

// one list of wall-function cells: boundary cells, or free-stream cells at
// no-slip domain faces (distance, normal, y+ and u_tau per entry)
struct WallList {
  int n;
  const int* cells;
  const double* y;
  const double* nv;
  const double* ypl;
  const double* utl;
};

// diffusion coefficient of the transported scalar (0: omega/eps, 1: k) from
// nu_t and, under SST, the blending F1 of the cell
__device__ __forceinline__ double gam_of(const Params& P, int eq, double nut, double f) {
  if (P.model == HFDIB_KEPS) return P.nu + nut * (eq == 0 ? P.isig_eps : P.isig_k);
  if (P.model == HFDIB_KOMEGA) return P.nu + nut * (eq == 0 ? P.isig_w_kw : P.isig_k_kw);
  if (P.model == HFDIB_RKEPS) return P.nu + nut * (eq == 0 ? P.isig_eps_rke : P.isig_k_rke);
  const double sg = eq == 0 ? f * P.sigma_w1 + (1.0 - f) * P.sigma_w2 : f * P.sigma_k1 + (1.0 - f) * P.sigma_k2;
  return P.nu + sg * nut;
}

// Turbulence inputs of the previous iterate, taken before this stage changes
// any k or omega/eps value: 2 S:S of the current velocity (Gauss gradient, the
// production term), the SST blending F1 and grad k . grad omega (the
// cross-diffusion term), the diffusivities of the omega/eps and k equations
// (nu_t and F1 do not change before both are assembled), and per block the
// maximum of omega/eps over the cells outside the in-solid group (the value
// imposed on in-solid cells)
__global__ void __launch_bounds__(256)
k_turb_inputs(Params P, const uint8_t* flags, Vel U, const double* kv, const double* wv, const double* dw,
              const double* nut, double* S2, double* F1, double* kwo, double* gam_w, double* gam_k, double* part) {
  double wmx = 0.0;
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i < P.nx && j < P.ny) {
    const long long c = cidx(P, i, j, k);
    const Nbr N = make_nbr(P, i, j, k, c);
    // loads first (clamped neighbours along all three axes; the terms beyond dim
    // are dropped by selects)
    const uint8_t fl = flags[c];
    const double kk = kv[c], ww = wv[c], nt = nut[c];
    double f1 = 0.0;
    double s2;
    {
      double G[3][3];
      gradu_all_bf(P, U.u, fl & F_SOLID, N, c, G);
      s2 = strain2(G);
    }
    if (P.model == HFDIB_KOMEGA_SST) {
      double kn[6], wn[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        kn[q] = kv[N.n[q]];
        wn[q] = wv[N.n[q]];
      }
      const double dwc = dw[c];
      const bool solid = fl & F_SOLID;
      double kw = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double kp = sel(is_bnd(N, 2 * d + 1), sc_bface(P, d, +1, solid, kk, P.k_in), 0.5 * (kk + kn[2 * d + 1]));
        const double km = sel(is_bnd(N, 2 * d), sc_bface(P, d, -1, solid, kk, P.k_in), 0.5 * (kn[2 * d] + kk));
        const double wp = sel(is_bnd(N, 2 * d + 1), sc_bface(P, d, +1, solid, ww, P.w_in), 0.5 * (ww + wn[2 * d + 1]));
        const double wm = sel(is_bnd(N, 2 * d), sc_bface(P, d, -1, solid, ww, P.w_in), 0.5 * (wn[2 * d] + ww));
        const double gk = (kp - km) * P.idelta[d], gw = (wp - wm) * P.idelta[d];
        kw = sel(d < P.dim, kw + gk * gw, kw);
      }
      double cd = 2.0 * P.sigma_w2 / ww * kw;
      cd = cd > P.cd_floor ? cd : P.cd_floor;
      const double a = sqrt(kk) / (P.Cmu * ww * dwc);
      const double bb = 500.0 * P.nu / (dwc * dwc * ww);
      const double m1 = a > bb ? a : bb;
      const double m2 = 4.0 * P.sigma_w2 * kk / (cd * dwc * dwc);
      const double arg1 = m1 < m2 ? m1 : m2;
      const double a2 = arg1 * arg1;
      f1 = tanh(a2 * a2);
      F1[c] = f1;
      kwo[c] = kw;
    }
    S2[c] = s2;
    gam_w[c] = gam_of(P, 0, nt, f1);
    gam_k[c] = gam_of(P, 1, nt, f1);
    wmx = (fl & F_IC) ? 0.0 : ww;
  }
  __shared__ double lmax[4];
  const double m = wave_max(wmx);
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  if ((tid & 63) == 0) lmax[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) part[block_linear()] = fmax(fmax(lmax[0], lmax[1]), fmax(lmax[2], lmax[3]));
}

// imposed omega/eps and production on the boundary cells and the domain-wall
// cells (one thread per list entry), and on the in-solid cells (omega/eps = the
// maximum over the other cells, no production), in one launch
// The logarithmic-branch production takes |n . grad u| as the wall-normal
// difference of the tangential velocity relative to the solid (0 at domain
// walls) over the wall distance y: (|u_t,P - u_s,t| / y)^2 (the wall-face normal
// gradient of the wall-function form of eq. omegaws; under the log law it makes
// P_ib the equilibrium production u_tau^3 / (kappa y)).
// k_ib of boundary cell c (list entry b): quadratic along n_P with the
// wall-function surface value k_S = k_vis(y+) u_tau^2 and free-stream values of
// k_old; 0 on cells off the viscous branch
struct KibIn {
  const uint8_t* flags;
  const double* L;
  const int* st1;
  const double* w1;
  const int* st2;
  const double* w2;
  double* kib;
};
__device__ __forceinline__ void k_ib_value(const Params& P, const KibIn& K, int b, int c, double yp, double ut,
                                           const double* kold) {
  if (!(K.flags[c] & F_ALPHA_U)) {
    K.kib[c] = 0.0;
    return;
  }
  double cc = P.C_wf;
  double t = yp + cc;
  double cf = 1.0 / (t * t) + 2.0 * yp / (cc * cc * cc) - 1.0 / (cc * cc);
  double kvis = 2400.0 * cf / (P.Ceps2_wf * P.Ceps2_wf);
  double kS = kvis * (ut * ut);
  double v1 = 0.0, v2 = 0.0;
  for (int q = 0; q < 8; ++q) v1 += K.w1[8 * b + q] * kold[K.st1[8 * b + q]];
  for (int q = 0; q < 8; ++q) v2 += K.w2[8 * b + q] * kold[K.st2[8 * b + q]];
  K.kib[c] = K.L[3 * b] * kS + K.L[3 * b + 1] * v1 + K.L[3 * b + 2] * v2;
}

struct Vel3 {
  const double* u[3];
  const double* us[3];
};

// (and k_ib of the boundary cells: it needs k_old and the boundary cells' y+
// and u_tau, all in place here)
__global__ void k_turb_imposed(Params P, WallList L0, WallList L1, int nic, const int* ic_cells, const double* wmax,
                               Vel3 V, const double* S2, const double* kold, const double* nut, double* Pk,
                               double* wib, double* w, KibIn K) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= L0.n + L1.n + nic) return;
  if (b >= L0.n + L1.n) {
    int c = ic_cells[b - L0.n - L1.n];
    double m = *wmax;
    Pk[c] = 0.0;
    wib[c] = m;
    w[c] = m;
    return;
  }
  const bool first = b < L0.n;
  const WallList& L = first ? L0 : L1;
  if (!first) b -= L0.n;
  int c = L.cells[b];
  double yp = L.ypl[b], ut = L.utl[b], y = L.y[b];
  if (first) k_ib_value(P, K, b, c, yp, ut, kold);
  double om = omega_ib(P, yp, y, ut);
  double kk = kold[c];
  double val = (P.model == HFDIB_KEPS || P.model == HFDIB_RKEPS) ? P.Cmu * kk * om : om;
  double ur[3], un = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    ur[q] = V.u[q][c] - (first ? V.us[q][c] : 0.0);
    un += ur[q] * L.nv[3 * b + q];
  }
  double t2 = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double tq = ur[q] - un * L.nv[3 * b + q];
    t2 += tq * tq;
  }
  double ng2 = t2 / (y * y);
  double Pm = model_production(P, S2[c], nut[c], kk, w[c]);
  Pk[c] = prod_ib(P, yp, Pm, ng2);
  wib[c] = val;
  w[c] = val;
}


// (each thread adds SUM_PER cells)
__global__ void k_sum1(long long n, const double* a, double* part, long long pstride) {
  const long long c0 = (long long)blockIdx.x * NTHREADS * SUM_PER + threadIdx.x;
  double v[1] = {0.0};
  double e[SUM_PER];
#pragma unroll
  for (int r = 0; r < SUM_PER; ++r) {
    const long long c = c0 + (long long)r * NTHREADS;
    e[r] = a[c < n ? c : n - 1];
  }
#pragma unroll
  for (int r = 0; r < SUM_PER; ++r) v[0] = sel(c0 + (long long)r * NTHREADS < n, v[0] + e[r], v[0]);
  block_sums_store<1>(v, part, pstride, blockIdx.x);
}

struct Scal {
  const double* phi[3];
  const double* S2;  // 2 S:S of the current velocity
  const uint8_t* flags;
  const double* nut;
  const double* F1;
  const double* kw;
  double* Pk;  // closure production on free rows (written by the omega assembly)
  const double* k;  // k_old
  double* w;        // omega/eps (fixed values already in place)
  const double* wib;
  const double* kib;
  Vel U;  // velocity (realizable k-epsilon: its gradient)
};

// neighbour coefficients of a scalar row (faces W, E, S, N, B, T; 0 on domain
// faces and beyond dim) from the stored diffusivities gam, loads from clamped
// indices
__device__ __forceinline__ void scal_anb(const Params& P, const Scal& S, double gP, const double* gam, const Nbr& N,
                                         int i, int j, int k, double (&anb)[6]) {
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int sh = 0; sh < 2; ++sh) {
      const int s = sh ? 1 : -1, q = 2 * d + sh;
      // loads from clamped indices for every face, chosen with selects
      const double mf = -outward_flux(P, S.phi, d, s, i, j, k);
      const double a = 0.5 * (gP + gam[N.n[q]]) * P.AoD[d] + (mf > 0.0 ? mf : 0.0);
      anb[q] = sel(d < P.dim && !is_bnd(N, q), a, 0.0);
    }
}

// assembly of the omega (eps, eq = 0) or k (eq = 1) rows; rhs -> rhs_out,
// relaxed diagonal -> aPr_out; residual sums of the solved rows
// (RKE: the realizable k-epsilon eps sources, instantiated separately so the
// other closures keep their register budget)
// gam: the equation's diffusivity per cell, stored by the stage's first pass
// (mixed policy: copied to gam_out32 for the FP32 sweeps)
template <bool RKE>
__global__ void k_scalar_assemble(Params P, Scal S, int eq, double* rhs_out, double* aPr_out, float* r32, float* a32,
                                  const double* gam, float* gam_out32, const double* xmean, double* part,
                                  long long pstride, double* xs_out) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  double red[3] = {0, 0, 0};
  if (i < P.nx && j < P.ny) {
    long long c = cidx(P, i, j, k);
    uint8_t fl = S.flags[c];
    bool solid = fl & F_SOLID;
    const double gP = gam[c];
    if (gam_out32) gam_out32[c] = (float)gP;
    Nbr N = make_nbr(P, i, j, k, c);
    double anb[6];
    scal_anb(P, S, gP, gam, N, i, j, k, anb);
    double aP = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) aP += anb[q];
    double vin = eq == 0 ? P.w_in : P.k_in;
    double b0 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int sh = 0; sh < 2; ++sh) {
        const int s = sh ? 1 : -1;
        if (d >= P.dim || face_kind(P, d, s) != HFDIB_BC_INLET) continue;
        if (!is_bnd(N, 2 * d + sh) || solid) continue;
        double F = outward_flux(P, S.phi, d, s, i, j, k);
        double mf = -F;
        double a = gP * P.Ab[d] + (mf > 0.0 ? mf : 0.0);
        aP += a;
        b0 += a * vin;
      }
    double V = P.V;
    double urf = P.urf_t;
    double kold = S.k[c];
    double x, rhs, aPr;
    bool skip;
    if (eq == 0) {
      double wo = S.w[c];
      double Pc;
      if (fl & F_ALPHA_W) {
        Pc = S.Pk[c];
      } else {
        Pc = model_production(P, S.S2[c], S.nut[c], kold, wo);
        S.Pk[c] = Pc;
      }
      if (P.model == HFDIB_KEPS) {
        aP = aP + P.C2 * wo / kold * V;
        b0 = b0 + P.C1 * Pc * wo / kold * V;
      } else if (RKE) {
        // C1 |S| eps explicit, C2 eps^2 / (k + sqrt(nu eps)) linearised in eps
        RkeInv I = rke_invariants(P, S.U, solid, N, c);
        double Sm = sqrt(2.0 * I.SS);
        double eta = Sm * kold / wo;
        double C1 = fmax(0.43, eta / (eta + 5.0));
        aP = aP + P.C2_rke * wo / (kold + sqrt(P.nu * wo)) * V;
        b0 = b0 + C1 * Sm * wo * V;
      } else if (P.model == HFDIB_KOMEGA) {
        // C_alpha1 (omega/k) P_k - C_beta1 omega^2, the sink linearised in omega
        aP = aP + P.beta_kw * wo * V;
        b0 = b0 + P.alpha_kw * (wo / kold) * Pc * V;
      } else {
        double f = S.F1[c];
        double beta = f * P.beta_1 + (1.0 - f) * P.beta_2;
        double gamma = f * P.gamma_1 + (1.0 - f) * P.gamma_2;
        aP = aP + beta * wo * V;
        b0 = b0 + gamma * (wo / kold) * Pc * V;
        double CD = (1.0 - f) * 2.0 * P.sigma_w2 * S.kw[c] / wo;
        b0 = b0 + (CD > 0.0 ? CD * V : 0.0);
        aP = aP + (CD < 0.0 ? -CD / wo * V : 0.0);
      }
      aPr = aP / urf;
      skip = fl & F_ALPHA_W;
      rhs = skip ? aPr * S.wib[c] : b0 + (1.0 - urf) / urf * aP * wo;
      x = wo;
    } else {
      double wv = S.w[c];
      double wmin = P.bound_frac * P.w_in;
      wv = wv > wmin ? wv : wmin;
      S.w[c] = wv;
      if (P.model == HFDIB_KEPS || P.model == HFDIB_RKEPS) aP = aP + wv / kold * V;
      else aP = aP + P.Cmu * wv * V;
      b0 = b0 + S.Pk[c] * V;
      aPr = aP / urf;
      double r = (1.0 - urf) / urf * aP * kold;
      skip = fl & F_ALPHA_U;
      if (skip) {
        double nbt = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          long long n = N.n[q];
          double kt = (S.flags[n] & F_ALPHA_U) ? S.kib[n] : S.k[n];
          nbt += anb[q] * kt;
        }
        rhs = (aP * S.kib[c] - nbt) + r;
      } else {
        rhs = b0 + r;
      }
      x = kold;
    }
    const long long sidx = rb_split(P, i, j, k);
    rhs_out[sidx] = rhs;
    aPr_out[sidx] = aPr;
    // FP64 policy: the colour-split copy the sweeps work on (the black half, and
    // the fixed rows, which no sweep writes: the first half sweep, red, reads the
    // black neighbours and writes the other red cells itself)
    if (xs_out && (((i + j + k) & 1) || (eq == 0 && (fl & F_ALPHA_W)))) xs_out[sidx] = x;
    // rows the sweeps update: all k rows; omega/eps rows outside alpha_omega
    bool swept = eq == 1 || !(fl & F_ALPHA_W);
    if (!skip || (a32 && swept)) {
      const double* xv = eq == 0 ? S.w : S.k;
      double nb = 0.0, one = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        nb += anb[q] * xv[N.n[q]];
        one += anb[q];
      }
      double Ax = aPr * x - nb;
      if (!skip) {
        double Axb = (aPr - one) * (*xmean);
        red[0] = fabs(rhs - Ax);
        red[1] = fabs(Ax - Axb);
        red[2] = fabs(rhs - Axb);
      }
      // mixed policy: FP64 defect of the row for the FP32 correction
      if (a32) r32[sidx] = (float)(rhs - Ax);
    }
    if (a32) {
      a32[sidx] = (float)aPr;
      if (!swept) r32[sidx] = 0.0f;
    }
  }
  block_sums_store<3>(red, part, pstride, block_linear());
}

// red-black Gauss-Seidel half sweep of a scalar equation; rows flagged `fixmask`
// are not updated
// (FP64) the diffusivity of each cell comes from the array the stage's first
// pass stored, rhs and a'_P from the colour-split arrays, so a one-colour
// launch streams only its own half of them
// The sweeps work on the colour-split copy xs of x that the assembly wrote (a
// one-colour pass reads only the other colour's half and writes only its
// own); fin: the last half sweep (black), which writes x in the natural order
// instead, for both cells of its pair (the red partner is a face neighbour);
// the split copy is dead after it.
__global__ void k_scalar_sweep(Params P, Scal S, const double* gamc, const double* rhs, const double* aPr, double* xs,
                               double* x, int color, uint8_t fixmask, int fin) {
  int i, j, k;
  tile_ijk_rb(P, color, i, j, k);
  if (j >= P.ny) return;
  if (i >= P.nx) {
    // only the partner of this pair lies in the grid (odd nx)
    const int io = i ^ 1;
    if (fin && io < P.nx) x[cidx(P, io, j, k)] = xs[rb_split(P, io, j, k)];
    return;
  }
  long long c = cidx(P, i, j, k);
  const Nbr N = make_nbr(P, i, j, k, c);
  const long long sidx = rb_split(P, i, j, k);
  // every load of the row is issued before any is used (also for fixed rows,
  // which then store nothing)
  const uint8_t fl = S.flags[c];
  const double gP = gamc[c], b = rhs[sidx], ap = aPr[sidx];
  double gn[6], xn[6], fo[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    gn[q] = gamc[N.n[q]];
    xn[q] = xs[nb_split(P, N, i, j, k, q)];
    fo[q] = outward_flux(P, S.phi, q >> 1, (q & 1) ? 1 : -1, i, j, k);
  }
  double nb = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int d = q >> 1;
    const double mf = -fo[q];
    double a = 0.5 * (gP + gn[q]) * P.AoD[d] + (mf > 0.0 ? mf : 0.0);
    a = sel(d < P.dim && !is_bnd(N, q), a, 0.0);
    nb += a * xn[q];
  }
  const bool upd = !(fl & fixmask);
  const double v = (b + nb) / ap;
  if (upd && !fin) xs[sidx] = v;
  if (fin) {
    // the partner (i ^ 1) is the west (i odd) or east (i even) neighbour
    const int io = i ^ 1;
    if (upd) x[c] = v;
    if (io < P.nx) x[cidx(P, io, j, k)] = sel((i & 1) != 0, xn[0], xn[1]);
  }
}

// Mixed policy: red-black sweep of the FP32 correction d of a scalar equation
// (A d = r from d = 0; rows flagged `fixmask` keep d = 0), coefficients from
// the FP32 mirrors; the last sweep of each colour writes x <- x_old + d (FP64).
struct Scal32 {
  const float* phi[3];
};

// (the diffusivity of each cell from the FP32 array the assembly stored; defect
// and diagonal colour-split)
__global__ void k_scalar_sweep32(Params P, Scal32 S, const uint8_t* flags, const float* gamc, const float* r,
                                 const float* a32, float* dv, double* x, int color, uint8_t fixmask, int init,
                                 int fin) {
  int i, j, k;
  tile_ijk_rb(P, color, i, j, k);
  if (j >= P.ny) return;
  if (init) {
    // the partner cell of the other colour in this pair starts from d = 0
    int io = i ^ 1;
    if (io < P.nx) dv[rb_split(P, io, j, k)] = 0.0f;
  }
  if (i >= P.nx) return;
  long long c = cidx(P, i, j, k);
  const long long sidx = rb_split(P, i, j, k);  // (d colour-split, like r and a)
  // loads first (clamped neighbours, selects), stores last
  const bool fixed = flags[c] & fixmask;
  const float rs = r[sidx], as = a32[sidx];
  float nb = 0.0f;
  if (!init) {
    const float gP = gamc[c];
    const Nbr N = make_nbr(P, i, j, k, c);
    float gn[6], fo[6], zn[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int d = q >> 1, s = (q & 1) ? 1 : -1;
      const long long n = N.n[q];
      gn[q] = gamc[n];
      fo[q] = S.phi[d][fidx(P, d, i, j, k) + (s > 0 ? stride(P, d) : 0)];
      zn[q] = dv[nb_split(P, N, i, j, k, q)];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int d = q >> 1;
      const float mf = (q & 1) ? -fo[q] : fo[q];
      const float a = 0.5f * (gP + gn[q]) * (float)P.AoD[d] + (mf > 0.0f ? mf : 0.0f);
      nb = sel(d < P.dim && !is_bnd(N, q), nb + a * zn[q], nb);
    }
  }
  if (fixed) {
    if (init) dv[sidx] = 0.0f;
    return;
  }
  const float e = (rs + nb) / as;
  const double xo = fin ? x[c] : 0.0;
  dv[sidx] = e;
  if (fin) x[c] = xo + (double)e;
}

// k <- k + alpha_k (k_ib - k), bounding, turbulent viscosity of the model
// (in-solid cells 0); eps/omega is already bounded
__global__ void k_turb_final(Params P, const uint8_t* flags, const double* S2, Vel U, const double* kib, double* k,
                             const double* w, const double* dw, double* nut, float* nut32) {
  int i, j, kz;
  tile_ijk(P, i, j, kz);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, kz);
  // loads first, stores last
  const uint8_t fl = flags[c];
  double kk = k[c];
  const double ww = w[c], dwc = dw[c], S2c = S2[c];
  if (fl & F_ALPHA_U) kk = kk + 1.0 * (kib[c] - kk);
  double kmin = P.bound_frac * P.k_in;
  kk = kk > kmin ? kk : kmin;
  double nt;
  if (P.model == HFDIB_KEPS) {
    nt = P.Cmu * kk * kk / ww;
  } else if (P.model == HFDIB_KOMEGA) {
    nt = kk / ww;
  } else if (P.model == HFDIB_RKEPS) {
    RkeInv I = rke_invariants(P, U, fl & F_SOLID, make_nbr(P, i, j, kz, c), c);
    nt = rke_cmu(P, I, kk, ww) * kk * kk / ww;
  } else {
    double d = dwc;
    double bs = P.Cmu;
    double a = 2.0 * sqrt(kk) / (bs * ww * d);
    double bb = 500.0 * P.nu / (d * d * ww);
    double arg2 = a > bb ? a : bb;
    double F2 = tanh(arg2 * arg2);
    double den1 = P.a1 * ww, den2 = sqrt(S2c) * F2;
    nt = P.a1 * kk / (den1 > den2 ? den1 : den2);
  }
  if (fl & F_IC) nt = 0.0;
  k[c] = kk;
  nut[c] = nt;
  if (nut32) nut32[c] = (float)nt;
}


// boundary cells on the logarithmic branch: the log-law wall viscosity, and the
// velocity-based friction velocity from the log law by Newton's method (0 off
// that branch)
__global__ void k_wall_bc(Params P, int nbc, const int* bc_cells, const double* bc_n, const double* bc_yeff,
                          const double* ypl, const double* utl, const double* u0, const double* u1, const double* u2,
                          const double* us0, const double* us1, const double* us2, double* out, double* nut,
                          float* nut32) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nbc) return;
  double yp = ypl[b];
  if (!(yp > P.ylam)) {
    out[b] = 0.0;
    return;
  }
  int c = bc_cells[b];
  {
    double v = P.kappa * yp / log(P.E * yp) - 1.0;
    double nt = P.nu * (v > 0.0 ? v : 0.0);
    nut[c] = nt;
    if (nut32) nut32[c] = (float)nt;
  }
  double ur[3] = {u0[c] - us0[c], u1[c] - us1[c], u2[c] - us2[c]};
  double n[3] = {bc_n[3 * b], bc_n[3 * b + 1], bc_n[3 * b + 2]};
  double un = ur[0] * n[0] + ur[1] * n[1] + ur[2] * n[2];
  double t0 = ur[0] - un * n[0], t1 = ur[1] - un * n[1], t2 = ur[2] - un * n[2];
  double mag = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
  double a = P.E * bc_yeff[b] / P.nu;
  double u = utl[b];
  double e0 = 2.718281828459045 / a;
  u = u > e0 ? u : e0;
  for (int it = 0; it < 20; ++it) {
    double lg = log(a * u);
    double f = u / P.kappa * lg - mag;
    double fp = (lg + 1.0) / P.kappa;
    double du = f / fp;
    u = u - du;
    if (!(fabs(du) > 1e-14 * fabs(u))) break;
  }
  out[b] = u;
}

}  // namespace hfdib

// ====================================================================== host
namespace hfdib {

int turbulence_stage(hfdib_ctx* c) {
  const Params& P = c->P;
  dim3 g = grid3(P), b = block3(P);
  long long nblk3 = (long long)g.x * g.y * g.z;
  double* S = c->scal + SCAL_PCG;
  double* wmax = S + SC_WMAX;
  const Vel U{{c->u[0], c->u[1], c->u[2]}};
  // per-cell diffusivities of the omega/eps and the k equations, stored by the
  // first pass for both assemblies and the FP64 sweeps (the momentum
  // right-hand sides are dead during this stage)
  double* gam_w = c->rhs[0];
  double* gam_k = c->rhs[1];
  // SST blending and cross diffusion of the previous iterate, the
  // diffusivities, maximum of omega/eps over cells outside the in-solid group
  hipLaunchKernelGGL(k_turb_inputs, g, b, 0, c->stream, P, (const uint8_t*)c->flags, U, (const double*)c->k,
                     (const double*)c->w, (const double*)c->dw, (const double*)c->nut, c->S2, c->F1, c->t2, gam_w,
                     gam_k, c->partials);
  launch_finalize(c, (int)nblk3, 1, SC_WMAX, 4);
  // imposed omega/eps and production on boundary, wall and in-solid cells
  {
    WallList L0{c->n_bc, c->bc_cells, c->bc_yeff, c->bc_n, c->bc_yplus, c->bc_utau};
    WallList L1{c->n_wall, c->wall_cells, c->wall_y, c->wall_n, c->wall_yplus, c->wall_utau};
    int ntot = c->n_bc + c->n_wall + c->n_ic;
    if (ntot > 0)
      hipLaunchKernelGGL(k_turb_imposed, dim3(nblocks1(ntot)), dim3(NTHREADS), 0, c->stream, P, L0, L1, c->n_ic,
                         c->ic_cells, wmax, Vel3{{c->u[0], c->u[1], c->u[2]}, {c->us[0], c->us[1], c->us[2]}},
                         c->S2, c->k, c->nut, c->Pk, c->wib, c->w,
                         KibIn{c->flags, c->bc_L, c->bc_s1, c->bc_w1, c->bc_s2, c->bc_w2, c->kib});
  }
  const int nbs = nblocks_sum(P.N);
  hipLaunchKernelGGL(k_sum1, dim3(nbs), dim3(NTHREADS), 0, c->stream, P.N, c->w, c->partials, c->pstride);
  launch_finalize(c, nbs, 1, SC_MEANS + 5, 0, (double)P.N);
  Scal Sc;
  for (int q = 0; q < 3; ++q) {
    Sc.phi[q] = c->phi[q];
  }
  Sc.flags = c->flags;
  Sc.S2 = c->S2;
  Sc.nut = c->nut;
  Sc.F1 = c->F1;
  Sc.kw = c->t2;
  Sc.Pk = c->Pk;
  Sc.k = c->k;
  Sc.w = c->w;
  Sc.wib = c->wib;
  Sc.kib = c->kib;
  Sc.U = U;
  bool mixed = P.precision == HFDIB_MIXED;
  float* r32 = mixed ? c->r32[0] : nullptr;
  float* a32 = mixed ? c->a32 : nullptr;
  Scal32 S32{{c->phi32[0], c->phi32[1], c->phi32[2]}};
  // n_s red-black sweeps of equation eq (FP64, or the FP32 correction)
  // (one timing span over the 2 n_s consecutive launches)
  auto sweeps = [&](const double* gam_c, double* x, uint8_t fixmask) {
    for (int s = 0; s < P.n_sweeps; ++s)
      for (int color = 0; color < 2; ++color) {
        const bool first = s == 0 && color == 0, last = s == P.n_sweeps - 1 && color == 1;
        LaunchEv ev = timer_launch(c, T_SCALSWEEP, first, last, 2 * P.n_sweeps);
        if (mixed)
          launch_ev(k_scalar_sweep32, grid3_rb(P), b, c->stream, ev, P, S32, c->flags, c->gam32, r32, a32, c->d32[0], x,
                    color, fixmask, first ? 1 : 0, s == P.n_sweeps - 1 ? 1 : 0);
        else
          launch_ev(k_scalar_sweep, grid3_rb(P), b, c->stream, ev, P, Sc, gam_c, c->t0, c->t1, c->xsp, x, color,
                    fixmask, last ? 1 : 0);
      }
  };
  // omega / eps equation, alpha_omega rows fixed
  auto assemble = P.model == HFDIB_RKEPS ? k_scalar_assemble<true> : k_scalar_assemble<false>;
  LaunchEv ev = timer_launch(c, T_SCALASM, true, true);
  launch_ev(assemble, g, b, c->stream, ev, P, Sc, 0, c->t0, c->t1, r32, a32, (const double*)gam_w,
            mixed ? c->gam32 : nullptr, S + SC_MEANS + 5, c->partials, c->pstride, c->xsp);
  launch_finalize(c, (int)nblk3, 3, SC_RESSUM + 9, 0);
  sweeps(gam_w, c->w, (uint8_t)F_ALPHA_W);
  // the k equation with S_ib (k_ib came with the imposed values; bounds
  // omega/eps on the way)
  ev = timer_launch(c, T_SCALASM, true, true);
  launch_ev(assemble, g, b, c->stream, ev, P, Sc, 1, c->t0, c->t1, r32, a32, (const double*)gam_k,
            mixed ? c->gam32 : nullptr, S + SC_MEANS + 4, c->partials, c->pstride, c->xsp);
  launch_finalize(c, (int)nblk3, 3, SC_RESSUM + 12, 0);
  sweeps(gam_k, c->k, (uint8_t)0);
  hipLaunchKernelGGL(k_turb_final, g, b, 0, c->stream, P, c->flags, c->S2, U, c->kib, c->k, c->w,
                     c->dw, c->nut, mixed ? c->nut32 : nullptr);
  if (c->n_bc > 0) {
    hipLaunchKernelGGL(k_wall_bc, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, P, c->n_bc, c->bc_cells,
                       c->bc_n, c->bc_yeff, c->bc_yplus, c->bc_utau, c->u[0], c->u[1], c->u[2], c->us[0], c->us[1],
                       c->us[2], c->bc_utauU, c->nut, mixed ? c->nut32 : nullptr);
  }
  HFDIB_CHECK_LAUNCH(c, "turbulence");
  return HFDIB_OK;
}

}  // namespace hfdib
