// Turbulence stage of the extended SIMPLE loop: alpha_omega, imposed omega
// (eps) and production, the omega (eps) equation with fixed rows, k_ib, the k
// equation with S_ib, the k correction and the turbulent viscosity
// (Sec. "Treatment of production and dissipation of k", eqs. for the imposed
// values, k_vis, u_tau, omega_ib and P_ib; k-epsilon and Menter SST closures).
#include "device_common.h"

namespace hfdib {

struct Turb {
  const double* u[3];
  const double* phi[3];
  const uint8_t* flags;
  double* grad[9];
  double* S2;
  double* Pk;
  double* F1;
  double* kw;  // grad k . grad omega (SST)
  const double* k;
  const double* w;
  const double* nut;
  const double* dw;
};

__device__ __forceinline__ double sc_bface(const Params& P, int d, int s, bool solid, double vP, double vin) {
  if (face_kind(P, d, s) == HFDIB_BC_INLET && !solid) return vin;
  return vP;
}
__device__ __forceinline__ double u_bface_t(const Params& P, int cc, int d, int s, bool solid, double uP) {
  if (solid) return uP;
  int kind = face_kind(P, d, s);
  if (kind == HFDIB_BC_INLET) return P.u_in[cc];
  if (kind == HFDIB_BC_NOSLIP) return 0.0;
  if (kind == HFDIB_BC_SLIP) return cc == d ? 0.0 : uP;
  return uP;
}

// (psi_+ - psi_-)/delta_d with linear face interpolation
__device__ __forceinline__ double ggrad(const Params& P, const double* a, long long c, int d, int i, int j, int k,
                                       double fb_p, double fb_m) {
  long long st = stride(P, d);
  double fp = on_bnd(P, d, +1, i, j, k) ? fb_p : 0.5 * (a[c] + a[c + st]);
  double fm = on_bnd(P, d, -1, i, j, k) ? fb_m : 0.5 * (a[c - st] + a[c]);
  return (fp - fm) / P.delta[d];
}

__device__ __forceinline__ void atomic_max_pos(double* addr, double v) {
  // positive doubles order like their bit patterns
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

// gradient tensor of u, 2 S:S, production, SST blending F1 and the maximum of
// omega (eps) over boundary and free-stream cells
__global__ void k_turb_grad(Params P, Turb T, double* wmax) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  int k = blockIdx.z;
  double mx = 0.0;
  bool act = i < P.nx && j < P.ny;
  if (act) {
    long long c = cidx(P, i, j, k);
    uint8_t fl = T.flags[c];
    bool solid = fl & F_SOLID;
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int jj = 0; jj < P.dim; ++jj) {
      const double* u = T.u[jj];
      double uP = u[c];
      for (int ii = 0; ii < P.dim; ++ii)
        G[ii][jj] = ggrad(P, u, c, ii, i, j, k, u_bface_t(P, jj, ii, +1, solid, uP),
                          u_bface_t(P, jj, ii, -1, solid, uP));
    }
    for (int ii = 0; ii < P.dim; ++ii)
      for (int jj = 0; jj < P.dim; ++jj) T.grad[ii * 3 + jj][c] = G[ii][jj];
    double S2 = 0.0;
    for (int ii = 0; ii < 3; ++ii)
      for (int jj = 0; jj < 3; ++jj) {
        double sij = 0.5 * (G[ii][jj] + G[jj][ii]);
        S2 = S2 + 2.0 * sij * sij;
      }
    T.S2[c] = S2;
    if (P.model != HFDIB_LAMINAR) {
      double kk = T.k[c], ww = T.w[c];
      double Gp = T.nut[c] * S2;
      if (P.model == HFDIB_KOMEGA_SST) {
        double gk[3] = {0, 0, 0}, gw[3] = {0, 0, 0};
        for (int d = 0; d < P.dim; ++d) {
          gk[d] = ggrad(P, T.k, c, d, i, j, k, sc_bface(P, d, +1, solid, kk, P.k_in),
                        sc_bface(P, d, -1, solid, kk, P.k_in));
          gw[d] = ggrad(P, T.w, c, d, i, j, k, sc_bface(P, d, +1, solid, ww, P.w_in),
                        sc_bface(P, d, -1, solid, ww, P.w_in));
        }
        double kw = gk[0] * gw[0] + gk[1] * gw[1] + gk[2] * gw[2];
        double dw = T.dw[c];
        double bs = P.Cmu;
        double cd = 2.0 * P.sigma_w2 / ww * kw;
        cd = cd > P.cd_floor ? cd : P.cd_floor;
        double a = sqrt(kk) / (bs * ww * dw);
        double bb = 500.0 * P.nu / (dw * dw * ww);
        double m1 = a > bb ? a : bb;
        double m2 = 4.0 * P.sigma_w2 * kk / (cd * dw * dw);
        double arg1 = m1 < m2 ? m1 : m2;
        double a2 = arg1 * arg1;
        T.F1[c] = tanh(a2 * a2);
        T.kw[c] = kw;
        double lim = P.c_lim * bs * kk * ww;
        T.Pk[c] = Gp < lim ? Gp : lim;
      } else {
        T.Pk[c] = Gp;
      }
      if (!(fl & F_IC)) mx = ww;
    }
  }
  if (P.model != HFDIB_LAMINAR) {
    double m = wave_max(mx);
    int tid = threadIdx.x + blockDim.x * threadIdx.y;
    if ((tid & 63) == 0 && m > 0.0) atomic_max_pos(wmax, m);
  }
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
struct Grad9 {
  const double* g[9];
};

__global__ void k_turb_ib(Params P, int n, const int* cells, const double* yv, const double* nv, const double* ypl,
                          const double* utl, const double* kold, Grad9 grad, double* Pk, double* wib, double* w) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= n) return;
  int c = cells[b];
  double yp = ypl[b], ut = utl[b], y = yv[b];
  double om = omega_ib(P, yp, y, ut);
  double val = P.model == HFDIB_KEPS ? P.Cmu * kold[c] * om : om;
  double ng[3] = {0.0, 0.0, 0.0};
  for (int jj = 0; jj < 3; ++jj)
    for (int ii = 0; ii < 3; ++ii) {
      double g = (ii < P.dim && jj < P.dim) ? grad.g[ii * 3 + jj][c] : 0.0;
      ng[jj] += nv[3 * b + ii] * g;
    }
  double ng2 = ng[0] * ng[0] + ng[1] * ng[1] + ng[2] * ng[2];
  Pk[c] = prod_ib(P, yp, Pk[c], ng2);
  wib[c] = val;
  w[c] = val;
}

__global__ void k_turb_ic(int n, const int* cells, const double* wmax, double* Pk, double* wib, double* w) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= n) return;
  int c = cells[b];
  double m = *wmax;
  Pk[c] = 0.0;
  wib[c] = m;
  w[c] = m;
}

__global__ void k_sum1(long long n, const double* a, double* part, long long pstride) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  double v[1] = {c < n ? a[c] : 0.0};
  block_sums_store<1>(v, part, pstride, blockIdx.x);
}

// diffusion coefficient of the transported scalar (0: omega/eps, 1: k)
__device__ __forceinline__ double gam(const Params& P, int eq, long long c, const double* nut, const double* F1) {
  if (P.model == HFDIB_KEPS) return P.nu + nut[c] / (eq == 0 ? P.sigma_eps : P.sigma_k);
  double f = F1[c];
  double sg = eq == 0 ? f * P.sigma_w1 + (1.0 - f) * P.sigma_w2 : f * P.sigma_k1 + (1.0 - f) * P.sigma_k2;
  return P.nu + sg * nut[c];
}

struct Scal {
  const double* phi[3];
  const uint8_t* flags;
  const double* nut;
  const double* F1;
  const double* kw;
  const double* Pk;
  const double* k;  // k_old
  double* w;        // omega/eps (fixed values already in place)
  const double* wib;
  const double* kib;
};

// assembly of the omega (eps, eq = 0) or k (eq = 1) rows; rhs -> rhs_out,
// relaxed diagonal -> aPr_out; residual sums of the solved rows
__global__ void k_scalar_assemble(Params P, Scal S, int eq, double* rhs_out, double* aPr_out, const double* xmean,
                                  double* part, long long pstride) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  int k = blockIdx.z;
  double red[3] = {0, 0, 0};
  if (i < P.nx && j < P.ny) {
    long long c = cidx(P, i, j, k);
    uint8_t fl = S.flags[c];
    bool solid = fl & F_SOLID;
    double gP = gam(P, eq, c, S.nut, S.F1);
    double anb[6];
    long long nbi[6];
    double aP = 0.0;
    for (int d = 0; d < P.dim; ++d)
      for (int s = -1; s <= 1; s += 2) {
        int q = 2 * d + (s > 0);
        if (on_bnd(P, d, s, i, j, k)) {
          anb[q] = 0.0;
          nbi[q] = c;
          continue;
        }
        long long n = c + s * stride(P, d);
        double F = outward_flux(P, S.phi, d, s, i, j, k);
        double mf = -F;
        anb[q] = 0.5 * (gP + gam(P, eq, n, S.nut, S.F1)) * P.area[d] / P.delta[d] + (mf > 0.0 ? mf : 0.0);
        nbi[q] = n;
        aP += anb[q];
      }
    double vin = eq == 0 ? P.w_in : P.k_in;
    double b0 = 0.0;
    for (int d = 0; d < P.dim; ++d)
      for (int s = -1; s <= 1; s += 2) {
        if (!on_bnd(P, d, s, i, j, k) || solid || face_kind(P, d, s) != HFDIB_BC_INLET) continue;
        double F = outward_flux(P, S.phi, d, s, i, j, k);
        double mf = -F;
        double a = gP * P.area[d] / (0.5 * P.delta[d]) + (mf > 0.0 ? mf : 0.0);
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
      if (P.model == HFDIB_KEPS) {
        aP = aP + P.C2 * wo / kold * V;
        b0 = b0 + P.C1 * S.Pk[c] * wo / kold * V;
      } else {
        double f = S.F1[c];
        double beta = f * P.beta_1 + (1.0 - f) * P.beta_2;
        double gamma = f * P.gamma_1 + (1.0 - f) * P.gamma_2;
        aP = aP + beta * wo * V;
        b0 = b0 + gamma * (wo / kold) * S.Pk[c] * V;
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
      if (P.model == HFDIB_KEPS) aP = aP + wv / kold * V;
      else aP = aP + P.Cmu * wv * V;
      b0 = b0 + S.Pk[c] * V;
      aPr = aP / urf;
      double r = (1.0 - urf) / urf * aP * kold;
      skip = fl & F_ALPHA_U;
      if (skip) {
        double nbt = 0.0;
        for (int q = 0; q < 2 * P.dim; ++q) {
          if (nbi[q] == c) continue;
          long long n = nbi[q];
          double kt = (S.flags[n] & F_ALPHA_U) ? S.kib[n] : S.k[n];
          nbt += anb[q] * kt;
        }
        rhs = (aP * S.kib[c] - nbt) + r;
      } else {
        rhs = b0 + r;
      }
      x = kold;
    }
    rhs_out[c] = rhs;
    aPr_out[c] = aPr;
    if (!skip) {
      const double* xv = eq == 0 ? S.w : S.k;
      double nb = 0.0, one = 0.0;
      for (int q = 0; q < 2 * P.dim; ++q) {
        if (nbi[q] == c) continue;
        nb += anb[q] * xv[nbi[q]];
        one += anb[q];
      }
      double Ax = aPr * x - nb;
      double Axb = (aPr - one) * (*xmean);
      red[0] = fabs(rhs - Ax);
      red[1] = fabs(Ax - Axb);
      red[2] = fabs(rhs - Axb);
    }
  }
  block_sums_store<3>(red, part, pstride, block_linear());
}

// red-black Gauss-Seidel half sweep of a scalar equation; rows flagged `fixmask`
// are not updated
__global__ void k_scalar_sweep(Params P, Scal S, int eq, const double* rhs, const double* aPr, double* x, int color,
                               uint8_t fixmask) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  int k = blockIdx.z;
  if (i >= P.nx || j >= P.ny) return;
  if (((i + j + k) & 1) != color) return;
  long long c = cidx(P, i, j, k);
  if (S.flags[c] & fixmask) return;
  double gP = gam(P, eq, c, S.nut, S.F1);
  double nb = 0.0;
  for (int d = 0; d < P.dim; ++d)
    for (int s = -1; s <= 1; s += 2) {
      if (on_bnd(P, d, s, i, j, k)) continue;
      long long n = c + s * stride(P, d);
      double F = outward_flux(P, S.phi, d, s, i, j, k);
      double mf = -F;
      double a = 0.5 * (gP + gam(P, eq, n, S.nut, S.F1)) * P.area[d] / P.delta[d] + (mf > 0.0 ? mf : 0.0);
      nb += a * x[n];
    }
  x[c] = (rhs[c] + nb) / aPr[c];
}

// k_ib on boundary cells: quadratic along n_P with the wall-function surface
// value k_S = k_vis(y+) u_tau^2 and free-stream values of k_old; 0 elsewhere
__global__ void k_kib(Params P, int nbc, const int* bc_cells, const uint8_t* flags, const double* bc_L,
                      const int* st1, const double* w1, const int* st2, const double* w2, const double* ypl,
                      const double* utl, const double* kold, double* kib) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nbc) return;
  int c = bc_cells[b];
  if (!(flags[c] & F_ALPHA_U)) {
    kib[c] = 0.0;
    return;
  }
  double yp = ypl[b], ut = utl[b];
  double cc = P.C_wf;
  double t = yp + cc;
  double cf = 1.0 / (t * t) + 2.0 * yp / (cc * cc * cc) - 1.0 / (cc * cc);
  double kvis = 2400.0 * cf / (P.Ceps2_wf * P.Ceps2_wf);
  double kS = kvis * (ut * ut);
  double v1 = 0.0, v2 = 0.0;
  for (int q = 0; q < 8; ++q) v1 += w1[8 * b + q] * kold[st1[8 * b + q]];
  for (int q = 0; q < 8; ++q) v2 += w2[8 * b + q] * kold[st2[8 * b + q]];
  kib[c] = bc_L[3 * b] * kS + bc_L[3 * b + 1] * v1 + bc_L[3 * b + 2] * v2;
}

// k <- k + alpha_k (k_ib - k), bounding, turbulent viscosity of the model
// (in-solid cells 0); eps/omega is already bounded
__global__ void k_turb_final(Params P, const uint8_t* flags, const double* kib, double* k, const double* w,
                             const double* S2, const double* dw, double* nut) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c >= P.N) return;
  uint8_t fl = flags[c];
  double kk = k[c];
  if (fl & F_ALPHA_U) kk = kk + 1.0 * (kib[c] - kk);
  double kmin = P.bound_frac * P.k_in;
  kk = kk > kmin ? kk : kmin;
  k[c] = kk;
  double ww = w[c];
  double nt;
  if (P.model == HFDIB_KEPS) {
    nt = P.Cmu * kk * kk / ww;
  } else {
    double d = dw[c];
    double bs = P.Cmu;
    double a = 2.0 * sqrt(kk) / (bs * ww * d);
    double bb = 500.0 * P.nu / (d * d * ww);
    double arg2 = a > bb ? a : bb;
    double F2 = tanh(arg2 * arg2);
    double den1 = P.a1 * ww, den2 = sqrt(S2[c]) * F2;
    nt = P.a1 * kk / (den1 > den2 ? den1 : den2);
  }
  if (fl & F_IC) nt = 0.0;
  nut[c] = nt;
}

// boundary cells on the logarithmic branch: log-law wall viscosity
__global__ void k_nut_bc(Params P, int nbc, const int* bc_cells, const double* ypl, double* nut) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nbc) return;
  double yp = ypl[b];
  if (!(yp > P.ylam)) return;
  double v = P.kappa * yp / log(P.E * yp) - 1.0;
  nut[bc_cells[b]] = P.nu * (v > 0.0 ? v : 0.0);
}

// velocity-based friction velocity from the log law by Newton's method
// (boundary cells on the logarithmic branch; 0 elsewhere)
__global__ void k_loglaw(Params P, int nbc, const int* bc_cells, const double* bc_n, const double* bc_yeff,
                         const double* ypl, const double* utl, const double* u0, const double* u1, const double* u2,
                         const double* us0, const double* us1, const double* us2, double* out) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nbc) return;
  double yp = ypl[b];
  if (!(yp > P.ylam)) {
    out[b] = 0.0;
    return;
  }
  int c = bc_cells[b];
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

__global__ void k_set1(double* a, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *a = v;
}

static Turb make_turb(hfdib_ctx* c) {
  Turb T;
  for (int q = 0; q < 3; ++q) {
    T.u[q] = c->u[q];
    T.phi[q] = c->phi[q];
  }
  T.flags = c->flags;
  for (int q = 0; q < 9; ++q) T.grad[q] = c->grad[q];
  T.S2 = c->S2;
  T.Pk = c->Pk;
  T.F1 = c->F1;
  T.kw = c->t2;
  T.k = c->k;
  T.w = c->w;
  T.nut = c->nut;
  T.dw = c->dw;
  return T;
}

int gradient_only(hfdib_ctx* c) {
  Params P = c->P;
  P.model = HFDIB_LAMINAR;
  Turb T = make_turb(c);
  hipLaunchKernelGGL(k_turb_grad, grid3(P), block3(), 0, c->stream, P, T, c->scal + SCAL_PCG + SC_WMAX);
  HFDIB_CHECK_LAUNCH(c, "gradient");
  return HFDIB_OK;
}

int turbulence_stage(hfdib_ctx* c) {
  const Params& P = c->P;
  dim3 g = grid3(P), b = block3();
  long long nblk3 = (long long)g.x * g.y * g.z;
  int nb1 = nblocks1(P.N);
  double* S = c->scal + SCAL_PCG;
  double* wmax = S + SC_WMAX;
  hipLaunchKernelGGL(k_set1, dim3(1), dim3(64), 0, c->stream, wmax, 0.0);
  Turb T = make_turb(c);
  hipLaunchKernelGGL(k_turb_grad, g, b, 0, c->stream, P, T, wmax);
  Grad9 G9;
  for (int q = 0; q < 9; ++q) G9.g[q] = c->grad[q];
  // imposed omega/eps and production on boundary, wall and in-solid cells
  if (c->n_bc > 0)
    hipLaunchKernelGGL(k_turb_ib, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, P, c->n_bc, c->bc_cells,
                       c->bc_yeff, c->bc_n, c->bc_yplus, c->bc_utau, c->k, G9, c->Pk, c->wib, c->w);
  if (c->n_wall > 0)
    hipLaunchKernelGGL(k_turb_ib, dim3(nblocks1(c->n_wall)), dim3(NTHREADS), 0, c->stream, P, c->n_wall,
                       c->wall_cells, c->wall_y, c->wall_n, c->wall_yplus, c->wall_utau, c->k, G9, c->Pk,
                       c->wib, c->w);
  if (c->n_ic > 0)
    hipLaunchKernelGGL(k_turb_ic, dim3(nblocks1(c->n_ic)), dim3(NTHREADS), 0, c->stream, c->n_ic, c->ic_cells,
                       wmax, c->Pk, c->wib, c->w);
  hipLaunchKernelGGL(k_sum1, dim3(nb1), dim3(NTHREADS), 0, c->stream, P.N, c->w, c->partials, c->pstride);
  launch_finalize(c, nb1, 1, SC_MEANS + 5, 0, (double)P.N);
  Scal Sc;
  for (int q = 0; q < 3; ++q) Sc.phi[q] = c->phi[q];
  Sc.flags = c->flags;
  Sc.nut = c->nut;
  Sc.F1 = c->F1;
  Sc.kw = c->t2;
  Sc.Pk = c->Pk;
  Sc.k = c->k;
  Sc.w = c->w;
  Sc.wib = c->wib;
  Sc.kib = c->kib;
  // omega / eps equation, alpha_omega rows fixed
  hipLaunchKernelGGL(k_scalar_assemble, g, b, 0, c->stream, P, Sc, 0, c->t0, c->t1, S + SC_MEANS + 5, c->partials,
                     c->pstride);
  launch_finalize(c, (int)nblk3, 3, SC_RESSUM + 9, 0);
  for (int s = 0; s < P.n_sweeps; ++s)
    for (int color = 0; color < 2; ++color)
      hipLaunchKernelGGL(k_scalar_sweep, g, b, 0, c->stream, P, Sc, 0, c->t0, c->t1, c->w, color,
                         (uint8_t)F_ALPHA_W);
  // k_ib, then the k equation with S_ib (bounds omega/eps on the way)
  if (c->n_bc > 0)
    hipLaunchKernelGGL(k_kib, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, P, c->n_bc, c->bc_cells,
                       c->flags, c->bc_L, c->bc_s1, c->bc_w1, c->bc_s2, c->bc_w2, c->bc_yplus, c->bc_utau, c->k,
                       c->kib);
  hipLaunchKernelGGL(k_scalar_assemble, g, b, 0, c->stream, P, Sc, 1, c->t0, c->t1, S + SC_MEANS + 4, c->partials,
                     c->pstride);
  launch_finalize(c, (int)nblk3, 3, SC_RESSUM + 12, 0);
  for (int s = 0; s < P.n_sweeps; ++s)
    for (int color = 0; color < 2; ++color)
      hipLaunchKernelGGL(k_scalar_sweep, g, b, 0, c->stream, P, Sc, 1, c->t0, c->t1, c->k, color, (uint8_t)0);
  hipLaunchKernelGGL(k_turb_final, dim3(nb1), dim3(NTHREADS), 0, c->stream, P, c->flags, c->kib, c->k, c->w, c->S2,
                     c->dw, c->nut);
  if (c->n_bc > 0) {
    hipLaunchKernelGGL(k_nut_bc, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, P, c->n_bc, c->bc_cells,
                       c->bc_yplus, c->nut);
    hipLaunchKernelGGL(k_loglaw, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, P, c->n_bc, c->bc_cells,
                       c->bc_n, c->bc_yeff, c->bc_yplus, c->bc_utau, c->u[0], c->u[1], c->u[2], c->us[0], c->us[1],
                       c->us[2], c->bc_utauU);
  }
  HFDIB_CHECK_LAUNCH(c, "turbulence");
  return HFDIB_OK;
}

}  // namespace hfdib
