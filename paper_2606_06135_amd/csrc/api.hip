// C ABI of the HFDIB SIMPLE library: workspace layout, context lifecycle,
// iteration driver, field access and kernel timing.
#include "device_common.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

namespace hfdib {

int set_hip_error(hfdib_ctx* c, hipError_t e, const char* where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return HFDIB_EDEVICE;
}

struct Timers {
  bool on = false;
  int every = 1;      // record every `every`-th SIMPLE iteration
  long long n_it = 0; // SIMPLE iterations seen while on
  bool skip = false;  // the current iteration is not recorded
  struct Span {
    hipEvent_t e0, e1;
    int launches;
  };
  std::vector<Span> pend[T_NCLASS];
  hipEvent_t open[T_NCLASS] = {};
  double ms[T_NCLASS] = {};
  long long cnt[T_NCLASS] = {};
  // events whose spans were read back, reused by later spans (creating an event
  // per span would cost a runtime call inside the timed iterations)
  std::vector<hipEvent_t> pool;
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  ~Timers() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : open)
      if (e) (void)hipEventDestroy(e);
  }
};

static void timers_flush(hfdib_ctx* c) {
  Timers* T = c->timers;
  bool any = false;
  for (int k = 0; k < T_NCLASS; ++k) any = any || !T->pend[k].empty();
  if (!any) return;
  (void)hipStreamSynchronize(c->stream);
  for (int k = 0; k < T_NCLASS; ++k) {
    for (auto& sp : T->pend[k]) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, sp.e0, sp.e1) == hipSuccess) {
        T->ms[k] += ms;
        T->cnt[k] += sp.launches;
      }
      T->pool.push_back(sp.e0);
      T->pool.push_back(sp.e1);
    }
    T->pend[k].clear();
  }
}

void timer_iteration(hfdib_ctx* c, bool begin) {
  Timers* T = c->timers;
  if (!T || !T->on) return;
  T->skip = begin && (T->n_it++ % T->every) != 0;
}

void timer_begin(hfdib_ctx* c, int cls) {
  Timers* T = c->timers;
  if (!T || !T->on || T->skip) return;
  if (!T->open[cls]) T->open[cls] = T->take();
  if (T->open[cls]) (void)hipEventRecord(T->open[cls], c->stream);
}

void timer_end(hfdib_ctx* c, int cls, int launches) {
  Timers* T = c->timers;
  if (!T || !T->on || !T->open[cls]) return;
  hipEvent_t e = T->take();
  if (!e) return;
  (void)hipEventRecord(e, c->stream);
  T->pend[cls].push_back({T->open[cls], e, launches});
  T->open[cls] = nullptr;
  if (T->pend[cls].size() > 4096) timers_flush(c);
}

LaunchEv timer_launch(hfdib_ctx* c, int cls, bool first, bool last, int launches) {
  LaunchEv ev{nullptr, nullptr};
  Timers* T = c->timers;
  if (!T || !T->on || T->skip) return ev;
  if (first) {
    if (T->pend[cls].size() > 4096) timers_flush(c);
    if (!T->open[cls]) T->open[cls] = T->take();
    ev.start = T->open[cls];
  }
  if (last && T->open[cls]) {
    ev.stop = T->take();
    if (ev.stop) T->pend[cls].push_back({T->open[cls], ev.stop, launches});
    T->open[cls] = nullptr;
  }
  return ev;
}

// ---------------------------------------------------------------- layout
struct Bump {
  char* base;
  size_t off;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

static void level_dims(hfdib_ctx* c) {
  const Params& P = c->P;
  c->nlev = 1;
  Level& L0 = c->lev[0];
  L0.nx = P.nx;
  L0.ny = P.ny;
  L0.nz = P.nz;
  L0.N = P.N;
  while (c->nlev < MAX_LEVELS) {
    Level& F = c->lev[c->nlev - 1];
    bool ok = F.nx % 2 == 0 && F.ny % 2 == 0 && F.nx / 2 >= 2 && F.ny / 2 >= 2 && F.N > 64;
    if (P.dim == 3) ok = ok && F.nz % 2 == 0 && F.nz / 2 >= 2;
    if (!ok) break;
    Level& L = c->lev[c->nlev];
    L.nx = F.nx / 2;
    L.ny = F.ny / 2;
    L.nz = P.dim == 3 ? F.nz / 2 : 1;
    L.N = (long long)L.nx * L.ny * L.nz;
    c->nlev++;
  }
}

static size_t layout(hfdib_ctx* c, char* base) {
  const Params& P = c->P;
  long long N = P.N;
  Bump B{base, 0};
  for (int q = 0; q < 3; ++q) c->u[q] = B.take<double>(N);
  c->p = B.take<double>(N);
  c->pnew = B.take<double>(N);
  c->k = B.take<double>(N);
  c->w = B.take<double>(N);
  c->nut = B.take<double>(N);
  c->lam = B.take<double>(N);
  c->dw = B.take<double>(N);
  // rhs and a'_P of the momentum rows, colour-split (see Params::nrb)
  const long long nsplit_u = 2 * P.nrb > N ? 2 * P.nrb : N;
  for (int q = 0; q < 3; ++q) c->rhs[q] = B.take<double>(nsplit_u);
  c->aPr = B.take<double>(nsplit_u);
  for (int q = 0; q < 3; ++q) c->hbya[q] = B.take<double>(N);
  c->rAU = B.take<double>(N);
  c->F1 = B.take<double>(N);
  for (int q = 0; q < 3; ++q) c->uib[q] = B.take<double>(N);
  c->kib = B.take<double>(N);
  c->wib = B.take<double>(N);
  c->Pk = B.take<double>(N);
  for (int q = 0; q < 3; ++q) c->us[q] = B.take<double>(N);
  // t0, t1: colour-split right-hand side and diagonal of the k and omega/eps rows
  const long long nsplit = 2 * P.nrb > N ? 2 * P.nrb : N;
  c->t0 = B.take<double>(nsplit);
  c->t1 = B.take<double>(nsplit);
  c->t2 = B.take<double>(N);
  c->wallD = B.take<double>(N);
  c->S2 = B.take<double>(N);
  for (int q = 0; q < 3; ++q) c->ex[q] = B.take<double>(N);
  c->rhs_p = B.take<double>(N);
  c->px = B.take<double>(N);
  c->pr = B.take<double>(N);
  c->pz = B.take<double>(N);
  c->pd = B.take<double>(N);
  c->pd2 = B.take<double>(N);
  c->pq = B.take<double>(N);
  {
    // the V-cycle's colour-split fine-level vectors (FP64 policy; FP32 below)
    const long long ns = 2 * P.nrb > N ? 2 * P.nrb : N;
    c->invD = B.take<double>(ns);
    const bool fp64 = P.precision != HFDIB_MIXED;
    c->pzs = fp64 ? B.take<double>(ns) : nullptr;
    c->prs = fp64 ? B.take<double>(ns) : nullptr;
    // the sweeps' colour-split copies of the state (FP64 policy)
    for (int q = 0; q < 3; ++q) c->usp[q] = fp64 ? B.take<double>(ns) : nullptr;
    c->xsp = fp64 ? B.take<double>(ns) : nullptr;
  }
  c->flags = B.take<uint8_t>(N);
  c->phi[0] = B.take<double>((long long)(P.nx + 1) * P.ny * P.nz);
  c->phi[1] = B.take<double>((long long)P.nx * (P.ny + 1) * P.nz);
  c->phi[2] = B.take<double>((long long)P.nx * P.ny * (P.nz + 1));
  int cap = c->cap;
  c->bc_cells = B.take<int>(cap);
  c->ic_cells = B.take<int>(cap);
  c->wall_cells = B.take<int>(cap);
  c->bc_n = B.take<double>(3LL * cap);
  c->bc_yperp = B.take<double>(cap);
  c->bc_yeff = B.take<double>(cap);
  c->bc_L = B.take<double>(3LL * cap);
  c->bc_w1 = B.take<double>(8LL * cap);
  c->bc_w2 = B.take<double>(8LL * cap);
  c->bc_s1 = B.take<int>(8LL * cap);
  c->bc_s2 = B.take<int>(8LL * cap);
  c->bc_mode = B.take<int>(cap);
  c->bc_yplus = B.take<double>(cap);
  c->bc_utau = B.take<double>(cap);
  c->bc_utauU = B.take<double>(cap);
  c->wall_y = B.take<double>(cap);
  c->wall_n = B.take<double>(3LL * cap);
  c->wall_yplus = B.take<double>(cap);
  c->wall_utau = B.take<double>(cap);
  c->ipts = B.take<double>(3LL * cap);
  // partial rows hold one entry per block of the largest tile-shape candidate
  // (every width, and the momentum assembly's 32 x 2 x 4 tiles)
  long long nblk3 = 0;
  for (int lx = TILE_LOG2_MIN; lx <= TILE_LOG2_MAX + 1; ++lx) {
    Params Q = P;
    Q.tx_log2 = lx <= TILE_LOG2_MAX ? lx : 5;
    if (lx > TILE_LOG2_MAX) {
      if (P.dim != 3 || P.nz % 4 != 0) continue;
      Q.tz_log2 = 2;
    }
    dim3 g = grid3(Q);
    long long nb = (long long)g.x * g.y * g.z;
    nblk3 = nb > nblk3 ? nb : nblk3;
  }
  long long nb1 = nblocks1(N);
  long long ps = nblk3 > nb1 ? nblk3 : nb1;
  c->pstride = (ps + 63) / 64 * 64;
  c->partials = B.take<double>(16 * c->pstride);
  c->partials2 = B.take<double>(16 * FIN2_STRIDE);
  c->scal = B.take<double>(512);
  c->iscal = B.take<int>(64);
  bool mixed = P.precision == HFDIB_MIXED;
  for (int l = 1; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    long long fx = (long long)(L.nx + 1) * L.ny * L.nz, fy = (long long)L.nx * (L.ny + 1) * L.nz,
              fz = (long long)L.nx * L.ny * (L.nz + 1);
    L.r = L.z = L.diag = L.cx = L.cy = L.cz = nullptr;
    L.r32 = L.z32 = L.diag32 = L.cx32 = L.cy32 = L.cz32 = nullptr;
    if (mixed) {
      L.r32 = B.take<float>(L.N);
      L.z32 = B.take<float>(L.N);
      L.diag32 = B.take<float>(L.N);
      L.cx32 = B.take<float>(fx);
      L.cy32 = B.take<float>(fy);
      L.cz32 = B.take<float>(fz);
    } else {
      L.r = B.take<double>(L.N);
      L.z = B.take<double>(L.N);
      L.diag = B.take<double>(L.N);
      L.cx = B.take<double>(fx);
      L.cy = B.take<double>(fy);
      L.cz = B.take<double>(fz);
    }
  }
  // FP32 arrays of the mixed policy
  for (int q = 0; q < 3; ++q) c->r32[q] = c->d32[q] = c->phi32[q] = nullptr;
  c->a32 = c->nut32 = c->rAU32 = c->pr32 = c->pz32 = c->invD32 = c->gam32 = nullptr;
  c->pzs32 = c->prs32 = nullptr;
  if (mixed) {
    // FP32 defects and relaxed diagonals, colour-split like their FP64 counterparts
    const long long n32 = 2 * P.nrb > N ? 2 * P.nrb : N;
    for (int q = 0; q < 3; ++q) c->r32[q] = B.take<float>(n32);
    for (int q = 0; q < 3; ++q) c->d32[q] = B.take<float>(n32);  // (colour-split)
    c->a32 = B.take<float>(n32);
    c->gam32 = B.take<float>(N);
    c->phi32[0] = B.take<float>((long long)(P.nx + 1) * P.ny * P.nz);
    c->phi32[1] = B.take<float>((long long)P.nx * (P.ny + 1) * P.nz);
    c->phi32[2] = B.take<float>((long long)P.nx * P.ny * (P.nz + 1));
    c->nut32 = B.take<float>(N);
    c->rAU32 = B.take<float>(N);
    c->pr32 = B.take<float>(N);
    c->pz32 = B.take<float>(N);
    c->invD32 = B.take<float>(n32);
    c->pzs32 = B.take<float>(n32);
    c->prs32 = B.take<float>(n32);
  }
  return B.off + 256;
}

// Inlet turbulence values: given, or (turb_intensity > 0) derived from the
// intensity and length scale by the paper's inlet condition (eq. bcspkoein):
// k = 3/2 |u_in|^2 I^2, eps = C_nu k^(3/2) / l_t, omega = eps / (C_nu k); without a
// length scale omega is given and eps = C_nu k omega.
static void inlet_values(const hfdib_grid_desc& d, const hfdib_config& c, double* k, double* eps, double* om) {
  *k = d.k_in;
  *eps = d.eps_in;
  *om = d.omega_in;
  if (!(d.turb_intensity > 0.0)) return;
  const double U2 = d.u_in[0] * d.u_in[0] + d.u_in[1] * d.u_in[1] + d.u_in[2] * d.u_in[2];
  *k = 1.5 * U2 * d.turb_intensity * d.turb_intensity;
  if (d.turb_length > 0.0) {
    *eps = c.Cmu * std::pow(*k, 1.5) / d.turb_length;
    *om = *eps / (c.Cmu * *k);
  } else {
    *eps = c.Cmu * *k * *om;
  }
}

static int check_inputs(const hfdib_grid_desc* d, const hfdib_config* c, std::string* why) {
  if (!d || !c) {
    *why = "null descriptor";
    return HFDIB_EINVAL;
  }
  if (c->abi_version != HFDIB_ABI_VERSION) {
    *why = "config abi_version mismatch";
    return HFDIB_EINVAL;
  }
  if (d->dim != 2 && d->dim != 3) {
    *why = "dim must be 2 or 3";
    return HFDIB_EINVAL;
  }
  if (d->nx < 4 || d->ny < 4 || d->nz < 1 || (d->dim == 2 && d->nz != 1) || (d->dim == 3 && d->nz < 4)) {
    *why = "grid too small (>= 4 cells per active axis; nz = 1 in 2D)";
    return HFDIB_EINVAL;
  }
  if ((long long)d->nx * d->ny * d->nz >= (1LL << 31)) {
    *why = "grid too large (at most 2^31 - 1 cells)";
    return HFDIB_EINVAL;
  }
  if (!(d->dx > 0.0 && d->dy > 0.0 && d->dz > 0.0)) {
    *why = "cell sizes must be positive";
    return HFDIB_EINVAL;
  }
  for (int f = 0; f < 6; ++f) {
    int b = d->bc[f];
    if (b < HFDIB_BC_INLET || b > HFDIB_BC_EMPTY) {
      *why = "invalid boundary kind";
      return HFDIB_EINVAL;
    }
    bool zf = f >= 4;
    if (d->dim == 2 && zf && b != HFDIB_BC_EMPTY) {
      *why = "2D grids need EMPTY z faces";
      return HFDIB_EINVAL;
    }
    if ((d->dim == 3 || !zf) && b == HFDIB_BC_EMPTY) {
      *why = "EMPTY is only valid for the z faces of 2D grids";
      return HFDIB_EINVAL;
    }
  }
  if (!(c->nu > 0.0)) {
    *why = "nu must be positive";
    return HFDIB_EINVAL;
  }
  if (!(c->urf_u > 0.0 && c->urf_u <= 1.0 && c->urf_p > 0.0 && c->urf_p <= 1.0 && c->urf_t > 0.0 && c->urf_t <= 1.0)) {
    *why = "under-relaxation factors must lie in (0, 1]";
    return HFDIB_EINVAL;
  }
  if (c->n_sweeps < 1 || c->p_maxit < 1 || !(c->p_rtol > 0.0)) {
    *why = "n_sweeps >= 1, p_maxit >= 1 and p_rtol > 0 are required";
    return HFDIB_EINVAL;
  }
  if (c->p_sweeps < 1 || c->p_sweeps > 4 || c->p_sweeps_coarse < 1 || c->p_sweeps_coarse > 4) {
    *why = "p_sweeps and p_sweeps_coarse must lie in 1..4";
    return HFDIB_EINVAL;
  }
  if (c->model < HFDIB_LAMINAR || c->model > HFDIB_RKEPS) {
    *why = "invalid model";
    return HFDIB_EINVAL;
  }
  if (c->continuity != 0 && c->continuity != 1) {
    *why = "continuity must be 0 or 1";
    return HFDIB_EINVAL;
  }
  if (c->yplus_dist != HFDIB_YPLUS_EFF && c->yplus_dist != HFDIB_YPLUS_PERP) {
    *why = "yplus_dist must be HFDIB_YPLUS_EFF or HFDIB_YPLUS_PERP";
    return HFDIB_EINVAL;
  }
  if (c->conv_scheme < HFDIB_CONV_UPWIND || c->conv_scheme > HFDIB_CONV_VANLEER) {
    *why = "conv_scheme must be HFDIB_CONV_UPWIND, HFDIB_CONV_LINEAR_UPWIND or HFDIB_CONV_VANLEER";
    return HFDIB_EINVAL;
  }
  if (c->precision != HFDIB_FP64 && c->precision != HFDIB_MIXED) {
    *why = "precision must be HFDIB_FP64 or HFDIB_MIXED";
    return HFDIB_EINVAL;
  }
  if (c->model != HFDIB_LAMINAR) {
    double kin, ein, oin;
    inlet_values(*d, *c, &kin, &ein, &oin);
    double win = (c->model == HFDIB_KEPS || c->model == HFDIB_RKEPS) ? ein : oin;
    if (!(kin > 0.0 && win > 0.0 && std::isfinite(kin) && std::isfinite(win))) {
      *why = "turbulent models need positive inlet k and eps/omega";
      return HFDIB_EINVAL;
    }
  }
  return HFDIB_OK;
}

static void fill_params(hfdib_ctx* c) {
  const hfdib_grid_desc& d = c->desc;
  const hfdib_config& g = c->cfg;
  Params& P = c->P;
  memset(&P, 0, sizeof(P));
  P.dim = d.dim;
  P.nx = d.nx;
  P.ny = d.ny;
  P.nz = d.nz;
  P.N = (long long)d.nx * d.ny * d.nz;
  P.nxh = (d.nx + 1) / 2;
  P.nrb = (long long)P.nxh * d.ny * d.nz;
  P.x0 = d.x0;
  P.y0 = d.y0;
  P.z0 = d.z0;
  P.dx = d.dx;
  P.dy = d.dy;
  P.dz = d.dz;
  P.area[0] = d.dy * d.dz;
  P.area[1] = d.dx * d.dz;
  P.area[2] = d.dx * d.dy;
  P.delta[0] = d.dx;
  P.delta[1] = d.dy;
  P.delta[2] = d.dz;
  P.V = d.dx * d.dy * d.dz;
  P.h = d.dim == 2 ? std::sqrt(d.dx * d.dy) : std::pow(P.V, 1.0 / 3.0);
  for (int f = 0; f < 6; ++f) P.bc[f] = d.bc[f];
  for (int q = 0; q < 3; ++q) P.u_in[q] = d.u_in[q];
  double kin, ein, oin;
  inlet_values(d, g, &kin, &ein, &oin);
  P.k_in = kin;
  P.w_in = (g.model == HFDIB_KEPS || g.model == HFDIB_RKEPS)
               ? ein
               : ((g.model == HFDIB_KOMEGA_SST || g.model == HFDIB_KOMEGA) ? oin : 0.0);
  P.model = g.model;
  P.n_sweeps = g.n_sweeps;
  P.nu = g.nu;
  P.urf_u = g.urf_u;
  P.urf_p = g.urf_p;
  P.urf_t = g.urf_t;
  P.Cmu = g.Cmu;
  P.kappa = g.kappa;
  P.E = g.E;
  P.beta1_wf = g.beta1_wf;
  P.Ceps2_wf = g.Ceps2_wf;
  P.C_wf = g.C_wf;
  P.ylam = g.ylam;
  P.C1 = g.C1;
  P.C2 = g.C2;
  P.sigma_k = g.sigma_k;
  P.sigma_eps = g.sigma_eps;
  P.sigma_k1 = g.sigma_k1;
  P.sigma_w1 = g.sigma_w1;
  P.beta_1 = g.beta_1;
  P.gamma_1 = g.gamma_1;
  P.sigma_k2 = g.sigma_k2;
  P.sigma_w2 = g.sigma_w2;
  P.beta_2 = g.beta_2;
  P.gamma_2 = g.gamma_2;
  P.a1 = g.a1;
  P.c_lim = g.c_lim;
  P.alpha_kw = g.alpha_kw;
  P.beta_kw = g.beta_kw;
  P.isig_k_kw = 1.0 / g.sigma_k_kw;
  P.isig_w_kw = 1.0 / g.sigma_w_kw;
  P.A0_rke = g.A0_rke;
  P.C2_rke = g.C2_rke;
  P.isig_k_rke = 1.0 / g.sigma_k_rke;
  P.isig_eps_rke = 1.0 / g.sigma_eps_rke;
  P.yplus_perp = g.yplus_dist == HFDIB_YPLUS_PERP;
  P.conv = g.conv_scheme;
  P.bound_frac = g.bound_frac;
  P.yperp_min_frac = g.yperp_min_frac;
  P.cd_floor = g.cd_floor;
  P.Cmu25 = std::pow(g.Cmu, 0.25);
  P.sqrtCmu = std::sqrt(g.Cmu);
  for (int d = 0; d < 3; ++d) {
    P.AoD[d] = P.area[d] / P.delta[d];
    P.Ab[d] = P.area[d] / (0.5 * P.delta[d]);
    P.idelta[d] = 1.0 / P.delta[d];
  }
  for (int f = 0; f < 6; ++f) {
    int kind = d.bc[f], dn = f / 2;
    for (int cc = 0; cc < 3; ++cc) {
      double A = 1.0, Bv = 0.0;  // outlet, empty: zero gradient
      if (kind == HFDIB_BC_INLET) {
        A = 0.0;
        Bv = d.u_in[cc];
      } else if (kind == HFDIB_BC_NOSLIP || (kind == HFDIB_BC_SLIP && cc == dn)) {
        A = 0.0;
      }
      P.ubA[f][cc] = A;
      P.ubB[f][cc] = Bv;
    }
    P.sc_inlet[f] = kind == HFDIB_BC_INLET ? 1 : 0;
    P.p_outlet[f] = kind == HFDIB_BC_OUTLET ? 1 : 0;
  }
  P.isig_k = 1.0 / g.sigma_k;
  P.isig_eps = 1.0 / g.sigma_eps;
  P.recorrect = g.recorrect;
  P.continuity = g.continuity;
  P.precision = g.precision;
  P.p_nu = g.p_sweeps;
  P.p_nu_c = g.p_sweeps_coarse;
  P.tx_log2 = 6;
}

static int capacity_for(long long N, int requested) {
  if (requested > 0) return requested;
  long long cap = N <= (1LL << 20) ? N : N / 8 + 4096;
  return (int)cap;
}

// small field conversion kernels
__global__ void k_flag_field(long long n, const uint8_t* flags, int which, double* out) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c >= n) return;
  uint8_t f = flags[c];
  if (which == 0) out[c] = (f & F_IC) ? 2.0 : ((f & F_BC) ? 1.0 : 0.0);
  else out[c] = (f & F_ALPHA_U) ? 1.0 : 0.0;
}
__global__ void k_scatter_list(int n, const int* cells, const double* v, double* dst) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b < n) dst[cells[b]] = v[b];
}

__global__ void k_fill0(long long n, double* a) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c < n) a[c] = 0.0;
}

}  // namespace hfdib

using namespace hfdib;

extern "C" {

int hfdib_abi_version(void) { return HFDIB_ABI_VERSION; }

void hfdib_default_config(hfdib_config* c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
  c->abi_version = HFDIB_ABI_VERSION;
  c->model = HFDIB_KEPS;
  c->precision = HFDIB_FP64;
  c->n_sweeps = 2;
  c->nu = 1e-5;
  c->urf_u = 0.7;
  c->urf_p = 0.3;
  c->urf_t = 0.85;
  c->p_rtol = 1e-2;
  c->p_maxit = 200;
  c->recorrect = 1;
  c->bc_capacity = 0;
  c->Cmu = 0.09;
  c->kappa = 0.41;
  c->E = 9.8;
  c->beta1_wf = 0.075;
  c->Ceps2_wf = 1.9;
  c->C_wf = 11.0;
  c->ylam = 11.0;
  c->C1 = 1.44;
  c->C2 = 1.92;
  c->sigma_k = 1.0;
  c->sigma_eps = 1.3;
  c->sigma_k1 = 0.85;
  c->sigma_w1 = 0.5;
  c->beta_1 = 0.075;
  c->gamma_1 = 0.5532;
  c->sigma_k2 = 1.0;
  c->sigma_w2 = 0.856;
  c->beta_2 = 0.0828;
  c->gamma_2 = 0.4404;
  c->a1 = 0.31;
  c->c_lim = 10.0;
  c->sigma_k_kw = 1.0 / 0.6;
  c->sigma_w_kw = 2.0;
  c->alpha_kw = 0.52;
  c->beta_kw = 0.0708;
  c->A0_rke = 4.0;
  c->C2_rke = 1.9;
  c->sigma_k_rke = 1.0;
  c->sigma_eps_rke = 1.2;
  c->bound_frac = 1e-10;
  c->yperp_min_frac = 1e-6;
  c->cd_floor = 1e-10;
  c->keep_state = 0;
  c->div_factor = 1e6;
  c->p_sweeps = 2;
  c->p_sweeps_coarse = 2;
}

int hfdib_workspace_bytes(const hfdib_grid_desc* d, const hfdib_config* c, size_t* bytes) {
  std::string why;
  int st = check_inputs(d, c, &why);
  if (st != HFDIB_OK) return st;
  if (!bytes) return HFDIB_EINVAL;
  hfdib_ctx tmp;
  tmp.desc = *d;
  tmp.cfg = *c;
  fill_params(&tmp);
  tmp.cap = capacity_for(tmp.P.N, c->bc_capacity);
  level_dims(&tmp);
  *bytes = layout(&tmp, nullptr);
  return HFDIB_OK;
}

int hfdib_init_grid(const hfdib_grid_desc* d, const hfdib_config* c, void* workspace, size_t bytes, void* hip_stream,
                    hfdib_ctx** out) {
  if (!out) return HFDIB_EINVAL;
  *out = nullptr;
  std::string why;
  int st = check_inputs(d, c, &why);
  if (st != HFDIB_OK) return st;
  if (!workspace || ((uintptr_t)workspace & 255)) return HFDIB_EINVAL;
  hfdib_ctx* ctx = new (std::nothrow) hfdib_ctx();
  if (!ctx) return HFDIB_ENOMEM;
  ctx->desc = *d;
  ctx->cfg = *c;
  fill_params(ctx);
  ctx->cap = capacity_for(ctx->P.N, c->bc_capacity);
  level_dims(ctx);
  size_t need = layout(ctx, nullptr);
  if (bytes < need) {
    delete ctx;
    return HFDIB_ENOMEM;
  }
  ctx->ws = (char*)workspace;
  ctx->ws_bytes = bytes;
  layout(ctx, ctx->ws);
  ctx->stream = (hipStream_t)hip_stream;
  ctx->ready = 0;
  {
    int dev = 0, n = 0;
    ctx->ncu = (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
                   ? n
                   : 256;
  }
  ctx->timers = new (std::nothrow) Timers();
  memset(ctx->stats, 0, sizeof(ctx->stats));
  *out = ctx;
  return HFDIB_OK;
}

int hfdib_set_indicator(hfdib_ctx* c, const double* lambda_dev, const double* solid_vel_dev) {
  if (!c || !lambda_dev) return HFDIB_EINVAL;
  const Params& P = c->P;
  size_t nb = (size_t)P.N * sizeof(double);
  HFDIB_CHECK(c, hipMemcpyAsync(c->lam, lambda_dev, nb, hipMemcpyDeviceToDevice, c->stream), "copy lambda");
  int n1 = nblocks1(P.N);
  for (int q = 0; q < 3; ++q) {
    if (solid_vel_dev)
      HFDIB_CHECK(c, hipMemcpyAsync(c->us[q], solid_vel_dev + (size_t)q * P.N, nb, hipMemcpyDeviceToDevice, c->stream),
                  "copy solid velocity");
    else
      hipLaunchKernelGGL(k_fill0, dim3(n1), dim3(NTHREADS), 0, c->stream, P.N, c->us[q]);
  }
  hipLaunchKernelGGL(k_fill0, dim3(n1), dim3(NTHREADS), 0, c->stream, P.N, c->dw);
  HFDIB_CHECK_LAUNCH(c, "set_indicator");
  // (keep_state needs a state: a context whose indicator was set before)
  const bool keep = c->cfg.keep_state && c->ready;
  c->ready = 0;
  int st = geometry_precompute(c);
  if (st != HFDIB_OK) return st;
  if (keep) {
    // the state stays; the FP32 mirrors are refreshed
    st = refresh_mirrors(c);
  } else {
    st = init_state(c);
  }
  if (st != HFDIB_OK) return st;
  c->ready = 1;
  return HFDIB_OK;
}

int hfdib_simple_iterate(hfdib_ctx* c, int max_iters, double tol, int check_every, int* iters_done,
                         double* res_out) {
  if (!c) return HFDIB_EINVAL;
  if (!c->ready) {
    c->err = "hfdib_set_indicator has not been called";
    return HFDIB_ESTATE;
  }
  if (max_iters < 0) return HFDIB_EINVAL;
  memset(c->stats, 0, sizeof(c->stats));
  // residuals of the checks: the six normalised ones, then the sum of the
  // absolute momentum residuals (the blow-up guard)
  double res[7] = {0, 0, 0, 0, 0, 0, 0};
  double abs0 = -1.0;
  int done = 0;
  int status = HFDIB_OK;
  for (int it = 0; it < max_iters; ++it) {
    bool check = (tol > 0.0 && check_every > 0 && (it + 1) % check_every == 0) || it == max_iters - 1;
    timer_iteration(c, true);
    int st = simple_step(c, it, check ? res : nullptr);
    timer_iteration(c, false);
    ++done;
    if (st != HFDIB_OK) {
      status = st;
      break;
    }
    if (check) {
      bool finite = true;
      double mx = 0.0;
      for (int q = 0; q < 6; ++q) {
        if (!std::isfinite(res[q])) finite = false;
        mx = res[q] > mx ? res[q] : mx;
      }
      if (!finite || !std::isfinite(res[6])) {
        c->err = "non-finite residual";
        status = HFDIB_EDIVERGED;
        break;
      }
      if (abs0 < 0.0) abs0 = res[6];
      if (c->cfg.div_factor > 0.0 && res[6] > c->cfg.div_factor * abs0) {
        c->err = "momentum residual grew by more than div_factor since the first check";
        status = HFDIB_EDIVERGED;
        break;
      }
      if (tol > 0.0 && mx <= tol) break;
    }
  }
  c->stats[1] = done;
  if (iters_done) *iters_done = done;
  if (res_out) memcpy(res_out, res, 6 * sizeof(double));
  return status;
}

static double* field_ptr(hfdib_ctx* c, int id, size_t* n) {
  const Params& P = c->P;
  *n = (size_t)P.N;
  switch (id) {
    case HFDIB_FIELD_UX: return c->u[0];
    case HFDIB_FIELD_UY: return c->u[1];
    case HFDIB_FIELD_UZ: return c->u[2];
    case HFDIB_FIELD_P: return c->p;
    case HFDIB_FIELD_K: return c->k;
    case HFDIB_FIELD_EPS_OR_OMEGA: return c->w;
    case HFDIB_FIELD_NUT: return c->nut;
    case HFDIB_FIELD_PHI_X: *n = (size_t)(P.nx + 1) * P.ny * P.nz; return c->phi[0];
    case HFDIB_FIELD_PHI_Y: *n = (size_t)P.nx * (P.ny + 1) * P.nz; return c->phi[1];
    case HFDIB_FIELD_PHI_Z: *n = (size_t)P.nx * P.ny * (P.nz + 1); return c->phi[2];
    case HFDIB_FIELD_LAMBDA: return c->lam;
    case HFDIB_FIELD_WALLDIST: return c->dw;
    case HFDIB_FIELD_UIB_X: return c->uib[0];
    case HFDIB_FIELD_UIB_Y: return c->uib[1];
    case HFDIB_FIELD_UIB_Z: return c->uib[2];
    case HFDIB_FIELD_KIB: return c->kib;
    case HFDIB_FIELD_WIB: return c->wib;
    case HFDIB_FIELD_PK: return c->Pk;
    default: return nullptr;
  }
}

int hfdib_get_field(hfdib_ctx* c, int id, double* dst) {
  if (!c || !dst) return HFDIB_EINVAL;
  if (id == HFDIB_FIELD_CLASS || id == HFDIB_FIELD_ALPHA_U) {
    hipLaunchKernelGGL(k_flag_field, dim3(nblocks1(c->P.N)), dim3(NTHREADS), 0, c->stream, c->P.N, c->flags,
                       id == HFDIB_FIELD_CLASS ? 0 : 1, dst);
    HFDIB_CHECK_LAUNCH(c, "get_field");
    return HFDIB_OK;
  }
  if (id == HFDIB_FIELD_YPLUS) {
    // y+ of the boundary and domain-wall cells, 0 elsewhere
    hipLaunchKernelGGL(k_fill0, dim3(nblocks1(c->P.N)), dim3(NTHREADS), 0, c->stream, c->P.N, dst);
    if (c->n_bc > 0)
      hipLaunchKernelGGL(k_scatter_list, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, c->n_bc,
                         (const int*)c->bc_cells, (const double*)c->bc_yplus, dst);
    if (c->n_wall > 0)
      hipLaunchKernelGGL(k_scatter_list, dim3(nblocks1(c->n_wall)), dim3(NTHREADS), 0, c->stream, c->n_wall,
                         (const int*)c->wall_cells, (const double*)c->wall_yplus, dst);
    HFDIB_CHECK_LAUNCH(c, "get_field");
    return HFDIB_OK;
  }
  size_t n;
  double* src = field_ptr(c, id, &n);
  if (!src) return HFDIB_EINVAL;
  HFDIB_CHECK(c, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "get_field");
  return HFDIB_OK;
}

int hfdib_set_field(hfdib_ctx* c, int id, const double* src) {
  if (!c || !src) return HFDIB_EINVAL;
  if (id > HFDIB_FIELD_PHI_Z) return HFDIB_EINVAL;
  size_t n;
  double* dst = field_ptr(c, id, &n);
  if (!dst) return HFDIB_EINVAL;
  HFDIB_CHECK(c, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "set_field");
  return hfdib::refresh_mirrors(c);
}

int hfdib_forces(hfdib_ctx* c, double* out8) {
  if (!c || !out8) return HFDIB_EINVAL;
  if (!c->ready) {
    c->err = "hfdib_forces before hfdib_set_indicator";
    return HFDIB_ESTATE;
  }
  return hfdib::body_forces(c, out8);
}

int hfdib_force_coefficients(hfdib_ctx* c, double ref_area, double u_ref, const double* drag_dir,
                             const double* lift_dir, double* out2) {
  if (!c || !drag_dir || !lift_dir || !out2 || !(ref_area > 0.0) || u_ref == 0.0) return HFDIB_EINVAL;
  if (!c->ready) {
    c->err = "hfdib_force_coefficients before hfdib_set_indicator";
    return HFDIB_ESTATE;
  }
  double f[8];
  int st = hfdib::body_forces(c, f);
  if (st != HFDIB_OK) return st;
  const double q = 0.5 * u_ref * u_ref * ref_area;
  double cd = 0.0, cl = 0.0;
  for (int d = 0; d < 3; ++d) {
    cd += (f[d] + f[3 + d]) * drag_dir[d];
    cl += (f[d] + f[3 + d]) * lift_dir[d];
  }
  out2[0] = cd / q;
  out2[1] = cl / q;
  return HFDIB_OK;
}

int hfdib_forces_noalloc(hfdib_ctx* c, double* out8_dev) {
  if (!c || !out8_dev) return HFDIB_EINVAL;
  if (!c->ready) {
    c->err = "hfdib_forces_noalloc before hfdib_set_indicator";
    return HFDIB_ESTATE;
  }
  return hfdib::body_forces_noalloc(c, out8_dev);
}

int hfdib_autotune_tiles(hfdib_ctx* c, int reps, int* best_width, double* ms_out) {
  if (!c || reps < 1) return HFDIB_EINVAL;
  if (!c->ready) {
    c->err = "hfdib_autotune_tiles before hfdib_set_indicator";
    return HFDIB_ESTATE;
  }
  hipEvent_t e0, e1;
  HFDIB_CHECK(c, hipEventCreate(&e0), "autotune event");
  HFDIB_CHECK(c, hipEventCreate(&e1), "autotune event");
  int best = c->P.tx_log2;
  double best_ms = 0.0;
  int status = HFDIB_OK;
  for (int lx = TILE_LOG2_MIN; lx <= TILE_LOG2_MAX && status == HFDIB_OK; ++lx) {
    if (lx + c->P.tz_log2 > 8) {  // too wide for the current depth
      if (ms_out) ms_out[lx - TILE_LOG2_MIN] = -1.0;
      continue;
    }
    c->P.tx_log2 = lx;
    status = tile_bench_round(c);  // warm-up
    if (status != HFDIB_OK) break;
    (void)hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps && status == HFDIB_OK; ++r) status = tile_bench_round(c);
    (void)hipEventRecord(e1, c->stream);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) status = set_hip_error(c, e, "autotune timing");
    double avg = (double)ms / reps;
    if (ms_out) ms_out[lx - TILE_LOG2_MIN] = avg;
    if (best_ms == 0.0 || avg < best_ms) {
      best_ms = avg;
      best = lx;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->P.tx_log2 = best;
  if (best_width) *best_width = 1 << best;
  return status;
}

int hfdib_set_tile_width(hfdib_ctx* c, int width) {
  if (!c) return HFDIB_EINVAL;
  for (int lx = TILE_LOG2_MIN; lx <= TILE_LOG2_MAX; ++lx)
    if (width == (1 << lx)) {
      if (lx + c->P.tz_log2 > 8) {
        c->err = "tile width times depth exceeds 256 cells";
        return HFDIB_EINVAL;
      }
      c->P.tx_log2 = lx;
      return HFDIB_OK;
    }
  return HFDIB_EINVAL;
}

int hfdib_set_tile_order(hfdib_ctx* c, int zfirst) {
  if (!c || (zfirst != 0 && zfirst != 1)) return HFDIB_EINVAL;
  c->P.tile_zfirst = zfirst;
  return HFDIB_OK;
}

int hfdib_set_tile_depth(hfdib_ctx* c, int depth) {
  if (!c) return HFDIB_EINVAL;
  for (int lz = 0; lz <= 2; ++lz)
    if (depth == (1 << lz)) {
      if (c->P.nz % depth != 0 || (lz > 0 && c->P.dim != 3) || c->P.tx_log2 + lz > 8) {
        c->err = "tile depth must divide nz (3-D grids) and width times depth must not exceed 256";
        return HFDIB_EINVAL;
      }
      c->P.tz_log2 = lz;
      return HFDIB_OK;
    }
  return HFDIB_EINVAL;
}

int hfdib_get_counts(hfdib_ctx* c, int* counts) {
  if (!c || !counts) return HFDIB_EINVAL;
  if (!c->ready) return HFDIB_ESTATE;
  counts[0] = c->n_bc;
  counts[1] = c->n_ic;
  counts[2] = c->n_wall;
  return HFDIB_OK;
}

int hfdib_get_ib_array(hfdib_ctx* c, int id, void* dst) {
  if (!c || !dst) return HFDIB_EINVAL;
  if (!c->ready) return HFDIB_ESTATE;
  const void* src = nullptr;
  size_t bytes = 0;
  size_t nb = (size_t)c->n_bc, nw = (size_t)c->n_wall;
  switch (id) {
    case HFDIB_IB_BC_CELLS: src = c->bc_cells; bytes = nb * 4; break;
    case HFDIB_IB_IC_CELLS: src = c->ic_cells; bytes = (size_t)c->n_ic * 4; break;
    case HFDIB_IB_WALL_CELLS: src = c->wall_cells; bytes = nw * 4; break;
    case HFDIB_IB_NORMAL: src = c->bc_n; bytes = nb * 24; break;
    case HFDIB_IB_YPERP: src = c->bc_yperp; bytes = nb * 8; break;
    case HFDIB_IB_YEFF: src = c->bc_yeff; bytes = nb * 8; break;
    case HFDIB_IB_MODE: src = c->bc_mode; bytes = nb * 4; break;
    case HFDIB_IB_LAGRANGE: src = c->bc_L; bytes = nb * 24; break;
    case HFDIB_IB_ST1_IDX: src = c->bc_s1; bytes = nb * 32; break;
    case HFDIB_IB_ST1_W: src = c->bc_w1; bytes = nb * 64; break;
    case HFDIB_IB_ST2_IDX: src = c->bc_s2; bytes = nb * 32; break;
    case HFDIB_IB_ST2_W: src = c->bc_w2; bytes = nb * 64; break;
    case HFDIB_IB_YPLUS: src = c->bc_yplus; bytes = nb * 8; break;
    case HFDIB_IB_UTAU_LOGLAW: src = c->bc_utauU; bytes = nb * 8; break;
    case HFDIB_IB_WALL_Y: src = c->wall_y; bytes = nw * 8; break;
    case HFDIB_IB_UTAU: src = c->bc_utau; bytes = nb * 8; break;
    case HFDIB_IB_WALL_YPLUS: src = c->wall_yplus; bytes = nw * 8; break;
    case HFDIB_IB_WALL_UTAU: src = c->wall_utau; bytes = nw * 8; break;
    default: return HFDIB_EINVAL;
  }
  if (bytes == 0) return HFDIB_OK;
  HFDIB_CHECK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream), "get_ib_array");
  return HFDIB_OK;
}

int hfdib_pressure_solve(hfdib_ctx* c, const double* rAU, const double* rhs, double* p, double rtol, int maxit,
                         int* iters, double* relres) {
  if (!c || !rAU || !rhs || !p || !(rtol > 0.0) || maxit < 1) return HFDIB_EINVAL;
  if (!c->ready) return HFDIB_ESTATE;
  int it = 0;
  double rr = 0.0;
  int st = pressure_solve(c, rAU, rhs, p, rtol, maxit, &it, &rr, nullptr);
  if (iters) *iters = it;
  if (relres) *relres = rr;
  if (st == HFDIB_OK) HFDIB_CHECK(c, hipStreamSynchronize(c->stream), "pressure solve sync");
  return st;
}

int hfdib_last_stats(hfdib_ctx* c, double* out8) {
  if (!c || !out8) return HFDIB_EINVAL;
  memcpy(out8, c->stats, sizeof(c->stats));
  return HFDIB_OK;
}

int hfdib_timing_enable(hfdib_ctx* c, int enable) {
  if (!c || !c->timers || enable < 0) return HFDIB_EINVAL;
  if (!enable) timers_flush(c);
  c->timers->on = enable != 0;
  c->timers->every = enable > 0 ? enable : 1;
  c->timers->n_it = 0;
  c->timers->skip = false;
  return HFDIB_OK;
}

int hfdib_timing_query(hfdib_ctx* c, int cls, double* total_ms, long long* count) {
  if (!c || !c->timers || cls < 0 || cls >= T_NCLASS) return HFDIB_EINVAL;
  timers_flush(c);
  if (total_ms) *total_ms = c->timers->ms[cls];
  if (count) *count = c->timers->cnt[cls];
  return HFDIB_OK;
}

void hfdib_destroy(hfdib_ctx* c) {
  if (!c) return;
  if (c->timers) {
    timers_flush(c);
    delete c->timers;
  }
  if (c->hmir) (void)hipHostFree(c->hmir);
  delete c;
}

const char* hfdib_status_string(int s) {
  switch (s) {
    case HFDIB_OK: return "ok";
    case HFDIB_EINVAL: return "invalid argument";
    case HFDIB_ENOMEM: return "workspace too small";
    case HFDIB_EDEVICE: return "HIP runtime error";
    case HFDIB_EDIVERGED: return "diverged";
    case HFDIB_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

const char* hfdib_last_error(const hfdib_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
