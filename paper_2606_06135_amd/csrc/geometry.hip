// Per-lambda precompute (Sec. "Mask fields construction" and "Calculation of
// y+ at the immersed boundary"): validation, cell groups, ordered compaction of
// the boundary / in-solid / wall-function lists, per-boundary-cell geometry
// (normal, sigma, in-solid neighbour, y_perp, y_eff, interpolation stencils)
// and the SST wall distance.
#include "device_common.h"

namespace hfdib {

// ---------------------------------------------------------------- validation
__global__ void k_validate(Params P, const double* lam, int* bad) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (c >= P.N) return;
  double l = lam[c];
  if (!(l >= 0.0 && l <= 1.0)) atomicOr(bad, 1);
}

// ---------------------------------------------------------------- groups
// in-solid: lambda >= 0.5; boundary: 0 < lambda < 0.5, or lambda = 0 with an
// in-solid Moore neighbour; free-stream otherwise.  Also marks lambda > 0
// (walls inside the solid on domain faces), the red colour and the free-stream
// cells touching a no-slip domain face.
__global__ void k_classify(Params P, const double* lam, uint8_t* flags) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, k);
  double l = lam[c];
  uint8_t f = 0;
  bool ic = l >= 0.5;
  bool nbic = false;
  int zr = P.dim == 3 ? 1 : 0;
  for (int ox = -1; ox <= 1; ++ox)
    for (int oy = -1; oy <= 1; ++oy)
      for (int oz = -zr; oz <= zr; ++oz) {
        if (ox == 0 && oy == 0 && oz == 0) continue;
        int ii = i + ox, jj = j + oy, kk = k + oz;
        if (ii < 0 || ii >= P.nx || jj < 0 || jj >= P.ny || kk < 0 || kk >= P.nz) continue;
        if (lam[cidx(P, ii, jj, kk)] >= 0.5) nbic = true;
      }
  bool bc = (l > 0.0 && l < 0.5) || (l == 0.0 && nbic);
  // in-solid cells are always forced (alpha_u = alpha_k = alpha_omega = 1);
  // boundary cells always carry alpha_omega
  if (ic) f |= F_IC | F_ALPHA_U | F_ALPHA_W;
  else if (bc) f |= F_BC | F_ALPHA_W;
  if (l > 0.0) f |= F_SOLID;
  if (((i + j + k) & 1) == 0) f |= F_RED;
  if (!ic && !bc && l == 0.0) {
    for (int d = 0; d < P.dim; ++d)
      for (int s = -1; s <= 1; s += 2)
        if (on_bnd(P, d, s, i, j, k) && face_kind(P, d, s) == HFDIB_BC_NOSLIP) f |= F_WALL | F_ALPHA_W;
  }
  flags[c] = f;
}

// ---------------------------------------------------------------- compaction
// Ordered stream compaction of the cells whose flags match `mask`: per-block
// counts, one-block exclusive scan, then an in-order scatter (the lists are in
// increasing cell index, as their consumers expect).
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
  __shared__ int wsum[NTHREADS / 64];
  int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  unsigned long long m = __ballot(v != 0);
  int pre = __popcll(m & ((1ULL << lane) - 1ULL));
  if (lane == 0) wsum[wid] = __popcll(m);
  __syncthreads();
  int base = 0, tot = 0;
  for (int w = 0; w < NTHREADS / 64; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  *total = tot;
  return base + pre;
}

__global__ void k_count(Params P, const uint8_t* flags, uint8_t mask, int* counts) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  int v = (c < P.N && (flags[c] & mask)) ? 1 : 0;
  int tot;
  block_excl_scan(v, &tot);
  if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// exclusive scan of nb counts in place by a single block; total -> *total
__global__ void k_scan_counts(int* counts, int nb, int* total) {
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += NTHREADS) {
    int idx = base + threadIdx.x;
    int v = idx < nb ? counts[idx] : 0;
    // inclusive scan within the block (Hillis-Steele in LDS)
    __shared__ int buf[NTHREADS];
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < NTHREADS; off <<= 1) {
      int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    int incl = buf[threadIdx.x];
    if (idx < nb) counts[idx] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == NTHREADS - 1) carry += incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scatter(Params P, const uint8_t* flags, uint8_t mask, const int* offsets, int* list, int cap) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  int v = (c < P.N && (flags[c] & mask)) ? 1 : 0;
  int tot;
  int pos = block_excl_scan(v, &tot) + offsets[blockIdx.x];
  if (v && pos < cap) list[pos] = (int)c;
}

// ---------------------------------------------------------------- boundary cells
__device__ __forceinline__ bool inside_domain(const Params& P, V3 X) {
  if (!(P.x0 <= X.x && X.x <= P.x0 + P.nx * P.dx)) return false;
  if (!(P.y0 <= X.y && X.y <= P.y0 + P.ny * P.dy)) return false;
  if (P.dim == 3 && !(P.z0 <= X.z && X.z <= P.z0 + P.nz * P.dz)) return false;
  return true;
}

// multilinear interpolation stencil at X: cells ordered x-outer, z-inner
__device__ void stencil(const Params& P, V3 X, int* cells, double* w) {
  int i0[3];
  double f[3];
  double xs[3] = {X.x, X.y, X.z};
  double os[3] = {P.x0, P.y0, P.z0};
  for (int d = 0; d < 3; ++d) {
    if (d >= P.dim) {
      i0[d] = 0;
      f[d] = 0.0;
      continue;
    }
    double t = (xs[d] - os[d]) / P.delta[d] - 0.5;
    int a = (int)floor(t);
    int n = ncell(P, d);
    a = a < 0 ? 0 : a;
    a = a > n - 2 ? n - 2 : a;
    double ff = t - (double)a;
    ff = ff < 0.0 ? 0.0 : (ff > 1.0 ? 1.0 : ff);
    i0[d] = a;
    f[d] = ff;
  }
  int q = 0;
  int nzs = P.dim == 3 ? 2 : 1;
  for (int a = 0; a < 2; ++a) {
    double wx = a == 0 ? 1.0 - f[0] : f[0];
    for (int b = 0; b < 2; ++b) {
      double wy = b == 0 ? 1.0 - f[1] : f[1];
      for (int cc = 0; cc < nzs; ++cc) {
        double wz = P.dim == 3 ? (cc == 0 ? 1.0 - f[2] : f[2]) : 1.0;
        cells[q] = (int)cidx(P, i0[0] + a, i0[1] + b, i0[2] + cc);
        w[q] = wx * wy * wz;
        ++q;
      }
    }
  }
  for (; q < 8; ++q) {
    cells[q] = -1;
    w[q] = 0.0;
  }
}

__device__ bool usable(const Params& P, const uint8_t* flags, V3 X, int* cells, double* w) {
  if (!inside_domain(P, X)) return false;
  stencil(P, X, cells, w);
  for (int q = 0; q < 8; ++q)
    if (cells[q] >= 0 && w[q] > 1e-9 && (flags[cells[q]] & F_IC)) return false;
  return true;
}

__global__ void k_bc_geometry(Params P, int nbc, const int* bc_cells, const double* lam, const uint8_t* flags,
                              double* bc_n, double* bc_yperp, double* bc_yeff, int* bc_mode, double* bc_L,
                              int* st1, double* w1, int* st2, double* w2) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nbc) return;
  int c = bc_cells[b];
  int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / (P.nx * P.ny);
  V3 Pc = center(P, i, j, k);
  V3 nP = cell_normal(P, lam, flags, i, j, k);
  bc_n[3 * b + 0] = nP.x;
  bc_n[3 * b + 1] = nP.y;
  bc_n[3 * b + 2] = nP.z;
  double h = P.h;
  double lp = lam[c];
  double yp;
  if (lp > 0.0 && lp < 0.5) {
    yp = fabs(h * atanh(1.0 - 2.0 * lp));  // first case: |sigma_P|
  } else {
    // in-solid neighbour minimising -n_P.(P - N); among equal values (1e-12 h) the
    // nearer one; y_perp is the mean over neighbours that remain tied
    bool have = false;
    double bv = 0.0, bd = 0.0, ysum = 0.0;
    int ycnt = 0;
    int zr = P.dim == 3 ? 1 : 0;
    for (int ox = -1; ox <= 1; ++ox)
      for (int oy = -1; oy <= 1; ++oy)
        for (int oz = -zr; oz <= zr; ++oz) {
          if (ox == 0 && oy == 0 && oz == 0) continue;
          int ii = i + ox, jj = j + oy, kk = k + oz;
          if (ii < 0 || ii >= P.nx || jj < 0 || jj >= P.ny || kk < 0 || kk >= P.nz) continue;
          int cn = (int)cidx(P, ii, jj, kk);
          if (!(flags[cn] & F_IC)) continue;
          V3 N = center(P, ii, jj, kk);
          double px = Pc.x - N.x, py = Pc.y - N.y, pz = Pc.z - N.z;
          double v = -(nP.x * px + nP.y * py + nP.z * pz);
          double dist = sqrt(px * px + py * py + pz * pz);
          bool better = !have || v < bv - 1e-12 * h || (fabs(v - bv) <= 1e-12 * h && dist < bd - 1e-12 * h);
          bool tie = have && !better && fabs(v - bv) <= 1e-12 * h && fabs(dist - bd) <= 1e-12 * h;
          if (!better && !tie) continue;
          double yv;
          double ln = lam[cn];
          if (ln < 1.0) {
            // second case: distance to the plane through N + |sigma_N| n_N
            V3 nN = cell_normal(P, lam, flags, ii, jj, kk);
            double sN = fabs(h * atanh(1.0 - 2.0 * ln));
            double qx = Pc.x - (N.x + sN * nN.x), qy = Pc.y - (N.y + sN * nN.y), qz = Pc.z - (N.z + sN * nN.z);
            yv = nN.x * qx + nN.y * qy + nN.z * qz;
          } else {
            // third case: distance to the mean of the vertices shared by P and N
            double mx = (double)i + 0.5 + 0.5 * (double)ox;
            double my = (double)j + 0.5 + 0.5 * (double)oy;
            double vx = P.x0 + mx * P.dx, vy = P.y0 + my * P.dy, vz = 0.0;
            if (P.dim == 3) {
              double mz = (double)k + 0.5 + 0.5 * (double)oz;
              vz = P.z0 + mz * P.dz;
            }
            double qx = Pc.x - vx, qy = Pc.y - vy, qz = Pc.z - vz;
            yv = sqrt(qx * qx + qy * qy + qz * qz);
          }
          if (better) {
            have = true;
            bv = v;
            bd = dist;
            ysum = yv;
            ycnt = 1;
          } else {
            ysum += yv;
            ycnt += 1;
          }
        }
    // a boundary cell with lambda = 0 always has an in-solid neighbour
    yp = ycnt > 0 ? ysum / ycnt : 0.0;
  }
  double ymin = P.yperp_min_frac * h;
  yp = yp > ymin ? yp : ymin;
  bc_yperp[b] = yp;
  // y_eff of the y+ definition, or y_perp alone for the appendix variant
  bc_yeff[b] = P.yplus_perp ? yp : 0.5 * (yp + 0.5 * h);
  // interpolation points along n_P
  int c1[8], c2[8];
  double q1[8], q2[8];
  int mode = 1;
  double L0 = 1.0, L1 = 0.0, L2 = 0.0;
  bool done = false;
  for (int m = 1; m <= 3 && !done; ++m) {
    V3 X1 = {Pc.x + m * h * nP.x, Pc.y + m * h * nP.y, Pc.z + m * h * nP.z};
    V3 X2 = {Pc.x + (m + 1) * h * nP.x, Pc.y + (m + 1) * h * nP.y, Pc.z + (m + 1) * h * nP.z};
    if (usable(P, flags, X1, c1, q1) && usable(P, flags, X2, c2, q2)) {
      double s = yp, s1 = yp + m * h, s2 = yp + (m + 1) * h;
      L0 = (s - s1) * (s - s2) / (s1 * s2);
      L1 = s * (s - s2) / (s1 * (s1 - s2));
      L2 = s * (s - s1) / (s2 * (s2 - s1));
      mode = 3;
      done = true;
    }
  }
  if (!done) {
    for (int m = 1; m <= 3 && !done; ++m) {
      V3 X1 = {Pc.x + m * h * nP.x, Pc.y + m * h * nP.y, Pc.z + m * h * nP.z};
      if (usable(P, flags, X1, c1, q1)) {
        double s1 = yp + m * h;
        L0 = 1.0 - yp / s1;
        L1 = yp / s1;
        L2 = 0.0;
        for (int q = 0; q < 8; ++q) {
          c2[q] = -1;
          q2[q] = 0.0;
        }
        mode = 2;
        done = true;
      }
    }
  }
  if (!done) {
    for (int q = 0; q < 8; ++q) {
      c1[q] = -1;
      q1[q] = 0.0;
      c2[q] = -1;
      q2[q] = 0.0;
    }
  }
  bc_mode[b] = mode;
  bc_L[3 * b + 0] = L0;
  bc_L[3 * b + 1] = L1;
  bc_L[3 * b + 2] = L2;
  for (int q = 0; q < 8; ++q) {
    st1[8 * b + q] = c1[q] < 0 ? c : c1[q];
    w1[8 * b + q] = q1[q];
    st2[8 * b + q] = c2[q] < 0 ? c : c2[q];
    w2[8 * b + q] = q2[q];
  }
}

// first cells at no-slip domain faces: distance half a cell width of the
// first (in face order) nearest face; unit normal pointing into the domain
__global__ void k_wall_geometry(Params P, int nw, const int* wall_cells, double* wall_y, double* wall_n) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  if (b >= nw) return;
  int c = wall_cells[b];
  int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / (P.nx * P.ny);
  double best = 1e300;
  double n[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < P.dim; ++d)
    for (int s = -1; s <= 1; s += 2) {
      if (!on_bnd(P, d, s, i, j, k) || face_kind(P, d, s) != HFDIB_BC_NOSLIP) continue;
      double y = 0.5 * P.delta[d];
      if (y < best) {
        best = y;
        n[0] = n[1] = n[2] = 0.0;
        n[d] = -(double)s;
      }
    }
  wall_y[b] = best;
  wall_n[3 * b + 0] = n[0];
  wall_n[3 * b + 1] = n[1];
  wall_n[3 * b + 2] = n[2];
}

// ---------------------------------------------------------------- wall distance
// Interface points: S-points P - sigma_P n_P of cut cells (0 < lambda < 1) and
// midpoints of faces between lambda = 0 and lambda = 1 face neighbours.  Each
// cell contributes at most 1 + dim points; slots are compacted afterwards.
__global__ void k_iface_points(Params P, const double* lam, const uint8_t* flags, double* pts, int* cnt, int cap) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  if (i >= P.nx || j >= P.ny) return;
  long long c = cidx(P, i, j, k);
  double l = lam[c];
  V3 Pc = center(P, i, j, k);
  if (l > 0.0 && l < 1.0) {
    V3 n = cell_normal(P, lam, flags, i, j, k);
    double sg = P.h * atanh(1.0 - 2.0 * l);
    int s = atomicAdd(cnt, 1);
    if (s < cap) {
      pts[3 * s + 0] = Pc.x - sg * n.x;
      pts[3 * s + 1] = Pc.y - sg * n.y;
      pts[3 * s + 2] = Pc.z - sg * n.z;
    }
  }
  for (int d = 0; d < P.dim; ++d) {
    if (on_bnd(P, d, +1, i, j, k)) continue;
    double ln = lam[c + stride(P, d)];
    if ((l == 0.0 && ln == 1.0) || (l == 1.0 && ln == 0.0)) {
      int s = atomicAdd(cnt, 1);
      if (s < cap) {
        double q[3] = {Pc.x, Pc.y, Pc.z};
        q[d] += 0.5 * P.delta[d];
        pts[3 * s + 0] = q[0];
        pts[3 * s + 1] = q[1];
        pts[3 * s + 2] = q[2];
      }
    }
  }
}

// brute-force minimum distance to the point set (LDS-tiled) and to no-slip walls
__global__ void k_wall_distance(Params P, const double* pts, int npts, double* dw) {
  __shared__ double sp[3 * NTHREADS];
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  bool act = c < P.N;
  int i = 0, j = 0, k = 0;
  if (act) {
    i = (int)(c % P.nx);
    j = (int)((c / P.nx) % P.ny);
    k = (int)(c / ((long long)P.nx * P.ny));
  }
  V3 X = center(P, i, j, k);
  double best2 = 1e300;
  for (int base = 0; base < npts; base += NTHREADS) {
    int q = base + threadIdx.x;
    if (q < npts) {
      sp[3 * threadIdx.x + 0] = pts[3 * q + 0];
      sp[3 * threadIdx.x + 1] = pts[3 * q + 1];
      sp[3 * threadIdx.x + 2] = pts[3 * q + 2];
    }
    __syncthreads();
    int m = npts - base < NTHREADS ? npts - base : NTHREADS;
    for (int t = 0; t < m; ++t) {
      double ex = X.x - sp[3 * t], ey = X.y - sp[3 * t + 1], ez = X.z - sp[3 * t + 2];
      double d2 = ex * ex + ey * ey + ez * ez;
      best2 = d2 < best2 ? d2 : best2;
    }
    __syncthreads();
  }
  if (!act) return;
  double best = best2 < 1e299 ? sqrt(best2) : 1e30;
  double xs[3] = {X.x, X.y, X.z};
  double os[3] = {P.x0, P.y0, P.z0};
  for (int d = 0; d < P.dim; ++d)
    for (int s = -1; s <= 1; s += 2) {
      if (face_kind(P, d, s) != HFDIB_BC_NOSLIP) continue;
      double wall = os[d] + (s < 0 ? 0.0 : ncell(P, d) * P.delta[d]);
      double dd = fabs(xs[d] - wall);
      best = dd < best ? dd : best;
    }
  dw[c] = best;
}

// ---------------------------------------------------------------- host driver
static int compact(hfdib_ctx* c, uint8_t mask, int* list, int* n_out) {
  const Params& P = c->P;
  int nb = nblocks1(P.N);
  int* counts = (int*)c->t0;  // scratch (>= N doubles)
  int* total = c->iscal + 8;
  hipLaunchKernelGGL(k_count, dim3(nb), dim3(NTHREADS), 0, c->stream, P, c->flags, mask, counts);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(NTHREADS), 0, c->stream, counts, nb, total);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(NTHREADS), 0, c->stream, P, c->flags, mask, counts, list, c->cap);
  HFDIB_CHECK_LAUNCH(c, "compaction");
  int h = 0;
  HFDIB_CHECK(c, hipMemcpyAsync(&h, total, sizeof(int), hipMemcpyDeviceToHost, c->stream), "compaction copy");
  HFDIB_CHECK(c, hipStreamSynchronize(c->stream), "compaction sync");
  *n_out = h;
  if (h > c->cap) {
    c->err = "list capacity exceeded (raise hfdib_config.bc_capacity)";
    return HFDIB_EINVAL;
  }
  return HFDIB_OK;
}

int geometry_precompute(hfdib_ctx* c) {
  const Params& P = c->P;
  int nb = nblocks1(P.N);
  int* bad = c->iscal;
  HFDIB_CHECK(c, hipMemsetAsync(c->iscal, 0, 64 * sizeof(int), c->stream), "memset");
  hipLaunchKernelGGL(k_validate, dim3(nb), dim3(NTHREADS), 0, c->stream, P, c->lam, bad);
  HFDIB_CHECK_LAUNCH(c, "validate");
  int hb = 0;
  HFDIB_CHECK(c, hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
  HFDIB_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  if (hb) {
    c->err = "lambda contains NaN or values outside [0,1]";
    return HFDIB_EINVAL;
  }
  hipLaunchKernelGGL(k_classify, grid3(P), block3(P), 0, c->stream, P, c->lam, c->flags);
  HFDIB_CHECK_LAUNCH(c, "classify");
  int st;
  if ((st = compact(c, F_BC, c->bc_cells, &c->n_bc)) != HFDIB_OK) return st;
  if ((st = compact(c, F_IC, c->ic_cells, &c->n_ic)) != HFDIB_OK) return st;
  if ((st = compact(c, F_WALL, c->wall_cells, &c->n_wall)) != HFDIB_OK) return st;
  if (c->n_bc > 0)
    hipLaunchKernelGGL(k_bc_geometry, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, P, c->n_bc,
                       c->bc_cells, c->lam, c->flags, c->bc_n, c->bc_yperp, c->bc_yeff, c->bc_mode, c->bc_L,
                       c->bc_s1, c->bc_w1, c->bc_s2, c->bc_w2);
  if (c->n_wall > 0)
    hipLaunchKernelGGL(k_wall_geometry, dim3(nblocks1(c->n_wall)), dim3(NTHREADS), 0, c->stream, P, c->n_wall,
                       c->wall_cells, c->wall_y, c->wall_n);
  HFDIB_CHECK_LAUNCH(c, "bc geometry");
  if (P.model == HFDIB_KOMEGA_SST) {
    int* cnt = c->iscal + 16;
    hipLaunchKernelGGL(k_iface_points, grid3(P), block3(P), 0, c->stream, P, c->lam, c->flags, c->ipts, cnt,
                       c->cap);
    HFDIB_CHECK_LAUNCH(c, "interface points");
    int h = 0;
    HFDIB_CHECK(c, hipMemcpyAsync(&h, cnt, sizeof(int), hipMemcpyDeviceToHost, c->stream), "copy");
    HFDIB_CHECK(c, hipStreamSynchronize(c->stream), "sync");
    if (h > c->cap) {
      c->err = "interface point capacity exceeded (raise hfdib_config.bc_capacity)";
      return HFDIB_EINVAL;
    }
    c->n_ipts = h;
    hipLaunchKernelGGL(k_wall_distance, dim3(nb), dim3(NTHREADS), 0, c->stream, P, c->ipts, h, c->dw);
    HFDIB_CHECK_LAUNCH(c, "wall distance");
  }
  return HFDIB_OK;
}

}  // namespace hfdib
