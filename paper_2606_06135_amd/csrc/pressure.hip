// Pressure-correction system of the lambda-masked continuity equation:
//   sum_f c_f (p_P - p_nb) + sum_outlet c_b p_P = rhs,
//   c_f = mean(rAU) |S_f| / d_f,  c_b = rAU_P |S| / (d/2)  (SPD, 5/7-point).
// Conjugate gradients preconditioned by one symmetric geometric-multigrid
// V-cycle (red-black Gauss-Seidel, 1 pre- and 1 post-sweep per level,
// piecewise-constant transfer, rediscretised coarse operators).  The fine
// level is matrix free (coefficients from rAU); coarse levels store face
// coefficients.  All dot products are deterministic two-pass reductions.
// Precision: the CG vectors, the operator apply, the residual and every dot
// product are FP64.  The V-cycle is templated on its storage type: FP64, or
// FP32 in the mixed policy (FP32 mirrors of rAU, of the residual and of every
// coarse operator; the preconditioner output is read back by the FP64 CG).
#include "device_common.h"

#include <utility>

#include <cmath>
#include <vector>

namespace hfdib {

enum {
  S_RHO = 0, S_ALPHA, S_BETA, S_RR, S_BB, S_DQ, S_RZ, S_RES0, S_RES1, S_RES2,  // pcg scalars
};

// ---------------------------------------------------------------- fine level
template <typename T>
struct FineOpT {
  const T* rAU;
  const uint8_t* flags;
};
using FineOp = FineOpT<double>;

template <typename T>
__device__ __forceinline__ T fine_coef(const Params& P, const FineOpT<T>& O, long long c, int d, int s, int i, int j,
                                       int k, long long* nb) {
  // both values from clamped loads, chosen with selects
  const bool b = on_bnd(P, d, s, i, j, k);
  const long long n = b ? c : c + s * stride(P, d);
  *nb = b ? -1 : n;
  const T rc = O.rAU[c], rn = O.rAU[n];
  const bool outl = face_kind(P, d, s) == HFDIB_BC_OUTLET && !(O.flags[c] & F_SOLID);
  return sel(b, sel(outl, rc * (T)P.Ab[d], (T)0), (T)0.5 * (rc + rn) * (T)P.AoD[d]);
}

// The six face coefficients of a fine-level row from clamped loads (no branch
// around a load): c_f = mean(rAU) |S|/d inside, rAU_P |S|/(d/2) on outlet faces
// of cells with lambda = 0, 0 on other domain faces and beyond dim.
template <typename T>
__device__ __forceinline__ void fine_row(const Params& P, const FineOpT<T>& O, const Nbr& N, long long c,
                                         T (&cf)[6]) {
  const T rc = O.rAU[c];
  T rn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) rn[q] = O.rAU[N.n[q]];  // all six (clamped) loads in flight together
  const bool solid = O.flags[c] & F_SOLID;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int d = q >> 1;
    const T inner = (T)0.5 * (rc + rn[q]) * (T)P.AoD[d];
    const T outl = sel(P.p_outlet[q] != 0 && !solid, rc * (T)P.Ab[d], (T)0);
    cf[q] = sel(d < P.dim, sel(is_bnd(N, q), outl, inner), (T)0);
  }
}

// (A x)_c of a fine row and the sum of its coefficients (0: uncoupled row)
template <typename T>
__device__ __forceinline__ T fine_Ax(const T (&cf)[6], const Nbr& N, const T* x, long long c, T& dg,
                                     T& bnd_sum) {
  const T xc = x[c];
  T xn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) xn[q] = x[N.n[q]];
  T acc = (T)0, bs = (T)0;
  dg = (T)0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const bool b = is_bnd(N, q);
    acc = sel(b, acc + cf[q] * xc, acc + cf[q] * (xc - xn[q]));
    bs = sel(b, bs + cf[q], bs);
    dg += cf[q];
  }
  bnd_sum = bs;
  return acc;
}

// Inside the V-cycle the fine-level vectors of the smoother (z, the residual r
// and the inverse diagonal) are stored colour-split (rb_split: all cells of one
// colour, then the other, each row's cells of a colour contiguous), so that a
// one-colour half sweep reads and writes only the halves it needs; the
// V-cycle's input r and output z are in the natural order (nb_split gives the
// split index of a face neighbour).

// y = A x (and partial sums of x.y)
__global__ void k_fine_apply(Params P, FineOp O, const double* x, double* y, double* part, long long pstride) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  double v[1] = {0.0};
  if (i < P.nx && j < P.ny) {
    long long c = cidx(P, i, j, k);
    Nbr N = make_nbr(P, i, j, k, c);
    double cf[6], dg, bs;
    fine_row(P, O, N, c, cf);
    double xc = x[c];
    double acc = fine_Ax(cf, N, x, c, dg, bs);
    if (dg == 0.0) acc = xc;  // uncoupled row: identity
    y[c] = acc;
    v[0] = xc * acc;
  }
  block_sums_store<1>(v, part, pstride, block_linear());
}

// the direction update d = z + beta d_old fused with y = A d (and partial sums
// of d.y): each cell forms d at itself and its neighbours as the update would
// (the same operations, so the same values), writes its own d to d_new and y
template <typename TZ>
__global__ void k_fine_apply_dir(Params P, FineOp O, const TZ* z, const double* d_old, double* d_new, double* y,
                                 const double* scal, double* part, long long pstride) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  double v[1] = {0.0};
  if (i < P.nx && j < P.ny) {
    long long c = cidx(P, i, j, k);
    Nbr N = make_nbr(P, i, j, k, c);
    double cf[6];
    fine_row(P, O, N, c, cf);
    const double beta = scal[S_BETA];
    const double dc = (double)z[c] + beta * d_old[c];
    double dn[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) dn[q] = (double)z[N.n[q]] + beta * d_old[N.n[q]];
    double acc = 0.0, dg = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      acc = sel(is_bnd(N, q), acc + cf[q] * dc, acc + cf[q] * (dc - dn[q]));
      dg += cf[q];
    }
    if (dg == 0.0) acc = dc;  // uncoupled row: identity
    d_new[c] = dc;
    y[c] = acc;
    v[0] = dc * acc;
  }
  block_sums_store<1>(v, part, pstride, block_linear());
}

// r = b - A x (and its FP32 copy when r32 is given); partial sums of r.r, b.b
// and (for the SIMPLE residual) |r|, |Ax - A xbar|, |b - A xbar| with
// xbar = *xmean (nullable)
// (also the inverse diagonal of the fine smoother, colour-split, in FP64
// (invD64) or FP32 (invD32, with the FP32 mirror of rAU): the row sum the
// residual forms anyway)
__global__ void k_fine_residual(Params P, FineOp O, const double* b, const double* x, double* r, float* r32,
                                const double* xmean, double* part, long long pstride, double* invD64,
                                float* invD32, float* rAU32) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  double v[5] = {0, 0, 0, 0, 0};
  if (i < P.nx && j < P.ny) {
    long long c = cidx(P, i, j, k);
    Nbr N = make_nbr(P, i, j, k, c);
    double cf[6], dg, bnd;
    fine_row(P, O, N, c, cf);
    double xc = x[c];
    double acc = fine_Ax(cf, N, x, c, dg, bnd);
    const bool ident = dg == 0.0;  // uncoupled row: identity
    if (ident) acc = xc;
    double bc = b[c];
    double rc = bc - acc;
    r[c] = rc;
    if (r32) r32[c] = (float)rc;
    const double idg = ident ? 1.0 : 1.0 / dg;
    if (invD64) invD64[rb_split(P, i, j, k)] = idg;
    if (invD32) {
      invD32[rb_split(P, i, j, k)] = (float)idg;
      rAU32[c] = (float)O.rAU[c];
    }
    v[0] = rc * rc;
    // |b| of the relative tolerance and the normalised residual: coupled rows only
    // (an identity row's right-hand side is a pressure value, not a source)
    if (!ident) {
      v[1] = bc * bc;
      if (xmean) {
        double Axb = bnd * (*xmean);
        v[2] = fabs(rc);
        v[3] = fabs(acc - Axb);
        v[4] = fabs(bc - Axb);
      }
    }
  }
  block_sums_store<5>(v, part, pstride, block_linear());
}

// Fine-level smoothing.  The V-cycle uses one red-black Gauss-Seidel sweep
// before (red first, from z = 0) and one after (black first) the coarse
// correction; the inverse diagonal D^-1 of the fine operator (1 for uncoupled
// rows) is formed once per pressure solve, by the initial residual pass.

// Pre-smoothing sweep in one pass: the red value of a cell is r D^-1 (its
// neighbours are 0 before the sweep), so each thread takes one red/black pair
// of a row, writes the red value and the black value
// (r + sum_f c_f r_nb D^-1_nb) D^-1 from recomputed red neighbour values.  It
// reads r in the natural order and leaves z and r colour-split (zs, rs) for
// the rest of the V-cycle.
template <typename T>
__global__ void k_fine_presmooth(Params P, FineOpT<T> O, const T* invD, const T* r, T* zs, T* rs) {
  int i, j, k;
  tile_ijk_rb(P, 0, i, j, k);  // i: the red cell of the pair
  if (j >= P.ny) return;
  if (i < P.nx) {
    const long long c = cidx(P, i, j, k), sp = rb_split(P, i, j, k);
    const T rc = r[c];
    zs[sp] = rc * invD[sp];
    rs[sp] = rc;
  }
  int ib = i ^ 1;  // the black cell of the pair
  if (ib >= P.nx) return;
  long long c = cidx(P, ib, j, k);
  Nbr N = make_nbr(P, ib, j, k, c);
  T cf[6];
  fine_row(P, O, N, c, cf);
  T rn[6], dn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    rn[q] = r[N.n[q]];
    dn[q] = invD[nb_split(P, N, ib, j, k, q)];
  }
  T nb = (T)0;
#pragma unroll
  for (int q = 0; q < 6; ++q) nb = sel(is_bnd(N, q), nb, nb + cf[q] * (rn[q] * dn[q]));
  const long long sp = rb_split(P, ib, j, k);
  const T rc = r[c];
  zs[sp] = (rc + nb) * invD[sp];
  rs[sp] = rc;
}

// One colour of a red-black half sweep (all neighbours are of the other
// colour): z = (r + sum_f c_f z_nb) D^-1, on the colour-split z, r and D^-1.
// When zc is given (first sweep after the coarse correction, black), the
// neighbour values are taken as z_nb + zc(parent of nb): the prolongation is
// applied on the fly (the prolonged values of this colour are overwritten,
// those of the other colour are only read here and overwritten by the next
// sweep).
template <typename T>
__global__ void k_fine_smooth(Params P, FineOpT<T> O, const T* invD, const T* r, T* z, int color, const T* zc,
                              int cnx, int cny, const double* rdot, double* part, long long pstride, double* dcopy,
                              T* zout) {
  int i, j, k;
  tile_ijk_rb(P, color, i, j, k);
  const bool own = i < P.nx && j < P.ny;
  T znew = (T)0;
  long long c = 0;
  if (own) {
    c = cidx(P, i, j, k);
    Nbr N = make_nbr(P, i, j, k, c);
    T cf[6];
    fine_row(P, O, N, c, cf);
    T nb = (T)0;
    T zn[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) zn[q] = z[nb_split(P, N, i, j, k, q)];
    if (zc) {
      const int i2 = i >> 1, j2 = j >> 1, k2 = P.dim == 3 ? k >> 1 : 0;
      T zp[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int d = q >> 1, s = (q & 1) ? 1 : -1;
        // parent of the neighbour: only its coordinate along d differs (the
        // own parent for a domain face, whose term is not used)
        const bool b = is_bnd(N, q);
        const int pi = (d == 0 && !b) ? (i + s) >> 1 : i2, pj = (d == 1 && !b) ? (j + s) >> 1 : j2;
        const int pk = (d == 2 && !b) ? (k + s) >> 1 : k2;
        zp[q] = zc[(long long)pi + (long long)cnx * ((long long)pj + (long long)cny * pk)];
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) nb = sel(is_bnd(N, q), nb, nb + cf[q] * (zn[q] + zp[q]));
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) nb = sel(is_bnd(N, q), nb, nb + cf[q] * zn[q]);
    }
    const long long sp = rb_split(P, i, j, k);
    znew = (r[sp] + nb) * invD[sp];
    z[sp] = znew;
  }
  // the last sweep of a V-cycle writes z in the natural order (zout: both cells
  // of its pair, the other one's z being already final) and forms the partial
  // sums of r . z (FP64 r); optionally it copies both cells' z to the FP64
  // search direction (dcopy)
  if (rdot) {
    double v[1] = {0.0};
    if (j < P.ny) {
      if (own) {
        v[0] = rdot[c] * (double)znew;
        zout[c] = znew;
        if (dcopy) dcopy[c] = (double)znew;
      }
      const int io = i ^ 1;
      if (io < P.nx) {
        const long long co = cidx(P, io, j, k);
        const T zo = z[rb_split(P, io, j, k)];
        v[0] += rdot[co] * (double)zo;
        zout[co] = zo;
        if (dcopy) dcopy[co] = (double)zo;
      }
    }
    block_sums_store<1>(v, part, pstride, block_linear());
  }
}

// ---------------------------------------------------------------- coarse levels
template <typename T>
struct LevelDevT {
  int nx, ny, nz, dim;
  long long N;
  T* r;
  T* z;
  const T* cx;
  const T* cy;
  const T* cz;
  const T* diag;
};

template <typename T>
__device__ __forceinline__ long long lidx(const LevelDevT<T>& L, int i, int j, int k) {
  return (long long)i + (long long)L.nx * ((long long)j + (long long)L.ny * k);
}

// coefficients of level 1 from the fine operator (always evaluated in FP64 from
// rAU, then stored as T): sum of the fine face coefficients on each coarse
// face, halved (rediscretisation on the 2h grid)
// Coarse operator of level L in one pass per cell: its six face coefficients
// (half the sum of the fine faces they cover, each interior face computed alike by
// both cells that share it), stored as the low faces of each cell plus the high
// faces on the domain boundary, and the diagonal (sum of the six; an uncoupled
// cell gets 1).  From the fine operator (FROM_FINE) or from level F.
template <typename T>
__device__ __forceinline__ T cface_fine(const Params& P, const FineOp& O, const LevelDevT<T>& L, int d, int I, int J,
                                        int K) {
  // the fine faces under coarse face (d; I, J, K): the low faces of the first
  // fine layer of the coarse cell, or on the high domain boundary the high faces
  // of the last fine layer; all four read (in 2-D the second layer along z
  // repeats the first and is not added)
  const bool d3 = L.dim == 3;
  double v[4];
  long long n;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int i, j, k, sg;
      if (d == 0) {
        const bool low = I < L.nx;
        i = low ? 2 * I : 2 * I - 1, j = 2 * J + a, k = d3 ? 2 * K + b : 0, sg = low ? -1 : 1;
      } else if (d == 1) {
        const bool low = J < L.ny;
        i = 2 * I + a, j = low ? 2 * J : 2 * J - 1, k = d3 ? 2 * K + b : 0, sg = low ? -1 : 1;
      } else {
        const bool low = K < L.nz;
        i = 2 * I + a, j = 2 * J + b, k = low ? 2 * K : 2 * K - 1, sg = low ? -1 : 1;
      }
      v[2 * a + b] = fine_coef(P, O, cidx(P, i, j, k), d, sg, i, j, k, &n);
    }
  // summed in the order of the loops over the two tangential directions
  double s = 0.0;
  if (d == 2) {
    s = v[0] + v[1] + v[2] + v[3];
  } else {
    s = s + v[0];
    s = sel(d3, s + v[1], s);
    s = s + v[2];
    s = sel(d3, s + v[3], s);
  }
  return (T)(0.5 * s);
}
template <typename T>
__device__ __forceinline__ T cface_level(const LevelDevT<T>& F, const LevelDevT<T>& L, int d, int I, int J, int K) {
  const int nzs = L.dim == 3 ? 2 : 1;
  T s = (T)0;
  if (d == 0) {
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < nzs; ++e) {
        int j = 2 * J + b, k = L.dim == 3 ? 2 * K + e : 0;
        s += F.cx[(long long)(2 * I) + (long long)(F.nx + 1) * ((long long)j + (long long)F.ny * k)];
      }
  } else if (d == 1) {
    for (int a = 0; a < 2; ++a)
      for (int e = 0; e < nzs; ++e) {
        int i = 2 * I + a, k = L.dim == 3 ? 2 * K + e : 0;
        s += F.cy[(long long)i + (long long)F.nx * ((long long)(2 * J) + (long long)(F.ny + 1) * k)];
      }
  } else {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        int i = 2 * I + a, j = 2 * J + b;
        s += F.cz[(long long)i + (long long)F.nx * ((long long)j + (long long)F.ny * (2 * K))];
      }
  }
  return (T)0.5 * s;
}
template <typename T, bool FROM_FINE>
__global__ void k_coarsen_diag(Params P, FineOp O, LevelDevT<T> F, LevelDevT<T> L, T* cx, T* cy, T* cz, T* diag) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= L.nx || J >= L.ny) return;
  auto face = [&](int d, int a, int b, int e) {
    return FROM_FINE ? cface_fine<T>(P, O, L, d, a, b, e) : cface_level<T>(F, L, d, a, b, e);
  };
  const T xl = face(0, I, J, K), xh = face(0, I + 1, J, K);
  const T yl = face(1, I, J, K), yh = face(1, I, J + 1, K);
  const bool d3 = L.dim == 3;
  const T zl = d3 ? face(2, I, J, K) : (T)0, zh = d3 ? face(2, I, J, K + 1) : (T)0;
  cx[(long long)I + (long long)(L.nx + 1) * ((long long)J + (long long)L.ny * K)] = xl;
  if (I == L.nx - 1) cx[(long long)L.nx + (long long)(L.nx + 1) * ((long long)J + (long long)L.ny * K)] = xh;
  cy[(long long)I + (long long)L.nx * ((long long)J + (long long)(L.ny + 1) * K)] = yl;
  if (J == L.ny - 1) cy[(long long)I + (long long)L.nx * ((long long)L.ny + (long long)(L.ny + 1) * K)] = yh;
  if (d3) {
    cz[(long long)I + (long long)L.nx * ((long long)J + (long long)L.ny * K)] = zl;
    if (K == L.nz - 1) cz[(long long)I + (long long)L.nx * ((long long)J + (long long)L.ny * L.nz)] = zh;
  }
  T sd = xl + xh + yl + yh;
  if (d3) sd += zl + zh;
  diag[lidx(L, I, J, K)] = sd == (T)0 ? (T)1 : sd;  // uncoupled coarse cells: identity
}


// coefficients of level l+1 from the stored coefficients of level l (F)


// off-diagonal sum sum_nb c z_nb at (i,j,k) of a stored level
template <typename T>
__device__ __forceinline__ T level_nbsum(const LevelDevT<T>& L, const T* z, int i, int j, int k) {
  long long c = lidx(L, i, j, k);
  T s = (T)0;
  if (i > 0) s += L.cx[(long long)i + (long long)(L.nx + 1) * ((long long)j + (long long)L.ny * k)] * z[c - 1];
  if (i < L.nx - 1)
    s += L.cx[(long long)(i + 1) + (long long)(L.nx + 1) * ((long long)j + (long long)L.ny * k)] * z[c + 1];
  if (j > 0) s += L.cy[(long long)i + (long long)L.nx * ((long long)j + (long long)(L.ny + 1) * k)] * z[c - L.nx];
  if (j < L.ny - 1)
    s += L.cy[(long long)i + (long long)L.nx * ((long long)(j + 1) + (long long)(L.ny + 1) * k)] * z[c + L.nx];
  if (L.dim == 3) {
    long long sz = (long long)L.nx * L.ny;
    if (k > 0) s += L.cz[(long long)i + (long long)L.nx * ((long long)j + (long long)L.ny * k)] * z[c - sz];
    if (k < L.nz - 1) s += L.cz[(long long)i + (long long)L.nx * ((long long)j + (long long)L.ny * (k + 1))] * z[c + sz];
  }
  return s;
}

// Coarse-level smoothing with the structure of the fine level: one pass for
// the pre-smoothing sweep (red r/diag from zero, then black from the
// recomputed red values), the restriction of the red rows' residuals only,
// and the prolongation applied on the fly by the first post-smoothing sweep.
// Thread t of a row (j, k) takes the pair of cells 2t, 2t+1.
template <typename T>
__device__ __forceinline__ bool level_pair(const LevelDevT<T>& L, int color, int& i, int& j, int& k) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  j = blockIdx.y * blockDim.y + threadIdx.y;
  k = blockIdx.z;
  i = 2 * t + ((j + k + color) & 1);
  return j < L.ny;
}

// sum_nb c_nb f(nb) at (i,j,k) of a stored level (f gives the neighbour value)
template <typename T, typename F>
__device__ __forceinline__ T level_nbsum_f(const LevelDevT<T>& L, int i, int j, int k, F f) {
  // all six terms from clamped loads (a face on the domain boundary takes the
  // cell itself and offset 0, and its term is dropped by a select): the loads of
  // the stencil are in flight together
  const long long c = lidx(L, i, j, k);
  const long long sz = (long long)L.nx * L.ny;
  const bool in[6] = {i > 0, i < L.nx - 1, j > 0, j < L.ny - 1, L.dim == 3 && k > 0, L.dim == 3 && k < L.nz - 1};
  const long long cf[6] = {
      (long long)i + (long long)(L.nx + 1) * ((long long)j + (long long)L.ny * k),
      (long long)(i + 1) + (long long)(L.nx + 1) * ((long long)j + (long long)L.ny * k),
      (long long)i + (long long)L.nx * ((long long)j + (long long)(L.ny + 1) * k),
      (long long)i + (long long)L.nx * ((long long)(j + 1) + (long long)(L.ny + 1) * k),
      (long long)i + (long long)L.nx * ((long long)j + (long long)L.ny * k),
      (long long)i + (long long)L.nx * ((long long)j + (long long)L.ny * (k + 1))};
  const T* coef[6] = {L.cx, L.cx, L.cy, L.cy, L.cz, L.cz};
  const long long st[6] = {-1, 1, -(long long)L.nx, (long long)L.nx, -sz, sz};
  T a[6], v[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int s = (q & 1) ? 1 : -1, d = q >> 1;
    const bool use = in[q];
    a[q] = coef[q][cf[q]];  // (the z-face arrays have nz + 1 planes in 2-D as well)
    v[q] = f(use ? c + st[q] : c, (d == 0 && use) ? s : 0, (d == 1 && use) ? s : 0, (d == 2 && use) ? s : 0);
  }
  T sum = (T)0;
#pragma unroll
  for (int q = 0; q < 6; ++q) sum = sel(in[q], sum + a[q] * v[q], sum);
  return sum;
}

template <typename T>
__global__ void k_level_presmooth(LevelDevT<T> L) {
  int i, j, k;
  if (!level_pair(L, 0, i, j, k)) return;  // i: the red cell of the pair
  if (i < L.nx) {
    long long c = lidx(L, i, j, k);
    L.z[c] = L.r[c] / L.diag[c];
  }
  int ib = i ^ 1;
  if (ib >= L.nx) return;
  long long c = lidx(L, ib, j, k);
  T nb = level_nbsum_f(L, ib, j, k, [&](long long n, int, int, int) { return L.r[n] / L.diag[n]; });
  L.z[c] = (L.r[c] + nb) / L.diag[c];
}

// one colour of a half sweep; with zc (coarse correction of the next level),
// the neighbour values are z_nb + zc(parent of nb)
template <typename T>
__global__ void k_level_smooth(LevelDevT<T> L, int color, LevelDevT<T> C, int prolong) {
  int i, j, k;
  if (!level_pair(L, color, i, j, k) || i >= L.nx) return;
  long long c = lidx(L, i, j, k);
  T nb;
  if (prolong) {
    const int k2 = L.dim == 3 ? k : 0;
    nb = level_nbsum_f(L, i, j, k, [&](long long n, int di, int dj, int dk) {
      return L.z[n] + C.z[lidx(C, (i + di) >> 1, (j + dj) >> 1, (k2 + dk) >> 1)];
    });
  } else {
    nb = level_nbsum_f(L, i, j, k, [&](long long n, int, int, int) { return L.z[n]; });
  }
  L.z[c] = (L.r[c] + nb) / L.diag[c];
}

// Restriction of the fine residual onto level 1 (sum over the children) after
// the pre-smoothing sweep: black rows are satisfied exactly, and a red row's
// residual is r - D r D^-1 + sum_f c_f z_nb = sum_f c_f z_nb (its neighbours
// are black), so only the red children contribute, each by that sum.
// (z colour-split)
template <typename T>
__global__ void k_restrict_fine(Params P, FineOpT<T> O, const T* z, LevelDevT<T> C) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  int J = blockIdx.y * blockDim.y + threadIdx.y;
  int K = blockIdx.z;
  if (I >= C.nx || J >= C.ny) return;
  const int nzs = C.dim == 3 ? 2 : 1;
  T s = (T)0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < nzs; ++e) {
        if ((a + b + e) & 1) continue;  // black child (2I+a+2J+b+2K+e odd)
        int i = 2 * I + a, j = 2 * J + b, k = C.dim == 3 ? 2 * K + e : 0;
        long long c = cidx(P, i, j, k);
        Nbr N = make_nbr(P, i, j, k, c);
        T cf[6], zn[6];
        fine_row(P, O, N, c, cf);
#pragma unroll
        for (int q = 0; q < 6; ++q) zn[q] = z[nb_split(P, N, i, j, k, q)];
#pragma unroll
        for (int q = 0; q < 6; ++q) s = sel(is_bnd(N, q), s, s + cf[q] * zn[q]);
      }
  C.r[lidx(C, I, J, K)] = s;
}

// Restriction after further pre-smoothing sweeps (the V-cycle's nu > 1): the
// last half sweep was black, so black rows are satisfied and only the red
// children contribute, each by its full residual r - A z (r, z colour-split;
// the operator and its order of terms as fine_Ax).
template <typename T>
__global__ void k_restrict_fine_res(Params P, FineOpT<T> O, const T* r, const T* z, LevelDevT<T> C) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  int J = blockIdx.y * blockDim.y + threadIdx.y;
  int K = blockIdx.z;
  if (I >= C.nx || J >= C.ny) return;
  const int nzs = C.dim == 3 ? 2 : 1;
  T s = (T)0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < nzs; ++e) {
        if ((a + b + e) & 1) continue;  // black child
        int i = 2 * I + a, j = 2 * J + b, k = C.dim == 3 ? 2 * K + e : 0;
        long long c = cidx(P, i, j, k);
        Nbr N = make_nbr(P, i, j, k, c);
        T cf[6];
        fine_row(P, O, N, c, cf);
        const long long sp = rb_split(P, i, j, k);
        const T xc = z[sp];
        T xn[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) xn[q] = z[nb_split(P, N, i, j, k, q)];
        T Az = (T)0, dg = (T)0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const bool b = is_bnd(N, q);
          Az = sel(b, Az + cf[q] * xc, Az + cf[q] * (xc - xn[q]));
          dg += cf[q];
        }
        Az = sel(dg == (T)0, xc, Az);  // uncoupled row: identity
        s += r[sp] - Az;
      }
  C.r[lidx(C, I, J, K)] = s;
}

template <typename T>
__global__ void k_restrict_level_res(LevelDevT<T> F, LevelDevT<T> C) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  int J = blockIdx.y * blockDim.y + threadIdx.y;
  int K = blockIdx.z;
  if (I >= C.nx || J >= C.ny) return;
  int nzs = C.dim == 3 ? 2 : 1;
  T s = (T)0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < nzs; ++e) {
        if ((a + b + e) & 1) continue;
        int i = 2 * I + a, j = 2 * J + b, k = C.dim == 3 ? 2 * K + e : 0;
        const long long c = lidx(F, i, j, k);
        const T nb = level_nbsum_f(F, i, j, k, [&](long long n, int, int, int) { return F.z[n]; });
        s += F.r[c] - (F.diag[c] * F.z[c] - nb);
      }
  C.r[lidx(C, I, J, K)] = s;
}

// restriction after the pre-smoothing sweep of a stored level: the residual of
// a red row is sum_nb c z_nb (black rows are satisfied), summed over the red
// children of each coarse cell
template <typename T>
__global__ void k_restrict_level(LevelDevT<T> F, LevelDevT<T> C) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  int J = blockIdx.y * blockDim.y + threadIdx.y;
  int K = blockIdx.z;
  if (I >= C.nx || J >= C.ny) return;
  int nzs = C.dim == 3 ? 2 : 1;
  T s = (T)0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < nzs; ++e) {
        if ((a + b + e) & 1) continue;
        int i = 2 * I + a, j = 2 * J + b, k = C.dim == 3 ? 2 * K + e : 0;
        s += level_nbsum_f(F, i, j, k, [&](long long n, int, int, int) { return F.z[n]; });
      }
  C.r[lidx(C, I, J, K)] = s;
}

// ---------------------------------------------------------------- tail V-cycle
// The small coarse levels (each <= TAIL_MAX cells) are processed by one
// workgroup: pre-smoothing, restriction, the coarsest solve, prolongation and
// post-smoothing with barriers between the passes (one launch instead of ~5 per
// level).  Same arithmetic as the per-level kernels.  The coarsest solve is a
// symmetric red-black Gauss-Seidel from zero (m forward then m backward colour
// pairs).  Two variants: every level staged in LDS (the normal case), and a
// global-memory one for a coarsest level too large for LDS (grids whose
// coarsening stops early).
constexpr long long TAIL_MAX = 1024;
constexpr int TAIL_LDS = 1024;
constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_LDS_BYTES = 64 * 1024;  // the LDS tail keeps every tail level in LDS
template <typename T>
struct TailLevelsT {
  LevelDevT<T> L[MAX_LEVELS];
  int off[MAX_LEVELS];  // LDS tail: element offset of each level's block r, z, diag, cx, cy, cz
  int n;
};

template <typename T>
__device__ __forceinline__ void tail_smooth(const LevelDevT<T>& L, int color, int init) {
  for (long long c = threadIdx.x; c < L.N; c += TAIL_THREADS) {
    int i = (int)(c % L.nx), j = (int)((c / L.nx) % L.ny), k = (int)(c / ((long long)L.nx * L.ny));
    bool mine = ((i + j + k) & 1) == color;
    if (init && !mine) {
      L.z[c] = (T)0;
      continue;
    }
    if (!mine) continue;
    T nb = init ? (T)0 : level_nbsum(L, L.z, i, j, k);
    L.z[c] = (L.r[c] + nb) / L.diag[c];
  }
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(TAIL_THREADS) k_tail_vcycle_global(TailLevelsT<T> TL, int m, int nu) {
  int n = TL.n;
  for (int t = 0; t < n - 1; ++t) {
    const LevelDevT<T>& F = TL.L[t];
    const LevelDevT<T>& C = TL.L[t + 1];
    tail_smooth(F, 0, 1);
    tail_smooth(F, 1, 0);
    for (int s = 1; s < nu; ++s) {
      tail_smooth(F, 0, 0);
      tail_smooth(F, 1, 0);
    }
    int nzs = C.dim == 3 ? 2 : 1;
    for (long long q = threadIdx.x; q < C.N; q += TAIL_THREADS) {
      int I = (int)(q % C.nx), J = (int)((q / C.nx) % C.ny), K = (int)(q / ((long long)C.nx * C.ny));
      T sacc = (T)0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int e = 0; e < nzs; ++e) {
            int i = 2 * I + a, j = 2 * J + b, k = C.dim == 3 ? 2 * K + e : 0;
            long long c = lidx(F, i, j, k);
            T Az = F.diag[c] * F.z[c] - level_nbsum(F, F.z, i, j, k);
            sacc += F.r[c] - Az;
          }
      C.r[q] = sacc;
    }
    __syncthreads();
  }
  const LevelDevT<T>& L = TL.L[n - 1];
  if (L.N <= TAIL_LDS) {
    __shared__ T zs[TAIL_LDS], rs[TAIL_LDS], ds[TAIL_LDS];
    for (long long c = threadIdx.x; c < L.N; c += TAIL_THREADS) {
      zs[c] = (T)0;
      rs[c] = L.r[c];
      ds[c] = L.diag[c];
    }
    __syncthreads();
    for (int it = 0; it < 2 * m; ++it)
      for (int h = 0; h < 2; ++h) {
        int color = it < m ? h : 1 - h;
        for (long long c = threadIdx.x; c < L.N; c += TAIL_THREADS) {
          int i = (int)(c % L.nx), j = (int)((c / L.nx) % L.ny), k = (int)(c / ((long long)L.nx * L.ny));
          if (((i + j + k) & 1) != color) continue;
          zs[c] = (rs[c] + level_nbsum(L, (const T*)zs, i, j, k)) / ds[c];
        }
        __syncthreads();
      }
    for (long long c = threadIdx.x; c < L.N; c += TAIL_THREADS) L.z[c] = zs[c];
    __syncthreads();
  } else {
    for (long long c = threadIdx.x; c < L.N; c += TAIL_THREADS) L.z[c] = (T)0;
    __syncthreads();
    for (int it = 0; it < 2 * m; ++it)
      for (int h = 0; h < 2; ++h) tail_smooth(L, it < m ? h : 1 - h, 0);
  }
  for (int t = n - 2; t >= 0; --t) {
    const LevelDevT<T>& F = TL.L[t];
    const LevelDevT<T>& C = TL.L[t + 1];
    for (long long c = threadIdx.x; c < F.N; c += TAIL_THREADS) {
      int i = (int)(c % F.nx), j = (int)((c / F.nx) % F.ny), k = (int)(c / ((long long)F.nx * F.ny));
      F.z[c] += C.z[lidx(C, i / 2, j / 2, F.dim == 3 ? k / 2 : 0)];
    }
    __syncthreads();
    for (int s = 0; s < nu; ++s) {
      tail_smooth(F, 1, 0);
      tail_smooth(F, 0, 0);
    }
  }
}

// LDS tail: every tail level (r, z, diag, cx, cy, cz) staged in dynamic LDS,
// 32-bit indices; the top level's r comes from the restriction above, its z
// goes back to global memory for the prolongation.
template <typename T>
struct LdsLev {
  int nx, ny, nz, dim, N;
  float inx, iny;  // 1/nx, 1/ny for split3
  T *r, *z, *diag, *cx, *cy, *cz;
};
// (i, j, k) of the flat index c of an nx x ny x nz block without integer
// division: (c + 0.5) / nx lies at least 0.5 / nx from an integer and the float
// product is accurate to ~1e-7 relative, so the floor is exact for c < 2^20
__device__ __forceinline__ void split3(int c, int nx, int ny, float inx, float iny, int& i, int& j, int& k) {
  const int jk = (int)(((float)c + 0.5f) * inx);
  i = c - jk * nx;
  k = (int)(((float)jk + 0.5f) * iny);
  j = jk - k * ny;
}
template <typename T>
__device__ __forceinline__ LdsLev<T> lds_lev(const TailLevelsT<T>& TL, int t, T* base) {
  const LevelDevT<T>& L = TL.L[t];
  LdsLev<T> v;
  v.nx = L.nx;
  v.ny = L.ny;
  v.nz = L.nz;
  v.dim = L.dim;
  v.N = (int)L.N;
  v.inx = 1.0f / (float)L.nx;
  v.iny = 1.0f / (float)L.ny;
  T* p = base + TL.off[t];
  v.r = p;
  v.z = p + v.N;
  v.diag = p + 2 * v.N;
  v.cx = p + 3 * v.N;
  v.cy = v.cx + (v.nx + 1) * v.ny * v.nz;
  v.cz = v.cy + v.nx * (v.ny + 1) * v.nz;
  return v;
}
template <typename T>
__device__ __forceinline__ T lds_nbsum(const LdsLev<T>& L, const T* z, int i, int j, int k) {
  // the x and y terms from clamped LDS reads issued together, dropped by selects
  // on the domain boundary (a 2-D level stages no z coefficients: its z block
  // is skipped as a whole)
  const int c = i + L.nx * (j + L.ny * k);
  const bool xm = i > 0, xp = i < L.nx - 1, ym = j > 0, yp = j < L.ny - 1;
  const T axm = L.cx[i + (L.nx + 1) * (j + L.ny * k)], axp = L.cx[i + 1 + (L.nx + 1) * (j + L.ny * k)];
  const T aym = L.cy[i + L.nx * (j + (L.ny + 1) * k)], ayp = L.cy[i + L.nx * (j + 1 + (L.ny + 1) * k)];
  const T zxm = z[xm ? c - 1 : c], zxp = z[xp ? c + 1 : c], zym = z[ym ? c - L.nx : c], zyp = z[yp ? c + L.nx : c];
  T s = (T)0;
  s = sel(xm, s + axm * zxm, s);
  s = sel(xp, s + axp * zxp, s);
  s = sel(ym, s + aym * zym, s);
  s = sel(yp, s + ayp * zyp, s);
  if (L.dim == 3) {
    const int sz = L.nx * L.ny;
    const bool zm = k > 0, zp = k < L.nz - 1;
    const T azm = L.cz[i + L.nx * (j + L.ny * k)], azp = L.cz[i + L.nx * (j + L.ny * (k + 1))];
    const T zzm = z[zm ? c - sz : c], zzp = z[zp ? c + sz : c];
    s = sel(zm, s + azm * zzm, s);
    s = sel(zp, s + azp * zzp, s);
  }
  return s;
}
template <typename T>
__device__ __forceinline__ void lds_smooth(const LdsLev<T>& L, int color, int init) {
  for (int c = threadIdx.x; c < L.N; c += TAIL_THREADS) {
    int i, j, k;
    split3(c, L.nx, L.ny, L.inx, L.iny, i, j, k);
    bool mine = ((i + j + k) & 1) == color;
    if (init && !mine) {
      L.z[c] = (T)0;
      continue;
    }
    if (!mine) continue;
    T nb = init ? (T)0 : lds_nbsum(L, (const T*)L.z, i, j, k);
    L.z[c] = (L.r[c] + nb) / L.diag[c];
  }
  __syncthreads();
}
template <typename T>
__device__ __forceinline__ void lds_copy(T* dst, const T* src, int n) {
  for (int q = threadIdx.x; q < n; q += TAIL_THREADS) dst[q] = src[q];
}

template <typename T>
__global__ void __launch_bounds__(TAIL_THREADS) k_tail_vcycle(TailLevelsT<T> TL, int m, int nu) {
  extern __shared__ unsigned char tail_lds_raw[];
  T* base = reinterpret_cast<T*>(tail_lds_raw);
  const int n = TL.n;
  // staging: per level, every thread issues all its loads (two elements of each
  // array; tail levels have at most TAIL_MAX cells, so their arrays fit in
  // 2 TAIL_THREADS elements, the loop after covers any rest) before its first LDS
  // store, so the level arrives in one memory round trip
  for (int t = 0; t < n; ++t) {
    const LevelDevT<T>& G = TL.L[t];
    LdsLev<T> L = lds_lev(TL, t, base);
    const int nr = t == 0 ? L.N : 0;
    const int nfx = (L.nx + 1) * L.ny * L.nz, nfy = L.nx * (L.ny + 1) * L.nz;
    const int nfz = L.dim == 3 ? L.nx * L.ny * (L.nz + 1) : 0;
    T v[2][5];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = (int)threadIdx.x + h * TAIL_THREADS;
      v[h][0] = q < nr ? G.r[q] : (T)0;
      v[h][1] = q < L.N ? G.diag[q] : (T)0;
      v[h][2] = q < nfx ? G.cx[q] : (T)0;
      v[h][3] = q < nfy ? G.cy[q] : (T)0;
      v[h][4] = q < nfz ? G.cz[q] : (T)0;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = (int)threadIdx.x + h * TAIL_THREADS;
      if (q < nr) L.r[q] = v[h][0];
      if (q < L.N) L.diag[q] = v[h][1];
      if (q < nfx) L.cx[q] = v[h][2];
      if (q < nfy) L.cy[q] = v[h][3];
      if (q < nfz) L.cz[q] = v[h][4];
    }
    for (int q = (int)threadIdx.x + 2 * TAIL_THREADS; q < nfx || q < nfy || q < nfz || q < L.N; q += TAIL_THREADS) {
      if (q < nr) L.r[q] = G.r[q];
      if (q < L.N) L.diag[q] = G.diag[q];
      if (q < nfx) L.cx[q] = G.cx[q];
      if (q < nfy) L.cy[q] = G.cy[q];
      if (q < nfz) L.cz[q] = G.cz[q];
    }
  }
  __syncthreads();
  for (int t = 0; t < n - 1; ++t) {
    LdsLev<T> F = lds_lev(TL, t, base), C = lds_lev(TL, t + 1, base);
    lds_smooth(F, 0, 1);
    lds_smooth(F, 1, 0);
    for (int s = 1; s < nu; ++s) {
      lds_smooth(F, 0, 0);
      lds_smooth(F, 1, 0);
    }
    int nzs = C.dim == 3 ? 2 : 1;
    for (int q = threadIdx.x; q < C.N; q += TAIL_THREADS) {
      int I, J, K;
      split3(q, C.nx, C.ny, C.inx, C.iny, I, J, K);
      T sacc = (T)0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int e = 0; e < nzs; ++e) {
            int i = 2 * I + a, j = 2 * J + b, k = C.dim == 3 ? 2 * K + e : 0;
            int c = i + F.nx * (j + F.ny * k);
            T Az = F.diag[c] * F.z[c] - lds_nbsum(F, (const T*)F.z, i, j, k);
            sacc += F.r[c] - Az;
          }
      C.r[q] = sacc;
    }
    __syncthreads();
  }
  {
    LdsLev<T> L = lds_lev(TL, n - 1, base);
    for (int c = threadIdx.x; c < L.N; c += TAIL_THREADS) L.z[c] = (T)0;
    __syncthreads();
    for (int it = 0; it < 2 * m; ++it)
      for (int h = 0; h < 2; ++h) lds_smooth(L, it < m ? h : 1 - h, 0);
  }
  for (int t = n - 2; t >= 0; --t) {
    LdsLev<T> F = lds_lev(TL, t, base), C = lds_lev(TL, t + 1, base);
    for (int c = threadIdx.x; c < F.N; c += TAIL_THREADS) {
      int i, j, k;
      split3(c, F.nx, F.ny, F.inx, F.iny, i, j, k);
      F.z[c] += C.z[(i / 2) + C.nx * ((j / 2) + C.ny * (F.dim == 3 ? k / 2 : 0))];
    }
    __syncthreads();
    for (int s = 0; s < nu; ++s) {
      lds_smooth(F, 1, 0);
      lds_smooth(F, 0, 0);
    }
  }
  LdsLev<T> L0 = lds_lev(TL, 0, base);
  for (int c = threadIdx.x; c < L0.N; c += TAIL_THREADS) TL.L[0].z[c] = L0.z[c];
}

// ---------------------------------------------------------------- vector ops


// x += alpha d, r -= alpha q (and its FP32 copy when r32 is given); partial r.r
__global__ void k_axpy2(long long n, const double* scal, double* x, const double* d, double* r, float* r32,
                        const double* q, double* part, long long pstride) {
  long long c = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  double a = scal[S_ALPHA];
  double v[1] = {0.0};
  if (c < n) {
    x[c] += a * d[c];
    double rc = r[c] - a * q[c];
    r[c] = rc;
    if (r32) r32[c] = (float)rc;
    v[0] = rc * rc;
  }
  block_sums_store<1>(v, part, pstride, blockIdx.x);
}


// first stage of a large reduction: workgroup (b, v) reduces entries
// [b chunk, (b+1) chunk) of partial row v (sum, or max when is_max) into
// out[v * FIN2_STRIDE + b]
constexpr int RED_THREADS = 256;
constexpr int FIN2_CHUNKS = 512;
__global__ void __launch_bounds__(RED_THREADS)
k_reduce_chunks(const double* part, long long pstride, int nblk, int chunk, int is_max, double* out) {
  __shared__ double lds[RED_THREADS / 64];
  const double* row = part + (long long)blockIdx.y * pstride;
  int b0 = blockIdx.x * chunk;
  int b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  double s = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += RED_THREADS) s = is_max ? fmax(s, row[b]) : s + row[b];
  s = is_max ? wave_max(s) : wave_sum(s);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = lds[0];
    for (int w = 1; w < RED_THREADS / 64; ++w) t = is_max ? fmax(t, lds[w]) : t + lds[w];
    out[(long long)blockIdx.y * FIN2_STRIDE + blockIdx.x] = t;
  }
}

// finalize: reduces `nval` rows of per-block partials -> scal[out+v] (sums, or
// maxima for op 4), then an optional PCG scalar update (only with one row).
// Workgroup v of 1024 threads reduces row v; thread t takes entries t, t+1024,
// ... in that order (loads issued eight at a time, summed in the same order),
// then the waves and the workgroup in fixed order: deterministic, and the
// result does not depend on how many rows are reduced together.
// op: 0 none, 1 alpha = rho / dq, 2 beta = rz / rho, rho = rz, 3 rho = value, 4 max
constexpr int FIN_THREADS = 1024;
constexpr int FIN_BATCH = 8;
__global__ void __launch_bounds__(FIN_THREADS)
k_finalize(const double* part, long long pstride, int nblk, double* scal, int out, int op, double divisor,
           double* hmir, double seq) {
  __shared__ double lds[FIN_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, v = blockIdx.x;
  const double* row = part + (long long)v * pstride;
  const bool mx = op == 4;
  double s = 0.0;
  int b = tid;
  for (; b + (FIN_BATCH - 1) * FIN_THREADS < nblk; b += FIN_BATCH * FIN_THREADS) {
    double e[FIN_BATCH];
#pragma unroll
    for (int q = 0; q < FIN_BATCH; ++q) e[q] = row[b + q * FIN_THREADS];
#pragma unroll
    for (int q = 0; q < FIN_BATCH; ++q) s = mx ? fmax(s, e[q]) : s + e[q];
  }
  for (; b < nblk; b += FIN_THREADS) s = mx ? fmax(s, row[b]) : s + row[b];
  s = mx ? wave_max(s) : wave_sum(s);
  if (lane == 0) lds[wid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = lds[0];
    for (int w = 1; w < FIN_THREADS / 64; ++w) t = mx ? fmax(t, lds[w]) : t + lds[w];
    scal[out + v] = divisor == 1.0 ? t : t / divisor;
    if (op == 1) {
      scal[S_ALPHA] = t != 0.0 ? scal[S_RHO] / t : 0.0;
    } else if (op == 2) {
      scal[S_BETA] = scal[S_RHO] != 0.0 ? t / scal[S_RHO] : 0.0;
      scal[S_RHO] = t;
    } else if (op == 3) {
      scal[S_RHO] = t;
    }
    if (hmir) {
      // the scalars, then (once they are visible to the host) the sequence
      // number the host waits for
      for (int q = 0; q < NMIR; ++q) hmir[q] = scal[q];
      __threadfence_system();
      *(volatile double*)(hmir + NMIR) = seq;
      __threadfence_system();
    }
  }
}

// ---------------------------------------------------------------- host side
template <typename T>
struct LevelPick;
template <>
struct LevelPick<double> {
  static LevelDevT<double> get(hfdib_ctx* c, int l) {
    Level& L = c->lev[l];
    return LevelDevT<double>{L.nx, L.ny, L.nz, c->P.dim, L.N, L.r, L.z, L.cx, L.cy, L.cz, L.diag};
  }
};
template <>
struct LevelPick<float> {
  static LevelDevT<float> get(hfdib_ctx* c, int l) {
    Level& L = c->lev[l];
    return LevelDevT<float>{L.nx, L.ny, L.nz, c->P.dim, L.N, L.r32, L.z32, L.cx32, L.cy32, L.cz32, L.diag32};
  }
};
template <typename T>
static LevelDevT<T> levdev(hfdib_ctx* c, int l) {
  return LevelPick<T>::get(c, l);
}
static dim3 lgrid(int nx, int ny, int nz) { return dim3((nx + 63) / 64, (ny + 3) / 4, nz); }
// pair-mapped grid of a stored level (half the x extent)
static dim3 lgrid_rb(int nx, int ny, int nz) { return dim3(((nx + 1) / 2 + 63) / 64, (ny + 3) / 4, nz); }

// finalize helper; partial slots live in ctx->partials with row stride c->pstride
// Large partial rows are first reduced in fixed chunks by many workgroups
// (deterministic: fixed chunk boundaries and order), then by one workgroup.
void launch_finalize(hfdib_ctx* c, int nblk, int nval, int out, int op, double divisor, int row0, double* hmir,
                     double seq) {
  const double* part = c->partials + (long long)row0 * c->pstride;
  if (nblk > 32 * FIN_THREADS) {
    int chunk = (nblk + FIN2_CHUNKS - 1) / FIN2_CHUNKS;
    int nchunks = (nblk + chunk - 1) / chunk;
    LaunchEv e0 = timer_launch(c, T_FINALIZE, true, false, 2);
    launch_ev(k_reduce_chunks, dim3(nchunks, nval), dim3(RED_THREADS), c->stream, e0, part, c->pstride, nblk, chunk,
              op == 4 ? 1 : 0, c->partials2);
    LaunchEv e1 = timer_launch(c, T_FINALIZE, false, true, 2);
    launch_ev(k_finalize, dim3(nval), dim3(FIN_THREADS), c->stream, e1, (const double*)c->partials2,
              (long long)FIN2_STRIDE, nchunks, c->scal + SCAL_PCG, out, op, divisor, hmir, seq);
    return;
  }
  LaunchEv ev = timer_launch(c, T_FINALIZE, true, true);
  launch_ev(k_finalize, dim3(nval), dim3(FIN_THREADS), c->stream, ev, part, c->pstride, nblk, c->scal + SCAL_PCG, out,
            op, divisor, hmir, seq);
}

// the colour-split work vectors of the V-cycle's fine level (z and r) in
// storage type T
template <typename T>
struct SplitBuf {
  T* z;
  T* r;
};
template <typename T>
static SplitBuf<T> split_buf(hfdib_ctx* c);
template <>
SplitBuf<double> split_buf<double>(hfdib_ctx* c) {
  return SplitBuf<double>{c->pzs, c->prs};
}
template <>
SplitBuf<float> split_buf<float>(hfdib_ctx* c) {
  return SplitBuf<float>{c->pzs32, c->prs32};
}

// the first pass of a V-cycle: fine-level pre-smoothing of z from zero (it
// writes only the colour-split z and r of the V-cycle)
template <typename T>
static void vcycle_presmooth(hfdib_ctx* c, const FineOpT<T>& O, const T* invD, const T* r) {
  const Params& P = c->P;
  const SplitBuf<T> S = split_buf<T>(c);
  LaunchEv ev = timer_launch(c, T_PPRESMOOTH, true, true);
  launch_ev(k_fine_presmooth<T>, grid3_rb(P), block3(P), c->stream, ev, P, O, invD, r, S.z, S.r);
}

// one fine-level half sweep of the V-cycle (timed as its own class), on the
// colour-split vectors; with rdot (the last one) it also writes z to zout
template <typename T>
static void fine_smooth(hfdib_ctx* c, const FineOpT<T>& O, const T* invD, int color, const T* zc, int cnx, int cny,
                        const double* rdot, double* part, long long pstride, double* dcopy, T* zout) {
  const Params& P = c->P;
  const SplitBuf<T> S = split_buf<T>(c);
  LaunchEv ev = timer_launch(c, T_PSMOOTH, true, true);
  launch_ev(k_fine_smooth<T>, grid3_rb(P), block3(P), c->stream, ev, P, O, invD, (const T*)S.r, S.z, color, zc, cnx,
            cny, rdot, part, pstride, dcopy, zout);
}

// one V-cycle z = M^-1 r in storage type T; the last sweep also leaves the
// block partial sums of rdot . z in the partials (rdot: the FP64 residual) and,
// with dcopy, writes z to that FP64 vector as well; returns the partial count.
// presmoothed: the first pass (vcycle_presmooth) is already enqueued.
template <typename T>
static int vcycle(hfdib_ctx* c, const FineOpT<T>& O, const T* invD, const T* r, T* z, const double* rdot,
                  double* dcopy = nullptr, bool presmoothed = false) {
  const Params& P = c->P;
  const int nu = P.p_nu, nuc = P.p_nu_c;  // sweeps per side on the fine level and on the coarse levels
  dim3 g = grid3_rb(P), b = block_lv();
  const SplitBuf<T> S = split_buf<T>(c);
  if (!presmoothed) vcycle_presmooth<T>(c, O, invD, r);
  // further pre-smoothing sweeps (red, then black)
  for (int s = 1; s < nu; ++s)
    for (int color = 0; color < 2; ++color)
      fine_smooth<T>(c, O, invD, color, (const T*)nullptr, 0, 0, (const double*)nullptr, (double*)nullptr, 0LL,
                     (double*)nullptr, (T*)nullptr);
  const T* zc = nullptr;
  int cnx = 0, cny = 0;
  if (c->nlev > 1) {
    LevelDevT<T> L1 = levdev<T>(c, 1);
    LaunchEv er = timer_launch(c, T_PRESTRICT, true, true);
    if (nu == 1)
      launch_ev(k_restrict_fine<T>, lgrid(L1.nx, L1.ny, L1.nz), b, c->stream, er, P, O, (const T*)S.z, L1);
    else
      launch_ev(k_restrict_fine_res<T>, lgrid(L1.nx, L1.ny, L1.nz), b, c->stream, er, P, O, (const T*)S.r,
                (const T*)S.z, L1);
    // the coarse levels are timed as one span: opened by their first launch,
    // closed by the last
    bool opened = false;
    auto cev = [&](bool last) {
      LaunchEv e = timer_launch(c, T_PCOARSE, !opened, last);
      opened = true;
      return e;
    };
    // large coarse levels: one kernel per pass
    int l = 1;
    while (l < c->nlev - 1 && c->lev[l].N > TAIL_MAX) {
      LevelDevT<T> L = levdev<T>(c, l);
      dim3 gr = lgrid_rb(L.nx, L.ny, L.nz);
      launch_ev(k_level_presmooth<T>, gr, b, c->stream, cev(false), L);
      for (int s = 1; s < nuc; ++s)
        for (int color = 0; color < 2; ++color)
          hipLaunchKernelGGL(k_level_smooth<T>, gr, b, 0, c->stream, L, color, L, 0);
      LevelDevT<T> C = levdev<T>(c, l + 1);
      if (nuc == 1)
        hipLaunchKernelGGL(k_restrict_level<T>, lgrid(C.nx, C.ny, C.nz), b, 0, c->stream, L, C);
      else
        hipLaunchKernelGGL(k_restrict_level_res<T>, lgrid(C.nx, C.ny, C.nz), b, 0, c->stream, L, C);
      ++l;
    }
    // small levels l..nlev-1 (and the coarsest solve) in one workgroup, staged
    // in LDS when they fit
    TailLevelsT<T> TL;
    TL.n = c->nlev - l;
    long long elems = 0;
    for (int t = 0; t < TL.n; ++t) {
      TL.L[t] = levdev<T>(c, l + t);
      const LevelDevT<T>& L = TL.L[t];
      TL.off[t] = (int)elems;
      elems += 3 * L.N + (long long)(L.nx + 1) * L.ny * L.nz + (long long)L.nx * (L.ny + 1) * L.nz +
               (L.dim == 3 ? (long long)L.nx * L.ny * (L.nz + 1) : 0);
    }
    size_t lds = (size_t)elems * sizeof(T);
    {
      const bool tail_last = l == 1;
      LaunchEv et = cev(tail_last);
      if (lds <= (size_t)TAIL_LDS_BYTES) {
        if (et.start || et.stop)
          hipExtLaunchKernelGGL(k_tail_vcycle<T>, dim3(1), dim3(TAIL_THREADS), lds, c->stream, et.start, et.stop, 0,
                                TL, 6, nuc);
        else
          hipLaunchKernelGGL(k_tail_vcycle<T>, dim3(1), dim3(TAIL_THREADS), lds, c->stream, TL, 6, nuc);
      } else {
        launch_ev(k_tail_vcycle_global<T>, dim3(1), dim3(TAIL_THREADS), c->stream, et, TL, 6, nuc);
      }
    }
    for (int q = l - 1; q >= 1; --q) {
      LevelDevT<T> L = levdev<T>(c, q);
      LevelDevT<T> C = levdev<T>(c, q + 1);
      dim3 gr = lgrid_rb(L.nx, L.ny, L.nz);
      for (int s = 0; s < nuc; ++s) {
        hipLaunchKernelGGL(k_level_smooth<T>, gr, b, 0, c->stream, L, 1, C, s == 0 ? 1 : 0);
        launch_ev(k_level_smooth<T>, gr, b, c->stream, cev(q == 1 && s == nuc - 1), L, 0, C, 0);
      }
    }
    zc = L1.z;
    cnx = L1.nx;
    cny = L1.ny;
  }
  // post-smoothing sweeps, black first (the first one with the prolongation on
  // the fly), then red; the last red half sweep also forms the r . z partials
  for (int s = 0; s < nu; ++s) {
    const bool last = s == nu - 1;
    fine_smooth<T>(c, O, invD, 1, s == 0 ? zc : (const T*)nullptr, cnx, cny, (const double*)nullptr,
                   (double*)nullptr, 0LL, (double*)nullptr, (T*)nullptr);
    fine_smooth<T>(c, O, invD, 0, (const T*)nullptr, 0, 0, last ? rdot : (const double*)nullptr,
                   last ? c->partials : (double*)nullptr, last ? c->pstride : 0LL, last ? dcopy : (double*)nullptr,
                   z);
  }
  return (int)g.x;
}

// coarse operators of every level from the FP64 fine operator
template <typename T>
static void build_levels(hfdib_ctx* c, const FineOp& O) {
  const Params& P = c->P;
  dim3 b = block_lv();
  for (int l = 1; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    LevelDevT<T> Ld = levdev<T>(c, l);
    T* cx = const_cast<T*>(Ld.cx);
    T* cy = const_cast<T*>(Ld.cy);
    T* cz = const_cast<T*>(Ld.cz);
    T* dg = const_cast<T*>(Ld.diag);
    if (l == 1)
      hipLaunchKernelGGL((k_coarsen_diag<T, true>), lgrid(L.nx, L.ny, L.nz), b, 0, c->stream, P, O, Ld, Ld, cx, cy, cz,
                         dg);
    else
      hipLaunchKernelGGL((k_coarsen_diag<T, false>), lgrid(L.nx, L.ny, L.nz), b, 0, c->stream, P, O,
                         levdev<T>(c, l - 1), Ld, cx, cy, cz, dg);
  }
}

// Preconditioned CG on the pressure system.  The preconditioner storage type
// is T (FP64; FP32 under the mixed policy, where r32/z32 hold the FP32 copies
// of the residual and of the preconditioned residual).
template <typename T>
struct PcgSet {
  FineOp O;         // FP64 fine operator (residual, operator apply)
  FineOpT<T> OM;    // fine operator of the preconditioner
  const T* invD;    // its inverse diagonal
  T* r_m;           // preconditioner input (the residual, or its FP32 copy)
  T* z_m;           // preconditioner output
  float* r32;       // FP32 copy of the residual (mixed policy) or null
};
template <typename T>
static PcgSet<T> pcg_set(hfdib_ctx* c, const double* rAU);
template <>
PcgSet<double> pcg_set<double>(hfdib_ctx* c, const double* rAU) {
  return PcgSet<double>{FineOp{rAU, c->flags}, FineOp{rAU, c->flags}, c->invD, c->pr, c->pz, nullptr};
}
template <>
PcgSet<float> pcg_set<float>(hfdib_ctx* c, const double* rAU) {
  return PcgSet<float>{FineOp{rAU, c->flags}, FineOpT<float>{c->rAU32, c->flags}, c->invD32, c->pr32, c->pz32,
                       c->pr32};
}

// the coarse operators from the FP64 fine operator (the fine smoother's
// inverse diagonal comes with the initial residual)
template <typename T>
static void pcg_operators(hfdib_ctx* c, const PcgSet<T>& A) {
  build_levels<T>(c, A.O);
}

// r = b - A x, |b| and the SIMPLE residual sums, then d = z = M^-1 r
template <typename T>
static void pcg_start(hfdib_ctx* c, const PcgSet<T>& A, const double* rhs, double* x, const double* xmean_dev) {
  const Params& P = c->P;
  dim3 g = grid3(P), b = block3(P);
  const bool f32 = sizeof(T) == sizeof(float);
  hipLaunchKernelGGL(k_fine_residual, g, b, 0, c->stream, P, A.O, rhs, x, c->pr, A.r32, xmean_dev, c->partials,
                     c->pstride, f32 ? (double*)nullptr : (double*)A.invD, f32 ? (float*)A.invD : (float*)nullptr,
                     f32 ? c->rAU32 : (float*)nullptr);
  // [20] = rr0, [21] = bb, [22..24] = residual sums
  launch_finalize(c, (int)((long long)g.x * g.y * g.z), 5, S_BB + 16, 0);
  launch_finalize(c, vcycle<T>(c, A.OM, A.invD, A.r_m, A.z_m, c->pr, c->pd), 1, S_RZ, 3);  // d = z
}

// one CG step: q = A d, alpha, x += alpha d, r -= alpha q, r.r (the reduction of
// r.r also copies the PCG scalars to the pinned host mirror hmir when given)
// (dir: the direction update d = z + beta d is fused into the operator apply,
// which writes the new d to the other direction buffer; the buffers then swap)
template <typename T>
static void pcg_step(hfdib_ctx* c, const PcgSet<T>& A, double* x, double* hmir, bool dir = false) {
  const Params& P = c->P;
  dim3 g = grid3(P), b = block3(P);
  const int nb1 = nblocks1(P.N);
  double* S = c->scal + SCAL_PCG;
  if (dir) {
    LaunchEv ed = timer_launch(c, T_PAPPLYDIR, true, true);
    launch_ev(k_fine_apply_dir<T>, g, b, c->stream, ed, P, A.O, (const T*)A.z_m, (const double*)c->pd, c->pd2, c->pq,
              (const double*)S, c->partials, c->pstride);
    std::swap(c->pd, c->pd2);
  } else {
    // (the timed class of the operator apply is this plain launch)
    LaunchEv ev = timer_launch(c, T_PAPPLY, true, true);
    launch_ev(k_fine_apply, g, b, c->stream, ev, P, A.O, (const double*)c->pd, c->pq, c->partials, c->pstride);
  }
  launch_finalize(c, (int)((long long)g.x * g.y * g.z), 1, S_DQ, 1);
  LaunchEv ea = timer_launch(c, T_PAXPY, true, true);
  launch_ev(k_axpy2, dim3(nb1), dim3(NTHREADS), c->stream, ea, P.N, (const double*)S, x, (const double*)c->pd, c->pr,
            A.r32, (const double*)c->pq, c->partials, c->pstride);
  launch_finalize(c, nb1, 1, S_RR, 0, 1.0, 0, hmir, hmir ? (double)++c->mir_seq : 0.0);
}

// z = M^-1 r, beta = r.z / rho (the direction update d = z + beta d is done by
// the next CG step's operator apply)
template <typename T>
static void pcg_direction(hfdib_ctx* c, const PcgSet<T>& A, bool presmoothed = false) {
  launch_finalize(c, vcycle<T>(c, A.OM, A.invD, A.r_m, A.z_m, c->pr, nullptr, presmoothed), 1, S_RZ, 2);
}

// The adaptive solve in the pieces between which the host reads the
// convergence scalars: the set-up with the first CG step, and each further
// step (both end with the reduction that writes the pinned host mirror).
// While the host waits for a step's scalars the first pass of the next
// V-cycle is already queued (it only writes the preconditioner output z, so it
// is harmless when the solve has converged): the device does not idle for the
// host's round trip.  It is left out at the step where the previous solve
// converged (consecutive solves mostly take the same number of steps, and a
// pass queued after a converged step is thrown away); values are the same
// either way.
template <typename T>
static void pcg_begin_t(hfdib_ctx* c, const double* rAU, const double* rhs, double* x, const double* xmean_dev) {
  PcgSet<T> A = pcg_set<T>(c, rAU);
  pcg_operators<T>(c, A);
  pcg_start<T>(c, A, rhs, x, xmean_dev);
  pcg_step<T>(c, A, x, c->hmir_dev);
}
template <typename T>
static void pcg_ahead_t(hfdib_ctx* c, const double* rAU) {
  PcgSet<T> A = pcg_set<T>(c, rAU);
  vcycle_presmooth<T>(c, A.OM, A.invD, A.r_m);
}
template <typename T>
static void pcg_continue_t(hfdib_ctx* c, const double* rAU, double* x, bool presmoothed) {
  PcgSet<T> A = pcg_set<T>(c, rAU);
  pcg_direction<T>(c, A, presmoothed);
  pcg_step<T>(c, A, x, c->hmir_dev, true);
}
static void pcg_begin(hfdib_ctx* c, const double* rAU, const double* rhs, double* x, const double* xmean_dev) {
  if (c->P.precision == HFDIB_MIXED)
    pcg_begin_t<float>(c, rAU, rhs, x, xmean_dev);
  else
    pcg_begin_t<double>(c, rAU, rhs, x, xmean_dev);
}
static void pcg_ahead(hfdib_ctx* c, const double* rAU) {
  if (c->P.precision == HFDIB_MIXED)
    pcg_ahead_t<float>(c, rAU);
  else
    pcg_ahead_t<double>(c, rAU);
}
static void pcg_continue(hfdib_ctx* c, const double* rAU, double* x, bool presmoothed) {
  if (c->P.precision == HFDIB_MIXED)
    pcg_continue_t<float>(c, rAU, x, presmoothed);
  else
    pcg_continue_t<double>(c, rAU, x, presmoothed);
}

// Waits until the host mirror holds the scalars of the last CG step: spins on
// its sequence number (the device writes it after the scalars), checking the
// stream now and then so that a device error ends the wait.
static int wait_mirror(hfdib_ctx* c) {
  volatile const double* m = c->hmir;
  const double want = (double)c->mir_seq;
  for (unsigned long n = 1; m[NMIR] != want; ++n) {
    if ((n & 255) == 0) {
      hipError_t e = hipStreamQuery(c->stream);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return set_hip_error(c, e, "pcg wait");
      if (m[NMIR] == want) break;
      c->err = "pcg wait: the stream is idle but the scalars of the last step did not arrive";
      return HFDIB_EDEVICE;
    }
  }
  return HFDIB_OK;
}

// fixed iteration count, no host read (the step may be captured in a graph);
// the scalar updates guard zero denominators on the device
template <typename T>
static void pcg_fixed(hfdib_ctx* c, const double* rAU, const double* rhs, double* x, const double* xmean_dev,
                      int nit) {
  PcgSet<T> A = pcg_set<T>(c, rAU);
  pcg_operators<T>(c, A);
  pcg_start<T>(c, A, rhs, x, xmean_dev);
  for (int it = 1; it <= nit; ++it) {
    pcg_step<T>(c, A, x, nullptr, it > 1);
    if (it == nit) break;
    pcg_direction<T>(c, A);
  }
}

void pressure_apply_bench(hfdib_ctx* c) {
  const Params& P = c->P;
  FineOp O{c->rAU, c->flags};
  hipLaunchKernelGGL(k_fine_apply, grid3(P), block3(P), 0, c->stream, P, O, (const double*)c->pd, c->pq, c->partials,
                     c->pstride);
}

int pressure_solve(hfdib_ctx* c, const double* rAU, const double* rhs, double* x, double rtol, int maxit, int* iters,
                   double* relres, const double* xmean_dev) {
  const Params& P = c->P;
  timer_begin(c, T_PSOLVE);
  if (c->graph_mode) {
    if (P.precision == HFDIB_MIXED)
      pcg_fixed<float>(c, rAU, rhs, x, xmean_dev, c->graph_pcg);
    else
      pcg_fixed<double>(c, rAU, rhs, x, xmean_dev, c->graph_pcg);
    HFDIB_CHECK_LAUNCH(c, "pcg (fixed)");
    timer_end(c, T_PSOLVE);
    if (iters) *iters = c->graph_pcg;
    if (relres) *relres = 0.0;
    return HFDIB_OK;
  }
  if (!c->hmir) {
    // host-coherent pinned mirror of the PCG scalars, allocated on first use
    void *hm = nullptr, *hm_dev = nullptr;
    HFDIB_CHECK(c, hipHostMalloc(&hm, (NMIR + 1) * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent),
                "pinned scalar mirror");
    hipError_t e = hipHostGetDevicePointer(&hm_dev, hm, 0);
    if (e != hipSuccess) {
      (void)hipHostFree(hm);
      return set_hip_error(c, e, "pinned scalar mirror");
    }
    c->hmir = (double*)hm;
    c->hmir_dev = (double*)hm_dev;
    c->hmir[NMIR] = 0.0;
    c->mir_seq = 0;
  }
  // at least one CG step is done; the host reads the residual after each step
  // (one synchronisation per step, none before the first)
  double rr = 0.0, bnorm = 1.0, target = 0.0;
  int it;
  pcg_begin(c, rAU, rhs, x, xmean_dev);
  HFDIB_CHECK_LAUNCH(c, "pcg set-up");
  for (it = 1; it <= maxit; ++it) {
    const bool ahead = it < maxit && it != c->pcg_prev_iters;
    if (ahead) pcg_ahead(c, rAU);
    HFDIB_CHECK_LAUNCH(c, "pcg look-ahead");
    int st = wait_mirror(c);
    if (st != HFDIB_OK) return st;
    const volatile double* hs = c->hmir;
    if (it == 1) {
      double bb = hs[S_BB + 17];
      bnorm = sqrt(bb) > 0.0 ? sqrt(bb) : 1.0;
      target = rtol * bnorm;
      c->last_pres[0] = hs[22];
      c->last_pres[1] = hs[23];
      c->last_pres[2] = hs[24];
    }
    rr = hs[S_RR];
    if (!std::isfinite(rr)) {
      c->err = "non-finite residual in the pressure solve";
      return HFDIB_EDIVERGED;
    }
    if (sqrt(rr) <= target || it == maxit) break;
    pcg_continue(c, rAU, x, ahead);
    HFDIB_CHECK_LAUNCH(c, "pcg iteration");
  }
  if (it > maxit) it = maxit;
  c->pcg_prev_iters = it;
  timer_end(c, T_PSOLVE);
  if (iters) *iters = it;
  if (relres) *relres = sqrt(rr) / bnorm;
  return HFDIB_OK;
}

}  // namespace hfdib
