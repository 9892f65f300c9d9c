// Device helpers shared by the HFDIB kernels: indexing, boundary faces,
// deterministic block reductions (wave64 shuffles + LDS), geometric helpers.
#pragma once

#include "hfdib_internal.h"

namespace hfdib {

// ---------------------------------------------------------------- indexing
__device__ __forceinline__ long long cidx(const Params& P, int i, int j, int k) {
  return (long long)i + (long long)P.nx * ((long long)j + (long long)P.ny * k);
}
// face index of the face on the low side of cell (i,j,k), normal d
__device__ __forceinline__ long long fidx(const Params& P, int d, int i, int j, int k) {
  if (d == 0) return (long long)i + (long long)(P.nx + 1) * ((long long)j + (long long)P.ny * k);
  if (d == 1) return (long long)i + (long long)P.nx * ((long long)j + (long long)(P.ny + 1) * k);
  return (long long)i + (long long)P.nx * ((long long)j + (long long)P.ny * k);
}
__device__ __forceinline__ int ncell(const Params& P, int d) { return d == 0 ? P.nx : (d == 1 ? P.ny : P.nz); }
__device__ __forceinline__ long long stride(const Params& P, int d) {
  return d == 0 ? 1LL : (d == 1 ? (long long)P.nx : (long long)P.nx * P.ny);
}
__device__ __forceinline__ int comp(int d, int i, int j, int k) { return d == 0 ? i : (d == 1 ? j : k); }

// true when the cell touches the domain face (d, s)
// index of cell (i, j, k) in a colour-split array (see Params::nrb)
__device__ __forceinline__ long long rb_split(const Params& P, int i, int j, int k) {
  return (long long)((i + j + k) & 1) * P.nrb + ((long long)k * P.ny + j) * P.nxh + (i >> 1);
}
__device__ __forceinline__ bool on_bnd(const Params& P, int d, int s, int i, int j, int k) {
  int a = comp(d, i, j, k);
  return s < 0 ? (a == 0) : (a == ncell(P, d) - 1);
}
__device__ __forceinline__ int face_kind(const Params& P, int d, int s) { return P.bc[2 * d + (s > 0 ? 1 : 0)]; }

// outward flux of cell (i,j,k) through its face (d, s)
__device__ __forceinline__ double outward_flux(const Params& P, const double* const* phi, int d, int s, int i,
                                               int j, int k) {
  long long f = fidx(P, d, i, j, k);
  if (s > 0) {
    long long off = d == 0 ? 1LL : (d == 1 ? (long long)P.nx : (long long)P.nx * P.ny);
    return phi[d][f + off];
  }
  return -phi[d][f];
}

struct Phi3 {
  const double* a[3];
  __device__ __forceinline__ const double* const* ptr() const { return a; }
};

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide sums of NV values (256 threads = 4 waves), result written by
// thread 0 to part[v*pstride + blk].  Fixed reduction order: deterministic.
template <int NV>
__device__ __forceinline__ void block_sums_store(const double (&v)[NV], double* part, long long pstride,
                                                 long long blk) {
  __shared__ double lds[4][NV];
  int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  int lane = tid & 63, wid = tid >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) lds[wid][q] = s;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = lds[0][q];
      for (int w = 1; w < 4; ++w) s += lds[w][q];
      part[(long long)q * pstride + blk] = s;
    }
  }
}

// Full-grid kernels run on a 1D grid of 256-thread tiles (grid3()) of
// 2^tx_log2 x 2^(8 - tx_log2 - tz_log2) x 2^tz_log2 cells.  Consecutive
// workgroups are dispatched round-robin over the 8 XCDs; the logical tile order
// is remapped so that each XCD works on a contiguous run of tiles (x fastest,
// then y, then z) and the y/z halo rows a tile needs stay in that XCD's L2.
// tile coordinates of logical tile L on a grid of tx x ty x (nz >> tz_log2)
// tiles: x fastest, then y, then z; or z fastest, then x, then y.  Written with
// selects on the (uniform) order flag so the three results stay in registers.
struct TileXYZ {
  int x, y, z;
};
__device__ __forceinline__ TileXYZ tile_coords(const Params& P, unsigned L, int tx, int ty) {
  const bool zf = P.tile_zfirst != 0;
  const unsigned m0 = zf ? (unsigned)(P.nz >> P.tz_log2) : (unsigned)tx;
  const unsigned m1 = zf ? (unsigned)tx : (unsigned)ty;
  const unsigned a = L % m0, rest = L / m0;
  const unsigned b = rest % m1, c = rest / m1;
  TileXYZ t;
  t.x = (int)(zf ? b : a);
  t.y = (int)(zf ? c : b);
  t.z = (int)(zf ? a : c);
  return t;
}
__device__ __forceinline__ void tile_ijk(const Params& P, int& i, int& j, int& k) {
  unsigned nb = gridDim.x, b = blockIdx.x;
  unsigned q = nb >> 3, r = nb & 7u, x = b & 7u, id = b >> 3;
  unsigned L = x < r ? x * (q + 1) + id : r * (q + 1) + (x - r) * q + id;
  const int lx = P.tx_log2, lz = P.tz_log2, ly = 8 - lx - lz;
  int tx = (P.nx + (1 << lx) - 1) >> lx, ty = (P.ny + (1 << ly) - 1) >> ly;
  const TileXYZ t = tile_coords(P, L, tx, ty);
  k = (t.z << lz) + (int)threadIdx.z;
  i = (t.x << lx) + (int)threadIdx.x;
  j = (t.y << ly) + (int)threadIdx.y;
}

// Red-black half sweeps run on a grid of half the x extent: thread t of a row
// handles the cell i = 2 t + ((j + k + color) & 1), the one of the active
// colour (no idle lanes); same XCD-contiguous tile order as tile_ijk.
__device__ __forceinline__ void tile_ijk_rb(const Params& P, int color, int& i, int& j, int& k) {
  unsigned nb = gridDim.x, b = blockIdx.x;
  unsigned q = nb >> 3, r = nb & 7u, x = b & 7u, id = b >> 3;
  unsigned L = x < r ? x * (q + 1) + id : r * (q + 1) + (x - r) * q + id;
  int nxh = (P.nx + 1) >> 1;
  const int lx = P.tx_log2, lz = P.tz_log2, ly = 8 - lx - lz;
  int tx = (nxh + (1 << lx) - 1) >> lx, ty = (P.ny + (1 << ly) - 1) >> ly;
  const TileXYZ t = tile_coords(P, L, tx, ty);
  k = (t.z << lz) + (int)threadIdx.z;
  j = (t.y << ly) + (int)threadIdx.y;
  // t >= nxh gives i >= nx and i ^ 1 >= nx (both cells of the pair outside)
  int tp = (t.x << lx) + (int)threadIdx.x;
  i = 2 * tp + ((j + k + color) & 1);
}

__device__ __forceinline__ long long block_linear() {
  return (long long)blockIdx.x + (long long)gridDim.x * ((long long)blockIdx.y + (long long)gridDim.y * blockIdx.z);
}

// ---------------------------------------------------------------- gradients
// Gauss face value of velocity component cc on the domain face (d, s)
// (inlet u_in, no-slip 0, slip: normal component 0, outlet: owner value;
// faces of cells with lambda > 0: owner value).  Branch free: affine map with
// host-computed coefficients, exact for finite uP.
__device__ __forceinline__ double u_bface(const Params& P, int cc, int d, int s, bool solid, double uP) {
  const int f = 2 * d + (s > 0 ? 1 : 0);
  double v = P.ubA[f][cc] * uP + P.ubB[f][cc];
  return solid ? uP : v;
}
// Gauss face value of a transported scalar (inlet value at inlets, else zero gradient)
__device__ __forceinline__ double sc_bface(const Params& P, int d, int s, bool solid, double vP, double vin) {
  const bool inl = P.sc_inlet[2 * d + (s > 0 ? 1 : 0)] != 0;
  return (inl && !solid) ? vin : vP;
}
// b ? x : y with both operands evaluated before the choice.  Stencil code
// writes its conditional terms this way: a conditional expression whose arms
// contain a load is emitted as a branch around the load, and the loads of a
// stencil then wait one after another instead of being in flight together.
template <typename T>
__device__ __forceinline__ T sel(bool b, T x, T y) {
  return b ? x : y;
}

// 2 S:S with S the symmetric part of G (summed over all nine entries)
__device__ __forceinline__ double strain2(const double (&G)[3][3]) {
  double S2 = 0.0;
#pragma unroll
  for (int ii = 0; ii < 3; ++ii)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      double sij = 0.5 * (G[ii][jj] + G[jj][ii]);
      S2 = S2 + 2.0 * sij * sij;
    }
  return S2;
}

// ---------------------------------------------------------------- neighbourhood
// Clamped neighbour indices of a cell (the cell itself across a domain face)
// and the mask of domain faces.  Stencil kernels load every neighbour value
// unconditionally from these indices (always in bounds) and select boundary
// values afterwards, so no load sits inside a divergent branch.  Face
// q = 2 d + (s > 0) in the order W, E, S, N, B, T; faces beyond dim count as
// domain faces.
struct Nbr {
  int n[6];      // neighbour cell indices (grids hold fewer than 2^31 cells; 32-bit to save registers)
  unsigned bnd;  // bit q: face q is a domain face
};
__device__ __forceinline__ Nbr make_nbr(const Params& P, int i, int j, int k, long long c) {
  Nbr N;
  N.bnd = 0u;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    long long st = stride(P, d);
    int a = comp(d, i, j, k);
    bool lo = d >= P.dim || a == 0, hi = d >= P.dim || a == ncell(P, d) - 1;
    N.n[2 * d] = (int)(lo ? c : c - st);
    N.n[2 * d + 1] = (int)(hi ? c : c + st);
    N.bnd |= (lo ? 1u : 0u) << (2 * d);
    N.bnd |= (hi ? 1u : 0u) << (2 * d + 1);
  }
  return N;
}
__device__ __forceinline__ bool is_bnd(const Nbr& N, int q) { return (N.bnd >> q) & 1u; }
// index in a colour-split array (rb_split) of the face neighbour q of cell
// (i, j, k): the cell itself across a domain face, like the clamped natural
// indices of Nbr
__device__ __forceinline__ long long nb_split(const Params& P, const Nbr& N, int i, int j, int k, int q) {
  const int d = q >> 1, sg = (q & 1) ? 1 : -1;
  const int o = is_bnd(N, q) ? 0 : sg;
  return rb_split(P, i + (d == 0 ? o : 0), j + (d == 1 ? o : 0), k + (d == 2 ? o : 0));
}

// d u_jc / d x_a at cell x (Gauss, linear face interpolation) from clamped
// loads; lo / hi: x lies on the low / high domain face along a; solid: lambda > 0
__device__ __forceinline__ double gradu_bf(const Params& P, const double* uj, int jc, int a, long long x, bool lo,
                                           bool hi, bool solid) {
  long long st = stride(P, a);
  double uP = uj[x];
  double up = uj[hi ? x : x + st];
  double um = uj[lo ? x : x - st];
  double fp = sel(hi, u_bface(P, jc, a, +1, solid, uP), 0.5 * (uP + up));
  double fm = sel(lo, u_bface(P, jc, a, -1, solid, uP), 0.5 * (um + uP));
  return (fp - fm) * P.idelta[a];
}
// d u_jc / d x_b at the (clamped) face neighbour q of cell (i, j, k), the value
// the cell gradient above takes at that cell: across the axis of q the
// neighbour has the cell's domain faces, along it its own position decides;
// sn: the neighbour has lambda > 0.  (Across a domain face the neighbour index
// is the cell itself and the value is to be discarded.)
__device__ __forceinline__ double gradu_nb(const Params& P, const double* uj, int jc, int b, const Nbr& N, int q, int i,
                                           int j, int k, bool sn) {
  const int a = q >> 1;
  bool lo = is_bnd(N, 2 * b), hi = is_bnd(N, 2 * b + 1);
  if (a == b) {
    const int x = comp(a, i, j, k) + (is_bnd(N, q) ? 0 : ((q & 1) ? 1 : -1));
    lo = x == 0;
    hi = x == ncell(P, a) - 1;
  }
  return gradu_bf(P, uj, jc, b, N.n[q], lo, hi, sn);
}
// full velocity gradient G[a][jc] = d u_jc / d x_a at a cell (zero outside dim)
__device__ __forceinline__ void gradu_all_bf(const Params& P, const double* const* u, bool solid, const Nbr& N,
                                             long long c, double (&G)[3][3]) {
#pragma unroll
  for (int jc = 0; jc < 3; ++jc)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      G[a][jc] = sel(a < P.dim && jc < P.dim,
                     gradu_bf(P, u[jc], jc, a, c, is_bnd(N, 2 * a), is_bnd(N, 2 * a + 1), solid), 0.0);
}

// ---------------------------------------------------------------- geometry
struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 center(const Params& P, int i, int j, int k) {
  V3 c;
  c.x = P.x0 + ((double)i + 0.5) * P.dx;
  c.y = P.y0 + ((double)j + 0.5) * P.dy;
  c.z = P.dim == 3 ? P.z0 + ((double)k + 0.5) * P.dz : 0.0;
  return c;
}

// central-difference gradient of lambda, one-sided at the domain edges
__device__ __forceinline__ V3 grad_lambda(const Params& P, const double* lam, int i, int j, int k) {
  V3 g = {0.0, 0.0, 0.0};
  long long c = cidx(P, i, j, k);
  for (int d = 0; d < P.dim; ++d) {
    int n = ncell(P, d);
    if (n <= 1) continue;
    int a = comp(d, i, j, k);
    long long st = stride(P, d);
    double D = P.delta[d];
    double val;
    if (a == 0)
      val = (lam[c + st] - lam[c]) / D;
    else if (a == n - 1)
      val = (lam[c] - lam[c - st]) / D;
    else
      val = (lam[c + st] - lam[c - st]) / (2.0 * D);
    if (d == 0) g.x = val;
    else if (d == 1) g.y = val;
    else g.z = val;
  }
  return g;
}

// outward normal n = -grad(lambda)/|grad(lambda)|, with the fallback to the
// normalised sum of (P - N) over in-solid Moore neighbours
__device__ V3 cell_normal(const Params& P, const double* lam, const uint8_t* flags, int i, int j, int k) {
  V3 g = grad_lambda(P, lam, i, j, k);
  double nrm = sqrt(g.x * g.x + g.y * g.y + g.z * g.z);
  V3 n;
  if (nrm * P.h >= 1e-12) {
    n.x = -g.x / nrm;
    n.y = -g.y / nrm;
    n.z = -g.z / nrm;
    return n;
  }
  V3 acc = {0.0, 0.0, 0.0};
  int zr = P.dim == 3 ? 1 : 0;
  for (int ox = -1; ox <= 1; ++ox)
    for (int oy = -1; oy <= 1; ++oy)
      for (int oz = -zr; oz <= zr; ++oz) {
        if (ox == 0 && oy == 0 && oz == 0) continue;
        int ii = i + ox, jj = j + oy, kk = k + oz;
        if (ii < 0 || ii >= P.nx || jj < 0 || jj >= P.ny || kk < 0 || kk >= P.nz) continue;
        if (flags[cidx(P, ii, jj, kk)] & F_IC) {
          acc.x -= ox * P.dx;
          acc.y -= oy * P.dy;
          acc.z -= oz * P.dz;
        }
      }
  double a = sqrt(acc.x * acc.x + acc.y * acc.y + acc.z * acc.z);
  if (a > 0.0) {
    acc.x /= a;
    acc.y /= a;
    acc.z /= a;
  }
  return acc;
}

}  // namespace hfdib
