// Force on the immersed body (per unit density, kinematic units), from the
// discrete interface measure of the indicator: the surface element of a cell
// is |grad lambda| V and its outward normal n = -grad lambda / |grad lambda|
// (Sec. of the drag and lift coefficients; eq. for sigma and n).
//
//   pressure part  F_p = - sum_cells p n |grad lambda| V = sum_cells p grad(lambda) V
//   viscous part   F_v = A_G * (sum_BC tau_w t |grad lambda| V) / (sum_BC |grad lambda| V)
//
// with A_G = sum_cells |grad lambda| V the interface area, t the direction of
// the tangential velocity relative to the solid at a boundary cell and tau_w
// the wall shear stress: u_tau^2 from the log-law Newton solve on cells of the
// logarithmic branch, nu |u_t| / y_eff on cells of the viscous branch.
#include <mutex>

#include "device_common.h"

namespace hfdib {

// sums over all cells: p grad(lambda) V (3) and |grad lambda| V (1)
__global__ void k_force_cells(Params P, const double* p, const double* lam, double* part, long long pstride) {
  int i, j, k;
  tile_ijk(P, i, j, k);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < P.nx && j < P.ny) {
    long long c = cidx(P, i, j, k);
    V3 g = grad_lambda(P, lam, i, j, k);
    double pc = p[c];
    v[0] = pc * g.x * P.V;
    v[1] = pc * g.y * P.V;
    v[2] = pc * g.z * P.V;
    v[3] = sqrt(g.x * g.x + g.y * g.y + g.z * g.z) * P.V;
  }
  block_sums_store<4>(v, part, pstride, block_linear());
}

// sums over the boundary cells: tau_w t |grad lambda| V (3) and |grad lambda| V (1)
__global__ void k_force_bc(Params P, int nbc, const int* bc_cells, const double* bc_n, const double* bc_yeff,
                           const double* bc_yplus, const double* bc_utauU, const double* lam, const double* u0,
                           const double* u1, const double* u2, const double* us0, const double* us1,
                           const double* us2, double* part, long long pstride) {
  int b = blockIdx.x * NTHREADS + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (b < nbc) {
    int c = bc_cells[b];
    int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / (P.nx * P.ny);
    V3 g = grad_lambda(P, lam, i, j, k);
    double dS = sqrt(g.x * g.x + g.y * g.y + g.z * g.z) * P.V;
    double ur[3] = {u0[c] - us0[c], u1[c] - us1[c], P.dim == 3 ? u2[c] - us2[c] : 0.0};
    double n[3] = {bc_n[3 * b], bc_n[3 * b + 1], bc_n[3 * b + 2]};
    double un = ur[0] * n[0] + ur[1] * n[1] + ur[2] * n[2];
    double t[3] = {ur[0] - un * n[0], ur[1] - un * n[1], ur[2] - un * n[2]};
    double mag = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    double ut = bc_utauU[b];
    double tau = bc_yplus[b] > P.ylam ? ut * ut : P.nu * mag / bc_yeff[b];
    double s = mag > 0.0 ? tau * dS / mag : 0.0;
    v[0] = s * t[0];
    v[1] = s * t[1];
    v[2] = s * t[2];
    v[3] = dS;
  }
  block_sums_store<4>(v, part, pstride, blockIdx.x);
}

int body_forces(hfdib_ctx* c, double* out8) {
  const Params& P = c->P;
  dim3 g = grid3(P), b = block3(P);
  long long nblk3 = (long long)g.x * g.y * g.z;
  double* S = c->scal + SCAL_PCG;
  hipLaunchKernelGGL(k_force_cells, g, b, 0, c->stream, P, c->p, c->lam, c->partials, c->pstride);
  launch_finalize(c, (int)nblk3, 4, SC_FORCE, 0);
  double h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (c->n_bc > 0) {
    hipLaunchKernelGGL(k_force_bc, dim3(nblocks1(c->n_bc)), dim3(NTHREADS), 0, c->stream, P, c->n_bc, c->bc_cells,
                       c->bc_n, c->bc_yeff, c->bc_yplus, c->bc_utauU, c->lam, c->u[0], c->u[1], c->u[2], c->us[0],
                       c->us[1], c->us[2], c->partials, c->pstride);
    launch_finalize(c, nblocks1(c->n_bc), 4, SC_FORCE + 4, 0);
  }
  HFDIB_CHECK_LAUNCH(c, "forces");
  HFDIB_CHECK(c, hipMemcpyAsync(h, S + SC_FORCE, (c->n_bc > 0 ? 8 : 4) * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream), "forces copy");
  HFDIB_CHECK(c, hipStreamSynchronize(c->stream), "forces sync");
  double area = h[3], bc_area = h[7];
  out8[0] = h[0];
  out8[1] = h[1];
  out8[2] = h[2];
  for (int d = 0; d < 3; ++d) out8[3 + d] = bc_area > 0.0 ? area * h[4 + d] / bc_area : 0.0;
  out8[6] = area;
  out8[7] = bc_area;
  return HFDIB_OK;
}

// ---------------------------------------------------------------- no allocation
// The variant of body_forces for callers that cannot allocate or synchronise:
// the block partial sums live in a file-scope device array (one copy per GPU,
// shared by every context on it) instead of the context's workspace, and the
// eight results go to a caller device buffer without a host read.  Every
// partial slot the final kernel reads is written by the partial kernels of the
// same call, so nothing has to be cleared; calls that overlap on one GPU race
// on the array.
constexpr size_t FORCE_SCRATCH_DOUBLES = (4u << 20) / sizeof(double);  // 4 MiB
static __device__ __align__(256) double scratch[FORCE_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
static double* g_scratch_dev[MAX_DEVICES];  // device address of scratch, per device
static std::mutex g_scratch_mu;

// device address of this device's copy of scratch (looked up once per device)
static int scratch_address(hfdib_ctx* c, double** out) {
  int dev = -1;
  HFDIB_CHECK(c, hipGetDevice(&dev), "forces_noalloc: current device");
  if (dev < 0 || dev >= MAX_DEVICES) {
    c->err = "forces_noalloc: device ordinal out of range";
    return HFDIB_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HFDIB_CHECK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "forces_noalloc: scratch address");
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return HFDIB_OK;
}

// sums the 4 cell rows and (nbb > 0) the 4 boundary-cell rows of partials and
// writes the force record (the same composition as body_forces) to out8
__global__ void __launch_bounds__(256) k_force_finish(const double* pc, long long nbc3, const double* pb, int nbb,
                                                      double* out8) {
  __shared__ double lds[4][8];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  for (long long b = tid; b < nbc3; b += 256)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += pc[(long long)q * nbc3 + b];
  for (int b = tid; b < nbb; b += 256)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[4 + q] += pb[(long long)q * nbb + b];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double sq = wave_sum(acc[q]);
    if (lane == 0) lds[wid][q] = sq;
  }
  __syncthreads();
  if (tid == 0) {
    double h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) h[q] = lds[0][q] + lds[1][q] + lds[2][q] + lds[3][q];
    const double area = h[3], bc_area = h[7];
    out8[0] = h[0];
    out8[1] = h[1];
    out8[2] = h[2];
    for (int d = 0; d < 3; ++d) out8[3 + d] = bc_area > 0.0 ? area * h[4 + d] / bc_area : 0.0;
    out8[6] = area;
    out8[7] = bc_area;
  }
}

int body_forces_noalloc(hfdib_ctx* c, double* out8_dev) {
  const Params& P = c->P;
  dim3 g = grid3(P), b = block3(P);
  const long long nblk3 = (long long)g.x * g.y * g.z;
  const int nbb = c->n_bc > 0 ? nblocks1(c->n_bc) : 0;
  const long long need = 4 * nblk3 + 4LL * nbb;
  if (need > (long long)FORCE_SCRATCH_DOUBLES) {
    c->err = "hfdib_forces_noalloc: the grid needs " + std::to_string(need * 8) +
             " bytes of partial sums, more than the fixed scratch of " +
             std::to_string(FORCE_SCRATCH_DOUBLES * 8) + " bytes (about 33 M cells)";
    return HFDIB_EINVAL;
  }
  double* sc = nullptr;
  int st = scratch_address(c, &sc);
  if (st != HFDIB_OK) return st;
  double* pc = sc;                 // 4 rows of nblk3 cell partials
  double* pb = sc + 4 * nblk3;     // 4 rows of nbb boundary-cell partials
  hipLaunchKernelGGL(k_force_cells, g, b, 0, c->stream, P, c->p, c->lam, pc, nblk3);
  if (nbb > 0)
    hipLaunchKernelGGL(k_force_bc, dim3(nbb), dim3(NTHREADS), 0, c->stream, P, c->n_bc, c->bc_cells, c->bc_n,
                       c->bc_yeff, c->bc_yplus, c->bc_utauU, c->lam, c->u[0], c->u[1], c->u[2], c->us[0], c->us[1],
                       c->us[2], pb, (long long)nbb);
  hipLaunchKernelGGL(k_force_finish, dim3(1), dim3(256), 0, c->stream, (const double*)pc, nblk3,
                     (const double*)pb, nbb, out8_dev);
  HFDIB_CHECK_LAUNCH(c, "forces_noalloc");
  return HFDIB_OK;
}

}  // namespace hfdib
