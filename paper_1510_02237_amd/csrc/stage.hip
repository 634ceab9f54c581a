// Point-stencil stage kernel for right-hand sides whose advective weights
// vary from row to row (x-direction) and from column to column
// (z-direction):
//   f(q)_field = sum_{m=-3..3} (wx[j][m] q(i+m, j) + wz[i][m] q(i, j+m))
//                - acoustic centred differences + grad-div damping.
// It serves three right-hand sides:
//  * the propagator pair of the instability example (Section 3.1): RK-3
//    stages with the sixth-order centred (F) or first-order upwind (G)
//    advective flux, second-order acoustics, no damping, constant velocity
//    (every row and every column has the same weights);
//  * the fine propagator of Section 3.2 with an advection velocity that
//    varies in space, (U + gamma (z - Lz/2), V - gamma (x - Lx/2)) (eq.
//    adVel): the x-velocity is constant along a row and the z-velocity
//    along a column, so the flux-form fifth-order upwind advection has one
//    weight set (and one upwind side) per row and one per column;
//  * the frozen slow tendency of the split coarse step with that velocity
//    (first-order upwind weights, no acoustics, no damping, no base).
// With d1(q) = q(+1) - q(-1) and d2(q) = q(+2) - q(-2) along an axis the
// acoustic terms are
//   u: -(ax1 d1x(p) + ax2 d2x(p))      w: -(az1 d1z(p) + az2 d2z(p))
//   p: -((ax1 d1x(u) + ax2 d2x(u)) + (az1 d1z(w) + az2 d2z(w)))
// (second order: ax1 = c_s/(2 dx), ax2 = 0; fourth order: ax1 = 8 c_s/(12
// dx), ax2 = -c_s/(12 dx)) and the damping is that of the fused fine step.
// These runs use small grids, where a step is bound by launch latency;
// one point per thread with neighbours read from global memory (cached)
// is the simple form that fits.
#include "pr_internal.h"

namespace prh {
namespace {

// Periodic index for i in [-3, n + 3) (a grid index plus a stencil offset
// of at most 3; grids have n >= 8): two compares instead of a division.
__device__ __forceinline__ int wrap(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

__global__ __launch_bounds__(256) void k_stage(
    const double* __restrict__ in, int64_t is, const double* __restrict__ base,
    int64_t bs, double* __restrict__ out, int64_t os, int nx, int nz,
    const StageCoef c, double beta) {
  const int64_t n = (int64_t)nx * nz;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int64_t sl = blockIdx.y;
  const double* U = in + sl * is;
  const double* W = U + n;
  const double* Pf = U + 2 * n;
  const int i = (int)(idx % nx), j = (int)(idx / nx);
  const int64_t row = (int64_t)j * nx;
  const double* wx = c.wx + 7 * (int64_t)j;
  const double* wz = c.wz + 7 * (int64_t)i;
  double au = 0.0, aw = 0.0, ap = 0.0;
#pragma unroll
  for (int m = -3; m <= 3; ++m) {
    const int64_t o = row + wrap(i + m, nx);
    au += wx[m + 3] * U[o];
    aw += wx[m + 3] * W[o];
    ap += wx[m + 3] * Pf[o];
  }
#pragma unroll
  for (int m = -3; m <= 3; ++m) {
    const int64_t o = (int64_t)wrap(j + m, nz) * nx + i;
    au += wz[m + 3] * U[o];
    aw += wz[m + 3] * W[o];
    ap += wz[m + 3] * Pf[o];
  }
  auto X = [&](int di) { return row + wrap(i + di, nx); };
  auto Z = [&](int dj) { return (int64_t)wrap(j + dj, nz) * nx + i; };
  auto ZX = [&](int dj, int di) {
    return (int64_t)wrap(j + dj, nz) * nx + wrap(i + di, nx);
  };
  const double dpx = c.ax1 * (Pf[X(1)] - Pf[X(-1)]) + c.ax2 * (Pf[X(2)] - Pf[X(-2)]);
  const double dpz = c.az1 * (Pf[Z(1)] - Pf[Z(-1)]) + c.az2 * (Pf[Z(2)] - Pf[Z(-2)]);
  const double dux = c.ax1 * (U[X(1)] - U[X(-1)]) + c.ax2 * (U[X(2)] - U[X(-2)]);
  const double dwz = c.az1 * (W[Z(1)] - W[Z(-1)]) + c.az2 * (W[Z(2)] - W[Z(-2)]);
  const double gxx = (U[X(1)] + U[X(-1)]) - 2.0 * U[idx];
  const double gzz = (W[Z(1)] + W[Z(-1)]) - 2.0 * W[idx];
  const double wxz = (W[ZX(1, 1)] - W[ZX(-1, 1)]) - (W[ZX(1, -1)] - W[ZX(-1, -1)]);
  const double uxz = (U[ZX(1, 1)] - U[ZX(1, -1)]) - (U[ZX(-1, 1)] - U[ZX(-1, -1)]);
  const double fu = au - dpx + c.kxx * gxx + c.kxzu * wxz;
  const double fw = aw - dpz + c.kzz * gzz + c.kxzw * uxz;
  const double fp = ap - (dux + dwz);
  double* O = out + sl * os;
  if (base) {
    const double* B = base + sl * bs;
    O[idx] = B[idx] + beta * fu;
    O[n + idx] = B[n + idx] + beta * fw;
    O[2 * n + idx] = B[2 * n + idx] + beta * fp;
  } else {
    O[idx] = beta * fu;
    O[n + idx] = beta * fw;
    O[2 * n + idx] = beta * fp;
  }
}

}  // namespace

hipError_t launch_stage(const double* in, int64_t in_stride,
                        const double* base, int64_t base_stride, double* out,
                        int64_t out_stride, int nx, int nz, int nstates,
                        const StageCoef& c, double beta, hipStream_t s) {
  if (nstates <= 0) return hipSuccess;
  const int64_t n = (int64_t)nx * nz;
  hipLaunchKernelGGL(k_stage, dim3((unsigned)((n + 255) / 256), nstates),
                     dim3(256), 0, s, in, in_stride, base, base_stride, out,
                     out_stride, nx, nz, c, beta);
  return hipGetLastError();
}

}  // namespace prh
