// Stage kernel of the propagator pair of the instability example (Section
// 3.1): both F and G are three-stage Runge-Kutta schemes (stages at 1/3,
// 1/2 and 1 of the step, each from q^n), F with the sixth-order centred
// advective flux, G with the first-order upwind flux, both with
// second-order centred acoustic fluxes and no damping, advection along x
// and z.  In point-stencil form the right-hand side of each field is
//   sum_{m=-3..3} (wx[m] q(i+m, j) + wz[m] q(i, j+m))
// plus the acoustic terms
//   u: -c_s (p(i+1) - p(i-1)) / (2 dx)
//   w: -c_s (p(j+1) - p(j-1)) / (2 dz)
//   p: -c_s ((u(i+1) - u(i-1)) / (2 dx) + (w(j+1) - w(j-1)) / (2 dz)).
// The example runs on small grids, where a step is bound by launch latency;
// one point per thread with neighbours read from global memory (cached) is
// the simple form that fits.
#include "pr_internal.h"

namespace prh {
namespace {

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__global__ __launch_bounds__(256) void k_rk3_stage(
    const double* __restrict__ in, int64_t is, const double* __restrict__ base,
    int64_t bs, double* __restrict__ out, int64_t os, int nx, int nz,
    const Rk3Coef c, double beta) {
  const int64_t n = (int64_t)nx * nz;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int64_t sl = blockIdx.y;
  const double* U = in + sl * is;
  const double* W = U + n;
  const double* Pf = U + 2 * n;
  const int i = (int)(idx % nx), j = (int)(idx / nx);
  const int64_t row = (int64_t)j * nx;
  double au = 0.0, aw = 0.0, ap = 0.0;
#pragma unroll
  for (int m = -3; m <= 3; ++m) {
    const int64_t o = row + wrap(i + m, nx);
    au += c.wx[m + 3] * U[o];
    aw += c.wx[m + 3] * W[o];
    ap += c.wx[m + 3] * Pf[o];
  }
#pragma unroll
  for (int m = -3; m <= 3; ++m) {
    const int64_t o = (int64_t)wrap(j + m, nz) * nx + i;
    au += c.wz[m + 3] * U[o];
    aw += c.wz[m + 3] * W[o];
    ap += c.wz[m + 3] * Pf[o];
  }
  const int64_t ip = row + wrap(i + 1, nx), im = row + wrap(i - 1, nx);
  const int64_t jp = (int64_t)wrap(j + 1, nz) * nx + i;
  const int64_t jm = (int64_t)wrap(j - 1, nz) * nx + i;
  const double fu = au - c.cx2 * (Pf[ip] - Pf[im]);
  const double fw = aw - c.cz2 * (Pf[jp] - Pf[jm]);
  const double fp = ap - (c.cx2 * (U[ip] - U[im]) + c.cz2 * (W[jp] - W[jm]));
  const double* B = base + sl * bs;
  double* O = out + sl * os;
  O[idx] = B[idx] + beta * fu;
  O[n + idx] = B[n + idx] + beta * fw;
  O[2 * n + idx] = B[2 * n + idx] + beta * fp;
}

}  // namespace

hipError_t launch_rk3_stage(const double* in, int64_t in_stride,
                            const double* base, int64_t base_stride,
                            double* out, int64_t out_stride, int nx, int nz,
                            int nstates, const Rk3Coef& c, double beta,
                            hipStream_t s) {
  if (nstates <= 0) return hipSuccess;
  const int64_t n = (int64_t)nx * nz;
  hipLaunchKernelGGL(k_rk3_stage, dim3((unsigned)((n + 255) / 256), nstates),
                     dim3(256), 0, s, in, in_stride, base, base_stride, out,
                     out_stride, nx, nz, c, beta);
  return hipGetLastError();
}

}  // namespace prh
