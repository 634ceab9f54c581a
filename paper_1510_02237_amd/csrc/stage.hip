// RK-3 step kernel for right-hand sides whose advective weights vary from
// row to row (x-direction) and from column to column (z-direction):
//   f(q)_field = sum_{m=-3..3} (wx[j][m] q(i+m, j) + wz[i][m] q(i, j+m))
//                - acoustic centred differences + grad-div damping.
// It serves:
//  * the propagator pair of the instability example (Section 3.1): RK-3
//    steps with the sixth-order centred (F) or first-order upwind (G)
//    advective flux, second-order acoustics, no damping, constant velocity
//    (every row and every column has the same weights);
//  * the fine propagator of Section 3.2 with an advection velocity that
//    varies in space, (U + gamma (z - Lz/2), V - gamma (x - Lx/2)) (eq.
//    adVel): the x-velocity is constant along a row and the z-velocity
//    along a column, so the flux-form fifth-order upwind advection has one
//    weight set (and one upwind side) per row and one per column.
// (The frozen slow tendency of the split coarse step with that velocity
// uses the same kind of tables and is evaluated inside the coarse kernel.)
// With d1(q) = q(+1) - q(-1) and d2(q) = q(+2) - q(-2) along an axis the
// acoustic terms are
//   u: -(ax1 d1x(p) + ax2 d2x(p))      w: -(az1 d1z(p) + az2 d2z(p))
//   p: -((ax1 d1x(u) + ax2 d2x(u)) + (az1 d1z(w) + az2 d2z(w)))
// (second order: ax1 = c_s/(2 dx), ax2 = 0; fourth order: ax1 = 8 c_s/(12
// dx), ax2 = -c_s/(12 dx)) and the damping is that of the fused fine step.
// These runs use small grids, where a step is bound by launch latency, so
// one launch does all three stages of a step on a tile held in LDS.
#include "pr_internal.h"

namespace prh {
namespace {

// f at one point; at(field, dx, dz) returns field 0 (u), 1 (w) or 2 (p) at
// offset (dx, dz) from the point, wx and wz are the point's row and column
// weights.
template <class At>
__device__ __forceinline__ void stage_point(const At& at, const double* wx,
                                            const double* wz,
                                            const StageCoef& c, double& fu,
                                            double& fw, double& fp) {
  double au = 0.0, aw = 0.0, ap = 0.0;
#pragma unroll
  for (int m = -3; m <= 3; ++m) {
    au += wx[m + 3] * at(0, m, 0);
    aw += wx[m + 3] * at(1, m, 0);
    ap += wx[m + 3] * at(2, m, 0);
  }
#pragma unroll
  for (int m = -3; m <= 3; ++m) {
    au += wz[m + 3] * at(0, 0, m);
    aw += wz[m + 3] * at(1, 0, m);
    ap += wz[m + 3] * at(2, 0, m);
  }
  const double dpx = c.ax1 * (at(2, 1, 0) - at(2, -1, 0)) + c.ax2 * (at(2, 2, 0) - at(2, -2, 0));
  const double dpz = c.az1 * (at(2, 0, 1) - at(2, 0, -1)) + c.az2 * (at(2, 0, 2) - at(2, 0, -2));
  const double dux = c.ax1 * (at(0, 1, 0) - at(0, -1, 0)) + c.ax2 * (at(0, 2, 0) - at(0, -2, 0));
  const double dwz = c.az1 * (at(1, 0, 1) - at(1, 0, -1)) + c.az2 * (at(1, 0, 2) - at(1, 0, -2));
  const double gxx = (at(0, 1, 0) + at(0, -1, 0)) - 2.0 * at(0, 0, 0);
  const double gzz = (at(1, 0, 1) + at(1, 0, -1)) - 2.0 * at(1, 0, 0);
  const double wxz = (at(1, 1, 1) - at(1, 1, -1)) - (at(1, -1, 1) - at(1, -1, -1));
  const double uxz = (at(0, 1, 1) - at(0, -1, 1)) - (at(0, 1, -1) - at(0, -1, -1));
  fu = au - dpx + c.kxx * gxx + c.kxzu * wxz;
  fw = aw - dpz + c.kzz * gzz + c.kxzw * uxz;
  fp = ap - (dux + dwz);
}

// All three stages of one RK-3 step in one launch.  A workgroup owns a
// S3_T x S3_T tile of one state and loads it with a halo of 9 cells (3 per
// stage) into LDS; stage s is evaluated on the region shrunk by 3 s, so the
// third stage covers exactly the tile.  Per tile 784 + 484 + 256 point
// evaluations for 256 outputs, against 3 launches of the one-point kernel.
constexpr int S3_T = 16, S3_H = 9, S3_R = S3_T + 2 * S3_H, S3_RN = S3_R * S3_R;
constexpr int S3_NT = 256;

__device__ __forceinline__ int wrap_any(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__global__ __launch_bounds__(S3_NT) void k_stage3(
    const double* __restrict__ in, int64_t is, double* __restrict__ out,
    int64_t os, int nx, int nz, int xtiles, const StageCoef c, double b1,
    double b2, double b3) {
  __shared__ double q0[3 * S3_RN], s1[3 * S3_RN], s2[3 * S3_RN];
  __shared__ int gi[S3_R], gj[S3_R];  // grid column / row of a region index
  const int64_t n = (int64_t)nx * nz;
  const int xt = blockIdx.x % xtiles, zt = blockIdx.x / xtiles;
  const int64_t sl = blockIdx.y;
  const double* src = in + sl * is;
  double* dst = out + sl * os;
  const int t = threadIdx.x;
  const int gx0 = xt * S3_T - S3_H, gz0 = zt * S3_T - S3_H;
  if (t < S3_R) {
    gi[t] = wrap_any(gx0 + t, nx);
    gj[t] = wrap_any(gz0 + t, nz);
  }
  __syncthreads();
  for (int r = t; r < S3_RN; r += S3_NT) {
    const int64_t g = (int64_t)gj[r / S3_R] * nx + gi[r % S3_R];
    q0[r] = src[g];
    q0[S3_RN + r] = src[n + g];
    q0[2 * S3_RN + r] = src[2 * n + g];
  }
  __syncthreads();
  // Stage s over the region points at least 3 s from its edge.
  auto stage = [&](int s, const double* q, double beta, double* o,
                   bool last) {
    const int lo = 3 * s, side = S3_R - 6 * s;
    for (int r = t; r < side * side; r += S3_NT) {
      const int a = lo + r % side, b = lo + r / side;
      const int p = b * S3_R + a;
      auto at = [&](int f, int dx, int dz) {
        return q[f * S3_RN + p + dz * S3_R + dx];
      };
      double fu, fw, fp;
      stage_point(at, c.wx + 7 * (int64_t)gj[b], c.wz + 7 * (int64_t)gi[a], c,
                  fu, fw, fp);
      const double nu = q0[p] + beta * fu, nw = q0[S3_RN + p] + beta * fw,
                   np = q0[2 * S3_RN + p] + beta * fp;
      if (!last) {
        o[p] = nu;
        o[S3_RN + p] = nw;
        o[2 * S3_RN + p] = np;
      } else {
        const int x = xt * S3_T + a - S3_H, z = zt * S3_T + b - S3_H;
        if (x < nx && z < nz) {
          const int64_t g = (int64_t)z * nx + x;
          dst[g] = nu;
          dst[n + g] = nw;
          dst[2 * n + g] = np;
        }
      }
    }
  };
  stage(1, q0, b1, s1, false);
  __syncthreads();
  stage(2, s1, b2, s2, false);
  __syncthreads();
  stage(3, s2, b3, nullptr, true);
}

}  // namespace

hipError_t launch_stage3(const double* in, int64_t in_stride, double* out,
                         int64_t out_stride, int nx, int nz, int nstates,
                         const StageCoef& c, double beta1, double beta2,
                         double beta3, hipStream_t s) {
  if (nstates <= 0) return hipSuccess;
  const int xtiles = (nx + S3_T - 1) / S3_T, ztiles = (nz + S3_T - 1) / S3_T;
  hipLaunchKernelGGL(k_stage3, dim3((unsigned)(xtiles * ztiles), nstates),
                     dim3(S3_NT), 0, s, in, in_stride, out, out_stride, nx, nz,
                     xtiles, c, beta1, beta2, beta3);
  return hipGetLastError();
}

}  // namespace prh
