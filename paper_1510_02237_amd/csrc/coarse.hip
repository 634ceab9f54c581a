// Coarse propagator kernel: the partially split forward-Euler step of
// Section 3.2.  The slow (advective) tendency R = -U dq/dx (first-order
// upwind, the diffusive low-order operator that stabilises the split
// scheme) is evaluated once from q^n and frozen; then N_sound
// forward-backward acoustic substeps of length dtau = Delta t / N_sound:
//   u' = u + dtau (R_u - c_s dp/dx + alpha_1 (div u)_x)
//   w' = w + dtau (R_w - c_s dp/dz + alpha_2 (div u)_z)
//   p' = p + dtau (R_p - c_s (du'/dx + dw'/dz))
// with second-order centred acoustic differences, the compact grad-div
// damping and alpha = nu_c h^2 / dtau (eq. dampingCoeff with the split-step
// coefficients).  Momentum goes forward with the old pressure, pressure
// backward with the new velocities.
//
// One launch performs up to kCoarseMaxSubPerLaunch substeps: a workgroup
// loads a TX x TZ tile plus a halo of 2 cells per substep (and one more
// column on the upwind side when it evaluates R) into LDS, runs the
// substeps there, and writes the tile interior.  States are batched along
// blockIdx.y.
#include "pr_internal.h"

namespace prh {
namespace {

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

constexpr int TX = 32, TZ = 32, NT = 256;
constexpr int HXM = 2 * kCoarseMaxSubPerLaunch + 1;
constexpr int HZM = 2 * kCoarseMaxSubPerLaunch;
constexpr int RXM = TX + 2 * HXM, RZM = TZ + 2 * HZM;
constexpr int MPT = (RXM * RZM + NT - 1) / NT;  // points per thread

__global__ __launch_bounds__(NT) void k_coarse(const CoarseLaunch L) {
  __shared__ double su[RZM * RXM], sw[RZM * RXM], sp[RZM * RXM];
  const int nx = L.nx, nz = L.nz;
  const int64_t n = (int64_t)nx * nz;
  const int xtiles = (nx + TX - 1) / TX;
  const int xt = blockIdx.x % xtiles, zt = blockIdx.x / xtiles;
  const int64_t off = (int64_t)blockIdx.y * L.stride;
  const double* __restrict__ in = L.in + off;
  double* __restrict__ out = L.out + off;
  double* __restrict__ Rg = L.R ? L.R + off : nullptr;
  const bool computeR = (L.flags & kCoarseComputeR) != 0;
  const bool storeR = (L.flags & kCoarseStoreR) != 0;
  const int hx = 2 * L.nsub + (computeR ? 1 : 0);
  const int hz = 2 * L.nsub;
  const int RX = TX + 2 * hx, RZ = TZ + 2 * hz;
  const int npts = RX * RZ;
  const int gx0 = xt * TX - hx, gz0 = zt * TZ - hz;
  const int t = threadIdx.x;
  const CoarseCoef k = L.c;

  for (int q = t; q < npts; q += NT) {
    const int a = q % RX, b = q / RX;
    const int64_t g = (int64_t)wrap(gz0 + b, nz) * nx + wrap(gx0 + a, nx);
    su[q] = in[g];
    sw[q] = in[n + g];
    sp[q] = in[2 * n + g];
  }
  __syncthreads();

  double Ru[MPT], Rw[MPT], Rp[MPT];
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    const int q = t + m * NT;
    Ru[m] = Rw[m] = Rp[m] = 0.0;
    if (q < npts) {
      const int a = q % RX, b = q / RX;
      if (computeR) {
        if (k.upwind_left) {
          const int qm = b * RX + (a > 0 ? a - 1 : 0);
          Ru[m] = k.cR * (su[q] - su[qm]);
          Rw[m] = k.cR * (sw[q] - sw[qm]);
          Rp[m] = k.cR * (sp[q] - sp[qm]);
        } else {
          const int qp = b * RX + (a < RX - 1 ? a + 1 : RX - 1);
          Ru[m] = k.cR * (su[qp] - su[q]);
          Rw[m] = k.cR * (sw[qp] - sw[q]);
          Rp[m] = k.cR * (sp[qp] - sp[q]);
        }
        if (storeR && a >= hx && a < hx + TX && b >= hz && b < hz + TZ) {
          const int x = xt * TX + a - hx, z = zt * TZ + b - hz;
          if (x < nx && z < nz) {
            const int64_t g = (int64_t)z * nx + x;
            Rg[g] = Ru[m];
            Rg[n + g] = Rw[m];
            Rg[2 * n + g] = Rp[m];
          }
        }
      } else {
        const int64_t g = (int64_t)wrap(gz0 + b, nz) * nx + wrap(gx0 + a, nx);
        Ru[m] = Rg[g];
        Rw[m] = Rg[n + g];
        Rp[m] = Rg[2 * n + g];
      }
    }
  }

  const double dtau = k.dtau;
  for (int s = 0; s < L.nsub; ++s) {
    double un[MPT], wn[MPT];
#pragma unroll
    for (int m = 0; m < MPT; ++m) {
      const int q = t + m * NT;
      un[m] = wn[m] = 0.0;
      if (q < npts) {
        const int a = q % RX, b = q / RX;
        const int am = a > 0 ? a - 1 : 0, ap = a < RX - 1 ? a + 1 : RX - 1;
        const int bm = (b > 0 ? b - 1 : 0) * RX, bp = (b < RZ - 1 ? b + 1 : RZ - 1) * RX;
        const int bc = b * RX;
        const double u = su[q], w = sw[q];
        const double dpx = sp[bc + ap] - sp[bc + am];
        const double dpz = sp[bp + a] - sp[bm + a];
        const double gxx = (su[bc + ap] + su[bc + am]) - 2.0 * u;
        const double gzz = (sw[bp + a] + sw[bm + a]) - 2.0 * w;
        const double wx = (sw[bp + ap] - sw[bm + ap]) - (sw[bp + am] - sw[bm + am]);
        const double uz = (su[bp + ap] - su[bp + am]) - (su[bm + ap] - su[bm + am]);
        un[m] = u + dtau * (Ru[m] - k.cx2 * dpx + k.kxx * gxx + k.kxzu * wx);
        wn[m] = w + dtau * (Rw[m] - k.cz2 * dpz + k.kzz * gzz + k.kxzw * uz);
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MPT; ++m) {
      const int q = t + m * NT;
      if (q < npts) {
        su[q] = un[m];
        sw[q] = wn[m];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MPT; ++m) {
      const int q = t + m * NT;
      if (q < npts) {
        const int a = q % RX, b = q / RX;
        const int am = a > 0 ? a - 1 : 0, ap = a < RX - 1 ? a + 1 : RX - 1;
        const int bm = (b > 0 ? b - 1 : 0) * RX, bp = (b < RZ - 1 ? b + 1 : RZ - 1) * RX;
        const int bc = b * RX;
        const double dux = su[bc + ap] - su[bc + am];
        const double dwz = sw[bp + a] - sw[bm + a];
        sp[q] = sp[q] + dtau * (Rp[m] - k.cx2 * dux - k.cz2 * dwz);
      }
    }
    __syncthreads();
  }

  for (int q = t; q < npts; q += NT) {
    const int a = q % RX, b = q / RX;
    if (a < hx || a >= hx + TX || b < hz || b >= hz + TZ) continue;
    const int x = xt * TX + a - hx, z = zt * TZ + b - hz;
    if (x >= nx || z >= nz) continue;
    const int64_t g = (int64_t)z * nx + x;
    out[g] = su[q];
    out[n + g] = sw[q];
    out[2 * n + g] = sp[q];
  }
}

}  // namespace

hipError_t launch_coarse(const CoarseLaunch& L, hipStream_t s) {
  if (L.nsub < 1 || L.nsub > kCoarseMaxSubPerLaunch || L.nstates < 1)
    return hipErrorInvalidValue;
  const int tiles = ((L.nx + TX - 1) / TX) * ((L.nz + TZ - 1) / TZ);
  hipLaunchKernelGGL(k_coarse, dim3(tiles, L.nstates), dim3(NT), 0, s, L);
  return hipGetLastError();
}

}  // namespace prh
