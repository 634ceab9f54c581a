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
// column on each side when it evaluates R) into LDS, runs the substeps
// there and writes the tile interior.  u and w are double-buffered in LDS
// (the momentum update writes the other buffer, so two barriers per
// substep suffice) and each thread keeps its own points' values in
// registers.  The LDS region carries one more
// ring of cells that is never written with valid data, so every neighbour
// is a fixed offset and the points near the edge (whose results are
// discarded) need no clamping.  Each thread owns the same MPT points in
// every phase; their indices are computed once.  States are batched along
// blockIdx.y.
//
// With a z-velocity, a rotation or the third-order slow tendency, R is the
// sum of per-row x-weights and per-column z-weights times q (stencil within
// 2 cells); the TAB instantiation evaluates it in the launch from a region
// 2 cells wider on each side, where points closer than 2 cells to the
// region's edge (more than 2 N_sound cells from the tile, so outside what
// the substeps carry into it) keep R = 0.
#include "pr_internal.h"

namespace prh {
namespace {

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Largest halo: 2 cells per substep, plus 1 in x for the upwind R or 2 in
// both directions for the table-driven R.
template <bool TAB>
constexpr int kHXM = 2 * kCoarseMaxSubPerLaunch + (TAB ? 2 : 1);
template <bool TAB>
constexpr int kHZM = 2 * kCoarseMaxSubPerLaunch + (TAB ? 2 : 0);

// TX x TZ interior tile, NT threads.  A single state uses the shorter tile
// (twice the workgroups for a latency-bound launch); batches use 32 x 32.
template <int TX, int TZ, int NT, bool TAB>
__global__ __launch_bounds__(NT) void k_coarse(const CoarseLaunch L) {
  constexpr int HXM = kHXM<TAB>, HZM = kHZM<TAB>;
  constexpr int RXM = TX + 2 * HXM, RZM = TZ + 2 * HZM;
  constexpr int SX = RXM + 2;                     // padded LDS row stride
  constexpr int LDSN = (RZM + 2) * SX;
  constexpr int MPT = (RXM * RZM + NT - 1) / NT;  // points per thread
  __shared__ double su[LDSN], sw[LDSN], sp[LDSN], su2[LDSN], sw2[LDSN];
  const int nx = L.nx, nz = L.nz;
  const int64_t n = (int64_t)nx * nz;
  const int xtiles = (nx + TX - 1) / TX;
  // Workgroups go to the 8 XCDs round-robin; up to kXcdMaxTiles tiles
  // (a few rounds of the machine) each XCD gets a contiguous range of
  // tiles, so that the halo a tile reads was mostly written by the same XCD
  // in the previous step and sits in its L2.  With many rounds (4096 x 1024:
  // 8192 tiles) the tiles keep their natural order, which measured faster
  // there.  The grid is padded to a multiple of 8; blocks past the last
  // tile leave before any barrier.
  constexpr int kXcdMaxTiles = 2048;
  const int ntiles = xtiles * ((nz + TZ - 1) / TZ);
  const int per = (ntiles + 7) >> 3;
  const int lt = ntiles <= kXcdMaxTiles
                     ? (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3)
                     : (int)blockIdx.x;
  if (lt >= ntiles) return;
  const int xt = lt % xtiles, zt = lt / xtiles;
  const int64_t off = (int64_t)blockIdx.y * L.stride;
  const double* __restrict__ in = L.in + off;
  double* __restrict__ out = L.out + off;
  double* __restrict__ Rg = L.R ? L.R + off : nullptr;
  const bool computeR = TAB || (L.flags & kCoarseComputeR) != 0;
  const bool storeR = (L.flags & kCoarseStoreR) != 0;
  const int hx = 2 * L.nsub + (TAB ? 2 : (computeR ? 1 : 0));
  const int hz = 2 * L.nsub + (TAB ? 2 : 0);
  const int RX = TX + 2 * hx, RZ = TZ + 2 * hz;
  const int npts = RX * RZ;
  const int gx0 = xt * TX - hx, gz0 = zt * TZ - hz;
  const int t = threadIdx.x;
  const CoarseCoef k = L.c;

  // Zero the whole LDS region once (the outer ring stays zero).
  for (int q = t; q < LDSN; q += NT) su[q] = sw[q] = sp[q] = su2[q] = sw2[q] = 0.0;
  // Table-driven R: the x-weights of the region's rows and the z-weights
  // of its columns, 7 each.
  __shared__ double swt[TAB ? 7 * (RZM + RXM) : 1];
  static_assert(!TAB || 7 * (RZM + RXM) <= NT, "one weight per thread");
  if (TAB) {
    if (t < 7 * RZ) {
      const int b = t / 7;
      swt[t] = L.wx[7 * (int64_t)wrap(gz0 + b, nz) + (t - 7 * b)];
    } else if (t < 7 * (RZ + RX)) {
      const int a = (t - 7 * RZ) / 7;
      swt[7 * RZM + (t - 7 * RZ)] =
          L.wz[7 * (int64_t)wrap(gx0 + a, nx) + (t - 7 * RZ - 7 * a)];
    }
  }

  int qi[MPT];       // LDS index of each owned point, -1 if none
  int64_t gi[MPT];   // global index of each owned point (wrapped)
  int cflag[MPT];    // 1 if the point is in the tile interior and inside
                     // the grid (stored at the end)
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    const int q = t + m * NT;
    qi[m] = -1;
    gi[m] = 0;
    cflag[m] = 0;
    if (q < npts) {
      const int a = q % RX, b = q / RX;
      qi[m] = (b + 1) * SX + a + 1;
      gi[m] = (int64_t)wrap(gz0 + b, nz) * nx + wrap(gx0 + a, nx);
      const int x = xt * TX + a - hx, z = zt * TZ + b - hz;
      cflag[m] = (a >= hx && a < hx + TX && b >= hz && b < hz + TZ && x < nx &&
                  z < nz) ? 1 : 0;
    }
  }
  double vu[MPT], vw[MPT], vp[MPT];
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    if (qi[m] >= 0) {
      vu[m] = in[gi[m]];
      vw[m] = in[n + gi[m]];
      vp[m] = in[2 * n + gi[m]];
    }
  }
  __syncthreads();  // zeroing done before the region is filled
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    if (qi[m] >= 0) {
      su[qi[m]] = vu[m];
      sw[qi[m]] = vw[m];
      sp[qi[m]] = vp[m];
    }
  }
  __syncthreads();

  double Ru[MPT], Rw[MPT], Rp[MPT];
  const int dR = k.upwind_left ? -1 : 1;  // upwind neighbour offset
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    Ru[m] = Rw[m] = Rp[m] = 0.0;
    if (qi[m] < 0) continue;
    if (TAB) {
      const int q = qi[m];
      const int a = q % SX - 1, b = q / SX - 1;
      if (a < 2 || a >= RX - 2 || b < 2 || b >= RZ - 2) continue;
      const double* wx = swt + 7 * b;
      const double* wz = swt + 7 * RZM + 7 * a;
      double au = 0.0, aw = 0.0, ap = 0.0;
#pragma unroll
      for (int o = -3; o <= 3; ++o) {
        au += wx[o + 3] * su[q + o];
        aw += wx[o + 3] * sw[q + o];
        ap += wx[o + 3] * sp[q + o];
      }
#pragma unroll
      for (int o = -3; o <= 3; ++o) {
        au += wz[o + 3] * su[q + o * SX];
        aw += wz[o + 3] * sw[q + o * SX];
        ap += wz[o + 3] * sp[q + o * SX];
      }
      Ru[m] = au;
      Rw[m] = aw;
      Rp[m] = ap;
    } else if (computeR) {
      const int q = qi[m], qn = q + dR;
      // cR (q_i - q_{i-1}) for U >= 0, cR (q_{i+1} - q_i) for U < 0
      Ru[m] = k.cR * (dR < 0 ? su[q] - su[qn] : su[qn] - su[q]);
      Rw[m] = k.cR * (dR < 0 ? sw[q] - sw[qn] : sw[qn] - sw[q]);
      Rp[m] = k.cR * (dR < 0 ? sp[q] - sp[qn] : sp[qn] - sp[q]);
    } else {
      Ru[m] = Rg[gi[m]];
      Rw[m] = Rg[n + gi[m]];
      Rp[m] = Rg[2 * n + gi[m]];
    }
  }
  if (computeR && storeR) {
#pragma unroll
    for (int m = 0; m < MPT; ++m) {
      if (cflag[m]) {
        Rg[gi[m]] = Ru[m];
        Rg[n + gi[m]] = Rw[m];
        Rg[2 * n + gi[m]] = Rp[m];
      }
    }
  }

  const double dtau = k.dtau;
  double* cu = su;   // u, w of the current substep
  double* cw = sw;
  double* nu_ = su2; // u, w being written
  double* nw_ = sw2;
  for (int s = 0; s < L.nsub; ++s) {
#pragma unroll
    for (int m = 0; m < MPT; ++m) {
      if (qi[m] < 0) continue;
      const int q = qi[m];
      const double u = vu[m], w = vw[m];
      const double dpx = sp[q + 1] - sp[q - 1];
      const double dpz = sp[q + SX] - sp[q - SX];
      const double gxx = (cu[q + 1] + cu[q - 1]) - 2.0 * u;
      const double gzz = (cw[q + SX] + cw[q - SX]) - 2.0 * w;
      const double wx = (cw[q + SX + 1] - cw[q - SX + 1]) -
                        (cw[q + SX - 1] - cw[q - SX - 1]);
      const double uz = (cu[q + SX + 1] - cu[q + SX - 1]) -
                        (cu[q - SX + 1] - cu[q - SX - 1]);
      vu[m] = u + dtau * (Ru[m] - k.cx2 * dpx + k.kxx * gxx + k.kxzu * wx);
      vw[m] = w + dtau * (Rw[m] - k.cz2 * dpz + k.kzz * gzz + k.kxzw * uz);
      nu_[q] = vu[m];
      nw_[q] = vw[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MPT; ++m) {
      if (qi[m] < 0) continue;
      const int q = qi[m];
      const double dux = nu_[q + 1] - nu_[q - 1];
      const double dwz = nw_[q + SX] - nw_[q - SX];
      vp[m] = vp[m] + dtau * (Rp[m] - k.cx2 * dux - k.cz2 * dwz);
      sp[q] = vp[m];
    }
    __syncthreads();
    double* tu = cu;  // the buffers written become the current ones
    cu = nu_;
    nu_ = tu;
    double* tw = cw;
    cw = nw_;
    nw_ = tw;
  }

#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    if (cflag[m]) {
      out[gi[m]] = vu[m];
      out[n + gi[m]] = vw[m];
      out[2 * n + gi[m]] = vp[m];
    }
  }
}

}  // namespace

hipError_t launch_coarse(const CoarseLaunch& L, hipStream_t s) {
  if (L.nsub < 1 || L.nsub > kCoarseMaxSubPerLaunch || L.nstates < 1)
    return hipErrorInvalidValue;
  const bool tab = (L.flags & kCoarseTablesR) != 0;
  if (tab && (!L.wx || !L.wz)) return hipErrorInvalidValue;
  const int big = ((L.nx + 31) / 32) * ((L.nz + 31) / 32);
  auto pad8 = [](int t) { return (unsigned)(8 * ((t + 7) / 8)); };
  // The table-driven R has a halo 2 cells wider.  Few tiles (the paper's
  // 40 x 40 grids): 16 x 8 tiles, whose 36 x 28 region gives every thread
  // one point (the launch is latency-bound, so redundant halo work is
  // cheaper than more points per thread); otherwise 32 x 32 (a 32 x 16
  // tile would need more than the 128 VGPRs of a 1024-thread group).
  if (tab && (int64_t)big * L.nstates < 256) {
    const int tiles = ((L.nx + 15) / 16) * ((L.nz + 7) / 8);
    hipLaunchKernelGGL((k_coarse<16, 8, 1024, true>), dim3(pad8(tiles), L.nstates),
                       dim3(1024), 0, s, L);
  } else if (tab) {
    hipLaunchKernelGGL((k_coarse<32, 32, 1024, true>), dim3(pad8(big), L.nstates),
                       dim3(1024), 0, s, L);
  } else if ((int64_t)big * L.nstates < 256) {
    const int tiles = ((L.nx + 31) / 32) * ((L.nz + 15) / 16);
    hipLaunchKernelGGL((k_coarse<32, 16, 1024, false>), dim3(pad8(tiles), L.nstates),
                       dim3(1024), 0, s, L);
  } else {
    hipLaunchKernelGGL((k_coarse<32, 32, 1024, false>), dim3(pad8(big), L.nstates),
                       dim3(1024), 0, s, L);
  }
  return hipGetLastError();
}

}  // namespace prh
