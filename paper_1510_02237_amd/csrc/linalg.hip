// Dense FP64 kernels of the Krylov-subspace part of KSE-Parareal
// (Section 2.2): projections c = S^T x, the fine part of the modified coarse
// propagator F(P x) = sum_i alpha_i F(s_i) (eq. Genhance), and the
// orthonormalisation of the subspace update (eq. subspaceUpdate).
//
// Vectors of a block are stored one after the other (V[j*ld + x]); every
// reduction is split into fixed chunks and summed in a fixed order, so the
// results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pr_internal.h"

namespace prh {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GEMV_NT = 256;
constexpr int GEMV_E = 8;   // elements of x per thread (column norms)
constexpr int GEMV_JG = 8;  // columns per workgroup
constexpr int GEMV_CHUNK = GEMV_NT * GEMV_E;
constexpr int GEMV_RESIDENT = 256;  // workgroups of one c = V^T x launch
constexpr int LINCOMB_RESIDENT = 512;  // workgroups of one D c launch

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums v over the workgroup of NT threads; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += sh[q];
  }
  return s;
}

// c = V^T x, partial sums.  One workgroup per (group of GEMV_JG columns,
// slice of d) item, with few enough items (about one workgroup per compute
// unit) that the grid stays resident beside a concurrent coarse step, which
// then finds its compute units free.  Each thread keeps four elements of x
// and 4 * GEMV_JG column loads in flight and reduces once at the end:
// part[slice * ncols + j] = sum over the slice of V[j][x] x[x].
__global__ __launch_bounds__(GEMV_NT) void k_gemv_t(
    const double* __restrict__ V, int64_t ld, int ncols,
    const double* __restrict__ x, int64_t d, int nsl, int64_t len,
    double* __restrict__ part) {
  __shared__ double sh[GEMV_JG][GEMV_NT / 64];
  const int grp = blockIdx.x / nsl, sl = blockIdx.x % nsl;
  const int j0 = grp * GEMV_JG;
  const int64_t xs = (int64_t)sl * len;
  const int64_t xe = xs + len < d ? xs + len : d;
  const double* col[GEMV_JG];
#pragma unroll
  for (int q = 0; q < GEMV_JG; ++q)
    col[q] = V + (int64_t)(j0 + q < ncols ? j0 + q : ncols - 1) * ld;
  double acc[GEMV_JG];
#pragma unroll
  for (int q = 0; q < GEMV_JG; ++q) acc[q] = 0.0;
  int64_t i = xs + threadIdx.x;
  for (; i + 3 * GEMV_NT < xe; i += 4 * GEMV_NT) {
    double xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = x[i + u * GEMV_NT];
#pragma unroll
    for (int q = 0; q < GEMV_JG; ++q) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = col[q][i + u * GEMV_NT];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[q] += v[u] * xv[u];
    }
  }
  for (; i < xe; i += GEMV_NT) {
    const double xv = x[i];
#pragma unroll
    for (int q = 0; q < GEMV_JG; ++q) acc[q] += col[q][i] * xv;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < GEMV_JG; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) sh[q][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < GEMV_JG && j0 + (int)threadIdx.x < ncols) {
    double sacc = 0.0;
#pragma unroll
    for (int w = 0; w < GEMV_NT / 64; ++w) sacc += sh[threadIdx.x][w];
    part[(int64_t)sl * ncols + j0 + threadIdx.x] = sacc;
  }
}

template <int E>
__global__ __launch_bounds__(GEMV_NT) void k_colnorm2_part(
    const double* __restrict__ V, int64_t ld, int ncols, int64_t d,
    double* __restrict__ part) {
  __shared__ double sh[GEMV_JG][GEMV_NT / 64];
  const int64_t x0 = (int64_t)blockIdx.x * GEMV_NT * E;
  const int j0 = blockIdx.y * GEMV_JG;
  double acc[GEMV_JG];
#pragma unroll
  for (int q = 0; q < GEMV_JG; ++q) {
    acc[q] = 0.0;
    const int j = j0 + q < ncols ? j0 + q : ncols - 1;
    const double* col = V + (int64_t)j * ld;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t i = x0 + threadIdx.x + e * GEMV_NT;
      if (i < d) acc[q] += col[i] * col[i];
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < GEMV_JG; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) sh[q][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < GEMV_JG && j0 + (int)threadIdx.x < ncols) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < GEMV_NT / 64; ++w) s += sh[threadIdx.x][w];
    part[(int64_t)blockIdx.x * ncols + j0 + threadIdx.x] = s;
  }
}

// c[j] = sum_b part[b*ncols + j]: one wave per column; lane l sums the
// blocks l, l + 64, ... in order, then a fixed butterfly across the wave.
__global__ __launch_bounds__(256) void k_reduce_cols(
    const double* __restrict__ part, int nblk, int ncols,
    double* __restrict__ c) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= ncols) return;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += part[(int64_t)b * ncols + j];
  s = wave_sum(s);
  if (lane == 0) c[j] = s;
}

constexpr int COMB_NT = 256;
constexpr int COMB_E = 2;
constexpr int COMB_MAXC = 4096;

// nw = qt + (g + sum_j D[j] c[j]); delta = nw - q; q = nw.   (mode 0)
// out = g + sum_j D[j] c[j]                                   (mode 1)
template <int MODE>
__global__ __launch_bounds__(COMB_NT) void k_combine(
    double* __restrict__ q, double* __restrict__ delta,
    const double* __restrict__ qt, const double* __restrict__ g,
    const double* __restrict__ D, int64_t ld, int ncols,
    const double* __restrict__ c, int64_t d) {
  __shared__ double cs[COMB_MAXC];
  for (int j = threadIdx.x; j < ncols; j += COMB_NT) cs[j] = c[j];
  __syncthreads();
  const int64_t x0 = (int64_t)blockIdx.x * COMB_NT * COMB_E + threadIdx.x;
  double acc[COMB_E];
#pragma unroll
  for (int e = 0; e < COMB_E; ++e) acc[e] = 0.0;
  int j = 0;
  for (; j + 8 <= ncols; j += 8) {
    const double* d0 = D + (int64_t)j * ld;
#pragma unroll
    for (int e = 0; e < COMB_E; ++e) {
      const int64_t i = x0 + e * COMB_NT;
      if (i < d) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = d0[(int64_t)q * ld + i];
        acc[e] += ((v[0] * cs[j] + v[1] * cs[j + 1]) +
                   (v[2] * cs[j + 2] + v[3] * cs[j + 3])) +
                  ((v[4] * cs[j + 4] + v[5] * cs[j + 5]) +
                   (v[6] * cs[j + 6] + v[7] * cs[j + 7]));
      }
    }
  }
  for (; j + 4 <= ncols; j += 4) {
    const double c0 = cs[j], c1 = cs[j + 1], c2 = cs[j + 2], c3 = cs[j + 3];
    const double* d0 = D + (int64_t)j * ld;
    const double* d1 = d0 + ld;
    const double* d2 = d1 + ld;
    const double* d3 = d2 + ld;
#pragma unroll
    for (int e = 0; e < COMB_E; ++e) {
      const int64_t i = x0 + e * COMB_NT;
      if (i < d) acc[e] += (d0[i] * c0 + d1[i] * c1) + (d2[i] * c2 + d3[i] * c3);
    }
  }
  for (; j < ncols; ++j) {
    const double c0 = cs[j];
    const double* d0 = D + (int64_t)j * ld;
#pragma unroll
    for (int e = 0; e < COMB_E; ++e) {
      const int64_t i = x0 + e * COMB_NT;
      if (i < d) acc[e] += d0[i] * c0;
    }
  }
#pragma unroll
  for (int e = 0; e < COMB_E; ++e) {
    const int64_t i = x0 + e * COMB_NT;
    if (i >= d) continue;
    const double k = (g ? g[i] : 0.0) + acc[e];
    if (MODE == 0) {
      const double nw = qt[i] + k;
      if (delta) delta[i] = nw - q[i];
      q[i] = nw;
    } else {
      q[i] = k;
    }
  }
}

// out = g + sum_j D[j] c[j], with the per-element association of
// k_combine and a resident grid: workgroup b owns elements
// [b*len, (b+1)*len) and each thread four elements per pass, eight basis
// vectors per inner step (32 loads in flight).
__global__ __launch_bounds__(COMB_NT) void k_lincomb(
    double* __restrict__ out, const double* __restrict__ g,
    const double* __restrict__ D, int64_t ld, int ncols,
    const double* __restrict__ c, int64_t d, int64_t len) {
  __shared__ double cs[COMB_MAXC];
  for (int j = threadIdx.x; j < ncols; j += COMB_NT) cs[j] = c[j];
  __syncthreads();
  const int64_t xs = (int64_t)blockIdx.x * len;
  const int64_t xe = xs + len < d ? xs + len : d;
  for (int64_t x0 = xs + threadIdx.x; x0 < xe; x0 += 4 * COMB_NT) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int j = 0;
    for (; j + 8 <= ncols; j += 8) {
      const double* d0 = D + (int64_t)j * ld;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = x0 + e * COMB_NT;
        if (i < xe) {
          double v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = d0[(int64_t)q * ld + i];
          acc[e] += ((v[0] * cs[j] + v[1] * cs[j + 1]) +
                     (v[2] * cs[j + 2] + v[3] * cs[j + 3])) +
                    ((v[4] * cs[j + 4] + v[5] * cs[j + 5]) +
                     (v[6] * cs[j + 6] + v[7] * cs[j + 7]));
        }
      }
    }
    for (; j + 4 <= ncols; j += 4) {
      const double* d0 = D + (int64_t)j * ld;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = x0 + e * COMB_NT;
        if (i < xe)
          acc[e] += (d0[i] * cs[j] + d0[ld + i] * cs[j + 1]) +
                    (d0[2 * ld + i] * cs[j + 2] + d0[3 * ld + i] * cs[j + 3]);
      }
    }
    for (; j < ncols; ++j) {
      const double* d0 = D + (int64_t)j * ld;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = x0 + e * COMB_NT;
        if (i < xe) acc[e] += d0[i] * cs[j];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = x0 + e * COMB_NT;
      if (i < xe) out[i] = (g ? g[i] : 0.0) + acc[e];
    }
  }
}

// nw = qt + (g + y); delta = nw - q (if delta); q = nw.  Same association
// as k_combine<0> with y = sum_j D[j] c[j] computed beforehand.
// Optionally gacc += g (running G of the iterate being corrected).
__global__ __launch_bounds__(256) void k_combine3(
    double* __restrict__ q, double* __restrict__ delta,
    const double* __restrict__ qt, const double* __restrict__ g,
    const double* __restrict__ y, double* __restrict__ gacc, int64_t d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double gi = g ? g[i] : 0.0;
    const double k = gi + (y ? y[i] : 0.0);
    const double nw = qt[i] + k;
    if (delta) delta[i] = nw - q[i];
    q[i] = nw;
    if (gacc) gacc[i] += gi;
  }
}

__global__ void k_sub(double* __restrict__ y, const double* a,
                      const double* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] - b[i];
}

__global__ void k_check_finite(const double* __restrict__ v, int64_t n,
                               int* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(v[i]);
  if (bad) atomicOr(flag, 1);
}

// ----------------------------------------------------------------- GEMM TN
// C = A^T B over d, A = [M][lda], B = [N][ldb].  A workgroup of four waves
// owns a 64 x 64 tile of C and one chunk of d; each wave a 32 x 32 quarter
// made of 2 x 2 MFMA blocks (v_mfma_f64_16x16x4f64).  For the MFMA operands
// lane l supplies A[m0 + l%16][k] and B[k][n0 + l%16] at k-slot l/16; the
// k-slots of four consecutive instructions are mapped to four consecutive
// x so that each lane reads 32 contiguous bytes of its vector.  The output
// of a block sits in lane l, register i at row l/16 + 4*i, column l%16.
// Partial tiles of each chunk go to work[split][M][N], summed in order by
// k_reduce_splits.
constexpr int TN_T = 64;

__device__ __forceinline__ int xcd_logical(int nlogical) {
  const int b = blockIdx.x;
  const int per = (nlogical + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__global__ __launch_bounds__(256) void k_gemm_tn_mfma(
    const double* __restrict__ A, int64_t lda, int M,
    const double* __restrict__ B, int64_t ldb, int N, int64_t d,
    int64_t kc, int mt, int nt, int nsplit, double* __restrict__ work) {
  const int tiles = mt * nt;
  const int lb = xcd_logical(tiles * nsplit);
  if (lb >= tiles * nsplit) return;
  const int split = lb / tiles, tile = lb % tiles;
  const int tm = tile % mt, tn = tile / mt;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m0 = tm * TN_T + (wv >> 1) * 32;
  const int n0 = tn * TN_T + (wv & 1) * 32;
  // A quarter wholly beyond M or N has nothing to compute (N <= 32 leaves
  // half the waves of every tile idle); no barrier follows.
  if (m0 >= M || n0 >= N) return;
  const int64_t xs = (int64_t)split * kc;
  const int64_t xe = xs + kc < d ? xs + kc : d;
  const int r16 = lane & 15, kq = lane >> 4;
  int ra0 = m0 + r16, ra1 = m0 + 16 + r16;
  int rb0 = n0 + r16, rb1 = n0 + 16 + r16;
  ra0 = ra0 < M ? ra0 : M - 1;
  ra1 = ra1 < M ? ra1 : M - 1;
  rb0 = rb0 < N ? rb0 : N - 1;
  rb1 = rb1 < N ? rb1 : N - 1;
  const double* pa0 = A + (int64_t)ra0 * lda + 4 * kq;
  const double* pa1 = A + (int64_t)ra1 * lda + 4 * kq;
  const double* pb0 = B + (int64_t)rb0 * ldb + 4 * kq;
  const double* pb1 = B + (int64_t)rb1 * ldb + 4 * kq;
  d4 c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
  // The second 16-row (16-column) block of the quarter is computed only if
  // it reaches into M (N): an FP64 MFMA occupies the SIMD for 64 cycles,
  // and small blocks (M, N <= 16) would otherwise spend three quarters of
  // them on padding.  The blocks kept run the same MFMA sequence.
  const bool m1 = m0 + 16 < M, n1 = n0 + 16 < N;
  // lda, ldb are multiples of 16 and the buffers are zero beyond d, so the
  // loop runs over whole groups of 16 without a tail.  The operands of the
  // next group are loaded before the MFMAs of the current one, so each wave
  // keeps two groups of loads in flight.  The blocks not computed load
  // nothing (their operands stay zero and unused).
  const d4 z4 = {0, 0, 0, 0};
  d4 a0 = z4, b0 = z4, a1 = z4, b1 = z4;
  if (xs < xe) {
    a0 = *(const d4*)(pa0 + xs);
    b0 = *(const d4*)(pb0 + xs);
    if (m1) a1 = *(const d4*)(pa1 + xs);
    if (n1) b1 = *(const d4*)(pb1 + xs);
  }
  for (int64_t x = xs; x < xe; x += 16) {
    const d4 ca0 = a0, cb0 = b0, ca1 = a1, cb1 = b1;
    const int64_t xn = x + 16;
    if (xn < xe) {
      a0 = *(const d4*)(pa0 + xn);
      b0 = *(const d4*)(pb0 + xn);
      if (m1) a1 = *(const d4*)(pa1 + xn);
      if (n1) b1 = *(const d4*)(pb1 + xn);
    }
    if (m1 && n1) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca0[s], cb0[s], c00, 0, 0, 0);
        c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca0[s], cb1[s], c01, 0, 0, 0);
        c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca1[s], cb0[s], c10, 0, 0, 0);
        c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca1[s], cb1[s], c11, 0, 0, 0);
      }
    } else if (m1) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca0[s], cb0[s], c00, 0, 0, 0);
        c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca1[s], cb0[s], c10, 0, 0, 0);
      }
    } else if (n1) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca0[s], cb0[s], c00, 0, 0, 0);
        c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca0[s], cb1[s], c01, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca0[s], cb0[s], c00, 0, 0, 0);
    }
  }
  double* W = work + (int64_t)split * M * N;
  auto put = [&](const d4& v, int mb, int nb) {
    const int col = nb + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = mb + kq + 4 * i;
      if (row < M && col < N) W[(int64_t)row * N + col] = v[i];
    }
  };
  put(c00, m0, n0);
  put(c01, m0, n0 + 16);
  put(c10, m0 + 16, n0);
  put(c11, m0 + 16, n0 + 16);
}

// Plain-FMA variant with the same chunking (used to cross-check MFMA).
__global__ __launch_bounds__(256) void k_gemm_tn_fma(
    const double* __restrict__ A, int64_t lda, int M,
    const double* __restrict__ B, int64_t ldb, int N, int64_t d,
    int64_t kc, int mt, int nt, int nsplit, double* __restrict__ work) {
  const int tiles = mt * nt;
  const int lb = blockIdx.x;
  if (lb >= tiles * nsplit) return;
  const int split = lb / tiles, tile = lb % tiles;
  const int tm = tile % mt, tn = tile / mt;
  const int64_t xs = (int64_t)split * kc;
  const int64_t xe = xs + kc < d ? xs + kc : d;
  double* W = work + (int64_t)split * M * N;
  for (int q = threadIdx.x; q < TN_T * TN_T; q += 256) {
    const int m = tm * TN_T + q / TN_T, nn = tn * TN_T + q % TN_T;
    if (m >= M || nn >= N) continue;
    const double* a = A + (int64_t)m * lda;
    const double* b = B + (int64_t)nn * ldb;
    double s = 0.0;
    for (int64_t x = xs; x < xe; ++x) s += a[x] * b[x];
    W[(int64_t)m * N + nn] = s;
  }
}

// C[q] = sum_k work[k*mn + q]: one wave per output element, lanes over the
// splits in a fixed order, then a fixed butterfly.
__global__ __launch_bounds__(256) void k_reduce_splits(
    const double* __restrict__ work, int nsplit, int64_t mn,
    double* __restrict__ C) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= mn) return;
  double s = 0.0;
  for (int k = lane; k < nsplit; k += 64) s += work[(int64_t)k * mn + q];
  s = wave_sum(s);
  if (lane == 0) C[q] = s;
}

// ----------------------------------------------------------------- GEMM NN
// Y[l][x] = beta Y[l][x] + alpha sum_j A[j][x] C[j*ldc + l], l < N.
// Computed as the transposed product (N x 16 strip of x per wave):
// MFMA A-operand = C^T (lane l: C[(j0 + l/16)*ldc + l0 + l%16]) from LDS,
// B-operand = A (lane l: A[(j0 + l/16)*lda + x0 + l%16], 128-byte runs).
// Output lane l, register i: Y row l0 + l/16 + 4*i, column x0 + l%16, so
// each group of 16 lanes stores 128 contiguous bytes.
constexpr int NN_JC = 32;  // rows of C staged in LDS per pass

template <int NB>
__global__ __launch_bounds__(256) void k_gemm_nn_mfma(
    double* __restrict__ Y, int64_t ldy, const double* __restrict__ A,
    int64_t lda, int K, const double* __restrict__ C, int ldc, int N,
    int64_t d, double alpha, double beta) {
  __shared__ double cs[NN_JC][NB * 16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t x0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
  const int r16 = lane & 15, kq = lane >> 4;
  d4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = d4{0, 0, 0, 0};
  const bool active = x0 < d;
  const double* pa = A + x0 + r16;
  for (int j0 = 0; j0 < K; j0 += NN_JC) {
    __syncthreads();
    for (int q = threadIdx.x; q < NN_JC * NB * 16; q += 256) {
      const int jj = q / (NB * 16), l = q % (NB * 16);
      const int j = j0 + jj;
      cs[jj][l] = (j < K && l < N) ? C[(int64_t)j * ldc + l] : 0.0;
    }
    __syncthreads();
    if (active) {
      // All loads of the chunk are issued before its MFMAs, so that a wave
      // keeps NN_JC / 4 of them in flight; rows past K contribute zero
      // (their rows of C in LDS are zero too).
      double bv[NN_JC / 4];
#pragma unroll
      for (int u = 0; u < NN_JC / 4; ++u) {
        const int j = j0 + 4 * u + kq;
        bv[u] = j < K ? pa[(int64_t)j * lda] : 0.0;
      }
      const int jn = K - j0 < NN_JC ? K - j0 : NN_JC;
#pragma unroll
      for (int u = 0; u < NN_JC / 4; ++u) {
        if (4 * u >= jn) break;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double av = cs[4 * u + kq][b * 16 + r16];
          acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[u], acc[b], 0, 0, 0);
        }
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int l = b * 16 + kq + 4 * i;
      if (l < N) {
        double* y = Y + (int64_t)l * ldy + x0 + r16;
        const double v = alpha * acc[b][i];
        *y = beta == 0.0 ? v : beta * *y + v;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_gemm_nn_fma(
    double* __restrict__ Y, int64_t ldy, const double* __restrict__ A,
    int64_t lda, int K, const double* __restrict__ C, int ldc, int N,
    int64_t d, double alpha, double beta) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= d) return;
  for (int l = 0; l < N; ++l) {
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += A[(int64_t)j * lda + x] * C[(int64_t)j * ldc + l];
    double* y = Y + (int64_t)l * ldy + x;
    *y = beta == 0.0 ? alpha * s : beta * *y + alpha * s;
  }
}

// ------------------------------------------------------ pivoted Cholesky
// G = X^T X (b x b).  Left-looking Cholesky with diagonal pivoting on the
// remaining residual norms: L[k][i] (row-major, position-indexed) holds the
// factor; perm maps positions to columns of X.  With pivoting, column k is
// accepted while its residual exceeds max(abs2, rel2 * n0[col]), where
// abs2 = rank_tol2 * max(r11sq, max n0) and r11sq is updated in place.
// Then R = L^T restricted to the rank, Rinv by back substitution per
// column, and T[perm[i]][c] = Rinv[i][c].
constexpr int PC_NT = 256;

__global__ __launch_bounds__(PC_NT) void k_pchol(
    const double* __restrict__ G, int b, const double* __restrict__ n0,
    double* r11sq, double rank_tol2, double rel2, int pivot,
    double* __restrict__ T, int* rank_out, double* __restrict__ work) {
  double* L = work;                 // b*b
  double* diag = work + (int64_t)b * b;  // b
  int* perm = (int*)(diag + b);     // b
  __shared__ double sv[PC_NT];
  __shared__ int si[PC_NT];
  __shared__ double s_abs2;
  __shared__ int s_rank, s_piv;
  const int t = threadIdx.x;

  for (int q = t; q < b; q += PC_NT) {
    diag[q] = G[(int64_t)q * b + q];
    perm[q] = q;
  }
  if (t == 0) {
    double m = r11sq ? *r11sq : 0.0;
    if (pivot && n0)
      for (int q = 0; q < b; ++q) m = fmax(m, n0[q]);
    if (r11sq && pivot) *r11sq = m;
    s_abs2 = rank_tol2 * m;
    s_rank = b;
  }
  __syncthreads();

  for (int k = 0; k < b; ++k) {
    int p = k;
    if (pivot) {
      double best = -1.0;
      int bi = k;
      for (int q = k + t; q < b; q += PC_NT) {
        if (diag[q] > best) { best = diag[q]; bi = q; }
      }
      sv[t] = best;
      si[t] = bi;
      __syncthreads();
      for (int o = PC_NT / 2; o > 0; o >>= 1) {
        if (t < o) {
          const double v2 = sv[t + o];
          const int i2 = si[t + o];
          if (v2 > sv[t] || (v2 == sv[t] && i2 < si[t])) {
            sv[t] = v2;
            si[t] = i2;
          }
        }
        __syncthreads();
      }
      if (t == 0) {
        const int pp = si[0];
        const double thr = fmax(s_abs2, rel2 * n0[perm[pp]]);
        s_piv = sv[0] > thr ? pp : -1;
      }
      __syncthreads();
      p = s_piv;
      if (p < 0) {
        if (t == 0) s_rank = k;
        break;
      }
      if (p != k) {
        // swap positions k and p: factor rows (columns < k), diag, perm
        for (int i = t; i < k; i += PC_NT) {
          const double a = L[(int64_t)k * b + i];
          L[(int64_t)k * b + i] = L[(int64_t)p * b + i];
          L[(int64_t)p * b + i] = a;
        }
        if (t == 0) {
          const double a = diag[k];
          diag[k] = diag[p];
          diag[p] = a;
          const int pi = perm[k];
          perm[k] = perm[p];
          perm[p] = pi;
        }
        __syncthreads();
      }
    } else {
      if (t == 0) s_piv = diag[k] > 0.0 ? k : -1;
      __syncthreads();
      if (s_piv < 0) {
        if (t == 0) s_rank = k;
        break;
      }
    }
    const double lkk = sqrt(diag[k]);
    const int ck = perm[k];
    // column k of the factor for positions j > k (left-looking)
    for (int jj = k + 1 + t; jj < b; jj += PC_NT) {
      const int cj = perm[jj];
      double s = G[(int64_t)cj * b + ck];
      for (int i = 0; i < k; ++i) s -= L[(int64_t)jj * b + i] * L[(int64_t)k * b + i];
      const double l = s / lkk;
      L[(int64_t)jj * b + k] = l;
      diag[jj] -= l * l;
    }
    if (t == 0) L[(int64_t)k * b + k] = lkk;
    __syncthreads();
  }
  __syncthreads();
  const int rho = s_rank;
  // T = Pi R^{-1}; R[i][m] = L[m][i] for i <= m < rho.
  for (int q = t; q < b * b; q += PC_NT) T[q] = 0.0;
  __syncthreads();
  for (int cc = t; cc < rho; cc += PC_NT) {
    // column cc of Rinv, rows cc down to 0, kept in T through perm
    // Rinv[i][cc] is stored at T[perm[i]][cc]; this thread owns column cc.
    const double rcc = L[(int64_t)cc * b + cc];
    T[(int64_t)perm[cc] * b + cc] = 1.0 / rcc;
    for (int i = cc - 1; i >= 0; --i) {
      double s = 0.0;
      for (int m = i + 1; m <= cc; ++m)
        s += L[(int64_t)m * b + i] * T[(int64_t)perm[m] * b + cc];
      T[(int64_t)perm[i] * b + cc] = -s / L[(int64_t)i * b + i];
    }
  }
  if (t == 0) *rank_out = rho;
}

// Same factorisation for b <= BMAX by one wavefront with the factor L, the
// Gram matrix (when it fits) and R^{-1} in LDS: the pivot search is a wave
// reduction, and no workgroup barrier is needed inside the factorisation.
// L is stored by columns (Lc[i][j] = L[j][i]) and the Gram read by rows, so
// the lanes of a wave, one per position j, touch consecutive LDS words.
// R^{-1} is formed by back substitution one row at a time, lane c owning
// column c: row i of R^{-1} needs rows i+1.. of its own column only.
template <int BMAX, bool GLDS>
__global__ __launch_bounds__(64) void k_pchol_wave(
    const double* __restrict__ G, int b, const double* __restrict__ n0,
    double* r11sq, double rank_tol2, double rel2, int pivot,
    double* __restrict__ T, int* rank_out) {
  __shared__ double Lc[BMAX * BMAX];
  __shared__ double Gs[GLDS ? BMAX * BMAX : 1];
  __shared__ double diag[BMAX];
  __shared__ int perm[BMAX];
  const int t = threadIdx.x;
  if (GLDS)
    for (int q = t; q < b * b; q += 64) Gs[(q / b) * BMAX + q % b] = G[q];
  for (int q = t; q < b; q += 64) {
    diag[q] = G[(int64_t)q * b + q];
    perm[q] = q;
  }
  // G is symmetric: entry (ck, j) is read along row ck.
  auto grow = [&](int i, int j) {
    return GLDS ? Gs[i * BMAX + j] : G[(int64_t)i * b + j];
  };
  double m = 0.0;
  if (pivot && n0)
    for (int q = t; q < b; q += 64) m = fmax(m, n0[q]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if (r11sq) m = fmax(m, *r11sq);
  const double abs2 = rank_tol2 * m;
  __syncthreads();
  if (t == 0 && r11sq && pivot) *r11sq = m;
  int rho = b;
  for (int k = 0; k < b; ++k) {
    if (pivot) {
      // The search starts at position k, a valid index: when no diagonal
      // exceeds -1 (a non-finite Gram) the reduction returns k, its
      // threshold test fails and the factorisation ends with rank k.
      double best = -1.0;
      int bi = k;
      for (int q = k + t; q < b; q += 64)
        if (diag[q] > best) { best = diag[q]; bi = q; }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(best, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (v2 > best || (v2 == best && i2 < bi)) { best = v2; bi = i2; }
      }
      const int p = bi;
      const double thr = fmax(abs2, rel2 * n0[perm[p]]);
      if (!(best > thr)) { rho = k; break; }
      if (p != k) {
        for (int i = t; i < k; i += 64) {
          const double a = Lc[i * BMAX + k];
          Lc[i * BMAX + k] = Lc[i * BMAX + p];
          Lc[i * BMAX + p] = a;
        }
        __syncthreads();
        if (t == 0) {
          const double a = diag[k]; diag[k] = diag[p]; diag[p] = a;
          const int pi = perm[k]; perm[k] = perm[p]; perm[p] = pi;
        }
        __syncthreads();
      }
    } else if (!(diag[k] > 0.0)) {
      rho = k;
      break;
    }
    const double lkk = sqrt(diag[k]);
    const int ck = perm[k];
    for (int jj = k + 1 + t; jj < b; jj += 64) {
      double sacc = grow(ck, perm[jj]);
      for (int i = 0; i < k; ++i) sacc -= Lc[i * BMAX + jj] * Lc[i * BMAX + k];
      const double l = sacc / lkk;
      Lc[k * BMAX + jj] = l;
      diag[jj] -= l * l;
    }
    if (t == 0) Lc[k * BMAX + k] = lkk;
    __syncthreads();
  }
  // X = R^{-1} (upper triangular, R[i][mm] = Lc[i][mm]).  With the Gram in
  // LDS, X takes its place; T[perm[i]][c] = X[i][c] at the end.  Otherwise X
  // is built in T directly through perm.
  __syncthreads();
  auto xat = [&](int i, int c) -> double& {
    return GLDS ? Gs[i * BMAX + c] : T[(int64_t)perm[i] * b + c];
  };
  if (!GLDS) {
    for (int q = t; q < b * b; q += 64) T[q] = 0.0;
    __syncthreads();
  }
  for (int c = t; c < rho; c += 64) {
    for (int i = rho - 1; i >= 0; --i) {
      if (i > c) {
        if (GLDS) xat(i, c) = 0.0;
        continue;
      }
      double sacc = i == c ? 1.0 : 0.0;
      for (int mm = i + 1; mm <= c; ++mm) sacc -= Lc[i * BMAX + mm] * xat(mm, c);
      xat(i, c) = sacc / Lc[i * BMAX + i];
    }
  }
  __syncthreads();
  if (GLDS) {
    for (int q = t; q < b * b; q += 64) {
      const int i = q / b, c = q % b;  // position i, column c
      T[(int64_t)perm[i] * b + c] = (i < rho && c < rho) ? Gs[i * BMAX + c] : 0.0;
    }
  }
  if (t == 0) *rank_out = rho;
}

__global__ void k_small_matmul(const double* __restrict__ T1, int b, int rho1,
                               const double* __restrict__ T2, int rho2,
                               double* __restrict__ T3) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= b * b) return;
  const int i = q / b, c = q % b;
  double s = 0.0;
  if (c < rho2)
    for (int m = 0; m < rho1; ++m)
      s += T1[(int64_t)i * b + m] * T2[(int64_t)m * rho1 + c];
  T3[q] = s;
}

}  // namespace

int gemv_t_blocks(int64_t d) { return (int)((d + GEMV_CHUNK - 1) / GEMV_CHUNK); }

// Below 64 chunks of d the column norms take one element per thread, so
// that small states (the paper's 40 x 40 grids: d = 4800) spread over more
// workgroups instead of a few long dependent chains.
int colnorm_blocks(int64_t d) {
  return d < 64 * (int64_t)GEMV_CHUNK ? (int)((d + GEMV_NT - 1) / GEMV_NT)
                                      : gemv_t_blocks(d);
}

namespace {
// Slices of d for a projection onto ncols vectors: about GEMV_RESIDENT
// workgroups in all, each slice at least GEMV_CHUNK elements.
int gemv_slices(int64_t d, int ncols) {
  const int ngrp = (ncols + GEMV_JG - 1) / GEMV_JG;
  int nsl = GEMV_RESIDENT / ngrp;
  const int64_t cap = (d + GEMV_CHUNK - 1) / GEMV_CHUNK;
  if (nsl > cap) nsl = (int)cap;
  return nsl < 1 ? 1 : nsl;
}
}  // namespace

size_t gemv_t_part(int64_t d, int ncols) {
  return (size_t)gemv_slices(d, ncols) * (size_t)(ncols > 0 ? ncols : 0);
}

hipError_t launch_gemv_t(const double* V, int64_t ld, int ncols,
                         const double* x, int64_t d, double* part, double* c,
                         hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  const int nsl = gemv_slices(d, ncols);
  const int ngrp = (ncols + GEMV_JG - 1) / GEMV_JG;
  int64_t len = (d + nsl - 1) / nsl;
  len = (len + GEMV_NT - 1) / GEMV_NT * GEMV_NT;
  hipLaunchKernelGGL(k_gemv_t, dim3(ngrp * nsl), dim3(GEMV_NT), 0, s, V, ld,
                     ncols, x, d, nsl, len, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_cols(part, nsl, ncols, c, s);
}

hipError_t launch_reduce_cols(const double* part, int nblk, int ncols,
                              double* c, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_cols, dim3((ncols + 3) / 4), dim3(256), 0, s,
                     part, nblk, ncols, c);
  return hipGetLastError();
}

hipError_t launch_colnorm2(const double* V, int64_t ld, int ncols, int64_t d,
                           double* part, double* nrm2, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  const int nblk = colnorm_blocks(d);
  const dim3 grid(nblk, (ncols + GEMV_JG - 1) / GEMV_JG);
  if (nblk == gemv_t_blocks(d))
    hipLaunchKernelGGL(k_colnorm2_part<GEMV_E>, grid, dim3(GEMV_NT), 0, s, V,
                       ld, ncols, d, part);
  else
    hipLaunchKernelGGL(k_colnorm2_part<1>, grid, dim3(GEMV_NT), 0, s, V, ld,
                       ncols, d, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_cols(part, nblk, ncols, nrm2, s);
}

hipError_t launch_combine(double* q, double* delta_out, const double* qt,
                          const double* g, const double* D, int64_t ld,
                          int ncols, const double* c, int64_t d,
                          hipStream_t s) {
  if (ncols > COMB_MAXC) return hipErrorInvalidValue;
  const int64_t per = (int64_t)COMB_NT * COMB_E;
  hipLaunchKernelGGL(k_combine<0>, dim3((unsigned)((d + per - 1) / per)),
                     dim3(COMB_NT), 0, s, q, delta_out, qt, g, D, ld, ncols,
                     c, d);
  return hipGetLastError();
}

hipError_t launch_lincomb(double* out, const double* g, const double* D,
                          int64_t ld, int ncols, const double* c, int64_t d,
                          hipStream_t s) {
  if (ncols > COMB_MAXC) return hipErrorInvalidValue;
  if (d <= 0) return hipSuccess;
  // About LINCOMB_RESIDENT workgroups (few enough to stay resident, see
  // k_gemv_t; enough loads in flight), at least 1024 elements each.
  int64_t nb = (d + 1023) / 1024;
  if (nb > LINCOMB_RESIDENT) nb = LINCOMB_RESIDENT;
  int64_t len = (d + nb - 1) / nb;
  len = (len + COMB_NT - 1) / COMB_NT * COMB_NT;
  nb = (d + len - 1) / len;
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)nb), dim3(COMB_NT), 0, s, out,
                     g, D, ld, ncols, c, d, len);
  return hipGetLastError();
}

hipError_t launch_combine3(double* q, double* delta_out, const double* qt,
                           const double* g, const double* y, double* gacc,
                           int64_t d, hipStream_t s) {
  int64_t blocks = (d + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_combine3, dim3((unsigned)blocks), dim3(256), 0, s, q,
                     delta_out, qt, g, y, gacc, d);
  return hipGetLastError();
}

hipError_t launch_sub(double* y, const double* a, const double* b, int64_t n,
                      hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_sub, dim3((unsigned)blocks), dim3(256), 0, s, y, a, b, n);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* v, int64_t n, int* flag,
                               hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, s,
                     v, n, flag);
  return hipGetLastError();
}

namespace {
// Most splits of d: at least 1024 elements a split, but down to 256 while
// that leaves at most 64 splits, so that small problems still spread over
// several compute units.
// Splits of d for a product with `tiles` 64 x 64 tiles: about 1024
// workgroups, chunks of at least 1024 elements (or 256 for small d).
int64_t tn_tile_splits(int64_t d, int tiles) {
  const int64_t big = (d + 1023) / 1024, small = (d + 255) / 256;
  const int64_t maxs = std::max<int64_t>(big, std::min<int64_t>(small, 64));
  return std::max<int64_t>(1, std::min<int64_t>((1024 + tiles - 1) / tiles, maxs));
}

// Shortest chunk of a small product: 512 elements, or d / 64 (at least 64)
// on small states, which would otherwise give only a few workgroups.
int64_t tn_min_chunk(int64_t d) {
  return std::max<int64_t>(64, std::min<int64_t>(512, d / 64));
}

// Upper bound of the splits tn_shape picks at this d.
int64_t tn_max_splits(int64_t d) {
  const int64_t mc = tn_min_chunk(d);
  return std::max<int64_t>(tn_tile_splits(d, 1), (d + mc - 1) / mc);
}

void tn_shape(int M, int N, int64_t d, int* mt, int* nt, int* nsplit,
              int64_t* kc) {
  *mt = (M + TN_T - 1) / TN_T;
  *nt = (N + TN_T - 1) / TN_T;
  const int tiles = *mt * *nt;
  int64_t ns = tn_tile_splits(d, tiles);
  // A wave computes one 32 x 32 quarter of a tile, and quarters beyond M
  // or N exit at once.  A small product (one or two active quarters per
  // split) takes more, shorter chunks, down to tn_min_chunk(d) elements, so
  // that about 1024 waves load operands at once; the partials to sum grow
  // with them.  active >= tiles, so ns stays <= ceil(1024 / tiles).
  const int64_t active = (int64_t)((M + 31) / 32) * ((N + 31) / 32);
  const int64_t mc = tn_min_chunk(d);
  if (active <= 2)
    ns = std::max<int64_t>(ns, std::min<int64_t>((1024 + active - 1) / active,
                                                 (d + mc - 1) / mc));
  int64_t k = (d + ns - 1) / ns;
  k = (k + 15) / 16 * 16;
  *kc = k;
  *nsplit = (int)((d + k - 1) / k);
}
}  // namespace

// Upper bound of nsplit * M * N over every M <= Mmax, N <= Nmax at this d:
// nsplit <= ceil(1024 / tiles) with M N <= 4096 tiles gives
// (1024 + tiles) * 4096, and nsplit <= tn_max_splits(d) gives the second
// bound.
size_t gemm_tn_work(int Mmax, int Nmax, int64_t d) {
  const int64_t tiles = (int64_t)((Mmax + TN_T - 1) / TN_T) * ((Nmax + TN_T - 1) / TN_T);
  const int64_t a = (1024 + tiles) * TN_T * TN_T;
  const int64_t b = tn_max_splits(d) * (int64_t)Mmax * Nmax;
  return (size_t)std::min(a, b);
}

hipError_t launch_gemm_tn(const double* A, int64_t lda, int M,
                          const double* B, int64_t ldb, int N, int64_t d,
                          double* C, double* work, bool use_mfma,
                          hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (lda % 16 || ldb % 16) return hipErrorInvalidValue;
  int mt, nt, ns;
  int64_t kc;
  tn_shape(M, N, d, &mt, &nt, &ns, &kc);
  const int nlog = mt * nt * ns;
  if (use_mfma)
    hipLaunchKernelGGL(k_gemm_tn_mfma, dim3(8 * ((nlog + 7) / 8)), dim3(256),
                       0, s, A, lda, M, B, ldb, N, d, kc, mt, nt, ns, work);
  else
    hipLaunchKernelGGL(k_gemm_tn_fma, dim3(nlog), dim3(256), 0, s, A, lda, M,
                       B, ldb, N, d, kc, mt, nt, ns, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t mn = (int64_t)M * N;
  hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((mn + 3) / 4)),
                     dim3(256), 0, s, work, ns, mn, C);
  return hipGetLastError();
}

hipError_t launch_gemm_nn(double* Y, int64_t ldy, const double* A,
                          int64_t lda, int K, const double* C, int ldc, int N,
                          int64_t d, double alpha, double beta, bool use_mfma,
                          hipStream_t s) {
  if (N <= 0) return hipSuccess;
  if (N > 128) return hipErrorInvalidValue;
  if (!use_mfma) {
    hipLaunchKernelGGL(k_gemm_nn_fma, dim3((unsigned)((d + 255) / 256)),
                       dim3(256), 0, s, Y, ldy, A, lda, K, C, ldc, N, d,
                       alpha, beta);
    return hipGetLastError();
  }
  const unsigned grid = (unsigned)((d + 63) / 64);
  const int nb = (N + 15) / 16;
#define PR_NN(NBV)                                                          \
  hipLaunchKernelGGL(k_gemm_nn_mfma<NBV>, dim3(grid), dim3(256), 0, s, Y,   \
                     ldy, A, lda, K, C, ldc, N, d, alpha, beta)
  if (nb <= 1) PR_NN(1);
  else if (nb <= 2) PR_NN(2);
  else if (nb <= 4) PR_NN(4);
  else PR_NN(8);
#undef PR_NN
  return hipGetLastError();
}

hipError_t launch_pchol(const double* G, int b, const double* n0,
                        double* r11sq, double rank_tol2, double rel2,
                        int pivot, double* T, int* rank, double* work,
                        hipStream_t s) {
  if (b <= 64)
    hipLaunchKernelGGL((k_pchol_wave<64, true>), dim3(1), dim3(64), 0, s, G, b,
                       n0, r11sq, rank_tol2, rel2, pivot, T, rank);
  else if (b <= 128)
    hipLaunchKernelGGL((k_pchol_wave<128, false>), dim3(1), dim3(64), 0, s, G,
                       b, n0, r11sq, rank_tol2, rel2, pivot, T, rank);
  else
    hipLaunchKernelGGL(k_pchol, dim3(1), dim3(PC_NT), 0, s, G, b, n0, r11sq,
                       rank_tol2, rel2, pivot, T, rank, work);
  return hipGetLastError();
}

hipError_t launch_small_matmul(const double* T1, int b, int rho1,
                               const double* T2, int rho2, double* T3,
                               hipStream_t s) {
  const int n = b * b;
  hipLaunchKernelGGL(k_small_matmul, dim3((n + 255) / 256), dim3(256), 0, s,
                     T1, b, rho1, T2, rho2, T3);
  return hipGetLastError();
}

}  // namespace prh
