// Internal interfaces of libpararealhip: kernel parameter blocks and the
// host-side launchers of the HIP kernels.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace prh {

// ---------------------------------------------------------------------------
// Fine propagator (Section 3.2: non-split three-stage Runge-Kutta with
// 5th-order upwind advection, 4th-order centred acoustic terms and
// divergence damping alpha = nu_f h^2 / dt_f, eq. dampingCoeff).
// ---------------------------------------------------------------------------

// Point-stencil weights of the fine right-hand side on one grid.
//   f_u = sum_k adv[k] u(i+m0+k) - cx4 (p(i-2) - 8p(i-1) + 8p(i+1) - p(i+2))
//         + kxx (u(i+1) - 2u + u(i-1))
//         + kxzu (w(i+1,j+1) - w(i+1,j-1) - w(i-1,j+1) + w(i-1,j-1))
//   f_w = sum_k adv[k] w(i+m0+k) - cz4 (p(j-2) - 8p(j-1) + 8p(j+1) - p(j+2))
//         + kzz (w(j+1) - 2w + w(j-1))
//         + kxzw (u(i+1,j+1) - u(i-1,j+1) - u(i+1,j-1) + u(i-1,j-1))
//   f_p = sum_k adv[k] p(i+m0+k) - cx4 (u(i-2) - 8u(i-1) + 8u(i+1) - u(i+2))
//         - cz4 (w(j-2) - 8w(j-1) + 8w(j+1) - w(j+2))
// m0 = -3 for U >= 0 and -2 for U < 0 (upwind side).
struct FineCoef {
  double adv[6];
  double cx4, cz4;
  double kxx, kxzu, kzz, kxzw;
  double dt;
};

// One group of slices of one problem advanced by one RK-3 step.
struct FineJob {
  const double* in;      // [nslices][3][nz][nx]
  double* out;           // [nslices][3][nz][nx]
  int64_t in_stride;     // doubles between consecutive input slices
  int64_t out_stride;
  int32_t nx, nz, nslices;
  int32_t xtiles, ztiles;
  int32_t block_begin;   // first logical workgroup of this job
  FineCoef c;
};

constexpr int kMaxFineJobs = 12;

// Kernel argument of one fused-step launch; every job shares the sign of U
// and the tile shape.
struct FineLaunch {
  int32_t njobs;
  int32_t nblocks;       // logical workgroups over all jobs
  int32_t zc;            // output rows per workgroup
  FineJob job[kMaxFineJobs];
};

// Output columns per workgroup of the fused step kernel with nt threads:
// the three stages consume a halo of 15 columns (3 on the upwind side and
// 2 on the other, per stage).
// Rows of nx in {128, 256, 512} can be spanned by one workgroup (nt = nx):
// the full-row variant has no x-halo.
bool fine_full_row(int nx);
// Output columns of one workgroup of nt threads on rows of nx points.
inline int fine_tile_cols(int nt, int nx) {
  return (nt == nx && fine_full_row(nx)) ? nt : nt - 15;
}
bool fine_nt_supported(int nt, int nx);
// Workgroups of the fused step kernel with nt threads that one compute unit
// holds at once (registers and LDS), 0 if unknown.
int fine_blocks_per_cu(int nt, int nx, int sgn);

// One fused RK-3 step for every job (all three stages in one pass over the
// data, z-marching with LDS row rings).  sgn = +1 for U >= 0, -1 for U < 0.
hipError_t launch_fine_step(const FineLaunch& L, int nt, int sgn,
                            hipStream_t s);

// One RK-3 stage over nslices states (unfused form, reads neighbours from
// global memory): out = base + beta * f(in); each array has its own slice
// stride.
hipError_t launch_fine_stage(const double* in, int64_t in_stride,
                             const double* base, int64_t base_stride,
                             double* out, int64_t out_stride, int nx, int nz,
                             int nslices, const FineCoef& c, double beta,
                             int sgn, hipStream_t s);

// ---------------------------------------------------------------------------
// Stage kernel with advective weights per row and per column (the Section
// 3.1 propagator pair; the Section 3.2 propagators with an advection
// velocity that varies in space, eq. adVel):
//   f(q)_field = sum_{m=-3..3} (wx[j][m] q(i+m, j) + wz[i][m] q(i, j+m))
//              - acoustic centred differences + grad-div damping
// (see stage.hip for the acoustic and damping terms).
// ---------------------------------------------------------------------------
struct StageCoef {
  const double* wx;      // device, [nz][7]: x-weights of row j, offsets -3..3
  const double* wz;      // device, [nx][7]: z-weights of column i
  double ax1, ax2;       // acoustic x-difference ax1 d1x + ax2 d2x (times c_s)
  double az1, az2;       // acoustic z-difference
  double kxx, kxzu, kzz, kxzw;  // damping weights as in FineCoef (0 = none)
};

// One RK-3 step of the same right-hand side: out = q + beta3 f(q2) with
// q2 = q + beta2 f(q1), q1 = q + beta1 f(q), q = in; one launch, tiles of
// 16 x 16 points with their halo in LDS.  in and out must not alias.
hipError_t launch_stage3(const double* in, int64_t in_stride, double* out,
                         int64_t out_stride, int nx, int nz, int nstates,
                         const StageCoef& c, double beta1, double beta2,
                         double beta3, hipStream_t s);

// ---------------------------------------------------------------------------
// Coarse propagator (Section 3.2: partially split forward Euler; the slow
// advective tendency -U * (first-order upwind derivative) is frozen over
// N_sound forward-backward acoustic substeps with divergence damping
// alpha = nu_c h^2 / (Delta t / N_sound)).
// ---------------------------------------------------------------------------
struct CoarseCoef {
  double cR;             // -U/dx; slow tendency cR*(q_i - q_{i-1}) for U>=0,
                         // cR*(q_{i+1} - q_i) for U<0
  double dtau;           // Delta t / N_sound
  double cx2, cz2;       // c_s/(2 dx), c_s/(2 dz)
  double kxx, kxzu, kzz, kxzw;  // damping weights as in FineCoef
  int32_t upwind_left;   // 1 if U >= 0
};

struct CoarseLaunch {
  const double* in;      // [nstates][3][nz][nx]
  double* out;           // [nstates][3][nz][nx]; may not alias in
  double* R;             // [nstates][3][nz][nx] frozen slow tendency
  int64_t stride;        // doubles between states (all three arrays)
  int32_t nx, nz, nstates;
  int32_t nsub;          // acoustic substeps done by this launch
  int32_t flags;         // kCoarseComputeR or kCoarseTablesR, either with
                         // kCoarseStoreR; or 0 = load R
  CoarseCoef c;
  const double* wx;      // kCoarseTablesR: device, [nz][7] x-weights of the
  const double* wz;      // slow tendency per row, [nx][7] z-weights per
                         // column (offsets -3..3; nonzero within -2..2)
};
constexpr int kCoarseComputeR = 1;
constexpr int kCoarseStoreR = 2;
constexpr int kCoarseTablesR = 4;  // R = sum of the row and column weights
                                   // times q, evaluated in the launch
constexpr int kCoarseMaxSubPerLaunch = 4;

hipError_t launch_coarse(const CoarseLaunch& L, hipStream_t s);

// ---------------------------------------------------------------------------
// Dense linear algebra on tall-skinny FP64 blocks.  A block of n vectors of
// length d is stored vector after vector: V[j*ld + x].
// ---------------------------------------------------------------------------

// Chunks of d of the projections' partials (launch_gemv_t uses at most
// this many slices).
int gemv_t_blocks(int64_t d);
// Partials per column of launch_colnorm2 (>= gemv_t_blocks(d)): one per 256
// elements below 64 chunks, else gemv_t_blocks(d).  Not monotone in d.
int colnorm_blocks(int64_t d);
// c = V^T x (deterministic: fixed slices of d, partial sums in part, summed
// in a fixed order).  part needs gemv_t_part(d, ncols) doubles, at most
// max(2048, ncols).
size_t gemv_t_part(int64_t d, int ncols);
hipError_t launch_gemv_t(const double* V, int64_t ld, int ncols,
                         const double* x, int64_t d, double* part, double* c,
                         hipStream_t s);
// c[j] = sum_b part[b*ncols + j] in a fixed order.
hipError_t launch_reduce_cols(const double* part, int nblk, int ncols,
                              double* c, hipStream_t s);

// Serial-correction combine (delta form of the correction step):
//   nw = qt + g + sum_j D[j] c[j];  if (delta_out) delta_out = nw - q;  q = nw
// with g and D optional (NULL / ncols = 0).
hipError_t launch_combine(double* q, double* delta_out, const double* qt,
                          const double* g, const double* D, int64_t ld,
                          int ncols, const double* c, int64_t d,
                          hipStream_t s);
// Serial-correction combine with the fine part precomputed:
//   nw = qt + (g + y);  if (delta_out) delta_out = nw - q;  q = nw;
//   if (gacc) gacc += g
// (g, y, gacc optional).
hipError_t launch_combine3(double* q, double* delta_out, const double* qt,
                           const double* g, const double* y, double* gacc,
                           int64_t d, hipStream_t s);
// out = g + sum_j D[j] c[j] (out may alias g).
hipError_t launch_lincomb(double* out, const double* g, const double* D,
                          int64_t ld, int ncols, const double* c, int64_t d,
                          hipStream_t s);
// y = a - b over n doubles (y may alias a or b).
hipError_t launch_sub(double* y, const double* a, const double* b, int64_t n,
                      hipStream_t s);
// flag[0] |= 1 if any of the n doubles is not finite.
hipError_t launch_check_finite(const double* v, int64_t n, int* flag,
                               hipStream_t s);
// nrm2[j] = ||V[j]||^2 (deterministic; uses part[colnorm_blocks(d)*ncols]).
hipError_t launch_colnorm2(const double* V, int64_t ld, int ncols, int64_t d,
                           double* part, double* nrm2, hipStream_t s);

// C (M x N, row-major, ldc = N) = A^T B for A = [M][d] and B = [N][d]
// (Gram-type product, FP64 MFMA, split over d with a fixed-order reduction).
// work needs gemm_tn_work(Mmax, Nmax, d) doubles for any M <= Mmax,
// N <= Nmax; lda and ldb are multiples of 16 and both blocks are zero from
// d up to the next multiple of 16.
size_t gemm_tn_work(int M, int N, int64_t d);
hipError_t launch_gemm_tn(const double* A, int64_t lda, int M,
                          const double* B, int64_t ldb, int N, int64_t d,
                          double* C, double* work, bool use_mfma,
                          hipStream_t s);

// Y[l][x] = beta Y[l][x] + alpha sum_{j<K} A[j][x] C[j*ldc + l] for l < N
// (update-type product, FP64 MFMA).  Y must not alias A.  N <= 128.
hipError_t launch_gemm_nn(double* Y, int64_t ldy, const double* A,
                          int64_t lda, int K, const double* C, int ldc, int N,
                          int64_t d, double alpha, double beta, bool use_mfma,
                          hipStream_t s);

// Rank-revealing pivoted Cholesky of the b x b Gram matrix G (row-major),
// single workgroup.  With pivot != 0, column j is kept while its residual
// exceeds max(rank_tol2 * R11^2, rel2 * n0[j]), where R11^2 is the largest
// squared raw-column norm seen so far: *r11sq (device, updated in place
// with max_j n0[j]).  With pivot == 0 no pivoting is done and a column
// stops the factorisation only if its pivot is not positive (second CholQR
// pass).  Writes the rank to *rank and the b x b row-major matrix
// T = Pi R^{-1} (columns >= rank zero), so that X T has orthonormal
// columns.  work: b*b + 2*b doubles.
hipError_t launch_pchol(const double* G, int b, const double* n0,
                        double* r11sq, double rank_tol2, double rel2,
                        int pivot, double* T, int* rank, double* work,
                        hipStream_t s);
// T3 (row stride b) = T1 (row stride b, rho1 columns used) * T2 (rho1 x
// rho2, row stride rho1); columns >= rho2 of T3 are zero.
hipError_t launch_small_matmul(const double* T1, int b, int rho1,
                               const double* T2, int rho2, double* T3,
                               hipStream_t s);

}  // namespace prh
