// Fine propagator kernels: one step of the three-stage Runge-Kutta scheme
// (stages at 1/3, 1/2 and 1 of the step, each restarting from q^n) applied
// to the semi-discrete acoustic-advection system with 5th-order upwind
// advection, 4th-order centred acoustic terms and divergence damping
// (Section 3, Section 3.2, eq. acousticAd, eq. dampingCoeff).
//
// k_fine_step: all three stages of one step fused in a single pass.  A
// workgroup owns an x-range of NT input columns (one per thread, x fastest
// in memory so every row load is coalesced) and marches down a chunk of
// rows in z.  Each input row goes once into an LDS ring; stage 1 runs two
// rows behind the loads, stage 2 two rows behind stage 1 and stage 3 two
// rows behind stage 2, so that every row a stage needs has been produced in
// an earlier iteration and one barrier per row suffices.  Neighbours along
// x come from the LDS rings, neighbours along z from per-thread register
// windows.  The halo is 3 columns on the upwind side and 2 on the other per
// stage (15 per step) and 6 rows above and below the chunk.
//
// When one workgroup spans a whole periodic row (NT = nx, FULL) there is no
// x-halo at all: the three columns beyond each end of an LDS row hold copies
// of the columns at the other end, written with the row, so every thread
// computes an output column.
//
// Odd chunks march upwards, so that the halo rows two neighbouring chunks
// share are read by both at the same time (both at the start or both at the
// end of their march) and the second read hits in L2.
#include "pr_internal.h"

namespace prh {
namespace {

__device__ __forceinline__ void lds_barrier() {
  // Wait for this wave's LDS traffic only, then join the workgroup; global
  // loads of prefetched rows stay in flight across the barrier.
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Workgroups are handed to the 8 XCDs round-robin; give each XCD a
// contiguous range of logical tiles so neighbouring tiles, which read the
// same halo rows, share an L2.
__device__ __forceinline__ int xcd_logical_block(int nlogical) {
  const int b = blockIdx.x;
  const int per = (nlogical + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

struct Coef {
  double a0, a1, a2, a3, a4, a5, cx4, cz4, kxx, kxzu, kzz, kxzw;
};

__device__ __forceinline__ Coef load_coef(const FineCoef& c) {
  return Coef{c.adv[0], c.adv[1], c.adv[2], c.adv[3], c.adv[4], c.adv[5],
              c.cx4,    c.cz4,    c.kxx,    c.kxzu,   c.kzz,    c.kxzw};
}

// Coefficients of the fused kernel with the damping terms that lie on the
// advection stencil folded in: the x-damping of u, kxx (u(i+1) - 2 u(i) +
// u(i-1)), joins the upwind weights of u at offsets -1, 0, +1, and the
// centre part -2 kzz w of the z-damping of w joins the centre weight of w.
struct FusedCoef {
  double a0, a1, a2, a3, a4, a5;  // upwind weights
  double um, uc, up;   // weights of u at offsets -1, 0, +1 with kxx folded in
  double wc;           // centre weight of w with -2 kzz folded in
  double cx4, cz4, kxzu, kzz, kxzw;
};

template <int SGN>
__device__ __forceinline__ FusedCoef load_fused_coef(const FineCoef& c) {
  FusedCoef k;
  k.a0 = c.adv[0]; k.a1 = c.adv[1]; k.a2 = c.adv[2];
  k.a3 = c.adv[3]; k.a4 = c.adv[4]; k.a5 = c.adv[5];
  // weight index of offset 0: 3 for offsets -3 .. +2, 2 for -2 .. +3
  const double am = SGN > 0 ? k.a2 : k.a1, ac = SGN > 0 ? k.a3 : k.a2,
               ap = SGN > 0 ? k.a4 : k.a3;
  k.um = am + c.kxx;
  k.uc = ac - 2.0 * c.kxx;
  k.up = ap + c.kxx;
  k.wc = ac - 2.0 * c.kzz;
  k.cx4 = c.cx4; k.cz4 = c.cz4; k.kxzu = c.kxzu; k.kzz = c.kzz; k.kxzw = c.kxzw;
  return k;
}

// Values a stage carries from row to row (registers): the x-neighbours
// i-1, i+1 of u and w on the row r about to be computed, and the centred
// x-differences D_u = u(i+1) - u(i-1), D_w = w(i+1) - w(i-1) on rows r - 1
// and r.  The grad-div cross terms are differences of these along z:
//   w(i+1,j+1) - w(i+1,j-1) - w(i-1,j+1) + w(i-1,j-1) = D_w(j+1) - D_w(j-1),
// so every x-neighbour of u and w at offset +-1 is read from LDS once.
struct Carry {
  double xum, xup, xwm, xwp;  // u, w at (r, i-1), (r, i+1)
  double dum, dwm;            // D_u, D_w at row r - 1
  double du0, dw0;            // D_u, D_w at row r
};

// LDS ring layout: column-major, one LDS column of CS doubles per x
// position holding the 3 levels x 4 row slots of that position.  The pair
// (u, w) of ring row s = level * 4 + slot sits at 2 s, 16-byte aligned, so
// one 128-bit read fetches both; p sits at 24 + s.  With CS = 38 a column
// starts every 304 bytes: 16 consecutive lanes of a 128-bit read start on
// distinct groups of 4 banks, and of a 64-bit read on distinct bank pairs.
// A thread addresses everything from one base, its own column, with small
// constant offsets.
constexpr int CS = 38;
constexpr int PB = 24;  // p of ring row s at PB + s

__device__ __forceinline__ double2 ld2(const double* a) {
  return *reinterpret_cast<const double2*>(a);
}

// Reads u, w at offsets +-1 of the next row (rn: (u, w) pair of the own
// column of that row).
__device__ __forceinline__ void carry_read(const double* rn, double& um,
                                           double& up, double& wm,
                                           double& wp) {
  const double2 m = ld2(rn - CS), q = ld2(rn + CS);
  um = m.x;
  wm = m.y;
  up = q.x;
  wp = q.y;
}

// Right-hand side at one point of row r.  rc: this thread's (u, w) pair of
// LDS row s = r's ring row of the level, p at rc[PB - s];
// the own-column values along z come from registers, the +-1 neighbours
// of u and w and the D differences from the carry, D_u, D_w of row r + 1
// from the caller.
template <int SGN>
__device__ __forceinline__ void rhs_point(
    const double* rc, const double* rp, const Carry& cy, double dup,
    double dwp,
    double u0, double wm2, double wm1, double w0, double wp1, double wp2,
    double pm2, double pm1, double p0, double pp1, double pp2,
    const FusedCoef& k, double& fu, double& fw, double& fp) {
  // (u, w) pair and p at x-offset dx
  auto UW = [&](int dx) { return ld2(rc + dx * CS); };
  auto Pr = [&](int dx) { return rp[dx * CS]; };
  const double um1 = cy.xum, up1 = cy.xup, wxm1 = cy.xwm, wxp1 = cy.xwp;
  const double2 m2 = UW(-2), p2 = UW(2);
  const double um2 = m2.x, up2 = p2.x;
  const double wxm2 = m2.y, wxp2 = p2.y;
  const double pxm2 = Pr(-2), pxm1 = Pr(-1), pxp1 = Pr(1), pxp2 = Pr(2);
  double au, aw, ap;
  if (SGN > 0) {  // offsets -3 .. +2
    const double2 m3 = UW(-3);
    au = k.a0 * m3.x + k.a1 * um2 + k.um * um1 + k.uc * u0 + k.up * up1 +
         k.a5 * up2;
    aw = k.a0 * m3.y + k.a1 * wxm2 + k.a2 * wxm1 + k.wc * w0 +
         k.a4 * wxp1 + k.a5 * wxp2;
    ap = k.a0 * Pr(-3) + k.a1 * pxm2 + k.a2 * pxm1 + k.a3 * p0 +
         k.a4 * pxp1 + k.a5 * pxp2;
  } else {  // offsets -2 .. +3
    const double2 p3 = UW(3);
    au = k.a0 * um2 + k.um * um1 + k.uc * u0 + k.up * up1 + k.a4 * up2 +
         k.a5 * p3.x;
    aw = k.a0 * wxm2 + k.a1 * wxm1 + k.wc * w0 + k.a3 * wxp1 + k.a4 * wxp2 +
         k.a5 * p3.y;
    ap = k.a0 * pxm2 + k.a1 * pxm1 + k.a2 * p0 + k.a3 * pxp1 + k.a4 * pxp2 +
         k.a5 * Pr(3);
  }
  const double dx4p = (pxm2 - pxp2) + 8.0 * (pxp1 - pxm1);
  const double dz4p = (pm2 - pp2) + 8.0 * (pp1 - pm1);
  const double dx4u = (um2 - up2) + 8.0 * (up1 - um1);
  const double dz4w = (wm2 - wp2) + 8.0 * (wp1 - wm1);
  fu = au - k.cx4 * dx4p + k.kxzu * (dwp - cy.dwm);
  fw = aw - k.cz4 * dz4p + k.kzz * (wp1 + wm1) + k.kxzw * (dup - cy.dum);
  fp = ap - k.cx4 * dx4u - k.cz4 * dz4w;
}

template <int SGN, int NT, int PF, bool FULL>
__global__ __launch_bounds__(NT, NT >= 512 ? 1 : 2) void k_fine_step(
    const FineLaunch L) {
  constexpr int HL = SGN > 0 ? 3 : 2;  // reach on the upwind side
  constexpr int HR = 5 - HL;
  constexpr int TX = FULL ? NT : NT - 15;
  constexpr int PAD = 3;
  constexpr int W = NT + 2 * PAD;
  static_assert(4 % PF == 0, "prefetch depth must divide the 4-row tail");
  __shared__ __align__(16) double ring[W * CS];  // column-major, see CS

  const int lb = xcd_logical_block(L.nblocks);
  if (lb >= L.nblocks) return;
  int j = 0;
#pragma unroll 1
  while (j + 1 < L.njobs && lb >= L.job[j + 1].block_begin) ++j;
  const FineJob& J = L.job[j];

  const int local = lb - J.block_begin;
  const int xt = local % J.xtiles;
  const int rest = local / J.xtiles;
  const int zt = rest % J.ztiles;
  const int sl = rest / J.ztiles;
  const int nx = J.nx, nz = J.nz;
  const int64_t n = (int64_t)nx * nz;
  const double* __restrict__ in = J.in + sl * J.in_stride;
  double* __restrict__ out = J.out + sl * J.out_stride;
  // Odd chunks march upwards (decreasing z), so that two neighbouring
  // chunks read the rows they share at the same time.  Marching backwards
  // flips the sign of every odd z-difference; negating their coefficients
  // gives bitwise the same results.
  const bool rev = (zt & 1) != 0;
  FusedCoef k = load_fused_coef<SGN>(J.c);
  if (rev) { k.cz4 = -k.cz4; k.kxzu = -k.kxzu; k.kxzw = -k.kxzw; }
  const double dt = J.c.dt;
  const double b1 = dt / 3.0, b2 = 0.5 * dt;

  const int t = threadIdx.x;
  const int c = PAD + t;
  const int zc = L.zc;
  const int x0 = xt * TX;
  const int z0 = zt * zc;
  const int zdir = rev ? -1 : 1;
  const int zbase = rev ? z0 + zc + 5 : z0 - 6;  // input row of iteration 0
  const int gx = FULL ? t : wrap(x0 - 3 * HL + t, nx);
  const int xo = FULL ? t : x0 + t - 3 * HL;
  const bool store_col =
      FULL || ((t >= 3 * HL) && (t < NT - 3 * HR) && (xo < nx));
  // FULL: the lanes whose column is copied into a pad of the row
  const bool pad_lo = FULL && t < PAD, pad_hi = FULL && t >= NT - PAD;
  const int nrows = zc + 12;

  // Pads of every ring row are read by the edge columns (whose results are
  // discarded, or, for FULL, overwritten with copies); keep them finite.
  for (int q = t; q < 2 * PAD * CS; q += NT) {
    const int col = q / CS, e = q % CS;
    ring[(col < PAD ? col : NT + col) * CS + e] = 0.0;
  }
  double* const own = ring + c * CS;  // this thread's LDS column
  // (u, w) pair and p of ring row (level, slot)
  auto slot = [&](int lvl, int sl) { return own + 2 * (lvl * 4 + sl); };
  auto pslot = [&](int lvl, int sl) { return own + PB + lvl * 4 + sl; };

  double fu_[PF], fw_[PF], fp_[PF];  // prefetched input rows
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    const double* src = in + (int64_t)wrap(zbase + zdir * q, nz) * nx + gx;
    fu_[q] = src[0];
    fw_[q] = src[n];
    fp_[q] = src[2 * n];
  }

  double iu[8], iw[8], ip[8];  // input rows, indexed by iteration & 7
  double au[8], aw[8], ap[8];  // stage-1 rows
  double bu[8], bw[8], bp[8];  // stage-2 rows
  Carry c1{}, c2{}, c3{};      // per-stage carries

  // Writes this thread's column of one ring row (and, for FULL, its copy in
  // the pad at the other end of the row).
  auto ring_put = [&](double* r, double* rp, double vu, double vw,
                      double vp) {
    *reinterpret_cast<double2*>(r) = double2{vu, vw};
    *rp = vp;
    if (FULL && (pad_lo || pad_hi)) {
      const int o = (pad_lo ? NT : -NT) * CS;
      *reinterpret_cast<double2*>(r + o) = double2{vu, vw};
      rp[o] = vp;
    }
  };

  // One row iteration.  For each stage L, PREL reads the +-1 neighbours of
  // the row after the one it computes (from an earlier iteration) and
  // advances the carry; DOL computes the row.  All flags are compile-time
  // after unrolling, so in the steady state the three stages (which read
  // only rows produced in earlier iterations) are straight-line code the
  // scheduler interleaves.  The row count zc + 12 is a multiple of 4: whole
  // blocks of 8 rows, then at most one block of 4.  The prefetch never
  // reaches past the chunk's last input row (it re-reads that row, which is
  // still in cache).
#define PR_STAGE(PRE, DO, LVL, CY, ZU, ZW, ZP, BU, BW, BP, OU, OW, OP, BETA, STORE) \
  if (PRE) {                                                                  \
    double xum, xup, xwm, xwp;                                                \
    carry_read(slot(LVL, ((uu) - 1) & 3), xum, xup, xwm, xwp);                \
    const double dup = xup - xum, dwp = xwp - xwm;                            \
    if (DO) {                                                                 \
      double fu, fw, fp;                                                      \
      rhs_point<SGN>(slot(LVL, ((uu) - 2) & 3), pslot(LVL, ((uu) - 2) & 3),   \
                     CY, dup, dwp,                                            \
                        ZU[((uu) - 2) & 7], ZW[((uu) - 4) & 7],               \
                        ZW[((uu) - 3) & 7], ZW[((uu) - 2) & 7],               \
                        ZW[((uu) - 1) & 7], ZW[(uu) & 7], ZP[((uu) - 4) & 7], \
                        ZP[((uu) - 3) & 7], ZP[((uu) - 2) & 7],               \
                        ZP[((uu) - 1) & 7], ZP[(uu) & 7], k, fu, fw, fp);     \
      const double nu = BU + (BETA) * fu, nw = BW + (BETA) * fw,              \
                   np = BP + (BETA) * fp;                                     \
      STORE                                                                   \
    }                                                                         \
    CY.dum = CY.du0;                                                          \
    CY.dwm = CY.dw0;                                                          \
    CY.du0 = dup;                                                             \
    CY.dw0 = dwp;                                                             \
    CY.xum = xum;                                                             \
    CY.xup = xup;                                                             \
    CY.xwm = xwm;                                                             \
    CY.xwp = xwp;                                                             \
  }

#define PR_ROW(uu, it, P1, D1, P2, D2, P3, D3)                                 \
  {                                                                           \
    lds_barrier();                                                            \
    {                                                                         \
      const int q = (uu) % PF;                                                \
      iu[uu] = fu_[q];                                                        \
      iw[uu] = fw_[q];                                                        \
      ip[uu] = fp_[q];                                                        \
      ring_put(slot(0, (uu) & 3), pslot(0, (uu) & 3), iu[uu], iw[uu], ip[uu]); \
      const int zp = (it) + PF < nrows ? (it) + PF : nrows - 1;               \
      const double* src = in + (int64_t)wrap(zbase + zdir * zp, nz) * nx + gx; \
      fu_[q] = src[0];                                                        \
      fw_[q] = src[n];                                                        \
      fp_[q] = src[2 * n];                                                    \
    }                                                                         \
    PR_STAGE(P1, D1, 0, c1, iu, iw, ip, iu[((uu) - 2) & 7],                   \
             iw[((uu) - 2) & 7], ip[((uu) - 2) & 7], au, aw, ap, b1,          \
             au[uu] = nu; aw[uu] = nw; ap[uu] = np;                           \
             ring_put(slot(1, (uu) & 3), pslot(1, (uu) & 3), nu, nw, np);)    \
    PR_STAGE(P2, D2, 1, c2, au, aw, ap, iu[((uu) - 4) & 7],                   \
             iw[((uu) - 4) & 7], ip[((uu) - 4) & 7], bu, bw, bp, b2,          \
             bu[uu] = nu; bw[uu] = nw; bp[uu] = np;                           \
             ring_put(slot(2, (uu) & 3), pslot(2, (uu) & 3), nu, nw, np);)    \
    PR_STAGE(P3, D3, 2, c3, bu, bw, bp, iu[((uu) - 6) & 7],                   \
             iw[((uu) - 6) & 7], ip[((uu) - 6) & 7], bu, bw, bp, dt,          \
             const int z3 = zbase + zdir * ((it) - 6);                        \
             if (store_col && (it) < nrows && z3 < nz) {                      \
               double* dst = out + (int64_t)z3 * nx + xo;                     \
               dst[0] = nu;                                                   \
               dst[n] = nw;                                                   \
               dst[2 * n] = np;                                               \
             })                                                               \
  }

  // Warm-up: stage L starts carrying two rows before it first computes
  // (stage 1 computes from row 4, stage 2 from 8, stage 3 from 12).
#pragma unroll
  for (int uu = 0; uu < 8; ++uu)
    PR_ROW(uu, uu, uu >= 2, uu >= 4, uu >= 6, false, false, false)
#pragma unroll
  for (int uu = 0; uu < 8; ++uu)
    PR_ROW(uu, 8 + uu, true, true, true, true, uu >= 2, uu >= 4)
  int base = 16;
  for (; base + 8 <= nrows; base += 8) {
#pragma unroll
    for (int uu = 0; uu < 8; ++uu)
      PR_ROW(uu, base + uu, true, true, true, true, true, true)
  }
  if (base < nrows) {
#pragma unroll
    for (int uu = 0; uu < 4; ++uu)
      PR_ROW(uu, base + uu, true, true, true, true, true, true)
  }
#undef PR_ROW
#undef PR_STAGE
}

// Unfused stage: out = base + beta f(in), one point per thread, neighbours
// straight from global memory.
template <int SGN>
__global__ __launch_bounds__(256) void k_fine_stage(
    const double* __restrict__ in, int64_t is, const double* __restrict__ base,
    int64_t bs, double* __restrict__ out, int64_t os, int nx, int nz,
    const FineCoef cc, double beta) {
  const int64_t n = (int64_t)nx * nz;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int64_t sl = blockIdx.y;
  const double* U = in + sl * is;
  const double* Wf = U + n;
  const double* Pf = U + 2 * n;
  const int i = (int)(idx % nx), jz = (int)(idx / nx);
  auto X = [&](int di) { return wrap(i + di, nx); };
  auto Z = [&](int dj) { return (int64_t)wrap(jz + dj, nz) * nx; };
  const int64_t zr = (int64_t)jz * nx;
  const Coef k = load_coef(cc);
  const int m0 = SGN > 0 ? -3 : -2;
  const double a[6] = {k.a0, k.a1, k.a2, k.a3, k.a4, k.a5};
  double au = 0.0, aw = 0.0, ap = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int64_t o = zr + X(m0 + q);
    au += a[q] * U[o];
    aw += a[q] * Wf[o];
    ap += a[q] * Pf[o];
  }
  const double u0 = U[idx], w0 = Wf[idx];
  const double dx4p = (Pf[zr + X(-2)] - Pf[zr + X(2)]) +
                      8.0 * (Pf[zr + X(1)] - Pf[zr + X(-1)]);
  const double dz4p = (Pf[Z(-2) + i] - Pf[Z(2) + i]) +
                      8.0 * (Pf[Z(1) + i] - Pf[Z(-1) + i]);
  const double dx4u = (U[zr + X(-2)] - U[zr + X(2)]) +
                      8.0 * (U[zr + X(1)] - U[zr + X(-1)]);
  const double dz4w = (Wf[Z(-2) + i] - Wf[Z(2) + i]) +
                      8.0 * (Wf[Z(1) + i] - Wf[Z(-1) + i]);
  const double gxx = (U[zr + X(1)] + U[zr + X(-1)]) - 2.0 * u0;
  const double gzz = (Wf[Z(1) + i] + Wf[Z(-1) + i]) - 2.0 * w0;
  const double wx = (Wf[Z(1) + X(1)] - Wf[Z(-1) + X(1)]) -
                    (Wf[Z(1) + X(-1)] - Wf[Z(-1) + X(-1)]);
  const double uz = (U[Z(1) + X(1)] - U[Z(1) + X(-1)]) -
                    (U[Z(-1) + X(1)] - U[Z(-1) + X(-1)]);
  const double fu = au - k.cx4 * dx4p + k.kxx * gxx + k.kxzu * wx;
  const double fw = aw - k.cz4 * dz4p + k.kzz * gzz + k.kxzw * uz;
  const double fp = ap - k.cx4 * dx4u - k.cz4 * dz4w;
  const double* B = base + sl * bs;
  double* O = out + sl * os;
  O[idx] = B[idx] + beta * fu;
  O[n + idx] = B[n + idx] + beta * fw;
  O[2 * n + idx] = B[2 * n + idx] + beta * fp;
}

// Prefetch depth in rows: the halo variants hold more per-thread state and
// stay within 256 VGPRs only with 2.
constexpr int fine_pf(bool full) { return full ? 4 : 2; }

template <int SGN, int NT, bool FULL>
hipError_t launch_nt(const FineLaunch& L, hipStream_t s) {
  const int grid = 8 * ((L.nblocks + 7) / 8);
  hipLaunchKernelGGL((k_fine_step<SGN, NT, fine_pf(FULL), FULL>), dim3(grid),
                     dim3(NT), 0, s, L);
  return hipGetLastError();
}

template <int SGN>
hipError_t launch_sgn(const FineLaunch& L, int nt, bool full, hipStream_t s) {
  if (full) {
    switch (nt) {
      case 128: return launch_nt<SGN, 128, true>(L, s);
      case 256: return launch_nt<SGN, 256, true>(L, s);
      case 512: return launch_nt<SGN, 512, true>(L, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nt) {
    case 128: return launch_nt<SGN, 128, false>(L, s);
    case 192: return launch_nt<SGN, 192, false>(L, s);
    case 256: return launch_nt<SGN, 256, false>(L, s);
    default: return hipErrorInvalidValue;
  }
}

template <int SGN, int NT, bool FULL>
int blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb,
          reinterpret_cast<const void*>(&k_fine_step<SGN, NT, fine_pf(FULL), FULL>),
          NT, 0) != hipSuccess)
    return 0;
  return nb;
}

template <int SGN>
int blocks_per_cu_sgn(int nt, bool full) {
  if (full) {
    switch (nt) {
      case 128: return blocks_per_cu<SGN, 128, true>();
      case 256: return blocks_per_cu<SGN, 256, true>();
      case 512: return blocks_per_cu<SGN, 512, true>();
      default: return 0;
    }
  }
  switch (nt) {
    case 128: return blocks_per_cu<SGN, 128, false>();
    case 192: return blocks_per_cu<SGN, 192, false>();
    case 256: return blocks_per_cu<SGN, 256, false>();
    default: return 0;
  }
}

}  // namespace

bool fine_nt_supported(int nt, int nx) {
  if (nt == nx) return fine_full_row(nx);
  return nt == 128 || nt == 192 || nt == 256;
}

bool fine_full_row(int nx) { return nx == 128 || nx == 256 || nx == 512; }

int fine_blocks_per_cu(int nt, int nx, int sgn) {
  const bool full = nt == nx && fine_full_row(nx);
  return sgn >= 0 ? blocks_per_cu_sgn<1>(nt, full)
                  : blocks_per_cu_sgn<-1>(nt, full);
}

hipError_t launch_fine_step(const FineLaunch& L, int nt, int sgn,
                            hipStream_t s) {
  if (L.nblocks <= 0) return hipSuccess;
  // One tile width for every job of the launch; FULL when it is the row.
  const bool full = nt == L.job[0].nx && fine_full_row(nt);
  for (int j = 1; j < L.njobs; ++j)
    if ((L.job[j].nx == nt && fine_full_row(nt)) != full)
      return hipErrorInvalidValue;
  return sgn >= 0 ? launch_sgn<1>(L, nt, full, s)
                  : launch_sgn<-1>(L, nt, full, s);
}

hipError_t launch_fine_stage(const double* in, int64_t in_stride,
                             const double* base, int64_t base_stride,
                             double* out, int64_t out_stride, int nx, int nz,
                             int nslices, const FineCoef& c, double beta,
                             int sgn, hipStream_t s) {
  const int64_t n = (int64_t)nx * nz;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)nslices);
  if (sgn >= 0)
    hipLaunchKernelGGL(k_fine_stage<1>, grid, dim3(256), 0, s, in, in_stride,
                       base, base_stride, out, out_stride, nx, nz, c, beta);
  else
    hipLaunchKernelGGL(k_fine_stage<-1>, grid, dim3(256), 0, s, in, in_stride,
                       base, base_stride, out, out_stride, nx, nz, c, beta);
  return hipGetLastError();
}

}  // namespace prh
