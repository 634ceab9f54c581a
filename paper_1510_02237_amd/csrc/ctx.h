// Host-side state of one KSE-Parareal problem (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/libpararealhip.h"
#include "pr_internal.h"

struct pr_ctx {
  // ----- problem (Section 2.1 time slicing, Section 3 grid) -----
  pr_grid g{};
  double c_s = 1.0, U = 0.0, dt_f = 0.0, dt_g = 0.0;
  int32_t P = 1;
  pr_opts o{};
  int n_f = 0, n_g = 0;
  int64_t n = 0;   // points per field
  int64_t d = 0;   // doubles per state (3 n)
  int64_t ld = 0;  // padded state stride of internal buffers (multiple of 64)
  prh::FineCoef fc{};
  prh::CoarseCoef cc{};
  // Stage kernels with advective weights per row and per column: the
  // Section 3.1 pair (rk3), and the split scheme with a z-velocity, a
  // rotation or second-order fine acoustics (tables_f: F runs as stages;
  // tables_g: the slow tendency of G comes from the stage kernel).
  prh::StageCoef sf{}, sg{};
  std::vector<double> h_tabs;  // F x, F z, G x, G z weights ([n][7] each)
  double* tabs = nullptr;      // device copy of h_tabs
  bool rk3 = false, tables_f = false, tables_g = false;
  int sgn = 1;
  std::vector<int> coarse_chunks;  // substeps per launch within a coarse step

  // ----- runtime -----
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t side = nullptr;      // projections overlap the coarse step
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  int nt = 256, zc = 64;  // fine-sweep tile (threads, rows)
  bool tuned = false;

  // ----- device arena -----
  int wcap = 0;           // states in each work block
  int rcap = 0;           // basis capacity (vectors)
  double* Q = nullptr;    // (P+1) iterates q^k_i
  double* Qt = nullptr;   // (P+1) fine results qt^k_i
  double* GQ = nullptr;   // (P) G(q^k_i), kept current by linearity
  double* Wk = nullptr;   // wcap: sweep ping-pong, batched-G ping
  double* X = nullptr;    // wcap: new raw columns (projected in place)
  double* DX = nullptr;   // wcap: their F - G images
  double* Yb = nullptr;   // wcap: CholQR intermediate, batched-G pong
  double* Rb = nullptr;   // wcap: frozen slow tendency when N_sound > 4 or
                          // tables_g, or the step buffer of the RK-3 coarse
                          // propagator
  double* st = nullptr;   // kSingle single states
  double* S = nullptr;    // rcap basis vectors
  double* D = nullptr;    // rcap vectors F(s_j) - G(s_j)
  double* small = nullptr;
  int* ism = nullptr;     // device ints: rank1, rank2, finite flag
  int* h_ism = nullptr;   // pinned host mirror
  double* nrm = nullptr;    // stopping criterion: 2 (P + 1) squared norms
  double* h_nrm = nullptr;  // pinned host mirror
  size_t small_len = 0;
  int r = 0;              // current basis dimension
  double* d_r11sq = nullptr;
  // carved out of `small`
  double *part = nullptr, *cvec = nullptr, *gram = nullptr, *T1 = nullptr,
         *T2 = nullptr, *T3 = nullptr, *pcw = nullptr, *tnw = nullptr,
         *n0 = nullptr, *Cm = nullptr;
  double* ext_ping = nullptr;  // sweep ping buffer for caller buffers
  size_t ext_ping_len = 0;
  double* ext_io = nullptr;    // staging for host-memory calls
  size_t ext_io_len = 0;

  // ----- graphs -----
  std::map<long long, hipGraphExec_t> graphs;

  // ----- subspace update in progress -----
  int upd_b = 0, upd_rho = 0;
  int upd_verify = 0;  // columns the last second Cholesky-QR pass must have
                       // kept, checked at the next wait (0: nothing pending)

  // ----- statistics -----
  pr_stats stats{};
  bool use_mfma = true;
};

enum { kIo = 0, kG = 1, kTa = 2, kTb = 3, kDa = 4, kDb = 5, kRs = 6,
       kTmp = 7, kY = 8, kSingle = 9 };

namespace prh {

// Implemented in solver.cpp
int set_error(pr_ctx* c, int code, const char* fmt, ...);
int hip_check(pr_ctx* c, hipError_t e, const char* what);
int ensure_arena(pr_ctx* c, int wcap, int rcap);
double* single(pr_ctx* c, int which);
// Fine sweep: out[s] = F(in[s]) for s < ns (strides in doubles), ping has
// ns states at stride ping_stride.  form: PR_FORM_*.
int run_sweep(pr_ctx* c, const double* in, int64_t in_stride, double* out,
              int64_t out_stride, double* ping, int64_t ping_stride, int ns,
              int form);
// Coarse propagator over one slice for ns states at stride `stride`:
// out = G(in); pa, pb: ping buffers (ns states each), R: slow-tendency
// buffer (ns states) needed when N_sound > 4, tables_g or rk3.  in must not
// alias out.
int run_coarse(pr_ctx* c, const double* in, double* out, int ns,
               int64_t stride, double* pa, double* pb, double* R);
// Appends span of b columns X0 (stride ld) with fine images FX0 (stride ld)
// (synchronous); the three asynchronous stages it is made of.  Between the
// stages the caller must wait for the context stream (the stage reads a rank
// the previous one copied to pinned host memory).  ensure_arena(c, b, r + b)
// must have been called before update_begin.
int krylov_append(pr_ctx* c, const double* X0, const double* FX0, int b);
// GX0: G of the columns (stride ld), or NULL to compute it here.
int update_begin(pr_ctx* c, const double* X0, const double* FX0,
                 const double* GX0, int b);
int update_mid(pr_ctx* c);
// defer_check: the second pass's rank is checked by verify_second_pass at
// the caller's next wait on the stream instead of now.
int update_end(pr_ctx* c, bool defer_check = false);
int verify_second_pass(pr_ctx* c);
// Coarse initialisation q^0_{i+1} = G(q^0_i) (Algorithm 2, initialisation)
// and the serial correction of iteration k, enqueued on the context stream.
int coarse_init(pr_ctx* c);
int chain(pr_ctx* c, int k);
// Applies new physical parameters to a context with the same grid and P
// (buffers kept); used by the server to reuse arenas.
int retarget(pr_ctx* c, double c_s, double U, double dt_f, double dt_g,
             const pr_opts* o, double T, double Lx, double Lz);
// Autotune the fused sweep tile for ns slices.
int autotune(pr_ctx* c, int ns);

}  // namespace prh
