// libpararealhip: context, propagator orchestration and Krylov-subspace-
// enhanced Parareal (Algorithm 2 of Ruprecht & Krause, Section 2.2).
//
// Device-side design (MI355X):
//  * every state lives in HBM in the C-ABI layout [3][nz][nx], internal
//    buffers padded to a stride `ld` (multiple of 64 doubles, zero pad) so
//    the tall-skinny MFMA products run over whole 16-element groups;
//  * the fine sweep advances all slices with one fused-step launch per RK-3
//    step (batched form), replayed from a captured HIP graph;
//  * the subspace update keeps an orthonormal basis S and the images
//    D(S) = F(S) - G(S); by linearity (eq. Genhance) the modified coarse
//    propagator of eq. modifiedCoarse is K(x) = G(x) + D(S) S^T x, which
//    is algebraically G((I - P)x) + F(P x) and reads the basis twice
//    instead of three times;
//  * the serial correction uses the difference form
//    q^{k+1}_{i+1} = qt^k_{i+1} + K(q^{k+1}_i - q^k_i), equal to Algorithm
//    2's K(q^{k+1}_i) + qt^k_{i+1} - K(q^k_i) by linearity, one K per slice;
//    slices already converged contribute exact zeros.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "ctx.h"

using namespace prh;

namespace {
thread_local std::string g_err;
}

int prh::set_error(pr_ctx* c, int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_err = buf;
  return code;
}

int prh::hip_check(pr_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return PR_OK;
  (void)hipGetLastError();
  return set_error(c, e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EDEVICE,
                   "%s: %s", what, hipGetErrorString(e));
}

#define HC(expr)                                         \
  do {                                                   \
    int rc_ = prh::hip_check(c, (expr), #expr);          \
    if (rc_) return rc_;                                 \
  } while (0)
#define RC(expr)          \
  do {                    \
    int rc_ = (expr);     \
    if (rc_) return rc_;  \
  } while (0)

// ---------------------------------------------------------------- helpers

static int int_ratio(double a, double b, int* out) {
  if (!(a > 0.0) || !(b > 0.0)) return -1;
  const double q = a / b;
  if (!(q < 2e9)) return -1;
  const long long k = llround(q);
  if (k < 1 || std::fabs((double)k * b - a) > 1e-9 * std::fabs(a)) return -1;
  *out = (int)k;
  return 0;
}

extern "C" void pr_opts_default(pr_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->nu_f = 0.005;
  o->nu_c = 0.1;
  o->n_sound = 4;
  o->rank_tol = 1e-10;
  o->form = PR_FORM_BATCHED;
  o->skip_converged = 1;
  o->tile_nt = 0;
  o->tile_zc = 0;
  o->windows = 1;
  o->fine_acoustic_order = 4;
  o->coarse_order = 1;
}

// Validates the problem; fills n_f, n_g.  Shared with the server.
int pr_validate(const pr_grid* g, double c_s, double U, double dt_f,
                double dt_g, int32_t P, const pr_opts* o, int* nf, int* ng,
                std::string* msg) {
  char buf[256];
  auto fail = [&](const char* m) {
    if (msg) *msg = m;
    return PR_EINVAL;
  };
  if (!g || !o) return fail("null argument");
  if (g->nx < 8 || g->nz < 8) return fail("nx and nz must be >= 8");
  if ((int64_t)g->nx * g->nz > (int64_t)1 << 30) return fail("grid too large");
  if (!(g->Lx > 0) || !(g->Lz > 0) || !(g->T > 0))
    return fail("Lx, Lz and T must be positive");
  if (P < 1 || P > 4096) return fail("P must be in [1, 4096]");
  if (!(c_s >= 0) || !std::isfinite(c_s) || !std::isfinite(U))
    return fail("c_s must be finite and >= 0, U finite");
  if (!(dt_f > 0) || !(dt_g > 0)) return fail("time steps must be positive");
  if (o->n_sound < 1 || o->n_sound > 256) return fail("n_sound must be in [1, 256]");
  if (!(o->nu_f >= 0) || !(o->nu_c >= 0)) return fail("nu_f, nu_c must be >= 0");
  if (!(o->rank_tol > 0) || !(o->rank_tol < 1)) return fail("rank_tol must be in (0, 1)");
  if (o->form < 0 || o->form > PR_FORM_STAGEWISE) return fail("unknown form");
  if (o->tile_nt && !fine_nt_supported(o->tile_nt, g->nx))
    return fail("tile_nt must be 0, 128, 192, 256, or nx when nx is 128, "
                "256 or 512");
  if (o->tile_zc < 0 || o->tile_zc > 4096 || (o->tile_zc % 4))
    return fail("tile_zc must be a multiple of 4 in [0, 4096]");
  if (o->windows < 1 || o->windows > (1 << 20))
    return fail("windows must be in [1, 2^20]");
  if (o->scheme != PR_SCHEME_SPLIT && o->scheme != PR_SCHEME_RK3)
    return fail("scheme must be PR_SCHEME_SPLIT or PR_SCHEME_RK3");
  if (!std::isfinite(o->V) || !std::isfinite(o->gamma))
    return fail("V and gamma must be finite");
  if (o->scheme == PR_SCHEME_RK3 && o->gamma != 0.0)
    return fail("gamma must be 0 with PR_SCHEME_RK3 (constant velocity)");
  if (o->fine_acoustic_order != 2 && o->fine_acoustic_order != 4)
    return fail("fine_acoustic_order must be 2 or 4");
  if (o->coarse_order != 1 && o->coarse_order != 3)
    return fail("coarse_order must be 1 or 3");
  if (o->scheme == PR_SCHEME_RK3 && o->coarse_order != 1)
    return fail("coarse_order must be 1 with PR_SCHEME_RK3");
  if (!(o->stop_tol >= 0) || !std::isfinite(o->stop_tol))
    return fail("stop_tol must be finite and >= 0");
  const double slice = g->T / ((double)o->windows * P);
  if (int_ratio(slice, dt_f, nf)) {
    snprintf(buf, sizeof buf, "(T/(windows*P))/dt_f = %.17g is not an integer",
             slice / dt_f);
    return fail(buf);
  }
  if (int_ratio(slice, dt_g, ng)) {
    snprintf(buf, sizeof buf, "(T/(windows*P))/dt_g = %.17g is not an integer",
             slice / dt_g);
    return fail(buf);
  }
  return PR_OK;
}

static void make_coef(pr_ctx* c) {
  const double dx = c->g.Lx / c->g.nx, dz = c->g.Lz / c->g.nz;
  const double U = c->U, cs = c->c_s;
  c->sgn = U >= 0 ? 1 : -1;
  // Fifth-order upwind derivative (Wicker-Skamarock flux of order 5,
  // differenced): weights /(60 dx) at offsets -3..2 for U >= 0, mirrored
  // (-2..3) for U < 0.
  static const double wpos[6] = {-2.0, 15.0, -60.0, 20.0, 30.0, -3.0};
  static const double wneg[6] = {3.0, -30.0, -20.0, 60.0, -15.0, 2.0};
  const double* w = U >= 0 ? wpos : wneg;
  for (int k = 0; k < 6; ++k) c->fc.adv[k] = -U * w[k] / (60.0 * dx);
  c->fc.cx4 = cs / (12.0 * dx);
  c->fc.cz4 = cs / (12.0 * dz);
  // alpha = nu h^2 / tau (eq. dampingCoeff) times the 1/h^2 and 1/(4 dx dz)
  // of the compact grad-div stencil.
  const double tf = c->dt_f, nuf = c->o.nu_f;
  c->fc.kxx = nuf / tf;
  c->fc.kxzu = nuf * dx / (4.0 * tf * dz);
  c->fc.kzz = nuf / tf;
  c->fc.kxzw = nuf * dz / (4.0 * tf * dx);
  c->fc.dt = tf;
  const double dtau = c->dt_g / c->o.n_sound, nuc = c->o.nu_c;
  c->cc.cR = -U / dx;
  c->cc.upwind_left = U >= 0 ? 1 : 0;
  c->cc.dtau = dtau;
  c->cc.cx2 = cs / (2.0 * dx);
  c->cc.cz2 = cs / (2.0 * dz);
  c->cc.kxx = nuc / dtau;
  c->cc.kxzu = nuc * dx / (4.0 * dtau * dz);
  c->cc.kzz = nuc / dtau;
  c->cc.kxzw = nuc * dz / (4.0 * dtau * dx);
  const int ns = c->o.n_sound;
  const int nch = (ns + kCoarseMaxSubPerLaunch - 1) / kCoarseMaxSubPerLaunch;
  c->coarse_chunks.assign(nch, ns / nch);
  for (int q = 0; q < ns % nch; ++q) c->coarse_chunks[q] += 1;
  // Stage-kernel weights, stored as weights of f = -advection at offsets
  // -3..3 of each row (x) and each column (z).  The velocity of row j
  // along x and of column i along z is U + gamma (z_j - Lz/2) and
  // V - gamma (x_i - Lx/2) (eq. adVel with a constant part).
  //  * Section 3.1 pair.  F: sixth-order centred flux differenced, point
  //    weights (-1, 9, -45, 0, 45, -9, 1)/(60 h).  G: first-order upwind,
  //    vel (q_i - q_{i-1})/h for vel >= 0, vel (q_{i+1} - q_i)/h for vel < 0.
  //  * Split scheme.  F: the fifth-order upwind weights above, per row and
  //    column; G: the first-order (or third-order) upwind slow tendency, no
  //    acoustics.  Third order: the Wicker-Skamarock flux of order 3
  //    differenced, point weights (1, -6, 3, 2)/(6 h) at offsets -2..1 for
  //    vel >= 0, (-2, -3, 6, -1)/(6 h) at -1..2 for vel < 0.
  c->rk3 = c->o.scheme == PR_SCHEME_RK3;
  const double V = c->o.V, gam = c->o.gamma;
  c->tables_f = c->rk3 || V != 0.0 || gam != 0.0 || c->o.fine_acoustic_order == 2;
  c->tables_g = !c->rk3 && (V != 0.0 || gam != 0.0 || c->o.coarse_order == 3);
  c->h_tabs.clear();
  c->sf = prh::StageCoef{};
  c->sg = prh::StageCoef{};
  if (!c->tables_f && !c->tables_g) return;
  const int nx = c->g.nx, nz = c->g.nz;
  c->h_tabs.assign((size_t)14 * (nx + nz), 0.0);
  double* fwx = c->h_tabs.data();
  double* fwz = fwx + 7 * (size_t)nz;
  double* gwx = fwz + 7 * (size_t)nx;
  double* gwz = gwx + 7 * (size_t)nz;
  static const double c6[7] = {-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0};
  auto fine_w = [&](double vel, double h, double* out) {
    if (c->rk3) {
      for (int k = 0; k < 7; ++k) out[k] = -vel * c6[k] / (60.0 * h);
    } else {
      const double* wv = vel >= 0 ? wpos : wneg;
      const int k0 = vel >= 0 ? 0 : 1;  // offset -3 or -2 first
      for (int k = 0; k < 6; ++k) out[k0 + k] = -vel * wv[k] / (60.0 * h);
    }
  };
  static const double u3pos[4] = {1.0, -6.0, 3.0, 2.0};
  static const double u3neg[4] = {-2.0, -3.0, 6.0, -1.0};
  const bool third = !c->rk3 && c->o.coarse_order == 3;
  auto up1_w = [&](double vel, double h, double* out) {
    if (third) {
      const double* wv = vel >= 0 ? u3pos : u3neg;
      const int k0 = vel >= 0 ? 1 : 2;  // offset -2 or -1 first
      for (int k = 0; k < 4; ++k) out[k0 + k] = -vel * wv[k] / (6.0 * h);
    } else if (vel >= 0) {
      out[3] = -vel / h;
      out[2] = vel / h;
    } else {
      out[4] = -vel / h;
      out[3] = vel / h;
    }
  };
  for (int j = 0; j < nz; ++j) {
    const double vel = U + gam * ((j + 0.5) * dz - 0.5 * c->g.Lz);
    fine_w(vel, dx, fwx + 7 * (size_t)j);
    up1_w(vel, dx, gwx + 7 * (size_t)j);
  }
  for (int i = 0; i < nx; ++i) {
    const double vel = V - gam * ((i + 0.5) * dx - 0.5 * c->g.Lx);
    fine_w(vel, dz, fwz + 7 * (size_t)i);
    up1_w(vel, dz, gwz + 7 * (size_t)i);
  }
  if (c->rk3) {
    c->sf.ax1 = c->sg.ax1 = cs / (2.0 * dx);
    c->sf.az1 = c->sg.az1 = cs / (2.0 * dz);
  } else {
    if (c->o.fine_acoustic_order == 2) {
      c->sf.ax1 = cs / (2.0 * dx);
      c->sf.az1 = cs / (2.0 * dz);
    } else {
      c->sf.ax1 = 8.0 * cs / (12.0 * dx);
      c->sf.ax2 = -cs / (12.0 * dx);
      c->sf.az1 = 8.0 * cs / (12.0 * dz);
      c->sf.az2 = -cs / (12.0 * dz);
    }
    c->sf.kxx = c->fc.kxx;
    c->sf.kxzu = c->fc.kxzu;
    c->sf.kzz = c->fc.kzz;
    c->sf.kxzw = c->fc.kxzw;
  }
}

// Copies the stage-kernel weights to the device (once, at create time, so
// that no allocation happens inside a captured graph) and points the
// coefficient blocks at them.
static int upload_tables(pr_ctx* c) {
  if (c->h_tabs.empty()) return PR_OK;
  const size_t bytes = c->h_tabs.size() * sizeof(double);
  HC(hipMalloc((void**)&c->tabs, bytes));
  HC(hipMemcpy(c->tabs, c->h_tabs.data(), bytes, hipMemcpyHostToDevice));
  const int nx = c->g.nx, nz = c->g.nz;
  c->sf.wx = c->tabs;
  c->sf.wz = c->sf.wx + 7 * (size_t)nz;
  c->sg.wx = c->sf.wz + 7 * (size_t)nx;
  c->sg.wz = c->sg.wx + 7 * (size_t)nz;
  return PR_OK;
}

static void clear_graphs(pr_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

double* prh::single(pr_ctx* c, int which) { return c->st + (int64_t)which * c->ld; }

static int dalloc(pr_ctx* c, double** p, size_t ndoubles, const char* what) {
  if (*p) {
    (void)hipFree(*p);
    *p = nullptr;
  }
  if (ndoubles == 0) return PR_OK;
  hipError_t e = hipMalloc((void**)p, ndoubles * sizeof(double));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(c, PR_ENOMEM, "hipMalloc(%s, %zu bytes) failed: %s", what,
                     ndoubles * sizeof(double), hipGetErrorString(e));
  }
  e = hipMemsetAsync(*p, 0, ndoubles * sizeof(double), c->stream);
  return hip_check(c, e, "hipMemsetAsync");
}

int prh::ensure_arena(pr_ctx* c, int wcap, int rcap) {
  wcap = std::max(wcap, c->P);
  rcap = std::max(rcap, 1);
  const int64_t ld = c->ld;
  bool changed = false;
  if (!c->Q) {
    RC(dalloc(c, &c->Q, (size_t)(c->P + 1) * ld, "iterates"));
    RC(dalloc(c, &c->Qt, (size_t)(c->P + 1) * ld, "fine results"));
    RC(dalloc(c, &c->GQ, (size_t)c->P * ld, "coarse images"));
    RC(dalloc(c, &c->st, (size_t)kSingle * ld, "single states"));
    HC(hipMalloc((void**)&c->ism, 16 * sizeof(int)));
    HC(hipHostMalloc((void**)&c->h_ism, 16 * sizeof(int), hipHostMallocDefault));
    HC(hipMalloc((void**)&c->nrm, 2 * (size_t)(c->P + 1) * sizeof(double)));
    HC(hipHostMalloc((void**)&c->h_nrm, 2 * (size_t)(c->P + 1) * sizeof(double),
                     hipHostMallocDefault));
    changed = true;
  }
  if (wcap > c->wcap) {
    const size_t w = (size_t)wcap * ld;
    RC(dalloc(c, &c->Wk, w, "work"));
    RC(dalloc(c, &c->X, w, "work"));
    RC(dalloc(c, &c->DX, w, "work"));
    RC(dalloc(c, &c->Yb, w, "work"));
    // third scratch block of run_coarse: the stored slow tendency (split
    // scheme with more than one substep chunk) or an RK-3 step (rk3)
    if (c->coarse_chunks.size() > 1 || c->rk3)
      RC(dalloc(c, &c->Rb, w, "work"));
    c->wcap = wcap;
    changed = true;
  }
  if (rcap > c->rcap) {
    double *S2 = nullptr, *D2 = nullptr;
    RC(dalloc(c, &S2, (size_t)rcap * ld, "basis S"));
    int rc = dalloc(c, &D2, (size_t)rcap * ld, "basis D");
    if (rc) {
      (void)hipFree(S2);
      return rc;
    }
    if (c->r > 0) {
      HC(hipMemcpyAsync(S2, c->S, (size_t)c->r * ld * 8, hipMemcpyDeviceToDevice, c->stream));
      HC(hipMemcpyAsync(D2, c->D, (size_t)c->r * ld * 8, hipMemcpyDeviceToDevice, c->stream));
    }
    HC(hipStreamSynchronize(c->stream));
    if (c->S) (void)hipFree(c->S);
    if (c->D) (void)hipFree(c->D);
    c->S = S2;
    c->D = D2;
    c->rcap = rcap;
    changed = true;
  }
  if (changed) {
    const int m = std::max(c->wcap, c->rcap);
    const int w = c->wcap;
    // Partials: column norms use colnorm_blocks(d) per column, projections
    // at most as many (their slice count is capped by gemv_t_blocks).
    // colnorm_blocks is not monotone (it drops where small states switch to
    // longer chunks), so take the larger of d and ld.
    const size_t nblk =
        (size_t)std::max(colnorm_blocks(c->d), colnorm_blocks(c->ld));
    size_t off = 0;
    const size_t part = nblk * m, cvec = m, cm = (size_t)c->rcap * w,
                 gram = (size_t)w * w, t = (size_t)w * w,
                 pcw = (size_t)w * w + 2 * w + 8,
                 tnw = gemm_tn_work(m, w, c->ld), n0 = w;
    const size_t total = part + cvec + cm + gram + 3 * t + pcw + tnw + n0 + 8;
    RC(dalloc(c, &c->small, total, "small"));
    c->small_len = total;
    auto carve = [&](size_t len) {
      double* p = c->small + off;
      off += (len + 7) / 8 * 8;
      return p;
    };
    c->part = carve(part);
    c->cvec = carve(cvec);
    c->Cm = carve(cm);
    c->gram = carve(gram);
    c->T1 = carve(t);
    c->T2 = carve(t);
    c->T3 = carve(t);
    c->pcw = carve(pcw);
    c->tnw = carve(tnw);
    c->n0 = carve(n0);
    c->d_r11sq = c->small + total - 8;
    clear_graphs(c);
  }
  return PR_OK;
}

int prh::retarget(pr_ctx* c, double c_s, double U, double dt_f, double dt_g,
                  const pr_opts* o, double T, double Lx, double Lz) {
  pr_grid g = c->g;
  g.T = T;
  g.Lx = Lx;
  g.Lz = Lz;
  int nf = 0, ng = 0;
  std::string msg;
  if (pr_validate(&g, c_s, U, dt_f, dt_g, c->P, o, &nf, &ng, &msg) != PR_OK)
    return set_error(c, PR_EINVAL, "%s", msg.c_str());
  c->g = g;
  c->c_s = c_s;
  c->U = U;
  c->dt_f = dt_f;
  c->dt_g = dt_g;
  c->o = *o;
  c->n_f = nf;
  c->n_g = ng;
  make_coef(c);
  if (!c->h_tabs.empty())
    return set_error(c, PR_EINVAL, "retarget: only the split scheme with "
                     "advection along x, fourth-order fine acoustics and a "
                     "first-order coarse slow tendency");
  clear_graphs(c);
  c->r = 0;
  if (c->coarse_chunks.size() > 1 && !c->Rb && c->wcap > 0)
    RC(dalloc(c, &c->Rb, (size_t)c->wcap * c->ld, "work"));
  return PR_OK;
}

// ------------------------------------------------------------- fine sweep

struct TileKey {
  int nx, nz, ns, sgn;
  bool operator<(const TileKey& o) const {
    return std::tie(nx, nz, ns, sgn) < std::tie(o.nx, o.nz, o.ns, o.sgn);
  }
};
static std::mutex g_tile_mu;
static std::map<TileKey, std::pair<int, int>> g_tiles;

static void fill_job(const pr_ctx* c, FineJob* j, const double* in, int64_t is,
                     double* out, int64_t os, int ns, int nt, int zc,
                     int block_begin) {
  j->in = in;
  j->out = out;
  j->in_stride = is;
  j->out_stride = os;
  j->nx = c->g.nx;
  j->nz = c->g.nz;
  j->nslices = ns;
  const int tc = fine_tile_cols(nt, c->g.nx);
  j->xtiles = (c->g.nx + tc - 1) / tc;
  j->ztiles = (c->g.nz + zc - 1) / zc;
  j->block_begin = block_begin;
  j->c = c->fc;
}

static hipError_t fine_step_launch(const pr_ctx* c, const double* src,
                                   int64_t ss, double* dst, int64_t ds, int ns,
                                   int nt, int zc) {
  FineLaunch L;
  std::memset(&L, 0, sizeof L);
  L.njobs = 1;
  L.zc = zc;
  fill_job(c, &L.job[0], src, ss, dst, ds, ns, nt, zc, 0);
  L.nblocks = ns * L.job[0].xtiles * L.job[0].ztiles;
  return launch_fine_step(L, nt, c->sgn, c->stream);
}

static void tile_for(pr_ctx* c, int ns, int* nt, int* zc) {
  if (c->o.tile_nt && c->o.tile_zc) {
    *nt = c->o.tile_nt;
    *zc = c->o.tile_zc;
    return;
  }
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tiles.find(TileKey{c->g.nx, c->g.nz, ns, c->sgn});
  if (it != g_tiles.end()) {
    *nt = it->second.first;
    *zc = it->second.second;
  } else {
    *nt = c->o.tile_nt ? c->o.tile_nt : 256;
    *zc = c->o.tile_zc ? c->o.tile_zc : 64;
  }
}

// Picks (threads, rows) of the fused step kernel for ns slices by timing
// every candidate on the context's own buffers (Q -> Qt); the choice only
// changes the speed, never the result.
int prh::autotune(pr_ctx* c, int ns) {
  if (c->tables_f || (c->o.tile_nt && c->o.tile_zc)) return PR_OK;
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    if (g_tiles.count(TileKey{c->g.nx, c->g.nz, ns, c->sgn})) return PR_OK;
  }
  RC(ensure_arena(c, ns, 1));
  if (ns > c->P + 1) return PR_OK;
  // One workgroup per row (no x-halo, the least traffic) is tried first, so
  // that a halo tile has to beat it clearly to be chosen.
  std::vector<int> nts;
  if (fine_full_row(c->g.nx)) nts.push_back(c->g.nx);
  for (int nt : {128, 192, 256})
    if (std::find(nts.begin(), nts.end(), nt) == nts.end()) nts.push_back(nt);
  static const int zcs[] = {12, 20, 28, 32, 60, 64, 124, 128, 252};
  int ncu = 0;
  HC(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount,
                           c->device));
  hipEvent_t e0, e1;
  HC(hipEventCreate(&e0));
  HC(hipEventCreate(&e1));
  float best = 1e30f;
  int bnt = 256, bzc = 64;
  const int zmax = std::max(16, (c->g.nz + 15) / 16 * 16);
  for (int nt : nts) {
    if (c->o.tile_nt && nt != c->o.tile_nt) continue;
    // Besides the fixed list, the chunk heights whose workgroup count fills
    // whole rounds of the machine (m rounds of ncu * blocks-per-CU): a
    // partial last round leaves compute units idle for a whole chunk.
    std::vector<int> cand(zcs, zcs + sizeof zcs / sizeof zcs[0]);
    const int bpc = fine_blocks_per_cu(nt, c->g.nx, c->sgn);
    const int tc = fine_tile_cols(nt, c->g.nx);
    const int64_t strips = (int64_t)ns * ((c->g.nx + tc - 1) / tc);
    for (int m = 1; m <= 4 && bpc > 0; ++m) {
      const int64_t nch = (int64_t)m * ncu * bpc / strips;
      if (nch < 1) continue;
      const int z = (int)((c->g.nz + nch - 1) / nch);
      const int r4 = (z + 3) / 4 * 4;          // multiple of 4
      const int r8 = (z + 3) / 8 * 8 + 4;      // 4 mod 8: zc + 12 fills the unroll
      for (int zc : {r4, r8})
        if (zc >= 8 && std::find(cand.begin(), cand.end(), zc) == cand.end())
          cand.push_back(zc);
    }
    for (int zc : cand) {
      if (c->o.tile_zc && zc != c->o.tile_zc) continue;
      if (zc > zmax && zc != 12) continue;
      HC(fine_step_launch(c, c->Q, c->ld, c->Qt, c->ld, ns, nt, zc));
      float ms = 1e30f;
      for (int r = 0; r < 3; ++r) {
        HC(hipEventRecord(e0, c->stream));
        HC(fine_step_launch(c, c->Q, c->ld, c->Qt, c->ld, ns, nt, zc));
        HC(hipEventRecord(e1, c->stream));
        HC(hipEventSynchronize(e1));
        float one = 0;
        HC(hipEventElapsedTime(&one, e0, e1));
        ms = std::min(ms, one);
      }
      // A later candidate must win by 3% to displace an earlier one, which
      // keeps the choice stable against timing noise.
      if (ms < 0.97f * best) {
        best = ms;
        bnt = nt;
        bzc = zc;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tiles[TileKey{c->g.nx, c->g.nz, ns, c->sgn}] = {bnt, bzc};
  return PR_OK;
}

int prh::run_sweep(pr_ctx* c, const double* in, int64_t is, double* out,
                   int64_t os, double* ping, int64_t ps, int ns, int form) {
  if (ns <= 0) return PR_OK;
  const int nf = c->n_f;
  if (form == PR_FORM_STAGEWISE) {
    // ping holds three blocks of ns states: ping-pong, stage 1, stage 2.
    double* A = ping + (int64_t)ns * ps;
    double* B = ping + 2 * (int64_t)ns * ps;
    const double* src = in;
    int64_t sst = is;
    for (int s = 0; s < nf; ++s) {
      const bool to_out = ((nf - 1 - s) % 2) == 0;
      double* dst = to_out ? out : ping;
      const int64_t dst_s = to_out ? os : ps;
      const double dt = c->fc.dt;
      if (c->tables_f) {
        // the three stages in one launch (the stage buffers stay unused)
        HC(launch_stage3(src, sst, dst, dst_s, c->g.nx, c->g.nz, ns, c->sf,
                         dt / 3.0, 0.5 * dt, dt, c->stream));
      } else {
        HC(launch_fine_stage(src, sst, src, sst, A, ps, c->g.nx, c->g.nz, ns,
                             c->fc, dt / 3.0, c->sgn, c->stream));
        HC(launch_fine_stage(A, ps, src, sst, B, ps, c->g.nx, c->g.nz, ns,
                             c->fc, 0.5 * dt, c->sgn, c->stream));
        HC(launch_fine_stage(B, ps, src, sst, dst, dst_s, c->g.nx, c->g.nz, ns,
                             c->fc, dt, c->sgn, c->stream));
      }
      src = dst;
      sst = dst_s;
    }
    return PR_OK;
  }
  const int tile_ns = form == PR_FORM_PLAIN ? 1 : ns;
  int nt, zc;
  tile_for(c, tile_ns, &nt, &zc);
  const double* src = in;
  int64_t sst = is;
  for (int s = 0; s < nf; ++s) {
    const bool to_out = ((nf - 1 - s) % 2) == 0;
    double* dst = to_out ? out : ping;
    const int64_t dst_s = to_out ? os : ps;
    if (form == PR_FORM_PLAIN) {
      for (int q = 0; q < ns; ++q)
        HC(fine_step_launch(c, src + q * sst, sst, dst + q * dst_s, dst_s, 1,
                            nt, zc));
    } else {
      HC(fine_step_launch(c, src, sst, dst, dst_s, ns, nt, zc));
    }
    src = dst;
    sst = dst_s;
  }
  return PR_OK;
}

// --------------------------------------------------------- coarse propagator

int prh::run_coarse(pr_ctx* c, const double* in, double* out, int ns,
                    int64_t stride, double* pa, double* pb, double* R) {
  if (ns <= 0) return PR_OK;
  if (c->rk3) {
    // n_g RK-3 steps of the upwind right-hand side, one launch each (all
    // three stages), alternating between out and R so that the last one
    // lands in out and no step writes its own input.
    const double dt = c->dt_g;
    const double* src = in;
    for (int st = 0; st < c->n_g; ++st) {
      double* dst = ((c->n_g - 1 - st) % 2 == 0) ? out : R;
      HC(launch_stage3(src, stride, dst, stride, c->g.nx, c->g.nz, ns, c->sg,
                       dt / 3.0, 0.5 * dt, dt, c->stream));
      src = dst;
    }
    return PR_OK;
  }
  const int nch = (int)c->coarse_chunks.size();
  const int total = c->n_g * nch;
  const double* src = in;
  int q = 0;
  for (int step = 0; step < c->n_g; ++step) {
    // The first launch of a step evaluates the frozen slow tendency (from
    // the upwind difference, or with a z-velocity, a rotation or third
    // order from the per-row and per-column weights) and, when the
    // substeps take more than one launch, stores it for the others.
    for (int ch = 0; ch < nch; ++ch, ++q) {
      double* dst = (q == total - 1) ? out : ((q % 2 == 0) ? pa : pb);
      CoarseLaunch L;
      L.in = src;
      L.out = dst;
      L.R = R;
      L.stride = stride;
      L.nx = c->g.nx;
      L.nz = c->g.nz;
      L.nstates = ns;
      L.nsub = c->coarse_chunks[ch];
      L.flags = ch == 0 ? ((c->tables_g ? kCoarseTablesR : kCoarseComputeR) |
                           (nch > 1 ? kCoarseStoreR : 0))
                        : 0;
      L.c = c->cc;
      L.wx = c->sg.wx;
      L.wz = c->sg.wz;
      HC(launch_coarse(L, c->stream));
      src = dst;
    }
  }
  return PR_OK;
}

// -------------------------------------------------------- subspace update

static int gemm_nn_chunked(pr_ctx* c, double* Y, const double* A, int K,
                           const double* C, int ldc, int N, double alpha,
                           double beta) {
  for (int l0 = 0; l0 < N; l0 += 128) {
    const int nn = std::min(128, N - l0);
    HC(launch_gemm_nn(Y + (int64_t)l0 * c->ld, c->ld, A, c->ld, K, C + l0,
                      ldc, nn, c->ld, alpha, beta, c->use_mfma, c->stream));
  }
  return PR_OK;
}

// Subspace update S^{k-1} -> S^k of eq. subspaceUpdate for the b new raw
// columns X0 with fine images FX0 (both at stride ld).  Orthonormalisation
// by two block classical Gram-Schmidt passes against S, then Cholesky QR
// twice on the new block, the first with diagonal pivoting as the rank
// test; every transformation is applied to D(X) = F(X) - G(X) as well, so
// D(S) stays the image of S (eq. Genhance).  Three stages separated by the
// two points where the host needs a rank: update_begin enqueues up to the
// pivoted factorisation and the copy of its rank to pinned memory;
// update_mid (after that copy landed) the second pass; update_end the
// append.
int prh::update_begin(pr_ctx* c, const double* X0, const double* FX0,
                      const double* GX0, int b) {
  c->upd_b = b;
  if (b <= 0) return PR_OK;
  hipStream_t s = c->stream;
  const int64_t ld = c->ld, d = c->d;
  HC(hipMemcpyAsync(c->X, X0, (size_t)b * ld * 8, hipMemcpyDeviceToDevice, s));
  if (GX0) {
    HC(launch_sub(c->DX, FX0, GX0, (int64_t)b * ld, s));
  } else {
    RC(run_coarse(c, c->X, c->DX, b, ld, c->Yb, c->Wk, c->Rb));
    HC(launch_sub(c->DX, FX0, c->DX, (int64_t)b * ld, s));
  }
  HC(launch_colnorm2(c->X, ld, b, d, c->part, c->n0, s));
  if (c->r > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      HC(launch_gemm_tn(c->S, ld, c->r, c->X, ld, b, d, c->Cm, c->tnw,
                        c->use_mfma, s));
      RC(gemm_nn_chunked(c, c->X, c->S, c->r, c->Cm, b, b, -1.0, 1.0));
      RC(gemm_nn_chunked(c, c->DX, c->D, c->r, c->Cm, b, b, -1.0, 1.0));
    }
  }
  HC(launch_gemm_tn(c->X, ld, b, c->X, ld, b, d, c->gram, c->tnw, c->use_mfma, s));
  const double tol2 = c->o.rank_tol * c->o.rank_tol;
  // Gram-based residuals carry an absolute error of about eps * |x|^2, so a
  // direction is trusted only above 1e-7 of its raw norm as well.
  const double rel2 = 1e-14;
  HC(launch_pchol(c->gram, b, c->n0, c->d_r11sq, tol2, rel2, 1, c->T1, c->ism,
                  c->pcw, s));
  HC(hipMemcpyAsync(c->h_ism, c->ism, sizeof(int), hipMemcpyDeviceToHost, s));
  return PR_OK;
}

int prh::update_mid(pr_ctx* c) {
  const int b = c->upd_b;
  if (b <= 0) return PR_OK;
  const int rho = c->h_ism[0];
  c->upd_rho = rho;
  if (rho <= 0) return PR_OK;
  hipStream_t s = c->stream;
  const int64_t ld = c->ld, d = c->d;
  RC(gemm_nn_chunked(c, c->Yb, c->X, b, c->T1, b, rho, 1.0, 0.0));
  HC(launch_gemm_tn(c->Yb, ld, rho, c->Yb, ld, rho, d, c->gram, c->tnw, c->use_mfma, s));
  HC(launch_pchol(c->gram, rho, nullptr, nullptr, 0.0, 0.0, 0, c->T2, c->ism + 1,
                  c->pcw, s));
  HC(hipMemcpyAsync(c->h_ism + 1, c->ism + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  return PR_OK;
}

// The second pass must keep every column the first one kept; its rank
// lands in h_ism[1] once the stream has passed the copy.
int prh::verify_second_pass(pr_ctx* c) {
  const int rho = c->upd_verify;
  c->upd_verify = 0;
  if (rho > 0 && c->h_ism[1] != rho)
    return set_error(c, PR_EDEVICE,
                     "second Cholesky-QR pass broke down (%d of %d columns)",
                     c->h_ism[1], rho);
  return PR_OK;
}

int prh::update_end(pr_ctx* c, bool defer_check) {
  const int b = c->upd_b, rho = c->upd_rho;
  c->upd_b = 0;
  if (b <= 0 || rho <= 0) return PR_OK;
  c->upd_verify = rho;
  if (!defer_check) RC(verify_second_pass(c));
  const int64_t ld = c->ld;
  RC(gemm_nn_chunked(c, c->S + (int64_t)c->r * ld, c->Yb, rho, c->T2, rho, rho,
                     1.0, 0.0));
  HC(launch_small_matmul(c->T1, b, rho, c->T2, rho, c->T3, c->stream));
  RC(gemm_nn_chunked(c, c->D + (int64_t)c->r * ld, c->DX, b, c->T3, b, rho,
                     1.0, 0.0));
  c->r += rho;
  return PR_OK;
}

int prh::krylov_append(pr_ctx* c, const double* X0, const double* FX0, int b) {
  if (b <= 0) return PR_OK;
  RC(ensure_arena(c, b, c->r + b));
  RC(update_begin(c, X0, FX0, nullptr, b));
  HC(hipStreamSynchronize(c->stream));
  RC(update_mid(c));
  HC(hipStreamSynchronize(c->stream));
  return update_end(c);
}

// ------------------------------------------------------------- graphs

template <class F>
static int with_graph(pr_ctx* c, long long key, F&& record) {
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    HC(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = record();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    HC(e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HC(e);
    it = c->graphs.emplace(key, exec).first;
  }
  HC(hipGraphLaunch(it->second, c->stream));
  return PR_OK;
}

static long long gkey(int kind, long long a, long long b) {
  return ((long long)kind << 56) | (a << 28) | b;
}

// ------------------------------------------------------------ the solver

// Grows a lazily allocated device scratch buffer to at least n doubles.
static int ensure_ext(pr_ctx* c, double** p, size_t* len, size_t n) {
  if (*len >= n && *p) return PR_OK;
  RC(dalloc(c, p, n, "scratch"));
  *len = n;
  clear_graphs(c);
  return PR_OK;
}

int prh::coarse_init(pr_ctx* c) {
  for (int i = 0; i < c->P; ++i)
    RC(run_coarse(c, c->Q + (int64_t)i * c->ld, c->Q + (int64_t)(i + 1) * c->ld,
                  1, c->ld, single(c, kTa), single(c, kTb), single(c, kRs)));
  // G(q^0_i) = q^0_{i+1}: the coarse images of the first iterates.
  HC(hipMemcpyAsync(c->GQ, c->Q + c->ld, (size_t)c->P * c->ld * 8,
                    hipMemcpyDeviceToDevice, c->stream));
  return PR_OK;
}

int prh::chain(pr_ctx* c, int k) {
  const int P = c->P;
  const int64_t ld = c->ld, d = c->d;
  double* da = single(c, kDa);
  double* db = single(c, kDb);
  double* g = single(c, kG);
  hipStream_t s = c->stream;
  // Slice k is converged (q^{k+1}_k = q^k_k), so q^{k+1}_{k+1} = qt^k_{k+1}.
  HC(launch_combine(c->Q + (int64_t)(k + 1) * ld, k + 1 < P ? da : nullptr,
                    c->Qt + (int64_t)(k + 1) * ld, nullptr, nullptr, ld, 0,
                    nullptr, d, s));
  double* y = single(c, kY);
  for (int i = k + 1; i < P; ++i) {
    // K(delta) = G(delta) + D(S) (S^T delta): the fine part (two passes over
    // the basis) runs on the side stream while the coarse step runs here;
    // both join before the combine.
    if (c->r > 0) {
      HC(hipEventRecord(c->ev_fork, s));
      HC(hipStreamWaitEvent(c->side, c->ev_fork, 0));
      HC(launch_gemv_t(c->S, ld, c->r, da, d, c->part, c->cvec, c->side));
      HC(launch_lincomb(y, nullptr, c->D, ld, c->r, c->cvec, d, c->side));
      HC(hipEventRecord(c->ev_join, c->side));
    }
    RC(run_coarse(c, da, g, 1, ld, single(c, kTa), single(c, kTb), single(c, kRs)));
    if (c->r > 0) HC(hipStreamWaitEvent(s, c->ev_join, 0));
    // G(q^{k+1}_i) = G(q^k_i) + G(delta_i) by linearity.
    HC(launch_combine3(c->Q + (int64_t)(i + 1) * ld, i + 1 < P ? db : nullptr,
                       c->Qt + (int64_t)(i + 1) * ld, g, c->r > 0 ? y : nullptr,
                       c->GQ + (int64_t)i * ld, d, s));
    std::swap(da, db);
  }
  return PR_OK;
}

static int copy_state_in(pr_ctx* c, double* dst, const double* src, int mem) {
  HC(hipMemcpyAsync(dst, src, (size_t)c->d * 8,
                    mem == PR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                    c->stream));
  return PR_OK;
}

static int copy_state_out(pr_ctx* c, double* dst, const double* src, int mem) {
  HC(hipMemcpyAsync(dst, src, (size_t)c->d * 8,
                    mem == PR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                    c->stream));
  return PR_OK;
}

// One window (parallel step) of Algorithm 2 (or 1): u0 in memory kind
// mem_in, or NULL to start from the previous window's final state Q[P];
// U_K (optional) and slices (optional) in memory kind mem.  The final state
// stays in Q[P].
static int solve_window(pr_ctx* c, const double* u0, int mem_in, int32_t K,
                        double* U_K, double* slices, int mem, bool krylov) {
  const int P = c->P;
  int Keff = std::min<int>(K, P);  // lowered by the stopping criterion
  const int64_t ld = c->ld;
  const int form = c->o.form;
  RC(ensure_arena(c, P, krylov ? P * std::max(Keff, 1) : 1));
  hipStream_t s = c->stream;
  if (form == PR_FORM_BATCHED) {
    for (int k = 0; k < Keff; ++k) {
      const int i0 = c->o.skip_converged ? k : 0;
      RC(autotune(c, P - i0));
      if (!c->o.skip_converged) break;
    }
  } else if (form == PR_FORM_PLAIN) {
    RC(autotune(c, 1));
  }
  std::vector<hipEvent_t> ev(3 * Keff + 3);
  for (auto& e : ev) HC(hipEventCreate(&e));
  struct EvGuard {
    std::vector<hipEvent_t>& v;
    ~EvGuard() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } guard{ev};

  c->r = 0;
  c->upd_verify = 0;
  HC(hipMemsetAsync(c->d_r11sq, 0, sizeof(double), s));
  HC(hipMemsetAsync(c->ism + 2, 0, sizeof(int), s));
  if (u0)
    RC(copy_state_in(c, c->Q, u0, mem_in));
  else
    HC(hipMemcpyAsync(c->Q, c->Q + (int64_t)P * ld, (size_t)c->d * 8,
                      hipMemcpyDeviceToDevice, s));
  HC(hipEventRecord(ev[0], s));
  RC(with_graph(c, gkey(1, 0, 0), [&] { return coarse_init(c); }));
  HC(hipEventRecord(ev[1], s));
  c->stats = pr_stats{};
  int64_t pts = 0;
  for (int k = 0; k < Keff; ++k) {
    const int i0 = c->o.skip_converged ? k : 0;
    const int ns = P - i0;
    auto sweep = [&] {
      return run_sweep(c, c->Q + (int64_t)i0 * ld, ld, c->Qt + (int64_t)(i0 + 1) * ld,
                       ld, c->Wk, ld, ns, form);
    };
    if (form == PR_FORM_BATCHED)
      RC(with_graph(c, gkey(2, i0, 0), sweep));
    else if (form == PR_FORM_STAGEWISE) {
      // the stage buffers are allocated before the capture; growing them
      // later drops the captured graphs
      RC(ensure_ext(c, &c->ext_ping, &c->ext_ping_len, (size_t)3 * ns * ld));
      RC(with_graph(c, gkey(5, i0, 0), [&] {
        return run_sweep(c, c->Q + (int64_t)i0 * ld, ld,
                         c->Qt + (int64_t)(i0 + 1) * ld, ld, c->ext_ping, ld,
                         ns, form);
      }));
    } else
      RC(sweep());
    pts += (int64_t)ns * c->n * c->n_f;
    HC(hipEventRecord(ev[2 + 3 * k], s));
    if (krylov) {
      RC(ensure_arena(c, P - k, c->r + P - k));
      RC(update_begin(c, c->Q + (int64_t)k * ld, c->Qt + (int64_t)(k + 1) * ld,
                      c->GQ + (int64_t)k * ld, P - k));
      HC(hipStreamSynchronize(s));
      // the rank of the previous update's second pass has landed too
      RC(verify_second_pass(c));
      RC(update_mid(c));
      // the append needs only the first pass's rank; the second pass's is
      // checked at the next wait, so the host does not stop the stream here
      RC(update_end(c, true));
    }
    HC(hipEventRecord(ev[3 + 3 * k], s));
    const int rr = c->r;
    // Stopping criterion (Section 2.1): the chain changes slices k+1..P;
    // keep their old values in the (now free) work block X.
    const bool stop = c->o.stop_tol > 0;
    if (stop) {
      RC(ensure_arena(c, P - k, c->r));
      HC(hipMemcpyAsync(c->X, c->Q + (int64_t)(k + 1) * ld,
                        (size_t)(P - k) * ld * 8, hipMemcpyDeviceToDevice, s));
    }
    RC(with_graph(c, gkey(3, k, rr), [&] { return chain(c, k); }));
    HC(hipEventRecord(ev[4 + 3 * k], s));
    if (k < 64) c->stats.rank[k] = c->r;
    if (stop) {
      // ||q^{k+1}_i - q^k_i||^2 for i = k+1..P (the others are unchanged)
      // and ||q^{k+1}_i||^2 for i = 1..P.
      HC(launch_sub(c->X, c->Q + (int64_t)(k + 1) * ld, c->X,
                    (int64_t)(P - k) * ld, s));
      HC(launch_colnorm2(c->X, ld, P - k, c->d, c->part, c->nrm, s));
      HC(launch_colnorm2(c->Q + ld, ld, P, c->d, c->part, c->nrm + (P + 1), s));
      HC(hipMemcpyAsync(c->h_nrm, c->nrm, 2 * (size_t)(P + 1) * 8,
                        hipMemcpyDeviceToHost, s));
      HC(hipStreamSynchronize(s));
      double dmax = 0, qmax = 0;
      for (int i = 0; i < P - k; ++i) dmax = std::max(dmax, c->h_nrm[i]);
      for (int i = 0; i < P; ++i) qmax = std::max(qmax, c->h_nrm[P + 1 + i]);
      const double rk = qmax > 0 ? std::sqrt(dmax) / std::sqrt(qmax) : 0.0;
      if (k < 64) c->stats.residual[k] = rk;
      if (rk <= c->o.stop_tol) {
        Keff = k + 1;
        break;
      }
    }
  }
  HC(launch_check_finite(c->Q + (int64_t)P * ld, c->d, c->ism + 2, s));
  HC(hipMemcpyAsync(c->h_ism + 2, c->ism + 2, sizeof(int), hipMemcpyDeviceToHost, s));
  HC(hipEventRecord(ev[2 + 3 * Keff], s));
  HC(hipStreamSynchronize(s));
  RC(verify_second_pass(c));
  if (c->h_ism[2]) return set_error(c, PR_EDIVERGED, "iterate is not finite");
  auto el = [&](int a, int b) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return (double)ms;
  };
  c->stats.iterations = Keff;
  c->stats.ms_coarse_init = el(0, 1);
  for (int k = 0; k < Keff; ++k) {
    c->stats.ms_fine += el(1 + 3 * k, 2 + 3 * k);
    c->stats.ms_update += el(2 + 3 * k, 3 + 3 * k);
    c->stats.ms_chain += el(3 + 3 * k, 4 + 3 * k);
  }
  c->stats.ms_total = el(0, 2 + 3 * Keff);
  c->stats.fine_point_steps = pts;
  if (form != PR_FORM_STAGEWISE && Keff > 0) {
    // the first sweep covers the most slices (the plain form tunes for one)
    int nt = 0, zc = 0;
    tile_for(c, form == PR_FORM_PLAIN ? 1 : P, &nt, &zc);
    c->stats.tile_nt = nt;
    c->stats.tile_zc = zc;
  }
  if (U_K) RC(copy_state_out(c, U_K, c->Q + (int64_t)P * ld, mem));
  if (slices) {
    HC(hipMemcpy2DAsync(slices, (size_t)c->d * 8, c->Q, (size_t)ld * 8,
                        (size_t)c->d * 8, P + 1,
                        mem == PR_MEM_HOST ? hipMemcpyDeviceToHost
                                           : hipMemcpyDeviceToDevice,
                        s));
  }
  HC(hipStreamSynchronize(s));
  return PR_OK;
}

// Section 2.1: windows (parallel steps) run one after the other, each from
// the previous window's final state and with an empty subspace.  Timings
// and fine point-steps are summed over the windows; iterations, ranks and
// residuals are the last window's.
static int solve_impl(pr_ctx* c, const double* u0, int32_t K, double* U_K,
                      double* slices, int mem, bool krylov) {
  if (!u0 || !U_K) return set_error(c, PR_EINVAL, "null state pointer");
  if (K < 0) return set_error(c, PR_EINVAL, "K must be >= 0");
  if (mem != PR_MEM_HOST && mem != PR_MEM_DEVICE)
    return set_error(c, PR_EINVAL, "bad mem kind");
  const int M = c->o.windows;
  if (M <= 1) return solve_window(c, u0, mem, K, U_K, slices, mem, krylov);
  pr_stats acc{};
  for (int w = 0; w < M; ++w) {
    const bool last = w == M - 1;
    RC(solve_window(c, w == 0 ? u0 : nullptr, mem, K,
                    last ? U_K : nullptr, last ? slices : nullptr, mem,
                    krylov));
    acc.ms_total += c->stats.ms_total;
    acc.ms_coarse_init += c->stats.ms_coarse_init;
    acc.ms_fine += c->stats.ms_fine;
    acc.ms_update += c->stats.ms_update;
    acc.ms_chain += c->stats.ms_chain;
    acc.fine_point_steps += c->stats.fine_point_steps;
  }
  acc.iterations = c->stats.iterations;
  acc.tile_nt = c->stats.tile_nt;
  acc.tile_zc = c->stats.tile_zc;
  std::memcpy(acc.rank, c->stats.rank, sizeof acc.rank);
  std::memcpy(acc.residual, c->stats.residual, sizeof acc.residual);
  c->stats = acc;
  return PR_OK;
}

// ------------------------------------------------------------------ C ABI

int pr_check_stability_impl(const pr_grid* g, double c_s, double U,
                            double dt_f, double dt_g, const pr_opts* o,
                            double* rho_f, double* rho_g);

extern "C" int pr_footprint(const pr_grid* g, int32_t P, int32_t K,
                            size_t* bytes) {
  if (!g || !bytes || P < 1 || K < 0 || g->nx < 8 || g->nz < 8) return PR_EINVAL;
  const int64_t d = 3LL * g->nx * g->nz;
  const int64_t ld = (d + 63) / 64 * 64;
  const int64_t states = 2LL * P * std::max(K, 1) + 2LL * (P + 1) + 5LL * P + kSingle;
  const int64_t m = std::max<int64_t>(P, (int64_t)P * std::max(K, 1));
  const int64_t small = (d + 2047) / 2048 * m + m * P + 4LL * P * P + m + 64 +
                        (int64_t)gemm_tn_work((int)m, P, ld);
  *bytes = (size_t)((states * ld + small) * 8);
  return PR_OK;
}

extern "C" int pr_create_ex(const pr_grid* g, double c_s, double U,
                            double dt_f, double dt_g, int32_t P,
                            const pr_opts* o, void* hip_stream, pr_ctx** out) {
  if (!out) return set_error(nullptr, PR_EINVAL, "null output pointer");
  *out = nullptr;
  pr_opts def;
  pr_opts_default(&def);
  if (!o) o = &def;
  int nf = 0, ng = 0;
  std::string msg;
  int rc = pr_validate(g, c_s, U, dt_f, dt_g, P, o, &nf, &ng, &msg);
  if (rc) return set_error(nullptr, rc, "%s", msg.c_str());
  double rf = 0, rg = 0;
  rc = pr_check_stability_impl(g, c_s, U, dt_f, dt_g, o, &rf, &rg);
  if (rc) return set_error(nullptr, rc, "stability scan failed");
  // Enforced for a constant velocity only: with a rotation the radii are a
  // frozen-coefficient estimate, which exceeds 1 for propagators that are
  // stable on the rotating flow (the coarse-CFL-4 runs of Section 3.2).
  if (o->gamma == 0.0 && (rf > 1.0 + 1e-12 || rg > 1.0 + 1e-12))
    return set_error(nullptr, PR_EUNSTABLE,
                     "unstable propagator: spectral radius fine %.15g, coarse %.15g",
                     rf, rg);
  pr_ctx* c = new pr_ctx();
  c->g = *g;
  c->c_s = c_s;
  c->U = U;
  c->dt_f = dt_f;
  c->dt_g = dt_g;
  c->P = P;
  c->o = *o;
  c->n_f = nf;
  c->n_g = ng;
  c->n = (int64_t)g->nx * g->nz;
  c->d = 3 * c->n;
  c->ld = (c->d + 63) / 64 * 64;
  make_coef(c);
  if (c->tables_f) c->o.form = PR_FORM_STAGEWISE;  // only stage kernels
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) {
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreate(&c->stream);
      c->own_stream = true;
    }
  }
  if (e == hipSuccess) e = hipStreamCreate(&c->side);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error(nullptr, PR_EDEVICE, "HIP device/stream: %s", hipGetErrorString(e));
    pr_destroy(c);
    return PR_EDEVICE;
  }
  if (upload_tables(c) != PR_OK) {
    const int rc = c->tabs ? PR_EDEVICE : PR_ENOMEM;
    set_error(nullptr, rc, "stage weights: %s", c->err.c_str());
    pr_destroy(c);
    return rc;
  }
  *out = c;
  return PR_OK;
}

extern "C" int pr_create(const pr_grid* g, double c_s, double U, double dt_f,
                         double dt_g, int32_t P, pr_ctx** out) {
  return pr_create_ex(g, c_s, U, dt_f, dt_g, P, nullptr, nullptr, out);
}

extern "C" void pr_destroy(pr_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  clear_graphs(c);
  double* bufs[] = {c->Q, c->Qt, c->GQ, c->Wk, c->X, c->DX, c->Yb, c->Rb, c->st,
                    c->S, c->D, c->small, c->ext_ping, c->ext_io};
  for (double* p : bufs)
    if (p) (void)hipFree(p);
  if (c->tabs) (void)hipFree(c->tabs);
  if (c->ism) (void)hipFree(c->ism);
  if (c->h_ism) (void)hipHostFree(c->h_ism);
  if (c->nrm) (void)hipFree(c->nrm);
  if (c->h_nrm) (void)hipHostFree(c->h_nrm);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" int pr_set_form(pr_ctx* c, int32_t form) {
  if (!c) return PR_EINVAL;
  if (form < 0 || form > PR_FORM_STAGEWISE)
    return set_error(c, PR_EINVAL, "unknown form %d", form);
  // Right-hand sides with per-row or per-column weights have only the
  // stage kernels.
  c->o.form = c->tables_f ? PR_FORM_STAGEWISE : form;
  return PR_OK;
}

extern "C" int pr_set_mfma(pr_ctx* c, int32_t on) {
  if (!c) return PR_EINVAL;
  c->use_mfma = on != 0;
  return PR_OK;
}

static int check_mem(pr_ctx* c, int mem) {
  if (mem != PR_MEM_HOST && mem != PR_MEM_DEVICE)
    return set_error(c, PR_EINVAL, "mem must be PR_MEM_HOST or PR_MEM_DEVICE");
  return PR_OK;
}

extern "C" int pr_fine_sweep(pr_ctx* c, const double* Q, double* FQ,
                             int32_t nslices, int mem) {
  if (!c) return PR_EINVAL;
  RC(check_mem(c, mem));
  if (!Q || !FQ) return set_error(c, PR_EINVAL, "null state pointer");
  if (nslices < 1 || nslices > 4096)
    return set_error(c, PR_EINVAL, "nslices must be in [1, 4096]");
  const int64_t d = c->d, ns = nslices;
  const int form = c->o.form;
  const size_t pingn = (size_t)(form == PR_FORM_STAGEWISE ? 3 : 1) * ns * d;
  RC(ensure_ext(c, &c->ext_ping, &c->ext_ping_len, pingn));
  if (form == PR_FORM_BATCHED) RC(autotune(c, nslices));
  else if (form == PR_FORM_PLAIN) RC(autotune(c, 1));
  const double* in = Q;
  double* out = FQ;
  if (mem == PR_MEM_HOST) {
    RC(ensure_ext(c, &c->ext_io, &c->ext_io_len, (size_t)2 * ns * d));
    HC(hipMemcpyAsync(c->ext_io, Q, (size_t)ns * d * 8, hipMemcpyHostToDevice, c->stream));
    in = c->ext_io;
    out = c->ext_io + ns * d;
  } else {
    const double* qe = Q + ns * d;
    const double* fe = FQ + ns * d;
    if (!(qe <= FQ || fe <= Q))
      return set_error(c, PR_EINVAL, "Q and FQ overlap");
  }
  RC(run_sweep(c, in, d, out, d, c->ext_ping, d, nslices, form));
  if (mem == PR_MEM_HOST)
    HC(hipMemcpyAsync(FQ, out, (size_t)ns * d * 8, hipMemcpyDeviceToHost, c->stream));
  HC(hipStreamSynchronize(c->stream));
  return PR_OK;
}

extern "C" int pr_coarse_step(pr_ctx* c, const double* q, double* gq,
                              int use_krylov, int mem) {
  if (!c) return PR_EINVAL;
  RC(check_mem(c, mem));
  if (!q || !gq) return set_error(c, PR_EINVAL, "null state pointer");
  RC(ensure_arena(c, c->P, 1));
  double* io = single(c, kIo);
  double* g = single(c, kG);
  RC(copy_state_in(c, io, q, mem));
  RC(run_coarse(c, io, g, 1, c->ld, single(c, kTa), single(c, kTb), single(c, kRs)));
  if (use_krylov && c->r > 0) {
    HC(launch_gemv_t(c->S, c->ld, c->r, io, c->d, c->part, c->cvec, c->stream));
    HC(launch_lincomb(g, g, c->D, c->ld, c->r, c->cvec, c->d, c->stream));
  }
  RC(copy_state_out(c, gq, g, mem));
  HC(hipStreamSynchronize(c->stream));
  return PR_OK;
}

extern "C" int pr_krylov_reset(pr_ctx* c) {
  if (!c) return PR_EINVAL;
  c->r = 0;
  if (c->d_r11sq) HC(hipMemsetAsync(c->d_r11sq, 0, sizeof(double), c->stream));
  HC(hipStreamSynchronize(c->stream));
  return PR_OK;
}

extern "C" int pr_reserve_basis(pr_ctx* c, int32_t max_vectors) {
  if (!c) return PR_EINVAL;
  if (max_vectors < 1 || max_vectors > 65536)
    return set_error(c, PR_EINVAL, "max_vectors must be in [1, 65536]");
  RC(ensure_arena(c, c->P, max_vectors));
  HC(hipStreamSynchronize(c->stream));
  return PR_OK;
}

extern "C" int pr_krylov_update(pr_ctx* c, const double* Q, const double* FQ,
                                int32_t m, int32_t* rank_out, int mem) {
  if (!c) return PR_EINVAL;
  RC(check_mem(c, mem));
  if (m < 0 || m > 4096) return set_error(c, PR_EINVAL, "m must be in [0, 4096]");
  if (m > 0 && (!Q || !FQ)) return set_error(c, PR_EINVAL, "null state pointer");
  if (m > 0) {
    if (!c->S) RC(ensure_arena(c, std::max<int>(c->P, m), c->P * c->P));
    if (c->r + m > c->rcap)
      return set_error(c, PR_ENOMEM, "basis capacity %d exceeded (have %d, adding %d)",
                       c->rcap, c->r, m);
    const int64_t ld = c->ld, d = c->d;
    RC(ensure_ext(c, &c->ext_io, &c->ext_io_len, (size_t)2 * m * ld));
    const hipMemcpyKind k =
        mem == PR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HC(hipMemsetAsync(c->ext_io, 0, (size_t)2 * m * ld * 8, c->stream));
    HC(hipMemcpy2DAsync(c->ext_io, ld * 8, Q, d * 8, d * 8, m, k, c->stream));
    HC(hipMemcpy2DAsync(c->ext_io + (int64_t)m * ld, ld * 8, FQ, d * 8, d * 8, m, k,
                        c->stream));
    RC(krylov_append(c, c->ext_io, c->ext_io + (int64_t)m * ld, m));
  }
  HC(hipStreamSynchronize(c->stream));
  if (rank_out) *rank_out = c->r;
  return PR_OK;
}

extern "C" int pr_solve(pr_ctx* c, const double* u0, int32_t K, double* U_K,
                        double* slices_or_NULL, int mem) {
  if (!c) return PR_EINVAL;
  return solve_impl(c, u0, K, U_K, slices_or_NULL, mem, true);
}

extern "C" int pr_solve_parareal(pr_ctx* c, const double* u0, int32_t K,
                                 double* U_K, double* slices_or_NULL, int mem) {
  if (!c) return PR_EINVAL;
  return solve_impl(c, u0, K, U_K, slices_or_NULL, mem, false);
}

extern "C" int pr_serial_fine(pr_ctx* c, const double* u0, int32_t nslices,
                              double* out, int mem) {
  if (!c) return PR_EINVAL;
  RC(check_mem(c, mem));
  if (!u0 || !out) return set_error(c, PR_EINVAL, "null state pointer");
  if (nslices < 0 || nslices > 1 << 20)
    return set_error(c, PR_EINVAL, "nslices out of range");
  RC(ensure_arena(c, c->P, 1));
  const int form = c->o.form == PR_FORM_STAGEWISE ? PR_FORM_STAGEWISE : PR_FORM_BATCHED;
  if (form == PR_FORM_STAGEWISE)
    RC(ensure_ext(c, &c->ext_ping, &c->ext_ping_len, (size_t)3 * c->ld));
  else
    RC(autotune(c, 1));
  double* a = single(c, kIo);
  double* b = single(c, kTa);
  double* ping = form == PR_FORM_STAGEWISE ? c->ext_ping : single(c, kTb);
  RC(copy_state_in(c, a, u0, mem));
  // Two slices per graph replay: a -> b -> a.
  const int pairs = nslices / 2;
  if (pairs > 0) {
    auto two = [&] {
      RC(run_sweep(c, a, c->ld, b, c->ld, ping, c->ld, 1, form));
      return run_sweep(c, b, c->ld, a, c->ld, ping, c->ld, 1, form);
    };
    // one graph per form: the batched and the stage form capture
    // different launches over the same buffers
    const long long key = gkey(form == PR_FORM_BATCHED ? 4 : 6, 0, 0);
    for (int p = 0; p < pairs; ++p) RC(with_graph(c, key, two));
  }
  double* res = a;
  if (nslices % 2) {
    RC(run_sweep(c, a, c->ld, b, c->ld, ping, c->ld, 1, form));
    res = b;
  }
  RC(copy_state_out(c, out, res, mem));
  HC(hipStreamSynchronize(c->stream));
  return PR_OK;
}

extern "C" int pr_get_stats(const pr_ctx* c, pr_stats* s) {
  if (!c || !s) return PR_EINVAL;
  *s = c->stats;
  return PR_OK;
}

extern "C" const char* pr_strerror(int code) {
  switch (code) {
    case PR_OK: return "ok";
    case PR_EINVAL: return "invalid argument";
    case PR_ENOMEM: return "out of device memory";
    case PR_EDEVICE: return "HIP device error";
    case PR_EUNSTABLE: return "unstable propagator";
    case PR_EAGAIN: return "pending";
    case PR_EBUSY: return "queue full";
    case PR_EDIVERGED: return "iterate not finite";
    case PR_ENOTFOUND: return "unknown ticket";
    default: return "unknown error";
  }
}

extern "C" const char* pr_last_error(const pr_ctx* c) {
  return c ? c->err.c_str() : g_err.c_str();
}
