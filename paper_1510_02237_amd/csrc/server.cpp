// Continuous-batching server for KSE-Parareal solves on one device.
//
// A scheduler thread owns all GPU work.  Each admitted solve keeps its
// iterates, basis S and images D(S) resident in its own context arena and
// runs as a state machine on its own stream:
//   coarse initialisation -> K x { fine sweep -> subspace update -> serial
//   correction } -> result copy.
// The fine sweeps of every resident solve that is in its sweep phase are
// fused: each scheduler tick issues one fused RK-3 step launch (on a shared
// sweep stream) whose job list holds the current step of each of those
// solves, so solves of different grids, slice counts and velocities share
// the device while the serial parts of others run on their own streams.
// Ordering between a solve's stream and the sweep stream uses events only;
// the host waits (by polling) only where it must read a rank in the
// subspace update and at completion.
//
// Requests are admitted in arrival order while their footprint fits the
// memory budget and a slot is free; contexts of finished solves are kept
// in a pool and reused by later solves with the same grid and slice count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "ctx.h"

using namespace prh;

int pr_validate(const pr_grid* g, double c_s, double U, double dt_f,
                double dt_g, int32_t P, const pr_opts* o, int* nf, int* ng,
                std::string* msg);
int pr_check_stability_impl(const pr_grid* g, double c_s, double U,
                            double dt_f, double dt_g, const pr_opts* o,
                            double* rho_f, double* rho_g);

namespace {

double now_s() {
  return std::chrono::duration<double>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket = 0;
  pr_grid g{};
  double c_s = 0, U = 0, dt_f = 0, dt_g = 0;
  int P = 0, K = 0;
  pr_opts o{};
  std::vector<double> u0;
  double t_submit = 0;
  size_t bytes = 0;
};

enum Phase { kSweep, kUpd1, kUpd2, kFinish, kDrain, kDone };

struct Active {
  Request req;
  pr_ctx* c = nullptr;
  int K = 0;
  int k = 0;
  Phase phase = kSweep;
  int step = 0;
  int i0 = 0, ns = 0;
  bool joined = false;
  const double* src = nullptr;
  hipEvent_t ev_ready = nullptr, ev_sweep = nullptr, ev_host = nullptr;
  double* h_buf = nullptr;  // pinned staging for u0 and U_K
  size_t bytes = 0;         // device memory held by the context
  int rc = PR_OK;
  bool cancelled = false;
};

struct Result {
  std::vector<double> uk;
  double latency = 0;
  int rc = PR_OK;
};

struct PoolKey {
  int nx, nz, P;
  bool operator<(const PoolKey& o) const {
    return std::tie(nx, nz, P) < std::tie(o.nx, o.nz, o.P);
  }
};

struct Pooled {
  pr_ctx* c;
  size_t bytes;
  double* h_buf;
};

constexpr size_t kQueueCap = 4096;
constexpr int kServerNT = 192, kServerZC = 28;

}  // namespace

struct pr_server {
  int device = 0;
  size_t budget = 0;
  int max_inflight = 1;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Request> queue;
  std::map<uint64_t, Result> done;
  std::set<uint64_t> cancel_req;
  std::set<uint64_t> live;  // tickets queued or active
  uint64_t next_ticket = 1;
  std::string err;
  std::atomic<bool> stop{false};
  std::thread th;
  // scheduler-owned
  size_t used = 0;  // bytes held by active and pooled contexts
  std::vector<Active*> active;
  std::multimap<PoolKey, Pooled> pool;
  std::deque<std::multimap<PoolKey, Pooled>::iterator> pool_lru;
  hipStream_t sweep_stream = nullptr;

  void run();
  bool admit();
  int start(Active* a);
  void release(Active* a, bool to_pool);
  bool progress();
  bool sweep_tick();
  void finish(Active* a);
  void evict_pool_one();
};

static int set_serr(pr_server* s, int code, const std::string& m) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->err = m;
  return code;
}

void pr_server::evict_pool_one() {
  if (pool_lru.empty()) return;
  auto it = pool_lru.front();
  pool_lru.pop_front();
  used -= it->second.bytes;
  pr_destroy(it->second.c);
  if (it->second.h_buf) (void)hipHostFree(it->second.h_buf);
  pool.erase(it);
}

// Returns true if something was admitted.
bool pr_server::admit() {
  bool any = false;
  while (true) {
    Request req;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (queue.empty() || (int)active.size() >= max_inflight) break;
      Request& head = queue.front();
      if (cancel_req.count(head.ticket)) {
        cancel_req.erase(head.ticket);
        live.erase(head.ticket);
        queue.pop_front();
        cv_done.notify_all();
        continue;
      }
      // Memory: reuse a pooled context of the same shape, else make room.
      const PoolKey key{head.g.nx, head.g.nz, head.P};
      const bool pooled = pool.count(key) > 0;
      if (!pooled) {
        while (used + head.bytes > budget && !pool_lru.empty()) evict_pool_one();
        if (used + head.bytes > budget) {
          if (active.empty()) {
            Result r;
            r.rc = PR_ENOMEM;
            done[head.ticket] = std::move(r);
            live.erase(head.ticket);
            err = "request footprint exceeds the memory budget";
            queue.pop_front();
            cv_done.notify_all();
            continue;
          }
          break;  // wait for a running solve to free memory
        }
      }
      req = std::move(head);
      queue.pop_front();
    }
    Active* a = new Active();
    a->req = std::move(req);
    const int rc = start(a);
    if (rc) {
      a->rc = rc;
      std::lock_guard<std::mutex> lk(mu);
      Result r;
      r.rc = rc;
      err = a->c ? a->c->err : "could not start the solve";
      done[a->req.ticket] = std::move(r);
      live.erase(a->req.ticket);
      cv_done.notify_all();
      release(a, false);
      delete a;
      continue;
    }
    active.push_back(a);
    any = true;
  }
  return any;
}

int pr_server::start(Active* a) {
  const Request& q = a->req;
  const PoolKey key{q.g.nx, q.g.nz, q.P};
  const int K = std::min(q.K, q.P);
  a->K = K;
  auto it = pool.find(key);
  bool reused = false;
  if (it != pool.end() && it->second.c->rcap >= q.P * std::max(K, 1)) {
    a->c = it->second.c;
    a->h_buf = it->second.h_buf;
    a->bytes = it->second.bytes;
    pool_lru.erase(std::find(pool_lru.begin(), pool_lru.end(), it));
    pool.erase(it);
    reused = true;
    const int rc = retarget(a->c, q.c_s, q.U, q.dt_f, q.dt_g, &q.o, q.g.T,
                            q.g.Lx, q.g.Lz);
    if (rc) return rc;
  } else {
    int rc = pr_create_ex(&q.g, q.c_s, q.U, q.dt_f, q.dt_g, q.P, &q.o, nullptr, &a->c);
    if (rc) return rc;
    a->bytes = q.bytes;
    used += a->bytes;
    rc = ensure_arena(a->c, q.P, q.P * std::max(K, 1));
    if (rc) return rc;
    if (hipHostMalloc((void**)&a->h_buf, (size_t)a->c->d * 8, hipHostMallocDefault) !=
        hipSuccess) {
      a->h_buf = nullptr;
      return PR_ENOMEM;
    }
  }
  (void)reused;
  pr_ctx* c = a->c;
  c->o.form = PR_FORM_BATCHED;
  if (hipEventCreateWithFlags(&a->ev_ready, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&a->ev_sweep, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&a->ev_host, hipEventDisableTiming) != hipSuccess)
    return PR_EDEVICE;
  std::memcpy(a->h_buf, q.u0.data(), (size_t)c->d * 8);
  c->r = 0;
  if (hipMemsetAsync(c->d_r11sq, 0, sizeof(double), c->stream) != hipSuccess ||
      hipMemsetAsync(c->ism + 2, 0, sizeof(int), c->stream) != hipSuccess ||
      hipMemcpyAsync(c->Q, a->h_buf, (size_t)c->d * 8, hipMemcpyHostToDevice,
                     c->stream) != hipSuccess)
    return PR_EDEVICE;
  int rc = coarse_init(c);
  if (rc) return rc;
  if (hipEventRecord(a->ev_ready, c->stream) != hipSuccess) return PR_EDEVICE;
  a->k = 0;
  if (K == 0) {
    finish(a);
  } else {
    a->phase = kSweep;
    a->step = 0;
    a->i0 = 0;
    a->ns = q.P;
    a->joined = false;
  }
  return PR_OK;
}

// Enqueues the finite check and the result copy; completion is polled.
void pr_server::finish(Active* a) {
  pr_ctx* c = a->c;
  const int64_t P = c->P;
  (void)launch_check_finite(c->Q + P * c->ld, c->d, c->ism + 2, c->stream);
  (void)hipMemcpyAsync(c->h_ism + 2, c->ism + 2, sizeof(int), hipMemcpyDeviceToHost,
                       c->stream);
  (void)hipMemcpyAsync(a->h_buf, c->Q + P * c->ld, (size_t)c->d * 8,
                       hipMemcpyDeviceToHost, c->stream);
  (void)hipEventRecord(a->ev_host, c->stream);
  a->phase = kFinish;
}

void pr_server::release(Active* a, bool to_pool) {
  if (a->ev_ready) (void)hipEventDestroy(a->ev_ready);
  if (a->ev_sweep) (void)hipEventDestroy(a->ev_sweep);
  if (a->ev_host) (void)hipEventDestroy(a->ev_host);
  if (!a->c) return;
  if (to_pool) {
    const PoolKey key{a->c->g.nx, a->c->g.nz, a->c->P};
    auto it = pool.emplace(key, Pooled{a->c, a->bytes, a->h_buf});
    pool_lru.push_back(it);
  } else {
    (void)hipStreamSynchronize(a->c->stream);
    pr_destroy(a->c);
    if (a->h_buf) (void)hipHostFree(a->h_buf);
    used -= std::min(used, a->bytes);
  }
  a->c = nullptr;
}

// Advances the host-polled phases.  Returns true if anything moved.
bool pr_server::progress() {
  bool moved = false;
  for (Active* a : active) {
    pr_ctx* c = a->c;
    switch (a->phase) {
      case kUpd1:
        if (hipEventQuery(a->ev_host) == hipSuccess) {
          a->rc = update_mid(c);
          (void)hipEventRecord(a->ev_host, c->stream);
          a->phase = a->rc ? kDrain : kUpd2;
          moved = true;
        }
        break;
      case kUpd2:
        if (hipEventQuery(a->ev_host) == hipSuccess) {
          a->rc = update_end(c);
          if (!a->rc) a->rc = chain(c, a->k);
          moved = true;
          a->k += 1;
          bool cancel;
          {
            std::lock_guard<std::mutex> lk(mu);
            cancel = cancel_req.count(a->req.ticket) > 0;
          }
          if (a->rc || cancel) {
            a->cancelled = cancel;
            (void)hipEventRecord(a->ev_host, c->stream);
            a->phase = kDrain;
          } else if (a->k < a->K) {
            (void)hipEventRecord(a->ev_ready, c->stream);
            a->phase = kSweep;
            a->step = 0;
            a->i0 = c->o.skip_converged ? a->k : 0;
            a->ns = c->P - a->i0;
            a->joined = false;
          } else {
            finish(a);
          }
        }
        break;
      case kFinish:
      case kDrain:
        if (hipEventQuery(a->ev_host) == hipSuccess) {
          a->phase = kDone;
          moved = true;
        }
        break;
      default:
        break;
    }
  }
  // Retire finished solves.
  std::vector<Active*> keep;
  for (Active* a : active) {
    if (a->phase != kDone) {
      keep.push_back(a);
      continue;
    }
    const double t = now_s();
    {
      std::lock_guard<std::mutex> lk(mu);
      const bool cancel = a->cancelled || cancel_req.count(a->req.ticket);
      cancel_req.erase(a->req.ticket);
      if (!cancel) {
        Result r;
        r.rc = a->rc;
        if (!r.rc && a->c->h_ism[2]) r.rc = PR_EDIVERGED;
        if (!r.rc) r.uk.assign(a->h_buf, a->h_buf + a->c->d);
        if (r.rc) err = a->c->err;
        r.latency = t - a->req.t_submit;
        done[a->req.ticket] = std::move(r);
      }
      live.erase(a->req.ticket);
      cv_done.notify_all();
    }
    release(a, a->rc == PR_OK);
    delete a;
  }
  active.swap(keep);
  return moved;
}

// One fused RK-3 step for every solve in its sweep phase.
bool pr_server::sweep_tick() {
  std::vector<Active*> sw;
  for (Active* a : active)
    if (a->phase == kSweep) sw.push_back(a);
  if (sw.empty()) return false;
  for (int sgn : {1, -1}) {
    std::vector<Active*> grp;
    for (Active* a : sw)
      if (a->c->sgn == sgn) grp.push_back(a);
    for (size_t g0 = 0; g0 < grp.size(); g0 += kMaxFineJobs) {
      const size_t g1 = std::min(grp.size(), g0 + kMaxFineJobs);
      FineLaunch L;
      std::memset(&L, 0, sizeof L);
      L.zc = kServerZC;
      int blocks = 0;
      for (size_t q = g0; q < g1; ++q) {
        Active* a = grp[q];
        pr_ctx* c = a->c;
        if (!a->joined) {
          (void)hipStreamWaitEvent(sweep_stream, a->ev_ready, 0);
          a->joined = true;
        }
        const int64_t ld = c->ld;
        const bool to_out = ((c->n_f - 1 - a->step) % 2) == 0;
        const double* src = a->step == 0 ? c->Q + (int64_t)a->i0 * ld : a->src;
        double* dst = to_out ? c->Qt + (int64_t)(a->i0 + 1) * ld : c->Wk;
        FineJob& j = L.job[L.njobs++];
        j.in = src;
        j.out = dst;
        j.in_stride = ld;
        j.out_stride = ld;
        j.nx = c->g.nx;
        j.nz = c->g.nz;
        j.nslices = a->ns;
        j.xtiles = (c->g.nx + fine_tile_cols(kServerNT, c->g.nx) - 1) /
                   fine_tile_cols(kServerNT, c->g.nx);
        j.ztiles = (c->g.nz + kServerZC - 1) / kServerZC;
        j.block_begin = blocks;
        j.c = c->fc;
        blocks += a->ns * j.xtiles * j.ztiles;
        a->src = dst;
      }
      L.nblocks = blocks;
      (void)launch_fine_step(L, kServerNT, sgn, sweep_stream);
      for (size_t q = g0; q < g1; ++q) {
        Active* a = grp[q];
        pr_ctx* c = a->c;
        a->step += 1;
        if (a->step == c->n_f) {
          (void)hipEventRecord(a->ev_sweep, sweep_stream);
          (void)hipStreamWaitEvent(c->stream, a->ev_sweep, 0);
          a->rc = update_begin(c, c->Q + (int64_t)a->k * c->ld,
                               c->Qt + (int64_t)(a->k + 1) * c->ld,
                               c->GQ + (int64_t)a->k * c->ld, c->P - a->k);
          (void)hipEventRecord(a->ev_host, c->stream);
          a->phase = a->rc ? kDrain : kUpd1;
        }
      }
    }
  }
  return true;
}

void pr_server::run() {
  (void)hipSetDevice(device);
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu);
      if (active.empty() && queue.empty()) {
        if (stop) break;
        cv.wait_for(lk, std::chrono::milliseconds(50));
        continue;
      }
    }
    bool did = admit();
    did |= sweep_tick();
    did |= progress();
    if (!did) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

// ----------------------------------------------------------------- C ABI

extern "C" int pr_server_create(int device, size_t hbm_budget_bytes,
                                int32_t max_inflight, pr_server** out) {
  if (!out || max_inflight < 1 || max_inflight > 1024) return PR_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return PR_EDEVICE;
  }
  pr_server* s = new pr_server();
  s->device = device;
  s->max_inflight = max_inflight;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return PR_EDEVICE;
  }
  s->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  if (hipStreamCreate(&s->sweep_stream) != hipSuccess) {
    delete s;
    return PR_EDEVICE;
  }
  s->th = std::thread([s] { s->run(); });
  *out = s;
  return PR_OK;
}

extern "C" int pr_submit_ex(pr_server* s, const pr_grid* g, double c_s,
                            double U, double dt_f, double dt_g, int32_t P,
                            int32_t K, const pr_opts* o, const double* u0,
                            uint64_t* ticket) {
  if (!s || !g || !u0 || !ticket) return PR_EINVAL;
  pr_opts def;
  pr_opts_default(&def);
  if (!o) o = &def;
  if (K < 0) return set_serr(s, PR_EINVAL, "K must be >= 0");
  if (o->windows != 1)
    return set_serr(s, PR_EINVAL, "the server solves one window (windows = 1)");
  if (o->scheme != PR_SCHEME_SPLIT)
    return set_serr(s, PR_EINVAL, "the server runs the split scheme only");
  if (o->stop_tol != 0.0)
    return set_serr(s, PR_EINVAL, "the server runs a fixed K (stop_tol = 0)");
  if (o->V != 0.0 || o->gamma != 0.0 || o->fine_acoustic_order != 4 ||
      o->coarse_order != 1)
    return set_serr(s, PR_EINVAL, "the server advects along x with "
                    "fourth-order fine acoustics and a first-order coarse "
                    "slow tendency (V = gamma = 0, fine_acoustic_order = 4, "
                    "coarse_order = 1)");
  int nf, ng;
  std::string msg;
  int rc = pr_validate(g, c_s, U, dt_f, dt_g, P, o, &nf, &ng, &msg);
  if (rc) return set_serr(s, rc, msg);
  double rf, rg;
  pr_check_stability_impl(g, c_s, U, dt_f, dt_g, o, &rf, &rg);
  if (rf > 1.0 + 1e-12 || rg > 1.0 + 1e-12)
    return set_serr(s, PR_EUNSTABLE, "unstable propagator");
  Request r;
  r.g = *g;
  r.c_s = c_s;
  r.U = U;
  r.dt_f = dt_f;
  r.dt_g = dt_g;
  r.P = P;
  r.K = K;
  r.o = *o;
  r.o.form = PR_FORM_BATCHED;
  const int64_t d = 3LL * g->nx * g->nz;
  r.u0.assign(u0, u0 + d);
  size_t fp = 0;
  pr_footprint(g, P, std::min(K, P), &fp);
  r.bytes = fp + (size_t)d * 8;
  r.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->queue.size() >= kQueueCap) {
      s->err = "queue full";
      return PR_EBUSY;
    }
    r.ticket = s->next_ticket++;
    *ticket = r.ticket;
    s->live.insert(r.ticket);
    s->queue.push_back(std::move(r));
  }
  s->cv.notify_all();
  return PR_OK;
}

extern "C" int pr_submit(pr_server* s, const pr_grid* g, double c_s, double U,
                         double dt_f, double dt_g, int32_t P, int32_t K,
                         const double* u0, uint64_t* ticket) {
  return pr_submit_ex(s, g, c_s, U, dt_f, dt_g, P, K, nullptr, u0, ticket);
}

extern "C" int pr_poll(pr_server* s, uint64_t ticket, double* U_K,
                       double* latency_s) {
  if (!s) return PR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it == s->done.end()) return s->live.count(ticket) ? PR_EAGAIN : PR_ENOTFOUND;
  const int rc = it->second.rc;
  if (rc == PR_OK && U_K)
    std::memcpy(U_K, it->second.uk.data(), it->second.uk.size() * 8);
  if (latency_s) *latency_s = it->second.latency;
  s->done.erase(it);
  return rc;
}

extern "C" int pr_cancel(pr_server* s, uint64_t ticket) {
  if (!s) return PR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->done.erase(ticket)) return PR_OK;
  if (!s->live.count(ticket)) return PR_ENOTFOUND;
  s->cancel_req.insert(ticket);
  return PR_OK;
}

extern "C" int pr_server_drain(pr_server* s) {
  if (!s) return PR_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return s->live.empty(); });
  return PR_OK;
}

extern "C" void pr_server_destroy(pr_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& r : s->queue) s->cancel_req.insert(r.ticket);
    for (Active* a : s->active) s->cancel_req.insert(a->req.ticket);
    s->stop = true;
  }
  s->cv.notify_all();
  // Queued requests are dropped by admit(); running ones stop at the end of
  // their current iteration.
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->live.empty(); });
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(s->device);
  while (!s->pool_lru.empty()) s->evict_pool_one();
  if (s->sweep_stream) (void)hipStreamDestroy(s->sweep_stream);
  delete s;
}

extern "C" const char* pr_server_last_error(const pr_server* s) {
  return s ? s->err.c_str() : "";
}
