// server.cpp -- the serving loop of libmils (mils_server_* in include/mils.h).
//
// Requests arrive from any host thread with host arrays, which submit copies.
// Each lane owns a HIP stream, a libmils context (workspace, plans, batch
// state) and pinned staging buffers, and runs in its own thread: when it is
// free it takes every compatible request that has arrived (same precision,
// tolerance, normalisation and flags), as far as the HBM budget allows, packs
// them into one batch, runs the batched launches on its stream and copies the
// results back.  While one lane's batch is on the device, the next
// arrivals are packed by another lane, so batches overlap on the GPU.
// Requests with many frequencies run through the single-series path instead.
//
// Plan classes: a request is computed on its frequency grid extended to the
// next class size (nf rounded up to ceil(64 * 2^(j/16)), at most 4.5% more
// frequencies), and the first nf values are returned.  Requests of fresh
// sizes then share the plans (kernel width, grid, FFT factorisation and their
// device tables) of a bounded set of classes, which mils_server_warm builds
// ahead of traffic, instead of building a plan per size on arrival.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mils.h"
#include "api_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// Above this many frequencies a request uses the single-series path: its
// own grids fill the GPU, and batching it would only hold back the small
// requests packed with it.
constexpr int64_t kBatchMaxNf = 200000;

// Smallest class size >= nf: ceil(64 * 2^(j/16)) for j >= 0 (64 for nf <= 64),
// capped at the largest frequency count a call accepts.
int64_t nf_class(int64_t nf) {
  constexpr int64_t kMaxNf = (int64_t)1 << 28;
  if (nf <= 64) return 64;
  if (nf >= kMaxNf) return nf;
  int j = (int)std::floor(16.0 * std::log2((double)nf / 64.0));
  if (j < 0) j = 0;
  for (;; ++j) {
    const int64_t v = (int64_t)std::ceil(64.0 * std::exp2((double)j / 16.0));
    if (v >= nf) return std::min(v, kMaxNf);
  }
}

struct Request {
  std::vector<double> t, y, dy;
  bool has_dy = false;
  mils_params p{};
  int64_t nfc = 0;  // frequencies computed: p.nf rounded up to its plan class
  int64_t nd = 0;
  std::vector<double> power;
  int state = MILS_REQ_PENDING;
  int status = MILS_OK;
  double submit_s = 0, start_s = 0, done_s = 0;
  int batch_size = 0;
};

// Device bytes a request needs while in flight: inputs, output, and three
// grids (plus their second buffers) of ~1.5 nf cells (nf: the class size).
uint64_t request_bytes(const mils_params& p, int64_t nf, int64_t nd) {
  const double c = p.precision == MILS_FP32 ? 8.0 : 16.0;
  return (uint64_t)(24.0 * nd + 8.0 * nf + 2.0 * 3.0 * 1.5 * (double)nf * c) + 4096;
}

struct Lane {
  mils_context* ctx = nullptr;
  hipStream_t stream = nullptr;
  double* h_in = nullptr;
  size_t h_in_cap = 0;
  double* h_out = nullptr;
  size_t h_out_cap = 0;
  double* d_in = nullptr;
  size_t d_in_cap = 0;
  double* d_out = nullptr;
  size_t d_out_cap = 0;
  bool dead = false;
  bool injected = false;  // stopped by the fault-injection switch
  // a plan warm-up posted by mils_server_warm (guarded by the server's mutex)
  bool warm_req = false;
  mils_params warm_p{};
  int64_t warm_nf_max = 0;
  int warm_rc = MILS_OK;
  int64_t plans_seen = 0;  // plans built by this lane's context, last counted
  double plan_s_seen = 0.0;
  int64_t runs = 0;       // batches run
  std::thread th;
};

bool grow_pinned(double** p, size_t* cap, size_t need) {
  if (need <= *cap) return true;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  size_t c = std::max(need, (size_t)(1 << 20));
  if (hipHostMalloc(reinterpret_cast<void**>(p), c * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  *cap = c;
  return true;
}

bool grow_device(double** p, size_t* cap, size_t need) {
  if (need <= *cap) return true;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  size_t c = std::max(need + need / 2, (size_t)(1 << 20));
  if (hipMalloc(reinterpret_cast<void**>(p), c * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  *cap = c;
  return true;
}

}  // namespace

struct mils_server {
  int device = 0;
  mils_server_config cfg{};
  int num_cu = 256;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<uint64_t> pending;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  uint64_t inflight = 0, peak = 0;
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, batched_reqs = 0;
  uint64_t failed = 0, dead_lanes = 0;
  std::string lane_error;  // message of the first device error that ended a lane
  // Fault injection for tests of the lane-failure handling: with
  // MILS_SERVER_FAIL_AFTER=N in the environment when the server is created,
  // each lane reports a device error once it has run N batches (the batch
  // that trips it is reported failed; the device is not touched).  -1: off.
  int64_t fail_after = -1;
  std::vector<double> lat_ms;
  double first_submit = -1.0, last_done = 0.0, sums_done = 0.0;
  uint64_t plans_built = 0;
  double plan_build_s = 0.0;
  std::vector<std::unique_ptr<Lane>> lanes;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void lane_loop(Lane* L);
  void run_batch(Lane* L, std::vector<Request*>& batch);
  void run_single(Lane* L, Request* r);
  int run_warm(Lane* L, const mils_params& p, int64_t nf_max);
  void count_plans(Lane* L);
  void lane_died(Lane* L);
};

namespace {

bool compatible(const Request& a, const Request& b) {
  return a.p.precision == b.p.precision && a.p.eps == b.p.eps &&
         a.p.normalization == b.p.normalization && a.p.flags == b.p.flags &&
         a.has_dy == b.has_dy && (a.nfc > kBatchMaxNf) == (b.nfc > kBatchMaxNf);
}

}  // namespace

void mils_server::run_single(Lane* L, Request* r) {
  const size_t nd = (size_t)r->nd, nf = (size_t)r->p.nf, nfc = (size_t)r->nfc;
  int st = MILS_OK;
  if (!grow_pinned(&L->h_in, &L->h_in_cap, 3 * nd) || !grow_pinned(&L->h_out, &L->h_out_cap, nf) ||
      !grow_device(&L->d_in, &L->d_in_cap, 3 * nd) || !grow_device(&L->d_out, &L->d_out_cap, nfc)) {
    st = MILS_ERR_OOM;
  } else {
    std::memcpy(L->h_in, r->t.data(), nd * sizeof(double));
    std::memcpy(L->h_in + nd, r->y.data(), nd * sizeof(double));
    if (r->has_dy) std::memcpy(L->h_in + 2 * nd, r->dy.data(), nd * sizeof(double));
    hipError_t he = hipMemcpyAsync(L->d_in, L->h_in, 3 * nd * sizeof(double),
                                   hipMemcpyHostToDevice, L->stream);
    if (he != hipSuccess) {
      st = MILS_ERR_DEVICE;
    } else {
      mils_params pc = r->p;
      pc.nf = r->nfc;
      st = mils_periodogram(L->ctx, L->d_in, L->d_in + nd, r->has_dy ? L->d_in + 2 * nd : nullptr,
                            r->nd, &pc, L->d_out, L->stream);
      if (st == MILS_OK || st == MILS_ERR_DEGENERATE || st == MILS_ERR_INVALID_ARG) {
        he = hipMemcpyAsync(L->h_out, L->d_out, nf * sizeof(double), hipMemcpyDeviceToHost,
                            L->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(L->stream);
        if (he != hipSuccess) st = MILS_ERR_DEVICE;
      }
    }
  }
  if (st == MILS_OK) r->power.assign(L->h_out, L->h_out + nf);
  r->status = st;
  if (st == MILS_ERR_DEVICE) L->dead = true;
}

void mils_server::run_batch(Lane* L, std::vector<Request*>& batch) {
  const size_t m = batch.size();
  std::vector<int64_t> nd_off(m + 1, 0), nf_off(m + 1, 0);
  std::vector<double> f0(m), df(m);
  for (size_t i = 0; i < m; ++i) {
    nd_off[i + 1] = nd_off[i] + batch[i]->nd;
    nf_off[i + 1] = nf_off[i] + batch[i]->nfc;
    f0[i] = batch[i]->p.f0;
    df[i] = batch[i]->p.df;
  }
  const size_t N = (size_t)nd_off[m], F = (size_t)nf_off[m];
  const bool has_dy = batch[0]->has_dy;
  std::vector<int32_t> stv(m, MILS_OK);
  int rc = MILS_OK;
  if (!grow_pinned(&L->h_in, &L->h_in_cap, 3 * N) || !grow_pinned(&L->h_out, &L->h_out_cap, F) ||
      !grow_device(&L->d_in, &L->d_in_cap, 3 * N) || !grow_device(&L->d_out, &L->d_out_cap, F)) {
    rc = MILS_ERR_OOM;
  } else {
    for (size_t i = 0; i < m; ++i) {
      const size_t o = (size_t)nd_off[i], n = (size_t)batch[i]->nd;
      std::memcpy(L->h_in + o, batch[i]->t.data(), n * sizeof(double));
      std::memcpy(L->h_in + N + o, batch[i]->y.data(), n * sizeof(double));
      if (has_dy) std::memcpy(L->h_in + 2 * N + o, batch[i]->dy.data(), n * sizeof(double));
    }
    hipError_t he = hipMemcpyAsync(L->d_in, L->h_in, 3 * N * sizeof(double),
                                   hipMemcpyHostToDevice, L->stream);
    if (he != hipSuccess) {
      rc = MILS_ERR_DEVICE;
    } else {
      mils_params common = batch[0]->p;
      rc = mils_batch_run(L->ctx, (int64_t)m, nd_off.data(), L->d_in, L->d_in + N,
                          has_dy ? L->d_in + 2 * N : nullptr, nf_off.data(), f0.data(), df.data(),
                          &common, L->d_out, stv.data(), L->stream, false);
      if (rc == MILS_OK || rc == MILS_ERR_INVALID_ARG || rc == MILS_ERR_DEGENERATE) {
        he = hipMemcpyAsync(L->h_out, L->d_out, F * sizeof(double), hipMemcpyDeviceToHost,
                            L->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(L->stream);
        if (he != hipSuccess) rc = MILS_ERR_DEVICE;
        else rc = MILS_OK;
      }
    }
  }
  for (size_t i = 0; i < m; ++i) {
    Request* r = batch[i];
    if (rc != MILS_OK) {
      r->status = rc;
      continue;
    }
    r->status = stv[i];
    if (stv[i] == MILS_OK)
      r->power.assign(L->h_out + nf_off[i], L->h_out + nf_off[i] + r->p.nf);
  }
  if (rc == MILS_ERR_DEVICE) L->dead = true;
}

// Adds the plans this lane's context built since the last count to the
// server's counters.  Called with mu held (only the lane's thread uses its
// context, and it calls this between its runs).
void mils_server::count_plans(Lane* L) {
  int64_t built = 0;
  double sec = 0.0;
  mils_context_plan_counters(L->ctx, &built, &sec);
  plans_built += (uint64_t)(built - L->plans_seen);
  plan_build_s += sec - L->plan_s_seen;
  L->plans_seen = built;
  L->plan_s_seen = sec;
}

// Runs every plan class up to nf_max once on this lane (parameters p apart
// from the grid): a one-series batch for the batched classes and a
// single-series call for the larger ones, on a short synthetic series (the
// single-series classes with nf / 12 points, so that the workspace also
// grows ahead of traffic).  Returns the first error.
int mils_server::run_warm(Lane* L, const mils_params& p, int64_t nf_max) {
  const int64_t top = nf_class(nf_max);
  std::vector<double> h;
  for (int64_t v = nf_class(1);; v = nf_class(v + 1)) {
    const bool single = v > kBatchMaxNf;
    const int64_t nd = single ? std::max<int64_t>(64, v / 12) : 64;
    // sorted times on [0, 20) with irregular spacing, a sinusoid, unit errors
    h.resize(3 * (size_t)nd);
    for (int64_t j = 0; j < nd; ++j) {
      const double u = ((double)j + 0.5 + 0.4 * std::sin(7.1 * (double)j)) / (double)nd;
      h[j] = 20.0 * u;
      h[nd + j] = std::sin(2.3 * h[j]) + 0.1 * std::cos(17.0 * (double)j);
      h[2 * nd + j] = 1.0;
    }
    if (!grow_device(&L->d_in, &L->d_in_cap, 3 * (size_t)nd) ||
        !grow_device(&L->d_out, &L->d_out_cap, (size_t)v))
      return MILS_ERR_OOM;
    if (hipMemcpyAsync(L->d_in, h.data(), 3 * (size_t)nd * sizeof(double), hipMemcpyHostToDevice,
                       L->stream) != hipSuccess)
      return MILS_ERR_DEVICE;
    mils_params q = p;
    q.nf = v;
    q.f0 = q.df = 0.01;
    int rc;
    if (single) {
      rc = mils_periodogram(L->ctx, L->d_in, L->d_in + nd, L->d_in + 2 * nd, nd, &q, L->d_out,
                            L->stream);
    } else {
      const int64_t nd_off[2] = {0, nd}, nf_off[2] = {0, v};
      int32_t st = MILS_OK;
      rc = mils_batch_run(L->ctx, 1, nd_off, L->d_in, L->d_in + nd, L->d_in + 2 * nd, nf_off,
                          &q.f0, &q.df, &q, L->d_out, &st, L->stream, false);
    }
    if (rc != MILS_OK && rc != MILS_ERR_DEGENERATE) return rc;
    if (hipStreamSynchronize(L->stream) != hipSuccess) return MILS_ERR_DEVICE;
    if (v >= top) break;
  }
  return MILS_OK;
}

// A lane whose context took a device error stops; once no lane is left, the
// pending requests end with MILS_ERR_DEVICE instead of waiting forever.
// Called with mu held.
void mils_server::lane_died(Lane* L) {
  ++dead_lanes;
  if (lane_error.empty()) {
    const char* m = mils_last_error(L->ctx);
    lane_error = L->injected ? "injected lane failure (MILS_SERVER_FAIL_AFTER)"
                 : (m && m[0]) ? m
                               : "device error";
  }
  if (dead_lanes < lanes.size()) return;
  const double t = now();
  for (uint64_t tk : pending) {
    Request* r = reqs[tk].get();
    r->state = MILS_REQ_DONE;
    r->status = MILS_ERR_DEVICE;
    r->start_s = r->done_s = t;
    ++completed;
    ++failed;
  }
  pending.clear();
  cv_done.notify_all();
}

void mils_server::lane_loop(Lane* L) {
  (void)hipSetDevice(device);
  const auto tick = std::chrono::microseconds(cfg.tick_us);
  std::unique_lock<std::mutex> lk(mu);
  while (!stop && !L->dead) {
    cv_work.wait(lk, [&] { return stop || !pending.empty() || L->warm_req; });
    if (stop) break;
    if (L->warm_req) {
      const mils_params wp = L->warm_p;
      const int64_t wmax = L->warm_nf_max;
      lk.unlock();
      const int rc = run_warm(L, wp, wmax);
      lk.lock();
      L->warm_rc = rc;
      L->warm_req = false;
      if (rc == MILS_ERR_DEVICE) {
        L->dead = true;
        lane_died(L);
      }
      count_plans(L);
      cv_done.notify_all();
      continue;
    }
    // let a small batch grow for up to one tick
    if ((int)pending.size() < cfg.max_batch) {
      const Request& head = *reqs[pending.front()];
      const double waited = now() - head.submit_s;
      if (waited * 1e6 < cfg.tick_us) {
        cv_work.wait_for(lk, tick, [&] { return stop || (int)pending.size() >= cfg.max_batch; });
        if (stop) break;
        if (pending.empty()) continue;
      }
    }
    // admit compatible requests in arrival order while the budget allows
    Request* first = reqs[pending.front()].get();
    const bool single = first->nfc > kBatchMaxNf;
    std::vector<uint64_t> take;
    std::vector<Request*> batch;
    uint64_t need = 0, data_bytes = 0, slot_max = 0;
    for (uint64_t tk : pending) {
      Request* r = reqs[tk].get();
      if (!compatible(*first, *r)) continue;
      const uint64_t rb = request_bytes(r->p, r->nfc, r->nd);
      const uint64_t d2 = data_bytes + (uint64_t)(24 * r->nd + 8 * r->nfc);
      const uint64_t s2 = std::max(slot_max, rb);
      const uint64_t n2 = d2 + std::min<uint64_t>(batch.size() + 1, 2 * (uint64_t)num_cu) * s2;
      if (inflight + n2 > cfg.hbm_budget_bytes) break;
      take.push_back(tk);
      batch.push_back(r);
      need = n2;
      data_bytes = d2;
      slot_max = s2;
      if (single || (int)batch.size() >= cfg.max_batch) break;
    }
    if (batch.empty()) {
      // nothing fits until something in flight completes
      cv_work.wait_for(lk, tick);
      continue;
    }
    std::deque<uint64_t> rest;
    size_t ti = 0;
    for (uint64_t tk : pending) {
      if (ti < take.size() && take[ti] == tk) {
        ++ti;
        continue;
      }
      rest.push_back(tk);
    }
    pending.swap(rest);
    const double t_start = now();
    for (Request* r : batch) {
      r->state = MILS_REQ_RUNNING;
      r->start_s = t_start;
      r->batch_size = (int)batch.size();
    }
    inflight += need;
    peak = std::max(peak, inflight);
    lk.unlock();
    if (single) run_single(L, batch[0]);
    else run_batch(L, batch);
    if (fail_after >= 0 && ++L->runs > fail_after) {
      for (Request* r : batch) r->status = MILS_ERR_DEVICE;
      L->dead = L->injected = true;
    }
    lk.lock();
    const double t_done = now();
    inflight -= need;
    ++batches;
    batched_reqs += batch.size();
    for (Request* r : batch) {
      r->state = MILS_REQ_DONE;
      r->done_s = t_done;
      ++completed;
      lat_ms.push_back((t_done - r->submit_s) * 1e3);
      if (r->status == MILS_OK) sums_done += (double)r->nd * (double)r->p.nf;
      else ++failed;
    }
    count_plans(L);
    if (L->dead) lane_died(L);
    last_done = t_done;
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" {

int mils_server_create(int device, const mils_server_config* cfg, mils_server** out) {
  if (!out) return MILS_ERR_INVALID_ARG;
  *out = nullptr;
  mils_server_config c{};
  if (cfg) c = *cfg;
  if (c.lanes < 0 || c.lanes > 16 || c.max_batch < 0 || c.queue_capacity < 0 || c.tick_us < 0)
    return MILS_ERR_INVALID_ARG;
  if (device < 0) return MILS_ERR_DEVICE;
  if (!c.hbm_budget_bytes) c.hbm_budget_bytes = 8ull << 30;
  if (!c.lanes) c.lanes = 2;
  if (!c.max_batch) c.max_batch = 4096;
  if (!c.queue_capacity) c.queue_capacity = 65536;
  if (!c.tick_us) c.tick_us = 200;
  std::unique_ptr<mils_server> s(new (std::nothrow) mils_server());
  if (!s) return MILS_ERR_OOM;
  s->device = device;
  s->cfg = c;
  if (const char* e = std::getenv("MILS_SERVER_FAIL_AFTER")) s->fail_after = std::atoll(e);
  s->t0 = Clock::now();
  if (hipSetDevice(device) != hipSuccess) return MILS_ERR_DEVICE;
  (void)hipDeviceGetAttribute(&s->num_cu, hipDeviceAttributeMultiprocessorCount, device);
  for (int i = 0; i < c.lanes; ++i) {
    auto L = std::make_unique<Lane>();
    int rc = mils_context_create(device, 0, &L->ctx);
    // a lane's single-series calls seldom repeat their arguments
    if (rc == MILS_OK) rc = mils_context_set_graphs(L->ctx, 0);
    if (rc == MILS_OK && hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess)
      rc = MILS_ERR_DEVICE;
    if (rc != MILS_OK) {
      if (L->ctx) mils_context_destroy(L->ctx);
      for (auto& M : s->lanes) {
        (void)hipStreamDestroy(M->stream);
        mils_context_destroy(M->ctx);
      }
      return rc;
    }
    s->lanes.push_back(std::move(L));
  }
  for (auto& L : s->lanes) {
    Lane* lp = L.get();
    mils_server* sp = s.get();
    L->th = std::thread([sp, lp] { sp->lane_loop(lp); });
  }
  *out = s.release();
  return MILS_OK;
}

int mils_server_submit(mils_server* srv, const mils_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket || !req->t || !req->y) return MILS_ERR_INVALID_ARG;
  int rc = mils_check_params(&req->params, req->nd);
  if (rc != MILS_OK) return rc;
  if (req->params.flags & MILS_DETERMINISTIC) return MILS_ERR_UNSUPPORTED;
  const int64_t nfc = nf_class(req->params.nf);
  const uint64_t rb = request_bytes(req->params, nfc, req->nd);
  auto r = std::make_unique<Request>();
  const size_t nd = (size_t)req->nd;
  r->t.assign(req->t, req->t + nd);
  r->y.assign(req->y, req->y + nd);
  r->has_dy = req->dy != nullptr;
  if (r->has_dy) r->dy.assign(req->dy, req->dy + nd);
  r->p = req->params;
  r->nfc = nfc;
  r->nd = req->nd;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return MILS_ERR_CANCELLED;
  if (srv->dead_lanes == srv->lanes.size()) return MILS_ERR_DEVICE;
  if (rb + (uint64_t)(24 * req->nd + 8 * nfc) > srv->cfg.hbm_budget_bytes) {
    ++srv->rejected;
    return MILS_ERR_OOM;
  }
  if ((int64_t)srv->pending.size() >= srv->cfg.queue_capacity) {
    ++srv->rejected;
    return MILS_ERR_BUSY;
  }
  r->submit_s = srv->now();
  if (srv->first_submit < 0) srv->first_submit = r->submit_s;
  const uint64_t tk = srv->next_ticket++;
  srv->reqs[tk] = std::move(r);
  srv->pending.push_back(tk);
  ++srv->submitted;
  *ticket = tk;
  srv->cv_work.notify_one();
  return MILS_OK;
}

int mils_server_warm(mils_server* srv, const mils_params* params, int64_t nf_max) {
  if (!srv || !params || nf_max < 1) return MILS_ERR_INVALID_ARG;
  mils_params p = *params;
  p.nf = nf_class(nf_max);
  int rc = mils_check_params(&p, 64);
  if (rc != MILS_OK) return rc;
  if (p.flags & MILS_DETERMINISTIC) return MILS_ERR_UNSUPPORTED;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->stop) return MILS_ERR_CANCELLED;
  for (auto& L : srv->lanes) {
    if (L->dead) continue;
    L->warm_p = p;
    L->warm_nf_max = nf_max;
    L->warm_rc = MILS_OK;
    L->warm_req = true;
  }
  srv->cv_work.notify_all();
  srv->cv_done.wait(lk, [&] {
    for (auto& L : srv->lanes)
      if (L->warm_req && !L->dead && !srv->stop) return false;
    return true;
  });
  rc = MILS_OK;
  int alive = 0;
  for (auto& L : srv->lanes) {
    if (L->dead) continue;
    ++alive;
    if (rc == MILS_OK && L->warm_rc != MILS_OK) rc = L->warm_rc;
  }
  if (rc == MILS_OK && !alive) rc = MILS_ERR_DEVICE;
  return rc;
}

int mils_server_poll(mils_server* srv, uint64_t ticket, int32_t* state) {
  if (!srv || !state) return MILS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return MILS_ERR_INVALID_ARG;
  *state = it->second->state;
  return MILS_OK;
}

int mils_server_wait(mils_server* srv, uint64_t ticket, int64_t timeout_us) {
  if (!srv) return MILS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto done = [&] {
    auto it = srv->reqs.find(ticket);
    return it == srv->reqs.end() || it->second->state == MILS_REQ_DONE;
  };
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, done);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
    return MILS_ERR_TIMEOUT;
  }
  return srv->reqs.count(ticket) ? MILS_OK : MILS_ERR_INVALID_ARG;
}

int mils_server_take(mils_server* srv, uint64_t ticket, double* power, mils_request_stats* st) {
  if (!srv) return MILS_ERR_INVALID_ARG;
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return MILS_ERR_INVALID_ARG;
    if (it->second->state != MILS_REQ_DONE) return MILS_ERR_BUSY;
    r = std::move(it->second);
    srv->reqs.erase(it);
  }
  if (power && r->status == MILS_OK) std::memcpy(power, r->power.data(), r->power.size() * sizeof(double));
  if (st) {
    st->submit_s = r->submit_s;
    st->start_s = r->start_s;
    st->done_s = r->done_s;
    st->status = r->status;
    st->batch_size = r->batch_size;
  }
  return r->status;
}

const char* mils_server_last_error(mils_server* srv) {
  if (!srv) return "";
  std::lock_guard<std::mutex> lk(srv->mu);
  return srv->lane_error.c_str();
}

int mils_server_stats(mils_server* srv, mils_server_counters* out) {
  if (!srv || !out) return MILS_ERR_INVALID_ARG;
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->batches = srv->batches;
    out->inflight_bytes = srv->inflight;
    out->peak_inflight_bytes = srv->peak;
    out->mean_batch = srv->batches ? (double)srv->batched_reqs / (double)srv->batches : 0.0;
    out->failed = srv->failed;
    out->dead_lanes = srv->dead_lanes;
    out->plans_built = srv->plans_built;
    out->plan_build_ms = srv->plan_build_s * 1e3;
    const double span = srv->last_done - srv->first_submit;
    out->sums_per_s = span > 0 ? srv->sums_done / span : 0.0;
    lat = srv->lat_ms;
  }
  out->latency_p50_ms = out->latency_p99_ms = out->latency_max_ms = 0.0;
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto q = [&](double f) {
      size_t i = (size_t)std::floor(f * (double)(lat.size() - 1) + 0.5);
      return lat[std::min(i, lat.size() - 1)];
    };
    out->latency_p50_ms = q(0.50);
    out->latency_p99_ms = q(0.99);
    out->latency_max_ms = lat.back();
  }
  return MILS_OK;
}

int mils_server_destroy(mils_server* srv) {
  if (!srv) return MILS_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& L : srv->lanes)
    if (L->th.joinable()) L->th.join();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->pending.clear();
    srv->reqs.clear();
  }
  srv->cv_done.notify_all();
  (void)hipSetDevice(srv->device);
  for (auto& L : srv->lanes) {
    if (L->stream) (void)hipStreamSynchronize(L->stream);
    if (L->h_in) (void)hipHostFree(L->h_in);
    if (L->h_out) (void)hipHostFree(L->h_out);
    if (L->d_in) (void)hipFree(L->d_in);
    if (L->d_out) (void)hipFree(L->d_out);
    if (L->stream) (void)hipStreamDestroy(L->stream);
    if (L->ctx) mils_context_destroy(L->ctx);
  }
  delete srv;
  return MILS_OK;
}

}  // extern "C"
