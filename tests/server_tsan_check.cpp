// Host check of the serving loop's threading (server.cpp) under
// ThreadSanitizer, with no GPU: the HIP runtime calls the server makes and
// the library entry points it drives are replaced by host stand-ins.  Device
// memory is host memory, a copy is a memcpy, a stream is a token, and a
// "periodogram" writes t[0] + k at frequency k (each request's t[0] is its
// own id), so every result can be traced to its request.  Several threads
// submit, poll, wait and take while three lanes run batches and single
// series, alongside a warm-up, stats readers, a shutdown with requests in
// flight, and injected lane failures (MILS_SERVER_FAIL_AFTER).  Prints
// "server ok"; any race, wrong result or lost ticket fails.
//
// Build: g++ -O1 -g -std=c++17 -fsanitize=thread -I/opt/rocm/include
//        -D__HIP_PLATFORM_AMD__ server_tsan_check.cpp server.cpp
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../include/mils.h"
#include "../paper_2409_08090_amd/csrc/api_internal.h"

// ---- host stand-ins for the HIP runtime -----------------------------------
extern "C" {
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  *v = 256;
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = reinterpret_cast<hipStream_t>(new int(0));
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<int*>(s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
}

// ---- host stand-ins for the library entry points --------------------------
struct mils_context {
  int64_t plans = 0;
};
static std::atomic<int64_t> g_calls{0};

static void tiny_pause(int64_t salt) {
  if (salt % 7 == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
}

extern "C" {
int mils_context_create(int, uint64_t, mils_context** out) {
  *out = new mils_context;
  return MILS_OK;
}
int mils_context_destroy(mils_context* ctx) {
  delete ctx;
  return MILS_OK;
}
int mils_context_set_graphs(mils_context*, int) { return MILS_OK; }
const char* mils_last_error(const mils_context*) { return ""; }
int mils_periodogram(mils_context* ctx, const double* t, const double*, const double*, int64_t nd,
                     const mils_params* p, double* power, void*) {
  if (nd < 1 || p->nf < 1) return MILS_ERR_INVALID_ARG;
  ++ctx->plans;
  for (int64_t k = 0; k < p->nf; ++k) power[k] = t[0] + (double)k;
  tiny_pause(++g_calls);
  return MILS_OK;
}
}

int mils_batch_run(mils_context* ctx, int64_t m, const int64_t* nd_off, const double* t,
                   const double*, const double*, const int64_t* nf_off, const double*,
                   const double*, const mils_params*, double* power, int32_t* st, void*, bool) {
  ++ctx->plans;
  for (int64_t c = 0; c < m; ++c) {
    for (int64_t k = 0; k < nf_off[c + 1] - nf_off[c]; ++k)
      power[nf_off[c] + k] = t[nd_off[c]] + (double)k;
    st[c] = MILS_OK;
  }
  tiny_pause(++g_calls);
  return MILS_OK;
}
void mils_context_plan_counters(const mils_context* ctx, int64_t* built, double* seconds) {
  *built = ctx->plans;
  *seconds = 1e-6 * (double)ctx->plans;
}
int mils_check_params(const mils_params* p, int64_t nd) {
  return (nd >= 1 && p->nf >= 1 && p->df > 0.0) ? MILS_OK : MILS_ERR_INVALID_ARG;
}

// ---- the check -------------------------------------------------------------
static std::atomic<int> g_fail{0};
#define FAIL(...)                  \
  do {                             \
    std::printf(__VA_ARGS__);      \
    std::printf("\n");             \
    g_fail.store(1);               \
  } while (0)

static mils_params params_for(int64_t nf, bool fp32) {
  mils_params p;
  std::memset(&p, 0, sizeof(p));
  p.f0 = 0.01;
  p.df = 0.01;
  p.nf = nf;
  p.eps = fp32 ? 1e-5 : 1e-9;
  p.precision = fp32 ? MILS_FP32 : MILS_FP64;
  p.flags = MILS_CENTER_DATA | MILS_FIT_MEAN;
  return p;
}

// Submits n requests (ids id0, id0 + 1, ...), then waits for and takes each,
// checking power[k] = id + k.  cancel_ok: the server may be destroyed
// meanwhile (then wait/take may fail, and nothing is checked).
static void client(mils_server* srv, int id0, int n, unsigned seed, bool cancel_ok,
                   std::atomic<int>* done) {
  std::mt19937 rng(seed);
  std::vector<uint64_t> tickets;
  std::vector<int64_t> nfs;
  for (int i = 0; i < n; ++i) {
    const int64_t nd = 20 + (int64_t)(rng() % 400);
    // mostly batched sizes, a few above the batch limit (single-series path)
    const int64_t nf = (rng() % 16 == 0) ? 40000 + (int64_t)(rng() % 30000) : 50 + (int64_t)(rng() % 4000);
    std::vector<double> t(nd), y(nd, 1.0), dy(nd, 0.5);
    for (int64_t j = 0; j < nd; ++j) t[j] = (double)(id0 + i) + 1e-3 * (double)j;
    mils_request rq;
    rq.t = t.data();
    rq.y = y.data();
    rq.dy = dy.data();
    rq.nd = nd;
    rq.params = params_for(nf, rng() % 2 == 0);
    uint64_t tk = 0;
    int rc;
    while ((rc = mils_server_submit(srv, &rq, &tk)) == MILS_ERR_BUSY)
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    if (rc != MILS_OK) {
      if (!cancel_ok) FAIL("submit failed: %d", rc);
      return;
    }
    tickets.push_back(tk);
    nfs.push_back(nf);
  }
  for (size_t i = 0; i < tickets.size(); ++i) {
    int32_t state = -1;
    if (mils_server_poll(srv, tickets[i], &state) != MILS_OK && !cancel_ok) FAIL("poll");
    const int rc = mils_server_wait(srv, tickets[i], 20 * 1000 * 1000);
    if (rc != MILS_OK) {
      if (!cancel_ok) FAIL("wait %d", rc);
      continue;
    }
    std::vector<double> pw((size_t)nfs[i]);
    mils_request_stats st;
    const int s = mils_server_take(srv, tickets[i], pw.data(), &st);
    if (cancel_ok) continue;
    if (s != MILS_OK) {
      FAIL("take %d", s);
      continue;
    }
    const double id = (double)(id0 + (int)i);
    for (int64_t k = 0; k < nfs[i]; ++k)
      if (pw[(size_t)k] != id + (double)k) {
        FAIL("request %d: power[%lld] = %g, expected %g", id0 + (int)i, (long long)k, pw[(size_t)k],
             id + (double)k);
        break;
      }
  }
  done->fetch_add(1);
}

static void stats_reader(mils_server* srv, std::atomic<bool>* stop) {
  while (!stop->load()) {
    mils_server_counters c;
    mils_server_stats(srv, &c);
    (void)mils_server_last_error(srv);
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

int main() {
  mils_server_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  cfg.lanes = 3;
  cfg.max_batch = 64;
  cfg.queue_capacity = 256;
  cfg.tick_us = 100;
  cfg.hbm_budget_bytes = (uint64_t)64 << 20;

  // phase 1: clients, a warm-up and stats readers together; every result checked
  {
    mils_server* srv = nullptr;
    if (mils_server_create(0, &cfg, &srv) != MILS_OK) {
      std::printf("create failed\n");
      return 1;
    }
    std::atomic<bool> stop{false};
    std::atomic<int> done{0};
    std::thread sr(stats_reader, srv, &stop);
    std::vector<std::thread> cl;
    for (int c = 0; c < 4; ++c) cl.emplace_back(client, srv, 100000 * (c + 1), 150, 11u + c, false, &done);
    mils_params wp = params_for(1, false);
    if (mils_server_warm(srv, &wp, 3000) != MILS_OK) FAIL("warm");
    for (auto& th : cl) th.join();
    stop.store(true);
    sr.join();
    mils_server_counters c;
    mils_server_stats(srv, &c);
    if (c.completed != 600 || c.failed != 0) FAIL("counters: completed %llu failed %llu",
                                                  (unsigned long long)c.completed,
                                                  (unsigned long long)c.failed);
    mils_server_destroy(srv);
  }
  // phase 2: shutdown with requests in flight (submitted, never waited for)
  {
    mils_server* srv = nullptr;
    if (mils_server_create(0, &cfg, &srv) != MILS_OK) return 1;
    std::vector<std::thread> sub;
    for (int c = 0; c < 2; ++c)
      sub.emplace_back([srv, c] {
        std::vector<double> t(200), y(200, 1.0), dy(200, 0.5);
        for (int i = 0; i < 100; ++i) {
          for (int j = 0; j < 200; ++j) t[j] = (double)(700000 * (c + 1) + i) + 1e-3 * j;
          mils_request rq;
          rq.t = t.data();
          rq.y = y.data();
          rq.dy = dy.data();
          rq.nd = 200;
          rq.params = params_for(2000 + 17 * i, i % 2 == 0);
          uint64_t tk;
          int rc;
          while ((rc = mils_server_submit(srv, &rq, &tk)) == MILS_ERR_BUSY)
            std::this_thread::sleep_for(std::chrono::microseconds(50));
          if (rc != MILS_OK) FAIL("submit before shutdown: %d", rc);
        }
      });
    for (auto& th : sub) th.join();
    mils_server_destroy(srv);  // cancels what is still queued, waits for running batches
  }
  // phase 3: lanes that fail after a few batches; pending requests must end
  {
    setenv("MILS_SERVER_FAIL_AFTER", "3", 1);
    mils_server* srv = nullptr;
    if (mils_server_create(0, &cfg, &srv) != MILS_OK) return 1;
    unsetenv("MILS_SERVER_FAIL_AFTER");
    std::atomic<int> done{0};
    std::vector<std::thread> cl;
    for (int c = 0; c < 3; ++c) cl.emplace_back(client, srv, 900000 * (c + 1), 80, 51u + c, true, &done);
    for (auto& th : cl) th.join();
    mils_server_counters c;
    mils_server_stats(srv, &c);
    if (c.dead_lanes != 3) FAIL("dead lanes %llu", (unsigned long long)c.dead_lanes);
    mils_server_destroy(srv);
  }
  if (g_fail.load()) return 1;
  std::printf("server ok\n");
  return 0;
}
