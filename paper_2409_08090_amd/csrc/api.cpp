// api.cpp -- the C ABI of libmils (include/mils.h): contexts, argument
// validation, plan cache, workspace and the synchronous / asynchronous
// periodogram and trig-sum calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mils.h"
#include "api_internal.h"
#include "batch.h"
#include "fft2.h"
#include "index_math.h"
#include "kernels.h"
#include "mils_internal.h"
#include "plan.h"

using namespace mils;

namespace {

struct PlanEntry {
  Plan plan;
  void* tw = nullptr;            // twiddles (FP64 or FP32 pairs)
  double* inv_phihat = nullptr;  // K + 1 doubles
  double* inv_phihat2 = nullptr; // two-pass plans: n doubles in last-pass order
  size_t bytes = 0;
};

// (nf, eps, precision, grids + 10 * batch, fixed grid size)
using PlanKey = std::tuple<int64_t, double, int, int, int64_t, int>;

std::mutex g_err_mu;
std::string g_create_err;

// Diagnostics on stderr, by MILS_LOG_LEVEL (read at each context's
// creation): 0 none (default), 1 errors, 2 also plans built, workspace
// growth and tuning decisions.
std::atomic<int> g_log_level{0};

void read_log_level() {
  const char* e = std::getenv("MILS_LOG_LEVEL");
  g_log_level.store(e ? std::atoi(e) : 0);
}

// Batch tuning decisions persisted across processes: with MILS_TUNE_CACHE
// naming a file, a context reads the decisions recorded there for its device
// when it is created, and the autotuner appends each new decision.  One line
// per decision: device key, N_f band, eps, precision, sigma, tile cap.  The
// device key is the architecture name, the CU count and the memory size, so
// that decisions of another GPU model are not reused.
std::string tune_device_key(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "";
  std::string arch(prop.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  return arch + ":" + std::to_string(prop.multiProcessorCount) + ":" +
         std::to_string((unsigned long long)(prop.totalGlobalMem >> 30));
}

void mils_log(int level, const char* fmt, ...) {
  if (g_log_level.load(std::memory_order_relaxed) < level) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[mils] %s\n", buf);
}

void host_dd_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double bb = x - a;
  *e = (a - (x - bb)) + (b - bb);
  *s = x;
}

// f_c = f0 + K df as a double-double (K df is exact as a two-product)
void centre_frequency(double f0, double df, int64_t K, double* fch, double* fcl) {
  const double Kd = (double)K;
  const double prod = Kd * df;
  const double perr = std::fma(Kd, df, -prod);
  double s, e;
  host_dd_sum(f0, prod, &s, &e);
  *fch = s;
  *fcl = e + perr;
}

// output index of the zero frequency: the k whose binary64 frequency
// fl(f0 + fl(k df)) is zero, or -1
int64_t zero_index(double f0, double df, int64_t nf) {
  const double kq = std::nearbyint(-f0 / df);
  int64_t kz = -1;
  for (double kk = kq - 1; kk <= kq + 1; kk += 1.0)
    if (kk >= 0.0 && kk < (double)nf && kk * df == -f0) kz = (int64_t)kk;
  return kz;
}

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// State of the batched path kept between calls: the uploaded descriptors, the
// slot workspace and the captured graph are reused when the next batch has
// the same layout and parameters.
// Per-series workspaces of one chunk of a batch are limited to this (the
// batch runs chunk after chunk when the series need more).
constexpr size_t kBatchWorkspaceCap = (size_t)24 << 30;

struct BatchState {
  uint64_t key = 0;
  bool valid = false;
  char* dev = nullptr;  // descriptors, plans, table pointers, workspaces' layout, items, status
  size_t dev_bytes = 0;
  char* ws = nullptr;   // per-series workspaces (of the largest chunk)
  size_t ws_bytes = 0;
  int64_t ncurves = 0;
  std::vector<mils::BatchLaunch> launches;  // one per chunk, in order
  int* status_dev = nullptr;
  int32_t* status_host = nullptr;  // pinned
  size_t status_cap = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  // (nf, prec, eps, sigma) -> grid size
  std::map<std::tuple<int64_t, int, double, double>, int64_t> grid_of_nf;
};

void free_batch_state(BatchState& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  if (b.cap_stream) (void)hipStreamDestroy(b.cap_stream);
  if (b.dev) (void)hipFree(b.dev);
  if (b.ws) (void)hipFree(b.ws);
  if (b.status_host) (void)hipHostFree(b.status_host);
  b = BatchState{};
}

}  // namespace

struct mils_context {
  int device = -1;
  uint64_t budget = 0;
  std::string err;
  bool poisoned = false;
  std::map<PlanKey, PlanEntry> plans;
  size_t plan_bytes = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // Set once a call has been captured into a caller's graph: that graph
  // holds pointers into the workspace, so a later growth keeps the old
  // buffer (freed with the context) instead of freeing it.
  bool captured = false;
  std::vector<char*> retired;
  // single-series calls may use the two-pass register-tile FFT (plans keyed
  // by this choice, so both kinds can coexist in the cache)
  bool fft2 = true;
  // batched series whose grids fit one workgroup's LDS run on chip
  bool batch_onchip = true;
  int64_t last_batch_onchip = 0;  // such series in the last batch built
  int* host_status = nullptr;  // pinned
  DevStats* last_stats = nullptr;
  int64_t last_illposed = 0;  // ill-posed frequencies of the last call whose status was read
  // plans built since the context was created, and the host time spent on them
  int64_t plans_built = 0;
  double plan_build_s = 0.0;
  hipStream_t last_stream = nullptr;
  bool have_pending = false;
  // per-stage event timing
  bool prof = false;
  uint32_t prof_mask = ~0u;  // stages timed while prof is on
  hipEvent_t prof_begin[kNumStages] = {};
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> prof_recs;
  std::vector<hipEvent_t> prof_pool;
  int num_cu = 256;
  // second stream (default priority) and fork/join events of a periodogram
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_mid = nullptr;
  BatchState batch;
  // the single-series call captured as a HIP graph: its key (arguments,
  // workspace layout, plan) was seen on the previous call; replayed while
  // the calls repeat it
  struct SingleGraph {
    bool enabled = true;
    bool have_key = false;
    unsigned char key[sizeof(CallArgs) + sizeof(Work) + sizeof(void*)] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    hipEvent_t done = nullptr;  // recorded after each replay
  } sg;
  // batch autotuner: (N_f band, eps, precision) -> (sigma, largest spreading tile)
  std::map<std::tuple<int, double, int>, std::pair<double, int>> tuned;
  std::string tune_file;  // MILS_TUNE_CACHE at creation ("" = none)
  std::string tune_key;   // this device's key in that file
};

namespace {

// Reads the decisions recorded for this context's device (missing or
// malformed lines are skipped).
void load_tuning(mils_context* ctx) {
  FILE* f = std::fopen(ctx->tune_file.c_str(), "r");
  if (!f) return;
  char key[256];
  int band = 0, prec = 0, tile = 0;
  double eps = 0.0, sigma = 0.0;
  int loaded = 0;
  while (std::fscanf(f, "%255s %d %lg %d %lg %d", key, &band, &eps, &prec, &sigma, &tile) == 6) {
    if (ctx->tune_key != key) continue;
    ctx->tuned[std::make_tuple(band, eps, prec)] = {sigma, tile};
    ++loaded;
  }
  std::fclose(f);
  mils_log(2, "tuning: %d decisions for %s from %s", loaded, ctx->tune_key.c_str(),
           ctx->tune_file.c_str());
}

void save_tuning(mils_context* ctx, int band, double eps, int prec, double sigma, int tile) {
  if (ctx->tune_file.empty()) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  FILE* f = std::fopen(ctx->tune_file.c_str(), "a");
  if (!f) {
    mils_log(1, "tuning cache %s cannot be written", ctx->tune_file.c_str());
    return;
  }
  std::fprintf(f, "%s %d %.17g %d %.17g %d\n", ctx->tune_key.c_str(), band, eps, prec, sigma,
               tile);
  std::fclose(f);
}

}  // namespace

namespace {

int fail(mils_context* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  // a handled failure (a refused allocation, say) must not stay the thread's
  // last HIP error, or a later launch check would report it
  (void)hipGetLastError();
  mils_log(1, "error %d: %s", code, msg.c_str());
  return code;
}

int hip_fail(mils_context* ctx, hipError_t e, const char* where) {
  if (ctx) {
    ctx->poisoned = true;
    ctx->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  mils_log(1, "device error in %s: %s (context unusable)", where, hipGetErrorString(e));
  return MILS_ERR_DEVICE;
}

int check_params(const mils_params* p) {
  if (!p) return MILS_ERR_INVALID_ARG;
  if (!(std::isfinite(p->f0)) || !(std::isfinite(p->df)) || !(p->df > 0.0))
    return MILS_ERR_INVALID_ARG;
  if (p->nf < 1) return MILS_ERR_INVALID_ARG;
  if (p->nf > ((int64_t)1 << 28)) return MILS_ERR_UNSUPPORTED;
  if (p->precision != MILS_FP64 && p->precision != MILS_FP32) return MILS_ERR_INVALID_ARG;
  if (p->normalization < 0 || p->normalization > 3) return MILS_ERR_INVALID_ARG;
  if (p->flags & ~(uint32_t)(MILS_CENTER_DATA | MILS_FIT_MEAN | MILS_DETERMINISTIC))
    return MILS_ERR_INVALID_ARG;
  if (!std::isfinite(p->eps) || !(p->eps > 0.0)) return MILS_ERR_INVALID_ARG;
  const double lo = p->precision == MILS_FP64 ? 1e-14 : 1e-6;
  if (p->eps < lo || p->eps > 1e-2) return MILS_ERR_UNSUPPORTED;
  if (!std::isfinite(p->f0 + (double)(p->nf - 1) * p->df)) return MILS_ERR_INVALID_ARG;
  return MILS_OK;
}

// Whether the caller is capturing `stream` into a graph (a NULL stream is
// never captured here).  On a query error the answer is "yes", so that the
// callers refuse rather than risk an allocation inside a capture.
bool capturing(hipStream_t stream) {
  if (!stream) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return cs != hipStreamCaptureStatusNone;
}

int check_nd(int64_t nd) {
  if (nd < 1 || nd > kMaxPoints) return MILS_ERR_INVALID_ARG;
  return MILS_OK;
}

// The two-pass register-tile FFT for single-series calls (MILS_FFT2=0 turns
// it off: those plans then use three or more LDS passes).
bool fft2_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("MILS_FFT2");
    return !(e && e[0] == '0');
  }();
  return on;
}

int get_plan(mils_context* ctx, int64_t nf, double eps, int prec, int G, PlanEntry** out,
             bool upload, bool batch = false, int64_t n_fixed = 0, int tile_max = 0,
             bool fft2 = false) {
  PlanKey key{nf, eps, prec, G + (batch ? 10 : 0) + (fft2 ? 20 : 0), n_fixed, tile_max};
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end() && (!upload || it->second.tw)) {
    *out = &it->second;
    return MILS_OK;
  }
  const auto t_build = std::chrono::steady_clock::now();
  PlanEntry e;
  std::string err;
  PlanRequest r{nf, eps, prec, G};
  r.batch = batch;
  r.n_fixed = n_fixed;
  r.tile_max = tile_max;
  r.fft2 = fft2;
  if (!make_plan(r, &e.plan, &err)) return fail(ctx, MILS_ERR_UNSUPPORTED, err);
  std::vector<double> tw;
  make_twiddles(&e.plan, &tw);
  if (upload) {
    const size_t twbytes = prec == 1 ? tw.size() * sizeof(float) : tw.size() * sizeof(double);
    const size_t phbytes = sizeof(double) * (e.plan.K + 1);
    std::vector<double> z, gphi;
    phihat_nodes(e.plan, &z, &gphi);
    const size_t nbytes = sizeof(double) * 2 * z.size();
    std::vector<double> hc;
    make_horner(e.plan, &hc);
    const size_t hbytes = hc.size() * (prec == 1 ? sizeof(float) : sizeof(double));
    const size_t p2bytes = e.plan.fft2 ? sizeof(double) * e.plan.n : 0;
    e.bytes = twbytes + phbytes + nbytes + hbytes + p2bytes;
    if (ctx->budget && ctx->plan_bytes + ctx->ws_bytes + e.bytes > ctx->budget)
      return fail(ctx, MILS_ERR_OOM, "plan tables exceed the HBM budget");
    char* buf = nullptr;
    hipError_t he = hipMalloc(&buf, twbytes + phbytes + nbytes + hbytes + p2bytes + 1280);
    if (he != hipSuccess) return fail(ctx, MILS_ERR_OOM, "hipMalloc of plan tables failed");
    e.inv_phihat = reinterpret_cast<double*>(buf);
    e.tw = buf + ((phbytes + 255) & ~(size_t)255);
    double* nodes = reinterpret_cast<double*>(
        reinterpret_cast<char*>(e.tw) + ((twbytes + 255) & ~(size_t)255));
    if (prec == 1) {
      std::vector<float> f(tw.begin(), tw.end());
      he = hipMemcpy(e.tw, f.data(), twbytes, hipMemcpyHostToDevice);
    } else {
      he = hipMemcpy(e.tw, tw.data(), twbytes, hipMemcpyHostToDevice);
    }
    if (he != hipSuccess) return hip_fail(ctx, he, "plan upload");
    std::vector<double> zn(z);
    zn.insert(zn.end(), gphi.begin(), gphi.end());
    he = hipMemcpy(nodes, zn.data(), nbytes, hipMemcpyHostToDevice);
    if (he != hipSuccess) return hip_fail(ctx, he, "plan upload");
    char* hdev = reinterpret_cast<char*>(nodes) + ((nbytes + 255) & ~(size_t)255);
    if (prec == 1) {
      std::vector<float> f(hc.begin(), hc.end());
      he = hipMemcpy(hdev, f.data(), hbytes, hipMemcpyHostToDevice);
    } else {
      he = hipMemcpy(hdev, hc.data(), hbytes, hipMemcpyHostToDevice);
    }
    if (he != hipSuccess) return hip_fail(ctx, he, "plan upload");
    e.plan.hcoef = hdev;
    if (e.plan.fft2)
      e.inv_phihat2 = reinterpret_cast<double*>(hdev + ((hbytes + 255) & ~(size_t)255));
    he = launch_phihat(e.inv_phihat, e.plan.K, (double)e.plan.w, (double)e.plan.n, nodes,
                       nodes + z.size(), (int)z.size(), nullptr);
    if (he == hipSuccess && e.plan.fft2)
      he = launch_phihat2(e.inv_phihat2, e.inv_phihat, e.plan.pass[0].L, e.plan.pass[1].L,
                          e.plan.n, e.plan.nf, e.plan.K, nullptr);
    if (he == hipSuccess) he = hipDeviceSynchronize();
    if (he != hipSuccess) return hip_fail(ctx, he, "phihat kernel");
    ctx->plan_bytes += e.bytes;
  }
  auto& slot = ctx->plans[key];
  if (slot.tw) {
    (void)hipFree(reinterpret_cast<char*>(slot.inv_phihat));
    ctx->plan_bytes -= slot.bytes;
  }
  slot = e;
  *out = &slot;
  ++ctx->plans_built;
  const double build_s =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build).count();
  ctx->plan_build_s += build_s;
  mils_log(2, "plan nf=%lld eps=%g %s%s: n=%lld w=%d passes=%d%s, %.2f ms", (long long)nf, eps,
           prec == 1 ? "fp32" : "fp64", batch ? " batch" : "", (long long)e.plan.n, e.plan.w,
           e.plan.npass, e.plan.fft2 ? " two-pass" : "", build_s * 1e3);
  return MILS_OK;
}

// Whether the single-series plan of (nf, eps, prec, G) exists with its device
// tables (a call may then run without allocating).
bool plan_ready(mils_context* ctx, int64_t nf, double eps, int prec, int G) {
  PlanKey key{nf, eps, prec, G + (ctx->fft2 ? 20 : 0), 0, 0};
  auto it = ctx->plans.find(key);
  return it != ctx->plans.end() && it->second.tw;
}

// Size for a buffer that must hold `need` bytes and holds `have`: half
// again as large as before at least, so that growing requests (a server's
// mix of sizes) reallocate rarely -- a reallocation waits for the device --
// and within `room` when room > 0.
size_t grow_to(size_t need, size_t have, size_t room) {
  size_t s = std::max(need, have + have / 2);
  if (room && s > room) s = std::max(need, room);
  return s;
}

// Device allocation of `want` bytes, or of `need` if that fails.
hipError_t malloc_grown(char** p, size_t want, size_t need, size_t* got) {
  if (want > need && hipMalloc(p, want) == hipSuccess) {
    *got = want;
    return hipSuccess;
  }
  (void)hipGetLastError();
  hipError_t he = hipMalloc(p, need);
  *got = he == hipSuccess ? need : 0;
  return he;
}

int ensure_workspace(mils_context* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return MILS_OK;
  if (ctx->budget && ctx->plan_bytes + bytes > ctx->budget)
    return fail(ctx, MILS_ERR_OOM, "workspace exceeds the HBM budget");
  const size_t room = ctx->budget ? ctx->budget - ctx->plan_bytes : 0;
  const size_t want = grow_to(bytes, ctx->ws_bytes, room);
  if (ctx->ws) {
    hipError_t he = hipDeviceSynchronize();
    if (he != hipSuccess) return hip_fail(ctx, he, "workspace resize");
    if (ctx->captured) ctx->retired.push_back(ctx->ws);
    else (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  char* p = nullptr;
  size_t got = 0;
  if (malloc_grown(&p, want, bytes, &got) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, MILS_ERR_OOM, "hipMalloc of the workspace failed");
  }
  ctx->ws = p;
  ctx->ws_bytes = got;
  mils_log(2, "workspace grown to %.1f MB", (double)got / 1e6);
  // the statistics block starts cleared (every call's statistics kernels
  // rewrite it before any other kernel reads it).  The memset runs on the
  // null stream and may still be in flight when hipMemset returns; a
  // caller's non-blocking stream (a server lane's) is not ordered after it,
  // so wait for it here: it once landed in the middle of a lane's first
  // call.
  hipError_t he = hipMemset(p, 0, 4096);
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he != hipSuccess) return hip_fail(ctx, he, "workspace init");
  return MILS_OK;
}

hipEvent_t prof_event(mils_context* ctx) {
  if (!ctx->prof_pool.empty()) {
    hipEvent_t e = ctx->prof_pool.back();
    ctx->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_hook(void* ud, int stage, int begin, hipStream_t s) {
  mils_context* ctx = static_cast<mils_context*>(ud);
  if (!((ctx->prof_mask >> stage) & 1u)) return;
  hipEvent_t e = prof_event(ctx);
  if (!e) return;
  (void)hipEventRecord(e, s);
  if (begin) {
    ctx->prof_begin[stage] = e;
  } else if (ctx->prof_begin[stage]) {
    ctx->prof_recs.emplace_back(stage, ctx->prof_begin[stage], e);
    ctx->prof_begin[stage] = nullptr;
  } else {
    ctx->prof_pool.push_back(e);
  }
}

// Graphs for repeated single-series calls (MILS_GRAPH=0 turns them off).
bool graphs_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("MILS_GRAPH");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Releases the context's single-series graph once its last replay has
// finished (the replay may still be queued when the caller did not wait).
void release_single_graph(mils_context* ctx) {
  auto& G = ctx->sg;
  if (G.exec) {
    if (G.done) (void)hipEventSynchronize(G.done);
    (void)hipGraphExecDestroy(G.exec);
  }
  if (G.graph) (void)hipGraphDestroy(G.graph);
  G.exec = nullptr;
  G.graph = nullptr;
}

// The launches of one single-series call: the first time a key repeats, they
// are captured (on a context-owned stream; the fork to the second stream and
// the join become graph edges) and the graph replays for as long as the key
// repeats; a new key launches directly.  Launching a graph costs one call
// and lets the runtime queue the kernels back to back.
hipError_t launch_single_graph(mils_context* ctx, const CallArgs& a, const Plan& plan,
                               const Work& w, hipStream_t stream, const AuxStream& aux) {
  auto& G = ctx->sg;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t he = hipStreamIsCapturing(stream, &cs);
  if (he != hipSuccess) return he;
  if (cs != hipStreamCaptureStatusNone) return launch_path(a, plan, w, stream, nullptr, &aux);
  unsigned char key[sizeof(G.key)];
  std::memcpy(key, &a, sizeof(CallArgs));
  std::memcpy(key + sizeof(CallArgs), &w, sizeof(Work));
  const Plan* pp = &plan;
  std::memcpy(key + sizeof(CallArgs) + sizeof(Work), &pp, sizeof(void*));
  const bool same = G.have_key && std::memcmp(key, G.key, sizeof(key)) == 0;
  if (!same) {
    release_single_graph(ctx);
    std::memcpy(G.key, key, sizeof(key));
    G.have_key = true;
    return launch_path(a, plan, w, stream, nullptr, &aux);
  }
  if (!G.exec) {
    if (!G.cap) he = hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking);
    if (he == hipSuccess && !G.done) he = hipEventCreateWithFlags(&G.done, hipEventDisableTiming);
    if (he == hipSuccess) he = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
      hipError_t le = launch_path(a, plan, w, G.cap, nullptr, &aux);
      he = hipStreamEndCapture(G.cap, &G.graph);
      if (le != hipSuccess) he = le;
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0);
    if (he != hipSuccess) return he;
  }
  he = hipGraphLaunch(G.exec, stream);
  if (he == hipSuccess) he = hipEventRecord(G.done, stream);
  return he;
}

// Arguments of a single-series call (zero padding: the bytes serve as a
// graph key).
CallArgs single_args(const double* t, const double* y, const double* dy, const double* h,
                     int64_t nd, const mils_params* p, const Plan& plan, double* power,
                     double* sums) {
  CallArgs a;
  std::memset(&a, 0, sizeof(a));
  a.t = t;
  a.y = y;
  a.dy = dy;
  a.h = h;
  a.nd = nd;
  a.nf = p->nf;
  a.f0 = p->f0;
  a.df = p->df;
  centre_frequency(p->f0, p->df, plan.K, &a.fch, &a.fcl);
  a.kzero = zero_index(p->f0, p->df, p->nf);
  a.norm = p->normalization;
  a.center = (p->flags & MILS_CENTER_DATA) ? 1 : 0;
  a.fit_mean = (p->flags & MILS_FIT_MEAN) ? 1 : 0;
  a.dmin = p->eps;
  a.periodogram = y ? 1 : 0;
  a.deterministic = (p->flags & MILS_DETERMINISTIC) ? 1 : 0;
  a.power = power;
  a.sums = sums;
  return a;
}

// Common body of the single-series calls.
int run_single(mils_context* ctx, const double* t, const double* y, const double* dy,
               const double* h, int64_t nd, const mils_params* p, double* power, double* sums,
               hipStream_t stream, bool sync) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  if (ctx->device < 0) return fail(ctx, MILS_ERR_DEVICE, "host-only context cannot compute");
  if (ctx->poisoned) return fail(ctx, MILS_ERR_DEVICE, "context unusable after a device error");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_fail(ctx, he, "hipSetDevice");
  const bool pg = (y != nullptr);
  const int G = pg ? 3 : 1;
  // A call captured into the caller's graph may use only what an earlier
  // uncaptured call of the same sizes left: the plan's tables and a large
  // enough workspace (their allocation, upload and the kernel-transform
  // kernel cannot run inside a capture), and it cannot wait for its result.
  const bool cap = capturing(stream);
  if (cap && sync)
    return fail(ctx, MILS_ERR_INVALID_ARG,
                "a synchronous call cannot be captured into a graph: use the _async variant");
  if (cap && !plan_ready(ctx, p->nf, p->eps, p->precision, G))
    return fail(ctx, MILS_ERR_BUSY,
                "captured call needs a plan that does not exist yet: make one uncaptured call "
                "with these sizes first");
  PlanEntry* pe = nullptr;
  int rc = get_plan(ctx, p->nf, p->eps, p->precision, G, &pe, true, false, 0, 0, ctx->fft2);
  if (rc != MILS_OK) return rc;
  const Plan& plan = pe->plan;
  const size_t need = layout_work(plan, nd, G, nullptr, nullptr);
  if (cap && need > ctx->ws_bytes)
    return fail(ctx, MILS_ERR_BUSY,
                "captured call needs a larger workspace: make one uncaptured call with these "
                "sizes first");
  rc = ensure_workspace(ctx, need);
  if (rc != MILS_OK) return rc;
  if (cap) ctx->captured = true;
  Work w{};
  layout_work(plan, nd, G, ctx->ws, &w);
  w.tw = pe->tw;
  w.inv_phihat = pe->inv_phihat;
  w.inv_phihat2 = pe->inv_phihat2;

  const CallArgs a = single_args(t, y, dy, h, nd, p, plan, power, sums);
  StageHook hook{prof_hook, ctx};
  AuxStream aux{ctx->aux, ctx->ev_fork, ctx->ev_join, ctx->ev_mid};
  if (!ctx->prof && ctx->aux && ctx->sg.enabled && graphs_enabled()) {
    he = launch_single_graph(ctx, a, plan, w, stream, aux);
  } else {
    he = launch_path(a, plan, w, stream, ctx->prof ? &hook : nullptr, ctx->aux ? &aux : nullptr);
  }
  if (he != hipSuccess) return hip_fail(ctx, he, "kernel launch");
  ctx->last_stats = w.stats;
  ctx->last_stream = stream;
  ctx->have_pending = true;
  if (!sync) return MILS_OK;
  return mils_context_status(ctx);
}

}  // namespace

void mils_context_plan_counters(const mils_context* ctx, int64_t* built, double* seconds) {
  *built = ctx->plans_built;
  *seconds = ctx->plan_build_s;
}

extern "C" {

int mils_version(void) { return MILS_VERSION; }

const char* mils_status_str(int s) {
  switch (s) {
    case MILS_OK: return "ok";
    case MILS_ERR_INVALID_ARG: return "invalid argument";
    case MILS_ERR_DEGENERATE: return "degenerate input (constant data)";
    case MILS_ERR_OOM: return "out of device memory or HBM budget";
    case MILS_ERR_DEVICE: return "device error";
    case MILS_ERR_UNSUPPORTED: return "unsupported parameters";
    case MILS_ERR_BUSY: return "busy";
    case MILS_ERR_CANCELLED: return "cancelled";
    case MILS_ERR_TIMEOUT: return "timed out";
    default: return "unknown status";
  }
}

const char* mils_last_error(const mils_context* ctx) {
  if (!ctx) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    return g_create_err.c_str();
  }
  return ctx->err.c_str();
}

int mils_context_create(int device, uint64_t hbm_budget_bytes, mils_context** out) {
  if (!out) return MILS_ERR_INVALID_ARG;
  *out = nullptr;
  if (device < -1) return MILS_ERR_INVALID_ARG;
  mils_context* c = new (std::nothrow) mils_context();
  if (!c) return MILS_ERR_OOM;
  c->device = device;
  c->budget = hbm_budget_bytes;
  c->fft2 = fft2_enabled();
  read_log_level();
  if (device >= 0) {
    int count = 0;
    hipError_t he = hipGetDeviceCount(&count);
    if (he != hipSuccess || device >= count) {
      std::lock_guard<std::mutex> lk(g_err_mu);
      g_create_err = "no such HIP device";
      delete c;
      return MILS_ERR_DEVICE;
    }
    he = hipSetDevice(device);
    if (he == hipSuccess) he = hipHostMalloc(reinterpret_cast<void**>(&c->host_status), 64);
    if (he == hipSuccess)
      he = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_mid, hipEventDisableTiming);
    if (he != hipSuccess) {
      std::lock_guard<std::mutex> lk(g_err_mu);
      g_create_err = std::string("context init: ") + hipGetErrorString(he);
      delete c;
      return MILS_ERR_DEVICE;
    }
    if (const char* tf = std::getenv("MILS_TUNE_CACHE")) {
      c->tune_file = tf;
      c->tune_key = tune_device_key(device);
      if (!c->tune_key.empty()) load_tuning(c);
      else c->tune_file.clear();
    }
  }
  *out = c;
  return MILS_OK;
}

int mils_context_destroy(mils_context* ctx) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->plans)
      if (kv.second.tw) (void)hipFree(reinterpret_cast<char*>(kv.second.inv_phihat));
    if (ctx->ws) (void)hipFree(ctx->ws);
    for (char* r : ctx->retired) (void)hipFree(r);
    free_batch_state(ctx->batch);
    release_single_graph(ctx);
    if (ctx->sg.cap) (void)hipStreamDestroy(ctx->sg.cap);
    if (ctx->sg.done) (void)hipEventDestroy(ctx->sg.done);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_mid) (void)hipEventDestroy(ctx->ev_mid);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->host_status) (void)hipHostFree(ctx->host_status);
    for (auto& r : ctx->prof_recs) {
      (void)hipEventDestroy(std::get<1>(r));
      (void)hipEventDestroy(std::get<2>(r));
    }
    for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
  }
  delete ctx;
  return MILS_OK;
}

int mils_check_periodogram_args(const double* t, const double* y, int64_t nd,
                                const mils_params* p, const double* power) {
  if (!t || !y || !power) return MILS_ERR_INVALID_ARG;
  int rc = check_nd(nd);
  if (rc != MILS_OK) return rc;
  return check_params(p);
}

int mils_plan_info(mils_context* ctx, int64_t nd, const mils_params* p, mils_plan_desc* out) {
  if (!ctx || !out) return MILS_ERR_INVALID_ARG;
  int rc = check_nd(nd);
  if (rc == MILS_OK) rc = check_params(p);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid plan query");
  PlanEntry* pe = nullptr;
  rc = get_plan(ctx, p->nf, p->eps, p->precision, 3, &pe, false, false, 0, 0, ctx->fft2);
  if (rc != MILS_OK) return rc;
  const Plan& pl = pe->plan;
  std::memset(out, 0, sizeof(*out));
  out->sigma = pl.sigma;
  out->width = pl.w;
  out->beta = pl.beta;
  out->n = pl.n;
  out->npass = pl.npass;
  for (int i = 0; i < pl.npass; ++i) out->len[i] = pl.pass[i].L;
  out->tile = pl.T;
  out->bin = pl.Tb;
  out->workspace_bytes = layout_work(pl, nd, 3, nullptr, nullptr);
  {
    // the launch sizes of kernels.hip
    const size_t elem = pl.prec == 1 ? 8 : 16;
    const FftPass& lp = pl.pass[pl.npass - 1];
    const int ntw_l = lp.big ? tw2_count(lp.L) : lp.L;
    out->last_rows = lp.C;
    out->last_lds_bytes = (int32_t)(elem * ((size_t)lp.L * last_pitch(3 * lp.C) + ntw_l));
    out->big = lp.big;
    if (pl.npass > 1) {
      const FftPass& fp = pl.pass[0];
      const int ntw_f = fp.big ? tw2_count(fp.L) : fp.L;
      out->first_cols = fp.C;
      out->first_lds_bytes = (int32_t)(elem * ((size_t)fp.L * fp.C + ntw_f) + fp.L + 16);
    }
    out->fft2 = pl.fft2;
    if (pl.fft2) {
      const bool h = pl.prec == 0;
      out->first_lds_bytes = (int32_t)(pl.prec == 1 ? f2_first_lds<float>(pl.pass[0].L, pl.pass[0].C, h)
                                                    : f2_first_lds<double>(pl.pass[0].L, pl.pass[0].C, h));
      // FP32: the three grids of a row one after another (one exchange line)
      out->last_lds_bytes = (int32_t)(pl.prec == 1 ? f2_last_seq_lds<float>(pl.pass[1].L, false)
                                                   : f2_last_lds<double>(pl.pass[1].L, 3, h));
    }
  }
  return MILS_OK;
}

int mils_kernel_table(mils_context* ctx, const mils_params* p, double* coef, int32_t* ncoef,
                      int32_t* kmax, int32_t* width, double* beta) {
  if (!ctx || !coef || !ncoef || !kmax || !width || !beta) return MILS_ERR_INVALID_ARG;
  int rc = check_params(p);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid plan query");
  PlanEntry* pe = nullptr;
  rc = get_plan(ctx, p->nf, p->eps, p->precision, 3, &pe, false, false, 0, 0, ctx->fft2);
  if (rc != MILS_OK) return rc;
  std::vector<double> hc;
  make_horner(pe->plan, &hc);
  std::copy(hc.begin(), hc.end(), coef);
  *ncoef = horner_n(pe->plan.prec);
  *kmax = kHornerK;
  *width = pe->plan.w;
  *beta = pe->plan.beta;
  return MILS_OK;
}

int mils_kernel_transform(mils_context* ctx, const mils_params* p, int64_t count,
                          const int64_t* modes, double* inv_phihat, int64_t* n_grid) {
  if (!ctx || (count > 0 && (!modes || !inv_phihat)) || count < 0 || !n_grid)
    return MILS_ERR_INVALID_ARG;
  int rc = check_params(p);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid plan query");
  PlanEntry* pe = nullptr;
  rc = get_plan(ctx, p->nf, p->eps, p->precision, 3, &pe, false, false, 0, 0, ctx->fft2);
  if (rc != MILS_OK) return rc;
  const Plan& pl = pe->plan;
  std::vector<double> z, gphi;
  phihat_nodes(pl, &z, &gphi);
  *n_grid = pl.n;
  for (int64_t i = 0; i < count; ++i) {
    if (modes[i] < 0 || modes[i] > pl.K) return fail(ctx, MILS_ERR_INVALID_ARG, "mode out of range");
    // the device table's sum (k_phihat), accumulated here in long double
    const long double alpha = (long double)modes[i] * (3.14159265358979323846264338327950288L *
                                                      (long double)pl.w / (long double)pl.n);
    long double sum = 0.0L;
    for (size_t r = 0; r < z.size(); ++r) sum += (long double)gphi[r] * cosl(alpha * z[r]);
    inv_phihat[i] = (double)(1.0L / ((long double)pl.w * sum));
  }
  return MILS_OK;
}

int mils_trig_sums(mils_context* ctx, const double* t, const double* h, int64_t nd, double f0,
                   double df, int64_t nf, double eps, int32_t precision, double* out,
                   void* hip_stream) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  if (!t || !h || !out) return fail(ctx, MILS_ERR_INVALID_ARG, "null pointer argument");
  int rc = check_nd(nd);
  if (rc != MILS_OK) return fail(ctx, rc, "nd out of range");
  mils_params p{f0, df, nf, eps, precision, 0, 0};
  rc = check_params(&p);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid parameters");
  return run_single(ctx, t, nullptr, nullptr, h, nd, &p, nullptr, out,
                    reinterpret_cast<hipStream_t>(hip_stream), true);
}

int mils_periodogram_async(mils_context* ctx, const double* t, const double* y, const double* dy,
                           int64_t nd, const mils_params* p, double* power, void* hip_stream) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  int rc = mils_check_periodogram_args(t, y, nd, p, power);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid periodogram arguments");
  return run_single(ctx, t, y, dy, nullptr, nd, p, power, nullptr,
                    reinterpret_cast<hipStream_t>(hip_stream), false);
}

int mils_periodogram(mils_context* ctx, const double* t, const double* y, const double* dy,
                     int64_t nd, const mils_params* p, double* power, void* hip_stream) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  int rc = mils_check_periodogram_args(t, y, nd, p, power);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid periodogram arguments");
  return run_single(ctx, t, y, dy, nullptr, nd, p, power, nullptr,
                    reinterpret_cast<hipStream_t>(hip_stream), true);
}

static int mils_periodogram_noalloc_impl(mils_context* ctx, const double* t, const double* y,
                                         const double* dy, int64_t nd, const mils_params* p,
                                         double* power, hipStream_t stream);

int mils_periodogram_noalloc(mils_context* ctx, const double* t, const double* y,
                             const double* dy, int64_t nd, const mils_params* p, double* power,
                             void* hip_stream) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  return mils_periodogram_noalloc_impl(ctx, t, y, dy, nd, p, power,
                                       reinterpret_cast<hipStream_t>(hip_stream));
}

// The plan whose tables occupy each GPU's no-allocation scratch (so that a
// call repeating the previous one's sizes skips the upload).
struct ScratchTables {
  bool valid = false;
  int64_t nf = 0;
  double eps = 0.0;
  int prec = 0;
  bool fft2 = false;
};
static std::mutex g_scratch_mu;
static ScratchTables g_scratch_tables[kNoAllocDevices];

static int mils_periodogram_noalloc_impl(mils_context* ctx, const double* t, const double* y,
                                  const double* dy, int64_t nd, const mils_params* p,
                                  double* power, hipStream_t stream) {
  int rc = mils_check_periodogram_args(t, y, nd, p, power);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid periodogram arguments");
  // the plan on the host (host memory only), then the scratch layout:
  // [1/phihat][twiddles][quadrature nodes][kernel polynomials][1/phihat in
  // two-pass order][workspace]
  Plan plan;
  std::string err;
  PlanRequest r{p->nf, p->eps, p->precision, 3};
  r.fft2 = ctx->fft2;
  if (!make_plan(r, &plan, &err)) return fail(ctx, MILS_ERR_UNSUPPORTED, err);
  std::vector<double> tw;
  make_twiddles(&plan, &tw);
  std::vector<double> z, gphi, hc;
  phihat_nodes(plan, &z, &gphi);
  make_horner(plan, &hc);
  const bool f32 = plan.prec == 1;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t ph_b = up(sizeof(double) * (plan.K + 1));
  const size_t tw_b = up(tw.size() * (f32 ? sizeof(float) : sizeof(double)));
  const size_t nd_b = up(sizeof(double) * 2 * z.size());
  const size_t hc_b = up(hc.size() * (f32 ? sizeof(float) : sizeof(double)));
  const size_t p2_b = plan.fft2 ? up(sizeof(double) * plan.n) : 0;
  const size_t tables = ph_b + tw_b + nd_b + hc_b + p2_b;
  const size_t need = tables + layout_work(plan, nd, 3, nullptr, nullptr);
  if (need > kNoAllocBytes)
    return fail(ctx, MILS_ERR_UNSUPPORTED,
                "the call needs " + std::to_string(need) + " bytes of device scratch; the " +
                    "allocation-free call has " + std::to_string(kNoAllocBytes));
  if (ctx->device < 0) return fail(ctx, MILS_ERR_DEVICE, "host-only context cannot compute");
  if (ctx->poisoned) return fail(ctx, MILS_ERR_DEVICE, "context unusable after a device error");
  if (capturing(stream))
    return fail(ctx, MILS_ERR_UNSUPPORTED,
                "the allocation-free call may upload its plan and waits for its status: it "
                "cannot be captured");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_fail(ctx, he, "hipSetDevice");
  char* base = static_cast<char*>(noalloc_scratch(ctx->device, &he));
  if (!base) return hip_fail(ctx, he, "scratch address");
  double* inv_phihat = reinterpret_cast<double*>(base);
  char* twd = base + ph_b;
  double* nodes = reinterpret_cast<double*>(twd + tw_b);
  char* hdev = reinterpret_cast<char*>(nodes) + nd_b;
  double* iphi2 = plan.fft2 ? reinterpret_cast<double*>(hdev + hc_b) : nullptr;
  plan.hcoef = hdev;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchTables& res = g_scratch_tables[ctx->device];
    const bool same = res.valid && res.nf == p->nf && res.eps == p->eps &&
                      res.prec == p->precision && res.fft2 == (bool)plan.fft2;
    if (!same) {
      res.valid = false;
      std::vector<float> tw32, hc32;
      if (f32) {
        tw32.assign(tw.begin(), tw.end());
        hc32.assign(hc.begin(), hc.end());
      }
      std::vector<double> zn(z);
      zn.insert(zn.end(), gphi.begin(), gphi.end());
      he = hipMemcpyAsync(twd, f32 ? (const void*)tw32.data() : (const void*)tw.data(),
                          tw.size() * (f32 ? sizeof(float) : sizeof(double)),
                          hipMemcpyHostToDevice, stream);
      if (he == hipSuccess)
        he = hipMemcpyAsync(nodes, zn.data(), sizeof(double) * zn.size(), hipMemcpyHostToDevice,
                            stream);
      if (he == hipSuccess)
        he = hipMemcpyAsync(hdev, f32 ? (const void*)hc32.data() : (const void*)hc.data(),
                            hc.size() * (f32 ? sizeof(float) : sizeof(double)),
                            hipMemcpyHostToDevice, stream);
      if (he == hipSuccess)
        he = launch_phihat(inv_phihat, plan.K, (double)plan.w, (double)plan.n, nodes,
                           nodes + z.size(), (int)z.size(), stream);
      if (he == hipSuccess && plan.fft2)
        he = launch_phihat2(iphi2, inv_phihat, plan.pass[0].L, plan.pass[1].L, plan.n, plan.nf,
                            plan.K, stream);
      // the host copies of the tables go out of scope below
      if (he == hipSuccess) he = hipStreamSynchronize(stream);
      if (he != hipSuccess) return hip_fail(ctx, he, "scratch plan upload");
      res.valid = true;
      res.nf = p->nf;
      res.eps = p->eps;
      res.prec = p->precision;
      res.fft2 = plan.fft2;
    }
  }
  Work w{};
  layout_work(plan, nd, 3, base + tables, &w);
  w.tw = twd;
  w.inv_phihat = inv_phihat;
  w.inv_phihat2 = iphi2;
  const CallArgs a = single_args(t, y, dy, nullptr, nd, p, plan, power, nullptr);
  AuxStream aux{ctx->aux, ctx->ev_fork, ctx->ev_join, ctx->ev_mid};
  he = launch_path(a, plan, w, stream, nullptr, ctx->aux ? &aux : nullptr);
  if (he != hipSuccess) return hip_fail(ctx, he, "kernel launch");
  ctx->last_stats = w.stats;
  ctx->last_stream = stream;
  ctx->have_pending = true;
  return mils_context_status(ctx);
}

// Direct evaluation: statistics and the term-by-term sums; the workspace
// holds only the statistics block and its per-block partials.
static int run_direct(mils_context* ctx, const double* t, const double* y, const double* dy,
                      const double* h, int64_t nd, const mils_params* p, double* power,
                      double* sums, hipStream_t stream) {
  if (ctx->device < 0) return fail(ctx, MILS_ERR_DEVICE, "host-only context cannot compute");
  if (capturing(stream))
    return fail(ctx, MILS_ERR_UNSUPPORTED, "direct evaluation is synchronous: it cannot be captured");
  if (ctx->poisoned) return fail(ctx, MILS_ERR_DEVICE, "context unusable after a device error");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_fail(ctx, he, "hipSetDevice");
  const size_t sb = (sizeof(DevStats) + 255) & ~(size_t)255;
  int rc = ensure_workspace(ctx, sb + sizeof(double) * 8 * kStatsBlocks);
  if (rc != MILS_OK) return rc;
  Work w{};
  w.stats = reinterpret_cast<DevStats*>(ctx->ws);
  w.partials = reinterpret_cast<double*>(ctx->ws + sb);
  CallArgs a{};
  a.t = t;
  a.y = y;
  a.dy = dy;
  a.h = h;
  a.nd = nd;
  a.nf = p->nf;
  a.f0 = p->f0;
  a.df = p->df;
  a.kzero = zero_index(p->f0, p->df, p->nf);
  a.norm = p->normalization;
  a.center = (p->flags & MILS_CENTER_DATA) ? 1 : 0;
  a.fit_mean = (p->flags & MILS_FIT_MEAN) ? 1 : 0;
  a.periodogram = y ? 1 : 0;
  a.power = power;
  a.sums = sums;
  he = launch_direct(a, w, stream);
  if (he != hipSuccess) return hip_fail(ctx, he, "kernel launch");
  ctx->last_stats = w.stats;
  ctx->last_stream = stream;
  ctx->have_pending = true;
  return mils_context_status(ctx);
}

int mils_direct_periodogram(mils_context* ctx, const double* t, const double* y,
                            const double* dy, int64_t nd, const mils_params* p, double* power,
                            void* hip_stream) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  int rc = mils_check_periodogram_args(t, y, nd, p, power);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid periodogram arguments");
  return run_direct(ctx, t, y, dy, nullptr, nd, p, power, nullptr,
                    reinterpret_cast<hipStream_t>(hip_stream));
}

int mils_direct_trig_sums(mils_context* ctx, const double* t, const double* h, int64_t nd,
                          double f0, double df, int64_t nf, double* out_re_im,
                          void* hip_stream) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  if (!t || !h || !out_re_im) return fail(ctx, MILS_ERR_INVALID_ARG, "null pointer");
  mils_params p{};
  p.f0 = f0;
  p.df = df;
  p.nf = nf;
  p.eps = 1e-9;
  p.precision = MILS_FP64;
  int rc = check_nd(nd);
  if (rc == MILS_OK) rc = check_params(&p);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid trig-sum arguments");
  return run_direct(ctx, t, nullptr, nullptr, h, nd, &p, nullptr, out_re_im,
                    reinterpret_cast<hipStream_t>(hip_stream));
}

int mils_periodogram_shared_t(mils_context* ctx, const double* t, const double* y,
                              const double* dy, int64_t dy_stride, int64_t nd, int64_t nseries,
                              const mils_params* p, double* power, int32_t* status_per_series,
                              void* hip_stream) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  int rc = mils_check_periodogram_args(t, y, nd, p, power);
  if (rc != MILS_OK) return fail(ctx, rc, "invalid periodogram arguments");
  if (nseries < 1 || nseries > ((int64_t)1 << 24))
    return fail(ctx, MILS_ERR_INVALID_ARG, "nseries must be in [1, 2^24]");
  if (dy && dy_stride != 0 && dy_stride != nd)
    return fail(ctx, MILS_ERR_INVALID_ARG, "dy_stride must be 0 (shared dy) or nd");
  if (p->flags & MILS_DETERMINISTIC)
    return fail(ctx, MILS_ERR_UNSUPPORTED, "MILS_DETERMINISTIC applies to single-series calls");
  if (ctx->device < 0) return fail(ctx, MILS_ERR_DEVICE, "host-only context cannot compute");
  if (ctx->poisoned) return fail(ctx, MILS_ERR_DEVICE, "context unusable after a device error");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_fail(ctx, he, "hipSetDevice");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (capturing(stream))
    return fail(ctx, MILS_ERR_UNSUPPORTED,
                "the shared-times call reads its sort decision back: it cannot be captured");
  PlanEntry* pe = nullptr;
  rc = get_plan(ctx, p->nf, p->eps, p->precision, 3, &pe, true);
  if (rc != MILS_OK) return rc;
  const Plan& plan = pe->plan;
  // workspace: the single-series layout, then B and B2 per output
  // frequency and one statistics block per series plus one for the weights
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t base = up(layout_work(plan, nd, 3, nullptr, nullptr));
  const size_t bsum = up(sizeof(double) * 2 * (size_t)p->nf);
  const size_t nst = (size_t)nseries + 1;
  const size_t low = up(sizeof(double) * 6 * kLowMax * kLowParts);
  rc = ensure_workspace(ctx, base + 2 * bsum + 3 * low + up(sizeof(DevStats) * nst));
  if (rc != MILS_OK) return rc;
  Work w{};
  layout_work(plan, nd, 3, ctx->ws, &w);
  w.tw = pe->tw;
  w.inv_phihat = pe->inv_phihat;
  double* bsum_b = reinterpret_cast<double*>(ctx->ws + base);
  double* bsum_b2 = reinterpret_cast<double*>(ctx->ws + base + bsum);
  double* lowfix[3];
  for (int g = 0; g < 3; ++g)
    lowfix[g] = reinterpret_cast<double*>(ctx->ws + base + 2 * bsum + g * low);
  DevStats* stats = reinterpret_cast<DevStats*>(ctx->ws + base + 2 * bsum + 3 * low);

  CallArgs a{};
  a.t = t;
  a.dy = dy;
  a.nd = nd;
  a.nf = p->nf;
  a.f0 = p->f0;
  a.df = p->df;
  centre_frequency(p->f0, p->df, plan.K, &a.fch, &a.fcl);
  a.kzero = zero_index(p->f0, p->df, p->nf);
  a.norm = p->normalization;
  a.center = (p->flags & MILS_CENTER_DATA) ? 1 : 0;
  a.fit_mean = (p->flags & MILS_FIT_MEAN) ? 1 : 0;
  a.dmin = p->eps;
  a.periodogram = 1;
  const bool shared_w = (dy == nullptr || dy_stride == 0);
  if (shared_w) {
    // the weight-only sums B and B2, once
    CallArgs aw = a;
    aw.unit_y = 1;
    Work ww = w;
    ww.stats = stats + nseries;
    he = launch_weight_sums(aw, plan, ww, bsum_b, bsum_b2, stream);
    a.bsum_b = bsum_b;
    a.bsum_b2 = bsum_b2;
    a.wstats = ww.stats;
    // then groups of up to three series: their A grids go through the FFT
    // passes together and one last pass reads B and B2 once for the group
    // (one series per group with the optional two-pass FFT)
    bool big = false;
    for (int i = 0; i < plan.npass; ++i) big = big || plan.pass[i].big;
    const int64_t gmax = big ? 1 : 3;
    // the sort decision of the weights-only call: series need their own
    // binning only when the points go through the counting sort
    if (he == hipSuccess)
      he = hipMemcpyAsync(ctx->host_status, &ww.stats->need_sort, sizeof(int),
                          hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    const int need_sort = he == hipSuccess ? *ctx->host_status : 1;
    for (int64_t i0 = 0; i0 < nseries && he == hipSuccess; i0 += gmax) {
      SeriesGroup sg{};
      sg.m = (int)std::min<int64_t>(gmax, nseries - i0);
      sg.need_sort = need_sort;
      for (int g = 0; g < sg.m; ++g) {
        sg.y[g] = y + (i0 + g) * nd;
        sg.power[g] = power + (i0 + g) * p->nf;
        sg.stats[g] = stats + i0 + g;
        sg.lowfix[g] = lowfix[g];
      }
      he = launch_series_group(a, plan, ww, sg, stream);
    }
  } else {
    AuxStream aux{ctx->aux, ctx->ev_fork, ctx->ev_join, ctx->ev_mid};
    for (int64_t i = 0; i < nseries && he == hipSuccess; ++i) {
      CallArgs as = a;
      as.y = y + i * nd;
      as.dy = dy + i * nd;
      as.power = power + i * p->nf;
      Work ws = w;
      ws.stats = stats + i;
      he = launch_path(as, plan, ws, stream, nullptr, ctx->aux ? &aux : nullptr);
    }
  }
  if (he != hipSuccess) return hip_fail(ctx, he, "kernel launch");
  std::vector<DevStats> host(nst);
  he = hipMemcpyAsync(host.data(), stats, sizeof(DevStats) * nst, hipMemcpyDeviceToHost, stream);
  if (he == hipSuccess) he = hipStreamSynchronize(stream);
  if (he != hipSuccess) return hip_fail(ctx, he, "status readback");
  ctx->have_pending = false;
  int first = MILS_OK;
  for (int64_t i = 0; i < nseries; ++i) {
    const int st = host[i].status;
    const int code = st == -1 ? MILS_ERR_INVALID_ARG : st == -2 ? MILS_ERR_DEGENERATE : MILS_OK;
    if (status_per_series) status_per_series[i] = code;
    if (first == MILS_OK && code != MILS_OK) first = code;
  }
  if (first == MILS_ERR_INVALID_ARG) return fail(ctx, first, "non-finite input or dy <= 0");
  if (first == MILS_ERR_DEGENERATE) return fail(ctx, first, "constant data: zero reference chi^2");
  return MILS_OK;
}

}  // extern "C"

int mils_check_params(const mils_params* p, int64_t nd) {
  int rc = check_nd(nd);
  return rc != MILS_OK ? rc : check_params(p);
}

// Radix stages of the in-LDS transform of a series that runs on chip: radix
// 16, 8, 4, 2, 5, 3 factors of n in ascending order (the largest stage last,
// so that the stages' Ns stay at most n / R_last).  Returns the number of
// stages, or 0 when n does not qualify (too large, not 5-smooth, too many
// stages, an Ns above 1024 or more LDS than the cap).
int small_radices(int64_t n, signed char* rad) {
  if (n < 16 || n > kSmallMaxN || small_lds_bytes(n) > kSmallLdsCap) return 0;
  int64_t m = n;
  int cnt = 0;
  for (int r : {16, 8, 4, 2, 5, 3}) {
    while (m % r == 0 && cnt < kSmallMaxRad) {
      rad[cnt++] = (signed char)r;
      m /= r;
    }
  }
  if (m != 1) return 0;
  std::sort(rad, rad + cnt);
  if (n / rad[cnt - 1] > 1024) return 0;
  return cnt;
}

// Body of mils_periodogram_batch; the serving loop calls it with
// use_graph = false (its batches change with every call).
// Builds the launches of a batch in B: the series idx[0..m) (indices into the
// caller's arrays, which keep their offsets and output positions), series i
// planned with upsampling factor sig[i] (0: the planner's choice) and
// spreading tiles of at most tmax[i] cells.  nstatus: size of the status array
// (the caller's number of series).
int build_batch(mils_context* ctx, BatchState& B, const std::vector<int64_t>& idx,
                const std::vector<double>& sig, const std::vector<int>& tmax,
                const int64_t* nd_off, const double* t, const double* y, const double* dy,
                const int64_t* nf_off, const double* f0, const double* df,
                const mils_params* common, double* power, int64_t nstatus, hipStream_t stream) {
  const int64_t m = (int64_t)idx.size();
  const int prec = common->precision;
  hipError_t he = hipSuccess;
  // grid size of each series, then grid-size classes (ratio <= 1.06) that share a plan
  std::vector<int64_t> ngrid(m);
  for (int64_t c = 0; c < m; ++c) {
    const int64_t nf = nf_off[idx[c] + 1] - nf_off[idx[c]];
    auto k = std::make_tuple(nf, prec, common->eps, sig[c]);
    auto it = B.grid_of_nf.find(k);
    if (it == B.grid_of_nf.end()) {
      Plan pl;
      std::string err;
      PlanRequest r{nf, common->eps, prec, 3};
      r.batch = true;
      r.sigma = sig[c];
      if (!make_plan(r, &pl, &err)) return fail(ctx, MILS_ERR_UNSUPPORTED, err);
      it = B.grid_of_nf.emplace(k, pl.n).first;
    }
    ngrid[c] = it->second;
  }
  std::vector<std::pair<int64_t, int>> ns(m);
  for (int64_t c = 0; c < m; ++c) ns[c] = {ngrid[c], tmax[c]};
  std::sort(ns.begin(), ns.end(), [](const std::pair<int64_t, int>& x, const std::pair<int64_t, int>& y) {
    return x.second != y.second ? x.second < y.second : x.first < y.first;
  });
  ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
  // classes are keyed by (grid size, tile cap)
  std::map<std::pair<int64_t, int>, int> cls_of_n;
  std::vector<int64_t> cls_n;
  std::vector<int> cls_t;
  for (size_t i = 0; i < ns.size();) {
    size_t j = i;
    while (j + 1 < ns.size() && ns[j + 1].second == ns[i].second &&
           (double)ns[j + 1].first <= 1.06 * (double)ns[i].first)
      ++j;
    const int cid = (int)cls_n.size();
    cls_n.push_back(ns[j].first);
    cls_t.push_back(ns[i].second);
    for (size_t q = i; q <= j; ++q) cls_of_n[ns[q]] = cid;
    i = j + 1;
  }
  const int ncls = (int)cls_n.size();
  std::vector<int64_t> cls_nf(ncls, 1);
  std::vector<int> cls_of(m);
  std::vector<char> cls_tuned(ncls, 0);
  for (int64_t c = 0; c < m; ++c) {
    cls_of[c] = cls_of_n[{ngrid[c], tmax[c]}];
    cls_nf[cls_of[c]] = std::max<int64_t>(cls_nf[cls_of[c]], nf_off[idx[c] + 1] - nf_off[idx[c]]);
    if (sig[c] > 1.0) cls_tuned[cls_of[c]] = 1;
  }
  // A class of series planned with the default upsampling s takes the plan
  // of its grid n for floor(n / s) frequencies: every member's own grid was
  // at least s nf and at most n, so this covers all of them (kernel width for
  // upsampling s, deconvolution table long enough), and the plan depends on
  // the grid alone, not on which series happen to share the batch.
  const double s_def = planner_sigma(common->eps, prec, true);
  for (int k = 0; k < ncls; ++k)
    if (!cls_tuned[k])
      cls_nf[k] = std::max<int64_t>(cls_nf[k], (int64_t)std::floor((double)cls_n[k] / s_def));
  std::vector<Plan> plans(ncls);
  std::vector<const void*> twp(ncls);
  std::vector<const double*> php(ncls);
  for (int k = 0; k < ncls; ++k) {
    PlanEntry* pe = nullptr;
    int rc = get_plan(ctx, cls_nf[k], common->eps, prec, 3, &pe, true, true, cls_n[k], cls_t[k]);
    if (rc != MILS_OK) return rc;
    plans[k] = pe->plan;
    twp[k] = pe->tw;
    php[k] = pe->inv_phihat;
  }
  // series descriptors and their workspaces; chunks whose workspaces fit the cap
  std::vector<BatchCurve> cur(m);
  std::vector<size_t> wsz(m);
  for (int64_t c = 0; c < m; ++c) {
    const int64_t oc = idx[c];
    BatchCurve& d = cur[c];
    d.t_off = nd_off[oc];
    d.nd = nd_off[oc + 1] - nd_off[oc];
    d.out_off = nf_off[oc];
    d.nf = nf_off[oc + 1] - nf_off[oc];
    d.K = d.nf / 2;
    d.f0 = f0[oc];
    d.df = df[oc];
    centre_frequency(d.f0, d.df, d.K, &d.fch, &d.fcl);
    d.kzero = zero_index(d.f0, d.df, d.nf);
    d.plan = cls_of[c];
    d.index = (int)oc;
    d.nsrad = ctx->batch_onchip ? small_radices(plans[cls_of[c]].n, d.srad) : 0;
    d.small = d.nsrad > 0;
    wsz[c] = (layout_work(plans[cls_of[c]], d.nd, 3, nullptr, nullptr, true) + 255) & ~(size_t)255;
  }
  size_t cap = kBatchWorkspaceCap;
  if (ctx->budget) {
    const size_t used = ctx->plan_bytes + ctx->ws_bytes;
    cap = ctx->budget > used ? std::min<size_t>(cap, (ctx->budget - used) / 2) : 0;
  }
  std::vector<int64_t> chunk_begin{0};
  size_t acc = 0, ws_max = 0;
  for (int64_t c = 0; c < m; ++c) {
    if (wsz[c] > cap) return fail(ctx, MILS_ERR_OOM, "a series of the batch exceeds the HBM budget");
    if (acc + wsz[c] > cap) {
      chunk_begin.push_back(c);
      ws_max = std::max(ws_max, acc);
      acc = 0;
    }
    acc += wsz[c];
  }
  ws_max = std::max(ws_max, acc);
  chunk_begin.push_back(m);
  const int nchunks = (int)chunk_begin.size() - 1;
  // work items of every chunk
  struct ChunkItems {
    std::vector<BatchItem> spread, pass[kMaxPass - 1], last, small;
    size_t small_lds = 0;
  };
  std::vector<ChunkItems> ci(nchunks);
  for (int k = 0; k < nchunks; ++k) {
    for (int64_t c = chunk_begin[k]; c < chunk_begin[k + 1]; ++c) {
      const Plan& q = plans[cls_of[c]];
      const int lc = (int)(c - chunk_begin[k]);
      if (cur[c].small) {
        ci[k].small.push_back({lc, 0, cls_of[c]});
        ci[k].small_lds = std::max(ci[k].small_lds, small_lds_bytes(q.n));
        continue;
      }
      const int64_t ntl = (q.n + q.T - 1) / q.T;
      for (int64_t tl = 0; tl < ntl; ++tl) ci[k].spread.push_back({lc, (int)tl, cls_of[c]});
      for (int ip = 0; ip + 1 < q.npass; ++ip) {
        const FftPass& ps = q.pass[ip];
        const int64_t nblk = ps.P * ((ps.S + ps.C - 1) / ps.C);
        // one item per column block and grid, or per block for all three
        const int per_item = prec == 1 ? kBatchPassGrids<float> : kBatchPassGrids<double>;
        const int64_t nitems = nblk * (3 / per_item);
        for (int64_t x = 0; x < nitems; ++x) ci[k].pass[ip].push_back({lc, (int)x, cls_of[c]});
      }
      const FftPass& ls = q.pass[q.npass - 1];
      for (int64_t x = 0; x < (ls.P + ls.C - 1) / ls.C; ++x) ci[k].last.push_back({lc, (int)x, cls_of[c]});
    }
  }
  // dynamic LDS of each pass launch (largest class that takes part)
  size_t pass_lds[kMaxPass - 1] = {0, 0, 0}, last_lds = 0;
  const size_t elem = prec == 1 ? 8 : 16;
  for (int k = 0; k < ncls; ++k) {
    const Plan& q = plans[k];
    for (int ip = 0; ip + 1 < q.npass; ++ip) {
      const FftPass& ps = q.pass[ip];
      pass_lds[ip] = std::max(pass_lds[ip], elem * (size_t)(ps.L * ps.C + ps.L) + ps.L + 16);
    }
    const FftPass& ls = q.pass[q.npass - 1];
    last_lds = std::max(last_lds, elem * (size_t)(ls.L * last_pitch(3 * ls.C) + ls.L));
  }
  // device layout: curves, plans, table pointers, works, items, status
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  const size_t o_cur = off;
  off += al(sizeof(BatchCurve) * m);
  const size_t o_plan = off;
  off += al(sizeof(Plan) * ncls);
  const size_t o_tw = off;
  off += al(sizeof(void*) * ncls);
  const size_t o_ph = off;
  off += al(sizeof(void*) * ncls);
  const size_t o_work = off;
  off += al(sizeof(Work) * m);
  const size_t o_st = off;
  off += al(sizeof(int) * nstatus);
  // each of a chunk's item lists starts on a 256-byte boundary with 256
  // bytes to spare: the reservation adds up exactly what the upload below
  // advances by, list by list
  auto list_bytes = [&](size_t n) { return al(sizeof(BatchItem) * n) + 256; };
  std::vector<size_t> o_items(nchunks);
  for (int k = 0; k < nchunks; ++k) {
    o_items[k] = off;
    off += list_bytes(ci[k].spread.size()) + list_bytes(ci[k].last.size()) +
           list_bytes(ci[k].small.size());
    for (int ip = 0; ip < kMaxPass - 1; ++ip) off += list_bytes(ci[k].pass[ip].size());
  }
  const size_t dev_bytes = off + 256;
  if (ctx->budget && ctx->plan_bytes + ctx->ws_bytes + dev_bytes + ws_max > ctx->budget)
    return fail(ctx, MILS_ERR_OOM, "batch workspace exceeds the HBM budget");
  he = hipStreamSynchronize(stream);
  if (he == hipSuccess) he = batch_prepare();
  if (he != hipSuccess) return hip_fail(ctx, he, "batch setup");
  // room left by the budget for the batch's two buffers (0: no budget)
  const size_t room = ctx->budget ? ctx->budget - ctx->plan_bytes - ctx->ws_bytes : 0;
  if (B.dev_bytes < dev_bytes) {
    const size_t had = B.dev_bytes;
    if (B.dev) (void)hipFree(B.dev);
    B.dev = nullptr;
    B.dev_bytes = 0;
    const size_t want = grow_to(dev_bytes, had, room ? room - ws_max : 0);
    if (malloc_grown(&B.dev, want, dev_bytes, &B.dev_bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, MILS_ERR_OOM, "hipMalloc of batch descriptors failed");
    }
  }
  if (B.ws_bytes < ws_max) {
    const size_t had = B.ws_bytes;
    if (B.ws) (void)hipFree(B.ws);
    B.ws = nullptr;
    B.ws_bytes = 0;
    const size_t left = room > B.dev_bytes + ws_max ? room - B.dev_bytes : ws_max;
    const size_t want = grow_to(ws_max, had, room ? left : 0);
    if (malloc_grown(&B.ws, want, ws_max, &B.ws_bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, MILS_ERR_OOM, "hipMalloc of batch workspace failed");
    }
  }
  if (B.status_cap < (size_t)nstatus) {
    if (B.status_host) (void)hipHostFree(B.status_host);
    B.status_host = nullptr;
    he = hipHostMalloc(reinterpret_cast<void**>(&B.status_host), sizeof(int32_t) * nstatus);
    if (he != hipSuccess) return fail(ctx, MILS_ERR_OOM, "pinned status buffer");
    B.status_cap = nstatus;
  }
  // workspaces of each chunk start at the base of the shared buffer
  std::vector<Work> works(m);
  for (int k = 0; k < nchunks; ++k) {
    size_t woff = 0;
    for (int64_t c = chunk_begin[k]; c < chunk_begin[k + 1]; ++c) {
      layout_work(plans[cls_of[c]], cur[c].nd, 3, B.ws + woff, &works[c], true);
      woff += wsz[c];
    }
  }
  // descriptor uploads on the call's stream (then waited for below): the
  // batch's kernels follow on that stream, which may be a non-blocking one
  // that copies on the null stream would not precede
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (he == hipSuccess && bytes)
      he = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
  };
  up(B.dev + o_cur, cur.data(), sizeof(BatchCurve) * m);
  up(B.dev + o_plan, plans.data(), sizeof(Plan) * ncls);
  up(B.dev + o_tw, twp.data(), sizeof(void*) * ncls);
  up(B.dev + o_ph, php.data(), sizeof(void*) * ncls);
  up(B.dev + o_work, works.data(), sizeof(Work) * m);
  B.launches.assign(nchunks, BatchLaunch{});
  ctx->last_batch_onchip = 0;
  for (int k = 0; k < nchunks && he == hipSuccess; ++k) {
    BatchLaunch& L = B.launches[k];
    const int64_t c0 = chunk_begin[k];
    BatchArgs& ba = L.args;
    ba.curves = reinterpret_cast<const BatchCurve*>(B.dev + o_cur) + c0;
    ba.ncurves = (int)(chunk_begin[k + 1] - c0);
    ba.plans = reinterpret_cast<const Plan*>(B.dev + o_plan);
    ba.tw = reinterpret_cast<const void* const*>(B.dev + o_tw);
    ba.inv_phihat = reinterpret_cast<const double* const*>(B.dev + o_ph);
    ba.works = reinterpret_cast<const Work*>(B.dev + o_work) + c0;
    ba.t = t;
    ba.y = y;
    ba.dy = dy;
    ba.power = power;
    ba.norm = common->normalization;
    ba.center = (common->flags & MILS_CENTER_DATA) ? 1 : 0;
    ba.fit_mean = (common->flags & MILS_FIT_MEAN) ? 1 : 0;
    ba.dmin = common->eps;
    ba.status = reinterpret_cast<int*>(B.dev + o_st);
    L.prec = prec;
    size_t io = o_items[k];
    auto put = [&](const std::vector<BatchItem>& v) -> const BatchItem* {
      const BatchItem* ptr = reinterpret_cast<const BatchItem*>(B.dev + io);
      up(B.dev + io, v.data(), sizeof(BatchItem) * v.size());
      io += list_bytes(v.size());
      return ptr;
    };
    L.spread_items = put(ci[k].spread);
    L.nspread = (int)ci[k].spread.size();
    for (int ip = 0; ip < kMaxPass - 1; ++ip) {
      L.pass_items[ip] = put(ci[k].pass[ip]);
      L.npass_items[ip] = (int)ci[k].pass[ip].size();
      L.pass_lds[ip] = pass_lds[ip];
    }
    L.last_items = put(ci[k].last);
    L.nlast = (int)ci[k].last.size();
    L.last_lds = last_lds;
    L.small_items = put(ci[k].small);
    L.nsmall = (int)ci[k].small.size();
    L.small_lds = ci[k].small_lds;
    ctx->last_batch_onchip += L.nsmall;
  }
  // the host vectors are released on return
  if (he == hipSuccess) he = hipStreamSynchronize(stream);
  if (he != hipSuccess) return hip_fail(ctx, he, "batch descriptor upload");
  B.status_dev = reinterpret_cast<int*>(B.dev + o_st);
  if (B.exec) (void)hipGraphExecDestroy(B.exec);
  if (B.graph) (void)hipGraphDestroy(B.graph);
  B.exec = nullptr;
  B.graph = nullptr;
  B.ncurves = nstatus;
  return MILS_OK;
}

hipError_t launch_all(const BatchState& B, hipStream_t s) {
  for (const BatchLaunch& L : B.launches) {
    hipError_t e = launch_batch(L, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Half-octave band of a series by its number of frequencies (the unit of the
// batch autotuner).
int nf_band(int64_t nf) { return (int)std::floor(2.0 * std::log2((double)nf)); }

bool autotune_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("MILS_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Batch autotuner: for each band of N_f with at least kTuneMin series that
// has no decision yet for (eps, precision), time a sample of its series
// (up to kTuneSample, spread over the band) under each candidate (sigma,
// largest spreading tile) and keep the fastest.  Candidates: the planner's
// sigma and larger ones (a wider grid with a narrower kernel), tiles of 1024
// and 256 cells.  The sample runs through the same launches as the batch and
// writes the sampled series' own outputs (rewritten by the real run).
constexpr int kTuneMin = 16, kTuneSample = 48;
int autotune_batch(mils_context* ctx, int64_t ncurves, const int64_t* nd_off, const double* t,
                   const double* y, const double* dy, const int64_t* nf_off, const double* f0,
                   const double* df, const mils_params* common, double* power,
                   hipStream_t stream) {
  const int prec = common->precision;
  std::map<int, std::vector<int64_t>> bands;
  for (int64_t c = 0; c < ncurves; ++c) bands[nf_band(nf_off[c + 1] - nf_off[c])].push_back(c);
  std::vector<std::pair<double, int>> cand;
  // 0: the planner's sigma (1.25 in FP64, 1.5 for batched FP32 series)
  for (double sg : prec == 1 ? std::vector<double>{0.0, 2.0} : std::vector<double>{0.0, 1.5, 2.0})
    for (int tm : {1024, 256}) cand.push_back({sg, tm});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) return hip_fail(ctx, he, "autotuner events");
  int rc = MILS_OK;
  BatchState T;
  for (auto& kv : bands) {
    const auto key = std::make_tuple(kv.first, common->eps, prec);
    if (ctx->tuned.count(key) || (int)kv.second.size() < kTuneMin) continue;
    std::vector<int64_t> sample;
    const int64_t nb = (int64_t)kv.second.size();
    const int64_t ns = std::min<int64_t>(nb, kTuneSample);
    for (int64_t i = 0; i < ns; ++i) sample.push_back(kv.second[(size_t)(i * nb / ns)]);
    double best_ms = 1e300;
    std::pair<double, int> best = cand[0];
    for (const auto& cv : cand) {
      std::vector<double> sig(sample.size(), cv.first);
      std::vector<int> tm(sample.size(), cv.second);
      rc = build_batch(ctx, T, sample, sig, tm, nd_off, t, y, dy, nf_off, f0, df, common, power,
                       ncurves, stream);
      if (rc == MILS_ERR_UNSUPPORTED) {  // this sigma does not plan for the band
        rc = MILS_OK;
        continue;
      }
      if (rc != MILS_OK) break;
      he = launch_all(T, stream);  // warm-up
      if (he == hipSuccess) he = hipEventRecord(e0, stream);
      if (he == hipSuccess) he = launch_all(T, stream);
      if (he == hipSuccess) he = hipEventRecord(e1, stream);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) {
        rc = hip_fail(ctx, he, "autotuner run");
        break;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = cv;
      }
    }
    if (rc != MILS_OK) break;
    ctx->tuned[key] = best;
    mils_log(2, "tuning: band %d eps %g %s -> sigma %g, tile cap %d (%.3f ms)", kv.first,
             common->eps, prec == 1 ? "fp32" : "fp64", best.first, best.second, best_ms);
    save_tuning(ctx, kv.first, common->eps, prec, best.first, best.second);
  }
  (void)hipStreamSynchronize(stream);
  free_batch_state(T);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int mils_batch_run(mils_context* ctx, int64_t ncurves, const int64_t* nd_off, const double* t,
                   const double* y, const double* dy, const int64_t* nf_off, const double* f0,
                   const double* df, const mils_params* common, double* power,
                   int32_t* status_per_curve, void* hip_stream, bool use_graph) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  if (ncurves < 1 || ncurves > (int64_t)0x7fffffff || !nd_off || !nf_off || !f0 || !df ||
      !common || !t || !y || !power)
    return fail(ctx, MILS_ERR_INVALID_ARG, "invalid batch arguments");
  if (nd_off[0] != 0 || nf_off[0] != 0) return fail(ctx, MILS_ERR_INVALID_ARG, "offsets must start at 0");
  if (common->flags & MILS_DETERMINISTIC)
    return fail(ctx, MILS_ERR_UNSUPPORTED, "MILS_DETERMINISTIC applies to single-series calls");
  if (capturing(reinterpret_cast<hipStream_t>(hip_stream)))
    return fail(ctx, MILS_ERR_UNSUPPORTED,
                "the batched call uploads its layout synchronously: it cannot be captured");
  for (int64_t c = 0; c < ncurves; ++c) {
    mils_params p = *common;
    p.f0 = f0[c];
    p.df = df[c];
    p.nf = nf_off[c + 1] - nf_off[c];
    int rc = check_nd(nd_off[c + 1] - nd_off[c]);
    if (rc == MILS_OK) rc = check_params(&p);
    if (rc != MILS_OK) return fail(ctx, rc, "invalid curve " + std::to_string(c) + " in batch");
  }
  if (ctx->device < 0) return fail(ctx, MILS_ERR_DEVICE, "host-only context cannot compute");
  if (ctx->poisoned) return fail(ctx, MILS_ERR_DEVICE, "context unusable after a device error");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return hip_fail(ctx, he, "hipSetDevice");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  BatchState& B = ctx->batch;
  const int prec = common->precision;
  if (use_graph && autotune_enabled()) {
    int rc = autotune_batch(ctx, ncurves, nd_off, t, y, dy, nf_off, f0, df, common, power, stream);
    if (rc != MILS_OK) return rc;
  }
  // per-series plan choices: the band's tuned decision, else the planner's
  std::vector<int64_t> idx(ncurves);
  std::vector<double> sig(ncurves, 0.0);
  std::vector<int> tmax(ncurves, 0);
  for (int64_t c = 0; c < ncurves; ++c) {
    idx[c] = c;
    auto it = ctx->tuned.find(std::make_tuple(nf_band(nf_off[c + 1] - nf_off[c]), common->eps, prec));
    if (it != ctx->tuned.end()) {
      sig[c] = it->second.first;
      tmax[c] = it->second.second;
    }
  }

  uint64_t key = 1469598103934665603ull;
  key = fnv1a(key, &ncurves, sizeof(ncurves));
  key = fnv1a(key, nd_off, sizeof(int64_t) * (ncurves + 1));
  key = fnv1a(key, nf_off, sizeof(int64_t) * (ncurves + 1));
  key = fnv1a(key, f0, sizeof(double) * ncurves);
  key = fnv1a(key, df, sizeof(double) * ncurves);
  key = fnv1a(key, &common->eps, sizeof(double));
  key = fnv1a(key, &common->precision, sizeof(int32_t) * 2);
  key = fnv1a(key, &common->flags, sizeof(uint32_t));
  key = fnv1a(key, sig.data(), sizeof(double) * ncurves);
  key = fnv1a(key, tmax.data(), sizeof(int) * ncurves);
  key = fnv1a(key, &ctx->batch_onchip, sizeof(bool));
  const void* ptrs[4] = {t, y, dy, power};
  key = fnv1a(key, ptrs, sizeof(ptrs));

  if (!(B.valid && B.key == key)) {
    B.valid = false;
    int rc = build_batch(ctx, B, idx, sig, tmax, nd_off, t, y, dy, nf_off, f0, df, common, power,
                         ncurves, stream);
    if (rc != MILS_OK) return rc;
    B.key = key;
    B.valid = true;
  }
  if (use_graph && !B.exec) {
    // capture the launches once per batch layout
    if (!B.cap_stream) {
      he = hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking);
      if (he != hipSuccess) return hip_fail(ctx, he, "capture stream");
    }
    he = hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
      hipError_t le = launch_all(B, B.cap_stream);
      he = hipStreamEndCapture(B.cap_stream, &B.graph);
      if (le != hipSuccess) he = le;
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0);
    if (he != hipSuccess) return hip_fail(ctx, he, "batch graph capture");
  }
  he = use_graph ? hipGraphLaunch(B.exec, stream) : launch_all(B, stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(B.status_host, B.status_dev, sizeof(int32_t) * ncurves,
                        hipMemcpyDeviceToHost, stream);
  if (he == hipSuccess) he = hipStreamSynchronize(stream);
  if (he != hipSuccess) return hip_fail(ctx, he, "batch launch");
  int worst = MILS_OK;
  for (int64_t c = 0; c < ncurves; ++c) {
    int st = B.status_host[c];
    int rc = st == -1 ? MILS_ERR_INVALID_ARG : st == -2 ? MILS_ERR_DEGENERATE : MILS_OK;
    if (status_per_curve) status_per_curve[c] = rc;
    if (rc != MILS_OK && worst == MILS_OK) worst = rc;
  }
  if (worst != MILS_OK) ctx->err = "some series of the batch have invalid or constant data";
  return worst;
}

extern "C" {

int mils_periodogram_batch(mils_context* ctx, int64_t ncurves, const int64_t* nd_off,
                           const double* t, const double* y, const double* dy,
                           const int64_t* nf_off, const double* f0, const double* df,
                           const mils_params* common, double* power, int32_t* status_per_curve,
                           void* hip_stream) {
  return mils_batch_run(ctx, ncurves, nd_off, t, y, dy, nf_off, f0, df, common, power,
                        status_per_curve, hip_stream, true);
}

int mils_batch_tuning(mils_context* ctx, int64_t nf, double eps, int32_t precision, double* sigma,
                      int32_t* tile_max) {
  if (!ctx || !sigma || !tile_max || nf < 1) return MILS_ERR_INVALID_ARG;
  auto it = ctx->tuned.find(std::make_tuple(nf_band(nf), eps, (int)precision));
  if (it == ctx->tuned.end()) return MILS_ERR_INVALID_ARG;
  *sigma = it->second.first;
  *tile_max = it->second.second;
  return MILS_OK;
}

int mils_profile_enable(mils_context* ctx, int enable) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  ctx->prof = enable != 0;
  for (auto& r : ctx->prof_recs) {
    ctx->prof_pool.push_back(std::get<1>(r));
    ctx->prof_pool.push_back(std::get<2>(r));
  }
  ctx->prof_recs.clear();
  return MILS_OK;
}

int mils_context_set_fft2(mils_context* ctx, int enable) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  ctx->fft2 = enable != 0;
  return MILS_OK;
}

int mils_context_set_batch_onchip(mils_context* ctx, int enable) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  ctx->batch_onchip = enable != 0;
  return MILS_OK;
}

int64_t mils_context_batch_onchip(const mils_context* ctx) {
  return ctx ? ctx->last_batch_onchip : 0;
}

int mils_context_set_graphs(mils_context* ctx, int enable) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  ctx->sg.enabled = enable != 0;
  if (!ctx->sg.enabled && ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    release_single_graph(ctx);
    ctx->sg.have_key = false;
  }
  return MILS_OK;
}

int mils_profile_stages(mils_context* ctx, uint32_t mask) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  ctx->prof_mask = mask;
  return MILS_OK;
}

const char* mils_profile_stage_name(int stage) {
  static const char* names[kNumStages] = {"stats",      "bin_sort",       "spread_f",
                                          "spread_2f",  "fft_pass_0",     "fft_pass_1",
                                          "fft_pass_2", "fft_last_power", "lowfreq",
                                          "row_class",  "fft_out"};
  if (stage < 0 || stage >= kNumStages) return "";
  return names[stage];
}

int mils_profile_read(mils_context* ctx, double* ms_total, int64_t* launches) {
  if (!ctx || !ms_total || !launches) return MILS_ERR_INVALID_ARG;
  for (auto& r : ctx->prof_recs) {
    hipEvent_t b = std::get<1>(r), e = std::get<2>(r);
    hipError_t he = hipEventSynchronize(e);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, b, e);
    if (he != hipSuccess) return hip_fail(ctx, he, "profile read");
    ms_total[std::get<0>(r)] += ms;
    launches[std::get<0>(r)] += 1;
    ctx->prof_pool.push_back(b);
    ctx->prof_pool.push_back(e);
  }
  ctx->prof_recs.clear();
  return MILS_OK;
}

int64_t mils_context_illposed(const mils_context* ctx) { return ctx ? ctx->last_illposed : 0; }

int mils_context_status(mils_context* ctx) {
  if (!ctx) return MILS_ERR_INVALID_ARG;
  if (ctx->device < 0) return MILS_OK;
  if (!ctx->have_pending) return MILS_OK;
  static_assert(offsetof(DevStats, nill) == offsetof(DevStats, status) + sizeof(int),
                "status and count are read together");
  hipError_t he = hipMemcpyAsync(ctx->host_status, &ctx->last_stats->status, 2 * sizeof(int),
                                 hipMemcpyDeviceToHost, ctx->last_stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->last_stream);
  if (he != hipSuccess) return hip_fail(ctx, he, "status readback");
  ctx->have_pending = false;
  int st = ctx->host_status[0];
  ctx->last_illposed = st == 0 ? ctx->host_status[1] : 0;
  if (st == -1) return fail(ctx, MILS_ERR_INVALID_ARG, "non-finite input or dy <= 0");
  if (st == -2) return fail(ctx, MILS_ERR_DEGENERATE, "constant data: zero reference chi^2");
  return MILS_OK;
}

}  // extern "C"
