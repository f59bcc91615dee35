/*
 * mils.h -- C ABI of libmils, an MI355X (gfx950) implementation of the NUFFT
 * Lomb-Scargle periodogram of the nifty-ls paper.
 *
 * Method (nifty-ls paper, Sec. 1): the weighted trigonometric sums of Eq. 1,
 *     C_k + i S_k = sum_j h_j exp(+i 2 pi f_k t_j),   f_k = f0 + k df,
 * are a type-1 (non-uniform to uniform) NUFFT, Eq. 2.  They are evaluated by
 * spreading the points onto an upsampled uniform grid with the "exponential of
 * semicircle" kernel, taking an FFT, and dividing by the kernel's Fourier
 * transform (the diagonal rescaling), with kernel width and grid size chosen
 * from the user tolerance eps.  A periodogram needs the sums at f for the
 * weighted data and the weights, and at 2f for the weights; the power is then
 * assembled per frequency.
 *
 * Conventions shared by every entry point:
 *   - Array arguments marked (device) are device pointers (for example
 *     torch.Tensor.data_ptr() of a CUDA/HIP tensor) owned by the caller; the
 *     library never frees or retains them after the call has completed on its
 *     stream.  Arrays marked (host) are ordinary host memory.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  All device
 *     work of a call is enqueued on that stream.
 *   - Argument checks (null pointers, sizes, ranges, enum values) happen on
 *     the host before any device work; a failed check returns
 *     MILS_ERR_INVALID_ARG and enqueues nothing.  Content checks (non-finite
 *     values, dy <= 0, constant data) happen on the device and are reported
 *     by the synchronous call, or by mils_context_status after an _async call;
 *     the output is then unspecified.
 *   - Point counts nd are 1 <= nd <= 2^30 (per series in the batched call);
 *     larger counts return MILS_ERR_INVALID_ARG before any device work.
 *   - No C++ exception crosses this interface.  Every call returns a status
 *     code; mils_last_error gives a human-readable message for the context.
 *   - One context may be used by one host thread at a time.  Calls on one
 *     context share its workspace, so they must not overlap on the device:
 *     enqueue them on one stream, or use one context per stream.
 */
#ifndef MILS_H
#define MILS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MILS_VERSION 10000 /* 1.0.0 */

/* Status codes. */
enum {
  MILS_OK = 0,
  MILS_ERR_INVALID_ARG = -1, /* bad argument, or invalid values found on device */
  MILS_ERR_DEGENERATE = -2,  /* the data are constant: the reference chi^2 is 0 */
  MILS_ERR_OOM = -3,         /* device allocation failed or the HBM budget is exceeded */
  MILS_ERR_DEVICE = -4,      /* a HIP runtime error; the context is unusable */
  MILS_ERR_UNSUPPORTED = -5, /* eps outside the range of the precision, size too large */
  MILS_ERR_BUSY = -6,        /* server queue full; a captured call that would have to allocate */
  MILS_ERR_CANCELLED = -7,   /* server request cancelled (server shut down) */
  MILS_ERR_TIMEOUT = -8      /* server wait timed out */
};

/* Arithmetic of the spread and FFT.  Rescaling to grid coordinates, the f0
 * phase shift, deconvolution and the power assembly are FP64 in both. */
enum { MILS_FP64 = 0, MILS_FP32 = 1 };

/* Normalisation of the power; chi2_ref is the weighted residual of the model
 * without the sinusoid (the best constant with MILS_FIT_MEAN, else zero) and
 * chi2 the residual of the best fit including the sinusoid at f.
 *   STANDARD (chi2_ref - chi2) / chi2_ref
 *   MODEL    (chi2_ref - chi2) / chi2
 *   LOG      ln(chi2_ref / chi2)
 *   PSD      (chi2_ref - chi2) / 2, with weights 1/dy^2 (1 when dy is NULL) */
enum { MILS_NORM_STANDARD = 0, MILS_NORM_MODEL = 1, MILS_NORM_LOG = 2, MILS_NORM_PSD = 3 };

/* Flags. */
enum {
  MILS_CENTER_DATA = 1, /* subtract the weighted mean of y before the sums */
  MILS_FIT_MEAN = 2,    /* include a constant offset in the fitted model ("floating mean") */
  /* Bitwise-reproducible results (mils_periodogram, mils_periodogram_async):
   * every sum is accumulated in a fixed order -- the points are binned by a
   * sort on (bin, index) instead of the counting sort, and the spread adds
   * them to each grid cell in that order instead of with atomic adds.  Slower
   * (about 3x at N_d = 1e6); other calls reject it with MILS_ERR_UNSUPPORTED.
   * Without it, repeated calls agree to rounding. */
  MILS_DETERMINISTIC = 4
};

typedef struct mils_context mils_context;

/* Periodogram parameters.  The frequency grid is f_k = f0 + k df, k = 0..nf-1
 * (the paper's Eq. 1 writes k = 0..N_f; N_f values are computed here). */
typedef struct {
  double f0;             /* first frequency (cycles per unit of t), finite */
  double df;             /* frequency step, finite and > 0 */
  int64_t nf;            /* number of frequencies, 1 <= nf <= 2^28 */
  double eps;            /* requested NUFFT tolerance: FP64 [1e-14, 1e-2], FP32 [1e-6, 1e-2] */
  int32_t precision;     /* MILS_FP64 or MILS_FP32 */
  int32_t normalization; /* MILS_NORM_* */
  uint32_t flags;        /* MILS_CENTER_DATA | MILS_FIT_MEAN (the default), MILS_DETERMINISTIC */
} mils_params;

/* What the planner chose for a problem (host-only query). */
typedef struct {
  double sigma;        /* upsampling factor n / nf */
  int32_t width;       /* kernel width w in fine-grid cells */
  double beta;         /* exponential-of-semicircle shape parameter */
  int64_t n;           /* fine grid size */
  int32_t npass;       /* FFT passes through HBM (1 = the whole grid stays on chip) */
  int32_t len[4];      /* FFT length of each pass; n = len[0]*...*len[npass-1] */
  int32_t tile;        /* spreading tile, in cells */
  int32_t bin;         /* point-binning granularity, in cells */
  uint64_t workspace_bytes; /* device workspace the call needs */
  int32_t last_rows;   /* rows of length len[npass-1] per workgroup of the last pass */
  int32_t last_lds_bytes; /* dynamic LDS of one workgroup of the last pass */
  int32_t first_cols;  /* columns per workgroup of the first pass (npass > 1) */
  int32_t first_lds_bytes; /* dynamic LDS of one workgroup of the first pass (npass > 1) */
  int32_t big;         /* 1: the passes run as 1024-thread workgroups with up to 160 KB LDS */
  int32_t fft2;        /* 1: two-pass register-tile FFT, n = len[0] * len[1] (single-series calls) */
} mils_plan_desc;

/* Library version (MILS_VERSION of the build). */
int mils_version(void);

/* Static description of a status code. */
const char *mils_status_str(int status);

/* Last error message recorded on the context ("" if none).  ctx may be NULL,
 * which returns the message of the last failed mils_context_create. */
const char *mils_last_error(const mils_context *ctx);

/* Create a context on HIP device `device`.  device = -1 creates a host-only
 * context that can plan and validate but not compute (every compute call
 * returns MILS_ERR_DEVICE).  hbm_budget_bytes bounds the workspace the
 * context may hold (0 = no bound).  *out receives the context. */
int mils_context_create(int device, uint64_t hbm_budget_bytes, mils_context **out);

/* Release the context and its device workspace (synchronises its device). */
int mils_context_destroy(mils_context *ctx);

/* Graph replay of repeated single-series calls (mils_periodogram[_async],
 * mils_trig_sums).  While enabled (the default, unless the environment sets
 * MILS_GRAPH=0), a call whose arguments, workspace and plan repeat those of
 * the context's previous call is captured as a HIP graph, and the graph is
 * replayed for as long as they keep repeating; a call on a stream that is
 * itself being captured launches directly.  On a new key the host waits for
 * the previous replay before releasing its graph.  A context whose calls
 * seldom repeat (a server lane) turns it off: each capture costs more than
 * a replay saves.  Disabling releases the context's graph (after its last
 * replay has finished). */
int mils_context_set_graphs(mils_context *ctx, int enable);

/* Whether the context's single-series calls (mils_periodogram, _async,
 * mils_trig_sums) may use the two-pass register-tile FFT for grids that
 * would otherwise need three or more passes (Sec. 1: the FFT of the
 * upsampled grid; see mils_plan_desc.fft2).  On by default, off when the
 * environment has MILS_FFT2=0 at context creation; the plans of both
 * choices are cached side by side. */
int mils_context_set_fft2(mils_context *ctx, int enable);
/* Batched periodograms (mils_periodogram_batch and the serving loop): a
 * series whose three grids fit one workgroup's LDS (FP64 complex, at most
 * 3072 cells) runs its whole pipeline -- statistics, direct sums near f = 0,
 * spread, transforms, deconvolution and power -- in that workgroup, with no
 * grid in device memory.  Its grids are FP64 in either precision.  On by
 * default; 0 sends every series through the staged kernels. */
int mils_context_set_batch_onchip(mils_context *ctx, int enable);
/* Series of the last batch built on this context that ran on chip. */
int64_t mils_context_batch_onchip(const mils_context *ctx);

/* Fill *out with the plan for a periodogram of nd points with parameters p.
 * Host-only; valid on a host-only context. */
int mils_plan_info(mils_context *ctx, int64_t nd, const mils_params *p, mils_plan_desc *out);

/* The polynomial table the spreading kernel is evaluated from, for the plan of
 * a periodogram with parameters p (host-only; valid on a host-only context).
 * The kernel is the exponential of semicircle phi(z) = exp(beta (sqrt(1 - z^2)
 * - 1)) (Sec. 1 of the paper); at the w cells of a point whose first covered
 * cell lies t in [0, 1) cells past the left end of its support, cell k takes
 * phi((k + t) / (w/2) - 1) ~= sum_j coef[j * kmax + k] u^(ncoef - 1 - j),
 * u = 2t - 1.  coef receives ncoef * kmax doubles (caller-owned, at least
 * 15 * 20); *ncoef, *kmax, *width and *beta describe it.  The device uses
 * the same values (rounded to FP32 for the FP32 precision form). */
int mils_kernel_table(mils_context *ctx, const mils_params *p, double *coef, int32_t *ncoef,
                      int32_t *kmax, int32_t *width, double *beta);

/* The deconvolution factors 1 / phihat(m) of the single-series plan of p
 * (host-only): phihat(m) = w int_0^1 phi(z) cos(pi w m z / n) dz, the
 * Fourier transform of the spreading kernel at mode m of the n-cell grid
 * (Sec. 1, Eq. 2: the diagonal rescaling after the FFT), by the plan's
 * Gauss-Legendre rule (2w + 16 nodes), the rule and sum the device's table
 * uses (there in FP64).  modes: count values in [0, floor(nf / 2)] (host);
 * inv_phihat: count doubles (host, caller-owned); *n_grid: the plan's n. */
int mils_kernel_transform(mils_context *ctx, const mils_params *p, int64_t count,
                          const int64_t *modes, double *inv_phihat, int64_t *n_grid);

/* Check the arguments of mils_periodogram without touching the device;
 * returns MILS_OK or the code mils_periodogram would return before launching. */
int mils_check_periodogram_args(const double *t, const double *y, int64_t nd,
                                const mils_params *p, const double *power);

/*
 * Raw trigonometric sums (Eq. 1 / Eq. 2 of the paper):
 *   out[2k] + i out[2k+1] = sum_j h_j exp(+i 2 pi (f0 + k df) t_j),  k = 0..nf-1,
 * to relative accuracy ~eps (in the norm sum_j |h_j|).  t, h: nd doubles
 * (device); out: 2*nf doubles (device), interleaved re/im.  The time origin is
 * not shifted.  Synchronous: returns after the result is complete.
 */
int mils_trig_sums(mils_context *ctx, const double *t, const double *h, int64_t nd,
                   double f0, double df, int64_t nf, double eps, int32_t precision,
                   double *out, void *hip_stream);

/*
 * Lomb-Scargle periodogram of one series (the method of the paper, Sec. 1):
 * t, y: nd doubles (device); dy: nd doubles (device) or NULL for unit weights;
 * power: p->nf doubles (device), written with the power at f0 + k df.
 * The power is exactly 0 where fl(f0 + fl(k df)) == 0.  Where the fit is
 * ill-posed the power is NaN: the determinant D = CC SS - CS^2 of the 2x2
 * fit (sums normalised by the total weight, after the floating-mean
 * correction) is at most p->eps (below the accuracy of the transformed sums)
 * or at most 1e-12 CC SS -- e.g. evenly spaced t at a multiple of the
 * Nyquist frequency.  mils_context_illposed then counts those frequencies.
 * Synchronous: returns after the result is complete, with the status of the
 * device-side content checks.
 */
int mils_periodogram(mils_context *ctx, const double *t, const double *y, const double *dy,
                     int64_t nd, const mils_params *p, double *power, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation): the
 * same periodogram as mils_periodogram (same arguments, results and
 * statuses; synchronous), computed without any device allocation or free.
 * The plan's tables and the workspace live in a fixed device scratch array
 * of 128 MiB that each GPU the library runs on holds from its first use
 * until the process ends (mils_plan_desc.workspace_bytes plus the plan's
 * tables must fit: about N_f <= 1e6 in FP64, more in FP32; larger calls
 * return MILS_ERR_UNSUPPORTED before any device work).  The context must
 * exist already (its creation allocates its streams, events and status
 * buffer).  Every call on a GPU shares that GPU's scratch, which keeps the
 * last call's plan tables (a call with the same nf, eps and precision skips
 * their upload); nothing in it needs clearing between calls.  Calls that
 * overlap on one GPU race on the scratch: callers serialise them.  Not for
 * a capturing stream (MILS_ERR_UNSUPPORTED).
 */
int mils_periodogram_noalloc(mils_context *ctx, const double *t, const double *y,
                             const double *dy, int64_t nd, const mils_params *p, double *power,
                             void *hip_stream);

/* As mils_periodogram, but returns once the work is enqueued on hip_stream.
 * The device-side status is read by mils_context_status.
 *
 * Graph capture: the call may be captured into the caller's graph on
 * hip_stream once an uncaptured call with the same nf, eps, precision and an
 * nd at least as large has run on the context (its plan tables and workspace
 * then exist).  Otherwise it returns MILS_ERR_BUSY (allocation, upload and
 * the plan's setup kernel cannot run inside a capture); the context stays
 * usable.  The graph holds pointers to the context's workspace and plan:
 * its replays use them as a call would (they must not overlap other calls on
 * the context), and a later workspace growth keeps the captured buffer
 * allocated until mils_context_destroy.  The synchronous calls, the
 * batched, shared-times and direct calls refuse a capturing stream
 * (MILS_ERR_INVALID_ARG for mils_periodogram, MILS_ERR_UNSUPPORTED for the
 * others). */
int mils_periodogram_async(mils_context *ctx, const double *t, const double *y,
                           const double *dy, int64_t nd, const mils_params *p, double *power,
                           void *hip_stream);

/* Wait for the last call enqueued on the context and return its device-side
 * status (MILS_OK, MILS_ERR_INVALID_ARG or MILS_ERR_DEGENERATE). */
int mils_context_status(mils_context *ctx);

/* Number of frequencies whose power was NaN because the fit was ill-posed
 * (see mils_periodogram), for the last single-series call (mils_periodogram,
 * mils_periodogram_async, mils_direct_periodogram) whose status has been read
 * with status MILS_OK; 0 otherwise.  The batched, shared-times and served
 * forms mark such frequencies with NaN without counting them. */
int64_t mils_context_illposed(const mils_context *ctx);

/*
 * Direct evaluation (Sec. 1, Eq. 1 term by term; the brute-force method the
 * paper compares with, Sec. 2.1): the same periodogram as mils_periodogram
 * (same arguments, results and statuses) with every sum accumulated over the
 * points in FP64 for every frequency -- O(nd * nf) work, no transform, no
 * approximation beyond FP64 rounding (p->eps and p->precision are ignored).
 * Per point, the phase at the first of each thread's 12 consecutive
 * frequencies is reduced in double-double and the next ones follow by
 * multiplication with exp(2 pi i df (t - t_min)).  Synchronous.  About 5 s
 * at nd = 1e6, nf = 1.2e7 on one MI355X; a check of the transform path at
 * any size.
 */
int mils_direct_periodogram(mils_context *ctx, const double *t, const double *y,
                            const double *dy, int64_t nd, const mils_params *p, double *power,
                            void *hip_stream);

/* Direct raw sums: out[k] = sum_j h_j exp(+2 pi i (f0 + k df) t_j), k < nf,
 * as mils_trig_sums but evaluated term by term in FP64 (no time shift).
 * out_re_im: 2*nf doubles (device).  Synchronous. */
int mils_direct_trig_sums(mils_context *ctx, const double *t, const double *h, int64_t nd,
                          double f0, double df, int64_t nf, double *out_re_im,
                          void *hip_stream);

/*
 * Periodograms of nseries series observed at the same times (the batched
 * mode for series sharing their observation times, Sec. 2.1 of the paper).
 * t: nd doubles; y: nseries x nd doubles, series i at y + i*nd; power:
 * nseries x p->nf doubles, series i at power + i*p->nf (all device arrays).
 * dy is NULL (unit weights), one array of nd doubles shared by every series
 * (dy_stride = 0), or nseries x nd doubles (dy_stride = nd).  Every series
 * gets exactly the result of mils_periodogram on its own (t, y_i, dy_i).
 * With shared weights (dy NULL or dy_stride = 0) the weight-only sums
 * B = sum w^ e^{iwt} at f and B2 at 2f are the same for every series: they
 * run once, and each series adds its own A = sum w^ y~ e^{iwt} through one
 * grid; series go in groups of three, whose grids share the FFT launches
 * and one last pass that reads B and B2 once for the group.  With
 * per-series weights every series runs the whole path.  Everything runs on
 * hip_stream (and the context's second stream); the workspace holds the
 * single-series layout plus 32 bytes per frequency.  Many short series are
 * better served by mils_periodogram_batch.  status_per_series (host, nullable, nseries int32)
 * receives each series' status.  Synchronous; returns MILS_OK when every
 * series succeeded, else the status of the first that did not.  Errors:
 * MILS_ERR_INVALID_ARG (null pointers, nseries outside [1, 2^24], dy_stride
 * neither 0 nor nd, or any of mils_periodogram's argument errors).
 */
int mils_periodogram_shared_t(mils_context *ctx, const double *t, const double *y,
                              const double *dy, int64_t dy_stride, int64_t nd, int64_t nseries,
                              const mils_params *p, double *power, int32_t *status_per_series,
                              void *hip_stream);

/*
 * Batched periodograms: ncurves independent series in CSR layout.  Curve c
 * has points nd_off[c] .. nd_off[c+1]-1 of t, y, dy and writes power
 * nf_off[c] .. nf_off[c+1]-1 at frequencies f0[c] + k df[c].  nd_off, nf_off
 * (ncurves+1 int64), f0, df (ncurves doubles) are HOST arrays; t, y, dy, power
 * are device arrays (dy may be NULL).  common supplies eps, precision,
 * normalization and flags (its f0, df, nf are ignored).  status_per_curve
 * (host, nullable, ncurves int32) receives each curve's device-side status.
 * Synchronous.  The series run together, phase by phase (per-series
 * statistics, binning and low-frequency sums; both spreads; each FFT pass;
 * the last pass with power), each phase one launch over the tiles of every
 * series; the launches of a batch layout are captured once in a HIP graph
 * and replayed by later calls with the same layout and pointers.  Every
 * series has its own device workspace (its three grids, 48 bytes per grid
 * cell in FP64 and 24 in FP32, plus binning buffers); a batch that needs more
 * than the context's budget allows (or 24 GiB) runs in chunks.
 */
int mils_periodogram_batch(mils_context *ctx, int64_t ncurves, const int64_t *nd_off,
                           const double *t, const double *y, const double *dy,
                           const int64_t *nf_off, const double *f0, const double *df,
                           const mils_params *common, double *power,
                           int32_t *status_per_curve, void *hip_stream);

/* The batch autotuner's decision for series of nf frequencies at (eps,
 * precision): the first mils_periodogram_batch call on a context times, for
 * every half-octave band of N_f holding at least 16 of its series, a sample of
 * them under a few upsampling factors sigma (0 stands for the planner's own
 * choice; larger sigma: a wider grid with a narrower kernel) and largest
 * spreading tiles, and keeps the fastest for later batches of the context
 * (Sec. 1 of the paper sets the grid and the kernel width from eps; which
 * admissible pair is fastest depends on the size).  Returns MILS_OK with
 * *sigma and *tile_max set, or MILS_ERR_INVALID_ARG when the band has no
 * decision.  Setting MILS_AUTOTUNE=0 in the environment turns the tuner off.
 * With MILS_TUNE_CACHE naming a file when a context is created, the context
 * reads the decisions recorded there for its device (architecture, CU count
 * and memory size), and the tuner appends every new decision to it, so that
 * later processes skip the tuning.
 * Diagnostics: MILS_LOG_LEVEL (read when a context is created) = 1 writes
 * every error to stderr, 2 also each plan built, each workspace growth and
 * each tuning decision; 0 (the default) writes nothing. */
int mils_batch_tuning(mils_context *ctx, int64_t nf, double eps, int32_t precision,
                      double *sigma, int32_t *tile_max);

/*
 * Serving loop: requests of mixed sizes and precisions are submitted from host
 * memory, admitted while the device memory they need fits the HBM budget,
 * packed as they arrive into batches that run concurrently on `lanes`
 * streams (a lane that frees up takes everything that has arrived: continuous
 * batching), and read back to host memory.  Requests whose frequency count
 * exceeds the batch limit run through the single-series path on a lane.
 * Thread-safe: any host thread may submit, poll, wait and take.
 *
 * Plan classes: a request is computed on its frequency grid f0 + k df
 * extended to the next class size (nf rounded up to ceil(64 * 2^(j/16)),
 * j >= 0: at most 4.5% more frequencies), and its first nf values are
 * returned.  Requests of any size thus share the plans of a bounded set of
 * classes; mils_server_warm builds them before traffic arrives.  The values
 * agree with a call at nf within the tolerance eps of the request.
 */
typedef struct mils_server mils_server;

typedef struct {
  uint64_t hbm_budget_bytes; /* device bytes for requests in flight (0 = 8 GiB) */
  int32_t lanes;             /* concurrent batches / streams (0 = 2) */
  int32_t max_batch;         /* requests per batch (0 = 4096) */
  int32_t queue_capacity;    /* pending requests before submit returns MILS_ERR_BUSY (0 = 65536) */
  int32_t tick_us;           /* how long an idle lane waits for more arrivals (0 = 200) */
} mils_server_config;

typedef struct {
  const double *t;    /* host, nd values; copied by submit */
  const double *y;    /* host, nd values; copied by submit */
  const double *dy;   /* host, nd values or NULL; copied by submit */
  int64_t nd;
  mils_params params; /* grid, tolerance, precision, normalisation, flags */
} mils_request;

enum { MILS_REQ_PENDING = 0, MILS_REQ_RUNNING = 1, MILS_REQ_DONE = 2 };

typedef struct {
  double submit_s;    /* seconds since the server started */
  double start_s;     /* when its batch was launched */
  double done_s;      /* when its result reached host memory */
  int32_t status;     /* MILS_OK or the request's error */
  int32_t batch_size; /* requests in its batch */
} mils_request_stats;

typedef struct {
  uint64_t submitted, completed, rejected, batches;
  uint64_t inflight_bytes, peak_inflight_bytes;
  double latency_p50_ms, latency_p99_ms, latency_max_ms; /* submit -> result on host */
  double sums_per_s;  /* sum of nd*nf over completed requests / (last done - first submit) */
  double mean_batch;  /* requests per batch */
  uint64_t failed;     /* completed requests whose status is not MILS_OK */
  uint64_t dead_lanes; /* lanes stopped by a device error (their context is unusable) */
  uint64_t plans_built; /* plans built by the lanes (warm-up included) */
  double plan_build_ms; /* host time the lanes spent building them */
} mils_server_counters;

/* Create a server on HIP device `device` (cfg may be NULL for defaults). */
int mils_server_create(int device, const mils_server_config *cfg, mils_server **out);
/* Copy the request's arrays and queue it; *ticket identifies it.  Returns
 * MILS_ERR_BUSY when the queue is full, MILS_ERR_OOM when the request alone
 * exceeds the budget, MILS_ERR_INVALID_ARG for bad arguments. */
int mils_server_submit(mils_server *srv, const mils_request *req, uint64_t *ticket);
/* Build, on every lane, the plans of every class up to nf_max for requests
 * with the precision, tolerance, normalisation and flags of *params (its
 * grid fields are ignored): each lane runs one short synthetic series per
 * class.  Blocks until every lane is done; requests submitted meanwhile wait
 * behind the warm-up.  Returns the first error a lane met. */
int mils_server_warm(mils_server *srv, const mils_params *params, int64_t nf_max);
/* *state = MILS_REQ_PENDING / RUNNING / DONE. */
int mils_server_poll(mils_server *srv, uint64_t ticket, int32_t *state);
/* Wait until the request is done (timeout_us < 0: forever); MILS_ERR_TIMEOUT otherwise. */
int mils_server_wait(mils_server *srv, uint64_t ticket, int64_t timeout_us);
/* Copy a done request's power (params.nf doubles, host) and statistics (st
 * may be NULL; power may be NULL to discard), release the ticket, and return
 * the request's status. */
int mils_server_take(mils_server *srv, uint64_t ticket, double *power, mils_request_stats *st);
int mils_server_stats(mils_server *srv, mils_server_counters *out);
/* Message of the first device error that stopped a lane ("" if none).  Once
 * every lane has stopped, pending requests complete with MILS_ERR_DEVICE and
 * submit returns MILS_ERR_DEVICE.  For tests of this handling, the
 * environment variable MILS_SERVER_FAIL_AFTER=N (read by mils_server_create)
 * makes each lane report a device error once it has run N batches, without
 * touching the device. */
const char *mils_server_last_error(mils_server *srv);
/* Stop the lanes; requests not yet done are cancelled (their tickets become
 * invalid).  Waits for batches already on the device. */
int mils_server_destroy(mils_server *srv);

/*
 * Per-stage timing of the single-series path (measurement support).  While
 * enabled, every call records a pair of HIP events around each stage of the
 * path on the stream that runs it.  Stages: 0 statistics, 1 binning / sort,
 * 2 spread (geometry f), 3 spread (geometry 2f), 4-6 FFT passes through HBM
 * (first pass pruned), 7 last FFT pass fused with deconvolution, crop and
 * power, 8 direct sums near f = 0, 9 row classes of both geometries and
 * 10 the transpose into frequency order (9 and 10: two-pass register-tile
 * plans, whose first pass, stage 4, transforms all three grids in one
 * launch).  A periodogram runs stage 3, stage 8 and (multi-pass plans) the
 * first pass of the 2f grid on a second stream of the context, beside the f
 * geometry (stage 4 then counts two launches per call, and stages that
 * overlap share the GPU).  mils_profile_enable(ctx, 1) clears the
 * accumulators.
 * mils_profile_read waits for the recorded events and adds, per stage, the
 * total elapsed milliseconds and the number of timed launches to ms_total[s]
 * and launches[s] (host arrays of MILS_NUM_STAGES entries), then clears them.
 */
enum { MILS_NUM_STAGES = 11 };
int mils_profile_enable(mils_context *ctx, int enable);
/* Stages timed while profiling is enabled: bit s for stage s (default: all).
 * Each timed stage adds two events per call; timing one stage leaves the rest
 * of the call as it runs unprofiled. */
int mils_profile_stages(mils_context *ctx, uint32_t mask);
const char *mils_profile_stage_name(int stage);
int mils_profile_read(mils_context *ctx, double *ms_total, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* MILS_H */
