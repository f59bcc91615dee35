// api_internal.h -- entry points shared between the C-ABI runtime (api.cpp)
// and the serving loop (server.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mils.h"

// Batched periodograms; use_graph = false launches directly (no capture).
int mils_batch_run(mils_context* ctx, int64_t ncurves, const int64_t* nd_off, const double* t,
                   const double* y, const double* dy, const int64_t* nf_off, const double* f0,
                   const double* df, const mils_params* common, double* power,
                   int32_t* status_per_curve, void* hip_stream, bool use_graph);

// Plans the context has built and the host seconds spent building them
// (table generation, upload and the kernel-transform launch).
void mils_context_plan_counters(const mils_context* ctx, int64_t* built, double* seconds);

// Validation shared with the public entry points (MILS_OK or the error code).
int mils_check_params(const mils_params* p, int64_t nd);

namespace mils {
// Device scratch of mils_periodogram_noalloc (noalloc.hip): kNoAllocBytes per
// GPU, for up to kNoAllocDevices GPUs.  noalloc_scratch returns the device
// address of the array on `device` (looked up once per device, with that
// device current), or NULL with *err set.
constexpr size_t kNoAllocBytes = (size_t)128 << 20;
constexpr int kNoAllocDevices = 64;
void* noalloc_scratch(int device, hipError_t* err);
}  // namespace mils
