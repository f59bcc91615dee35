// api_internal.h -- entry points shared between the C-ABI runtime (api.cpp)
// and the serving loop (server.cpp).
#pragma once

#include <stdint.h>

#include "../../include/mils.h"

// Batched periodograms; use_graph = false launches directly (no capture).
int mils_batch_run(mils_context* ctx, int64_t ncurves, const int64_t* nd_off, const double* t,
                   const double* y, const double* dy, const int64_t* nf_off, const double* f0,
                   const double* df, const mils_params* common, double* power,
                   int32_t* status_per_curve, void* hip_stream, bool use_graph);

// Validation shared with the public entry points (MILS_OK or the error code).
int mils_check_params(const mils_params* p, int64_t nd);
