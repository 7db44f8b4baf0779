// Host-runtime pieces shared by the kernels of libopmm (fit path and learned seed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/opmm.h"

namespace opmm_rt {

// Device-side saccade record, built by the host from opmm_saccade.
struct SacDev {
    int64_t pos_off;   // first element of the trace in the packed position buffer
    int64_t proj_off;  // first element of the projected trace
    double cphi, sphi; // movement direction
    uint64_t seed;     // candidate-stream key
    int32_t T, C;
    float amp, dur;
    int32_t n_cand, tiles, tile_base, pad;
};

int fail(opmm_ctx* ctx, int code, const std::string& msg);
int hip_fail(opmm_ctx* ctx, hipError_t e, const char* what);
int ctx_device(const opmm_ctx* ctx);

// Validate and upload saccade records, then project every trace on its
// movement direction (ctx-owned scratch, valid until the next call on ctx).
int project_batch(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int S,
                  const SacDev** sacs_dev, const float** proj, hipStream_t st);

}  // namespace opmm_rt
