// Host-runtime pieces shared by the kernels of libopmm (fit path and learned seed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

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
    int32_t n_cand, tiles, tile_base;
    int32_t slot;      // index of this saccade's search state (box, status, keys)
    int32_t round;     // current round when a launch serves saccades at different rounds
    int32_t model;     // 18 or 9 (tied K_SE/K_LT, neural parameters fixed)
};

// Calls on one object (context, surrogate, plan) share that object's device scratch, so a call on
// one stream must not start on the scratch while an earlier call on another stream still uses it.
// While every call comes on one stream, stream order does it and nothing is added.  At the first
// call on a second stream the host waits once for the device to drain; from then on every call
// records `ev` on its stream when it has queued its work, and a call on a stream other than the
// last call's first makes its stream wait for that event (on the device).  A call queued under
// stream capture takes no part: inside a graph the caller orders its work.
struct StreamOrder {
    hipEvent_t ev = nullptr;      // created with the object, timing disabled
    hipStream_t last = nullptr;   // stream of the last call
    bool seen = false;            // a call has been made
    bool multi = false;           // calls have come on more than one stream
    bool recorded = false;        // ev holds the end of the last call
};
hipError_t order_init(StreamOrder& o);
void order_release(StreamOrder& o);
// Host-side wait for the last call, for a synchronous call about to use stream `st`.
hipError_t order_host_wait(const StreamOrder& o, hipStream_t st);

// Per-kernel timing of uncaptured fit launches (opmm_kernel_timing_*).  Event pairs come from a pool
// made when timing is switched on, so a timed call creates nothing; a launch that finds the pool
// empty (more than kPairs launches between two reads) is not timed.
struct KernelTimer {
    static constexpr int kPairs = 1024;
    bool on = false;
    std::vector<hipEvent_t> ev;            // 2 * kPairs, made by reserve()
    std::vector<int> free_pairs;           // pairs not waiting to be read
    std::vector<std::pair<int, int>> pending;  // (kernel, pair) recorded, not yet read
    double ms[OPMM_KERNEL_KINDS] = {};
    int64_t n[OPMM_KERNEL_KINDS] = {};

    hipError_t reserve()
    {
        if (!ev.empty()) return hipSuccess;
        ev.assign(2 * kPairs, nullptr);
        for (auto& e : ev) {
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) {
                release();
                return err;
            }
        }
        for (int i = kPairs - 1; i >= 0; --i) free_pairs.push_back(i);
        return hipSuccess;
    }
    int begin(hipStream_t st)
    {
        if (free_pairs.empty()) return -1;
        int i = free_pairs.back();
        if (hipEventRecord(ev[2 * i], st) != hipSuccess) return -1;
        free_pairs.pop_back();
        return i;
    }
    void end(int kernel, int i, hipStream_t st)
    {
        if (i < 0) return;
        if (hipEventRecord(ev[2 * i + 1], st) == hipSuccess) pending.emplace_back(kernel, i);
        else free_pairs.push_back(i);
    }
    // Wait for every recorded pair and add its time to its kernel's total.
    hipError_t collect()
    {
        for (auto& kp : pending) {
            int i = kp.second;
            float t = 0.f;
            hipError_t err = hipEventSynchronize(ev[2 * i + 1]);
            if (err == hipSuccess) err = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
            if (err != hipSuccess) return err;
            ms[kp.first] += t;
            n[kp.first] += 1;
            free_pairs.push_back(i);
        }
        pending.clear();
        return hipSuccess;
    }
    void release()
    {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        ev.clear();
        free_pairs.clear();
        pending.clear();
        on = false;
    }
};

// Scope of one call's use of an object's scratch on `st`: orders it after the previous call in the
// constructor, records its end in the destructor.
class Ordered {
  public:
    Ordered(StreamOrder& o, hipStream_t st);
    ~Ordered();
    Ordered(const Ordered&) = delete;
    Ordered& operator=(const Ordered&) = delete;
    hipError_t error() const { return err_; }

  private:
    StreamOrder& o_;
    hipStream_t st_;
    bool skip_ = false;
    hipError_t err_ = hipSuccess;
};
StreamOrder& ctx_order(opmm_ctx* ctx);

int fail(opmm_ctx* ctx, int code, const std::string& msg);
int hip_fail(opmm_ctx* ctx, hipError_t e, const char* what);
int ctx_device(const opmm_ctx* ctx);
int ctx_cu_count(const opmm_ctx* ctx);  // compute units of the context's device

// Validate and upload saccade records, then project every trace on its
// movement direction (ctx-owned scratch, valid until the next call on ctx).
int project_batch(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int S,
                  const SacDev** sacs_dev, const float** proj, hipStream_t st);

// A fit in two halves, for callers that queue work of their own on the batch between the upload
// and the search (the learned seed reads the projection).  fit_stage validates like opmm_fit,
// uploads the records into the context's fit scratch and queues the projection; *sacs_dev and
// *proj stay valid until the next fit on ctx.  fit_launch queues the search of that upload.
struct FitStage {
    int shape;
    int64_t total_T;
    int tiles;
};
int fit_stage(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int S,
              const opmm_fit_params* prm, float* opc_out, float* rmse_out, FitStage* fs, const SacDev** sacs_dev,
              const float** proj, hipStream_t st);
int fit_launch(opmm_ctx* ctx, const float* pos, int S, const FitStage& fs, const opmm_fit_params* prm,
               const float* seed_opc, float* opc_out, float* rmse_out, float* mae_out, int32_t* status_out,
               uint64_t* round_keys, hipStream_t st);

// Device array [S] of the last project_batch: the batch's indices sorted by T, longest first
// (ties in batch order).
const int* batch_order(const opmm_ctx* ctx);

// As project_batch, also returning the orthogonal energies and status words
// (both indexed by SacDev::slot = position in the batch).
int project_batch_full(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int S,
                       const SacDev** sacs_dev, const float** proj, const double** qorth, const int32_t** status,
                       hipStream_t st);

// Grow the learned seed's activation buffers to `batch` rows now.
int surrogate_reserve(opmm_surrogate* sg, int batch);
// Learned OPC [n][18] of n device records whose traces are already projected (proj at each
// record's proj_off): features, network, de-normalisation into the search box.
int surrogate_predict_projected(opmm_surrogate* sg, int n, const SacDev* sacs, const float* proj, float dt_ms,
                                float box_frac, float* opc_out, hipStream_t st);

int validate_saccade(opmm_ctx* ctx, const opmm_saccade& s, int64_t pos_len, int i);
SacDev make_record(const opmm_saccade& s, int n_cand_default);

// Search state of a set of slots (one saccade each), indexed by SacDev::slot.
struct SlotState {
    float *centre, *hw, *lo, *hi;  // [slots][18]
    int32_t* status;               // [slots]
    uint64_t* keys;                // [slots]: argmin key of the slot's current round
    float* proj;                   // projected traces (SacDev::proj_off)
    double* qorth;                 // [slots]
};

// Launchers over a compact device list of n records (each names its slot).
hipError_t launch_prep(const SacDev* sacs, int n, const float* pos, const SlotState& ss, hipStream_t st);
hipError_t launch_init(const SacDev* sacs, int n, float box_frac, float w_init_frac, const float* seed_opc,
                       const SlotState& ss, hipStream_t st);
hipError_t launch_reset_keys(const SacDev* sacs, int n, const SlotState& ss, hipStream_t st);
// one round for every listed saccade at its own SacDev::round (records carry tile_base/tiles)
hipError_t launch_round(int shape, const SacDev* sacs, int n, int tiles_total, float dt, const SlotState& ss,
                        hipStream_t st);
hipError_t launch_refine(const SacDev* sacs, int n, float shrink, const SlotState& ss, hipStream_t st);
hipError_t launch_report(const SacDev* sacs, int n, const float* pos, float dt, const SlotState& ss, float* opc_out,
                         float* rmse_out, float* mae_out, int32_t* status_out, hipStream_t st);
int shape_tile(int shape);
int default_shape(const opmm_ctx* ctx);
// default_shape, or a smaller-tile shape when a saccade has fewer candidates than its tile
int shape_for_candidates(const opmm_ctx* ctx, int64_t n_cand);
// `base`, or a smaller-tile shape when a launch of `tiles` tiles of `base` would leave CUs idle
int launch_shape(const opmm_ctx* ctx, int base, int64_t tiles);

// Gradient polish of n listed saccades (T <= max_T) on ctx's device: opc [n][18] in/out,
// rmse/mae [n] out, status indexed by SacDev::slot.
hipError_t launch_polish(const opmm_ctx* ctx, const SacDev* sacs, int n, int max_T, const float* pos,
                         const int32_t* status, int model, const opmm_polish_params& prm, float* opc, float* rmse,
                         float* mae, hipStream_t st);

}  // namespace opmm_rt
