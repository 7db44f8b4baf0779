// libopmm: continuous-batching estimation server.
//
// Saccades arrive one by one (a streamed recording, the paper's real-time goal
// of Section 5: estimation in the time it takes to record).  Each admitted
// request owns a device slot -- its trace, projection, search box, status and
// round key stay resident in HBM -- and every step advances *all* occupied
// slots by one search round in a single launch, whatever round each is at.
// Requests that arrive while others are on the GPU are admitted as slots free
// up (the slot count is set by an HBM budget), so their work overlaps on the
// device with requests admitted earlier.  A slot's arithmetic depends only on
// its own request (candidate stream keyed by the request's seed), so a result
// is the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/opmm.h"
#include "runtime.hpp"

using opmm_rt::SacDev;
using opmm_rt::SlotState;

namespace {

constexpr int P = OPMM_P;
constexpr int kMaxAdmitPerStep = 4096;
constexpr int kMaxRoundsPerStep = 64;
constexpr int kPolishBatches = 3;

struct Request {
    int64_t id;
    opmm_saccade sac;
    std::vector<float> trace;
    double t_arrival;
};

enum Phase { PH_FIRST = 0, PH_FALLBACK = 1 };

struct Slot {
    bool busy = false;
    int64_t id = 0;
    opmm_saccade sac{};
    double t_arrival = 0;
    int phase = PH_FIRST;
    int round = 0;
    int rounds = 0;
    int n_cand = 0;
    bool has_prev = false;  // seeded result kept while the fallback runs
    float prev_opc[P];
    float prev_rmse = 0, prev_mae = 0;
    int32_t prev_status = 0;
};

struct PolishBatch {
    hipStream_t stream = nullptr;  // batches run concurrently, each on its own stream
    hipEvent_t done = nullptr;
    SacDev* d_list = nullptr;  // [slots]
    float* d_out = nullptr;    // [slots][18 + 2]
    int32_t* d_st = nullptr;   // [slots]
    float* h_out = nullptr;
    int32_t* h_st = nullptr;
    std::vector<int> fin;      // slots of the batch
};

struct Done {
    int64_t id;
    float opc[P];
    float rmse, mae;
    int32_t status;
    double t_arrival, t_done;
};

// Admitted traces, staged contiguously (one copy per step), into their slots' rows of pos.
// Record i's trace is T * C <= stride floats (T <= max_T was checked at submission).
__global__ void scatter_traces_kernel(int n, const SacDev* __restrict__ list, const float* __restrict__ staged,
                                      int stride, float* __restrict__ pos)
{
    const int i = blockIdx.x;
    if (i >= n) return;
    const SacDev d = list[i];
    const int len = d.T * d.C;
    for (int k = threadIdx.x; k < len; k += blockDim.x) pos[d.pos_off + k] = staged[(size_t)i * stride + k];
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct opmm_server {
    opmm_ctx* ctx = nullptr;
    opmm_surrogate* sg = nullptr;
    opmm_serve_params prm{};
    int device = 0;
    int slots = 0;
    int max_T = 0;
    int shape = 0;
    int tile = 1;
    int max_admit = 1;  // requests admitted per step (bounds a step's work and its scratch)
    hipStream_t stream = nullptr;
    // device
    float* d_pos = nullptr;   // [slots][max_T * 2]
    float* d_box = nullptr;   // 4 x [slots][18]
    int32_t* d_status = nullptr;
    uint64_t* d_keys = nullptr;
    float* d_proj = nullptr;  // [slots][max_T]
    double* d_qorth = nullptr;
    SacDev* d_list = nullptr;  // [slots] active / admitted / finished lists
    float* d_seed = nullptr;   // [slots][18]
    float* d_out = nullptr;    // [slots][18 + 2] opc, rmse, mae
    int32_t* d_st = nullptr;   // [slots]
    float* d_adm_trace = nullptr;  // [max_admit][max_T * 2]: staged admitted traces
    // Polish of finished searches on streams of their own, so it overlaps the following steps'
    // rounds.  Up to kPolishBatches batches are in flight, each on its own stream with its
    // records, outputs (the d_out layout) and status, taken in order when their event completes.
    hipEvent_t ev_fin = nullptr;
    PolishBatch pb[kPolishBatches];
    int pb_head = 0, pb_count = 0;  // ring of in-flight batches, oldest at pb_head
    // pinned host staging
    SacDev* h_list = nullptr;  // 4 x [slots]: restart, admitted, active and finished lists of a step
    SacDev* h_more = nullptr;  // [rounds_per_step - 1][cus]: active lists of a step's further rounds
    int cus = 1;               // compute units of the device
    float* h_out = nullptr;
    int32_t* h_st = nullptr;
    float* h_adm_trace = nullptr;  // [max_admit][max_T * 2]: traces admitted in one step
    // host state
    std::vector<Slot> slot;
    std::vector<int> free_slots;
    std::vector<int> reinit;  // slots restarting with the plain search
    std::deque<Request> pending;
    std::deque<Done> done;
    int64_t next_id = 0;
    int64_t n_admitted = 0, n_completed = 0, n_fallback = 0, n_steps = 0;
    SlotState ss{};
};

namespace {

int sfail(opmm_server* sv, int code, const std::string& m) { return opmm_rt::fail(sv->ctx, code, m); }

#define SV_HIP(call)                                                        \
    do {                                                                    \
        hipError_t _e = (call);                                             \
        if (_e != hipSuccess) return opmm_rt::hip_fail(sv->ctx, _e, #call); \
    } while (0)

const opmm_fit_params& phase_params(const opmm_server* sv, int phase)
{
    return (phase == PH_FIRST && sv->sg) ? sv->prm.seeded : sv->prm.plain;
}

opmm_saccade slot_saccade(const opmm_server* sv, int k)
{
    opmm_saccade s = sv->slot[k].sac;
    s.pos_offset = (int64_t)k * sv->max_T * 2;
    s.n_cand = sv->slot[k].n_cand;
    return s;
}

SacDev slot_record(const opmm_server* sv, int k)
{
    SacDev d = opmm_rt::make_record(slot_saccade(sv, k), sv->slot[k].n_cand);
    d.proj_off = (int64_t)k * sv->max_T;
    d.slot = k;
    d.round = sv->slot[k].round;
    d.tiles = (d.n_cand + sv->tile - 1) / sv->tile;
    d.model = phase_params(sv, sv->slot[k].phase).model;
    return d;
}



}  // namespace

extern "C" {

void opmm_serve_params_default(opmm_serve_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->max_slots = 4096;
    p->hbm_budget_bytes = (size_t)1 << 30;
    p->max_T = 160;
    opmm_fit_params_default(&p->plain);
    p->plain.n_cand = 4096;
    p->plain.n_rounds = 10;
    opmm_fit_params_default(&p->seeded);
    p->seeded.n_cand = 1024;
    p->seeded.n_rounds = 3;
    p->seeded.w_init_frac = 0.25f;
    p->fallback_rmse = 0.075f;
    p->rounds_per_step = 16;
}

double opmm_server_now(void) { return now_s(); }

int opmm_server_create(opmm_ctx* ctx, opmm_surrogate* sg, const opmm_serve_params* prm, opmm_server** out)
{
    if (!ctx || !prm || !out) return OPMM_EINVAL;
    *out = nullptr;
    if (prm->max_slots < 1 || prm->max_T < 1 || prm->max_T > OPMM_MAX_T)
        return opmm_rt::fail(ctx, OPMM_EINVAL, "max_slots >= 1 and max_T in 1..OPMM_MAX_T required");
    for (const opmm_fit_params* fp : {&prm->plain, &prm->seeded}) {
        if (fp->n_cand < 1 || fp->n_rounds < 1 || !(fp->box_frac > 0 && fp->box_frac < 1) ||
            !(fp->shrink > 0 && fp->shrink <= 1) || !(fp->dt_ms > 0 && fp->dt_ms <= 1) ||
            !(fp->w_init_frac >= 0 && fp->w_init_frac <= 1))
            return opmm_rt::fail(ctx, OPMM_EINVAL, "bad search parameters");
    }
    if (prm->plain.dt_ms != prm->seeded.dt_ms || prm->plain.box_frac != prm->seeded.box_frac ||
        prm->plain.shrink != prm->seeded.shrink || (prm->plain.model != 18 && prm->plain.model != 9) ||
        prm->plain.model != prm->seeded.model)
        return opmm_rt::fail(ctx, OPMM_EINVAL, "plain and seeded searches must share dt_ms, box_frac, shrink and model");
    if (prm->polish_iter < 0 || prm->polish_iter > 100)
        return opmm_rt::fail(ctx, OPMM_EINVAL, "polish_iter must be in 0..100");
    if (prm->plain.screen_rounds != 0 || prm->seeded.screen_rounds != 0)
        return opmm_rt::fail(ctx, OPMM_EINVAL, "the server runs every round in FP64 (screen_rounds = 0)");
    if (prm->rounds_per_step < 1 || prm->rounds_per_step > kMaxRoundsPerStep)
        return opmm_rt::fail(ctx, OPMM_EINVAL, "rounds_per_step must be in 1..64");
    // slots admitted by memory: what one resident request costs on the device
    const size_t per_slot = sizeof(float) * (3 * (size_t)prm->max_T + 4 * P + P + P + 2) + sizeof(int32_t) * 2 +
                            sizeof(uint64_t) + sizeof(double) + sizeof(SacDev) +
                            (prm->polish_iter > 0
                                 ? kPolishBatches * (sizeof(SacDev) + sizeof(float) * (P + 2) + sizeof(int32_t))
                                 : 0);
    const int64_t by_budget = (int64_t)(prm->hbm_budget_bytes / per_slot);
    const int slots = (int)std::min<int64_t>(prm->max_slots, by_budget);
    if (slots < 1) return opmm_rt::fail(ctx, OPMM_ENOMEM, "HBM budget below one slot");
    opmm_server* sv = new (std::nothrow) opmm_server();
    if (!sv) return OPMM_ENOMEM;
    sv->ctx = ctx;
    sv->sg = sg;
    sv->prm = *prm;
    sv->device = opmm_rt::ctx_device(ctx);
    sv->slots = slots;
    sv->max_T = prm->max_T;
    sv->shape = opmm_rt::shape_for_candidates(
        ctx, sg ? std::min(prm->seeded.n_cand, prm->plain.n_cand) : prm->plain.n_cand);
    sv->tile = opmm_rt::shape_tile(sv->shape);
    int rc = OPMM_OK;
    if (hipSetDevice(sv->device) != hipSuccess || hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess)
        rc = OPMM_EDEVICE;
    auto dm = [&](void** p, size_t b) { if (rc == OPMM_OK && hipMalloc(p, b) != hipSuccess) rc = OPMM_ENOMEM; };
    auto hm = [&](void** p, size_t b) { if (rc == OPMM_OK && hipHostMalloc(p, b, 0) != hipSuccess) rc = OPMM_ENOMEM; };
    dm((void**)&sv->d_pos, sizeof(float) * (size_t)slots * sv->max_T * 2);
    dm((void**)&sv->d_box, sizeof(float) * 4 * P * (size_t)slots);
    dm((void**)&sv->d_status, sizeof(int32_t) * slots);
    dm((void**)&sv->d_keys, sizeof(uint64_t) * slots);
    dm((void**)&sv->d_proj, sizeof(float) * (size_t)slots * sv->max_T);
    dm((void**)&sv->d_qorth, sizeof(double) * slots);
    dm((void**)&sv->d_list, sizeof(SacDev) * slots);
    dm((void**)&sv->d_seed, sizeof(float) * P * (size_t)slots);
    dm((void**)&sv->d_out, sizeof(float) * (P + 2) * (size_t)slots);
    dm((void**)&sv->d_st, sizeof(int32_t) * slots);
    hm((void**)&sv->h_list, sizeof(SacDev) * 4 * (size_t)slots);
    sv->cus = opmm_rt::ctx_cu_count(ctx);
    if (prm->rounds_per_step > 1)
        hm((void**)&sv->h_more, sizeof(SacDev) * (size_t)(prm->rounds_per_step - 1) * sv->cus);
    hm((void**)&sv->h_out, sizeof(float) * (P + 2) * (size_t)slots);
    hm((void**)&sv->h_st, sizeof(int32_t) * slots);
    // a step admits at most max_admit requests; size the per-call scratch for that now, so no step
    // reallocates (which would synchronise the device) when a burst arrives
    sv->max_admit = std::min(slots, kMaxAdmitPerStep);
    hm((void**)&sv->h_adm_trace, sizeof(float) * (size_t)sv->max_admit * sv->max_T * 2);
    dm((void**)&sv->d_adm_trace, sizeof(float) * (size_t)sv->max_admit * sv->max_T * 2);
    if (prm->polish_iter > 0) {
        if (rc == OPMM_OK && hipEventCreateWithFlags(&sv->ev_fin, hipEventDisableTiming) != hipSuccess)
            rc = OPMM_EDEVICE;
        for (PolishBatch& b : sv->pb) {
            if (rc == OPMM_OK && (hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess ||
                                  hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess))
                rc = OPMM_EDEVICE;
            dm((void**)&b.d_list, sizeof(SacDev) * slots);
            dm((void**)&b.d_out, sizeof(float) * (P + 2) * (size_t)slots);
            dm((void**)&b.d_st, sizeof(int32_t) * slots);
            hm((void**)&b.h_out, sizeof(float) * (P + 2) * (size_t)slots);
            hm((void**)&b.h_st, sizeof(int32_t) * slots);
        }
    }
    if (rc == OPMM_OK && sg) rc = opmm_rt::surrogate_reserve(sg, sv->max_admit);
    if (rc != OPMM_OK) {
        opmm_server_destroy(sv);
        return opmm_rt::fail(ctx, rc, "server allocation failed");
    }
    sv->ss.centre = sv->d_box;
    sv->ss.hw = sv->d_box + (size_t)P * slots;
    sv->ss.lo = sv->d_box + 2 * (size_t)P * slots;
    sv->ss.hi = sv->d_box + 3 * (size_t)P * slots;
    sv->ss.status = sv->d_status;
    sv->ss.keys = sv->d_keys;
    sv->ss.proj = sv->d_proj;
    sv->ss.qorth = sv->d_qorth;
    sv->slot.resize(slots);
    for (int k = slots - 1; k >= 0; --k) sv->free_slots.push_back(k);
    *out = sv;
    return OPMM_OK;
}

int opmm_server_destroy(opmm_server* sv)
{
    if (!sv) return OPMM_OK;
    (void)hipSetDevice(sv->device);
    if (sv->stream) (void)hipStreamSynchronize(sv->stream);
    for (PolishBatch& b : sv->pb)
        if (b.stream) (void)hipStreamSynchronize(b.stream);
    for (void* p : {(void*)sv->d_pos, (void*)sv->d_box, (void*)sv->d_status, (void*)sv->d_keys, (void*)sv->d_proj,
                    (void*)sv->d_qorth, (void*)sv->d_list, (void*)sv->d_seed, (void*)sv->d_out, (void*)sv->d_st,
                    (void*)sv->d_adm_trace})
        if (p) (void)hipFree(p);
    for (void* p : {(void*)sv->h_list, (void*)sv->h_more, (void*)sv->h_out, (void*)sv->h_st, (void*)sv->h_adm_trace})
        if (p) (void)hipHostFree(p);
    for (PolishBatch& b : sv->pb) {
        for (void* p : {(void*)b.d_list, (void*)b.d_out, (void*)b.d_st})
            if (p) (void)hipFree(p);
        for (void* p : {(void*)b.h_out, (void*)b.h_st})
            if (p) (void)hipHostFree(p);
        if (b.done) (void)hipEventDestroy(b.done);
        if (b.stream) (void)hipStreamDestroy(b.stream);
    }
    if (sv->ev_fin) (void)hipEventDestroy(sv->ev_fin);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
    return OPMM_OK;
}

int opmm_server_slots(const opmm_server* sv) { return sv ? sv->slots : 0; }

int opmm_server_submit(opmm_server* sv, const float* host_trace, const opmm_saccade* sac, double t_arrival,
                       int64_t* id_out)
{
    if (!sv || !host_trace || !sac) return OPMM_EINVAL;
    opmm_saccade s = *sac;
    s.pos_offset = 0;
    int rc = opmm_rt::validate_saccade(sv->ctx, s, (int64_t)s.T * s.C, 0);
    if (rc != OPMM_OK) return rc;
    if (s.T > sv->max_T) return sfail(sv, OPMM_EINVAL, "trace longer than the server's max_T");
    Request r;
    r.id = sv->next_id++;
    r.sac = s;
    r.trace.assign(host_trace, host_trace + (size_t)s.T * s.C);
    r.t_arrival = t_arrival;
    sv->pending.push_back(std::move(r));
    if (id_out) *id_out = sv->pending.back().id;
    return OPMM_OK;
}

int opmm_server_submit_many(opmm_server* sv, const float* host_pos, int64_t pos_len, const opmm_saccade* sacs,
                            int32_t n, const double* t_arrival, int64_t* ids_out)
{
    if (!sv || n < 0 || (n > 0 && (!host_pos || !sacs || !t_arrival))) return OPMM_EINVAL;
    for (int i = 0; i < n; ++i) {
        int rc = opmm_rt::validate_saccade(sv->ctx, sacs[i], pos_len, i);
        if (rc != OPMM_OK) return rc;
        if (sacs[i].T > sv->max_T) return sfail(sv, OPMM_EINVAL, "trace longer than the server's max_T");
    }
    for (int i = 0; i < n; ++i) {
        opmm_saccade s = sacs[i];
        const float* tr = host_pos + s.pos_offset;
        s.pos_offset = 0;
        int64_t id = 0;
        int rc = opmm_server_submit(sv, tr, &s, t_arrival[i], &id);
        if (rc != OPMM_OK) return rc;
        if (ids_out) ids_out[i] = id;
    }
    return OPMM_OK;
}

// Results of the nf finished slots fin (host arrays: opc [nf][18], then rmse [nf] and mae [nf] at
// hout, status at hst): a seeded result above the fallback threshold restarts its slot with the
// plain search, every other one completes its request.  Returns the number completed.
static int take_results(opmm_server* sv, const std::vector<int>& fin, const float* hout, const int32_t* hst)
{
    const double t = now_s();
    const size_t nf = fin.size();
    int ndone = 0;
    for (size_t i = 0; i < nf; ++i) {
        const int k = fin[i];
        Slot& sl = sv->slot[k];
        const float r = hout[P * nf + i];
        const float m = hout[(P + 1) * nf + i];
        int32_t status = hst[i];
        const float* o = hout + (size_t)P * i;
        if (sv->sg && sl.phase == PH_FIRST && !(r <= sv->prm.fallback_rmse) && !(status & OPMM_ST_NONFINITE_INPUT)) {
            // the plain search judges: restart this slot from the nominal centre
            sl.has_prev = true;
            std::memcpy(sl.prev_opc, o, sizeof(float) * P);
            sl.prev_rmse = r;
            sl.prev_mae = m;
            sl.prev_status = status;
            sl.phase = PH_FALLBACK;
            sl.round = 0;
            sl.rounds = sv->prm.plain.n_rounds;
            sl.n_cand = sv->prm.plain.n_cand;
            sv->reinit.push_back(k);
            sv->n_fallback++;
            continue;
        }
        Done d;
        d.id = sl.id;
        if (sl.has_prev && sl.prev_rmse <= r) {
            std::memcpy(d.opc, sl.prev_opc, sizeof(float) * P);
            d.rmse = sl.prev_rmse;
            d.mae = sl.prev_mae;
        } else {
            std::memcpy(d.opc, o, sizeof(float) * P);
            d.rmse = r;
            d.mae = m;
        }
        if (sl.has_prev) status |= OPMM_ST_FALLBACK | sl.prev_status;
        d.status = status;
        d.t_arrival = sl.t_arrival;
        d.t_done = t;
        sv->done.push_back(d);
        sl.busy = false;
        sv->free_slots.push_back(k);
        sv->n_completed++;
        ndone++;
    }
    return ndone;
}

// The oldest polished batch, once its event has completed.
static int take_polished(opmm_server* sv)
{
    PolishBatch& b = sv->pb[sv->pb_head];
    sv->pb_head = (sv->pb_head + 1) % kPolishBatches;
    sv->pb_count--;
    return take_results(sv, b.fin, b.h_out, b.h_st);
}

int opmm_server_step(opmm_server* sv, int32_t* n_done_out)
{
    if (!sv) return OPMM_EINVAL;
    if (n_done_out) *n_done_out = 0;
    SV_HIP(hipSetDevice(sv->device));
    hipStream_t st = sv->stream;
    const float dt = sv->prm.plain.dt_ms;
    const float box = sv->prm.plain.box_frac;
    int rc;
    // Each list of the step is staged in its own part of h_list, so no copy has to finish before
    // the host writes the next list; the device list d_list is reused in stream order.  The step
    // ends with one synchronisation, after which every part may be rewritten.
    SacDev* h_re = sv->h_list;
    SacDev* h_adm = sv->h_list + sv->slots;
    SacDev* h_act = sv->h_list + 2 * (size_t)sv->slots;
    SacDev* h_fin = sv->h_list + 3 * (size_t)sv->slots;
    bool queued = false;
    // 1. slots restarting with the plain search (their seeded result was rejected)
    if (!sv->reinit.empty()) {
        const int n = (int)sv->reinit.size();
        for (int i = 0; i < n; ++i) h_re[i] = slot_record(sv, sv->reinit[i]);
        SV_HIP(hipMemcpyAsync(sv->d_list, h_re, sizeof(SacDev) * n, hipMemcpyHostToDevice, st));
        SV_HIP(opmm_rt::launch_init(sv->d_list, n, box, sv->prm.plain.w_init_frac, nullptr, sv->ss, st));
        sv->reinit.clear();
        queued = true;
    }
    // 2. admission: pending requests into free slots
    std::vector<int> adm;
    while (!sv->free_slots.empty() && !sv->pending.empty() && (int)adm.size() < sv->max_admit) {
        const int k = sv->free_slots.back();
        sv->free_slots.pop_back();
        Request& r = sv->pending.front();
        Slot& sl = sv->slot[k];
        sl = Slot();
        sl.busy = true;
        sl.id = r.id;
        sl.sac = r.sac;
        sl.t_arrival = r.t_arrival;
        sl.phase = PH_FIRST;
        sl.round = 0;
        sl.rounds = phase_params(sv, PH_FIRST).n_rounds;
        sl.n_cand = phase_params(sv, PH_FIRST).n_cand;
        std::memcpy(sv->h_adm_trace + adm.size() * sv->max_T * 2, r.trace.data(), sizeof(float) * r.trace.size());
        adm.push_back(k);
        sv->pending.pop_front();
        sv->n_admitted++;
    }
    if (!adm.empty()) {
        const int n = (int)adm.size();
        for (int i = 0; i < n; ++i) h_adm[i] = slot_record(sv, adm[i]);
        SV_HIP(hipMemcpyAsync(sv->d_adm_trace, sv->h_adm_trace, sizeof(float) * n * sv->max_T * 2,
                              hipMemcpyHostToDevice, st));
        SV_HIP(hipMemcpyAsync(sv->d_list, h_adm, sizeof(SacDev) * n, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(scatter_traces_kernel, dim3(n), dim3(64), 0, st, n, (const SacDev*)sv->d_list,
                           (const float*)sv->d_adm_trace, sv->max_T * 2, sv->d_pos);
        SV_HIP(hipGetLastError());
        SV_HIP(opmm_rt::launch_prep(sv->d_list, n, sv->d_pos, sv->ss, st));
        const float* seeds = nullptr;
        if (sv->sg) {
            // the network reads the projection just queued for the admitted slots
            rc = opmm_rt::surrogate_predict_projected(sv->sg, n, sv->d_list, sv->d_proj, dt, box, sv->d_seed, st);
            if (rc != OPMM_OK) return rc;
            seeds = sv->d_seed;
        }
        const opmm_fit_params& fp = phase_params(sv, PH_FIRST);
        SV_HIP(opmm_rt::launch_init(sv->d_list, n, box, fp.w_init_frac, seeds, sv->ss, st));
        queued = true;
    }
    // 3. one round for every occupied slot, each at its own round; a step too small to fill the
    // device takes the smaller-tile shape.  While a round's launch has fewer tiles than the device
    // has CUs, further rounds follow for the slots still searching (each runs its own sequence of
    // rounds, so results do not depend on how rounds fall into steps), up to rounds_per_step.  A
    // further round's list is a subset of the previous one (fewer than `cus` records), staged in its
    // own part of h_more.
    std::vector<int> act;
    for (int k = 0; k < sv->slots; ++k) {
        const Slot& sl = sv->slot[k];
        if (sl.busy && sl.round < sl.rounds) act.push_back(k);
    }
    const std::vector<int> act0 = act;
    for (int it = 0; it < sv->prm.rounds_per_step && !act.empty(); ++it) {
        SacDev* h_it = it == 0 ? h_act : sv->h_more + (size_t)(it - 1) * sv->cus;
        const int na = (int)act.size();
        int64_t base_tiles = 0;
        for (int i = 0; i < na; ++i) {
            h_it[i] = slot_record(sv, act[i]);
            base_tiles += h_it[i].tiles;
        }
        const int shape = opmm_rt::launch_shape(sv->ctx, sv->shape, base_tiles);
        const int tile = opmm_rt::shape_tile(shape);
        int tiles = 0;
        for (int i = 0; i < na; ++i) {
            h_it[i].tiles = (h_it[i].n_cand + tile - 1) / tile;
            h_it[i].tile_base = tiles;
            tiles += h_it[i].tiles;
        }
        SV_HIP(hipMemcpyAsync(sv->d_list, h_it, sizeof(SacDev) * na, hipMemcpyHostToDevice, st));
        SV_HIP(opmm_rt::launch_reset_keys(sv->d_list, na, sv->ss, st));
        SV_HIP(opmm_rt::launch_round(shape, sv->d_list, na, tiles, dt, sv->ss, st));
        SV_HIP(opmm_rt::launch_refine(sv->d_list, na, phase_params(sv, PH_FIRST).shrink, sv->ss, st));
        queued = true;
        std::vector<int> next;
        for (int k : act)
            if (++sv->slot[k].round < sv->slot[k].rounds) next.push_back(k);
        if (base_tiles >= sv->cus) break;  // this round filled the device: one round per step
        act.swap(next);
    }
    // 4. harvest slots whose search is complete
    std::vector<int> fin;
    for (int k : act0)
        if (sv->slot[k].round >= sv->slot[k].rounds) fin.push_back(k);
    int ndone = 0;
    if (!fin.empty()) {
        const int nf = (int)fin.size();
        for (int i = 0; i < nf; ++i) h_fin[i] = slot_record(sv, fin[i]);
        SV_HIP(hipMemcpyAsync(sv->d_list, h_fin, sizeof(SacDev) * nf, hipMemcpyHostToDevice, st));
        if (sv->prm.polish_iter > 0) {
            // with every batch buffer in flight, the oldest batch is taken first
            if (sv->pb_count == kPolishBatches) {
                SV_HIP(hipEventSynchronize(sv->pb[sv->pb_head].done));
                ndone += take_polished(sv);
            }
            PolishBatch& b = sv->pb[(sv->pb_head + sv->pb_count) % kPolishBatches];
            // outputs packed for nf: opc [nf][18], rmse [nf], mae [nf] (one copy down)
            float* opc = b.d_out;
            float* rm = b.d_out + (size_t)P * nf;
            float* ma = rm + nf;
            SV_HIP(opmm_rt::launch_report(sv->d_list, nf, sv->d_pos, dt, sv->ss, opc, rm, ma, b.d_st, st));
            SV_HIP(hipMemcpyAsync(b.d_list, sv->d_list, sizeof(SacDev) * nf, hipMemcpyDeviceToDevice, st));
            SV_HIP(hipEventRecord(sv->ev_fin, st));
            hipStream_t ps = b.stream;
            SV_HIP(hipStreamWaitEvent(ps, sv->ev_fin, 0));
            opmm_polish_params pp;
            opmm_polish_params_default(&pp);
            pp.max_iter = sv->prm.polish_iter;
            pp.box_frac = sv->prm.plain.box_frac;
            pp.dt_ms = dt;
            SV_HIP(opmm_rt::launch_polish(sv->ctx, b.d_list, nf, sv->max_T, sv->d_pos, sv->ss.status,
                                          sv->prm.plain.model, pp, opc, rm, ma, ps));
            SV_HIP(hipMemcpyAsync(b.h_out, opc, sizeof(float) * (P + 2) * nf, hipMemcpyDeviceToHost, ps));
            SV_HIP(hipMemcpyAsync(b.h_st, b.d_st, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, ps));
            SV_HIP(hipEventRecord(b.done, ps));
            b.fin = fin;
            sv->pb_count++;
            queued = true;
        } else {
            float* opc = sv->d_out;
            float* rm = sv->d_out + (size_t)P * nf;
            float* ma = rm + nf;
            SV_HIP(opmm_rt::launch_report(sv->d_list, nf, sv->d_pos, dt, sv->ss, opc, rm, ma, sv->d_st, st));
            SV_HIP(hipMemcpyAsync(sv->h_out, opc, sizeof(float) * (P + 2) * nf, hipMemcpyDeviceToHost, st));
            SV_HIP(hipMemcpyAsync(sv->h_st, sv->d_st, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, st));
            SV_HIP(hipStreamSynchronize(st));
            queued = false;
            ndone += take_results(sv, fin, sv->h_out, sv->h_st);
        }
    }
    if (queued) SV_HIP(hipStreamSynchronize(st));
    // 5. polish batches that finished meanwhile, oldest first
    while (sv->pb_count > 0) {
        const hipError_t e = hipEventQuery(sv->pb[sv->pb_head].done);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) return opmm_rt::hip_fail(sv->ctx, e, "polish batch");
        ndone += take_polished(sv);
    }
    if (n_done_out) *n_done_out = ndone;
    sv->n_steps++;
    return OPMM_OK;
}

int opmm_server_poll(opmm_server* sv, int64_t max, int64_t* ids, float* opc, float* rmse, float* mae, int32_t* status,
                     double* t_arrival, double* t_done, int64_t* n_out)
{
    if (!sv || max < 0 || !n_out) return OPMM_EINVAL;
    int64_t n = 0;
    while (n < max && !sv->done.empty()) {
        const Done& d = sv->done.front();
        if (ids) ids[n] = d.id;
        if (opc) std::memcpy(opc + n * P, d.opc, sizeof(float) * P);
        if (rmse) rmse[n] = d.rmse;
        if (mae) mae[n] = d.mae;
        if (status) status[n] = d.status;
        if (t_arrival) t_arrival[n] = d.t_arrival;
        if (t_done) t_done[n] = d.t_done;
        sv->done.pop_front();
        ++n;
    }
    *n_out = n;
    return OPMM_OK;
}

int opmm_server_stats(const opmm_server* sv, int64_t* out)
{
    if (!sv || !out) return OPMM_EINVAL;
    int64_t busy = 0;
    for (const Slot& s : sv->slot) busy += s.busy;
    out[0] = (int64_t)sv->pending.size();
    out[1] = busy;
    out[2] = sv->n_admitted;
    out[3] = sv->n_completed;
    out[4] = sv->n_fallback;
    out[5] = sv->n_steps;
    out[6] = sv->slots;
    return OPMM_OK;
}

}  // extern "C"
