// Continuous-batching planning server (include/plan_serve.h).
//
// Device residency: every slot owns a terrain cell grid, a [13][max_K] state block
// and a [max_K] running-cost block for the whole life of the server; a
// request's controls and plan output stay in the caller's buffers. A step
// launches one rollout over all resident requests (rollout_slots: each
// workgroup belongs to one slot, so per-slot arguments are wave-uniform);
// the requests that end in it select their plans in the same launch (fused
// per-slot argmin). The host runs at
// most two steps ahead of the GPU and learns of finished requests through
// one event per step; per-step result copies go to their own pinned buffer so
// nothing is overwritten before it is read.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/plan_serve.h"
#include "plan_internal.h"

using plan::RolloutArgs;
using plan::SelectOut;

namespace {

constexpr int RING = 4;          // pinned result buffers (> steps in flight)
constexpr int MAX_INFLIGHT = 2;  // steps the host may run ahead of the GPU

// One request admitted in this step: its launch arguments (state, cost and
// argmin key and ticket pointing at its slot's storage; the caller's plan
// buffer) and its terrain.
struct AdmitEntry {
    RolloutArgs args;
    const float *height;
    const float *costmap;
    float4 *cells;
    int slot, W, H;
    float inv_res;
};

// Admission of every request a step admits, in one launch: blockIdx.y picks
// the request; thread t writes candidate t's initial state and zero running
// cost, workgroup b packs tile b of its terrain (pack_tile); thread 0
// publishes the launch arguments. The slot's bad-terrain flag was cleared by
// the rollout that finished its previous request (or at server creation).
__global__ __launch_bounds__(256) void admit_batch(const AdmitEntry *__restrict__ ents,
                                                   RolloutArgs *__restrict__ slot_args,
                                                   int *__restrict__ bad) {
    __shared__ plan::PackLds lds;
    const AdmitEntry &e = ents[blockIdx.y];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t == 0) slot_args[e.slot] = e.args;
    const int K = e.args.K;
    if (t < K) {
#pragma unroll
        for (int q = 0; q < 13; ++q) e.args.state[(size_t)q * K + t] = e.args.s0[q];
        e.args.cost[t] = 0.0f;
    }
    const int tiles_x = (e.W + plan::PACK_TILE - 1) / plan::PACK_TILE;
    const int tiles_y = (e.H + plan::PACK_TILE - 1) / plan::PACK_TILE;
    if ((int)blockIdx.x < tiles_x * tiles_y) {  // uniform over the workgroup
        const int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
        if (!plan::pack_tile(e.height, e.costmap, e.W, e.H, e.inv_res, bx * plan::PACK_TILE,
                             by * plan::PACK_TILE, e.cells, lds))
            atomicOr(bad + e.slot, 1);
    }
}

struct Req {
    plan_request_t r;
    plan_result_t res;
    unsigned long long footprint;
};

struct Slot {
    int req = -1;
    int progress = 0;  // control intervals already simulated
};

struct Step {
    hipEvent_t ev;
    int ring;
    uint32_t seq;                               // published with each finished slot's result
    std::vector<std::pair<int, int>> finished;  // (slot, request)
};

}  // namespace

struct plan_server {
    int device = 0;
    int simds = 1024;  // SIMDs of the device (4 per compute unit)
    hipStream_t stream = nullptr;
    plan_vehicle_t veh{};
    int max_slots = 0, max_K = 0, max_N = 0, max_W = 0, max_H = 0, chunk = 1;
    unsigned long long budget = 0, used = 0;
    std::chrono::steady_clock::time_point t0;
    // device memory
    float4 *cells = nullptr;  // [max_slots][max_W * max_H][4]
    float *state = nullptr;
    float *cost = nullptr;
    RolloutArgs *slot_args = nullptr;
    int *bad = nullptr;
    SelectOut *sel = nullptr;
    unsigned long long *sel_key = nullptr;  // per-slot argmin key (all ones between uses)
    unsigned int *sel_ticket = nullptr;     // per-slot arrival ticket (zero between uses)
    SelectOut *ring_host[RING] = {};
    int ring_next = 0;
    uint32_t seq = 0;  // sequence number of the last launched step
    // admission staging: pinned entries per ring position (reused only after
    // the step that copied them has completed) and their device copy
    AdmitEntry *admit_host[RING] = {};
    AdmitEntry *admit_dev = nullptr;
    // host bookkeeping
    std::vector<Req> reqs;
    std::deque<int> queue;
    std::vector<Slot> slots;
    std::deque<Step> inflight;
    std::deque<int> completed;  // finished request ids not yet collected
    std::vector<hipEvent_t> ev_pool;
    std::string err;
};

static thread_local std::string g_server_create_err;

static plan_status_t sfail(plan_server *s, plan_status_t st, const char *msg) {
    if (s)
        s->err = msg;
    else
        g_server_create_err = msg;
    return st;
}

static plan_status_t shipfail(plan_server *s, const char *what, hipError_t e) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return sfail(s, e == hipErrorOutOfMemory ? PLAN_ENOMEM : PLAN_EDEVICE, buf);
}

#define SHIP(s, call)                                          \
    do {                                                       \
        hipError_t e__ = (call);                               \
        if (e__ != hipSuccess) return shipfail((s), #call, e__); \
    } while (0)

static double now_of(const plan_server *s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

static unsigned long long footprint(const plan_request_t &r) {
    return 64ull * r.W * r.H + 56ull * r.K + 8ull * r.K * r.N + 8ull * r.N;
}

static void server_release(plan_server *s) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->cells);
    (void)hipFree(s->state);
    (void)hipFree(s->cost);
    (void)hipFree(s->slot_args);
    (void)hipFree(s->sel_key);
    (void)hipFree(s->sel_ticket);
    (void)hipFree(s->bad);
    (void)hipFree(s->sel);
    (void)hipFree(s->admit_dev);
    for (int i = 0; i < RING; ++i) {
        if (s->ring_host[i]) (void)hipHostFree(s->ring_host[i]);
        if (s->admit_host[i]) (void)hipHostFree(s->admit_host[i]);
    }
    for (auto &st : s->inflight) (void)hipEventDestroy(st.ev);
    for (auto e : s->ev_pool) (void)hipEventDestroy(e);
}

// Retire the oldest in-flight step (its event has completed).
static void retire_front(plan_server *s) {
    Step st = std::move(s->inflight.front());
    s->inflight.pop_front();
    const double t = now_of(s);
    const SelectOut *res = s->ring_host[st.ring];
    for (auto &fr : st.finished) {
        Req &q = s->reqs[fr.second];
        const SelectOut &o = res[fr.first];
        q.res.best_k = o.best_k;
        q.res.best_cost = o.best_cost;
        q.res.status = o.status ? (int)o.status : 1;
        q.res.t_done = t;
        s->completed.push_back(fr.second);
    }
    s->ev_pool.push_back(st.ev);
}

// Whether every result of step st has landed in its pinned ring entry (each
// finishing slot's record carries the step's sequence number in each of the
// three 8-byte words the host reads: (k*, seq), (J*, seq), (status, seq)).
// A step that finishes no request has nothing to publish.
static bool results_landed(const plan_server *s, const Step &st) {
    if (st.finished.empty()) return false;
    const SelectOut *res = s->ring_host[st.ring];
    for (const auto &fr : st.finished) {
        const uint64_t *w = reinterpret_cast<const uint64_t *>(&res[fr.first]);
        const uint64_t w0 = __atomic_load_n(&w[0], __ATOMIC_ACQUIRE);
        const uint64_t w1 = __atomic_load_n(&w[1], __ATOMIC_ACQUIRE);
        const uint64_t w2 = __atomic_load_n(&w[2], __ATOMIC_ACQUIRE);
        if ((uint32_t)(w0 >> 32) != st.seq || (uint32_t)(w1 >> 32) != st.seq ||
            (uint32_t)(w2 >> 32) != st.seq)
            return false;
    }
    return true;
}

// Retire completed steps from the front: a step is complete when its event
// has fired or, sooner, when all its results have landed in host memory (its
// kernel may still be writing plans then; they stay ordered on the stream).
static plan_status_t poll(plan_server *s, bool block_until_below) {
    while (!s->inflight.empty()) {
        if (results_landed(s, s->inflight.front())) {
            retire_front(s);
            continue;
        }
        hipError_t q = hipEventQuery(s->inflight.front().ev);
        if (q == hipSuccess) {
            retire_front(s);
            continue;
        }
        if (q != hipErrorNotReady) return shipfail(s, "hipEventQuery", q);
        if (block_until_below && (int)s->inflight.size() >= MAX_INFLIGHT) {
            SHIP(s, hipEventSynchronize(s->inflight.front().ev));
            retire_front(s);
            continue;
        }
        break;
    }
    return PLAN_OK;
}

// Admit queued requests (FIFO) while a slot is free and the byte budget
// allows. The step's admissions go out as one staging copy and one launch;
// the staging entries belong to the ring position of the step about to be
// launched, whose event covers the copy.
static plan_status_t admit(plan_server *s) {
    AdmitEntry *stage = s->admit_host[s->ring_next];
    int count = 0;
    long long extent = 0;
    while (!s->queue.empty()) {
        const int id = s->queue.front();
        Req &q = s->reqs[id];
        if (s->used + q.footprint > s->budget) break;  // FIFO: wait for memory
        int slot = -1;
        for (int i = 0; i < s->max_slots; ++i)
            if (s->slots[i].req < 0) {
                slot = i;
                break;
            }
        if (slot < 0) break;
        s->queue.pop_front();
        const plan_request_t &r = q.r;
        AdmitEntry &e = stage[count++];
        memset(&e, 0, sizeof e);
        e.cells = s->cells + (size_t)slot * 4 * plan::terrain_cells(s->max_W, s->max_H);
        RolloutArgs &a = e.args;
        plan::fill_rollout_args(a, s->veh, r.cost, r.integ, e.cells, r.W, r.H, r.x0, r.y0,
                                r.res);
        for (int j = 0; j < 13; ++j) a.s0[j] = r.state0[j];
        a.controls = r.controls_dev;
        a.K = r.K;
        a.N = r.N;
        a.state = s->state + (size_t)slot * 13 * s->max_K;
        a.cost = s->cost + (size_t)slot * s->max_K;
        a.final_state = nullptr;
        a.sel_key = s->sel_key + slot;
        a.sel_ticket = s->sel_ticket + slot;
        a.plan = r.plan_dev;
        a.sel_out = s->sel + slot;
        a.sel_out_host = nullptr;  // the step's ring entry, passed at launch
        e.height = r.height_dev;
        e.costmap = r.costmap_dev;
        e.slot = slot;
        e.W = r.W;
        e.H = r.H;
        e.inv_res = 1.0f / r.res;
        // workgroups: one per 256 candidates, one per tile of the terrain
        const long long tiles = (long long)((r.W + plan::PACK_TILE - 1) / plan::PACK_TILE) *
                                ((r.H + plan::PACK_TILE - 1) / plan::PACK_TILE);
        const long long kb = ((long long)r.K + 255) / 256;
        const long long work = tiles > kb ? tiles : kb;
        extent = work > extent ? work : extent;
        s->slots[slot].req = id;
        s->slots[slot].progress = 0;
        s->used += q.footprint;
        q.res.slot = slot;
        q.res.t_admit = now_of(s);
    }
    if (count == 0) return PLAN_OK;
    SHIP(s, hipMemcpyAsync(s->admit_dev, stage, sizeof(AdmitEntry) * count,
                           hipMemcpyHostToDevice, s->stream));
    const dim3 grid((unsigned)extent, (unsigned)count);
    hipLaunchKernelGGL(admit_batch, grid, dim3(256), 0, s->stream, s->admit_dev, s->slot_args,
                       s->bad);
    SHIP(s, hipGetLastError());
    return PLAN_OK;
}

static plan_status_t launch_step(plan_server *s) {
    plan::TickTable t;
    memset(&t, 0, sizeof t);
    long long total_K = 0;
    for (int i = 0; i < s->max_slots; ++i)
        if (s->slots[i].req >= 0) total_K += s->reqs[s->slots[i].req].r.K;
    if (total_K == 0) return PLAN_OK;
    int lanes, block;
    plan::auto_launch(total_K, s->simds, &lanes, &block);
    // a tick's slots are small independent plans: one-wave workgroups spread
    // each over more compute units (four-wave workgroups lengthened a lone
    // request's latency at 200 req/s from 0.088 to 0.11 ms)
    block = (total_K * lanes + 63) / 64 < 4096 ? 64 : 256;
    Step st;
    int blocks = 0;
    for (int i = 0; i < s->max_slots; ++i) {
        Slot &sl = s->slots[i];
        if (sl.req < 0) continue;
        const plan_request_t &r = s->reqs[sl.req].r;
        plan::TickEntry &e = t.e[t.count++];
        e.slot = i;
        e.block_start = blocks;
        e.n0 = sl.progress;
        // a slice of `chunk` intervals while requests wait for a slot or for
        // memory; with nothing waiting, run to the horizon's end in this launch
        const int slice = s->queue.empty() ? r.N : s->chunk;
        e.n1 = sl.progress + slice < r.N ? sl.progress + slice : r.N;
        e.finalize = e.n1 == r.N;
        blocks += (int)(((long long)r.K * lanes + block - 1) / block);
        if (e.finalize) st.finished.emplace_back(i, sl.req);
    }
    t.total_blocks = blocks;
    // the requests that end in this launch select their plans in it and
    // write their results into this step's pinned ring entry
    st.ring = s->ring_next;
    s->ring_next = (s->ring_next + 1) % RING;
    s->seq = s->seq + 1u == 0u ? 1u : s->seq + 1u;
    st.seq = s->seq;
    bool s1 = true;
    for (int j = 0; j < t.count; ++j)
        s1 = s1 && s->reqs[s->slots[t.e[j].slot].req].r.integ.substeps == 1;
    SHIP(s, plan::launch_rollout_slots(s->slot_args, t, s->bad, s->ring_host[st.ring], st.seq,
                                       s1, lanes, block, s->stream));
    // per-candidate costs of the requests that asked for them, copied before
    // any later launch can reuse the slot
    for (const auto &fr : st.finished) {
        const plan_request_t &r = s->reqs[fr.second].r;
        if (r.cost_dev)
            SHIP(s, hipMemcpyAsync(r.cost_dev, s->cost + (size_t)fr.first * s->max_K,
                                   sizeof(float) * r.K, hipMemcpyDeviceToDevice, s->stream));
    }
    if (s->ev_pool.empty()) {
        hipEvent_t e;
        SHIP(s, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        s->ev_pool.push_back(e);
    }
    st.ev = s->ev_pool.back();
    s->ev_pool.pop_back();
    SHIP(s, hipEventRecord(st.ev, s->stream));
    // advance progress; a finished slot is free for requests enqueued later
    for (int j = 0; j < t.count; ++j) {
        Slot &sl = s->slots[t.e[j].slot];
        sl.progress = t.e[j].n1;
        if (t.e[j].finalize) {
            s->used -= s->reqs[sl.req].footprint;
            sl.req = -1;
            sl.progress = 0;
        }
    }
    s->inflight.push_back(std::move(st));
    return PLAN_OK;
}

extern "C" {

plan_status_t plan_server_create(plan_server **out, const plan_vehicle_t *veh, int max_slots,
                                 int max_K, int max_N, int max_W, int max_H,
                                 unsigned long long budget_bytes, int chunk_intervals,
                                 void *hip_stream) {
    if (!out || !veh) return sfail(nullptr, PLAN_EINVAL, "NULL argument");
    if (!plan::valid_vehicle(*veh)) return sfail(nullptr, PLAN_EINVAL, "invalid vehicle parameters");
    if (max_slots < 1 || max_slots > plan::MAX_TICK_SLOTS)
        return sfail(nullptr, PLAN_EINVAL, "max_slots outside [1, 128]");
    if (max_K < 1 || max_N < 1 || max_W < 2 || max_H < 2 || chunk_intervals < 1)
        return sfail(nullptr, PLAN_EINVAL, "sizes must be K,N,chunk >= 1 and W,H >= 2");
    if ((long long)max_K * 4 > 0x7fffffffll ||
        plan::terrain_cells(max_W, max_H) >= plan::MAX_TERRAIN_CELLS)
        return sfail(nullptr, PLAN_EINVAL,
                     "sizes too large (K*4 below 2^31, W*H below 2^26)");
    if (budget_bytes == 0) return sfail(nullptr, PLAN_EINVAL, "budget must be positive");
    plan_server *s = new (std::nothrow) plan_server;
    if (!s) return sfail(nullptr, PLAN_ENOMEM, "host allocation failed");
    s->veh = *veh;
    s->max_slots = max_slots;
    s->max_K = max_K;
    s->max_N = max_N;
    s->max_W = max_W;
    s->max_H = max_H;
    s->chunk = chunk_intervals;
    s->budget = budget_bytes;
    s->stream = (hipStream_t)hip_stream;
    s->t0 = std::chrono::steady_clock::now();
    s->slots.assign(max_slots, Slot{});
    hipError_t e = hipSuccess;
    const size_t S = (size_t)max_slots;
    if (e == hipSuccess) e = hipGetDevice(&s->device);
    if (e == hipSuccess) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
        if (e == hipSuccess && cus > 0) s->simds = 4 * cus;
    }
    if (e == hipSuccess)
        e = hipMalloc(&s->cells, sizeof(float4) * 4 * S * plan::terrain_cells(max_W, max_H));
    if (e == hipSuccess) e = hipMalloc(&s->state, sizeof(float) * S * 13 * max_K);
    if (e == hipSuccess) e = hipMalloc(&s->cost, sizeof(float) * S * max_K);
    if (e == hipSuccess) e = hipMalloc(&s->slot_args, sizeof(RolloutArgs) * S);
    if (e == hipSuccess) e = hipMalloc(&s->sel_key, sizeof(unsigned long long) * S);
    if (e == hipSuccess) e = hipMalloc(&s->sel_ticket, sizeof(unsigned int) * S);
    if (e == hipSuccess) e = hipMemset(s->sel_key, 0xFF, sizeof(unsigned long long) * S);
    if (e == hipSuccess) e = hipMemset(s->sel_ticket, 0, sizeof(unsigned int) * S);
    if (e == hipSuccess) e = hipMalloc(&s->bad, sizeof(int) * S);
    if (e == hipSuccess) e = hipMalloc(&s->sel, sizeof(SelectOut) * S);
    if (e == hipSuccess) e = hipMalloc(&s->admit_dev, sizeof(AdmitEntry) * S);
    for (int i = 0; i < RING && e == hipSuccess; ++i) {
        e = hipHostMalloc(&s->ring_host[i], sizeof(SelectOut) * S, hipHostMallocDefault);
        if (e == hipSuccess) memset(s->ring_host[i], 0, sizeof(SelectOut) * S);  // seq 0: none
    }
    for (int i = 0; i < RING && e == hipSuccess; ++i)
        e = hipHostMalloc(&s->admit_host[i], sizeof(AdmitEntry) * S, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(s->bad, 0, sizeof(int) * S);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        shipfail(nullptr, "plan_server_create", e);
        server_release(s);
        delete s;
        return e == hipErrorOutOfMemory ? PLAN_ENOMEM : PLAN_EDEVICE;
    }
    *out = s;
    return PLAN_OK;
}

plan_status_t plan_server_submit(plan_server *s, const plan_request_t *r, int *id) {
    if (!s) return PLAN_EINVAL;
    if (!r || !id) return sfail(s, PLAN_EINVAL, "NULL argument");
    if (!r->height_dev || !r->controls_dev || !r->plan_dev)
        return sfail(s, PLAN_EINVAL, "NULL device buffer");
    if (r->K < 1 || r->K > s->max_K || r->N < 1 || r->N > s->max_N)
        return sfail(s, PLAN_EINVAL, "K or N outside the server maxima");
    if (r->W < 2 || r->H < 2 || r->W > s->max_W || r->H > s->max_H)
        return sfail(s, PLAN_EINVAL, "terrain size outside the server maxima");
    if (!(r->res > 0) || !isfinite(r->res) || !isfinite(r->x0) || !isfinite(r->y0))
        return sfail(s, PLAN_EINVAL, "terrain origin/resolution invalid");
    if (!plan::valid_cost(r->cost) || !plan::valid_integ(r->integ))
        return sfail(s, PLAN_EINVAL, "invalid cost or integration parameters");
    if (r->integ.method != PLAN_EULER)
        return sfail(s, PLAN_EINVAL, "the server integrates with PLAN_EULER only");
    if (!plan::finite_all(r->state0, 13)) return sfail(s, PLAN_EINVAL, "state0 not finite");
    Req q;
    q.r = *r;
    q.footprint = footprint(*r);
    if (q.footprint > s->budget) return sfail(s, PLAN_EINVAL, "request larger than the budget");
    memset(&q.res, 0, sizeof q.res);
    q.res.status = 0;
    q.res.best_k = -1;
    q.res.best_cost = INFINITY;
    q.res.slot = -1;
    q.res.t_submit = now_of(s);
    q.res.t_admit = q.res.t_done = -1.0;
    *id = (int)s->reqs.size();
    s->reqs.push_back(q);
    s->queue.push_back(*id);
    return PLAN_OK;
}

plan_status_t plan_server_step(plan_server *s, int *active, int *queued) {
    if (!s) return PLAN_EINVAL;
    SHIP(s, hipSetDevice(s->device));
    plan_status_t st = poll(s, false);
    if (st != PLAN_OK) return st;
    st = admit(s);
    if (st != PLAN_OK) return st;
    bool any = false;
    for (auto &sl : s->slots) any = any || sl.req >= 0;
    if (any) {
        st = poll(s, true);  // at most MAX_INFLIGHT steps ahead of the GPU
        if (st != PLAN_OK) return st;
        st = launch_step(s);
        if (st != PLAN_OK) return st;
    }
    if (active) {
        int n = 0;
        for (auto &sl : s->slots) n += sl.req >= 0;
        *active = n;
    }
    if (queued) *queued = (int)s->queue.size();
    return PLAN_OK;
}

plan_status_t plan_server_drain(plan_server *s) {
    if (!s) return PLAN_EINVAL;
    for (;;) {
        int active = 0, queued = 0;
        plan_status_t st = plan_server_step(s, &active, &queued);
        if (st != PLAN_OK) return st;
        if (active == 0 && queued == 0) {
            while (!s->inflight.empty()) {
                if (!results_landed(s, s->inflight.front()))
                    SHIP(s, hipEventSynchronize(s->inflight.front().ev));
                retire_front(s);
            }
            // every plan buffer written before returning
            SHIP(s, hipStreamSynchronize(s->stream));
            return PLAN_OK;
        }
    }
}

plan_status_t plan_server_completions(plan_server *s, int *ids, int capacity, int *count) {
    if (!s) return PLAN_EINVAL;
    if (!count || capacity < 0 || (!ids && capacity > 0))
        return sfail(s, PLAN_EINVAL, "invalid completion buffer");
    int n = 0;
    while (n < capacity && !s->completed.empty()) {
        ids[n++] = s->completed.front();
        s->completed.pop_front();
    }
    *count = n;
    return PLAN_OK;
}

plan_status_t plan_server_stats(const plan_server *s, int *active, int *queued,
                                unsigned long long *used_bytes) {
    if (!s) return PLAN_EINVAL;
    if (active) {
        int n = 0;
        for (auto &sl : s->slots) n += sl.req >= 0;
        *active = n;
    }
    if (queued) *queued = (int)s->queue.size();
    if (used_bytes) *used_bytes = s->used;
    return PLAN_OK;
}

plan_status_t plan_server_result(const plan_server *s, int id, plan_result_t *out) {
    if (!s || !out || id < 0 || id >= (int)s->reqs.size()) return PLAN_EINVAL;
    *out = s->reqs[id].res;
    return PLAN_OK;
}

double plan_server_now(const plan_server *s) { return s ? now_of(s) : 0.0; }

void plan_server_destroy(plan_server *s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    server_release(s);
    delete s;
}

const char *plan_server_last_error(const plan_server *s) {
    return s ? s->err.c_str() : g_server_create_err.c_str();
}

}  // extern "C"
