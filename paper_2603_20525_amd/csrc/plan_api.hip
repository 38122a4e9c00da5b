// Host side of the libplan C ABI (include/plan.h): argument validation,
// workspace ownership, derived constants, kernel launches on the caller's
// stream. No exception or abort crosses the ABI.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <mutex>
#include <new>
#include <string>

#include "../../include/plan.h"
#include "plan_internal.h"

using plan::RolloutArgs;
using plan::SelectOut;
using plan::auto_launch;
using plan::finite_all;
using plan::valid_cost;
using plan::valid_integ;
using plan::valid_vehicle;

struct plan_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    plan_vehicle_t veh{};
    plan_cost_t cost{};
    plan_integ_t integ{};
    int max_K = 0, max_N = 0, max_W = 0, max_H = 0;
    // terrain cells [max_W * max_H][4]
    float4 *cells = nullptr;
    int W = 0, H = 0;
    float x0 = 0, y0 = 0, res = 0;
    bool has_terrain = false;
    bool has_costmap = false;
    int *bad_dev = nullptr;
    int *bad_host = nullptr;  // pinned
    // selection workspace
    unsigned long long *part_keys = nullptr;  // argmin slot, all ones between launches
    unsigned int *counters = nullptr;  // tickets: [0] argmin, [2] fused argmin
    unsigned long long *fused_key = nullptr;  // fused argmin slot, all ones between launches
    SelectOut *sel_dev = nullptr;
    SelectOut *sel_host = nullptr;  // pinned
    uint32_t seq = 0;               // sequence number of the last published selection
    // launch shape
    int simds = 1024;  // SIMDs of the device (4 per compute unit)
    int lanes_opt = 0, block_opt = 0;
    int last_lanes = 0, last_block = 0;
    // candidate order for gather locality (workspace for max_K)
    int order_mode = PLAN_ORDER_AUTO;
    bool last_ordered = false;
    plan::OrderArgs ow{};
    float *ctrl_lane = nullptr;  // lane-ordered controls, grown on demand
    size_t ctrl_lane_floats = 0;
    // terrain preparation: intermediate grid of the separable smoothing
    float *smooth_tmp = nullptr;
    // adjoint workspace (grown on demand): state, checkpoints, segment scratch
    float *gws = nullptr;
    size_t gws_floats = 0;
    // timing
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool ev_recorded = false;
    std::string err;
};

static thread_local std::string g_create_err;

// Fixed adjoint workspace of plan_rollout_grad_noalloc, for callers that
// cannot allocate device memory inside a call. One copy per GPU, held until
// the process ends; every call on a GPU shares it (overlapping calls race).
// Host code uses only the device address resolved per device at context
// creation, never the symbol itself.
constexpr size_t NOALLOC_FLOATS = (size_t)4 << 20;  // 16 MiB
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];
constexpr int MAX_DEVICES = 64;
static float *g_scratch_dev[MAX_DEVICES];
static std::mutex g_scratch_mu;

// With `device` current: resolve this device's copy of the workspace once.
static hipError_t resolve_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (g_scratch_dev[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_dev[device] = static_cast<float *>(p);
    return e;
}

static float *scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < MAX_DEVICES) ? g_scratch_dev[device] : nullptr;
}

static plan_status_t fail(plan_ctx *c, plan_status_t st, const char *fmt, const char *a = "") {
    char buf[512];
    snprintf(buf, sizeof buf, fmt, a);
    if (c)
        c->err = buf;
    else
        g_create_err = buf;
    return st;
}

static plan_status_t hip_fail(plan_ctx *c, const char *what, hipError_t e) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    if (c)
        c->err = buf;
    else
        g_create_err = buf;
    return PLAN_EDEVICE;
}

#define HIP_TRY(ctx, call)                                         \
    do {                                                           \
        hipError_t e__ = (call);                                   \
        if (e__ != hipSuccess) return hip_fail((ctx), #call, e__); \
    } while (0)

static void release(plan_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->cells);
    (void)hipFree(c->bad_dev);
    (void)hipFree(c->part_keys);
    (void)hipFree(c->counters);
    (void)hipFree(c->fused_key);
    (void)hipFree(c->sel_dev);
    (void)hipFree(c->gws);
    (void)hipFree(c->smooth_tmp);
    (void)hipFree(c->ow.lat);
    (void)hipFree(c->ctrl_lane);
    (void)hipFree(c->ow.range);
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(c->ow.keys[i]);
        (void)hipFree(c->ow.vals[i]);
    }
    (void)hipFree(c->ow.hist);
    (void)hipFree(c->ow.dtotal);
    if (c->sel_host) (void)hipHostFree(c->sel_host);
    if (c->bad_host) (void)hipHostFree(c->bad_host);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
}

namespace plan {

// Derived constants of one launch (double on the host, rounded once).
void fill_rollout_args(RolloutArgs &a, const plan_vehicle_t &v, const plan_cost_t &co,
                       const plan_integ_t &in, const float4 *cells, int W, int H, float x0,
                       float y0, float res) {
    memset(&a, 0, sizeof a);
    const double L = (double)v.Lf + v.Lr;
    a.invM = (float)(1.0 / v.M);
    a.invJxx = (float)(1.0 / v.Jxx);
    a.invJyy = (float)(1.0 / v.Jyy);
    a.invJzz = (float)(1.0 / v.Jzz);
    a.dJyz = (float)((double)v.Jyy - v.Jzz);
    a.dJxz = (float)((double)v.Jxx - v.Jzz);
    a.dJxy = (float)((double)v.Jxx - v.Jyy);
    a.Lf = v.Lf;
    a.Lr = v.Lr;
    a.half_e = 0.5f * v.e;
    a.hR = v.hR;
    a.Lf_g = (float)((double)v.Lf / res);
    a.Lr_g = (float)((double)v.Lr / res);
    a.half_e_g = (float)(0.5 * (double)v.e / res);
    a.hR_g = (float)((double)v.hR / res);
    a.kf = v.kf;
    a.kr = v.kr;
    a.bf = v.bf;
    a.br = v.br;
    a.Fsf = (float)(0.5 * v.g * v.M * v.Lr / L);
    a.Fsr = (float)(0.5 * v.g * v.M * v.Lf / L);
    a.Mhalf = 0.5f * v.M;
    a.C = v.C;
    a.mu = v.mu;
    a.mu2 = v.mu * v.mu;
    a.delta_max = v.delta_max;
    a.drate_max = v.delta_rate_max;
    a.g = v.g;
    const double he = 0.5 * (double)v.e;
    a.MgRbar = (float)((double)v.M * v.g * sqrt((double)v.hR * v.hR + he * he));
    a.phibar = (float)atan(2.0 * v.hR / v.e);
    a.Kzzf = (float)((double)v.M * v.Lr / L);
    a.Kzzr = (float)((double)v.M * v.Lf / L);
    a.Kzx = (float)((double)v.M * v.hR / L);
    const double a_bar_y = (double)v.g * v.e / (2.0 * v.hR);  // M g / (2 K_zy)
    a.a_bar_y = (float)a_bar_y;
    a.inv_eps_ay = (float)(1.0 / ((co.eps_ay > 0) ? (double)co.eps_ay : 0.1 * a_bar_y));
    a.w_t = co.w_t;
    a.w_c = co.w_c;
    a.w_g = co.w_g;
    a.goal_x = co.goal_x;
    a.goal_y = co.goal_y;
    a.goal_r2 = (float)((double)co.goal_r * co.goal_r);
    a.sigma = co.sigma;
    const double eps = (co.eps_esm > 0) ? (double)co.eps_esm : 0.1 * esm_level(v);
    a.inv_eps_esm = (float)(1.0 / eps);
    a.h = (float)((double)in.dt / in.substeps);
    a.h_half = (float)(0.5 * (double)in.dt / in.substeps);
    a.h_sixth = (float)((double)in.dt / in.substeps / 6.0);
    a.S = in.substeps;
    a.method = in.method;
    a.accel_max = in.accel_max;
    a.vx_min = in.vx_min;
    a.cells = cells;
    a.W = W;
    a.H = H;
    a.x0 = x0;
    a.y0 = y0;
    a.inv_res = (float)(1.0 / res);
    a.x0_g = (float)((double)x0 / res);
    a.y0_g = (float)((double)y0 / res);
    a.umax = (float)(W - 1);
    a.vmax = (float)(H - 1);
}

double esm_level(const plan_vehicle_t &v) {
    const double hR = v.hR, he = 0.5 * (double)v.e;
    return (double)v.M * v.g * (sqrt(hR * hR + he * he) - hR);
}

bool valid_vehicle(const plan_vehicle_t &v) {
    if (!finite_all(&v.M, sizeof(plan_vehicle_t) / sizeof(float))) return false;
    return v.M > 0 && v.Jxx > 0 && v.Jyy > 0 && v.Jzz > 0 && v.Lf + v.Lr > 0 && v.e > 0 &&
           v.hR > 0 && v.mu > 0 && v.g > 0 && v.delta_max >= 0 && v.delta_rate_max >= 0;
}

bool valid_cost(const plan_cost_t &c) {
    return finite_all(&c.w_t, sizeof(plan_cost_t) / sizeof(float)) && c.goal_r >= 0;
}

bool valid_integ(const plan_integ_t &i) {
    return isfinite(i.dt) && i.dt > 0 && i.substeps >= 1 && isfinite(i.accel_max) &&
           isfinite(i.vx_min) && (i.method == PLAN_EULER || i.method == PLAN_RK4);
}

bool finite_all(const float *p, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(p[i])) return false;
    return true;
}

void auto_launch(long long K, int simds, int *lanes, int *block) {
    // Spread small candidate sets over more lanes (wheel-parallel); sets
    // that give every SIMD a wave at one lane per candidate (65 536 on the
    // MI355X's 1 024 SIMDs) use one lane, avoiding redundant chassis work.
    if (K <= 16384) {
        *lanes = 4;
    } else if (K < 65536) {
        *lanes = 2;
    } else {
        *lanes = 1;
    }
    // Up to one wave per SIMD, four waves share each workgroup (and so a
    // compute unit, its L1 and the fused selection's atomics: measured 2 %
    // faster at both K = 4 096 x 4 lanes and K = 65 536 x 1 lane); with
    // several waves per SIMD, one-wave workgroups balance better (2 % at the
    // paper's 204 288 candidates).
    const long long waves = (K * *lanes + 63) / 64;
    *block = (waves <= simds) ? 256 : 64;
}

}  // namespace plan

static void fill_args(const plan_ctx *c, RolloutArgs &a) {
    plan::fill_rollout_args(a, c->veh, c->cost, c->integ, c->cells, c->W, c->H, c->x0, c->y0,
                            c->res);
    a.has_costmap = c->has_costmap;
}


extern "C" {

plan_status_t plan_create(plan_ctx **out, const plan_vehicle_t *veh, const plan_cost_t *cost,
                          const plan_integ_t *integ, int max_K, int max_N, int max_W, int max_H,
                          void *hip_stream) {
    if (!out || !veh || !cost || !integ) return fail(nullptr, PLAN_EINVAL, "NULL argument");
    if (!valid_vehicle(*veh)) return fail(nullptr, PLAN_EINVAL, "invalid vehicle parameters");
    if (!valid_cost(*cost)) return fail(nullptr, PLAN_EINVAL, "invalid cost parameters");
    if (!valid_integ(*integ)) return fail(nullptr, PLAN_EINVAL, "invalid integration parameters");
    if (max_K < 1 || max_N < 1 || max_W < 2 || max_H < 2)
        return fail(nullptr, PLAN_EINVAL, "max sizes must be K,N >= 1 and W,H >= 2");
    if (plan::terrain_cells(max_W, max_H) >= plan::MAX_TERRAIN_CELLS)
        return fail(nullptr, PLAN_EINVAL, "terrain grid too large (W*H must be below 2^26)");
    if ((long long)max_K * 4 > 0x7fffffffll) return fail(nullptr, PLAN_EINVAL, "max_K too large");

    plan_ctx *c = new (std::nothrow) plan_ctx;
    if (!c) return fail(nullptr, PLAN_ENOMEM, "host allocation failed");
    c->veh = *veh;
    c->cost = *cost;
    c->integ = *integ;
    c->max_K = max_K;
    c->max_N = max_N;
    c->max_W = max_W;
    c->max_H = max_H;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e;
#define CREATE_TRY(call)                                    \
    do {                                                    \
        e = (call);                                         \
        if (e != hipSuccess) {                              \
            hip_fail(nullptr, #call, e);                    \
            release(c);                                     \
            delete c;                                       \
            return e == hipErrorOutOfMemory ? PLAN_ENOMEM : PLAN_EDEVICE; \
        }                                                   \
    } while (0)
    CREATE_TRY(hipGetDevice(&c->device));
    {
        int cus = 0;
        CREATE_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        if (cus > 0) c->simds = 4 * cus;
    }
    CREATE_TRY(resolve_scratch(c->device));
    CREATE_TRY(hipMalloc(&c->cells, sizeof(float4) * 4 * plan::terrain_cells(max_W, max_H)));
    CREATE_TRY(hipMalloc(&c->smooth_tmp, sizeof(float) * (size_t)max_W * max_H));
    CREATE_TRY(hipMalloc(&c->bad_dev, sizeof(int)));
    CREATE_TRY(hipHostMalloc(&c->bad_host, sizeof(int), hipHostMallocDefault));
    CREATE_TRY(hipMalloc(&c->part_keys, sizeof(unsigned long long)));
    CREATE_TRY(hipMemset(c->part_keys, 0xFF, sizeof(unsigned long long)));
    CREATE_TRY(hipMalloc(&c->counters, sizeof(unsigned int) * 4));
    CREATE_TRY(hipMemset(c->counters, 0, sizeof(unsigned int) * 4));
    CREATE_TRY(hipMalloc(&c->fused_key, sizeof(unsigned long long)));
    CREATE_TRY(hipMemset(c->fused_key, 0xFF, sizeof(unsigned long long)));
    CREATE_TRY(hipMalloc(&c->sel_dev, sizeof(SelectOut)));
    CREATE_TRY(hipHostMalloc(&c->sel_host, sizeof(SelectOut), hipHostMallocDefault));
    memset(c->sel_host, 0, sizeof(SelectOut));  // no sequence number matches 0
    c->ow.lat_stride = max_K;
    c->ow.nt_max = plan::order_tiles(max_K);
    CREATE_TRY(hipMalloc(&c->ow.lat, sizeof(float) * 4 * (size_t)max_K));
    CREATE_TRY(hipMalloc(&c->ow.range, sizeof(unsigned) * 8));
    for (int i = 0; i < 2; ++i) {
        CREATE_TRY(hipMalloc(&c->ow.keys[i], sizeof(unsigned) * (size_t)max_K));
        CREATE_TRY(hipMalloc(&c->ow.vals[i], sizeof(int) * (size_t)max_K));
    }
    CREATE_TRY(hipMalloc(&c->ow.hist, sizeof(unsigned) * 256 * (size_t)c->ow.nt_max));
    CREATE_TRY(hipMalloc(&c->ow.dtotal, sizeof(unsigned) * 256));
    CREATE_TRY(plan::launch_order_reset(c->ow, c->stream));
    CREATE_TRY(hipEventCreate(&c->ev0));
    CREATE_TRY(hipEventCreate(&c->ev1));
    CREATE_TRY(hipDeviceSynchronize());
#undef CREATE_TRY
    *out = c;
    return PLAN_OK;
}

plan_status_t plan_set_stream(plan_ctx *c, void *hip_stream) {
    if (!c) return PLAN_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return PLAN_OK;
}

plan_status_t plan_set_cost(plan_ctx *c, const plan_cost_t *cost) {
    if (!c) return PLAN_EINVAL;
    if (!cost || !valid_cost(*cost)) return fail(c, PLAN_EINVAL, "invalid cost parameters");
    c->cost = *cost;
    return PLAN_OK;
}

plan_status_t plan_set_terrain(plan_ctx *c, const float *height_dev, int W, int H, float x0,
                               float y0, float res, const float *costmap_dev) {
    if (!c) return PLAN_EINVAL;
    if (!height_dev) return fail(c, PLAN_EINVAL, "height is NULL");
    if (W < 2 || H < 2 || W > c->max_W || H > c->max_H)
        return fail(c, PLAN_EINVAL, "terrain size outside [2, max] in W or H");
    if (!(res > 0) || !isfinite(res) || !isfinite(x0) || !isfinite(y0))
        return fail(c, PLAN_EINVAL, "terrain origin/resolution invalid");
    HIP_TRY(c, hipSetDevice(c->device));
    c->has_terrain = false;
    HIP_TRY(c, hipMemsetAsync(c->bad_dev, 0, sizeof(int), c->stream));
    HIP_TRY(c, plan::launch_pack_terrain(height_dev, costmap_dev, W, H, 1.0f / res, c->cells,
                                         c->bad_dev, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->bad_host, c->bad_dev, sizeof(int), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (*c->bad_host) return fail(c, PLAN_EINVAL, "terrain holds non-finite values");
    c->W = W;
    c->H = H;
    c->x0 = x0;
    c->y0 = y0;
    c->res = res;
    c->has_costmap = costmap_dev != nullptr;
    c->has_terrain = true;
    return PLAN_OK;
}

enum class Kind { plain, chunk, sampled, fused, fused_sampled };

// Automatic locality order: launches that draw uniform samples in the kernel
// with many Euler substeps per control interval (the paper's configuration:
// steering rates spread over the admissible set, 50 substeps), from this many
// candidates on. There the candidates of a wave spread over tens of metres,
// the steps are texture-bound and the sort is amortised over a long rollout:
// ordering at one lane per candidate beat the unordered automatic shape from
// 49 152 candidates on (by about a quarter at the paper's K). With one
// substep per interval (a control draw every step, a short rollout) it lost,
// with uniform and with Gaussian draws, and the spread of materialised
// controls is unknown, so those launches are ordered only on request.
constexpr int ORDER_AUTO_MIN_K_UNIFORM = 49152;
constexpr int ORDER_AUTO_MIN_SUBSTEPS = 8;

// Whether a full-horizon launch of K candidates at this lane count runs in
// locality order (ordered launches then use one lane per candidate).
// smp: the generator of a launch that draws its controls, else nullptr.
static bool order_wanted(const plan_ctx *c, int K, const plan::SampleArgs *smp) {
    return c->order_mode == PLAN_ORDER_ON ||
           (c->order_mode == PLAN_ORDER_AUTO && smp && smp->kind == PLAN_SAMPLE_UNIFORM &&
            c->integ.substeps >= ORDER_AUTO_MIN_SUBSTEPS && K >= ORDER_AUTO_MIN_K_UNIFORM);
}

// Sort the candidates of a one-lane full-horizon launch by their proxy
// trajectories and point a.order at the result. delta0 and vx0: the initial
// steering angle and forward speed.
static plan_status_t order_candidates(plan_ctx *c, RolloutArgs &a, float delta0, float vx0) {
    plan::OrderArgs o = c->ow;
    o.K = a.K;
    o.N = a.N;
    o.controls = a.controls;
    o.smp = a.smp;
    o.dt = c->integ.dt;
    o.drate_max = c->veh.delta_rate_max;
    o.delta_max = c->veh.delta_max;
    o.accel_max = c->integ.accel_max;
    o.vx_min = c->integ.vx_min;
    o.inv_wheelbase = (float)(1.0 / ((double)c->veh.Lf + (double)c->veh.Lr));
    o.mu_g = (float)((double)c->veh.mu * (double)c->veh.g);
    o.delta0 = delta0;
    o.vx0 = vx0;
    HIP_TRY(c, plan::launch_locality_order(o, c->stream));
    a.order = c->ow.vals[0];
    if (a.controls) {
        // materialised controls: one gather into lane order keeps the
        // rollout's control reads coalesced. The copy grows on demand; if it
        // cannot be allocated, the rollout reads the controls in place
        // (scattered, same results).
        const size_t need = 2 * (size_t)a.N * a.K;
        if (c->ctrl_lane_floats < need) {
            if (c->ctrl_lane) {
                // the previous copy may still be read by a launch in flight
                HIP_TRY(c, hipStreamSynchronize(c->stream));
                HIP_TRY(c, hipFree(c->ctrl_lane));
            }
            c->ctrl_lane = nullptr;
            c->ctrl_lane_floats = 0;
            if (hipMalloc(&c->ctrl_lane, sizeof(float) * need) == hipSuccess)
                c->ctrl_lane_floats = need;
            else
                c->ctrl_lane = nullptr;
            (void)hipGetLastError();  // an allocation failure is not sticky
        }
        if (c->ctrl_lane) {
            HIP_TRY(c, plan::launch_permute_controls(a.controls, a.order, a.K, a.N, c->ctrl_lane,
                                                     c->stream));
            a.controls_lane = c->ctrl_lane;
        }
    }
    c->last_ordered = true;
    return PLAN_OK;
}

static plan_status_t launch(plan_ctx *c, RolloutArgs &a, Kind kind) {
    int lanes, block;
    auto_launch(a.K, c->simds, &lanes, &block);
    if (c->lanes_opt) lanes = c->lanes_opt;
    if (c->block_opt) block = c->block_opt;
    a.order = nullptr;
    a.controls_lane = nullptr;
    c->last_ordered = false;
    const bool sampled = kind == Kind::sampled || kind == Kind::fused_sampled;
    const bool ordered = kind != Kind::chunk && order_wanted(c, a.K, sampled ? &a.smp : nullptr);
    if (ordered && lanes != 1) {
        lanes = 1;
        block = c->block_opt ? c->block_opt : (((long long)a.K + 63) / 64 <= c->simds ? 256 : 64);
    }
    c->last_lanes = lanes;
    c->last_block = block;
    // one lane per candidate with at most one wave per SIMD: the kernels
    // built for a wave that has its SIMD to itself
    const bool one_wave = lanes == 1 && ((long long)a.K + 63) / 64 <= c->simds;
    // automatic one-lane launches of the paper's shape (several substeps per
    // interval, no costmap, forward Euler) whose last round of waves would be
    // a small remainder: that remainder runs four lanes per candidate
    int split = 0;
    if (!c->lanes_opt && !c->block_opt && lanes == 1 && block == 64 && kind != Kind::chunk &&
        a.S > 1 && !a.has_costmap && a.method == 0)
        split = plan::balanced_split(a.K, c->simds);
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->timing) HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    if (ordered) {
        const plan_status_t st = order_candidates(c, a, a.s0[12], a.s0[6]);
        if (st != PLAN_OK) return st;
    }
    if (split > 0) {
        HIP_TRY(c, plan::launch_rollout_balanced(
                       a, split, kind == Kind::sampled || kind == Kind::fused_sampled,
                       kind == Kind::fused || kind == Kind::fused_sampled, c->stream));
        if (c->timing) {
            HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
            c->ev_recorded = true;
        }
        return PLAN_OK;
    }
    switch (kind) {
    case Kind::plain:
    case Kind::chunk:
        HIP_TRY(c, plan::launch_rollout(a, lanes, block, kind == Kind::chunk, c->stream, one_wave));
        break;
    case Kind::sampled:
        HIP_TRY(c, plan::launch_rollout_sampled(a, lanes, block, c->stream, one_wave));
        break;
    case Kind::fused:
    case Kind::fused_sampled:
        HIP_TRY(c, plan::launch_rollout_argmin(a, lanes, block, kind == Kind::fused_sampled,
                                               c->stream, one_wave));
        break;
    }
    if (c->timing) {
        HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
        c->ev_recorded = true;
    }
    return PLAN_OK;
}

plan_status_t plan_rollout(plan_ctx *c, const float state0[13], const float *controls_dev, int K,
                           int N, float *cost_dev, float *final_state_dev) {
    if (!c) return PLAN_EINVAL;
    if (!state0 || !controls_dev || !cost_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (!finite_all(state0, 13)) return fail(c, PLAN_EINVAL, "state0 not finite");
    if (!c->has_terrain) return fail(c, PLAN_ENOTERRAIN, "no terrain set");
    RolloutArgs a;
    fill_args(c, a);
    for (int q = 0; q < 13; ++q) a.s0[q] = state0[q];
    a.controls = controls_dev;
    a.K = K;
    a.N = N;
    a.n0 = 0;
    a.n1 = N;
    a.finalize = 1;
    a.cost = cost_dev;
    a.final_state = final_state_dev;
    return launch(c, a, Kind::plain);
}

// Validated generator arguments of a plan_sample_t.
static plan_status_t sample_args(plan_ctx *c, const plan_sample_t *spec, plan::SampleArgs &sa) {
    if (!spec) return fail(c, PLAN_EINVAL, "sample spec is NULL");
    if (spec->kind != PLAN_SAMPLE_UNIFORM && spec->kind != PLAN_SAMPLE_GAUSSIAN)
        return fail(c, PLAN_EINVAL, "sample kind must be PLAN_SAMPLE_UNIFORM or _GAUSSIAN");
    if (!finite_all(spec->scale, 2) || spec->scale[0] < 0 || spec->scale[1] < 0)
        return fail(c, PLAN_EINVAL, "sample scales must be finite and >= 0");
    sa.kind = spec->kind;
    sa.keep_nominal = spec->keep_nominal != 0;
    sa.key0 = spec->seed;
    sa.key1 = spec->stream;
    sa.scale0 = spec->scale[0];
    sa.scale1 = spec->scale[1];
    sa.nominal = spec->nominal_dev;
    return PLAN_OK;
}

plan_status_t plan_sample_controls(plan_ctx *c, const plan_sample_t *spec, int K, int N,
                                   float *controls_dev) {
    if (!c) return PLAN_EINVAL;
    if (!controls_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    plan::SampleArgs sa;
    plan_status_t st = sample_args(c, spec, sa);
    if (st != PLAN_OK) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, plan::launch_sample_controls(sa, K, N, controls_dev, c->stream));
    return PLAN_OK;
}

plan_status_t plan_rollout_sampled(plan_ctx *c, const float state0[13], const plan_sample_t *spec,
                                   int K, int N, float *cost_dev, float *final_state_dev) {
    if (!c) return PLAN_EINVAL;
    if (c->integ.method != PLAN_EULER)
        return fail(c, PLAN_EINVAL, "%s supports PLAN_EULER integration only", "plan_rollout_sampled");
    if (!state0 || !cost_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (!finite_all(state0, 13)) return fail(c, PLAN_EINVAL, "state0 not finite");
    RolloutArgs a;
    fill_args(c, a);
    plan_status_t st = sample_args(c, spec, a.smp);
    if (st != PLAN_OK) return st;
    if (!c->has_terrain) return fail(c, PLAN_ENOTERRAIN, "no terrain set");
    for (int q = 0; q < 13; ++q) a.s0[q] = state0[q];
    a.controls = nullptr;
    a.K = K;
    a.N = N;
    a.n0 = 0;
    a.n1 = N;
    a.finalize = 1;
    a.cost = cost_dev;
    a.final_state = final_state_dev;
    return launch(c, a, Kind::sampled);
}

// Sequence number for the next selection whose host copy is read: unique
// in the process (until it wraps) and never 0, so neither a zeroed record nor
// one left in recycled pinned memory by another context can match.
static std::atomic<uint32_t> g_seq{0};

static uint32_t next_seq(plan_ctx *c) {
    uint32_t s = g_seq.fetch_add(1u, std::memory_order_relaxed) + 1u;
    if (s == 0u) s = g_seq.fetch_add(1u, std::memory_order_relaxed) + 1u;
    c->seq = s;
    return s;
}

// Wait for the pinned copy of (k*, J*) published by selection `seq`: poll the
// two 8-byte words that carry it (each also holds seq) for up to about a
// millisecond, then fall back to a stream synchronisation, which also reports
// a failed launch. Polling returns as soon as the result lands in host memory,
// a few microseconds before the stream would report completion; the kernel
// may still be writing the plan then, and device outputs stay ordered on the
// context's stream.
static plan_status_t wait_result(plan_ctx *c, uint32_t seq, int *best_k, float *best_cost) {
    const uint64_t *w = reinterpret_cast<const uint64_t *>(c->sel_host);
    uint64_t w0 = 0, w1 = 0;
    bool seen = false;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned i = 1;; ++i) {
        w0 = __atomic_load_n(&w[0], __ATOMIC_ACQUIRE);
        w1 = __atomic_load_n(&w[1], __ATOMIC_ACQUIRE);
        if ((uint32_t)(w0 >> 32) == seq && (uint32_t)(w1 >> 32) == seq) {
            seen = true;
            break;
        }
        if ((i & 1023u) == 0u &&
            std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(1000))
            break;
        __builtin_ia32_pause();
    }
    if (!seen) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        w0 = __atomic_load_n(&w[0], __ATOMIC_ACQUIRE);
        w1 = __atomic_load_n(&w[1], __ATOMIC_ACQUIRE);
        if ((uint32_t)(w0 >> 32) != seq || (uint32_t)(w1 >> 32) != seq)
            return fail(c, PLAN_EDEVICE, "selection result was not published");
    }
    if (best_k) *best_k = (int)(uint32_t)w0;
    if (best_cost) {
        const uint32_t bits = (uint32_t)w1;
        memcpy(best_cost, &bits, sizeof bits);
    }
    return PLAN_OK;
}

plan_status_t plan_select_sampled(plan_ctx *c, const plan_sample_t *spec, const float *cost_dev,
                                  int K, int N, int *best_k, float *best_cost, float *plan_dev) {
    if (!c) return PLAN_EINVAL;
    if (!cost_dev || !plan_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    plan::SampleArgs sa;
    plan_status_t st = sample_args(c, spec, sa);
    if (st != PLAN_OK) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    const bool want = best_k || best_cost;
    const uint32_t seq = want ? next_seq(c) : 0u;
    HIP_TRY(c, plan::launch_select_sampled(sa, cost_dev, K, N, c->veh.delta_rate_max, plan_dev,
                                           c->part_keys, c->counters, c->sel_dev,
                                           want ? c->sel_host : nullptr, seq, c->stream));
    return want ? wait_result(c, seq, best_k, best_cost) : PLAN_OK;
}

plan_status_t plan_rollout_est(plan_ctx *c, const float state0[7], const float *controls_dev,
                               int K, int N, float *cost_dev, float *final_state_dev) {
    if (!c) return PLAN_EINVAL;
    if (c->integ.method != PLAN_EULER)
        return fail(c, PLAN_EINVAL, "%s supports PLAN_EULER integration only", "plan_rollout_est");
    if (!state0 || !controls_dev || !cost_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (!finite_all(state0, 7)) return fail(c, PLAN_EINVAL, "state0 not finite");
    if (!c->has_terrain) return fail(c, PLAN_ENOTERRAIN, "no terrain set");
    RolloutArgs a;
    fill_args(c, a);
    for (int q = 0; q < 7; ++q) a.s0[q] = state0[q];
    a.controls = controls_dev;
    a.K = K;
    a.N = N;
    a.n0 = 0;
    a.n1 = N;
    a.finalize = 1;
    a.cost = cost_dev;
    a.final_state = final_state_dev;
    const int block = ((long long)K + 63) / 64 < 4096 ? 64 : 256;
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->timing) HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    // state (x, y, psi, v_y, omega_z, delta, v_x): one lane per candidate
    c->last_ordered = false;
    if (order_wanted(c, K, nullptr)) {
        const plan_status_t st = order_candidates(c, a, state0[5], state0[6]);
        if (st != PLAN_OK) return st;
    }
    HIP_TRY(c, plan::launch_rollout_est(a, block, c->stream));
    if (c->timing) {
        HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
        c->ev_recorded = true;
    }
    return PLAN_OK;
}

// Shared tail of the fused entry points: outputs of the epilogue, launch,
// optional wait for the host copy of (k*, J*).
static plan_status_t fused_launch(plan_ctx *c, RolloutArgs &a, bool sampled, float *plan_dev,
                                  int *best_k, float *best_cost) {
    const bool want = best_k || best_cost;
    a.sel_key = c->fused_key;
    a.sel_ticket = c->counters + 2;
    a.plan = plan_dev;
    a.sel_out = c->sel_dev;
    a.sel_out_host = want ? c->sel_host : nullptr;
    a.sel_seq = want ? next_seq(c) : 0u;
    plan_status_t st = launch(c, a, sampled ? Kind::fused_sampled : Kind::fused);
    if (st != PLAN_OK || !want) return st;
    return wait_result(c, a.sel_seq, best_k, best_cost);
}

plan_status_t plan_rollout_argmin(plan_ctx *c, const float state0[13], const float *controls_dev,
                                  int K, int N, float *cost_dev, float *final_state_dev,
                                  float *plan_dev, int *best_k, float *best_cost) {
    if (!c) return PLAN_EINVAL;
    if (c->integ.method != PLAN_EULER)
        return fail(c, PLAN_EINVAL, "%s supports PLAN_EULER integration only", "plan_rollout_argmin");
    if (!state0 || !controls_dev || !cost_dev || !plan_dev)
        return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (!finite_all(state0, 13)) return fail(c, PLAN_EINVAL, "state0 not finite");
    if (!c->has_terrain) return fail(c, PLAN_ENOTERRAIN, "no terrain set");
    RolloutArgs a;
    fill_args(c, a);
    for (int q = 0; q < 13; ++q) a.s0[q] = state0[q];
    a.controls = controls_dev;
    a.K = K;
    a.N = N;
    a.n0 = 0;
    a.n1 = N;
    a.finalize = 1;
    a.cost = cost_dev;
    a.final_state = final_state_dev;
    return fused_launch(c, a, false, plan_dev, best_k, best_cost);
}

plan_status_t plan_rollout_sampled_argmin(plan_ctx *c, const float state0[13],
                                          const plan_sample_t *spec, int K, int N,
                                          float *cost_dev, float *final_state_dev,
                                          float *plan_dev, int *best_k, float *best_cost) {
    if (!c) return PLAN_EINVAL;
    if (c->integ.method != PLAN_EULER)
        return fail(c, PLAN_EINVAL, "%s supports PLAN_EULER integration only", "plan_rollout_sampled_argmin");
    if (!state0 || !cost_dev || !plan_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (!finite_all(state0, 13)) return fail(c, PLAN_EINVAL, "state0 not finite");
    RolloutArgs a;
    fill_args(c, a);
    plan_status_t st = sample_args(c, spec, a.smp);
    if (st != PLAN_OK) return st;
    if (!c->has_terrain) return fail(c, PLAN_ENOTERRAIN, "no terrain set");
    for (int q = 0; q < 13; ++q) a.s0[q] = state0[q];
    a.controls = nullptr;
    a.K = K;
    a.N = N;
    a.n0 = 0;
    a.n1 = N;
    a.finalize = 1;
    a.cost = cost_dev;
    a.final_state = final_state_dev;
    return fused_launch(c, a, true, plan_dev, best_k, best_cost);
}

plan_status_t plan_smooth_terrain(plan_ctx *c, const float *height_dev, int W, int H, float res,
                                  float sigma, float *out_dev) {
    if (!c) return PLAN_EINVAL;
    if (!height_dev || !out_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (W < 1 || H < 1 || W > c->max_W || H > c->max_H)
        return fail(c, PLAN_EINVAL, "terrain size outside [1, max] in W or H");
    if (!(res > 0) || !isfinite(res) || !(sigma > 0) || !isfinite(sigma))
        return fail(c, PLAN_EINVAL, "res and sigma must be finite and > 0");
    // 3-sigma truncation; the 1e-6 node slack keeps decimal inputs such as
    // 0.3 m at 0.1 m on 9 nodes although they arrive rounded to float
    const double rr = ceil(3.0 * (double)sigma / (double)res - 1e-6);
    if (rr > plan::MAX_SMOOTH_RADIUS)
        return fail(c, PLAN_EINVAL, "sigma / res too large (3 sigma / res > 127 nodes)");
    plan::SmoothTaps taps;
    memset(&taps, 0, sizeof taps);
    taps.r = (int)rr;
    double g[2 * plan::MAX_SMOOTH_RADIUS + 1], sum = 0.0;
    for (int k = -taps.r; k <= taps.r; ++k) {
        const double d = k * (double)res;
        g[k + taps.r] = exp(-d * d / (2.0 * (double)sigma * sigma));
        sum += g[k + taps.r];
    }
    for (int k = 0; k <= 2 * taps.r; ++k) taps.w[k] = (float)(g[k] / sum);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, plan::launch_smooth(height_dev, W, H, taps, c->smooth_tmp, out_dev, c->stream));
    return PLAN_OK;
}

plan_status_t plan_costmap_polygons(plan_ctx *c, const float *verts_dev, int V, const int *offsets,
                                    const int *kinds, int P, int W, int H, float x0, float y0,
                                    float res, float sigma, float eps_dist, int accumulate,
                                    float *costmap_dev) {
    if (!c) return PLAN_EINVAL;
    if (!costmap_dev) return fail(c, PLAN_EINVAL, "costmap is NULL");
    if (P < 0 || P > plan::MAX_POLYGONS) return fail(c, PLAN_EINVAL, "P outside [0, 64]");
    if (P > 0 && (!verts_dev || !offsets || !kinds))
        return fail(c, PLAN_EINVAL, "NULL polygon array");
    if (W < 1 || H < 1) return fail(c, PLAN_EINVAL, "W and H must be >= 1");
    if (!(res > 0) || !isfinite(res) || !isfinite(x0) || !isfinite(y0) || !(eps_dist > 0) ||
        !isfinite(eps_dist) || !(sigma >= 0) || !isfinite(sigma))
        return fail(c, PLAN_EINVAL, "grid or cost parameters invalid");
    plan::PolygonSet ps;
    memset(&ps, 0, sizeof ps);
    ps.count = P;
    if (P > 0) {
        if (offsets[0] != 0) return fail(c, PLAN_EINVAL, "offsets[0] must be 0");
        for (int p = 0; p < P; ++p) {
            if (offsets[p + 1] - offsets[p] < 3)
                return fail(c, PLAN_EINVAL, "a polygon needs at least 3 vertices");
            if (kinds[p] != 0 && kinds[p] != 1)
                return fail(c, PLAN_EINVAL, "polygon kind must be 0 (obstacle) or 1 (boundary)");
            ps.offsets[p] = offsets[p];
            ps.kinds[p] = kinds[p];
        }
        if (offsets[P] != V) return fail(c, PLAN_EINVAL, "offsets[P] must equal V");
        ps.offsets[P] = offsets[P];
    }
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, plan::launch_costmap_polygons(verts_dev, ps, W, H, x0, y0, res, sigma, eps_dist,
                                             accumulate != 0, costmap_dev, c->stream));
    return PLAN_OK;
}

plan_status_t plan_init_state(plan_ctx *c, const float state0[13], float *state_dev,
                              float *cost_dev, int K) {
    if (!c) return PLAN_EINVAL;
    if (!state0 || !state_dev || !cost_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (!finite_all(state0, 13)) return fail(c, PLAN_EINVAL, "state0 not finite");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, plan::launch_init_state(state0, state_dev, cost_dev, K, c->stream));
    return PLAN_OK;
}

plan_status_t plan_rollout_chunk(plan_ctx *c, float *state_dev, float *cost_dev,
                                 const float *controls_dev, int K, int N, int n0, int n1,
                                 int finalize) {
    if (!c) return PLAN_EINVAL;
    if (!state_dev || !cost_dev || !controls_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (n0 < 0 || n1 < n0 || n1 > N) return fail(c, PLAN_EINVAL, "need 0 <= n0 <= n1 <= N");
    if (!c->has_terrain) return fail(c, PLAN_ENOTERRAIN, "no terrain set");
    RolloutArgs a;
    fill_args(c, a);
    a.controls = controls_dev;
    a.K = K;
    a.N = N;
    a.n0 = n0;
    a.n1 = n1;
    a.finalize = finalize != 0;
    a.cost = cost_dev;
    a.state = state_dev;
    return launch(c, a, Kind::chunk);
}

// Validation shared by plan_rollout_grad and plan_rollout_grad_noalloc;
// *need receives the workspace size in floats.
static plan_status_t grad_check(plan_ctx *c, const char *fn, const float *state0,
                                const float *controls_dev, int K, int N, int checkpoint_every,
                                const float *cost_dev, const float *grad_dev, size_t *need) {
    if (c->integ.method != PLAN_EULER)
        return fail(c, PLAN_EINVAL, "%s supports PLAN_EULER integration only", fn);
    if (!state0 || !controls_dev || !cost_dev || !grad_dev)
        return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (checkpoint_every < 1) return fail(c, PLAN_EINVAL, "checkpoint_every must be >= 1");
    if (!finite_all(state0, 13)) return fail(c, PLAN_EINVAL, "state0 not finite");
    if (!c->has_terrain) return fail(c, PLAN_ENOTERRAIN, "no terrain set");
    const int C = checkpoint_every < N ? checkpoint_every : N;
    const int nseg = (N + C - 1) / C;
    const size_t Kz = (size_t)K;
    *need = (size_t)(nseg + 1) * 13 * Kz                 // checkpoints
            + (size_t)C * c->integ.substeps * 14 * Kz;   // segment scratch
    return PLAN_OK;
}

// Forward pass with checkpoints, then the backward pass, on workspace ws
// (at least grad_check's *need floats; every float of it that is read is
// first written by the same call).
static plan_status_t grad_launch(plan_ctx *c, const float *state0, const float *controls_dev,
                                 int K, int N, const float *weight_dev, int checkpoint_every,
                                 float *cost_dev, float *grad_dev, float *ws) {
    const int C = checkpoint_every < N ? checkpoint_every : N;
    const int nseg = (N + C - 1) / C;
    float *ckpt = ws;
    float *seg = ckpt + (size_t)(nseg + 1) * 13 * (size_t)K;
    RolloutArgs a;
    fill_args(c, a);
    for (int q = 0; q < 13; ++q) a.s0[q] = state0[q];
    a.controls = controls_dev;
    a.K = K;
    a.N = N;
    a.n0 = 0;
    a.n1 = N;
    a.finalize = 1;
    a.cost = cost_dev;
    a.final_state = nullptr;
    a.ckpt = ckpt;
    a.ckpt_every = C;
    // forward pass in one launch, storing the state at every C-th interval
    int lanes, block;
    auto_launch(K, c->simds, &lanes, &block);
    if (c->lanes_opt) lanes = c->lanes_opt;
    if (c->block_opt) block = c->block_opt;
    c->last_lanes = lanes;
    c->last_block = block;
    HIP_TRY(c, plan::launch_rollout_ckpt(a, lanes, block, c->stream));
    // the backward kernel splits the wheels over the same lanes
    if (c->timing) HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    HIP_TRY(c, plan::launch_adjoint_backward(a, C, ckpt, weight_dev, seg, grad_dev, lanes,
                                             c->stream));
    if (c->timing) {
        HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
        c->ev_recorded = true;
    }
    return PLAN_OK;
}

plan_status_t plan_rollout_grad(plan_ctx *c, const float state0[13], const float *controls_dev,
                                int K, int N, const float *weight_dev, int checkpoint_every,
                                float *cost_dev, float *grad_dev) {
    if (!c) return PLAN_EINVAL;
    size_t need = 0;
    const plan_status_t st = grad_check(c, "plan_rollout_grad", state0, controls_dev, K, N,
                                        checkpoint_every, cost_dev, grad_dev, &need);
    if (st != PLAN_OK) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    if (need > c->gws_floats) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipFree(c->gws));
        c->gws = nullptr;
        c->gws_floats = 0;
        hipError_t e = hipMalloc(&c->gws, sizeof(float) * need);
        if (e != hipSuccess) {
            hip_fail(c, "hipMalloc(adjoint workspace)", e);
            return e == hipErrorOutOfMemory ? PLAN_ENOMEM : PLAN_EDEVICE;
        }
        c->gws_floats = need;
    }
    return grad_launch(c, state0, controls_dev, K, N, weight_dev, checkpoint_every, cost_dev,
                       grad_dev, c->gws);
}

plan_status_t plan_rollout_grad_noalloc(plan_ctx *c, const float state0[13],
                                        const float *controls_dev, int K, int N,
                                        const float *weight_dev, int checkpoint_every,
                                        float *cost_dev, float *grad_dev) {
    if (!c) return PLAN_EINVAL;
    size_t need = 0;
    const plan_status_t st = grad_check(c, "plan_rollout_grad_noalloc", state0, controls_dev, K,
                                        N, checkpoint_every, cost_dev, grad_dev, &need);
    if (st != PLAN_OK) return st;
    if (need > NOALLOC_FLOATS) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "workspace of %zu bytes exceeds the fixed %zu-byte workspace "
                 "(4 (13 K (ceil(N/C) + 1) + 14 K C S) bytes)",
                 need * sizeof(float), NOALLOC_FLOATS * sizeof(float));
        return fail(c, PLAN_EINVAL, "%s", buf);
    }
    float *ws = scratch_of(c->device);
    if (!ws) return fail(c, PLAN_EDEVICE, "fixed workspace not resolved on this device");
    HIP_TRY(c, hipSetDevice(c->device));
    return grad_launch(c, state0, controls_dev, K, N, weight_dev, checkpoint_every, cost_dev,
                       grad_dev, ws);
}

plan_status_t plan_select(plan_ctx *c, int mode, float lambda, const float *controls_dev,
                          const float *cost_dev, int K, int N, int *best_k, float *best_cost,
                          float *plan_dev) {
    if (!c) return PLAN_EINVAL;
    if (!controls_dev || !cost_dev || !plan_dev) return fail(c, PLAN_EINVAL, "NULL argument");
    if (K < 1 || K > c->max_K) return fail(c, PLAN_EINVAL, "K outside [1, max_K]");
    if (N < 1 || N > c->max_N) return fail(c, PLAN_EINVAL, "N outside [1, max_N]");
    if (mode != PLAN_ARGMIN && mode != PLAN_SOFTMIN) return fail(c, PLAN_EINVAL, "bad mode");
    if (mode == PLAN_SOFTMIN && !(lambda > 0 && isfinite(lambda)))
        return fail(c, PLAN_EINVAL, "softmin needs a finite lambda > 0");
    HIP_TRY(c, hipSetDevice(c->device));
    const bool want = best_k || best_cost;
    const uint32_t seq = want ? next_seq(c) : 0u;
    HIP_TRY(c, plan::launch_select(mode, lambda, controls_dev, cost_dev, K, N,
                                   c->veh.delta_rate_max, plan_dev, c->part_keys, c->counters,
                                   c->sel_dev, want ? c->sel_host : nullptr, seq,
                                   c->stream));
    return want ? wait_result(c, seq, best_k, best_cost) : PLAN_OK;
}

plan_status_t plan_set_launch(plan_ctx *c, int lanes, int block) {
    if (!c) return PLAN_EINVAL;
    if (!(lanes == 0 || lanes == 1 || lanes == 2 || lanes == 4))
        return fail(c, PLAN_EINVAL, "lanes must be 0, 1, 2 or 4");
    if (!(block == 0 || block == 64 || block == 256))
        return fail(c, PLAN_EINVAL, "block must be 0, 64 or 256");
    c->lanes_opt = lanes;
    c->block_opt = block;
    return PLAN_OK;
}

plan_status_t plan_set_order(plan_ctx *c, int mode) {
    if (!c) return PLAN_EINVAL;
    if (!(mode == PLAN_ORDER_AUTO || mode == PLAN_ORDER_OFF || mode == PLAN_ORDER_ON))
        return fail(c, PLAN_EINVAL, "order mode must be PLAN_ORDER_AUTO, _OFF or _ON");
    c->order_mode = mode;
    return PLAN_OK;
}

plan_status_t plan_get_order(const plan_ctx *c, int *ordered) {
    if (!c || !ordered) return PLAN_EINVAL;
    *ordered = c->last_ordered ? 1 : 0;
    return PLAN_OK;
}

plan_status_t plan_get_launch(const plan_ctx *c, int *lanes, int *block) {
    if (!c || !lanes || !block) return PLAN_EINVAL;
    *lanes = c->last_lanes;
    *block = c->last_block;
    return PLAN_OK;
}

plan_status_t plan_enable_timing(plan_ctx *c, int on) {
    if (!c) return PLAN_EINVAL;
    c->timing = on != 0;
    c->ev_recorded = false;
    return PLAN_OK;
}

plan_status_t plan_last_rollout_ms(plan_ctx *c, float *ms) {
    if (!c || !ms) return PLAN_EINVAL;
    if (!c->ev_recorded) return fail(c, PLAN_EINVAL, "no timed rollout recorded");
    HIP_TRY(c, hipEventSynchronize(c->ev1));
    HIP_TRY(c, hipEventElapsedTime(ms, c->ev0, c->ev1));
    return PLAN_OK;
}

void plan_destroy(plan_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    release(c);
    delete c;
}

const char *plan_last_error(const plan_ctx *c) {
    return c ? c->err.c_str() : g_create_err.c_str();
}

}  // extern "C"
