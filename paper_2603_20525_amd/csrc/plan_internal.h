// Internal declarations shared by the libplan sources (kernels and host ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/plan.h"
#include "sample.h"

namespace plan {

struct SelectOut {
    // (k*, J*) of a selection and, for the serving loop, the request's
    // status. Each of the first three 8-byte words also holds the sequence
    // number of the call that produced it, so a host polling the pinned copy
    // knows every value it reads is that call's (a naturally aligned 8-byte
    // store is never torn, but the record's two 16-byte stores may land in
    // either order).
    int best_k;
    uint32_t seq_k;
    float best_cost;
    uint32_t seq_cost;
    int32_t status;  // serving: 0, or the plan_status_t of the request
    uint32_t seq_status;
    uint32_t pad[2];
};

// Everything one rollout needs, passed by value as the kernel argument
// (a few hundred bytes, well inside the kernarg limit). All derived constants
// are computed once on the host in double precision and rounded to float.
struct RolloutArgs {
    // vehicle
    float invM;
    float invJxx, invJyy, invJzz;
    float dJyz, dJxz, dJxy;        // Jyy-Jzz, Jxx-Jzz, Jxx-Jyy
    float Lf, Lr, half_e, hR;
    float Lf_g, Lr_g, half_e_g, hR_g;  // the same lever arms in grid units (times 1 / res)
    float kf, kr, bf, br;
    float Fsf, Fsr;                // nominal tire loads (g/2) K_zz,f / K_zz,r
    float Mhalf;                   // M/2 (rear longitudinal constraint force)
    float C, mu, mu2;
    float delta_max, drate_max, g;
    float MgRbar, phibar;          // ESM: M g R_bar, phi_bar
    // extended single-track baseline: load-transfer coefficients K_zz,f,
    // K_zz,r, K_zx (kg), lateral-acceleration boundary and its normaliser
    float Kzzf, Kzzr, Kzx;
    float a_bar_y, inv_eps_ay;
    // cost
    float w_t, w_c, w_g;
    float goal_x, goal_y, goal_r2;
    float sigma, inv_eps_esm;
    // integration
    float h;                       // integration step dt / substeps
    float h_half, h_sixth;         // h / 2 and h / 6 (fourth-order Runge-Kutta)
    int S;                         // substeps per control
    int method;                    // 0 forward Euler, 1 fourth-order Runge-Kutta
    float accel_max, vx_min;
    // terrain: a W x H node grid stored as W x H cells, each the bilinear
    // coefficients of the four channels (h, f_x, f_y, cost) over the cell
    // (pack_tile; the last column and row are the grid's edge, constant
    // outward)
    const float4 *cells;
    int W, H;
    float x0, y0, inv_res;
    float x0_g, y0_g;              // x0 / res, y0 / res
    float umax, vmax;              // W-1, H-1 as floats (clamp-to-edge)
    int has_costmap;               // the cost channel is not all zero
    // problem
    float s0[13];
    const float *controls;         // [N][2][K]
    int K, N;
    int n0, n1;                    // control intervals simulated by this launch
    int finalize;                  // add the terminal cost, apply the non-finite rule
    float *cost;                   // [K]: written (full) or read-modify-written (chunk)
    float *final_state;            // full: [13][K] or nullptr
    float *state;                  // chunk: [13][K], read and written
    SampleArgs smp;                // sampled launches: the candidate generator
    // checkpointing launches (adjoint forward): ckpt [nseg+1][13][K] receives
    // the state at intervals 0, C, 2C, ... and the final state
    float *ckpt;
    int ckpt_every;
    // fused argmin epilogue: packed-key slot (all ones between launches),
    // arrival ticket (zero between launches), plan [N][2], result copies
    unsigned long long *sel_key;
    unsigned int *sel_ticket;
    float *plan;
    SelectOut *sel_out, *sel_out_host;
    uint32_t sel_seq;  // sequence number published with the host copy
    // one-lane full-horizon launches: lane i simulates candidate order[i]
    // (a permutation of 0..K-1), or candidate i if order is nullptr; with an
    // order, controls_lane (if not nullptr) holds the controls [N][2][K] in
    // lane order (column i = candidate order[i]), so the reads stay coalesced
    const int *order;
    const float *controls_lane;
};

// Locality order of a full-horizon rollout (order.hip): the candidates
// sorted by a kinematic proxy of their trajectories, so that each wave
// gathers from nearby terrain cells.
struct OrderArgs {
    int K, N;
    const float *controls;  // [N][2][K], or nullptr: drawn from smp
    SampleArgs smp;
    float dt, drate_max, delta_max, accel_max, vx_min;
    float inv_wheelbase, mu_g;  // 1 / (L_f + L_r), mu g
    float delta0, vx0;          // initial steering angle and forward speed
    // workspace (sized for the context's max_K)
    float *lat;                 // [4][lat_stride] proxy lateral offsets
    int lat_stride;             // max_K
    unsigned *range;            // [8] ordered-bits minimum (0..3) and maximum (4..7)
    unsigned *keys[2];          // [max_K] each
    int *vals[2];               // [max_K] each; vals[0] receives the order
    unsigned *hist;             // [256][tiles of K] digit counts, then per-digit offsets
    unsigned *dtotal;           // [256] digit totals of the current pass
    int nt_max;                 // order_tiles(max_K)
};

// Scatter tiles of the order's radix sort for K candidates.
int order_tiles(int max_K);
// Reset the range (once, after allocation; each order leaves it reset).
hipError_t launch_order_reset(const OrderArgs &o, hipStream_t s);
// Fourteen launches: proxy, keys, and four histogram + scan + scatter passes.
hipError_t launch_locality_order(const OrderArgs &o, hipStream_t s);
// out[n][c][i] = controls[n][c][order[i]] for the N intervals of K candidates.
hipError_t launch_permute_controls(const float *controls, const int *order, int K, int N,
                                   float *out, hipStream_t s);

// Bilinear coefficients of one channel over a cell with corner values a00,
// a10 (next column), a01 (next row), a11: the interpolant is
// c0 + c_x t_x + c_y t_y + c_xy t_x t_y with t_x, t_y in [0, 1].
__device__ __forceinline__ float4 bilinear_coefs(float a00, float a10, float a01, float a11) {
    const float dx0 = a10 - a00, dx1 = a11 - a01;
    return make_float4(a00, dx0, a01 - a00, dx1 - dx0);
}

// Cell (i, j), 0 <= i < W, 0 <= j < H, of the packed terrain: 64 bytes, the
// coefficients of h, f_x, f_y and cost over the square from node (i, j) to
// node (i+1, j+1), one float4 each; node values are the height, its slopes
// by central differences (one-sided on the border) and the costmap's rate.
// Interpolating within a cell then takes one contiguous load and three
// multiply-adds per channel. The cells of the last column (row) take node
// i+1 = i (j+1 = j): the interpolant there is constant along x (y), so a
// query clamped to the grid's edge lands in such a cell at weight 0 and
// reads the edge nodes exactly.
//
// One 16 x 16 tile of cells packed by a 256-thread workgroup: the heights
// of the tile's nodes and their neighbours are staged in LDS once, each
// node's values computed once, and the cells written as consecutive float4
// by consecutive lanes (one 1 KB row of the tile per wave and store).
constexpr int PACK_TILE = 16;

struct PackLds {
    float h[PACK_TILE + 3][PACK_TILE + 3];       // heights of nodes i0-1 .. i0+17 (clamped)
    float4 node[PACK_TILE + 1][PACK_TILE + 1];   // node values of nodes i0 .. i0+16 (clamped)
};

// Packs the cells (i0 .. i0+15, j0 .. j0+15) that lie inside the grid;
// returns false in a thread that found a non-finite node. Every thread of
// the workgroup must call it (it synchronises the workgroup).
__device__ inline bool pack_tile(const float *__restrict__ hgt, const float *__restrict__ cm,
                                 int W, int H, float inv_res, int i0, int j0,
                                 float4 *__restrict__ cells, PackLds &L) {
    constexpr int T = PACK_TILE;
    const int t = threadIdx.x;
    for (int q = t; q < (T + 3) * (T + 3); q += 256) {
        const int li = q % (T + 3), lj = q / (T + 3);
        const int gi = min(max(i0 - 1 + li, 0), W - 1), gj = min(max(j0 - 1 + lj, 0), H - 1);
        L.h[lj][li] = hgt[(size_t)gj * W + gi];
    }
    __syncthreads();
    bool ok = true;
    for (int q = t; q < (T + 1) * (T + 1); q += 256) {
        const int li = q % (T + 1), lj = q / (T + 1);
        const int gi = min(i0 + li, W - 1), gj = min(j0 + lj, H - 1);
        const int hi = gi - i0 + 1, hj = gj - j0 + 1;
        const float hc = L.h[hj][hi];
        float fx, fy;
        if (gi == 0)
            fx = (L.h[hj][hi + 1] - hc) * inv_res;
        else if (gi == W - 1)
            fx = (hc - L.h[hj][hi - 1]) * inv_res;
        else
            fx = (L.h[hj][hi + 1] - L.h[hj][hi - 1]) * (0.5f * inv_res);
        if (gj == 0)
            fy = (L.h[hj + 1][hi] - hc) * inv_res;
        else if (gj == H - 1)
            fy = (hc - L.h[hj - 1][hi]) * inv_res;
        else
            fy = (L.h[hj + 1][hi] - L.h[hj - 1][hi]) * (0.5f * inv_res);
        const float cc = cm ? cm[(size_t)gj * W + gi] : 0.0f;
        L.node[lj][li] = make_float4(hc, fx, fy, cc);
        ok = ok && isfinite(hc) && isfinite(cc);
    }
    __syncthreads();
    // float4 q of the tile: cell q / 4 (row-major in the tile), channel q % 4
    for (int q = t; q < T * T * 4; q += 256) {
        const int ch = q & 3, cl = q >> 2;
        const int ci = cl % T, cj = cl / T;
        const int i = i0 + ci, j = j0 + cj;
        if (i >= W || j >= H) continue;
        const float4 n00 = L.node[cj][ci], n10 = L.node[cj][ci + 1];
        const float4 n01 = L.node[cj + 1][ci], n11 = L.node[cj + 1][ci + 1];
        float4 c;
        if (ch == 0)
            c = bilinear_coefs(n00.x, n10.x, n01.x, n11.x);
        else if (ch == 1)
            c = bilinear_coefs(n00.y, n10.y, n01.y, n11.y);
        else if (ch == 2)
            c = bilinear_coefs(n00.z, n10.z, n01.z, n11.z);
        else
            c = bilinear_coefs(n00.w, n10.w, n01.w, n11.w);
        cells[4 * ((size_t)j * W + i) + ch] = c;
    }
    return ok;
}

// Cells of a W x H node grid, and the largest grid the 32-bit byte offsets
// of the cell loads can address.
__host__ __device__ inline long long terrain_cells(long long W, long long H) { return W * H; }
constexpr long long MAX_TERRAIN_CELLS = 1ll << 26;

// One tick of the serving loop: which slots advance through which control
// intervals, and which blocks of the launch belong to each slot.
constexpr int MAX_TICK_SLOTS = 128;

struct TickEntry {
    int slot;
    int block_start;
    int n0, n1;
    int finalize;
};

struct TickTable {
    int count;
    int total_blocks;
    TickEntry e[MAX_TICK_SLOTS];
};

// chunk = false: candidates start from s0 with zero cost. chunk = true:
// they continue from a.state / a.cost. Both run the same step code.
// one_wave (one lane per candidate only): use the kernels built for launches
// of at most one wave per SIMD (no four-wave register bound; forward Euler of
// one substep per interval requests each node's terrain a step ahead); the
// arithmetic, and so every result, is the same either way.
hipError_t launch_rollout(const RolloutArgs &a, int lanes, int block, bool chunk, hipStream_t s,
                          bool one_wave = false);

// Full-horizon rollout that also stores every candidate's state at each
// checkpoint (a.ckpt, a.ckpt_every): the adjoint's forward pass in one launch.
hipError_t launch_rollout_ckpt(const RolloutArgs &a, int lanes, int block, hipStream_t s);

// Full-horizon rollout whose last workgroup to finish also selects the argmin
// (a.sel_* and a.plan), with controls read (sampled = false) or drawn.
hipError_t launch_rollout_argmin(const RolloutArgs &a, int lanes, int block, bool sampled,
                                 hipStream_t s, bool one_wave = false);

// As launch_rollout (full horizon from a.s0) with the controls drawn in the
// kernel from a.smp instead of read from a.controls.
hipError_t launch_rollout_sampled(const RolloutArgs &a, int lanes, int block, hipStream_t s,
                                  bool one_wave = false);

// One-lane full-horizon launches of several Euler substeps per interval
// without a costmap, whose K is R whole rounds of one wave per SIMD (R = 1..3)
// plus a remainder of at most a quarter round: the remainder runs four lanes
// per candidate in the same launch (rollout_balanced). balanced_split returns
// the number of one-lane 64-thread workgroups, or 0 when K is not of that
// form. Plain or fused (argmin epilogue), materialised or sampled controls.
int balanced_split(long long K, int simds);
hipError_t launch_rollout_balanced(const RolloutArgs &a, int split, bool sampled, bool fused,
                                   hipStream_t s);

// controls [N][2][K] from the generator.
hipError_t launch_sample_controls(const SampleArgs &sa, int K, int N, float *controls,
                                  hipStream_t s);

// Extended single-track formulation (state [7]: x, y, psi, v_y, omega_z,
// delta, v_x): full horizon from a.s0[0..6]; a.final_state is [7][K].
hipError_t launch_rollout_est(const RolloutArgs &a, int block, hipStream_t s);

// Slots whose entry finalizes also select their plan in the same launch
// (fused argmin per slot): result, status and sequence number seq to
// ring[slot], plan to the slot's plan buffer; bad[slot] (non-finite terrain)
// is reported and cleared. s1: every slot has one substep per interval.
hipError_t launch_rollout_slots(const RolloutArgs *slots, const TickTable &t, int *bad,
                                SelectOut *ring, uint32_t seq, bool s1, int lanes, int block,
                                hipStream_t s);

// lanes: 1, 2 or 4 lanes per candidate (wheels split as in the forward).
hipError_t launch_adjoint_backward(const RolloutArgs &a, int C, const float *ckpt,
                                   const float *weight, float *scratch, float *grad, int lanes,
                                   hipStream_t s);

hipError_t launch_init_state(const float *s0, float *state, float *cost, int K, hipStream_t s);

// Packs the cells of a W x H grid (heights h, optional costmap c) into
// cells; *bad is set if any node is not finite.
hipError_t launch_pack_terrain(const float *h, const float *c, int W, int H, float inv_res,
                               float4 *cells, int *bad, hipStream_t s);

// Terrain preparation. Gaussian taps w[0 .. 2r] (normalised, FP32) of the
// separable level-of-detail kernel; r <= MAX_SMOOTH_RADIUS.
constexpr int MAX_SMOOTH_RADIUS = 127;

struct SmoothTaps {
    int r;
    float w[2 * MAX_SMOOTH_RADIUS + 1];
};

// Polygons of one costmap call: vertices offsets[p] .. offsets[p+1]-1 of the
// vertex array, kind 0 obstacle / 1 path boundary.
constexpr int MAX_POLYGONS = 64;

struct PolygonSet {
    int count;
    int offsets[MAX_POLYGONS + 1];
    int kinds[MAX_POLYGONS];
};

// Row pass into tmp, column pass into out (both [H][W]).
hipError_t launch_smooth(const float *h, int W, int H, const SmoothTaps &taps, float *tmp,
                         float *out, hipStream_t s);

hipError_t launch_costmap_polygons(const float *verts, const PolygonSet &ps, int W, int H,
                                   float x0, float y0, float res, float sigma, float eps,
                                   int accumulate, float *cm, hipStream_t s);

// Selection workspace sizes for a given maximum K / N.
int select_blocks(int K);

hipError_t launch_select(int mode, float lambda, const float *controls, const float *cost,
                         int K, int N, float drate_max, float *plan_out,
                         unsigned long long *part_keys, unsigned int *counters,
                         SelectOut *out, SelectOut *out_host, uint32_t seq, hipStream_t s);

// Argmin whose plan is the winner's sequence regenerated from the sampler.
hipError_t launch_select_sampled(const SampleArgs &sa, const float *cost, int K, int N,
                                 float drate_max, float *plan_out,
                                 unsigned long long *part_keys, unsigned int *counters,
                                 SelectOut *out, SelectOut *out_host, uint32_t seq,
                                 hipStream_t s);

// Host helpers shared by the plan and server entry points.
void fill_rollout_args(RolloutArgs &a, const plan_vehicle_t &v, const plan_cost_t &co,
                       const plan_integ_t &in, const float4 *cells, int W, int H, float x0,
                       float y0, float res);
double esm_level(const plan_vehicle_t &v);
bool finite_all(const float *p, int n);
bool valid_vehicle(const plan_vehicle_t &v);
bool valid_cost(const plan_cost_t &c);
bool valid_integ(const plan_integ_t &i);
// Launch shape for K candidates on a device of `simds` SIMDs: lanes per
// candidate and the workgroup size.
void auto_launch(long long K, int simds, int *lanes, int *block);

}  // namespace plan
