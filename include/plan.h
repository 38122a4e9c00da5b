/*
 * plan.h -- C ABI of libplan: the data-parallel hot path of the off-road
 * sampling MPC planner of "High-Speed, All-Terrain Autonomy: Ensuring Safety
 * at the Limits of Mobility" (arXiv 2603.20525), for AMD Instinct MI355X
 * (gfx950).
 *
 * One optimal-control problem (section "OCP Formulation", the problem solved
 * at each MPC iteration) is: given the most recent state estimate xi_0, a
 * heightmap f, a costmap of obstacle/path-boundary cost, a goal and the model
 * parameters, evaluate the cost J (eq. framework:cost) of each of K sampled
 * control sequences by forward-simulating the single-rigid-body (SRB) vehicle
 * model (section "Single Rigid Body Vehicle Dynamics Model", eq.
 * models:6dof:A), then return the sequence of minimal cost -- the "empirical
 * argmin" of section "Real-Time Implementation" -- or, optionally, the
 * MPPI-style weighted average of the sequences described beside it.
 *
 * Conventions shared by every call
 *   - Status: every call returns plan_status_t; 0 (PLAN_OK) on success and a
 *     negative code on failure. No call throws, aborts or exits. After a
 *     failure plan_last_error() returns a one-line description.
 *   - Device pointers (suffix _dev) are plain device addresses on the
 *     context's device, owned by the caller, FP32, contiguous, 4-byte aligned.
 *     Host pointers are ordinary process memory.
 *   - Asynchrony: plan_set_terrain, plan_rollout and plan_select enqueue work
 *     on the context's HIP stream and return without waiting, except where a
 *     call states that it synchronises.
 *   - Threads: a context is not thread-safe; independent contexts may be used
 *     concurrently from different threads on different streams.
 *   - Units: SI (m, s, kg, rad); costs in the paper's cost units.
 */
#ifndef PLAN_H
#define PLAN_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct plan_ctx plan_ctx; /* opaque, owned by the library */

typedef enum {
    PLAN_OK = 0,
    PLAN_EINVAL = -1,     /* invalid argument (NULL, size out of range, non-finite) */
    PLAN_ENOMEM = -2,     /* device or host allocation failed */
    PLAN_EDEVICE = -3,    /* a HIP runtime call or kernel launch failed */
    PLAN_ENOTERRAIN = -4  /* rollout before any successful plan_set_terrain */
} plan_status_t;

/* Vehicle parameters (appendix "Vehicle Model Parameters": model parameter
 * table and tire tables; notation table). hR = h + R, the CoM height above the
 * contact patches at rest. C, mu: sigmoid tire (eq. models:tire). delta_max:
 * steering angle limit; delta_rate_max: steering rate limit (the admissible
 * control set of section "OCP Formulation"). g: gravity (positive). */
typedef struct {
    float M, Jxx, Jyy, Jzz;
    float Lf, Lr, e, hR;
    float kf, kr, bf, br;
    float C, mu;
    float delta_max, delta_rate_max;
    float g;
} plan_vehicle_t;

/* Cost parameters (section "OCP Formulation"): running cost
 * L = w_t + w_c delta_dot^2 + L_soft, terminal cost w_g * distance to the goal
 * (goal_x, goal_y), goal radius goal_r ending the horizon early
 * (eq. formulation:goal). sigma and eps_esm normalise the ESM soft constraint
 * (L_soft term sigma * max(0, 1 - U_ESM / eps_esm)^2); eps_esm <= 0 selects
 * 10 % of the ESM on level ground. eps_dist is the distance normaliser used
 * when building a costmap; the rollout itself reads costmap cost rates. */
typedef struct {
    float w_t, w_c, w_g;
    float goal_x, goal_y, goal_r;
    float sigma, eps_esm, eps_dist;
    float eps_ay; /* lateral-acceleration normaliser of plan_rollout_est;
                   * <= 0 selects 10 % of a_bar_y = g e / (2 hR) */
} plan_cost_t;

/* Integration (sections "OCP Formulation" and "Real-Time Implementation"):
 * dt = zero-order-hold period of one control; substeps = integration steps
 * per control (step h = dt / substeps); accel_max maps the throttle
 * channel in [-1, 1] to the prescribed longitudinal acceleration vx_dot;
 * vx_min is the floor kept on the CoM longitudinal speed (the model assumes it
 * positive). */
typedef struct {
    float dt;
    int substeps;
    float accel_max;
    float vx_min;
    int method; /* PLAN_EULER (the paper's forward Euler) or PLAN_RK4 */
} plan_integ_t;

/* Integration method. PLAN_EULER: forward Euler, running cost by the left
 * Riemann sum at the Euler nodes. PLAN_RK4: the classical fourth-order
 * Runge-Kutta method the paper compared Euler against, applied to (state, J)
 * with J' = L and the control held over the step; the steering limit and the
 * speed floor apply to each completed step. PLAN_RK4 is available through
 * plan_rollout and plan_rollout_chunk; the other rollout calls, the adjoint,
 * the serving loop and the EST rollout accept PLAN_EULER only. */
enum { PLAN_EULER = 0, PLAN_RK4 = 1 };

enum { PLAN_ARGMIN = 0, PLAN_SOFTMIN = 1 };

/* Create a context on the current HIP device. max_K, max_N, max_W, max_H bound
 * the sizes later calls may use; the library allocates its workspace for them
 * once here (terrain cells 64*max_W*max_H bytes: each cell of the grid
 * holds the bilinear coefficients of height, slopes and cost over it;
 * the candidate-order workspace about 32*max_K bytes, plus selection
 * scratch).
 * hip_stream is a hipStream_t, or NULL for the default stream.
 * Errors: PLAN_EINVAL for NULL pointers, non-positive sizes, a terrain grid
 * of max_W*max_H >= 2^26 nodes, or invalid parameters (M, J, Lf+Lr, e,
 * hR, dt <= 0, substeps < 1, non-finite values); PLAN_ENOMEM; PLAN_EDEVICE.
 * *out is set only on success. */
plan_status_t plan_create(plan_ctx **out, const plan_vehicle_t *veh,
                          const plan_cost_t *cost, const plan_integ_t *integ,
                          int max_K, int max_N, int max_W, int max_H,
                          void *hip_stream);

/* Replace the stream later calls enqueue on (a hipStream_t, NULL = default). */
plan_status_t plan_set_stream(plan_ctx *ctx, void *hip_stream);

/* Replace the cost parameters (e.g. a new goal for the next MPC iteration). */
plan_status_t plan_set_cost(plan_ctx *ctx, const plan_cost_t *cost);

/* Upload a terrain (the heightmap f of assumption A1; slopes f_x, f_y by
 * numerical first derivatives as the models require; costmap per section
 * "Real-Time Implementation", pre-computed distance cost interpolated at run
 * time). height_dev is [H][W] FP32, node (i, j) at (x0 + i*res, y0 + j*res),
 * row j contiguous. costmap_dev is [H][W] FP32 cost units per second at each
 * node, or NULL for zero. The library packs both into its own cell grid, so
 * the caller may reuse the buffers once the stream has passed this call.
 * Synchronises the stream (once per terrain, off the per-plan path) to check
 * the data. Errors: PLAN_EINVAL for NULL height, W or H < 2 or above the
 * create-time maxima, res <= 0, or any non-finite height or cost (the previous
 * terrain is then no longer valid); PLAN_EDEVICE. */
plan_status_t plan_set_terrain(plan_ctx *ctx, const float *height_dev, int W, int H,
                               float x0, float y0, float res,
                               const float *costmap_dev);

/* Terrain level-of-detail smoothing (section "Terrain Smoothing": the
 * models need terrain smooth at their own length scale; the paper smooths
 * with a Gaussian of standard deviation 0.3 m for the SRB model and 1.5 m for
 * the extended single-track model). out_dev [H][W] receives height_dev
 * [H][W] convolved with the Gaussian exp(-d^2 / (2 sigma^2)) over the square
 * of half-width r = ceil(3 sigma / res - 1e-6) nodes, normalised to sum 1, nodes
 * beyond the grid taking the nearest edge value. out_dev may equal
 * height_dev. Asynchronous. Errors: PLAN_EINVAL (NULL pointers, W or H
 * outside [1, max], res or sigma not finite and > 0, r > 127); PLAN_EDEVICE. */
plan_status_t plan_smooth_terrain(plan_ctx *ctx, const float *height_dev, int W, int H,
                                  float res, float sigma, float *out_dev);

/* Costmap of the distance constraints (section "OCP Formulation": signed
 * distances between each wheel and each obstacle or path-boundary
 * perimeter; section "Real-Time Implementation": pre-computed and summed for
 * all features into a costmap interpolated at run time). costmap_dev [H][W]
 * (node (i, j) at (x0 + i res, y0 + j res)) receives, or with accumulate != 0
 * has added to it, sum_p sigma * max(0, 1 - sdist_p / eps_dist)^2, where
 * sdist_p is the signed distance from the node to polygon p: negative inside
 * an obstacle (kind 0), negative outside a path boundary (kind 1); inside is
 * the even-odd rule. Polygon p is vertices offsets[p] .. offsets[p+1]-1 of
 * verts_dev ([V][2] FP32 x, y on the device), implicitly closed.
 * offsets ([P+1], offsets[0] = 0, offsets[P] = V, at least 3 vertices each)
 * and kinds ([P]) are host arrays; P <= 64 per call (accumulate for more).
 * Errors: PLAN_EINVAL (NULL pointers, bad offsets or kinds, P outside
 * [0, 64], W or H < 1, res or eps_dist <= 0, sigma < 0); PLAN_EDEVICE. */
plan_status_t plan_costmap_polygons(plan_ctx *ctx, const float *verts_dev, int V,
                                    const int *offsets, const int *kinds, int P, int W, int H,
                                    float x0, float y0, float res, float sigma,
                                    float eps_dist, int accumulate, float *costmap_dev);

/* Roll out K candidates for N zero-order-hold intervals of `substeps` Euler
 * steps each and write their costs (eq. framework:cost, horizon ended early
 * at the goal per eq. formulation:goal).
 *   state0:          host, 13 floats in the order of eq. models:6dof:state:
 *                    x, y, z, psi, theta, phi, vx, vy, vz, wx, wy, wz, delta
 *                    (3-2-1 Euler angles, body-frame velocities).
 *   controls_dev:    [N][2][K]: channel 0 steering rate (rad/s), channel 1
 *                    throttle in [-1, 1]; both are clamped to the admissible
 *                    set before use.
 *   cost_dev:        [K] output; +inf for a candidate whose cost or final
 *                    state is not finite.
 *   final_state_dev: [13][K] output (state at the horizon end or goal exit),
 *                    or NULL.
 * Errors: PLAN_EINVAL (NULL ctx/state0/controls/cost, K not in [1, max_K], N
 * not in [1, max_N], non-finite state0); PLAN_ENOTERRAIN; PLAN_EDEVICE. */
plan_status_t plan_rollout(plan_ctx *ctx, const float state0[13],
                           const float *controls_dev, int K, int N,
                           float *cost_dev, float *final_state_dev);

/* plan_rollout for the extended single-track (EST) baseline formulation the
 * paper compares against (appendix "Extended Single-Track Vehicle Dynamics
 * Model"; lateral-acceleration constraint of section "OCP Formulation"): a
 * planar single-track model on the plane tangent to the terrain under the
 * CoM, roll and pitch taken from that plane's normal, normal loads by load
 * transfer, the same sigmoid tire on a front and a rear virtual tire, and the
 * soft constraint sigma * max(0, 1 + pi_ay / eps_ay)^2 with
 * pi_ay = |a_y - g_y| - a_bar_y, a_bar_y = M g / (2 K_zy) = g e / (2 hR), in
 * place of the ESM term. Same controls, cost terms (costmap at the four
 * wheels), goal rule, clamps and +inf rule as plan_rollout.
 *   state0:          host, 7 floats in the order of eq. models:3dof:state:
 *                    x, y, psi, v_y, omega_z, delta, v_x.
 *   final_state_dev: [7][K] or NULL.
 * Uses M, Jzz, Lf, Lr, e, hR, C, mu and the limits of the vehicle (not Jxx,
 * Jyy or the suspension). Errors: as plan_rollout. */
plan_status_t plan_rollout_est(plan_ctx *ctx, const float state0[7],
                               const float *controls_dev, int K, int N,
                               float *cost_dev, float *final_state_dev);

/* Resumable form of plan_rollout, for callers that advance candidates a few
 * control intervals at a time (a serving loop interleaving requests, or a
 * backward pass recomputing from checkpoints). state_dev [13][K] and
 * cost_dev [K] hold each candidate's state (order of plan_rollout's state0)
 * and running cost; this call advances them in place through control
 * intervals n0 .. n1-1 of controls_dev [N][2][K]. finalize != 0 adds the
 * terminal cost and applies the +inf rule, as at the end of plan_rollout. A
 * candidate that reached the goal stays frozen (its next goal test fires
 * again). plan_init_state followed by chunks covering [0, N) with finalize on
 * the last gives bit-identical costs and states to one plan_rollout.
 * Errors: PLAN_EINVAL (NULL pointers, K or N out of range, not
 * 0 <= n0 <= n1 <= N); PLAN_ENOTERRAIN; PLAN_EDEVICE. */
plan_status_t plan_rollout_chunk(plan_ctx *ctx, float *state_dev, float *cost_dev,
                                 const float *controls_dev, int K, int N, int n0, int n1,
                                 int finalize);

/* Gradient of each candidate's cost with respect to its controls, by a
 * hand-written reverse pass through the forward-Euler rollout (gradient
 * refinement of sampled candidates; the paper's optimiser is sampling-only,
 * section "Real-Time Implementation").
 *   controls_dev [N][2][K] as for plan_rollout;
 *   weight_dev   [K] seeds w_k (the result is w_k dJ_k/du_k), or NULL for 1;
 *   checkpoint_every: the forward pass stores every candidate's state every
 *                this many control intervals; the backward pass recomputes
 *                one such segment at a time (memory O(N/C + C) states);
 *   cost_dev     [K] output: the costs, as plan_rollout computes them;
 *   grad_dev     [N][2][K] output: dJ/du for the raw controls (zero where a
 *                control lies outside the admissible set and is clamped, zero
 *                after the goal exit, zero rows for a +inf candidate).
 * Non-smooth points take the derivative of the branch the forward pass took.
 * The backward kernel splits each candidate's wheels over 1, 2 or 4 lanes
 * (the automatic choice of plan_rollout, or the lanes set by
 * plan_set_launch); the result is bit-identical for every choice.
 * The forward pass is one launch that stores the checkpoints; the backward
 * pass is a second. The library grows an internal workspace of
 * 4*(13 K (ceil(N/C) + 1) + 14 K C S) bytes when a call needs more than the
 * previous ones (may synchronise the stream then).
 * Errors: PLAN_EINVAL, PLAN_ENOTERRAIN, PLAN_ENOMEM, PLAN_EDEVICE. */
plan_status_t plan_rollout_grad(plan_ctx *ctx, const float state0[13],
                                const float *controls_dev, int K, int N,
                                const float *weight_dev, int checkpoint_every,
                                float *cost_dev, float *grad_dev);

/* plan_rollout_grad without any allocation, for callers that cannot allocate
 * device memory inside a call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Arguments, outputs and results are
 * those of plan_rollout_grad (same kernels, bit-identical outputs), but the
 * checkpoints and segment states live in a fixed workspace of 16 MiB per GPU
 * inside the library (held until the process ends) instead of the context's
 * growing one: the call needs 4*(13 K (ceil(N/C) + 1) + 14 K C S) <= 16 MiB,
 * with C = min(checkpoint_every, N) and S the context's substeps (e.g. K =
 * 4096 candidates at N = 100, C = 10, S = 1 use 4.6 MiB). The workspace is
 * shared by every call on that GPU, from any context or stream: calls that
 * overlap on one GPU race and must be serialised by the caller. Nothing in
 * it needs clearing between calls (each call writes what it reads).
 * Errors: those of plan_rollout_grad except PLAN_ENOMEM; PLAN_EINVAL also
 * when the workspace would exceed 16 MiB. */
plan_status_t plan_rollout_grad_noalloc(plan_ctx *ctx, const float state0[13],
                                        const float *controls_dev, int K, int N,
                                        const float *weight_dev, int checkpoint_every,
                                        float *cost_dev, float *grad_dev);

/* Fill state_dev [13][K] with state0 (host, 13 floats) for every candidate
 * and cost_dev [K] with zero, on the context's stream.
 * Errors: PLAN_EINVAL (NULL pointers, K out of range, non-finite state0). */
plan_status_t plan_init_state(plan_ctx *ctx, const float state0[13], float *state_dev,
                              float *cost_dev, int K);

/* Select over the K candidates of a rollout (section "Real-Time
 * Implementation"). mode PLAN_ARGMIN: the lowest index k* of minimal finite
 * cost; plan_dev [N][2] receives candidate k*'s clamped controls. mode
 * PLAN_SOFTMIN: MPPI-style average, weights exp(-(J_k - J_min) / lambda) over
 * finite costs (lambda > 0); plan_dev receives the weighted mean of the
 * clamped controls, and best_k / best_cost still report the argmin.
 * If no cost is finite, best_k = -1, best_cost = +inf, plan_dev is zeroed and
 * the status is still PLAN_OK.
 * best_k and best_cost are host pointers; if either is non-NULL the call
 * waits until the kernel has published them into pinned host memory (it
 * polls that memory briefly, then synchronises the stream). The device
 * outputs (plan_dev) are ordered on the context's stream like every other
 * launch: read them through that stream, or synchronise it first. Pass both
 * NULL to stay asynchronous.
 * Errors: PLAN_EINVAL (NULL ctx/controls/cost/plan, K or N out of range, bad
 * mode, lambda <= 0 for SOFTMIN); PLAN_EDEVICE. */
plan_status_t plan_select(plan_ctx *ctx, int mode, float lambda,
                          const float *controls_dev, const float *cost_dev,
                          int K, int N, int *best_k, float *best_cost,
                          float *plan_dev);

/* On-device candidate sampling (section "Real-Time Implementation": the
 * candidate control sequences are drawn on the GPU by a counter-based
 * generator; the published configuration draws the steering rate uniformly
 * in [-1, 1] rad/s and holds the longitudinal acceleration at zero).
 *
 * Generator: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011). Candidate k at control interval n
 * uses the 64-bit word n mod 4 of the output block for counter
 * (k, n div 4, 0, 0) and key (seed, stream); its bits 40..63 give a and bits
 * 16..39 give b (24-bit integers).
 *   PLAN_SAMPLE_UNIFORM:  u_c = nominal_c + scale_c (2 x_c - 1), x_0 = a/2^24,
 *                         x_1 = b/2^24;
 *   PLAN_SAMPLE_GAUSSIAN: u_c = nominal_c + scale_c z_c, with the Box-Muller
 *                         pair z_0 = r cos(2 pi q), z_1 = r sin(2 pi q),
 *                         r = sqrt(-2 ln p), p = (a+1)/2^24, q = b/2^24.
 * keep_nominal != 0 makes candidate 0 the nominal sequence itself.
 * nominal_dev is [N][2] FP32 on the device (steering rate, throttle) or NULL
 * for zeros; it must stay valid until the calls using it have run. The raw
 * u are what plan_rollout would read from controls_dev: they are clamped to
 * the admissible set when applied. A sequence depends only on (seed, stream,
 * k, n), so any call with the same spec and N sees the same candidates. */
enum { PLAN_SAMPLE_UNIFORM = 0, PLAN_SAMPLE_GAUSSIAN = 1 };

typedef struct {
    int kind;                  /* PLAN_SAMPLE_UNIFORM or PLAN_SAMPLE_GAUSSIAN */
    int keep_nominal;
    unsigned long long seed;   /* key word 0 */
    unsigned long long stream; /* key word 1 (e.g. the MPC iteration) */
    float scale[2];            /* half-width (uniform) or std (Gaussian), >= 0 */
    const float *nominal_dev;  /* [N][2] or NULL */
} plan_sample_t;

/* Write the sampled candidates to controls_dev [N][2][K] (the layout
 * plan_rollout reads). Errors: PLAN_EINVAL (NULL ctx/spec/controls, K or N
 * out of range, unknown kind, negative or non-finite scale); PLAN_EDEVICE. */
plan_status_t plan_sample_controls(plan_ctx *ctx, const plan_sample_t *spec, int K, int N,
                                   float *controls_dev);

/* plan_rollout with the candidates drawn inside the rollout kernel instead of
 * read from memory (no [N][2][K] array exists). Costs and final states are
 * bit-identical to plan_sample_controls followed by plan_rollout.
 * Errors: as plan_rollout, plus the spec errors of plan_sample_controls. */
plan_status_t plan_rollout_sampled(plan_ctx *ctx, const float state0[13],
                                   const plan_sample_t *spec, int K, int N,
                                   float *cost_dev, float *final_state_dev);

/* Argmin selection (as plan_select with PLAN_ARGMIN) over costs produced from
 * spec: plan_dev [N][2] receives the winner's clamped controls, regenerated
 * from the generator. Host outputs and synchronisation as plan_select.
 * Errors: PLAN_EINVAL (NULL ctx/spec/cost/plan, K or N out of range, bad
 * spec); PLAN_EDEVICE. */
plan_status_t plan_select_sampled(plan_ctx *ctx, const plan_sample_t *spec,
                                  const float *cost_dev, int K, int N, int *best_k,
                                  float *best_cost, float *plan_dev);

/* plan_rollout followed by plan_select(PLAN_ARGMIN), in ONE kernel launch:
 * the rollout kernel's last workgroup to finish reduces the candidates'
 * costs and writes the plan, so a plan costs one launch and (optionally) one
 * wait. cost_dev, final_state_dev and plan_dev receive bit-identical values
 * to the two-call sequence; best_k / best_cost (host, NULL to stay
 * asynchronous) as plan_select, written by the kernel into pinned memory.
 * Calls on one context must not overlap (they share the context's reduction
 * slot), which the single stream of a context already guarantees.
 * Errors: as plan_rollout, plus PLAN_EINVAL for a NULL plan_dev. */
plan_status_t plan_rollout_argmin(plan_ctx *ctx, const float state0[13],
                                  const float *controls_dev, int K, int N,
                                  float *cost_dev, float *final_state_dev,
                                  float *plan_dev, int *best_k, float *best_cost);

/* plan_rollout_sampled followed by plan_select_sampled, in one launch (the
 * winner's sequence is regenerated from spec for plan_dev). The paper's
 * configuration end to end: candidates drawn, simulated, scored and reduced
 * without any [N][2][K] array in memory. Errors: as plan_rollout_sampled,
 * plus PLAN_EINVAL for a NULL plan_dev. */
plan_status_t plan_rollout_sampled_argmin(plan_ctx *ctx, const float state0[13],
                                          const plan_sample_t *spec, int K, int N,
                                          float *cost_dev, float *final_state_dev,
                                          float *plan_dev, int *best_k, float *best_cost);

/* Launch shape of the rollout kernel: lanes per candidate (1, 2 or 4; the
 * four wheels are split over the lanes) and workgroup size (64 or 256).
 * 0 restores the automatic choice. Results are identical for every shape up
 * to FP32 rounding of the wheel sums' evaluation order, which is fixed. */
plan_status_t plan_set_launch(plan_ctx *ctx, int lanes, int block);

/* Launch shape chosen for the most recent rollout. */
plan_status_t plan_get_launch(const plan_ctx *ctx, int *lanes, int *block);

/* Candidate order of full-horizon rollouts (plan_rollout, plan_rollout_est,
 * plan_rollout_sampled, plan_rollout_argmin, plan_rollout_sampled_argmin).
 * Gather locality, not the paper: a wave of one-lane candidates gathers the
 * terrain cells under 64 different vehicles each step, and when the candidates are
 * far apart the texture path rather than arithmetic limits the rollout. With
 * ordering, the library first sorts the candidates by a kinematic proxy of
 * their trajectories (single-track kinematics under the model's control
 * limits and a friction-limited curvature; lateral offsets at four times of
 * the horizon, Morton-interleaved, stable radix sort; fourteen small
 * launches on the context's stream) and runs each wave on neighbouring
 * candidates, one lane per candidate (plan_set_launch's lane count applies
 * to unordered launches, its workgroup size to both); materialised
 * controls are first gathered into lane order (a buffer of 2 N K floats
 * that the context grows on demand; without it the controls are read in
 * place, with the same results). Only the
 * assignment of candidates to lanes changes: every output is bit-identical
 * with and without ordering. Ordering pays when the candidates of a wave
 * spread far apart and the steps are texture-bound, as with the paper's
 * configuration (uniform steering-rate samples, 50 Euler substeps per
 * control); with one substep per control it was slower, with uniform and
 * with Gaussian draws. Modes: PLAN_ORDER_AUTO (default: launches that draw
 * uniform samples in the kernel with at least 8 substeps per control, from
 * 49 152 candidates on), PLAN_ORDER_OFF,
 * PLAN_ORDER_ON (every full-horizon launch). Errors: PLAN_EINVAL for another
 * mode. plan_get_order reports whether the most recent full-horizon rollout
 * was ordered (1) or not (0). */
enum { PLAN_ORDER_AUTO = 0, PLAN_ORDER_OFF = 1, PLAN_ORDER_ON = 2 };
plan_status_t plan_set_order(plan_ctx *ctx, int mode);
plan_status_t plan_get_order(const plan_ctx *ctx, int *ordered);

/* Kernel timing: when enabled, HIP events bracket each rollout kernel on the
 * context's stream (for plan_rollout_grad and plan_rollout_grad_noalloc, the
 * backward kernel); plan_last_rollout_ms waits for the end event and returns
 * the kernel's elapsed time in milliseconds. */
plan_status_t plan_enable_timing(plan_ctx *ctx, int on);
plan_status_t plan_last_rollout_ms(plan_ctx *ctx, float *ms);

/* Release everything the context owns. NULL is ignored. Waits for the
 * context's stream first. */
void plan_destroy(plan_ctx *ctx);

/* Description of the most recent failure on ctx ("" if none). With ctx NULL,
 * the description of the most recent failed plan_create in this process. The
 * string stays valid until the next call on ctx. */
const char *plan_last_error(const plan_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PLAN_H */
