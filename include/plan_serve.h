/*
 * plan_serve.h -- continuous-batching planning server on top of libplan.
 *
 * The planner of arXiv 2603.20525 answers one optimal-control problem per MPC
 * iteration (section "OCP Formulation"; the closed loop of section "Plant
 * Co-Simulator" asks for a new plan every 40 ms). A server holding many such
 * planners receives problems of different sizes at unpredictable times. This
 * interface batches them: every admitted request occupies a device-resident
 * slot (its terrain cells, candidate states and running costs stay in HBM
 * between launches); each scheduling step launches ONE rollout kernel that
 * advances the candidates of every active slot by a few control intervals
 * and, in the same launch, selects the plans of the slots that finish.
 * Requests arriving while
 * others run join at the next step, as slots and the memory budget allow.
 * Each request's result is bit-identical to plan_rollout + plan_select on the
 * same inputs (same kernels, same arithmetic).
 *
 * Conventions are those of plan.h (status codes, caller-owned FP32 device
 * buffers, no exceptions). A server is not thread-safe: one host thread
 * submits, steps and polls.
 */
#ifndef PLAN_SERVE_H
#define PLAN_SERVE_H

#include "plan.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct plan_server plan_server; /* opaque, owned by the library */

/* One planning request. All device buffers are caller-owned and must stay
 * valid (and unmodified) until the request is reported done.
 *   height_dev  [H][W] heights, node (i, j) at (x0 + i*res, y0 + j*res);
 *   costmap_dev [H][W] cost rate or NULL;
 *   state0      initial state (host copy taken at submit), order of
 *               plan_rollout;
 *   controls_dev [N][2][K] candidate controls as for plan_rollout;
 *   cost, integ  per-request cost and integration parameters;
 *   plan_dev    [N][2] output: the argmin candidate's clamped controls;
 *   cost_dev    [K] output or NULL: every candidate's cost J_k (eq.
 *               framework:cost, +inf for a non-finite candidate), copied
 *               from the slot on the server's stream right after the launch
 *               that finishes the request. */
typedef struct {
    const float *height_dev;
    int W, H;
    float x0, y0, res;
    const float *costmap_dev;
    float state0[13];
    const float *controls_dev;
    int K, N;
    plan_cost_t cost;
    plan_integ_t integ;
    float *plan_dev;
    float *cost_dev;
} plan_request_t;

/* State of one request. Times are seconds on the server's monotonic clock
 * (plan_server_now). t_done is when plan_server_step first observed the
 * result on the host: the kernel publishes (k*, J*) into pinned memory, and
 * the host sees it there before the launch has completed. The request's
 * plan_dev is written by that same launch (and cost_dev by a copy right after
 * it), so read them through the server's stream (or after plan_server_drain,
 * which completes all device work). */
typedef struct {
    int status;       /* 0 pending, 1 done, < 0: plan_status_t of a failure */
    int best_k;       /* as plan_select; -1 if no candidate is finite */
    float best_cost;
    int slot;         /* slot used, -1 while queued */
    double t_submit, t_admit, t_done;
} plan_result_t;

/* Create a server on the current device. max_slots (<= 128) requests may be
 * resident at once, each with K <= max_K, N <= max_N, W <= max_W, H <= max_H
 * (max_W*max_H below 2^26).
 * A request's footprint is 64*W*H (terrain cells) + 56*K (state, cost) + 8*K*N
 * (controls) + 8*N (plan) bytes; a request is admitted only while the summed
 * footprint of resident requests stays within budget_bytes.
 * chunk_intervals (>= 1) is how many control intervals one step advances
 * while requests are waiting (for a slot or for memory), so that waiting
 * requests join after a short launch; when nothing waits, a step runs every
 * resident request to the end of its horizon.
 * Errors: PLAN_EINVAL, PLAN_ENOMEM, PLAN_EDEVICE. */
plan_status_t plan_server_create(plan_server **out, const plan_vehicle_t *veh, int max_slots,
                                 int max_K, int max_N, int max_W, int max_H,
                                 unsigned long long budget_bytes, int chunk_intervals,
                                 void *hip_stream);

/* Queue a request (FIFO). *id receives its handle. Nothing is launched until
 * the next plan_server_step. Errors: PLAN_EINVAL for NULL pointers, sizes
 * outside the create-time maxima, invalid parameters, non-finite state0, or
 * a footprint larger than the whole budget. */
plan_status_t plan_server_submit(plan_server *s, const plan_request_t *req, int *id);

/* One scheduling step: retire finished steps, admit queued requests, and
 * enqueue one rollout launch over all resident requests (plus the selects of
 * those that finish with it). Waits for the GPU only when two earlier steps
 * are still in flight. *active / *queued (optional) receive the number of
 * resident and waiting requests after the step. */
plan_status_t plan_server_step(plan_server *s, int *active, int *queued);

/* Step until every submitted request is done, then wait for the server's
 * stream, so every plan buffer is written on return. */
plan_status_t plan_server_drain(plan_server *s);

/* Resident requests, queued requests and bytes of budget in use (their summed
 * footprint) right now; any output pointer may be NULL. */
plan_status_t plan_server_stats(const plan_server *s, int *active, int *queued,
                                unsigned long long *used_bytes);

/* Copy the state of request id into *out. */
plan_status_t plan_server_result(const plan_server *s, int id, plan_result_t *out);

/* Completion queue: move up to capacity ids of requests that finished (done
 * or failed) since the previous call into ids[], in the order the host
 * observed them (plan_server_step and plan_server_drain observe them);
 * *count receives how many were moved. Ids not moved stay queued for the
 * next call. Errors: PLAN_EINVAL for NULL s or count, NULL ids with
 * capacity > 0, or capacity < 0. */
plan_status_t plan_server_completions(plan_server *s, int *ids, int capacity, int *count);

/* Seconds on the server's monotonic clock (the clock of the timestamps). */
double plan_server_now(const plan_server *s);

/* Release everything the server owns (waits for its stream). NULL is ignored. */
void plan_server_destroy(plan_server *s);

/* Description of the most recent failure on s ("" if none); with s NULL, of
 * the most recent failed plan_server_create. */
const char *plan_server_last_error(const plan_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PLAN_SERVE_H */
