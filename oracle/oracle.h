/*
 * FP64 CPU oracle for the single-rigid-body (SRB) sampling planner.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the correctness reference that the
 * GPU path is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no source, header, table or helper with the GPU library.
 *
 * What it computes (paper: "Proposed MPC Formulation" and "Real-Time
 * Implementation"): for K given candidate control sequences, the forward-Euler
 * rollout of the SRB model over a gridded heightmap, the running cost with the
 * energy-stability-margin (ESM) soft constraint and the costmap term, the
 * terminal distance cost, and the selection over candidates (empirical argmin,
 * or the MPPI-style weighted average).
 *
 * All internal arithmetic is double precision. Inputs that the GPU path also
 * receives (heights, costmap, controls, initial state) are taken as float
 * arrays and promoted, so both sides start from identical bits.
 */
#ifndef SRB_ORACLE_H
#define SRB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Vehicle parameters (paper, appendix "Vehicle Model Parameters", tables
 * of model and tire parameters; notation table). hR is h+R. */
typedef struct {
    double M, Jxx, Jyy, Jzz;
    double Lf, Lr, e, hR;
    double kf, kr, bf, br;
    double C, mu;
    double delta_max, delta_rate_max;
    double g;
} oracle_vehicle;

/* Cost parameters (paper, "OCP Formulation": running/terminal cost, soft
 * constraints, goal radius). eps_esm <= 0 selects the default: 10 % of the
 * ESM on level ground. */
typedef struct {
    double w_t, w_c, w_g;
    double goal_x, goal_y, goal_r;
    double sigma, eps_esm, eps_dist;
    double eps_ay; /* lateral-acceleration normaliser; <= 0: 10 % of a_bar_y */
} oracle_cost;

/* Integration: dt is the zero-order-hold period of one control, substeps is
 * the number of Euler steps per control (h = dt/substeps), accel_max maps the
 * normalised throttle channel to the prescribed longitudinal acceleration,
 * vx_min is the floor kept on the CoM longitudinal speed. */
typedef struct {
    double dt;
    int substeps;
    double accel_max, vx_min;
    int method; /* 0 forward Euler (the paper's), 1 classical fourth-order
                 * Runge-Kutta (the alternative the paper compared against) */
} oracle_integ;

/* Per-wheel diagnostic of one right-hand-side evaluation (wheel order
 * fl, fr, rl, rr). f is the force on the chassis at the wheel, in the body
 * frame: (F_x, F_y cos(delta_i), F_z). vi is the contact-point velocity in
 * the body frame. */
typedef struct {
    double P[4][3];
    double vi[4][3];
    double terr[4][4];  /* h, f_x, f_y, c at the wheel */
    double chi[4], chidot[4];
    double Fk[4], Fb[4], Fz[4], Fy[4], alpha[4];
    double f[4][3];
    double Fy_sum, Fz_sum, Mx, My, Mz, c_sum;
    double U_esm, L;    /* ESM and running cost at this state/control */
} oracle_diag;

typedef struct oracle_ctx oracle_ctx;

/* Returns NULL on invalid parameters. */
oracle_ctx *oracle_create(const oracle_vehicle *veh, const oracle_cost *cost,
                          const oracle_integ *integ);
void oracle_destroy(oracle_ctx *o);

/* Heights [H][W] (node (i,j) at (x0+i*res, y0+j*res), stored row j),
 * optional costmap [H][W] in cost units per second (NULL = zeros).
 * Returns 0, or -1 on invalid arguments. */
int oracle_set_terrain(oracle_ctx *o, const float *height, int W, int H,
                       double x0, double y0, double res, const float *costmap);

/* Bilinear sample of (h, f_x, f_y, c) at (x, y); clamp-to-edge. */
int oracle_sample_terrain(const oracle_ctx *o, double x, double y, double out[4]);

/* State derivative for state xi[13] and applied control (delta_dot, vx_dot),
 * with optional diagnostics. Returns 0, or -1 if no terrain is set. */
int oracle_rhs(const oracle_ctx *o, const double xi[13], double delta_dot,
               double vx_dot, double xidot[13], oracle_diag *diag);

/* ESM at roll phi and pitch theta. */
double oracle_esm(const oracle_ctx *o, double phi, double theta);

/* Normalised quadratic soft-constraint cost rate for violation measure pi. */
double oracle_soft(double sigma, double eps, double pi);

/* Rollout of K candidates. controls is [N][2][K] float (channel 0 steering
 * rate in rad/s, channel 1 normalised throttle). cost[K] and, if non-NULL,
 * final_state[13][K] are written in double. exit_step[K] (optional) receives
 * the Euler-node index at which the goal test fired, or -1.
 * Returns 0, -1 on invalid arguments, -4 if no terrain is set. */
int oracle_rollout(const oracle_ctx *o, const float state0[13],
                   const float *controls, int K, int N,
                   double *cost, double *final_state, int *exit_step);

/* Continue K candidates from per-candidate states over control intervals
 * [n0, n1) of the [N][2][K] control array. state_in is [13][K] float and
 * cost_in [K] float (running cost so far); state_out [13][K] and cost_out [K]
 * are double. With finalize, the terminal cost and the non-finite rule are
 * applied at the end (as after the last interval of oracle_rollout).
 * td_margin and slip_margin (optional, [K]) receive each candidate's smallest
 * distance over the span to the model's discontinuities: the damper's
 * touchdown switch (|F_s - k chi| / F_s on a compressing wheel) and the slip
 * angle's sign flip (|v_x| of a wheel, m/s); tilt_max (optional, [K]) the
 * largest |roll| or |pitch| (rad) met over the span.
 * Returns 0, -1 on invalid arguments, -4 if no terrain is set. */
int oracle_rollout_span(const oracle_ctx *o, const float *state_in, const float *cost_in,
                        const float *controls, int K, int N, int n0, int n1, int finalize,
                        double *state_out, double *cost_out, double *td_margin,
                        double *slip_margin, double *tilt_max);

/* As oracle_rollout with a double initial state and double controls
 * [N][2][K] (for finite-difference derivatives with steps below float
 * resolution). */
int oracle_rollout_d(const oracle_ctx *o, const double state0[13], const double *controls,
                     int K, int N, double *cost, double *final_state);

/* Conditioning probe (off by default): when on, rollouts round the state and
 * the running cost to float after every Euler step, while computing in
 * double. Comparing with the plain double run shows how far float storage
 * alone moves each trajectory, i.e. which candidates are well conditioned
 * enough for an element-wise float-vs-double comparison. */
void oracle_set_round32(oracle_ctx *o, int on);

/* Selection over candidates. mode 0 = argmin, 1 = softmin with temperature
 * lambda. cost is [K] float (the values being selected over). plan is
 * [N][2] double: the applied (clamped) controls of the selected candidate, or
 * their weighted average. best_k = -1 if no candidate is finite.
 * Returns 0 or -1 on invalid arguments. */
int oracle_select(const oracle_ctx *o, int mode, double lambda,
                  const float *controls, const float *cost, int K, int N,
                  int *best_k, double *best_cost, double *plan);

/* ---- extended single-track (EST) baseline formulation -------------------
 * Paper: appendix "Extended Single-Track Vehicle Dynamics Model" (state
 * eq. models:3dof:state, eqs. models:3dof:update / models:3dof:A, 1-2-3
 * rotation, terrain normal at the CoM, slip angles, load transfer
 * eqs. models:3dof:Fz_all / models:3dof:Fz_lon with the coefficients
 * models:3dof:Kzzf..Kzy and accelerations models:3dof:abx / models:3dof:aby)
 * and the lateral-acceleration soft constraint of "OCP Formulation"
 * (pi_ay = |a_y - g_y| - a_bar_y, a_bar_y = M g / (2 K_zy)). State order:
 * x, y, psi, v_y, omega_z, delta, v_x. */
typedef struct {
    double phi, theta;      /* roll and pitch from the normal under the CoM */
    double z;               /* CoM height f + (h+R) cos(phi) cos(theta) */
    double R[3][3];         /* 1-2-3 rotation W <- B */
    double gB[3];
    double alpha_f, alpha_r;
    double Fz_f, Fz_r;      /* virtual-tire normal loads */
    double Fy_f, Fy_r;
    double Fz_wheel[4];     /* physical tires fl, fr, rl, rr */
    double ax, ay;          /* CoM acceleration, body x and y */
    double pi_ay, a_bar_y;
    double P[4][3];         /* wheel contact points (costmap lookups) */
    double c_sum, L;        /* costmap sum and running cost */
} oracle_est_diag;

/* EST state derivative (7) for state xi[7] and control (delta_dot, vx_dot).
 * Returns 0, or -1 if no terrain is set. */
int oracle_est_rhs(const oracle_ctx *o, const double xi[7], double delta_dot, double vx_dot,
                   double xidot[7], oracle_est_diag *diag);

/* EST formulation rollout: same controls layout, goal test, quadrature,
 * clamps, +inf rule and conditioning probe (oracle_set_round32) as
 * oracle_rollout; final_state is [7][K]. */
int oracle_est_rollout(const oracle_ctx *o, const float state0[7], const float *controls,
                       int K, int N, double *cost, double *final_state, int *exit_step);

/* ---- terrain preparation (off the per-plan path) -------------------------
 * Level-of-detail smoothing (section "Terrain Smoothing"): the heightmap
 * convolved with a 2-D Gaussian of standard deviation sigma (m), weights
 * exp(-(di^2 + dj^2) res^2 / (2 sigma^2)) over the square of half-width
 * r = ceil(3 sigma / res - 1e-6) nodes, normalised to sum 1; nodes outside the grid
 * take the value of the nearest edge node (clamp-to-edge). out is [H][W].
 * Returns 0, or -1 on invalid arguments. */
int oracle_smooth_terrain(const float *height, int W, int H, double res, double sigma,
                          double *out);

/* Costmap of the distance constraints (sections "OCP Formulation" and
 * "Real-Time Implementation"): at every node, the sum over perimeters p of
 * sigma * max(0, 1 + pi_p / eps_dist)^2 with pi_p = -sdist_p, sdist_p the
 * signed 2-D distance from the node to perimeter p: for an obstacle
 * (kind 0) negative inside and positive outside, for a path boundary
 * (kind 1) the reverse. Polygon p has vertices verts[offsets[p]] ..
 * verts[offsets[p+1]-1] (x, y pairs, implicitly closed); inside is the
 * even-odd rule. out is [H][W], node (i, j) at (x0 + i res, y0 + j res).
 * Returns 0, or -1 on invalid arguments. */
int oracle_costmap_polygons(const double *verts, const int *offsets, const int *kinds, int P,
                            int W, int H, double x0, double y0, double res, double sigma,
                            double eps_dist, double *out);

/* Philox4x64-10 (Salmon et al., SC 2011): out = bijection of the 256-bit
 * counter under the 128-bit key. */
void oracle_philox4x64(const unsigned long long ctr[4], const unsigned long long key[2],
                       unsigned long long out[4]);

/* Candidate controls drawn from the counter-based generator: kind 0 uniform
 * (nominal + scale * U(-1, 1) per channel), kind 1 Gaussian (nominal +
 * scale * N(0, 1) by Box-Muller). Candidate k, interval n use word n mod 4
 * of Philox4x64-10 at counter (k, n div 4, 0, 0), key (seed, stream).
 * nominal is [N][2] float or NULL; keep_nominal makes candidate 0 the
 * nominal. controls is [N][2][K] double. Returns 0 or -1. */
int oracle_sample_controls(int kind, unsigned long long seed, unsigned long long stream,
                           const double scale[2], int keep_nominal, const float *nominal,
                           int K, int N, double *controls);

#ifdef __cplusplus
}
#endif
#endif
