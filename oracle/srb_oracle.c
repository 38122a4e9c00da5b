/*
 * FP64 CPU oracle for the single-rigid-body (SRB) sampling planner.
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU path is checked against.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code with the GPU library.
 *
 * Written plainly and sequentially from the paper (arXiv 2603.20525):
 *   - SRB model: section "Single Rigid Body Vehicle Dynamics Model"
 *     (state vector, eq. models:6dof:A, rotation matrix
 *     eq. models:6dof:rotation-matrix, Euler rates eq. models:6dof:euler-rates,
 *     contact point eq. models:6dof:P, extension eq. models:6dof:chi, suspension
 *     eq. models:6dof:Fs, slip angle, force and moment sums, rear constraint
 *     force F_x).
 *   - Tire: eq. models:tire (sigmoid lateral force).
 *   - Static loads: eqs. models:3dof:Kzzf, models:3dof:Kzzr.
 *   - ESM: eqs. esm and models:6dof:esm, with R-bar and phi-bar.
 *   - Cost: eq. framework:cost, baseline running cost
 *     eq. formulation:baseline_running_cost, terminal cost, L_soft, pi_ESM.
 *   - Goal: eq. formulation:goal; horizon and ZOH: section "OCP Formulation".
 *   - Optimiser: section "Real-Time Implementation" (empirical argmin; MPPI
 *     weighted average as the lambda > 0 variant; forward Euler).
 *
 * Readings where the paper is silent or ambiguous (the kernels take the same):
 *   - terrain normal taken as (-f_x, -f_y, 1), the upward normal of z=f(x,y);
 *   - ESM sign: negative once |phi| + phi_bar exceeds pi/2 (CoM past the
 *     wheel line);
 *   - eps_ESM default: 10 % of the level-ground ESM;
 *   - costmap holds the summed distance soft-cost rate; the four wheel
 *     lookups are added to the running cost;
 *   - cost quadrature: left Riemann sum at the Euler nodes;
 *   - goal test at each Euler node before the step, inclusive;
 *   - steering angle clamped to +-delta_max after each step, CoM speed floored
 *     at vx_min;
 *   - node slopes by central differences (one-sided on the border), bilinear
 *     interpolation of height, slopes and cost, clamp-to-edge queries;
 *   - slip angle literal atan(v_y/v_x); 0/0 gives alpha = -delta_i;
 *   - non-finite cost or final state makes the candidate cost +inf; argmin
 *     ties go to the lowest index.
 */
#define _DEFAULT_SOURCE
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

struct oracle_ctx {
    oracle_vehicle v;
    oracle_cost c;
    oracle_integ in;
    /* terrain, double precision, row j = y index */
    int W, H;
    double x0, y0, res;
    double *th, *tfx, *tfy, *tc;
    int has_terrain;
    int round32; /* conditioning probe, see oracle_set_round32 */
};

static double clampd(double x, double lo, double hi)
{
    if (x < lo) return lo;
    if (x > hi) return hi;
    return x;
}

/* ---------------------------------------------------------------- ESM ---- */

/* Eqs. esm and models:6dof:esm: Delta h = R_bar (1 - sin(|phi| + phi_bar)) cos(theta),
 * R_bar = sqrt((h+R)^2 + (e/2)^2), phi_bar = atan(2(h+R)/e).
 * U = +M g Delta h while the CoM is inside the footprint, -M g Delta h once it
 * is outside (|phi| + phi_bar > pi/2 under the rollover-only simplification). */
double oracle_esm(const oracle_ctx *o, double phi, double theta)
{
    const oracle_vehicle *v = &o->v;
    double Rbar = sqrt(v->hR * v->hR + (v->e / 2.0) * (v->e / 2.0));
    double phibar = atan(2.0 * v->hR / v->e);
    double a = fabs(phi) + phibar;
    double dh = Rbar * (1.0 - sin(a)) * cos(theta);
    double U = v->M * v->g * dh;
    if (a > 2.0 * atan(1.0)) U = -U; /* pi/2 */
    return U;
}

/* L_soft term for one constraint: sigma * max(0, 1 + pi/eps)^2. */
double oracle_soft(double sigma, double eps, double pi)
{
    double m = fmax(0.0, 1.0 + pi / eps);
    return sigma * m * m;
}

/* ------------------------------------------------------------ context ---- */

oracle_ctx *oracle_create(const oracle_vehicle *veh, const oracle_cost *cost,
                          const oracle_integ *integ)
{
    if (!veh || !cost || !integ) return NULL;
    if (!(veh->M > 0) || !(veh->Jxx > 0) || !(veh->Jyy > 0) || !(veh->Jzz > 0))
        return NULL;
    if (!(veh->Lf + veh->Lr > 0) || !(veh->e > 0) || !(veh->hR > 0)) return NULL;
    if (!(integ->dt > 0) || integ->substeps < 1) return NULL;
    if (integ->method != 0 && integ->method != 1) return NULL;
    oracle_ctx *o = (oracle_ctx *)calloc(1, sizeof(oracle_ctx));
    if (!o) return NULL;
    o->v = *veh;
    o->c = *cost;
    o->in = *integ;
    if (!(o->c.eps_esm > 0)) {
        /* 10 % of the ESM on level ground (the soft constraint starts adding
         * cost at a 10 % safety factor). */
        o->c.eps_esm = 0.1 * oracle_esm(o, 0.0, 0.0);
    }
    if (!(o->c.eps_ay > 0)) {
        /* same 10 % safety factor on the lateral-acceleration boundary
         * a_bar_y = M g / (2 K_zy) = g e / (2 (h+R)) */
        o->c.eps_ay = 0.1 * o->v.g * o->v.e / (2.0 * o->v.hR);
    }
    return o;
}

void oracle_destroy(oracle_ctx *o)
{
    if (!o) return;
    free(o->th);
    free(o->tfx);
    free(o->tfy);
    free(o->tc);
    free(o);
}

/* ------------------------------------------------------------ terrain ---- */

int oracle_set_terrain(oracle_ctx *o, const float *height, int W, int H,
                       double x0, double y0, double res, const float *costmap)
{
    if (!o || !height || W < 2 || H < 2 || !(res > 0)) return -1;
    size_t n = (size_t)W * (size_t)H;
    for (size_t q = 0; q < n; ++q)
        if (!isfinite((double)height[q]) || (costmap && !isfinite((double)costmap[q])))
            return -1;
    free(o->th);
    free(o->tfx);
    free(o->tfy);
    free(o->tc);
    o->th = (double *)malloc(n * sizeof(double));
    o->tfx = (double *)malloc(n * sizeof(double));
    o->tfy = (double *)malloc(n * sizeof(double));
    o->tc = (double *)malloc(n * sizeof(double));
    if (!o->th || !o->tfx || !o->tfy || !o->tc) return -1;
    o->W = W;
    o->H = H;
    o->x0 = x0;
    o->y0 = y0;
    o->res = res;
    for (int j = 0; j < H; ++j) {
        for (int i = 0; i < W; ++i) {
            size_t q = (size_t)j * W + i;
            o->th[q] = (double)height[q];
            o->tc[q] = costmap ? (double)costmap[q] : 0.0;
        }
    }
    /* Numerical first derivatives of the height function (the models only
     * need f, f_x, f_y; the paper asks for numerical derivatives of a
     * heightmap): central differences inside, one-sided on the border. */
    for (int j = 0; j < H; ++j) {
        for (int i = 0; i < W; ++i) {
            size_t q = (size_t)j * W + i;
            double fx, fy;
            if (i == 0)
                fx = (o->th[q + 1] - o->th[q]) / res;
            else if (i == W - 1)
                fx = (o->th[q] - o->th[q - 1]) / res;
            else
                fx = (o->th[q + 1] - o->th[q - 1]) / (2.0 * res);
            if (j == 0)
                fy = (o->th[q + W] - o->th[q]) / res;
            else if (j == H - 1)
                fy = (o->th[q] - o->th[q - W]) / res;
            else
                fy = (o->th[q + W] - o->th[q - W]) / (2.0 * res);
            o->tfx[q] = fx;
            o->tfy[q] = fy;
        }
    }
    o->has_terrain = 1;
    return 0;
}

/* Bilinear interpolation of the four node fields at (x, y), clamp-to-edge.
 * A non-finite query returns NaN in every channel. */
int oracle_sample_terrain(const oracle_ctx *o, double x, double y, double out[4])
{
    if (!o || !o->has_terrain) return -1;
    if (!isfinite(x) || !isfinite(y)) {
        out[0] = out[1] = out[2] = out[3] = NAN;
        return 0;
    }
    double u = clampd((x - o->x0) / o->res, 0.0, (double)(o->W - 1));
    double w = clampd((y - o->y0) / o->res, 0.0, (double)(o->H - 1));
    int i = (int)floor(u);
    int j = (int)floor(w);
    if (i > o->W - 2) i = o->W - 2;
    if (j > o->H - 2) j = o->H - 2;
    double tx = u - i, ty = w - j;
    size_t q00 = (size_t)j * o->W + i, q10 = q00 + 1;
    size_t q01 = q00 + o->W, q11 = q01 + 1;
    const double *F[4] = {o->th, o->tfx, o->tfy, o->tc};
    for (int ch = 0; ch < 4; ++ch) {
        const double *g = F[ch];
        out[ch] = (1.0 - tx) * (1.0 - ty) * g[q00] + tx * (1.0 - ty) * g[q10] +
                  (1.0 - tx) * ty * g[q01] + tx * ty * g[q11];
    }
    return 0;
}

/* ---------------------------------------------------------- SRB model ---- */

int oracle_rhs(const oracle_ctx *o, const double xi[13], double delta_dot,
               double vx_dot, double xidot[13], oracle_diag *diag)
{
    if (!o || !o->has_terrain) return -1;
    const oracle_vehicle *V = &o->v;

    /* state vector eq. models:6dof:state */
    double x = xi[0], y = xi[1], z = xi[2];
    double psi = xi[3], th = xi[4], ph = xi[5];
    double vb[3] = {xi[6], xi[7], xi[8]};
    double w[3] = {xi[9], xi[10], xi[11]};
    double delta = xi[12];

    /* 3-2-1 rotation matrix W <- B, eq. models:6dof:rotation-matrix */
    double cps = cos(psi), sps = sin(psi);
    double cth = cos(th), sth = sin(th);
    double cph = cos(ph), sph = sin(ph);
    double R[3][3] = {
        {cps * cth, cps * sph * sth - cph * sps, sph * sps + cph * cps * sth},
        {cth * sps, cph * cps + sph * sps * sth, cph * sps * sth - cps * sph},
        {-sth, cth * sph, cph * cth},
    };

    /* world-frame CoM velocity */
    double vw[3];
    for (int r = 0; r < 3; ++r) vw[r] = R[r][0] * vb[0] + R[r][1] * vb[1] + R[r][2] * vb[2];

    /* Euler-angle rates, eq. models:6dof:euler-rates */
    double psid = (sph / cth) * w[1] + (cph / cth) * w[2];
    double thd = cph * w[1] - sph * w[2];
    double phd = w[0] + (sph * sth / cth) * w[1] + (cph * sth / cth) * w[2];

    /* gravity resolved in the body frame: R^T (0, 0, -g) */
    double gB[3];
    for (int cidx = 0; cidx < 3; ++cidx) gB[cidx] = R[2][cidx] * (-V->g);

    /* static loads, eqs. models:3dof:Kzzf / models:3dof:Kzzr */
    double L = V->Lf + V->Lr;
    double Kzz_f = V->M * V->Lr / L;
    double Kzz_r = V->M * V->Lf / L;

    /* wheels fl, fr, rl, rr; body-frame lever arms rho^i */
    double rho[4][3] = {
        {V->Lf, V->e / 2.0, -V->hR},
        {V->Lf, -V->e / 2.0, -V->hR},
        {-V->Lr, V->e / 2.0, -V->hR},
        {-V->Lr, -V->e / 2.0, -V->hR},
    };

    double Fy_sum = 0.0, Fz_sum = 0.0, Msum[3] = {0.0, 0.0, 0.0}, c_sum = 0.0;
    for (int i = 0; i < 4; ++i) {
        int front = (i < 2);
        /* contact point and its velocity, eq. models:6dof:P */
        double P[3], vi[3];
        for (int r = 0; r < 3; ++r)
            P[r] = (r == 0 ? x : (r == 1 ? y : z)) +
                   R[r][0] * rho[i][0] + R[r][1] * rho[i][1] + R[r][2] * rho[i][2];
        /* v^i = v + omega x rho^i (body frame) */
        vi[0] = vb[0] + (w[1] * rho[i][2] - w[2] * rho[i][1]);
        vi[1] = vb[1] + (w[2] * rho[i][0] - w[0] * rho[i][2]);
        vi[2] = vb[2] + (w[0] * rho[i][1] - w[1] * rho[i][0]);

        /* terrain height and slope at the nominal contact patch */
        double T[4];
        oracle_sample_terrain(o, P[0], P[1], T);

        /* normal to the terrain, world frame (upward normal of z = f(x,y)),
         * resolved in the body frame */
        double nW[3] = {-T[1], -T[2], 1.0};
        double nB[3];
        for (int cidx = 0; cidx < 3; ++cidx)
            nB[cidx] = R[0][cidx] * nW[0] + R[1][cidx] * nW[1] + R[2][cidx] * nW[2];

        /* extension and rate, eq. models:6dof:chi; omega x b_z = (w_y, -w_x, 0) */
        double chi = (P[2] - T[0]) / nB[2];
        double rel[3] = {vi[0] - chi * w[1], vi[1] + chi * w[0], vi[2]};
        double chidot = (nB[0] * rel[0] + nB[1] * rel[1] + nB[2] * rel[2]) / nB[2];

        /* suspension with liftoff, eq. models:6dof:Fs */
        double Kzz = front ? Kzz_f : Kzz_r;
        double k = front ? V->kf : V->kr;
        double b = front ? V->bf : V->br;
        double Fs = (V->g / 2.0) * Kzz;
        double Fk = fmax(Fs - k * chi, 0.0);
        double Fb = (Fk > 0.0) ? fmax(-b * chidot, -Fk) : 0.0;
        double Fz = Fk + Fb;

        /* slip angle and sigmoid tire, eq. models:tire */
        double delta_i = front ? delta : 0.0;
        double alpha;
        if (vi[0] == 0.0 && vi[1] == 0.0)
            alpha = -delta_i;
        else
            alpha = atan(vi[1] / vi[0]) - delta_i;
        double Ca = V->C * alpha;
        double Fy = Fz * (-Ca * V->mu) / sqrt(V->mu * V->mu + Ca * Ca);

        /* longitudinal constraint force (rear wheels only) */
        double Fx = front ? 0.0
                          : (V->M / 2.0) * (vx_dot - gB[0] + w[1] * vb[2] - w[2] * vb[1]);

        /* force on the chassis at wheel i (body frame) */
        double f[3] = {Fx, Fy * cos(delta_i), Fz};
        /* summed forces and moments */
        Fy_sum += f[1];
        Fz_sum += f[2];
        Msum[0] += rho[i][1] * f[2] - rho[i][2] * f[1];
        Msum[1] += rho[i][2] * f[0] - rho[i][0] * f[2];
        Msum[2] += rho[i][0] * f[1] - rho[i][1] * f[0];
        c_sum += T[3];

        if (diag) {
            for (int r = 0; r < 3; ++r) {
                diag->P[i][r] = P[r];
                diag->vi[i][r] = vi[r];
                diag->f[i][r] = f[r];
            }
            for (int ch = 0; ch < 4; ++ch) diag->terr[i][ch] = T[ch];
            diag->chi[i] = chi;
            diag->chidot[i] = chidot;
            diag->Fk[i] = Fk;
            diag->Fb[i] = Fb;
            diag->Fz[i] = Fz;
            diag->Fy[i] = Fy;
            diag->alpha[i] = alpha;
        }
    }

    /* eq. models:6dof:A plus B zeta */
    xidot[0] = vw[0];
    xidot[1] = vw[1];
    xidot[2] = vw[2];
    xidot[3] = psid;
    xidot[4] = thd;
    xidot[5] = phd;
    xidot[6] = vx_dot;
    xidot[7] = Fy_sum / V->M + gB[1] + w[0] * vb[2] - w[2] * vb[0];
    xidot[8] = Fz_sum / V->M + gB[2] - w[0] * vb[1] + w[1] * vb[0];
    xidot[9] = (Msum[0] + (V->Jyy - V->Jzz) * w[1] * w[2]) / V->Jxx;
    xidot[10] = (Msum[1] - (V->Jxx - V->Jzz) * w[0] * w[2]) / V->Jyy;
    xidot[11] = (Msum[2] + (V->Jxx - V->Jyy) * w[0] * w[1]) / V->Jzz;
    xidot[12] = delta_dot;

    /* ESM constraint and running cost: L = w_t + w_c delta_dot^2 + L_soft,
     * with pi_ESM = -U_ESM and the costmap (distance) term at the wheels */
    double U = oracle_esm(o, ph, th);
    double Lrun = o->c.w_t + o->c.w_c * delta_dot * delta_dot +
                  oracle_soft(o->c.sigma, o->c.eps_esm, -U) + c_sum;

    if (diag) {
        diag->Fy_sum = Fy_sum;
        diag->Fz_sum = Fz_sum;
        diag->Mx = Msum[0];
        diag->My = Msum[1];
        diag->Mz = Msum[2];
        diag->c_sum = c_sum;
        diag->U_esm = U;
        diag->L = Lrun;
    }
    return 0;
}

/* ------------------------------------------------------------ rollout ---- */

static double goal_distance(const oracle_ctx *o, double x, double y)
{
    double dx = x - o->c.goal_x, dy = y - o->c.goal_y;
    return sqrt(dx * dx + dy * dy);
}

/* One candidate over control intervals [n0, n1): J accumulates h L at each
 * Euler node (left Riemann sum); the horizon ends early at the goal. With
 * finalize, Phi is added at the final (or goal-exit) state and a non-finite
 * cost or state makes J = +inf. With round32, the state and J are rounded to
 * float after every Euler step (a conditioning probe: how far float storage
 * alone moves the double-precision trajectory). */
/* Distance of one right-hand-side evaluation to the model's two
 * discontinuities (diagnostic for float-vs-double comparisons):
 *   - touchdown: the damper force is max(-b chi_dot, -F_k) while F_k > 0 and 0
 *     at F_k = 0, so a compressing wheel (chi_dot < 0) gains b|chi_dot| at the
 *     step where F_s - k chi crosses zero; margin |F_s - k chi| / F_s;
 *   - slip: atan(v_y / v_x) jumps by pi where a wheel's v_x changes sign;
 *     margin |v_x| in m/s;
 * and the largest roll or pitch magnitude (the paper scores a trial as a
 * rollover once either exceeds 72 degrees). */
static void discontinuity_margins(const oracle_ctx *o, const oracle_diag *d,
                                  const double xi[13], double *td, double *sl, double *tilt)
{
    double t = fmax(fabs(xi[4]), fabs(xi[5]));
    if (!(t <= *tilt)) *tilt = t;
    const oracle_vehicle *V = &o->v;
    double L = V->Lf + V->Lr;
    for (int i = 0; i < 4; ++i) {
        int front = (i < 2);
        double Fs = (V->g / 2.0) * V->M * (front ? V->Lr : V->Lf) / L;
        double k = front ? V->kf : V->kr;
        if (d->chidot[i] < 0.0) {
            double m = fabs(Fs - k * d->chi[i]) / Fs;
            if (!(m >= *td)) *td = m;
        }
        double vxm = fabs(d->vi[i][0]);
        if (!(vxm >= *sl)) *sl = vxm;
    }
}

/* Control u[n][c] of candidate k, from the float array or, when given, the
 * double one. */
static double control_at(const float *cf, const double *cd, int K, int k, int n, int c)
{
    size_t q = ((size_t)n * 2 + c) * K + k;
    return cd ? cd[q] : (double)cf[q];
}

static void span_one(const oracle_ctx *o, double xi[13], double *J_io,
                     const float *controls, const double *controls_d, int K, int k, int n0, int n1,
                     int finalize, int round32, int *exit_out, double *td, double *sl,
                     double *tilt)
{
    const int S = o->in.substeps;
    const double h = o->in.dt / S;
    double xd[13];
    double J = *J_io;
    int done = 0, exit_step = -1;

    for (int n = n0; n < n1 && !done; ++n) {
        /* zero-order hold: control n applies for the whole interval; the
         * sampled controls are restricted to the admissible set */
        double u0 = control_at(controls, controls_d, K, k, n, 0);
        double u1 = control_at(controls, controls_d, K, k, n, 1);
        double delta_dot = clampd(u0, -o->v.delta_rate_max, o->v.delta_rate_max);
        double vx_dot = o->in.accel_max * clampd(u1, -1.0, 1.0);
        for (int s = 0; s < S; ++s) {
            /* goal reached: horizon ends here (t_f) */
            if (goal_distance(o, xi[0], xi[1]) <= o->c.goal_r) {
                done = 1;
                exit_step = n * S + s;
                break;
            }
            oracle_diag d;
            oracle_rhs(o, xi, delta_dot, vx_dot, xd, &d);
            if (td && sl && tilt) discontinuity_margins(o, &d, xi, td, sl, tilt);
            if (o->in.method == 1) {
                /* classical fourth-order Runge-Kutta on (xi, J), J' = L, with
                 * the control held; the limits apply to the completed step */
                double k[4][13], Ls[4], stage[13];
                for (int q = 0; q < 13; ++q) k[0][q] = xd[q];
                Ls[0] = d.L;
                const double c[3] = {0.5 * h, 0.5 * h, h};
                for (int st = 1; st < 4; ++st) {
                    oracle_diag ds;
                    for (int q = 0; q < 13; ++q) stage[q] = xi[q] + c[st - 1] * k[st - 1][q];
                    oracle_rhs(o, stage, delta_dot, vx_dot, k[st], &ds);
                    Ls[st] = ds.L;
                }
                J += h / 6.0 * (Ls[0] + 2.0 * Ls[1] + 2.0 * Ls[2] + Ls[3]);
                for (int q = 0; q < 13; ++q)
                    xi[q] = xi[q] + h / 6.0 * (k[0][q] + 2.0 * k[1][q] + 2.0 * k[2][q] + k[3][q]);
            } else {
                J += h * d.L;
                for (int q = 0; q < 13; ++q) xi[q] = xi[q] + h * xd[q];
            }
            xi[12] = clampd(xi[12], -o->v.delta_max, o->v.delta_max);
            if (xi[6] < o->in.vx_min) xi[6] = o->in.vx_min;
            if (round32) {
                for (int q = 0; q < 13; ++q) xi[q] = (double)(float)xi[q];
                J = (double)(float)J;
            }
        }
    }
    if (finalize) {
        J += o->c.w_g * goal_distance(o, xi[0], xi[1]);
        int finite = isfinite(J);
        for (int q = 0; q < 13; ++q) finite = finite && isfinite(xi[q]);
        if (!finite) J = INFINITY;
    }
    *J_io = J;
    if (exit_out) *exit_out = exit_step;
}

int oracle_rollout(const oracle_ctx *o, const float state0[13],
                   const float *controls, int K, int N,
                   double *cost, double *final_state, int *exit_step)
{
    if (!o || !state0 || !controls || !cost || K < 1 || N < 1) return -1;
    if (!o->has_terrain) return -4;
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < K; ++k) {
        double xi[13], J = 0.0;
        int ex;
        for (int q = 0; q < 13; ++q) xi[q] = (double)state0[q];
        span_one(o, xi, &J, controls, NULL, K, k, 0, N, 1, o->round32, &ex, NULL, NULL, NULL);
        cost[k] = J;
        if (final_state)
            for (int q = 0; q < 13; ++q) final_state[(size_t)q * K + k] = xi[q];
        if (exit_step) exit_step[k] = ex;
    }
    return 0;
}

int oracle_rollout_span(const oracle_ctx *o, const float *state_in, const float *cost_in,
                        const float *controls, int K, int N, int n0, int n1, int finalize,
                        double *state_out, double *cost_out, double *td_margin,
                        double *slip_margin, double *tilt_max)
{
    if (!o || !state_in || !cost_in || !controls || !state_out || !cost_out) return -1;
    if (K < 1 || N < 1 || n0 < 0 || n1 < n0 || n1 > N) return -1;
    if (!o->has_terrain) return -4;
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < K; ++k) {
        double xi[13], J = (double)cost_in[k];
        double td = INFINITY, sl = INFINITY, tilt = 0.0;
        for (int q = 0; q < 13; ++q) xi[q] = (double)state_in[(size_t)q * K + k];
        span_one(o, xi, &J, controls, NULL, K, k, n0, n1, finalize, o->round32, NULL, &td, &sl,
                 &tilt);
        if (td_margin) td_margin[k] = td;
        if (slip_margin) slip_margin[k] = sl;
        if (tilt_max) tilt_max[k] = tilt;
        cost_out[k] = J;
        for (int q = 0; q < 13; ++q) state_out[(size_t)q * K + k] = xi[q];
    }
    return 0;
}

int oracle_rollout_d(const oracle_ctx *o, const double state0[13], const double *controls,
                     int K, int N, double *cost, double *final_state)
{
    if (!o || !state0 || !controls || !cost || K < 1 || N < 1) return -1;
    if (!o->has_terrain) return -4;
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < K; ++k) {
        double xi[13], J = 0.0;
        for (int q = 0; q < 13; ++q) xi[q] = state0[q];
        span_one(o, xi, &J, NULL, controls, K, k, 0, N, 1, 0, NULL, NULL, NULL, NULL);
        cost[k] = J;
        if (final_state)
            for (int q = 0; q < 13; ++q) final_state[(size_t)q * K + k] = xi[q];
    }
    return 0;
}

void oracle_set_round32(oracle_ctx *o, int on)
{
    if (o) o->round32 = on != 0;
}

/* ------------------------------------------------------------- select ---- */

int oracle_select(const oracle_ctx *o, int mode, double lambda,
                  const float *controls, const float *cost, int K, int N,
                  int *best_k, double *best_cost, double *plan)
{
    if (!o || !controls || !cost || !best_k || !best_cost || !plan) return -1;
    if (K < 1 || N < 1 || (mode != 0 && mode != 1)) return -1;
    if (mode == 1 && !(lambda > 0)) return -1;

    /* empirical argmin: lowest index among the minimal finite costs */
    int kb = -1;
    double Jb = INFINITY;
    for (int k = 0; k < K; ++k) {
        double J = (double)cost[k];
        if (!isfinite(J)) continue;
        if (kb < 0 || J < Jb) {
            kb = k;
            Jb = J;
        }
    }
    *best_k = kb;
    *best_cost = Jb;
    if (kb < 0) {
        for (int q = 0; q < 2 * N; ++q) plan[q] = 0.0;
        return 0;
    }

    for (int n = 0; n < N; ++n) {
        for (int ch = 0; ch < 2; ++ch) {
            double lim = (ch == 0) ? o->v.delta_rate_max : 1.0;
            if (mode == 0) {
                plan[n * 2 + ch] = clampd((double)controls[((size_t)n * 2 + ch) * K + kb], -lim, lim);
            } else {
                /* MPPI-style average: weights exp(-(J_k - J_min)/lambda) */
                double num = 0.0, den = 0.0;
                for (int k = 0; k < K; ++k) {
                    double J = (double)cost[k];
                    if (!isfinite(J)) continue;
                    double wk = exp(-(J - Jb) / lambda);
                    num += wk * clampd((double)controls[((size_t)n * 2 + ch) * K + k], -lim, lim);
                    den += wk;
                }
                plan[n * 2 + ch] = num / den;
            }
        }
    }
    return 0;
}

/* ----------------------------------------------------------- EST model ---- */

int oracle_est_rhs(const oracle_ctx *o, const double xi[7], double delta_dot, double vx_dot,
                   double xidot[7], oracle_est_diag *diag)
{
    if (!o || !o->has_terrain) return -1;
    const oracle_vehicle *V = &o->v;

    /* state vector eq. models:3dof:state */
    double x = xi[0], y = xi[1], psi = xi[2];
    double vy = xi[3], wz = xi[4], delta = xi[5], vx = xi[6];

    /* roll and pitch: the chassis z axis is the terrain's unit upward normal
     * under the CoM (the normal of z = f(x, y) is (-f_x, -f_y, 1)); under the
     * 1-2-3 convention b_z = (sin th, -cos th sin ph, cos ph cos th) */
    double T0[4];
    oracle_sample_terrain(o, x, y, T0);
    double nrm = sqrt(1.0 + T0[1] * T0[1] + T0[2] * T0[2]);
    double n[3] = {-T0[1] / nrm, -T0[2] / nrm, 1.0 / nrm};
    double th = asin(n[0]);
    double ph = atan2(-n[1], n[2]);

    /* 1-2-3 rotation W <- B, eq. app:models:3dof:rotation */
    double cps = cos(psi), sps = sin(psi);
    double cth = cos(th), sth = sin(th);
    double cph = cos(ph), sph = sin(ph);
    double R[3][3] = {
        {cth * cps, -cth * sps, sth},
        {cph * sps + cps * sph * sth, cph * cps - sph * sth * sps, -cth * sph},
        {sph * sps - cph * cps * sth, cps * sph + cph * sth * sps, cph * cth},
    };

    /* planar body velocity (v_x, v_y, 0) and yaw-only angular velocity */
    double vw0 = R[0][0] * vx + R[0][1] * vy;
    double vw1 = R[1][0] * vx + R[1][1] * vy;

    /* gravity in the body frame, R^T (0, 0, -g) */
    double gB[3] = {-V->g * R[2][0], -V->g * R[2][1], -V->g * R[2][2]};

    /* load-transfer coefficients, eqs. models:3dof:Kzzf .. models:3dof:Kzy */
    double L = V->Lf + V->Lr;
    double Kzz_f = V->M * V->Lr / L;
    double Kzz_r = V->M * V->Lf / L;
    double Kzx = V->M * V->hR / L;
    double Kzy = V->M * V->hR / V->e;

    /* longitudinal acceleration, eq. models:3dof:abx */
    double ax = vx_dot - wz * vy;

    /* virtual-tire normal loads, eq. models:3dof:Fz_lon */
    double Fz_f = -Kzz_f * gB[2] - Kzx * ax;
    double Fz_r = -Kzz_r * gB[2] + Kzx * ax;

    /* slip angles of the virtual tires and sigmoid tire, eq. models:tire */
    double alpha_f = atan((vy + wz * V->Lf) / vx) - delta;
    double alpha_r = atan((vy - wz * V->Lr) / vx);
    double Caf = V->C * alpha_f, Car = V->C * alpha_r;
    double Fy_f = Fz_f * (-Caf * V->mu) / sqrt(V->mu * V->mu + Caf * Caf);
    double Fy_r = Fz_r * (-Car * V->mu) / sqrt(V->mu * V->mu + Car * Car);

    /* eq. models:3dof:A plus B zeta */
    xidot[0] = vw0;
    xidot[1] = vw1;
    xidot[2] = wz;
    xidot[3] = (Fy_f + Fy_r) / V->M + gB[1] - wz * vx;
    xidot[4] = (Fy_f * V->Lf * cos(delta) - Fy_r * V->Lr) / V->Jzz;
    xidot[5] = delta_dot;
    xidot[6] = vx_dot;

    /* lateral acceleration, eq. models:3dof:aby, and its soft constraint */
    double ay = xidot[3] + wz * vx;
    double a_bar_y = V->M * V->g / (2.0 * Kzy);
    double pi_ay = fabs(ay - gB[1]) - a_bar_y;

    /* wheel contact points for the costmap: CoM at height f + (h+R) b_z.w_z,
     * wheels at the SRB lever arms rotated into the world frame */
    double z = T0[0] + V->hR * R[2][2];
    double rho[4][3] = {
        {V->Lf, V->e / 2.0, -V->hR},
        {V->Lf, -V->e / 2.0, -V->hR},
        {-V->Lr, V->e / 2.0, -V->hR},
        {-V->Lr, -V->e / 2.0, -V->hR},
    };
    double c_sum = 0.0, P[4][3];
    for (int i = 0; i < 4; ++i) {
        double p0[3] = {x, y, z};
        for (int r = 0; r < 3; ++r)
            P[i][r] = p0[r] + R[r][0] * rho[i][0] + R[r][1] * rho[i][1] + R[r][2] * rho[i][2];
        double Ti[4];
        oracle_sample_terrain(o, P[i][0], P[i][1], Ti);
        c_sum += Ti[3];
    }
    double Lrun = o->c.w_t + o->c.w_c * delta_dot * delta_dot +
                  oracle_soft(o->c.sigma, o->c.eps_ay, pi_ay) + c_sum;

    if (diag) {
        diag->phi = ph;
        diag->theta = th;
        diag->z = z;
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) diag->R[r][cc] = R[r][cc];
        for (int r = 0; r < 3; ++r) diag->gB[r] = gB[r];
        diag->alpha_f = alpha_f;
        diag->alpha_r = alpha_r;
        diag->Fz_f = Fz_f;
        diag->Fz_r = Fz_r;
        diag->Fy_f = Fy_f;
        diag->Fy_r = Fy_r;
        /* physical tires, eq. models:3dof:Fz_all */
        double lat = Kzy * ay / (-V->M * gB[2]);
        diag->Fz_wheel[0] = Fz_f * (0.5 - lat);
        diag->Fz_wheel[1] = Fz_f * (0.5 + lat);
        diag->Fz_wheel[2] = Fz_r * (0.5 - lat);
        diag->Fz_wheel[3] = Fz_r * (0.5 + lat);
        diag->ax = ax;
        diag->ay = ay;
        diag->pi_ay = pi_ay;
        diag->a_bar_y = a_bar_y;
        for (int i = 0; i < 4; ++i)
            for (int r = 0; r < 3; ++r) diag->P[i][r] = P[i][r];
        diag->c_sum = c_sum;
        diag->L = Lrun;
    }
    return 0;
}

int oracle_est_rollout(const oracle_ctx *o, const float state0[7], const float *controls,
                       int K, int N, double *cost, double *final_state, int *exit_step)
{
    if (!o || !state0 || !controls || !cost || K < 1 || N < 1) return -1;
    if (!o->has_terrain) return -4;
    const int S = o->in.substeps;
    const double h = o->in.dt / S;
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < K; ++k) {
        double xi[7], xd[7], J = 0.0;
        int done = 0, ex = -1;
        for (int q = 0; q < 7; ++q) xi[q] = (double)state0[q];
        for (int n = 0; n < N && !done; ++n) {
            double delta_dot = clampd((double)controls[((size_t)n * 2 + 0) * K + k],
                                      -o->v.delta_rate_max, o->v.delta_rate_max);
            double vx_dot = o->in.accel_max *
                            clampd((double)controls[((size_t)n * 2 + 1) * K + k], -1.0, 1.0);
            for (int s = 0; s < S; ++s) {
                if (goal_distance(o, xi[0], xi[1]) <= o->c.goal_r) {
                    done = 1;
                    ex = n * S + s;
                    break;
                }
                oracle_est_diag d;
                oracle_est_rhs(o, xi, delta_dot, vx_dot, xd, &d);
                J += h * d.L;
                for (int q = 0; q < 7; ++q) xi[q] = xi[q] + h * xd[q];
                xi[5] = clampd(xi[5], -o->v.delta_max, o->v.delta_max);
                if (xi[6] < o->in.vx_min) xi[6] = o->in.vx_min;
                if (o->round32) {
                    for (int q = 0; q < 7; ++q) xi[q] = (double)(float)xi[q];
                    J = (double)(float)J;
                }
            }
        }
        J += o->c.w_g * goal_distance(o, xi[0], xi[1]);
        int finite = isfinite(J);
        for (int q = 0; q < 7; ++q) finite = finite && isfinite(xi[q]);
        if (!finite) J = INFINITY;
        cost[k] = J;
        if (final_state)
            for (int q = 0; q < 7; ++q) final_state[(size_t)q * K + k] = xi[q];
        if (exit_step) exit_step[k] = ex;
    }
    return 0;
}

/* ------------------------------------------------- terrain preparation ---- */

int oracle_smooth_terrain(const float *height, int W, int H, double res, double sigma,
                          double *out)
{
    if (!height || !out || W < 1 || H < 1 || !(res > 0) || !(sigma > 0)) return -1;
    /* truncation at 3 sigma; the 1e-6 node slack keeps decimal inputs such as
     * sigma = 0.3 m at 0.1 m on 9 nodes whatever precision they arrive in */
    const int r = (int)ceil(3.0 * sigma / res - 1e-6);
    /* unnormalised 2-D weights and their sum */
    const int n = 2 * r + 1;
    double *wt = (double *)malloc(sizeof(double) * (size_t)n * n);
    if (!wt) return -1;
    double total = 0.0;
    for (int dj = -r; dj <= r; ++dj)
        for (int di = -r; di <= r; ++di) {
            double d2 = ((double)di * di + (double)dj * dj) * res * res;
            double w = exp(-d2 / (2.0 * sigma * sigma));
            wt[(size_t)(dj + r) * n + (di + r)] = w;
            total += w;
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j) {
        for (int i = 0; i < W; ++i) {
            double acc = 0.0;
            for (int dj = -r; dj <= r; ++dj) {
                int jj = j + dj;
                if (jj < 0) jj = 0;
                if (jj > H - 1) jj = H - 1;
                for (int di = -r; di <= r; ++di) {
                    int ii = i + di;
                    if (ii < 0) ii = 0;
                    if (ii > W - 1) ii = W - 1;
                    acc += wt[(size_t)(dj + r) * n + (di + r)] * (double)height[(size_t)jj * W + ii];
                }
            }
            out[(size_t)j * W + i] = acc / total;
        }
    }
    free(wt);
    return 0;
}

/* Distance from (px, py) to the segment a-b. */
static double segment_distance(double px, double py, double ax, double ay, double bx, double by)
{
    double ex = bx - ax, ey = by - ay;
    double len2 = ex * ex + ey * ey;
    double t = 0.0;
    if (len2 > 0.0) t = clampd(((px - ax) * ex + (py - ay) * ey) / len2, 0.0, 1.0);
    double qx = ax + t * ex - px, qy = ay + t * ey - py;
    return sqrt(qx * qx + qy * qy);
}

int oracle_costmap_polygons(const double *verts, const int *offsets, const int *kinds, int P,
                            int W, int H, double x0, double y0, double res, double sigma,
                            double eps_dist, double *out)
{
    if (!out || W < 1 || H < 1 || !(res > 0) || !(eps_dist > 0) || P < 0) return -1;
    if (P > 0 && (!verts || !offsets || !kinds)) return -1;
    for (int p = 0; p < P; ++p)
        if (offsets[p + 1] - offsets[p] < 3 || (kinds[p] != 0 && kinds[p] != 1)) return -1;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j) {
        for (int i = 0; i < W; ++i) {
            double px = x0 + i * res, py = y0 + j * res;
            double c = 0.0;
            for (int p = 0; p < P; ++p) {
                int a = offsets[p], b = offsets[p + 1], m = b - a;
                double dmin = INFINITY;
                int inside = 0;
                for (int e = 0; e < m; ++e) {
                    const double *v0 = verts + 2 * (size_t)(a + e);
                    const double *v1 = verts + 2 * (size_t)(a + (e + 1) % m);
                    double d = segment_distance(px, py, v0[0], v0[1], v1[0], v1[1]);
                    if (d < dmin) dmin = d;
                    /* even-odd rule: count edges crossing the ray to +x */
                    if ((v0[1] > py) != (v1[1] > py)) {
                        double xc = v0[0] + (py - v0[1]) * (v1[0] - v0[0]) / (v1[1] - v0[1]);
                        if (px < xc) inside = !inside;
                    }
                }
                /* obstacle: negative inside; path boundary: negative outside */
                double sdist = (inside == (kinds[p] == 0)) ? -dmin : dmin;
                c += oracle_soft(sigma, eps_dist, -sdist);
            }
            out[(size_t)j * W + i] = c;
        }
    }
    return 0;
}

/* ------------------------------------------------------------ sampling ---- */
/* The paper draws the candidate controls on the GPU with a counter-based
 * generator ("Real-Time Implementation": the random samples are produced with
 * cuRAND on the device; the published configuration draws the steering rate
 * uniformly and holds the acceleration). The generator here is Philox4x64-10
 * as defined by Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3" (SC 2011): ten rounds of two 64x64->128-bit products with
 * the published multipliers, the halves crossed and xored with the key, the
 * key advanced by the published Weyl increments between rounds. */
void oracle_philox4x64(const unsigned long long ctr[4], const unsigned long long key[2],
                       unsigned long long out[4])
{
    const uint64_t mul0 = 0xD2E7470EE14C6C93ull, mul1 = 0xCA5A826395121157ull;
    const uint64_t weyl0 = 0x9E3779B97F4A7C15ull, weyl1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        unsigned __int128 p0 = (unsigned __int128)mul0 * c0;
        unsigned __int128 p1 = (unsigned __int128)mul1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Controls [N][2][K] (double) for candidate k and interval n from the 64-bit
 * word w = word (n mod 4) of Philox4x64-10 at counter (k, floor(n/4), 0, 0)
 * and key (seed, stream). Two 24-bit integers are taken from w: a = bits
 * 40..63 and b = bits 16..39.
 *   kind 0 (uniform):  u_c = nominal_c + scale_c (2 x_c - 1), with
 *                      x_0 = a 2^-24, x_1 = b 2^-24 (uniform on [0, 1));
 *   kind 1 (Gaussian): Box-Muller (Box and Muller, 1958) on p = (a+1) 2^-24
 *                      in (0, 1] and q = b 2^-24: r = sqrt(-2 ln p),
 *                      u_0 = nominal_0 + scale_0 r cos(2 pi q),
 *                      u_1 = nominal_1 + scale_1 r sin(2 pi q).
 * nominal is [N][2] float or NULL (zeros). With keep_nominal, candidate 0 is
 * the nominal itself. Returns 0, or -1 on invalid arguments. */
int oracle_sample_controls(int kind, unsigned long long seed, unsigned long long stream,
                           const double scale[2],
                           int keep_nominal, const float *nominal, int K, int N,
                           double *controls)
{
    if ((kind != 0 && kind != 1) || !scale || !controls || K < 1 || N < 1) return -1;
    const double two_m24 = 1.0 / 16777216.0;
    const double two_pi = 8.0 * atan(1.0);
    const unsigned long long key[2] = {seed, stream};
    for (int k = 0; k < K; ++k) {
        for (int n = 0; n < N; ++n) {
            double nom0 = nominal ? (double)nominal[2 * n] : 0.0;
            double nom1 = nominal ? (double)nominal[2 * n + 1] : 0.0;
            double u0 = nom0, u1 = nom1;
            if (!(keep_nominal && k == 0)) {
                const unsigned long long ctr[4] = {(unsigned long long)k,
                                                   (unsigned long long)(n / 4), 0, 0};
                unsigned long long words[4];
                oracle_philox4x64(ctr, key, words);
                uint64_t w = words[n % 4];
                double a = (double)(w >> 40);
                double b = (double)((w >> 16) & 0xFFFFFFull);
                if (kind == 0) {
                    u0 = nom0 + scale[0] * (2.0 * (a * two_m24) - 1.0);
                    u1 = nom1 + scale[1] * (2.0 * (b * two_m24) - 1.0);
                } else {
                    double p = (a + 1.0) * two_m24;
                    double q = b * two_m24;
                    double r = sqrt(-2.0 * log(p));
                    u0 = nom0 + scale[0] * r * cos(two_pi * q);
                    u1 = nom1 + scale[1] * r * sin(two_pi * q);
                }
            }
            controls[((size_t)n * 2 + 0) * K + k] = u0;
            controls[((size_t)n * 2 + 1) * K + k] = u1;
        }
    }
    return 0;
}
