// Rollout of the extended single-track (EST) baseline formulation: the
// paper's comparison model (appendix "Extended Single-Track Vehicle Dynamics
// Model": state eq. models:3dof:state, eqs. models:3dof:update and
// models:3dof:A, 1-2-3 rotation, virtual-tire slip angles, load transfer
// eq. models:3dof:Fz_lon, sigmoid tire eq. models:tire) with the
// lateral-acceleration soft constraint of section "OCP Formulation"
// (pi_ay = |a_y - g_y| - a_bar_y, a_bar_y = M g / (2 K_zy)), in place of the
// SRB model and the ESM.
//
// One lane per candidate: the 7-component state stays in VGPRs; each Euler
// step interpolates the slopes of the terrain cell under the CoM (they give
// roll and pitch) and, when a costmap is set, the cost at the four wheels.
// Arithmetic is fixed by the source (no contraction, explicit fmaf), as in
// the SRB kernel.
#include "plan_internal.h"
#include "rollout_step.h"

namespace plan {
namespace {

// Bilinear interpolant of channel ch (0 h, 1 f_x, 2 f_y, 3 cost) at the
// world point (Px, Py), clamp-to-edge; a NaN coordinate clamps to the grid
// origin, so every cell is inside the grid.
template <int CH>
__device__ __forceinline__ float lookup(const RolloutArgs &a, const CellPos &c) {
    return bil(load_coefs(cell_rsrc(a), c.off, CH), c.tx, c.ty);
}

__device__ __forceinline__ CellPos cell_at(const RolloutArgs &a, float Px, float Py) {
    return cell_pos(a, (Px - a.x0) * a.inv_res, (Py - a.y0) * a.inv_res);
}

// One forward-Euler step of the EST formulation for one candidate: the
// running cost at the node is added to J and the state advanced in place.
__device__ __forceinline__ void est_step(const RolloutArgs &a, float (&st)[7], float &J,
                                         float dd, float ax) {
    const float h = a.h;
    float x = st[0], y = st[1], psi = st[2];
    float vy = st[3], wz = st[4], delta = st[5], vx = st[6];

    // Roll and pitch put b_z on the unit upward normal (-f_x, -f_y, 1)/s
    // under the CoM. With the 1-2-3 convention b_z = (sin th, -cos th sin ph,
    // cos ph cos th), so sin th = -f_x/s, cos th = sqrt(1 + f_y^2)/s,
    // sin ph = f_y/sqrt(1 + f_y^2), cos ph = 1/sqrt(1 + f_y^2).
    const CellPos cg = cell_at(a, x, y);
    const float Tfx = lookup<1>(a, cg), Tfy = lookup<2>(a, cg);
    const float q = fmaf(Tfy, Tfy, 1.0f);
    const float rq = frsq(q), rs = frsq(fmaf(Tfx, Tfx, q));
    const float sth = -Tfx * rs;
    const float cth = (q * rq) * rs;
    const float sph = Tfy * rq;
    const float cph = rq;
    float sps, cps;
    __sincosf(psi, &sps, &cps);
    // rows of the 1-2-3 rotation W <- B that the model uses
    const float R11 = cth * cps, R12 = -(cth * sps);
    const float R21 = fmaf(cps * sph, sth, cph * sps);
    const float R22 = fmaf(-(sph * sth), sps, cph * cps);
    const float R32 = fmaf(cph * sth, sps, cps * sph);
    const float R33 = cph * cth;

    // world velocity of the planar body velocity (v_x, v_y, 0)
    const float vWx = fmaf(R11, vx, R12 * vy);
    const float vWy = fmaf(R21, vx, R22 * vy);
    // gravity in the body frame, R^T (0, 0, -g): lateral and normal parts
    const float gBy = -a.g * R32;
    const float gBz = -a.g * R33;

    // load transfer to the virtual tires from the longitudinal acceleration
    // a_x = vx_dot - omega_z v_y
    const float axb = fmaf(-wz, vy, ax);
    const float Fzf = fmaf(-a.Kzzf, gBz, -(a.Kzx * axb));
    const float Fzr = fmaf(-a.Kzzr, gBz, a.Kzx * axb);
    // virtual-tire slip angles (v_x >= vx_min > 0) and sigmoid tire
    const float ivx = frcp(vx);
    const float af = atan_mm(fmaf(wz, a.Lf, vy) * ivx) - delta;
    const float ar = atan_mm(fmaf(-wz, a.Lr, vy) * ivx);
    const float Caf = a.C * af, Car = a.C * ar;
    const float Fyf = (Fzf * (-Caf * a.mu)) * frsq(fmaf(Caf, Caf, a.mu2));
    const float Fyr = (Fzr * (-Car * a.mu)) * frsq(fmaf(Car, Car, a.mu2));
    const float Fy = Fyf + Fyr;
    const float vyd = fmaf(Fy, a.invM, gBy) - wz * vx;
    const float wzd = fmaf(Fyf * a.Lf, __cosf(delta), -(Fyr * a.Lr)) * a.invJzz;

    // lateral-acceleration measure: a_y - g_y = (F_y,f + F_y,r) / M
    const float pi = fabsf(Fy * a.invM) - a.a_bar_y;
    const float mm = fmaxf(0.0f, fmaf(pi, a.inv_eps_ay, 1.0f));
    float L = fmaf(a.w_c * dd, dd, a.w_t) + (a.sigma * mm) * mm;
    if (a.has_costmap) {
        // costmap at the four wheels, P = p + R rho with the SRB lever arms
        const float R13 = sth, R23 = -(cth * sph);
        const float rz = -a.hR;
        const float bx = fmaf(R13, rz, x), by = fmaf(R23, rz, y);
        float c[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float rx = (w < 2) ? a.Lf : -a.Lr;
            const float ry = (w & 1) ? -a.half_e : a.half_e;
            const float Px = fmaf(R11, rx, fmaf(R12, ry, bx));
            const float Py = fmaf(R21, rx, fmaf(R22, ry, by));
            c[w] = lookup<3>(a, cell_at(a, Px, Py));
        }
        L = L + ((c[0] + c[1]) + (c[2] + c[3]));
    }
    J = fmaf(h, L, J);

    // forward Euler and the steering / speed limits
    x = fmaf(h, vWx, x);
    y = fmaf(h, vWy, y);
    psi = fmaf(h, wz, psi);
    vy = fmaf(h, vyd, vy);
    wz = fmaf(h, wzd, wz);
    delta = clampf_nan(fmaf(h, dd, delta), -a.delta_max, a.delta_max);
    vx = fmaf(h, ax, vx);
    vx = (vx < a.vx_min) ? a.vx_min : vx;
    st[0] = x;
    st[1] = y;
    st[2] = psi;
    st[3] = vy;
    st[4] = wz;
    st[5] = delta;
    st[6] = vx;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void rollout_est(const RolloutArgs a) {
    const int slot = blockIdx.x * BLOCK + threadIdx.x;
    if (slot >= a.K) return;
    const int k = a.order ? min(max(a.order[slot], 0), a.K - 1) : slot;
    const size_t K = (size_t)a.K;
    float st[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) st[q] = a.s0[q];
    float J = 0.0f;
    const float *up = a.controls_lane ? a.controls_lane + slot : a.controls + k;
    // uniform trip counts: a candidate that reaches the goal stays frozen
    for (int n = 0; n < a.N; ++n) {
        const float dd = clampf_nan(up[(2 * (size_t)n) * K], -a.drate_max, a.drate_max);
        const float ax = a.accel_max * clampf_nan(up[(2 * (size_t)n + 1) * K], -1.0f, 1.0f);
        for (int s = 0; s < a.S; ++s) {
            const float gdx = st[0] - a.goal_x, gdy = st[1] - a.goal_y;
            // a candidate at its goal is frozen, so the test stays true
            if (fmaf(gdx, gdx, gdy * gdy) <= a.goal_r2) continue;
            est_step(a, st, J, dd, ax);
        }
    }
    const float gdx = st[0] - a.goal_x, gdy = st[1] - a.goal_y;
    J = fmaf(a.w_g, sqrtf(fmaf(gdx, gdx, gdy * gdy)), J);
    bool fin = isfinite(J);
#pragma unroll
    for (int q = 0; q < 7; ++q) fin = fin && isfinite(st[q]);
    if (!fin) J = __builtin_inff();
    a.cost[k] = J;
    if (a.final_state) {
#pragma unroll
        for (int q = 0; q < 7; ++q) a.final_state[(size_t)q * K + k] = st[q];
    }
}

}  // namespace

hipError_t launch_rollout_est(const RolloutArgs &a, int block, hipStream_t s) {
    const unsigned grid = (unsigned)(((long long)a.K + block - 1) / block);
    if (block == 64) {
        hipLaunchKernelGGL(rollout_est<64>, dim3(grid), dim3(64), 0, s, a);
    } else if (block == 256) {
        hipLaunchKernelGGL(rollout_est<256>, dim3(grid), dim3(256), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace plan
