// Adjoint (reverse-mode) rollout: gradients of each candidate's cost J with
// respect to its control sequence, for gradient refinement of the best
// sampled candidates.
//
// The paper samples because its vehicle model is not analytically
// differentiable (section on the state of the art, and section "Real-Time
// Implementation"); the discretised model used here is differentiable almost
// everywhere, so this file differentiates exactly what the forward kernel
// computes. Conventions at the non-smooth points:
//   * max(a, b) and the clamps pass the gradient to the branch the forward
//     pass took (ties to the first argument / the unclamped value);
//   * the damper's switch at liftoff, the bilinear cell edges, |phi| at 0 and
//     the ESM sign change use the active branch's derivative;
//   * the goal test fixes the exit step: steps after it carry no gradient and
//     the exit time is not differentiated.
//
// Memory: states are checkpointed every C control intervals during the
// forward pass; the backward pass recomputes one segment at a time into a
// [C*S][14][M] scratch (13 state components plus an executed flag) and runs
// the step adjoints in reverse. One lane per candidate (LANES = 1 step code,
// the same arithmetic as the forward kernel).
#include <type_traits>

#include "plan_internal.h"
#include "rollout_step.h"

namespace plan {
namespace {

// Partial derivatives of a channel's bilinear interpolant (cell
// coefficients c = (c0, c_x, c_y, c_xy)) with respect to tx and ty.
__device__ __forceinline__ float dbil_dtx(const float4 &c, float ty) { return fmaf(ty, c.w, c.y); }
__device__ __forceinline__ float dbil_dty(const float4 &c, float tx) { return fmaf(tx, c.w, c.z); }

// Adjoint contributions of one wheel to the chassis quantities it reads:
// the rotation matrix, the rear constraint force, cos(delta), delta, the
// body velocities and rates, and the CoM position.
struct WheelAdj {
    float R11, R12, R13, R21, R22, R23, R31, R32, R33;
    float FxR, cosd, delta;
    float vx, vy, vz, wx, wy, wz;
    float x, y, z;
};

__device__ __forceinline__ WheelAdj adj_add(const WheelAdj &p, const WheelAdj &q) {
    WheelAdj o;
    o.R11 = p.R11 + q.R11; o.R12 = p.R12 + q.R12; o.R13 = p.R13 + q.R13;
    o.R21 = p.R21 + q.R21; o.R22 = p.R22 + q.R22; o.R23 = p.R23 + q.R23;
    o.R31 = p.R31 + q.R31; o.R32 = p.R32 + q.R32; o.R33 = p.R33 + q.R33;
    o.FxR = p.FxR + q.FxR; o.cosd = p.cosd + q.cosd; o.delta = p.delta + q.delta;
    o.vx = p.vx + q.vx; o.vy = p.vy + q.vy; o.vz = p.vz + q.vz;
    o.wx = p.wx + q.wx; o.wy = p.wy + q.wy; o.wz = p.wz + q.wz;
    o.x = p.x + q.x; o.y = p.y + q.y; o.z = p.z + q.z;
    return o;
}

// Sum over the candidate's lanes, in the forward pass's fixed order
// (w0 + w1) + (w2 + w3).
template <int LANES>
__device__ __forceinline__ WheelAdj adj_group_sum(WheelAdj v) {
    v.R11 = group_sum<LANES>(v.R11); v.R12 = group_sum<LANES>(v.R12);
    v.R13 = group_sum<LANES>(v.R13); v.R21 = group_sum<LANES>(v.R21);
    v.R22 = group_sum<LANES>(v.R22); v.R23 = group_sum<LANES>(v.R23);
    v.R31 = group_sum<LANES>(v.R31); v.R32 = group_sum<LANES>(v.R32);
    v.R33 = group_sum<LANES>(v.R33);
    v.FxR = group_sum<LANES>(v.FxR); v.cosd = group_sum<LANES>(v.cosd);
    v.delta = group_sum<LANES>(v.delta);
    v.vx = group_sum<LANES>(v.vx); v.vy = group_sum<LANES>(v.vy);
    v.vz = group_sum<LANES>(v.vz); v.wx = group_sum<LANES>(v.wx);
    v.wy = group_sum<LANES>(v.wy); v.wz = group_sum<LANES>(v.wz);
    v.x = group_sum<LANES>(v.x); v.y = group_sum<LANES>(v.y); v.z = group_sum<LANES>(v.z);
    return v;
}

// Vector-Jacobian product of one Euler step (state st, applied controls dd,
// ax) for one candidate whose wheels are split over LANES lanes (this lane
// holds `arms`). In: lam = dJ/d(next state), wJ = dJ/d(running cost). Out:
// lam = dJ/d(this state), *g_dd, *g_ax = dJ/d(dd), dJ/d(ax) through this
// step; identical in every lane of the group.
template <int LANES, class Hook = NoHook>
__device__ void step_vjp(const RolloutArgs &a, const Arm (&arms)[4 / LANES],
                         const float (&st)[13], float dd, float ax, float wJ, float (&lam)[13],
                         float *g_dd, float *g_ax, const Hook &hook = Hook()) {
    constexpr int WPL = 4 / LANES;
    const float h = a.h;
    const float half_pi = 1.57079632679489662f;
    const float x = st[0], y = st[1], z = st[2];
    const float psi = st[3], th = st[4], ph = st[5];
    const float vx = st[6], vy = st[7], vz = st[8];
    const float wx = st[9], wy = st[10], wz = st[11];
    const float delta = st[12];

    // ---------------------------------------------------------- forward
    float sps, cps;
    __sincosf(psi, &sps, &cps);
    const Attitude A = attitude(psi, th, ph);
    const float ss = A.sph * A.sth, cs = A.cph * A.sth;
    const float icth = frcp(A.cth);
    const float t1 = fmaf(A.sph, wy, A.cph * wz);
    const float psid = t1 * icth;
    const float cosd = __cosf(delta);
    const float sind = __sinf(delta);
    const float ang = fabsf(ph) + a.phibar;
    const float sang = __sinf(ang), cang = __cosf(ang);
    const float sgn = (ang > half_pi) ? -1.0f : 1.0f;
    float U = (a.MgRbar * (1.0f - sang)) * A.cth;
    U = sgn * U;
    const float mm_raw = fmaf(-U, a.inv_eps_esm, 1.0f);
    const float mm = fmaxf(0.0f, mm_raw);

    // this lane's wheels: forward quantities
    float P_z[WPL], cl_u[WPL], cl_v[WPL], txv[WPL], tyv[WPL];
    float4 CH[WPL], CFX[WPL], CFY[WPL], CC[WPL];
    float vix[WPL], viy[WPL], viz[WPL], th_[WPL], tfx[WPL], tfy[WPL];
    float nBx[WPL], nBy[WPL], nBz[WPL], inz[WPL], chi[WPL], relx[WPL], rely[WPL], Dv[WPL],
        chid[WPL];
    float Fkr[WPL], Fk[WPL], Fb[WPL], Fz[WPL], rr[WPL], alpha[WPL], Ca[WPL], qq[WPL], Fyv[WPL];
    bool guard[WPL], fb_first[WPL];
    // terrain requests of this lane's wheels first; the hook's loads are
    // issued after them
    const GridPos gp = grid_pos(a, x, y);
    Gather G[WPL];
#pragma unroll
    for (int i = 0; i < WPL; ++i) G[i] = gather(a, A, gp, z, arms[i]);
    if constexpr (!std::is_same<Hook, NoHook>::value) {
        __builtin_amdgcn_sched_barrier(0);
        hook();
    }
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
        const Arm r = arms[i];
        // the lookup coordinates as the gather computed them
        const float ur = fmaf(A.R11, r.gx, fmaf(A.R12, r.gy, fmaf(A.R13, r.gz, gp.xg)));
        const float vr = fmaf(A.R21, r.gx, fmaf(A.R22, r.gy, fmaf(A.R23, r.gz, gp.yg)));
        cl_u[i] = (ur > 0.0f && ur < a.umax) ? 1.0f : 0.0f;  // NaN: clamped
        cl_v[i] = (vr > 0.0f && vr < a.vmax) ? 1.0f : 0.0f;
        const Gather &g = G[i];
        P_z[i] = g.Pz;
        txv[i] = g.tx;
        tyv[i] = g.ty;
        CH[i] = g.ch;
        CFX[i] = g.cfx;
        CFY[i] = g.cfy;
        CC[i] = g.cc;
        vix[i] = fmaf(wy, r.rz, fmaf(-wz, r.ry, vx));
        viy[i] = fmaf(wz, r.rx, fmaf(-wx, r.rz, vy));
        viz[i] = fmaf(wx, r.ry, fmaf(-wy, r.rx, vz));
        th_[i] = bil(g.ch, g.tx, g.ty);
        tfx[i] = bil(g.cfx, g.tx, g.ty);
        tfy[i] = bil(g.cfy, g.tx, g.ty);
        nBx[i] = fmaf(-A.R11, tfx[i], fmaf(-A.R21, tfy[i], A.R31));
        nBy[i] = fmaf(-A.R12, tfx[i], fmaf(-A.R22, tfy[i], A.R32));
        nBz[i] = fmaf(-A.R13, tfx[i], fmaf(-A.R23, tfy[i], A.R33));
        inz[i] = frcp(nBz[i]);
        chi[i] = (P_z[i] - th_[i]) * inz[i];
        relx[i] = fmaf(-chi[i], wy, vix[i]);
        rely[i] = fmaf(chi[i], wx, viy[i]);
        Dv[i] = fmaf(nBx[i], relx[i], fmaf(nBy[i], rely[i], nBz[i] * viz[i]));
        chid[i] = Dv[i] * inz[i];
        const float Fs = r.front ? a.Fsf : a.Fsr;
        const float k = r.front ? a.kf : a.kr;
        const float b = r.front ? a.bf : a.br;
        Fkr[i] = fmaf(-k, chi[i], Fs);
        Fk[i] = fmaxf(Fkr[i], 0.0f);
        fb_first[i] = (-b * chid[i]) >= -Fk[i];
        Fb[i] = (Fk[i] > 0.0f) ? fmaxf(-b * chid[i], -Fk[i]) : 0.0f;
        Fz[i] = Fk[i] + Fb[i];
        const float dl = r.front ? delta : 0.0f;
        guard[i] = (vix[i] == 0.0f && viy[i] == 0.0f);
        rr[i] = guard[i] ? 0.0f : viy[i] * frcp(vix[i]);
        alpha[i] = guard[i] ? -dl : atan_mm(rr[i]) - dl;
        Ca[i] = a.C * alpha[i];
        qq[i] = frsq(fmaf(Ca[i], Ca[i], a.mu2));
        Fyv[i] = (Fz[i] * (-Ca[i] * a.mu)) * qq[i];
    }
    const float vx_new = fmaf(h, ax, vx);
    const float d_new = fmaf(h, dd, delta);
    const float gate_v = (vx_new < a.vx_min) ? 0.0f : 1.0f;
    const float gate_d = (d_new < -a.delta_max || d_new > a.delta_max) ? 0.0f : 1.0f;

    // ---------------------------------------------------------- reverse
    // Euler update and clamps
    float L_x = lam[0], L_y = lam[1], L_z = lam[2];
    float L_psi = lam[3], L_th = lam[4], L_ph = lam[5];
    float L_vx = gate_v * lam[6], L_vy = lam[7], L_vz = lam[8];
    float L_wx = lam[9], L_wy = lam[10], L_wz = lam[11];
    float L_delta = gate_d * lam[12];
    float L_dd = gate_d * h * lam[12];
    float L_ax = gate_v * h * lam[6];
    const float L_vWx = h * lam[0], L_vWy = h * lam[1], L_vWz = h * lam[2];
    const float L_psid0 = h * lam[3], L_thd = h * lam[4], L_phd = h * lam[5];
    const float L_vyd = h * lam[7], L_vzd = h * lam[8];
    const float L_wxd = h * lam[9], L_wyd = h * lam[10], L_wzd = h * lam[11];

    // running cost L = w_t + w_c dd^2 + sigma m^2 + csum, weight h*wJ
    const float L_L = h * wJ;
    L_dd += L_L * 2.0f * a.w_c * dd;
    const float L_mm = L_L * 2.0f * a.sigma * mm;
    const float L_csum = L_L;
    const float L_U = (mm_raw >= 0.0f) ? -a.inv_eps_esm * L_mm : 0.0f;
    // U = sgn * MgRbar (1 - sin ang) cos th
    const float L_ang = sgn * a.MgRbar * (-cang) * A.cth * L_U;
    float L_cth = sgn * a.MgRbar * (1.0f - sang) * L_U;
    L_ph += (ph < 0.0f ? -1.0f : 1.0f) * L_ang;

    // right-hand side rows
    float L_Fy = a.invM * L_vyd, L_Fz = a.invM * L_vzd;
    float L_gBy = L_vyd, L_gBz = L_vzd;
    L_wx += vz * L_vyd;
    L_vz += wx * L_vyd;
    L_wz -= vx * L_vyd;
    L_vx -= wz * L_vyd;
    L_wx -= vy * L_vzd;
    L_vy -= wx * L_vzd;
    L_wy += vx * L_vzd;
    L_vx += wy * L_vzd;
    const float L_Mx = a.invJxx * L_wxd, L_My = a.invJyy * L_wyd, L_Mz = a.invJzz * L_wzd;
    L_wy += a.dJyz * wz * L_Mx;
    L_wz += a.dJyz * wy * L_Mx;
    L_wx -= a.dJxz * wz * L_My;
    L_wz -= a.dJxz * wx * L_My;
    L_wx += a.dJxy * wy * L_Mz;
    L_wy += a.dJxy * wx * L_Mz;

    // per-wheel reverse: each of this lane's wheels into its own WheelAdj,
    // then the fixed-order sum over the candidate's wheels
    WheelAdj wadj[WPL];
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
        const Arm r = arms[i];
        WheelAdj W = {};
        // moments and force sums
        float L_fy = L_Fy - r.rz * L_Mx + r.rx * L_Mz;
        float L_Fzw = L_Fz + r.ry * L_Mx - r.rx * L_My;
        const float L_Fxw = r.rz * L_My - r.ry * L_Mz;
        if (!r.front) W.FxR += L_Fxw;
        float L_Fyw = L_fy;
        if (r.front) {
            W.cosd += Fyv[i] * L_fy;
            L_Fyw = cosd * L_fy;
        }
        // Fy = (Fz * (-Ca mu)) * q, q = rsqrt(mu^2 + Ca^2)
        const float P1 = Fz[i] * (-Ca[i] * a.mu);
        const float L_P1 = qq[i] * L_Fyw;
        const float L_q = P1 * L_Fyw;
        L_Fzw += (-Ca[i] * a.mu) * L_P1;
        float L_Ca = Fz[i] * (-a.mu) * L_P1;
        L_Ca += -Ca[i] * qq[i] * qq[i] * qq[i] * L_q;
        const float L_alpha = a.C * L_Ca;
        if (r.front) W.delta -= L_alpha;
        float L_vix = 0.0f, L_viy = 0.0f, L_viz = 0.0f;
        if (!guard[i]) {
            const float L_r = L_alpha / fmaf(rr[i], rr[i], 1.0f);
            const float ivx = frcp(vix[i]);
            L_viy += ivx * L_r;
            L_vix += -rr[i] * ivx * L_r;
        }
        // Fz = Fk + Fb
        float L_Fk = L_Fzw;
        float L_chid = 0.0f;
        if (Fk[i] > 0.0f) {
            const float b = r.front ? a.bf : a.br;
            if (fb_first[i])
                L_chid += -b * L_Fzw;
            else
                L_Fk += -L_Fzw;
        }
        float L_chi = 0.0f;
        if (Fkr[i] >= 0.0f) L_chi += -(r.front ? a.kf : a.kr) * L_Fk;
        // chid = D * inz
        const float L_D = inz[i] * L_chid;
        float L_inz = Dv[i] * L_chid;
        float L_nBx = relx[i] * L_D, L_nBy = rely[i] * L_D, L_nBz = viz[i] * L_D;
        const float L_relx = nBx[i] * L_D, L_rely = nBy[i] * L_D;
        L_viz += nBz[i] * L_D;
        L_vix += L_relx;
        L_chi += -wy * L_relx;
        W.wy += -chi[i] * L_relx;
        L_viy += L_rely;
        L_chi += wx * L_rely;
        W.wx += chi[i] * L_rely;
        // chi = (Pz - h) * inz
        float L_Pz = inz[i] * L_chi;
        const float L_hgt = -inz[i] * L_chi;
        L_inz += (P_z[i] - th_[i]) * L_chi;
        L_nBz += -inz[i] * inz[i] * L_inz;
        // normal in body frame
        W.R31 += L_nBx;
        W.R11 += -tfx[i] * L_nBx;
        W.R21 += -tfy[i] * L_nBx;
        W.R32 += L_nBy;
        W.R12 += -tfx[i] * L_nBy;
        W.R22 += -tfy[i] * L_nBy;
        W.R33 += L_nBz;
        W.R13 += -tfx[i] * L_nBz;
        W.R23 += -tfy[i] * L_nBz;
        const float L_tfx = -A.R11 * L_nBx - A.R12 * L_nBy - A.R13 * L_nBz;
        const float L_tfy = -A.R21 * L_nBx - A.R22 * L_nBy - A.R23 * L_nBz;
        // bilinear terrain: d/dtx, d/dty of (h, f_x, f_y, c)
        const float tx = txv[i], ty = tyv[i];
        const float L_tx = L_hgt * dbil_dtx(CH[i], ty) + L_tfx * dbil_dtx(CFX[i], ty) +
                           L_tfy * dbil_dtx(CFY[i], ty) + L_csum * dbil_dtx(CC[i], ty);
        const float L_ty = L_hgt * dbil_dty(CH[i], tx) + L_tfx * dbil_dty(CFX[i], tx) +
                           L_tfy * dbil_dty(CFY[i], tx) + L_csum * dbil_dty(CC[i], tx);
        const float L_Px = cl_u[i] * a.inv_res * L_tx;
        const float L_Py = cl_v[i] * a.inv_res * L_ty;
        // contact-point velocity
        W.vx += L_vix;
        W.wy += r.rz * L_vix;
        W.wz += -r.ry * L_vix;
        W.vy += L_viy;
        W.wz += r.rx * L_viy;
        W.wx += -r.rz * L_viy;
        W.vz += L_viz;
        W.wx += r.ry * L_viz;
        W.wy += -r.rx * L_viz;
        // contact point
        W.x += L_Px;
        W.R11 += r.rx * L_Px;
        W.R12 += r.ry * L_Px;
        W.R13 += r.rz * L_Px;
        W.y += L_Py;
        W.R21 += r.rx * L_Py;
        W.R22 += r.ry * L_Py;
        W.R23 += r.rz * L_Py;
        W.z += L_Pz;
        W.R31 += r.rx * L_Pz;
        W.R32 += r.ry * L_Pz;
        W.R33 += r.rz * L_Pz;
        wadj[i] = W;
    }
    WheelAdj wsum;
    if constexpr (WPL == 4)
        wsum = adj_add(adj_add(wadj[0], wadj[1]), adj_add(wadj[2], wadj[3]));
    else if constexpr (WPL == 2)
        wsum = adj_add(wadj[0], wadj[1]);
    else
        wsum = wadj[0];
    wsum = adj_group_sum<LANES>(wsum);
    float L_R11 = wsum.R11, L_R12 = wsum.R12, L_R13 = wsum.R13;
    float L_R21 = wsum.R21, L_R22 = wsum.R22, L_R23 = wsum.R23;
    float L_R31 = wsum.R31, L_R32 = wsum.R32, L_R33 = wsum.R33;
    const float L_FxR = wsum.FxR, L_cosd = wsum.cosd;
    L_delta += wsum.delta;
    L_vx += wsum.vx;
    L_vy += wsum.vy;
    L_vz += wsum.vz;
    L_wx += wsum.wx;
    L_wy += wsum.wy;
    L_wz += wsum.wz;
    L_x += wsum.x;
    L_y += wsum.y;
    L_z += wsum.z;


    // chassis
    L_delta += -sind * L_cosd;
    // FxR = Mhalf (wy vz - wz vy + ax - gBx)
    L_wy += a.Mhalf * vz * L_FxR;
    L_vz += a.Mhalf * wy * L_FxR;
    L_wz += -a.Mhalf * vy * L_FxR;
    L_vy += -a.Mhalf * wz * L_FxR;
    L_ax += a.Mhalf * L_FxR;
    const float L_gBx = -a.Mhalf * L_FxR;
    float L_sth = a.g * L_gBx;
    L_cth += -a.g * A.sph * L_gBy;
    float L_sph = -a.g * A.cth * L_gBy;
    float L_cph = -a.g * A.cth * L_gBz;
    L_cth += -a.g * A.cph * L_gBz;
    // Euler-angle rates
    float L_psid = L_psid0 + A.sth * L_phd;
    L_sth += psid * L_phd;
    L_wx += L_phd;
    L_cph += wy * L_thd;
    L_wy += A.cph * L_thd;
    L_sph += -wz * L_thd;
    L_wz += -A.sph * L_thd;
    const float L_t1 = icth * L_psid;
    const float L_icth = t1 * L_psid;
    L_sph += wy * L_t1;
    L_wy += A.sph * L_t1;
    L_cph += wz * L_t1;
    L_wz += A.cph * L_t1;
    L_cth += -icth * icth * L_icth;
    // world velocity v_W = R v
    L_R11 += vx * L_vWx;
    L_R12 += vy * L_vWx;
    L_R13 += vz * L_vWx;
    L_R21 += vx * L_vWy;
    L_R22 += vy * L_vWy;
    L_R23 += vz * L_vWy;
    L_R31 += vx * L_vWz;
    L_R32 += vy * L_vWz;
    L_R33 += vz * L_vWz;
    L_vx += A.R11 * L_vWx + A.R21 * L_vWy + A.R31 * L_vWz;
    L_vy += A.R12 * L_vWx + A.R22 * L_vWy + A.R32 * L_vWz;
    L_vz += A.R13 * L_vWx + A.R23 * L_vWy + A.R33 * L_vWz;
    // rotation matrix entries
    float L_cps = A.cth * L_R11, L_sps = 0.0f, L_ss = 0.0f, L_cs = 0.0f;
    L_cth += cps * L_R11;
    L_cps += ss * L_R12;
    L_ss += cps * L_R12;
    L_cph += -sps * L_R12;
    L_sps += -A.cph * L_R12;
    L_cps += cs * L_R13;
    L_cs += cps * L_R13;
    L_sph += sps * L_R13;
    L_sps += A.sph * L_R13;
    L_sps += A.cth * L_R21;
    L_cth += sps * L_R21;
    L_sps += ss * L_R22;
    L_ss += sps * L_R22;
    L_cph += cps * L_R22;
    L_cps += A.cph * L_R22;
    L_sps += cs * L_R23;
    L_cs += sps * L_R23;
    L_cps += -A.sph * L_R23;
    L_sph += -cps * L_R23;
    L_sth += -L_R31;
    L_cth += A.sph * L_R32;
    L_sph += A.cth * L_R32;
    L_cph += A.cth * L_R33;
    L_cth += A.cph * L_R33;
    L_sph += A.sth * L_ss;
    L_sth += A.sph * L_ss;
    L_cph += A.sth * L_cs;
    L_sth += A.cph * L_cs;
    // trigonometric functions of the angles
    L_psi += cps * L_sps - sps * L_cps;
    L_th += A.cth * L_sth - A.sth * L_cth;
    L_ph += A.cph * L_sph - A.sph * L_cph;

    lam[0] = L_x;
    lam[1] = L_y;
    lam[2] = L_z;
    lam[3] = L_psi;
    lam[4] = L_th;
    lam[5] = L_ph;
    lam[6] = L_vx;
    lam[7] = L_vy;
    lam[8] = L_vz;
    lam[9] = L_wx;
    lam[10] = L_wy;
    lam[11] = L_wz;
    lam[12] = L_delta;
    *g_dd = L_dd;
    *g_ax = L_ax;
}

// Backward pass over checkpointed segments; LANES lanes per candidate, the
// wheels split over them as in the forward kernel.
//   ckpt:    [nseg+1][13][K]: state at the start of each segment of C
//            intervals (segment nseg: the final state)
//   weight:  [K] dJ/dJ_k seeds (NULL = 1)
//   cost:    [K] the forward costs (+inf rows get zero gradients)
//   scratch: [C*S][14][K] recomputed states plus an executed flag (every
//            lane of a group writes and reads back the same values)
//   grad:    [N][2][K] output dJ/du
template <int LANES>
__global__ __launch_bounds__(64) void adjoint_backward(const RolloutArgs a, int C,
                                                       const float *__restrict__ ckpt,
                                                       const float *__restrict__ weight,
                                                       float *__restrict__ scratch,
                                                       float *__restrict__ grad) {
    constexpr int WPL = 4 / LANES;
    const int gtid = blockIdx.x * 64 + threadIdx.x;
    const int sub = gtid & (LANES - 1);
    const int k = gtid / LANES;
    // whole lane groups past K leave together (64 is a multiple of LANES)
    if (k >= a.K) return;
    const size_t K = (size_t)a.K;
    const int N = a.N, S = a.S;
    const int nseg = (N + C - 1) / C;
    const float wJ = weight ? weight[k] : 1.0f;
    const float Jk = a.cost[k];
    const float *up = a.controls + k;
    if (!isfinite(Jk)) {
        if (sub == 0)
            for (int e = 0; e < 2 * N; ++e) grad[(size_t)e * K + k] = 0.0f;
        return;
    }
    // terminal cost Phi = w_g |(x, y) - goal| at the final state
    float lam[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) lam[q] = 0.0f;
    {
        const float xf = ckpt[((size_t)nseg * 13 + 0) * K + k];
        const float yf = ckpt[((size_t)nseg * 13 + 1) * K + k];
        const float gdx = xf - a.goal_x, gdy = yf - a.goal_y;
        const float dist = sqrtf(fmaf(gdx, gdx, gdy * gdy));
        if (dist > 0.0f) {
            lam[0] = wJ * a.w_g * gdx / dist;
            lam[1] = wJ * a.w_g * gdy / dist;
        }
    }
    Arm arms[WPL];
#pragma unroll
    for (int q = 0; q < WPL; ++q) arms[q] = arm(a, sub * WPL + q);

    // Loads are issued one step ahead from inside the step (after its terrain
    // requests): the next interval's controls in the recomputation, the
    // previous step's recomputed state and controls in the reverse sweep.
    // Indices are clamped to the segment, so every load stays in bounds.
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int n0 = seg * C;
        const int n1 = min(N, n0 + C);
        // recompute the segment's states
        float st[13];
#pragma unroll
        for (int q = 0; q < 13; ++q) st[q] = ckpt[((size_t)seg * 13 + q) * K + k];
        float Jdummy = 0.0f;
        int idx = 0;
        float nu0 = up[(2 * (size_t)n0) * K], nu1 = up[(2 * (size_t)n0 + 1) * K];
        for (int n = n0; n < n1; ++n) {
            const float dd = clampf_nan(nu0, -a.drate_max, a.drate_max);
            const float ax = a.accel_max * clampf_nan(nu1, -1.0f, 1.0f);
            const size_t nn = (size_t)min(n + 1, n1 - 1);
            for (int s = 0; s < S; ++s, ++idx) {
                float *sl = scratch + ((size_t)idx * 14) * K + k;
#pragma unroll
                for (int q = 0; q < 13; ++q) sl[(size_t)q * K] = st[q];
                const float gdx = st[0] - a.goal_x, gdy = st[1] - a.goal_y;
                const bool live = !(fmaf(gdx, gdx, gdy * gdy) <= a.goal_r2);
                sl[(size_t)13 * K] = live ? 1.0f : 0.0f;
                // a step that is not live leaves the state frozen, so no later
                // step of this candidate is live and the stale controls are
                // never applied
                if (live)
                    euler_step<LANES>(a, arms, st, Jdummy, dd, ax, [&]() {
                        nu0 = up[(2 * nn) * K];
                        nu1 = up[(2 * nn + 1) * K];
                    });
            }
        }
        // reverse through the segment, one step at a time (flat index i)
        const int cnt = (n1 - n0) * S;
        float cur[14];
        {
            const float *sl = scratch + ((size_t)(cnt - 1) * 14) * K + k;
#pragma unroll
            for (int q = 0; q < 14; ++q) cur[q] = sl[(size_t)q * K];
        }
        float cu0 = up[(2 * (size_t)(n1 - 1)) * K], cu1 = up[(2 * (size_t)(n1 - 1) + 1) * K];
        float gdd = 0.0f, gax = 0.0f;
        // (n, s): interval and substep of flat index i, stepped down with i
        // (no divisions in the loop)
        int n = n1 - 1, s = S - 1;
        for (int i = cnt - 1; i >= 0; --i) {
            const float u0 = cu0, u1 = cu1;
            const float dd = clampf_nan(u0, -a.drate_max, a.drate_max);
            const float ax = a.accel_max * clampf_nan(u1, -1.0f, 1.0f);
            const int ip = max(i - 1, 0);
            const size_t np = (size_t)(i == 0 ? n0 : (s > 0 ? n : n - 1));
            const float *slp = scratch + ((size_t)ip * 14) * K + k;
            float nxt[14], nu0, nu1;
            auto prefetch = [&]() {
#pragma unroll
                for (int q = 0; q < 14; ++q) nxt[q] = slp[(size_t)q * K];
                nu0 = up[(2 * np) * K];
                nu1 = up[(2 * np + 1) * K];
            };
            if (cur[13] != 0.0f) {  // executed (not after the goal exit)
                float sti[13];
#pragma unroll
                for (int q = 0; q < 13; ++q) sti[q] = cur[q];
                float g1, g2;
                step_vjp<LANES>(a, arms, sti, dd, ax, wJ, lam, &g1, &g2, prefetch);
                gdd += g1;
                gax += g2;
            } else {
                prefetch();
            }
            if (s == 0) {
                // first substep of interval n: its gradient is complete;
                // through the admissible-set clamps (identity branch inside)
                const bool in0 = !(u0 < -a.drate_max) && !(u0 > a.drate_max);
                const bool in1 = !(u1 < -1.0f) && !(u1 > 1.0f);
                if (sub == 0) {
                    grad[(2 * (size_t)n) * K + k] = in0 ? gdd : 0.0f;
                    grad[(2 * (size_t)n + 1) * K + k] = in1 ? a.accel_max * gax : 0.0f;
                }
                gdd = 0.0f;
                gax = 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 14; ++q) cur[q] = nxt[q];
            cu0 = nu0;
            cu1 = nu1;
            if (s == 0) {
                s = S - 1;
                --n;
            } else {
                --s;
            }
        }
    }
}

}  // namespace

hipError_t launch_adjoint_backward(const RolloutArgs &a, int C, const float *ckpt,
                                   const float *weight, float *scratch, float *grad, int lanes,
                                   hipStream_t s) {
    const unsigned grid = (unsigned)(((long long)a.K * lanes + 63) / 64);
    if (lanes == 1)
        hipLaunchKernelGGL(adjoint_backward<1>, dim3(grid), dim3(64), 0, s, a, C, ckpt, weight,
                           scratch, grad);
    else if (lanes == 2)
        hipLaunchKernelGGL(adjoint_backward<2>, dim3(grid), dim3(64), 0, s, a, C, ckpt, weight,
                           scratch, grad);
    else if (lanes == 4)
        hipLaunchKernelGGL(adjoint_backward<4>, dim3(grid), dim3(64), 0, s, a, C, ckpt, weight,
                           scratch, grad);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace plan
