// Device code of one forward-Euler step of the SRB model with its stage
// cost, shared by the rollout kernels and the adjoint (which recomputes the
// forward pass from checkpoints and must see the same arithmetic).
// Arithmetic is fixed by the source: the library is compiled without
// floating-point contraction and every fused multiply-add is an explicit fmaf.
#pragma once

#include <type_traits>

#include "plan_internal.h"

namespace plan {

// ----------------------------------------------------------------- math ----
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// DPP quad permutations: swap with lane^1 and lane^2 inside each quad.
__device__ __forceinline__ float dpp_xor1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor2(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}

template <int LANES>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (LANES >= 2) v = v + dpp_xor1(v);
    if constexpr (LANES >= 4) v = v + dpp_xor2(v);
    return v;
}

// Arctangent of the slip angles: x + x^3 P(x^2) on [0, 1], P of degree 5
// with coefficients that minimise the largest absolute error over the
// interval (a discrete minimax fit solved as a linear program; fit_atan.py in
// the package prints them and the bound), and pi/2 - atan(1/|x|) beyond, with
// the sign of x. Largest absolute error in float32 evaluation 4.3e-7 on
// [-1, 1] and below 6e-7 beyond, where the reciprocal and the subtraction
// round as well (the library's sine and cosine are of order 1e-6);
// atan(+-inf) = +-pi/2. NAN_TO_ZERO: a NaN argument gives 0 (|x| is taken
// as the IEEE maximum of |x| and 0, which returns 0 for a NaN), the slip
// ratio's 0/0 convention at no extra instruction; otherwise NaN gives NaN.
template <bool NAN_TO_ZERO = false>
__device__ __forceinline__ float atan_mm(float x) {
    const float ax = NAN_TO_ZERO ? fmaxf(fabsf(x), 0.0f) : fabsf(x);
    const bool big = ax > 1.0f;
    const float r = big ? frcp(ax) : ax;
    const float t = r * r;
    float p = 7.331810426e-03f;
    p = fmaf(p, t, -3.539908305e-02f);
    p = fmaf(p, t, 8.204584569e-02f);
    p = fmaf(p, t, -1.339402497e-01f);
    p = fmaf(p, t, 1.986153722e-01f);
    p = fmaf(p, t, -3.332552314e-01f);
    float y = fmaf(r * t, p, r);
    y = big ? 1.57079632679489662f - y : y;
    return copysignf(y, x);
}

// NaN-propagating clamp (a NaN input stays NaN, as in the reference
// arithmetic; the candidate is then scored +inf at the end). v_med3 returns
// the clamped value for every non-NaN input, -0.0 included.
__device__ __forceinline__ float clampf_nan(float x, float lo, float hi) {
    const float m = __builtin_amdgcn_fmed3f(x, lo, hi);
    return x != x ? x : m;
}

// Attitude terms of the 3-2-1 rotation W <- B.
// Hardware sine/cosine (v_sin_f32 / v_cos_f32): absolute error of order 1e-6,
// far below the trajectory's own float32 sensitivity.
struct Attitude {
    float sth, cth, sph, cph;
    float R11, R12, R13, R21, R22, R23, R31, R32, R33;
};

__device__ __forceinline__ Attitude attitude(float psi, float th, float ph) {
    float sps, cps;
    Attitude A;
    __sincosf(psi, &sps, &cps);
    __sincosf(th, &A.sth, &A.cth);
    __sincosf(ph, &A.sph, &A.cph);
    const float ss = A.sph * A.sth, cs = A.cph * A.sth;
    A.R11 = cps * A.cth;
    A.R12 = fmaf(cps, ss, -(A.cph * sps));
    A.R13 = fmaf(cps, cs, A.sph * sps);
    A.R21 = A.cth * sps;
    A.R22 = fmaf(sps, ss, A.cph * cps);
    A.R23 = fmaf(sps, cs, -(cps * A.sph));
    A.R31 = -A.sth;
    A.R32 = A.cth * A.sph;
    A.R33 = A.cph * A.cth;
    return A;
}

// Body-frame lever arm of wheel wi (fl, fr, rl, rr): constant in the body
// frame; (gx, gy, gz) is the same arm in grid units (times 1 / res).
struct Arm {
    float rx, ry, rz;
    float gx, gy, gz;
    bool front, left;  // left: ry = +e/2
};

__device__ __forceinline__ Arm arm(const RolloutArgs &a, int wi) {
    Arm r;
    r.front = wi < 2;
    r.left = (wi & 1) == 0;
    r.rx = r.front ? a.Lf : -a.Lr;
    r.ry = (wi & 1) ? -a.half_e : a.half_e;
    r.rz = -a.hR;
    r.gx = r.front ? a.Lf_g : -a.Lr_g;
    r.gy = (wi & 1) ? -a.half_e_g : a.half_e_g;
    r.gz = -a.hR_g;
    return r;
}

// CoM position in grid units, (x - x0) / res and (y - y0) / res, from
// which every wheel's lookup coordinate follows as u = xg + (R rho)_x / res.
struct GridPos {
    float xg, yg;
};

__device__ __forceinline__ GridPos grid_pos(const RolloutArgs &a, float x, float y) {
    return GridPos{fmaf(x, a.inv_res, -a.x0_g), fmaf(y, a.inv_res, -a.y0_g)};
}

// The terrain cell under a wheel's contact point: the bilinear coefficients
// of its channels and the weights; the loads are issued here and consumed
// in wheel(), so the gathers are in flight while the chassis terms are
// computed.
struct Gather {
    float4 ch, cfx, cfy, cc;  // (c0, c_x, c_y, c_xy) of h, f_x, f_y, cost
    float tx, ty, Pz;
};

// Buffer resource over the W x H cells of 64 bytes (fewer than 2^26 cells, a
// limit plan_create and plan_server_create enforce, so every byte offset
// fits in 32 bits). A buffer load takes a 32-bit offset from a scalar base
// instead of a 64-bit address per lane.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cell_rsrc(const RolloutArgs &a) {
    const unsigned bytes = (unsigned)(a.W * a.H) << 6;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float4 *>(a.cells), 0, (int)bytes,
                                             0x00020000);
}

// One channel's coefficients: the cell's byte offset plus 16 x channel,
// the channel offset as the load's scalar offset.
__device__ __forceinline__ float4 load_coefs(__amdgpu_buffer_rsrc_t rs, unsigned off, int ch) {
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 16 * ch, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                       __uint_as_float(v.w));
}

// Cell index and weights of lookup coordinates (u, v) in grid units:
// clamp-to-edge with v_med3, which on gfx950 gives min(max(x, 0), umax) for
// every input and maps a NaN coordinate to 0, so the cell is always inside
// the grid. With u >= 0 the integer part (truncation) and the fraction
// (v_fract) split u exactly; u = W-1 on the edge selects the last column's
// cell at weight 0.
struct CellPos {
    unsigned off;  // byte offset of the cell
    float tx, ty;
};

__device__ __forceinline__ CellPos cell_pos(const RolloutArgs &a, float ur, float vr) {
    const float u = __builtin_amdgcn_fmed3f(ur, 0.0f, a.umax);
    const float v = __builtin_amdgcn_fmed3f(vr, 0.0f, a.vmax);
    CellPos p;
    p.tx = __builtin_amdgcn_fractf(u);
    p.ty = __builtin_amdgcn_fractf(v);
    p.off = (unsigned)((int)v * a.W + (int)u) << 6;
    return p;
}

// CM: the context has a costmap; without one only (h, f_x, f_y) are loaded
// and the cost channel is neither interpolated nor summed (it is 0 there, so
// the results are the same bits).
template <bool CM = true>
__device__ __forceinline__ Gather gather(const RolloutArgs &a, const Attitude &A,
                                         const GridPos &p, float z, const Arm &r) {
    // contact point P = p + R rho: its height in the world, its horizontal
    // position as lookup coordinates in grid units
    const float ur = fmaf(A.R11, r.gx, fmaf(A.R12, r.gy, fmaf(A.R13, r.gz, p.xg)));
    const float vr = fmaf(A.R21, r.gx, fmaf(A.R22, r.gy, fmaf(A.R23, r.gz, p.yg)));
    Gather g;
    g.Pz = fmaf(A.R31, r.rx, fmaf(A.R32, r.ry, fmaf(A.R33, r.rz, z)));
    const CellPos c = cell_pos(a, ur, vr);
    g.tx = c.tx;
    g.ty = c.ty;
    const __amdgpu_buffer_rsrc_t rs = cell_rsrc(a);
    g.ch = load_coefs(rs, c.off, 0);
    g.cfx = load_coefs(rs, c.off, 1);
    g.cfy = load_coefs(rs, c.off, 2);
    g.cc = CM ? load_coefs(rs, c.off, 3) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return g;
}

// Bilinear interpolant of one channel at (tx, ty) from its cell
// coefficients: c0 + tx c_x + ty (c_y + tx c_xy).
__device__ __forceinline__ float bil(const float4 &c, float tx, float ty) {
    return fmaf(tx, c.y, fmaf(ty, fmaf(tx, c.w, c.z), c.x));
}

// Force contributions of one wheel to the sums of the force and moment
// equations of the SRB section. The moments about the CoM are not formed
// per wheel: every wheel has the same lever arm rz = -hR and ry = +-e/2, and
// the rear traction force acts on both rear wheels, so
//   sum Mx = (e/2) (sum of +-Fz) - rz (sum fy),
//   sum My = rz (2 FxR) - sum rx Fz,
//   sum Mz = sum rx fy - (e/2) FxR + (e/2) FxR = sum rx fy,
// and each wheel contributes Fz with the sign of its ry (Sx), rx Fz (Tx) and
// rx fy (Ux).
struct WheelOut {
    float Fy, Fz, Sx, Tx, Ux, c;
};

struct Motion {
    float vx, vy, vz, wx, wy, wz;
    float delta, cosd, FxR;
};

// Terrain-independent part of one wheel: contact-point velocity, slip angle
// and the tire's force-per-load factor, computed while the gathers are in
// flight.
struct WheelPre {
    float vix, viy, viz;
    float tire, q;  // -C alpha mu and 1 / sqrt(mu^2 + (C alpha)^2)
};

__device__ __forceinline__ WheelPre wheel_pre(const RolloutArgs &a, const Motion &m,
                                              const Arm &r) {
    WheelPre p;
    // contact-point velocity v + w x rho (body)
    p.vix = fmaf(m.wy, r.rz, fmaf(-m.wz, r.ry, m.vx));
    p.viy = fmaf(m.wz, r.rx, fmaf(-m.wx, r.rz, m.vy));
    p.viz = fmaf(m.wx, r.ry, fmaf(-m.wy, r.rx, m.vz));
    // slip angle (literal atan of the velocity ratio; 0/0 gives -delta_i),
    // evaluated without a branch so the step stays one basic block. For
    // finite velocities the ratio is NaN only at 0/0 (v_rcp(0) is infinite),
    // whose arctangent is taken as 0; a NaN velocity means a non-finite
    // state, which scores +inf at the end whatever the slip angle.
    const float dl = r.front ? m.delta : 0.0f;
    const float alpha = atan_mm<true>(p.viy * frcp(p.vix)) - dl;
    const float Ca = a.C * alpha;
    p.tire = -Ca * a.mu;
    p.q = frsq(fmaf(Ca, Ca, a.mu2));
    return p;
}

template <bool CM = true>
__device__ __forceinline__ WheelOut wheel(const RolloutArgs &a, const Attitude &A,
                                          const Motion &m, const Arm &r, const Gather &g,
                                          const WheelPre &p) {
    const float vix = p.vix, viy = p.viy, viz = p.viz;
    // bilinear height, slopes and cost rate at the contact point
    const float th = bil(g.ch, g.tx, g.ty);
    const float tfx = bil(g.cfx, g.tx, g.ty);
    const float tfy = bil(g.cfy, g.tx, g.ty);
    const float tc = CM ? bil(g.cc, g.tx, g.ty) : 0.0f;
    // upward terrain normal (-f_x, -f_y, 1) resolved in the body frame
    const float nBx = fmaf(-A.R11, tfx, fmaf(-A.R21, tfy, A.R31));
    const float nBy = fmaf(-A.R12, tfx, fmaf(-A.R22, tfy, A.R32));
    const float nBz = fmaf(-A.R13, tfx, fmaf(-A.R23, tfy, A.R33));
    const float inz = frcp(nBz);
    // extension and its rate along b_z (omega x b_z = (w_y, -w_x, 0))
    const float chi = (g.Pz - th) * inz;
    const float relx = fmaf(-chi, m.wy, vix);
    const float rely = fmaf(chi, m.wx, viy);
    const float chid = fmaf(nBx, relx, fmaf(nBy, rely, nBz * viz)) * inz;
    // spring-damper with liftoff
    const float Fs = r.front ? a.Fsf : a.Fsr;
    const float k = r.front ? a.kf : a.kr;
    const float b = r.front ? a.bf : a.br;
    const float Fk = fmaxf(fmaf(-k, chi, Fs), 0.0f);
    const float Fb = (Fk > 0.0f) ? fmaxf(-b * chid, -Fk) : 0.0f;
    const float Fz = Fk + Fb;
    // sigmoid tire
    const float Fy = (Fz * p.tire) * p.q;
    const float fy = r.front ? Fy * m.cosd : Fy;
    WheelOut o;
    o.Fy = fy;
    o.Fz = Fz;
    o.Sx = r.left ? Fz : -Fz;
    o.Tx = r.rx * Fz;
    o.Ux = r.rx * fy;
    o.c = tc;
    return o;
}

__device__ __forceinline__ WheelOut wadd(const WheelOut &p, const WheelOut &q) {
    return WheelOut{p.Fy + q.Fy, p.Fz + q.Fz, p.Sx + q.Sx, p.Tx + q.Tx, p.Ux + q.Ux, p.c + q.c};
}

// Work a caller issues inside the step right after the terrain gathers (a
// load whose latency should overlap the rest of the step).
struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// Kinematic rows of the right-hand side: world velocity R v and the
// Euler-angle rates of the 3-2-1 sequence. They need only the attitude and
// the state, so the next node's position and angles (x + h of these, the
// update's own fmaf) are known before the wheel forces are.
struct Kin {
    float vWx, vWy, vWz, psid, thd, phd;
};

__device__ __forceinline__ Kin kinematics(const Attitude &A, const float (&st)[13]) {
    const float vx = st[6], vy = st[7], vz = st[8];
    const float wx = st[9], wy = st[10], wz = st[11];
    Kin k;
    k.vWx = fmaf(A.R11, vx, fmaf(A.R12, vy, A.R13 * vz));
    k.vWy = fmaf(A.R21, vx, fmaf(A.R22, vy, A.R23 * vz));
    k.vWz = fmaf(A.R31, vx, fmaf(A.R32, vy, A.R33 * vz));
    const float icth = frcp(A.cth);
    const float t1 = fmaf(A.sph, wy, A.cph * wz);
    k.psid = t1 * icth;
    k.thd = fmaf(A.cph, wy, -(A.sph * wz));
    k.phd = fmaf(k.psid, A.sth, wx);
    return k;
}

// The rest of the right-hand side once the attitude, this lane's terrain
// requests G and the kinematic rows are there: gravity, the rear constraint
// force, the running cost, the wheel forces (the first use of G) and the
// Newton-Euler rows. xd receives the state derivative and the return value
// is the running cost rate L at the state.
template <int LANES, bool CM = true>
__device__ __forceinline__ float srb_forces(const RolloutArgs &a, const Arm (&arms)[4 / LANES],
                                            const float (&st)[13], float dd, float ax,
                                            const Attitude &A, const Gather (&G)[4 / LANES],
                                            const Kin &kn, float (&xd)[13]) {
    constexpr int WPL = 4 / LANES;  // wheels per lane
    const float half_pi = 1.57079632679489662f;
    const float ph = st[5];
    const float vx = st[6], vy = st[7], vz = st[8];
    const float wx = st[9], wy = st[10], wz = st[11];
    const float delta = st[12];
    // gravity (0, 0, -g) in the body frame: -g times the third row of R
    const float gBx = a.g * A.sth;
    const float gBy = -a.g * A.R32;
    const float gBz = -a.g * A.R33;
    Motion m;
    m.vx = vx;
    m.vy = vy;
    m.vz = vz;
    m.wx = wx;
    m.wy = wy;
    m.wz = wz;
    m.delta = delta;
    m.cosd = __cosf(delta);
    m.FxR = a.Mhalf * fmaf(wy, vz, fmaf(-wz, vy, ax - gBx));

    // ESM soft-constraint and control terms of the running cost
    const float ang = fabsf(ph) + a.phibar;
    float U = (a.MgRbar * (1.0f - __sinf(ang))) * A.cth;
    U = (ang > half_pi) ? -U : U;
    const float mm = fmaxf(0.0f, fmaf(-U, a.inv_eps_esm, 1.0f));
    const float L0 = fmaf(a.w_c * dd, dd, a.w_t) + (a.sigma * mm) * mm;

    WheelPre pre[WPL];
#pragma unroll
    for (int q = 0; q < WPL; ++q) pre[q] = wheel_pre(a, m, arms[q]);
    // everything above is independent of the terrain: keep it between the
    // gather issue and the first use of a cell's coefficients
    __builtin_amdgcn_sched_barrier(0);

    // wheel forces: this lane's share, then the group sum in fixed
    // order (w0 + w1) + (w2 + w3)
    WheelOut sum;
    if constexpr (WPL == 4) {
        const WheelOut w0 = wheel<CM>(a, A, m, arms[0], G[0], pre[0]);
        const WheelOut w1 = wheel<CM>(a, A, m, arms[1], G[1], pre[1]);
        const WheelOut w2 = wheel<CM>(a, A, m, arms[2], G[2], pre[2]);
        const WheelOut w3 = wheel<CM>(a, A, m, arms[3], G[3], pre[3]);
        sum = wadd(wadd(w0, w1), wadd(w2, w3));
    } else if constexpr (WPL == 2) {
        sum = wadd(wheel<CM>(a, A, m, arms[0], G[0], pre[0]),
                   wheel<CM>(a, A, m, arms[1], G[1], pre[1]));
    } else {
        sum = wheel<CM>(a, A, m, arms[0], G[0], pre[0]);
    }
    const float Fy = group_sum<LANES>(sum.Fy);
    const float Fz = group_sum<LANES>(sum.Fz);
    const float Sx = group_sum<LANES>(sum.Sx);
    const float Tx = group_sum<LANES>(sum.Tx);
    const float Mz = group_sum<LANES>(sum.Ux);
    const float csum = CM ? group_sum<LANES>(sum.c) : 0.0f;
    // moments about the CoM (see WheelOut): rz = -hR
    const float Mx = fmaf(a.half_e, Sx, a.hR * Fy);
    const float My = fmaf(-a.hR, m.FxR + m.FxR, -Tx);

    // right-hand side rows (Newton-Euler in the body frame)
    const float vyd = fmaf(Fy, a.invM, gBy) + fmaf(wx, vz, -(wz * vx));
    const float vzd = fmaf(Fz, a.invM, gBz) + fmaf(wy, vx, -(wx * vy));
    const float wxd = fmaf(a.dJyz * wy, wz, Mx) * a.invJxx;
    const float wyd = fmaf(-a.dJxz * wx, wz, My) * a.invJyy;
    const float wzd = fmaf(a.dJxy * wx, wy, Mz) * a.invJzz;

    xd[0] = kn.vWx;
    xd[1] = kn.vWy;
    xd[2] = kn.vWz;
    xd[3] = kn.psid;
    xd[4] = kn.thd;
    xd[5] = kn.phd;
    xd[6] = ax;
    xd[7] = vyd;
    xd[8] = vzd;
    xd[9] = wxd;
    xd[10] = wyd;
    xd[11] = wzd;
    xd[12] = dd;
    // without a costmap the cost channel adds nothing (L0 + 0 is L0)
    return CM ? L0 + csum : L0;
}

// Right-hand side of the model for one candidate (this lane's wheels, group
// sums over the candidate's lanes): xd receives the state derivative and the
// return value is the running cost rate L at the state. A hook other than
// NoHook runs after the gathers are issued, behind a scheduling barrier so
// that its loads stay after them.
template <int LANES, bool CM = true, class Hook = NoHook>
__device__ __forceinline__ float srb_rhs(const RolloutArgs &a, const Arm (&arms)[4 / LANES],
                                         const float (&st)[13], float dd, float ax,
                                         float (&xd)[13], const Hook &hook = Hook()) {
    constexpr int WPL = 4 / LANES;  // wheels per lane
    // attitude and this lane's terrain requests first, so the
    // gathers overlap the chassis arithmetic
    const Attitude A = attitude(st[3], st[4], st[5]);
    const GridPos gp = grid_pos(a, st[0], st[1]);
    Gather G[WPL];
#pragma unroll
    for (int q = 0; q < WPL; ++q) G[q] = gather<CM>(a, A, gp, st[2], arms[q]);
    if constexpr (!std::is_same<Hook, NoHook>::value) {
        __builtin_amdgcn_sched_barrier(0);
        hook();
    }
    const Kin kn = kinematics(A, st);
    return srb_forces<LANES, CM>(a, arms, st, dd, ax, A, G, kn, xd);
}

// Steering-angle limit and speed floor, applied to a completed step.
__device__ __forceinline__ void apply_limits(const RolloutArgs &a, float (&st)[13]) {
    st[12] = clampf_nan(st[12], -a.delta_max, a.delta_max);
    st[6] = (st[6] < a.vx_min) ? a.vx_min : st[6];
}

// One forward-Euler step (the paper's integrator): the running cost at the
// node is added to J (left Riemann sum) and the state advanced in place.
template <int LANES, bool CM = true, class Hook = NoHook>
__device__ __forceinline__ void euler_step(const RolloutArgs &a, const Arm (&arms)[4 / LANES],
                                           float (&st)[13], float &J, float dd, float ax,
                                           const Hook &hook = Hook()) {
    float xd[13];
    const float L = srb_rhs<LANES, CM>(a, arms, st, dd, ax, xd, hook);
    J = fmaf(a.h, L, J);
#pragma unroll
    for (int q = 0; q < 13; ++q) st[q] = fmaf(a.h, xd[q], st[q]);
    apply_limits(a, st);
}

// The terrain requests of one Euler node: its attitude and the cell
// coefficients of this lane's wheels, whose loads stay in flight until the
// step at that node uses them.
template <int LANES, bool CM>
struct NodeRequest {
    Attitude A;
    Gather G[4 / LANES];
};

template <int LANES, bool CM>
__device__ __forceinline__ void request_node(const RolloutArgs &a, const Arm (&arms)[4 / LANES],
                                             float x, float y, float z, float psi, float th,
                                             float ph, NodeRequest<LANES, CM> &r) {
    r.A = attitude(psi, th, ph);
    const GridPos gp = grid_pos(a, x, y);
#pragma unroll
    for (int q = 0; q < 4 / LANES; ++q) r.G[q] = gather<CM>(a, r.A, gp, z, arms[q]);
}

// The same forward-Euler step with its node's terrain requested one step
// earlier (cur) and the next node's requested here (nxt): the update moves
// the position and angles by h times the kinematic rows, which the step has
// before its wheel forces, so the next node's cells are loaded a whole step
// ahead of their use. The arithmetic is that of euler_step, so the results
// are the same bits. The hook (the next control pair) is issued before the
// cell loads: loads complete in issue order, so waiting for the controls at
// the next interval never waits for the cells.
template <int LANES, bool CM = true, class Hook = NoHook>
__device__ __forceinline__ void euler_step_ahead(const RolloutArgs &a,
                                                 const Arm (&arms)[4 / LANES], float (&st)[13],
                                                 float &J, float dd, float ax,
                                                 const NodeRequest<LANES, CM> &cur,
                                                 NodeRequest<LANES, CM> &nxt,
                                                 const Hook &hook = Hook()) {
    const Kin kn = kinematics(cur.A, st);
    if constexpr (!std::is_same<Hook, NoHook>::value) {
        hook();
        __builtin_amdgcn_sched_barrier(0);
    }
    request_node<LANES, CM>(a, arms, fmaf(a.h, kn.vWx, st[0]), fmaf(a.h, kn.vWy, st[1]),
                            fmaf(a.h, kn.vWz, st[2]), fmaf(a.h, kn.psid, st[3]),
                            fmaf(a.h, kn.thd, st[4]), fmaf(a.h, kn.phd, st[5]), nxt);
    float xd[13];
    const float L = srb_forces<LANES, CM>(a, arms, st, dd, ax, cur.A, cur.G, kn, xd);
    J = fmaf(a.h, L, J);
#pragma unroll
    for (int q = 0; q < 13; ++q) st[q] = fmaf(a.h, xd[q], st[q]);
    apply_limits(a, st);
}

// One classical fourth-order Runge-Kutta step on (state, J) with J' = L and
// the control held (the alternative integrator the paper compared Euler
// with); the limits apply to the completed step.
template <int LANES, bool CM = true>
__device__ __forceinline__ void rk4_step(const RolloutArgs &a, const Arm (&arms)[4 / LANES],
                                         float (&st)[13], float &J, float dd, float ax) {
    float k[13], acc[13], stage[13];
    float L = srb_rhs<LANES, CM>(a, arms, st, dd, ax, k);
    float Lacc = L;
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        acc[q] = k[q];
        stage[q] = fmaf(a.h_half, k[q], st[q]);
    }
    L = srb_rhs<LANES, CM>(a, arms, stage, dd, ax, k);
    Lacc = fmaf(2.0f, L, Lacc);
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        acc[q] = fmaf(2.0f, k[q], acc[q]);
        stage[q] = fmaf(a.h_half, k[q], st[q]);
    }
    L = srb_rhs<LANES, CM>(a, arms, stage, dd, ax, k);
    Lacc = fmaf(2.0f, L, Lacc);
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        acc[q] = fmaf(2.0f, k[q], acc[q]);
        stage[q] = fmaf(a.h, k[q], st[q]);
    }
    L = srb_rhs<LANES, CM>(a, arms, stage, dd, ax, k);
    Lacc = Lacc + L;
    J = fmaf(a.h_sixth, Lacc, J);
#pragma unroll
    for (int q = 0; q < 13; ++q) st[q] = fmaf(a.h_sixth, acc[q] + k[q], st[q]);
    apply_limits(a, st);
}

}  // namespace plan
