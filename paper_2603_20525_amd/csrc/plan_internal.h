// Internal declarations shared by the libplan sources (kernels and host ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plan {

// Everything one rollout needs, passed by value as the kernel argument
// (a few hundred bytes, well inside the kernarg limit). All derived constants
// are computed once on the host in double precision and rounded to float.
struct RolloutArgs {
    // vehicle
    float invM;
    float invJxx, invJyy, invJzz;
    float dJyz, dJxz, dJxy;        // Jyy-Jzz, Jxx-Jzz, Jxx-Jyy
    float Lf, Lr, half_e, hR;
    float kf, kr, bf, br;
    float Fsf, Fsr;                // nominal tire loads (g/2) K_zz,f / K_zz,r
    float Mhalf;                   // M/2 (rear longitudinal constraint force)
    float C, mu, mu2;
    float delta_max, drate_max, g;
    float MgRbar, phibar;          // ESM: M g R_bar, phi_bar
    // cost
    float w_t, w_c, w_g;
    float goal_x, goal_y, goal_r2;
    float sigma, inv_eps_esm;
    // integration
    float h;                       // Euler step dt / substeps
    int S;                         // substeps per control
    float accel_max, vx_min;
    // terrain: float4 texels (h, f_x, f_y, cost) on a W x H grid
    const float4 *tex;
    int W, H;
    float x0, y0, inv_res;
    float umax, vmax;              // W-1, H-1 as floats (clamp-to-edge)
    // problem
    float s0[13];
    const float *controls;         // [N][2][K]
    int K, N;
    int n0, n1;                    // control intervals simulated by this launch
    int finalize;                  // add the terminal cost, apply the non-finite rule
    float *cost;                   // [K]: written (full) or read-modify-written (chunk)
    float *final_state;            // full: [13][K] or nullptr
    float *state;                  // chunk: [13][K], read and written
};

struct SelectOut {
    int best_k;
    float best_cost;
    uint32_t pad[2];
};

// chunk = false: candidates start from s0 with zero cost. chunk = true:
// they continue from a.state / a.cost. Both run the same step code.
hipError_t launch_rollout(const RolloutArgs &a, int lanes, int block, bool chunk, hipStream_t s);

hipError_t launch_init_state(const float *s0, float *state, float *cost, int K, hipStream_t s);

hipError_t launch_pack_terrain(const float *h, const float *c, int W, int H, float inv_res,
                               float4 *tex, int *bad, hipStream_t s);

// Selection workspace sizes for a given maximum K / N.
int select_blocks(int K);
int softmin_chunks(int K);
int softmin_row_groups(int N);

hipError_t launch_select(int mode, float lambda, const float *controls, const float *cost,
                         int K, int N, float drate_max, float *plan_out,
                         unsigned long long *part_keys, unsigned int *counters,
                         float *wpart, SelectOut *out, hipStream_t s);

}  // namespace plan
