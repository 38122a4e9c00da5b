// Terrain preparation kernels, off the per-plan path (run once per map):
//   * level-of-detail smoothing (section "Terrain Smoothing"): the heightmap
//     convolved with a Gaussian of standard deviation sigma, truncated at
//     r = ceil(3 sigma / res) nodes, clamp-to-edge; the kernel is separable,
//     so it runs as a row pass and a column pass, each staging its tile and
//     halo in LDS (HBM-bound: one read and one write of the grid per pass);
//   * the distance-constraint costmap (sections "OCP Formulation" and
//     "Real-Time Implementation": sdist pre-computed and summed over all
//     features, interpolated at run time): at each node the sum over
//     perimeters of sigma * max(0, 1 - sdist / eps)^2, sdist negative inside
//     an obstacle and outside a path boundary, inside by the even-odd rule.
#include "plan_internal.h"

namespace plan {
namespace {

constexpr int ROW_OUT = 4;                      // outputs per thread, row pass
constexpr int ROW_TILE = 256 * ROW_OUT;         // outputs per workgroup, row pass
constexpr int COL_W = 32;                       // columns per workgroup, column pass
constexpr int COL_RUN = 8;                      // consecutive rows per thread, column pass
constexpr int COL_T = (256 / COL_W) * COL_RUN;  // rows per workgroup, column pass (64)

// Row pass: tmp[j][i] = sum_k w[k] h[j][clamp(i + k - r)], k = 0 .. 2r in
// order. Each thread produces ROW_OUT neighbouring outputs from one sliding
// window of the LDS row tile.
__global__ __launch_bounds__(256) void smooth_rows(const float *__restrict__ h, int W, int H,
                                                   const SmoothTaps taps,
                                                   float *__restrict__ tmp) {
    __shared__ float tile[ROW_TILE + 2 * MAX_SMOOTH_RADIUS];
    const int r = taps.r;
    const int j = blockIdx.y;
    if (j >= H) return;  // whole workgroup (grid rows = H)
    const int i0 = blockIdx.x * ROW_TILE;
    const float *row = h + (size_t)j * W;
    for (int q = threadIdx.x; q < ROW_TILE + 2 * r; q += 256) {
        const int i = min(max(i0 + q - r, 0), W - 1);
        tile[q] = row[i];
    }
    __syncthreads();
    const int base = threadIdx.x * ROW_OUT;  // first output of this thread in the tile
    float acc[ROW_OUT];
#pragma unroll
    for (int o = 0; o < ROW_OUT; ++o) acc[o] = 0.0f;
    float win[ROW_OUT];
#pragma unroll
    for (int o = 0; o < ROW_OUT - 1; ++o) win[o + 1] = tile[base + o];
    for (int k = 0; k <= 2 * r; ++k) {
        // window = tile[base + k .. base + k + ROW_OUT - 1]
#pragma unroll
        for (int o = 0; o < ROW_OUT - 1; ++o) win[o] = win[o + 1];
        win[ROW_OUT - 1] = tile[base + k + ROW_OUT - 1];
        const float w = taps.w[k];
#pragma unroll
        for (int o = 0; o < ROW_OUT; ++o) acc[o] = fmaf(w, win[o], acc[o]);
    }
    float *dst = tmp + (size_t)j * W + i0 + base;
#pragma unroll
    for (int o = 0; o < ROW_OUT; ++o)
        if (i0 + base + o < W) dst[o] = acc[o];
}

// Column pass: out[j][i] = sum_k w[k] tmp[clamp(j + k - r)][i]; a tile of
// COL_T rows x COL_W columns plus the vertical halo is staged in LDS (at most
// 318 x 32 floats, 40.7 KB). Thread t owns column t % COL_W and the COL_RUN
// consecutive rows starting at (t / COL_W) * COL_RUN, swept with a sliding
// window of the column.
__global__ __launch_bounds__(256) void smooth_cols(const float *__restrict__ tmp, int W, int H,
                                                   const SmoothTaps taps,
                                                   float *__restrict__ out) {
    __shared__ float tile[(COL_T + 2 * MAX_SMOOTH_RADIUS) * COL_W];
    const int r = taps.r;
    const int i0 = blockIdx.x * COL_W, j0 = blockIdx.y * COL_T;
    const int rows = COL_T + 2 * r;
    const int c = threadIdx.x & (COL_W - 1);
    const int i = min(i0 + c, W - 1);
    for (int q = threadIdx.x / COL_W; q < rows; q += 256 / COL_W) {
        const int j = min(max(j0 + q - r, 0), H - 1);
        tile[q * COL_W + c] = tmp[(size_t)j * W + i];
    }
    __syncthreads();
    if (i0 + c >= W) return;
    const int t0 = (threadIdx.x / COL_W) * COL_RUN;  // first output row in the tile
    float acc[COL_RUN];
#pragma unroll
    for (int o = 0; o < COL_RUN; ++o) acc[o] = 0.0f;
    float win[COL_RUN];
#pragma unroll
    for (int o = 0; o < COL_RUN - 1; ++o) win[o + 1] = tile[(t0 + o) * COL_W + c];
    for (int k = 0; k <= 2 * r; ++k) {
#pragma unroll
        for (int o = 0; o < COL_RUN - 1; ++o) win[o] = win[o + 1];
        win[COL_RUN - 1] = tile[(t0 + k + COL_RUN - 1) * COL_W + c];
        const float w = taps.w[k];
#pragma unroll
        for (int o = 0; o < COL_RUN; ++o) acc[o] = fmaf(w, win[o], acc[o]);
    }
#pragma unroll
    for (int o = 0; o < COL_RUN; ++o) {
        const int j = j0 + t0 + o;
        if (j < H) out[(size_t)j * W + i0 + c] = acc[o];
    }
}

// Distance from (px, py) to the segment a-b (FP32).
__device__ __forceinline__ float seg_dist(float px, float py, float ax, float ay, float bx,
                                          float by) {
    const float ex = bx - ax, ey = by - ay;
    const float len2 = fmaf(ex, ex, ey * ey);
    float t = 0.0f;
    if (len2 > 0.0f) t = fminf(fmaxf(fmaf(px - ax, ex, (py - ay) * ey) / len2, 0.0f), 1.0f);
    const float qx = fmaf(t, ex, ax) - px, qy = fmaf(t, ey, ay) - py;
    return sqrtf(fmaf(qx, qx, qy * qy));
}

// One thread per node; the vertices are read with wave-uniform addresses.
__global__ __launch_bounds__(256) void costmap_polygons(const float2 *__restrict__ verts,
                                                        const PolygonSet ps, int W, int H,
                                                        float x0, float y0, float res,
                                                        float sigma, float inv_eps,
                                                        int accumulate,
                                                        float *__restrict__ cm) {
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= W || j >= H) return;
    const float px = fmaf((float)i, res, x0), py = fmaf((float)j, res, y0);
    float c = 0.0f;
    for (int p = 0; p < ps.count; ++p) {
        const int a = ps.offsets[p], m = ps.offsets[p + 1] - a;
        float dmin = __builtin_inff();
        bool inside = false;
        float2 v0 = verts[a + m - 1];
        for (int e = 0; e < m; ++e) {
            const float2 v1 = verts[a + e];
            dmin = fminf(dmin, seg_dist(px, py, v0.x, v0.y, v1.x, v1.y));
            if ((v0.y > py) != (v1.y > py)) {
                const float xc = v0.x + (py - v0.y) * (v1.x - v0.x) / (v1.y - v0.y);
                if (px < xc) inside = !inside;
            }
            v0 = v1;
        }
        // obstacle: negative inside; path boundary: negative outside
        const float sd = (inside == (ps.kinds[p] == 0)) ? -dmin : dmin;
        const float mm = fmaxf(0.0f, fmaf(-sd, inv_eps, 1.0f));
        c = fmaf(sigma * mm, mm, c);
    }
    const size_t q = (size_t)j * W + i;
    cm[q] = accumulate ? cm[q] + c : c;
}

}  // namespace

hipError_t launch_smooth(const float *h, int W, int H, const SmoothTaps &taps, float *tmp,
                         float *out, hipStream_t s) {
    hipLaunchKernelGGL(smooth_rows, dim3((W + ROW_TILE - 1) / ROW_TILE, H), dim3(256), 0, s, h, W,
                       H, taps, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(smooth_cols, dim3((W + COL_W - 1) / COL_W, (H + COL_T - 1) / COL_T),
                       dim3(256), 0, s, tmp, W, H, taps, out);
    return hipGetLastError();
}

hipError_t launch_costmap_polygons(const float *verts, const PolygonSet &ps, int W, int H,
                                   float x0, float y0, float res, float sigma, float eps,
                                   int accumulate, float *cm, hipStream_t s) {
    dim3 grid((W + 15) / 16, (H + 15) / 16);
    hipLaunchKernelGGL(costmap_polygons, grid, dim3(256), 0, s, (const float2 *)verts, ps, W, H,
                       x0, y0, res, sigma, 1.0f / eps, accumulate, cm);
    return hipGetLastError();
}

}  // namespace plan
