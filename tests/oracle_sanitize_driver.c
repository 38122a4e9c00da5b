/* Drives every entry point of the oracle on small, ragged and degenerate
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py compiles and runs it on the host). Exits 0
 * when every call returns its documented status; the sanitizers abort the
 * process on the first invalid access or undefined operation. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static unsigned long long rng_state = 0x9e3779b97f4a7c15ull;

/* splitmix64 in [0, 1) */
static double urand(void)
{
    unsigned long long z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static int run_grid(int W, int H, int with_costmap, int K, int N, int substeps, int method)
{
    const oracle_vehicle v = {900.0, 260.9, 642.8, 753.0, 1.1537, 0.8463, 1.5, 0.6,
                              4.2e4, 5.8e4, 3.1e3, 4.3e3, 6.1, 0.6, 0.639, 1.0, 9.81};
    const oracle_cost c = {5.0, 8.0, 15.0, 3.0, 1.0, 2.5, 1.0e6, 0.0, 0.25, 0.0};
    const oracle_integ in = {0.02, substeps, 3.0, 1.0, method};
    oracle_ctx *o = oracle_create(&v, &c, &in);
    CHECK(o != NULL);
    float *h = malloc(sizeof(float) * W * H);
    float *cm = malloc(sizeof(float) * W * H);
    for (int q = 0; q < W * H; ++q) {
        h[q] = (float)(0.3 * urand());
        cm[q] = (float)(5.0 * urand());
    }
    CHECK(oracle_set_terrain(o, h, W, H, -0.5, -0.5, 0.25, with_costmap ? cm : NULL) == 0);
    double tout[4];
    /* inside, on the far edge, far outside, and a NaN query */
    CHECK(oracle_sample_terrain(o, 0.1, 0.1, tout) == 0);
    CHECK(oracle_sample_terrain(o, -0.5 + 0.25 * (W - 1), -0.5 + 0.25 * (H - 1), tout) == 0);
    CHECK(oracle_sample_terrain(o, 1e3, -1e3, tout) == 0);
    oracle_sample_terrain(o, NAN, 0.0, tout);

    float s0[13] = {0.2f, 0.1f, 1.0f, 0.3f, 0.0f, 0.0f, 8.0f, 0, 0, 0, 0, 0, 0};
    float *u = malloc(sizeof(float) * 2 * N * K);
    for (int q = 0; q < 2 * N * K; ++q) u[q] = (float)(4.0 * urand() - 2.0); /* beyond the limits */
    if (K > 2) u[1] = NAN; /* a non-finite control on candidate 1 */
    double *J = malloc(sizeof(double) * K), *fs = malloc(sizeof(double) * 13 * K);
    int *ex = malloc(sizeof(int) * K);
    CHECK(oracle_rollout(o, s0, u, K, N, J, fs, ex) == 0);

    float *si = malloc(sizeof(float) * 13 * K), *ci = malloc(sizeof(float) * K);
    for (int k = 0; k < K; ++k) {
        for (int q = 0; q < 13; ++q) si[q * K + k] = s0[q];
        ci[k] = 0.0f;
    }
    double *so = malloc(sizeof(double) * 13 * K), *co = malloc(sizeof(double) * K);
    double *td = malloc(sizeof(double) * K), *sl = malloc(sizeof(double) * K);
    double *tl = malloc(sizeof(double) * K);
    CHECK(oracle_rollout_span(o, si, ci, u, K, N, 0, N, 1, so, co, td, sl, tl) == 0);
    CHECK(oracle_rollout_span(o, si, ci, u, K, N, N, N, 0, so, co, NULL, NULL, NULL) == 0);
    oracle_set_round32(o, 1);
    CHECK(oracle_rollout_span(o, si, ci, u, K, N, 0, N, 1, so, co, NULL, NULL, NULL) == 0);
    oracle_set_round32(o, 0);

    double sd[13], *ud = malloc(sizeof(double) * 2 * N * K);
    for (int q = 0; q < 13; ++q) sd[q] = s0[q];
    for (int q = 0; q < 2 * N * K; ++q) ud[q] = u[q];
    CHECK(oracle_rollout_d(o, sd, ud, K, N, J, fs) == 0);

    float *Jf = malloc(sizeof(float) * K);
    for (int k = 0; k < K; ++k) Jf[k] = (float)J[k];
    if (K > 3) Jf[2] = INFINITY;
    int best = -2;
    double bc = 0.0, *plan = malloc(sizeof(double) * 2 * N);
    CHECK(oracle_select(o, 0, 0.0, u, Jf, K, N, &best, &bc, plan) == 0);
    CHECK(oracle_select(o, 1, 50.0, u, Jf, K, N, &best, &bc, plan) == 0);
    for (int k = 0; k < K; ++k) Jf[k] = INFINITY; /* no finite candidate */
    CHECK(oracle_select(o, 0, 0.0, u, Jf, K, N, &best, &bc, plan) == 0);
    CHECK(best == -1);

    double xi[13], xd[13];
    oracle_diag dg;
    for (int q = 0; q < 13; ++q) xi[q] = s0[q];
    CHECK(oracle_rhs(o, xi, 0.1, 0.2, xd, &dg) == 0);
    (void)oracle_esm(o, 0.2, -0.1);
    (void)oracle_soft(1e6, 0.1, -0.3);

    float e0[7] = {0.2f, 0.1f, 0.3f, 0.0f, 0.0f, 0.0f, 8.0f};
    double *fe = malloc(sizeof(double) * 7 * K);
    CHECK(oracle_est_rollout(o, e0, u, K, N, J, fe, ex) == 0);
    double xe[7] = {0.2, 0.1, 0.3, 0.0, 0.0, 0.0, 8.0}, xde[7];
    oracle_est_diag de;
    CHECK(oracle_est_rhs(o, xe, 0.1, 0.2, xde, &de) == 0);

    free(h); free(cm); free(u); free(J); free(fs); free(ex); free(si); free(ci); free(so);
    free(co); free(td); free(sl); free(tl); free(ud); free(Jf); free(plan); free(fe);
    oracle_destroy(o);
    return 0;
}

int main(void)
{
    /* grids of one cell, one row or column of cells, and ragged sizes;
     * Euler and RK4; one and several substeps; K = 1 and N = 1 */
    static const int cases[][7] = {
        {2, 2, 0, 1, 1, 1, 0},   {2, 9, 1, 5, 3, 2, 0},  {13, 2, 0, 7, 4, 1, 1},
        {23, 17, 1, 37, 9, 3, 0}, {31, 5, 1, 16, 6, 1, 1},
    };
    for (size_t i = 0; i < sizeof cases / sizeof cases[0]; ++i) {
        const int *p = cases[i];
        if (run_grid(p[0], p[1], p[2], p[3], p[4], p[5], p[6])) {
            fprintf(stderr, "case %zu failed\n", i);
            return 1;
        }
    }

    /* terrain smoothing: radius beyond the grid, a single row */
    float hs[7 * 5];
    for (int q = 0; q < 35; ++q) hs[q] = (float)urand();
    double out[35];
    CHECK(oracle_smooth_terrain(hs, 7, 5, 0.1, 0.3, out) == 0);
    CHECK(oracle_smooth_terrain(hs, 7, 5, 0.1, 4.2, out) == 0);
    CHECK(oracle_smooth_terrain(hs, 35, 1, 0.1, 0.3, out) == 0);

    /* costmap: an obstacle triangle and a path-boundary square */
    const double verts[] = {0.0, 0.0, 1.0, 0.0, 0.5, 1.0, -1.0, -1.0, 2.0, -1.0, 2.0, 2.0, -1.0, 2.0};
    const int offsets[] = {0, 3, 7}, kinds[] = {0, 1};
    double cmo[9 * 6];
    CHECK(oracle_costmap_polygons(verts, offsets, kinds, 2, 9, 6, -1.0, -1.0, 0.4, 1e6, 0.25,
                                  cmo) == 0);

    /* sampler: both laws, with and without a nominal; N not a multiple of 4 */
    const double scale[2] = {1.0, 0.5};
    float nominal[2 * 7];
    for (int q = 0; q < 14; ++q) nominal[q] = (float)urand();
    double sc[2 * 7 * 5];
    CHECK(oracle_sample_controls(0, 6000, 0, scale, 0, NULL, 5, 7, sc) == 0);
    CHECK(oracle_sample_controls(1, 6000, 3, scale, 1, nominal, 5, 7, sc) == 0);
    printf("oracle sanitized driver: all entry points ran\n");
    return 0;
}
