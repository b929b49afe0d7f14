/*
 * Host driver that runs every entry point of the FP64 oracle on small seeded
 * inputs, built together with the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py (gcc, host
 * code only).  Any out-of-bounds access, use of freed memory, leak or
 * undefined operation in the oracle makes the sanitizer report and the
 * process fail; the driver also checks a few results and returns non-zero
 * when they are wrong.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpm_oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

/* splitmix64, mapped to [0, 1) */
static double uniform(void)
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) / 9007199254740992.0;
}

#define CHECK(cond, msg)                                           \
    do {                                                           \
        if (!(cond)) {                                             \
            fprintf(stderr, "driver check failed: %s\n", msg);     \
            return 1;                                              \
        }                                                          \
    } while (0)

int main(void)
{
    enum { N = 240, S = 4, RES = 12 };
    const int n = 16;
    orc_params P;
    memset(&P, 0, sizeof P);
    P.n = n; P.bound = 3; P.n_tools = 3; P.dt = 1e-4;
    P.g[1] = -9.8;
    P.E = 1e4; P.nu = 0.35; P.rho = 1e3; P.V0 = 0.3 * 0.1 * 0.3 / N;

    /* particles in a box, moving, slightly deformed; one leaves the grid, one is inverted */
    double *x = malloc(sizeof(double) * 3 * N), *v = malloc(sizeof(double) * 3 * N);
    double *C = malloc(sizeof(double) * 9 * N), *F = malloc(sizeof(double) * 9 * N);
    for (int p = 0; p < N; ++p) {
        x[3 * p + 0] = 0.35 + 0.3 * uniform();
        x[3 * p + 1] = 0.2 + 0.1 * uniform();
        x[3 * p + 2] = 0.35 + 0.3 * uniform();
        for (int a = 0; a < 3; ++a) v[3 * p + a] = 0.2 * (uniform() - 0.5);
        for (int k = 0; k < 9; ++k) {
            C[9 * p + k] = 0.5 * (uniform() - 0.5);
            F[9 * p + k] = (k % 4 == 0 ? 1.0 : 0.0) + 0.01 * (uniform() - 0.5);
        }
    }
    x[0] = 0.02;                                   /* stencil outside the grid */
    F[9 * 1 + 8] = -0.5;                           /* det F < 0 */

    /* three tools: slip capsule, sticky box, trilinear sampled SDF (a ball) */
    float *sdf = malloc(sizeof(float) * RES * RES * RES);
    const double h = 0.01;
    for (int i = 0; i < RES; ++i)
        for (int j = 0; j < RES; ++j)
            for (int k = 0; k < RES; ++k) {
                double px = (i - RES / 2) * h, py = (j - RES / 2) * h, pz = (k - RES / 2) * h;
                sdf[(i * RES + j) * RES + k] = (float)(sqrt(px * px + py * py + pz * pz) - 0.03);
            }
    orc_tool tools[3];
    memset(tools, 0, sizeof tools);
    for (int t = 0; t < 3; ++t) {
        tools[t].R[0] = tools[t].R[4] = tools[t].R[8] = 1.0;
        tools[t].theta = 1e-3;
        tools[t].friction = 0.3;
    }
    tools[0].shape = ORC_TOOL_CAPSULE; tools[0].contact = ORC_CONTACT_SLIP;
    tools[0].radius = 0.02; tools[0].half_len = 0.1;
    tools[1].shape = ORC_TOOL_BOX; tools[1].contact = ORC_CONTACT_STICKY;
    tools[1].half[0] = 0.04; tools[1].half[1] = 0.02; tools[1].half[2] = 0.01; tools[1].radius = 0.005;
    tools[2].shape = ORC_TOOL_SDF; tools[2].contact = ORC_CONTACT_SLIP; tools[2].sdf = sdf;
    tools[2].sdf_res = RES; tools[2].sdf_h = h; tools[2].sdf_interp = ORC_SDF_TRILINEAR;
    for (int a = 0; a < 3; ++a) tools[2].sdf_lo[a] = -(RES / 2) * h;
    double T0[9] = {0.5, 0.31, 0.5, 0.4, 0.3, 0.45, 0.6, 0.3, 0.55};
    double traj[3 * S * 3];
    for (int t = 0; t < 3; ++t)
        for (int s = 0; s < S; ++s) {
            traj[(t * S + s) * 3 + 0] = 0.05;
            traj[(t * S + s) * 3 + 1] = -0.3;
            traj[(t * S + s) * 3 + 2] = 0.02 * t;
        }

    /* serial run and threaded run must agree bit for bit */
    double *x2 = malloc(sizeof(double) * 3 * N), *v2 = malloc(sizeof(double) * 3 * N);
    double *C2 = malloc(sizeof(double) * 9 * N), *F2 = malloc(sizeof(double) * 9 * N);
    memcpy(x2, x, sizeof(double) * 3 * N); memcpy(v2, v, sizeof(double) * 3 * N);
    memcpy(C2, C, sizeof(double) * 9 * N); memcpy(F2, F, sizeof(double) * 9 * N);
    double T1[9], T2[9];
    memcpy(T1, T0, sizeof T1); memcpy(T2, T0, sizeof T2);
    uint32_t f1 = orc_run(&P, tools, traj, S, 0, S, T1, N, x, v, C, F);
    uint32_t f2 = orc_run_threads(&P, tools, traj, S, 0, S, T2, N, x2, v2, C2, F2, 3);
    CHECK(f1 == f2, "flags of serial and threaded runs");
    CHECK(f1 & ORC_FLAG_OUT_OF_DOMAIN, "out-of-domain flag");
    CHECK(f1 & ORC_FLAG_INVERTED, "inverted flag");
    CHECK(memcmp(x, x2, sizeof(double) * 3 * N) == 0 && memcmp(F, F2, sizeof(double) * 9 * N) == 0,
          "serial and threaded states");

    /* stages one by one, with node records */
    const size_t nn = (size_t)n * n * n;
    double *gm = malloc(sizeof(double) * nn), *gmv = malloc(sizeof(double) * 3 * nn);
    double *gv = malloc(sizeof(double) * 3 * nn);
    orc_node_rec *rec = malloc(sizeof(orc_node_rec) * nn);
    orc_p2g(&P, N, x, v, C, F, gm, gmv);
    double msum = 0.0;
    for (size_t i = 0; i < nn; ++i) msum += gm[i];
    CHECK(fabs(msum - (N - 1) * P.rho * P.V0) < 1e-12, "P2G mass conservation");
    orc_grid_update(&P, tools, T1, traj, gm, gmv, gv, rec);
    double *gvbar = malloc(sizeof(double) * 3 * nn), *gmbar = malloc(sizeof(double) * nn);
    double *gmvbar = malloc(sizeof(double) * 3 * nn);
    double *xb = calloc(3 * N, sizeof(double)), *vb = calloc(3 * N, sizeof(double));
    double *Cb = calloc(9 * N, sizeof(double)), *Fb = calloc(9 * N, sizeof(double));
    for (int p = 0; p < N; ++p) xb[3 * p + 1] = 1.0;
    double ubar[9] = {0}, Tbar[9] = {0}, mub = 0.0, lamb = 0.0;
    orc_g2p_adjoint(&P, N, x, F, gv, xb, vb, Cb, Fb, gvbar);
    orc_grid_adjoint(&P, tools, traj, gm, gmv, rec, gvbar, gmbar, gmvbar, ubar, Tbar);
    orc_p2g_adjoint(&P, N, x, v, C, F, gmbar, gmvbar, xb, vb, Cb, Fb, &mub, &lamb);
    orc_g2p(&P, N, x, v, C, F, gv);

    /* full adjoint with every output */
    double gE = 0.0, gnu = 0.0, gu[3 * S * 3], gT0[9];
    double *xb0 = calloc(3 * N, sizeof(double)), *vb0 = calloc(3 * N, sizeof(double));
    double *Cb0 = calloc(9 * N, sizeof(double)), *Fb0 = calloc(9 * N, sizeof(double));
    for (int p = 0; p < N; ++p) xb0[3 * p] = 1.0 / N;
    orc_adjoint(&P, tools, traj, S, S, T0, N, x2, v2, C2, F2, xb0, vb0, Cb0, Fb0, &gE, &gnu, gu, gT0);
    CHECK(isfinite(gE) && isfinite(gnu), "finite parameter gradients");

    /* point queries */
    double l[3], Jl[9], q[3], xr[3] = {0.01, 0.005, -0.002};
    int inside = 0, base[3];
    (void)orc_capsule_sdf(xr, 0.02, 0.1, q, &inside);
    (void)orc_box_sdf(xr, tools[1].half, 0.005, l, Jl);
    (void)orc_sampled_sdf(&tools[2], xr, l, Jl);
    double fx[3], w[3][3], dw[3][3], tau[9];
    orc_weights(x + 3 * 5, n, base, fx, w, dw);
    (void)orc_kirchhoff(F + 9 * 5, 1e3, 2e3, tau);

    /* marching cubes: every case, then the surface of the mass volume */
    int32_t tri[12][3];
    for (int mask = 0; mask < 256; ++mask) CHECK(orc_mc_case(mask, tri) >= 0, "case closes");
    int32_t *cells = malloc(sizeof(int32_t) * (size_t)(n - 1) * (n - 1) * (n - 1));
    double iso = 0.25 * P.rho * (1.0 / ((double)n * n * n));
    int64_t total = orc_surface(n, 1.0 / n, gm, iso, cells, NULL, NULL, 0);
    CHECK(total > 0, "surface has triangles");
    int32_t *edges = malloc(sizeof(int32_t) * 3 * (size_t)total);
    double *tris = malloc(sizeof(double) * 9 * (size_t)total);
    CHECK(orc_surface(n, 1.0 / n, gm, iso, NULL, edges, tris, total) == total, "surface count stable");

    free(x); free(v); free(C); free(F); free(x2); free(v2); free(C2); free(F2); free(sdf);
    free(gm); free(gmv); free(gv); free(rec); free(gvbar); free(gmbar); free(gmvbar);
    free(xb); free(vb); free(Cb); free(Fb); free(xb0); free(vb0); free(Cb0); free(Fb0);
    free(cells); free(edges); free(tris);
    printf("sanitized oracle driver: ok (%lld triangles, dL/dE %.3e)\n", (long long)total, gE);
    return 0;
}
