/*
 * A client of the C ABI alone: no Python, no torch, plain C and the HIP
 * runtime for device memory.  A block of 8,000 particles at rest in the air
 * of a 64^3 grid falls freely for 40 substeps (no tool, no wall in reach);
 * with F = I the stress vanishes and the transfers reproduce the uniform
 * velocity exactly, so every particle must follow the substep's symplectic
 * Euler in closed form, x = x0 + dt^2 g S (S + 1) / 2, v = S dt g, F = I.
 * Then the same block takes 40 more substeps pressed by a capsule tool, and
 * the status must stay clear.  Prints one line per check; exit code 0 when
 * all hold.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpm.h"

#define CHECK(x)                                                                     \
    do {                                                                             \
        int rc_ = (int)(x);                                                          \
        if (rc_ != 0) {                                                              \
            fprintf(stderr, "%s failed: %d (%s)\n", #x, rc_, mpm_last_error(NULL)); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

int main(void)
{
    const int side = 20, N = side * side * side, n = 64, S = 40;
    const float dt = 1e-4f, g[3] = {0.0f, -9.8f, 0.0f};
    float *x0 = calloc(3 * (size_t)N, sizeof(float)), *zero = calloc(9 * (size_t)N, sizeof(float));
    float *F0 = calloc(9 * (size_t)N, sizeof(float)), *xs = calloc(3 * (size_t)N, sizeof(float));
    float *vs = calloc(3 * (size_t)N, sizeof(float)), *Fs = calloc(9 * (size_t)N, sizeof(float));
    if (!x0 || !zero || !F0 || !xs || !vs || !Fs) return 1;
    /* lattice at half the grid spacing, inside [0.40, 0.56)^3 */
    for (int i = 0; i < side; ++i)
        for (int j = 0; j < side; ++j)
            for (int k = 0; k < side; ++k) {
                int p = (i * side + j) * side + k;
                x0[p] = 0.40f + (i + 0.5f) * 0.5f / n;
                x0[N + p] = 0.40f + (j + 0.5f) * 0.5f / n;
                x0[2 * N + p] = 0.40f + (k + 0.5f) * 0.5f / n;
                F0[p] = F0[4 * (size_t)N + p] = F0[8 * (size_t)N + p] = 1.0f;
            }
    const float side_len = side * 0.5f / n;
    const float material[4] = {1e4f, 0.3f, 1e3f, side_len * side_len * side_len / N};

    float *dx0, *dv0, *dC0, *dF0, *dmat, *du;
    CHECK(hipMalloc((void **)&dx0, 3 * (size_t)N * sizeof(float)));
    CHECK(hipMalloc((void **)&dv0, 3 * (size_t)N * sizeof(float)));
    CHECK(hipMalloc((void **)&dC0, 9 * (size_t)N * sizeof(float)));
    CHECK(hipMalloc((void **)&dF0, 9 * (size_t)N * sizeof(float)));
    CHECK(hipMalloc((void **)&dmat, sizeof material));
    CHECK(hipMalloc((void **)&du, 3 * sizeof(float)));
    CHECK(hipMemcpy(dx0, x0, 3 * (size_t)N * sizeof(float), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dv0, zero, 3 * (size_t)N * sizeof(float), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dC0, zero, 9 * (size_t)N * sizeof(float), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dF0, F0, 9 * (size_t)N * sizeof(float), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dmat, material, sizeof material, hipMemcpyHostToDevice));

    const int32_t np[1] = {N}, gn[1] = {n};
    mpm_desc d;
    memset(&d, 0, sizeof d);
    d.n_envs = 1;
    d.n_particles = np;
    d.grid_n = gn;
    d.dt = dt;
    memcpy(d.gravity, g, sizeof g);
    d.bound = 3;
    d.max_tools = 1;
    d.checkpoint_every = 1;
    d.max_tape_substeps = 0;
    d.x0 = dx0; d.v0 = dv0; d.C0 = dC0; d.F0 = dF0;
    d.material = dmat;
    size_t bytes = mpm_workspace_size(&d);
    if (bytes == 0) { fprintf(stderr, "workspace size: %s\n", mpm_last_error(NULL)); return 1; }
    void *ws;
    CHECK(hipMalloc(&ws, bytes));
    mpm_ctx *ctx = NULL;
    CHECK(mpm_create(&d, ws, bytes, NULL, &ctx));

    CHECK(mpm_substep(ctx, S, 0, NULL));
    CHECK(mpm_read_state(ctx, 0, MPM_F_X, xs, 3 * (size_t)N * sizeof(float), 0, NULL));
    CHECK(mpm_read_state(ctx, 0, MPM_F_V, vs, 3 * (size_t)N * sizeof(float), 0, NULL));
    CHECK(mpm_read_state(ctx, 0, MPM_F_F, Fs, 9 * (size_t)N * sizeof(float), 0, NULL));
    double ex = 0.0, ev = 0.0, eF = 0.0;
    for (int p = 0; p < N; ++p)
        for (int a = 0; a < 3; ++a) {
            double xe = x0[a * N + p] + (double)dt * dt * g[a] * S * (S + 1) / 2.0;
            ex = fmax(ex, fabs(xs[a * N + p] - xe));
            ev = fmax(ev, fabs(vs[a * N + p] - (double)S * dt * g[a]));
        }
    for (int c = 0; c < 9; ++c)
        for (int p = 0; p < N; ++p) eF = fmax(eF, fabs(Fs[c * (size_t)N + p] - ((c % 4) == 0 ? 1.0 : 0.0)));
    printf("free fall: |x - exact| %.2e  |v - exact| %.2e  |F - I| %.2e\n", ex, ev, eF);
    int ok = ex <= 1e-6 && ev <= 1e-5 && eF <= 1e-5;

    /* a capsule pressing on the block's top */
    const float u[3] = {0.0f, -0.3f, 0.0f};
    CHECK(hipMemcpy(du, u, sizeof u, hipMemcpyHostToDevice));
    mpm_tool t;
    memset(&t, 0, sizeof t);
    t.shape = MPM_TOOL_CAPSULE;
    t.contact = MPM_CONTACT_SLIP;
    t.radius = 0.02f;
    t.half_len = 0.05f;
    t.friction = 0.3f;
    t.theta = 1e-3f;
    t.R[0] = t.R[4] = t.R[8] = 1.0f;
    t.T0[0] = 0.48f;
    t.T0[1] = 0.40f + side_len + 0.015f;
    t.T0[2] = 0.48f;
    CHECK(mpm_set_tool(ctx, 0, 0, &t, du, 1));
    CHECK(mpm_substep(ctx, S, 0, NULL));
    uint32_t status = 99;
    int32_t steps = 0;
    CHECK(mpm_read_state(ctx, 0, MPM_F_STATUS, &status, sizeof status, 0, NULL));
    CHECK(mpm_read_state(ctx, 0, MPM_F_STEP, &steps, sizeof steps, 0, NULL));
    printf("pressed: status %u  substeps %d\n", status, steps);
    ok = ok && status == 0 && steps == 2 * S;

    mpm_destroy(ctx);
    hipFree(ws); hipFree(dx0); hipFree(dv0); hipFree(dC0); hipFree(dF0); hipFree(dmat); hipFree(du);
    free(x0); free(zero); free(F0); free(xs); free(vs); free(Fs);
    printf("%s\n", ok ? "ok" : "FAILED");
    return ok ? 0 : 1;
}
