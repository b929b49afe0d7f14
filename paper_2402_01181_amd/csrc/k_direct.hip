// Direct scheme: one thread per particle with global float atomics for P2G,
// one thread per node over the dense grid for the grid operation, one thread
// per particle for G2P.  Used for per-stage inspection and as the
// cross-check of the tiled scheme.
#include "mpm_kernels.h"

namespace mpm {

// P2G (Sec. III-B item 1): scatter mass and APIC momentum with the MLS stress
// term  w [m v + (m C - dt V0 (4/dx^2) tau) (x_i - x_p)]  to the 27 nodes.
__global__ __launch_bounds__(256) void k_p2g_direct(Dev d)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.ntot) return;
    int env = env_of_particle(d, q);
    const EnvDev e = load_env(d.env + env);
    const int N = d.ntot;
    float x0 = d.x[q], x1 = d.x[N + q], x2 = d.x[2 * N + q];
    Stencil s;
    make_stencil(x0, x1, x2, e.inv_dx, e.n, s);
    if (stencil_outside(s, e.n)) {
        set_flag(d.status, env, MPM_FLAG_OUT_OF_DOMAIN);
        return;
    }
    const float *mat = d.material + 4 * env;
    float mu, lam;
    lame(mat[0], mat[1], mu, lam);
    const float V0 = mat[3], m = mat[2] * mat[3];
    float H[9], tau[9], A[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) H[c] = gload(d.H + (size_t)c * N + q);
    if (kirchhoff(H, mu, lam, tau)) set_flag(d.status, env, MPM_FLAG_INVERTED);
    const float k = -d.dt * V0 * 4.0f * e.inv_dx * e.inv_dx;
#pragma unroll
    for (int c = 0; c < 9; ++c) A[c] = k * tau[c] + m * d.C[(size_t)c * N + q];
    float mv0 = m * d.v[q], mv1 = m * d.v[N + q], mv2 = m * d.v[2 * N + q];
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                float d0 = (o0 - s.fx[0]) * e.dx, d1 = (o1 - s.fx[1]) * e.dx, d2 = (o2 - s.fx[2]) * e.dx;
                float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                float p0 = mv0 + A[0] * d0 + A[1] * d1 + A[2] * d2;
                float p1 = mv1 + A[3] * d0 + A[4] * d1 + A[5] * d2;
                float p2 = mv2 + A[6] * d0 + A[7] * d1 + A[8] * d2;
                float *g = reinterpret_cast<float *>(d.gP + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2));
                gatomic_add(g + 0, w * m);
                gatomic_add(g + 1, w * p0);
                gatomic_add(g + 2, w * p1);
                gatomic_add(g + 3, w * p2);
            }
}

// Grid operation over every node of every environment (dense).  zero_P
// clears the momentum buffer behind it for the next P2G.
__global__ __launch_bounds__(256) void k_grid_dense(Dev d, const int64_t *env_gofs, int64_t total_nodes, int zero_P)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_nodes) return;
    int lo = 0, hi = d.n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (env_gofs[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const EnvDev e = load_env(d.env + lo);
    int64_t local = g - e.gofs;
    int i, j, k;
    brick_local_to_ijk(e, (int)(local >> 6), (int)(local & 63), i, j, k);
    float4 P = d.gP[g];
    float3 v = grid_node_velocity(d, e, lo, P, i, j, k, nullptr);
    d.gV[g] = make_float4(v.x, v.y, v.z, 0.0f);
    if (zero_P) d.gP[g] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// End of a substep: advance each active tool, T <- T + dt u_k, k <- k + 1
// (FP64 position), and count the substep of each environment.
__device__ __forceinline__ void advance_tools(const Dev &d, int t)
{
    if (t < d.n_envs) d.step[t] += 1;
    if (t < d.n_envs * d.max_tools) {
        ToolDev &T = d.tools[t];
        if (T.active) {
            advance_tool(T, d.dt);
        }
    }
}

// G2P (Sec. III-B item 3) + advection + F update (I + dt C) F (kept as H = F - I).
__global__ __launch_bounds__(256) void k_g2p_direct(Dev d)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    advance_tools(d, q);
    if (q >= d.ntot) return;
    int env = env_of_particle(d, q);
    const EnvDev e = load_env(d.env + env);
    const int N = d.ntot;
    float x0 = d.x[q], x1 = d.x[N + q], x2 = d.x[2 * N + q];
    Stencil s;
    make_stencil(x0, x1, x2, e.inv_dx, e.n, s);
    if (stencil_outside(s, e.n)) {
        set_flag(d.status, env, MPM_FLAG_OUT_OF_DOMAIN);
        return;
    }
    float vp0 = 0.f, vp1 = 0.f, vp2 = 0.f;
    float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                float d0 = (o0 - s.fx[0]), d1 = (o1 - s.fx[1]), d2 = (o2 - s.fx[2]);
                float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                float4 V = gload(d.gV + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2));
                float wx = w * V.x, wy = w * V.y, wz = w * V.z;
                vp0 += wx; vp1 += wy; vp2 += wz;
                B[0] += wx * d0; B[1] += wx * d1; B[2] += wx * d2;
                B[3] += wy * d0; B[4] += wy * d1; B[5] += wy * d2;
                B[6] += wz * d0; B[7] += wz * d1; B[8] += wz * d2;
            }
    // C = (4/dx^2) sum w v_i (x_i - x_p)^T with (x_i - x_p) = (o - fx) dx
    const float cs = 4.0f * e.inv_dx;
    float Cn[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) Cn[c] = cs * B[c];
    x0 += d.dt * vp0; x1 += d.dt * vp1; x2 += d.dt * vp2;
    float H[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) H[c] = gload(d.H + (size_t)c * N + q);
    update_h(H, Cn, d.dt);
    if (inverted_h(H)) set_flag(d.status, env, MPM_FLAG_INVERTED);
    if (!(isfinite(x0) && isfinite(x1) && isfinite(x2) && isfinite(vp0) && isfinite(vp1) && isfinite(vp2)))
        set_flag(d.status, env, MPM_FLAG_NONFINITE);
    d.x[q] = x0; d.x[N + q] = x1; d.x[2 * N + q] = x2;
    d.v[q] = vp0; d.v[N + q] = vp1; d.v[2 * N + q] = vp2;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        d.C[(size_t)c * N + q] = Cn[c];
        d.H[(size_t)c * N + q] = H[c];
    }
}

void launch_p2g_direct(const Dev &d, hipStream_t st)
{
    launch_k(k_p2g_direct, dim3((d.ntot + 255) / 256), dim3(256), 0, st, d);
}

void launch_grid_dense(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, int zero_P, hipStream_t st)
{
    launch_k(k_grid_dense, dim3((unsigned)((total_nodes + 255) / 256)), dim3(256), 0, st, d, env_gofs,
                       total_nodes, zero_P);
}

void launch_g2p_direct(const Dev &d, hipStream_t st)
{
    int n = d.ntot;
    if (n < d.n_envs * d.max_tools) n = d.n_envs * d.max_tools;
    if (n < d.n_envs) n = d.n_envs;
    launch_k(k_g2p_direct, dim3((n + 255) / 256), dim3(256), 0, st, d);
}

}  // namespace mpm
