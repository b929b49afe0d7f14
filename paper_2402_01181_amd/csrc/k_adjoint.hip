// Reverse-mode substep (adjoint of P2G, the grid operation, G2P and the F
// update), run over a tape recorded by a forward recompute.
//
// Per reverse substep j, with the adjoints of the state after substep j:
//   k_adj_g2p : F update, advection and G2P reversed; scatters the adjoint of
//               the node velocities (27 nodes x 3 floats per particle).
//   k_adj_grid: grid operation reversed node by node, using the contact
//               decisions the tape recorded; yields adjoints of (m, mv) and
//               the tool-velocity / tool-position gradients.
//   k_adj_p2g : P2G and the Neo-Hookean stress reversed; gathers the node
//               adjoints and accumulates dL/dmu, dL/dlambda.
// The last three also give the adjoints of the state before substep j.
#include <stdexcept>

#include "mpm_adjoint.h"
#include "mpm_tile_util.h"

namespace mpm {

// Grid pass of a tape recompute at node g (local index `local` in
// environment env's grid, tool slots at tl): like the grid operation, but it
// writes (m, vhat) back into P, the final velocity into V and the contact
// decision of the node.
__device__ __forceinline__ void grid_tape_node(const Dev &d, const EnvDev &e, const ToolDev *tl, int64_t g,
                                               int64_t local, ContactCode *dec)
{
    int i, j, k;
    brick_local_to_ijk(e, (int)(local >> 6), (int)(local & 63), i, j, k);
    const float4 P = gload(d.gP + g);
    ContactRec rec;
    const float3 v = grid_node_velocity_tl(d, e, tl, P, i, j, k, &rec);
    const float3 vh = node_vhat(d, P);
    gstore(d.gV + g, make_float4(v.x, v.y, v.z, 0.f));
    gstore(d.gP + g, make_float4(P.x, vh.x, vh.y, vh.z));
    gstore(dec + g, (ContactCode)(rec.tool < 0 || rec.branch == 0 ? -1 : rec.tool * 4 + rec.branch));
}

__device__ __forceinline__ int env_of_node(const Dev &d, const int64_t *env_gofs, int64_t g)
{
    int lo = 0, hi = d.n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (gload(env_gofs + mid) <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Calls body(env, environment entry, its tool slots, node, local index) for
// every node the pass visits: the listed bricks, a wavefront each, or every
// node.  The kernels that call it run 256 threads a workgroup; tls is their
// LDS room for one environment's tool slots.  The listed pass of a single
// environment reads its entry, grid offset and tool slots (into tls, with
// TOOLS) once, in the same round of loads as the list count and each wave's
// first brick, so a brick's nodes wait for one load (its id) before their own.
template <bool TOOLS, class Body>
__device__ __forceinline__ void tape_nodes(const Dev &d, const int64_t *env_gofs, int64_t total_nodes,
                                           const TapeList &tl, ToolDev *tls, Body &&body)
{
    constexpr int T = 256, nw = T >> 6;
    const int lane = threadIdx.x & 63, stride = gridDim.x * nw;
    int i = blockIdx.x * nw + (threadIdx.x >> 6);
    // the list holds at most one entry per brick of the grid
    const int64_t cap = total_nodes / BRICK_NODES;
    const int n = uload(tl.scount);
    int b0 = i < cap ? uload(tl.slist + i) : 0;
    const bool dense = tl.dense || uload(tl.far + tl.far_slot) == tl.far_stamp;
    if (dense) {
        const int64_t gs = (int64_t)gridDim.x * T;
        for (int64_t g = (int64_t)blockIdx.x * T + threadIdx.x; g < total_nodes; g += gs) {
            const int env = env_of_node(d, env_gofs, g);
            body(env, load_env(d.env + env), d.tools + (size_t)env * d.max_tools, g, g - gload(env_gofs + env));
        }
        return;
    }
    if (d.n_envs == 1) {
        const EnvDev e = load_env(d.env);
        const int64_t o = gload(env_gofs);
        const ToolDev *t = d.tools;
        if (TOOLS) {
            const int words = d.max_tools * (int)(sizeof(ToolDev) / 4);
            for (int w = threadIdx.x; w < words; w += T)
                reinterpret_cast<int *>(tls)[w] = gload(reinterpret_cast<const int *>(d.tools) + w);
            __syncthreads();
            t = tls;
        }
        for (; i < n; i += stride, b0 = i < cap ? uload(tl.slist + i) : 0) {
            const int64_t g = (int64_t)b0 * BRICK_NODES + lane;
            body(0, e, t, g, g - o);
        }
        return;
    }
    for (; i < n; i += stride, b0 = i < cap ? uload(tl.slist + i) : 0) {
        const int env = uload(tl.brick_env + b0);
        const int64_t g = (int64_t)b0 * BRICK_NODES + lane;
        body(env, load_env(d.env + env), d.tools + (size_t)env * d.max_tools, g, g - gload(env_gofs + env));
    }
}

__global__ __launch_bounds__(256) void k_grid_tape(Dev d, const int64_t *env_gofs, int64_t total_nodes,
                                                   ContactCode *dec, ToolDev *snap, int slots, TapeList tl)
{
    __shared__ ToolDev tls[MAX_TOOLS];
    if (snap)
        for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < slots; t += (int64_t)gridDim.x * 256)
            snap[t] = d.tools[t];
    tape_nodes<true>(d, env_gofs, total_nodes, tl, tls,
                     [&](int, const EnvDev &e, const ToolDev *t, int64_t g, int64_t local) {
                         grid_tape_node(d, e, t, g, local, dec);
                     });
}

__device__ __forceinline__ void weight_grads(const Stencil &s, float dw[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float f = s.fx[a];
        dw[a][0] = -(1.5f - f);
        dw[a][1] = -2.0f * (f - 1.0f);
        dw[a][2] = f - 0.5f;
    }
}

// Reverse of G2P + advection + F update for one particle.
__global__ __launch_bounds__(256) void k_adj_g2p(Dev d, AdjBuf a)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.ntot) return;
    const int N = d.ntot;
    int env = env_of_particle(d, q);
    const EnvDev e = load_env(d.env + env);
    float x0 = gload(d.x + q), x1 = gload(d.x + N + q), x2 = gload(d.x + 2 * N + q);
    Stencil s;
    make_stencil(x0, x1, x2, e.inv_dx, e.n, s);
    if (s.outside) return;   // frozen particle: state and adjoints pass through
    float dw[3][3];
    weight_grads(s, dw);
    // forward C' from the tape's node velocities
    float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float4 Vn[27];
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                int n = (o0 * 3 + o1) * 3 + o2;
                Vn[n] = gload(d.gV + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2));
                float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                float q0 = o0 - s.fx[0], q1 = o1 - s.fx[1], q2 = o2 - s.fx[2];
                float wx = w * Vn[n].x, wy = w * Vn[n].y, wz = w * Vn[n].z;
                B[0] += wx * q0; B[1] += wx * q1; B[2] += wx * q2;
                B[3] += wy * q0; B[4] += wy * q1; B[5] += wy * q2;
                B[6] += wz * q0; B[7] += wz * q1; B[8] += wz * q2;
            }
    const float cs = 4.0f * e.inv_dx;
    float Cn[9], H[9], Fb[9], Cb[9], xb[3], vb[3];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        Cn[c] = cs * B[c];
        H[c] = gload(d.H + (size_t)c * N + q);
        Fb[c] = gload(a.Fb + (size_t)c * N + q);
        Cb[c] = gload(a.Cb + (size_t)c * N + q);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xb[c] = gload(a.xb + (size_t)c * N + q);
        vb[c] = gload(a.vb + (size_t)c * N + q);
    }
    // F' = (I + dt C') F:  Fbar <- (I + dt C')^T Fbar',  Cbar' += dt Fbar' F^T  (F = I + H)
    float Fbn[9], Cbt[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Fbn[3 * r + c] = Fb[3 * r + c] + d.dt * (Cn[r] * Fb[c] + Cn[3 + r] * Fb[3 + c] + Cn[6 + r] * Fb[6 + c]);
            Cbt[3 * r + c] = Cb[3 * r + c] + d.dt * (Fb[3 * r + c] + Fb[3 * r] * H[3 * c] + Fb[3 * r + 1] * H[3 * c + 1] +
                                                     Fb[3 * r + 2] * H[3 * c + 2]);
        }
    // x' = x + dt v'
    float vbt[3] = {vb[0] + d.dt * xb[0], vb[1] + d.dt * xb[1], vb[2] + d.dt * xb[2]};
    float Bb[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) Bb[c] = cs * Cbt[c];
    float fxb[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                int n = (o0 * 3 + o1) * 3 + o2;
                float q0 = o0 - s.fx[0], q1 = o1 - s.fx[1], q2 = o2 - s.fx[2];
                float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                float g0 = vbt[0] + Bb[0] * q0 + Bb[1] * q1 + Bb[2] * q2;
                float g1 = vbt[1] + Bb[3] * q0 + Bb[4] * q1 + Bb[5] * q2;
                float g2 = vbt[2] + Bb[6] * q0 + Bb[7] * q1 + Bb[8] * q2;
                float *gv = reinterpret_cast<float *>(a.gVb + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2));
                gatomic_add(gv + 0, w * g0);
                gatomic_add(gv + 1, w * g1);
                gatomic_add(gv + 2, w * g2);
                const float4 V = Vn[n];
                float wb = V.x * g0 + V.y * g1 + V.z * g2;
                // qbar = w Bbar^T V; q = o - fx
                float qb0 = w * (Bb[0] * V.x + Bb[3] * V.y + Bb[6] * V.z);
                float qb1 = w * (Bb[1] * V.x + Bb[4] * V.y + Bb[7] * V.z);
                float qb2 = w * (Bb[2] * V.x + Bb[5] * V.y + Bb[8] * V.z);
                fxb[0] += -qb0 + wb * dw[0][o0] * s.w[1][o1] * s.w[2][o2];
                fxb[1] += -qb1 + wb * s.w[0][o0] * dw[1][o1] * s.w[2][o2];
                fxb[2] += -qb2 + wb * s.w[0][o0] * s.w[1][o1] * dw[2][o2];
            }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        gstore(a.xb + (size_t)c * N + q, xb[c] + e.inv_dx * fxb[c]);
        gstore(a.vb + (size_t)c * N + q, 0.0f);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        gstore(a.Fb + (size_t)c * N + q, Fbn[c]);
        gstore(a.Cb + (size_t)c * N + q, 0.0f);
    }
}

// Reverse of the grid operation at one node with mass; vb is the adjoint of
// the node's final velocity.  Returns the adjoint of vhat and adds the
// contact tool's velocity / position adjoints.
__device__ __forceinline__ float3 node_adjoint(const ToolDev *tl, const EnvDev &e, float3 vh, int i, int j, int k,
                                               ContactCode code, float3 vb, int &tool, float3 &ub, float3 &Tb)
{
    tool = -1;
    ub = make_float3(0.f, 0.f, 0.f);
    Tb = make_float3(0.f, 0.f, 0.f);
    if (boundary_node(e, i, j, k)) return make_float3(0.f, 0.f, 0.f);
    if (code < 0) return vb;
    const int t = code >> 2, branch = code & 3;
    const ToolDev &T = tl[t];
    tool = t;
    ub = vb;                                   // v = v_rel' + u
    if (branch == 2) return make_float3(0.f, 0.f, 0.f);
    // friction branch: v = s v_t + u with s = 1 + mu vn/|vt|
    float3 u = tool_velocity(T);
    float3 n = tool_hit(T, e, i, j, k).n;
    float r0 = vh.x - u.x, r1 = vh.y - u.y, r2 = vh.z - u.z;
    float vn = r0 * n.x + r1 * n.y + r2 * n.z;
    float t0 = r0 - vn * n.x, t1 = r1 - vn * n.y, t2 = r2 - vn * n.z;
    float nt = sqrtf(t0 * t0 + t1 * t1 + t2 * t2);
    float s = 1.0f + T.friction * vn / nt;
    float sb = vb.x * t0 + vb.y * t1 + vb.z * t2;
    float tb0 = s * vb.x, tb1 = s * vb.y, tb2 = s * vb.z;
    float vnb = sb * T.friction / nt;
    float ntb = -sb * T.friction * vn / (nt * nt);
    tb0 += ntb * t0 / nt; tb1 += ntb * t1 / nt; tb2 += ntb * t2 / nt;
    vnb -= tb0 * n.x + tb1 * n.y + tb2 * n.z;
    float rb0 = tb0 + vnb * n.x, rb1 = tb1 + vnb * n.y, rb2 = tb2 + vnb * n.z;
    float nb0 = -vn * tb0 + vnb * r0, nb1 = -vn * tb1 + vnb * r1, nb2 = -vn * tb2 + vnb * r2;
    ub.x -= rb0; ub.y -= rb1; ub.z -= rb2;
    Tb = tool_pose_bar(T, e, i, j, k, make_float3(nb0, nb1, nb2));
    return make_float3(rb0, rb1, rb2);
}

// Add a wavefront's tool-gradient terms c (dL/du, then dL/dT, of tool `tool`,
// -1: none) of environment env and reverse substep a.j: summed over the
// wavefront first when one tool is concerned, then one set of atomics.
__device__ __forceinline__ void wave_tool_add(const Dev &d, const AdjBuf &a, int env, int tool, const double c[6])
{
    const bool has = tool >= 0;
    const uint64_t m = __ballot(has);
    if (!m) return;
    const int lead = __ffsll((unsigned long long)m) - 1, t0 = __shfl(tool, lead);
    auto at = [&](int t) { return (((size_t)env * d.max_tools + t) * a.max_tape + a.j) * 3; };
    if (__all(!has || tool == t0)) {
        double s[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            s[q] = has ? c[q] : 0.0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off);
        }
        if ((threadIdx.x & 63) == lead) {
            const size_t o = at(t0);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                gatomic_add(a.ubar + o + q, s[q]);
                gatomic_add(a.Tbar + o + q, s[3 + q]);
            }
        }
    } else if (has) {
        const size_t o = at(tool);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            gatomic_add(a.ubar + o + q, c[q]);
            gatomic_add(a.Tbar + o + q, c[3 + q]);
        }
    }
}

// Reverse grid operation at node g; clears the node-velocity adjoint and the
// tape's (m, v-hat) there.
__device__ __forceinline__ void adj_grid_node(const Dev &d, const EnvDev &e, const ToolDev *tl, int env, int64_t g,
                                              int64_t local, const ContactCode *dec, const AdjBuf &a)
{
    // the node's tape entries and velocity adjoint, loaded together
    const float4 P = gload(d.gP + g);                                // (m, vhat)
    const float4 vb4 = gload(a.gVb + g);
    const ContactCode code = gload(dec + g);
    // a wavefront is one brick (environments' grids start at multiples of 64 nodes);
    // a brick without mass is in no particle's stencil: its velocity adjoint was
    // never scattered to (still zero), its (m, mv) adjoint is never gathered and
    // its tape entry is already zero
    if (!__any(P.x > 0.0f)) return;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    gstore(a.gVb + g, zero);                // ready for the next reverse substep
    gstore(d.gP + g, zero);                 // the tape grid is zero between recomputes
    int tool = -1;
    float3 ub = make_float3(0.f, 0.f, 0.f), Tb = make_float3(0.f, 0.f, 0.f);
    if (P.x > 0.0f) {
        int i, j, k;
        brick_local_to_ijk(e, (int)(local >> 6), (int)(local & 63), i, j, k);
        const float3 vh = make_float3(P.y, P.z, P.w);
        const float3 vhb = node_adjoint(tl, e, vh, i, j, k, code, make_float3(vb4.x, vb4.y, vb4.z), tool, ub, Tb);
        // vhat = P/m + dt g:  Pbar = vhbar/m,  mbar = -vhbar . (P/m) / m
        const float pm0 = vh.x - d.dt * d.gx, pm1 = vh.y - d.dt * d.gy, pm2 = vh.z - d.dt * d.gz;
        const float mb = -(vhb.x * pm0 + vhb.y * pm1 + vhb.z * pm2) / P.x;
        gstore(a.gPb + g, make_float4(mb, vhb.x / P.x, vhb.y / P.x, vhb.z / P.x));
    } else {
        gstore(a.gPb + g, zero);
    }
    // the tool gradients of the brick's contact nodes (every lane of the wavefront is here)
    const double c6[6] = {ub.x, ub.y, ub.z, Tb.x, Tb.y, Tb.z};
    wave_tool_add(d, a, env, tool, c6);
}

__global__ __launch_bounds__(256) void k_adj_grid(Dev d, const int64_t *env_gofs, int64_t total_nodes,
                                                  const ContactCode *dec, AdjBuf a, TapeList tl)
{
    __shared__ ToolDev tls[MAX_TOOLS];
    tape_nodes<true>(d, env_gofs, total_nodes, tl, tls,
                     [&](int env, const EnvDev &e, const ToolDev *t, int64_t g, int64_t local) {
                         adj_grid_node(d, e, t, env, g, local, dec, a);
                     });
}

// Sum per environment over a wavefront, then one double atomic per wave.
__device__ __forceinline__ void wave_env_add(double *dst, int env, double v, bool active)
{
    int env0 = __shfl(env, 0);
    bool uniform = __all(!active || env == env0);
    if (uniform) {
        double s = active ? v : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((threadIdx.x & 63) == 0 && __any(active)) gatomic_add(dst + env0, s);
    } else if (active) {
        gatomic_add(dst + env, v);
    }
}

// Reverse of P2G and of the stress for one particle.
__global__ __launch_bounds__(256) void k_adj_p2g(Dev d, AdjBuf a)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = d.ntot;
    bool active = q < N;
    int env = 0;
    double mub = 0.0, lamb = 0.0;
    if (active) {
        env = env_of_particle(d, q);
        const EnvDev e = load_env(d.env + env);
        float x0 = gload(d.x + q), x1 = gload(d.x + N + q), x2 = gload(d.x + 2 * N + q);
        Stencil s;
        make_stencil(x0, x1, x2, e.inv_dx, e.n, s);
        if (!s.outside) {
            const float *mat = d.material + 4 * env;
            float E = gload(mat), nu = gload(mat + 1), rho = gload(mat + 2), V0 = gload(mat + 3);
            float mu, lam;
            lame(E, nu, mu, lam);
            const float m = rho * V0;
            const float kf = -d.dt * V0 * 4.0f * e.inv_dx * e.inv_dx;
            float H[9], F[9], C[9], v[3], tau[9], A[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                H[c] = gload(d.H + (size_t)c * N + q);
                F[c] = H[c] + ((c & 3) == 0 ? 1.0f : 0.0f);
                C[c] = gload(d.C + (size_t)c * N + q);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = gload(d.v + (size_t)c * N + q);
            bool inverted = kirchhoff(H, mu, lam, tau);
#pragma unroll
            for (int c = 0; c < 9; ++c) A[c] = kf * tau[c] + m * C[c];
            float dw[3][3];
            weight_grads(s, dw);
            float vbp[3] = {0.f, 0.f, 0.f}, Ab[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float fxb[3] = {0.f, 0.f, 0.f};
            const float dx = e.dx;
#pragma unroll
            for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
                for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
                    for (int o2 = 0; o2 < 3; ++o2) {
                        float4 Pb = gload(a.gPb + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2));
                        float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                        float d0 = (o0 - s.fx[0]) * dx, d1 = (o1 - s.fx[1]) * dx, d2 = (o2 - s.fx[2]) * dx;
                        vbp[0] += m * w * Pb.y; vbp[1] += m * w * Pb.z; vbp[2] += m * w * Pb.w;
                        float wy = w * Pb.y, wz = w * Pb.z, ww = w * Pb.w;
                        Ab[0] += wy * d0; Ab[1] += wy * d1; Ab[2] += wy * d2;
                        Ab[3] += wz * d0; Ab[4] += wz * d1; Ab[5] += wz * d2;
                        Ab[6] += ww * d0; Ab[7] += ww * d1; Ab[8] += ww * d2;
                        float c0 = m * v[0] + A[0] * d0 + A[1] * d1 + A[2] * d2;
                        float c1 = m * v[1] + A[3] * d0 + A[4] * d1 + A[5] * d2;
                        float c2 = m * v[2] + A[6] * d0 + A[7] * d1 + A[8] * d2;
                        float wb = m * Pb.x + Pb.y * c0 + Pb.z * c1 + Pb.w * c2;
                        // dpos = q dx, q = o - fx:  fxbar -= dx * w A^T Pbar
                        float db0 = w * (A[0] * Pb.y + A[3] * Pb.z + A[6] * Pb.w);
                        float db1 = w * (A[1] * Pb.y + A[4] * Pb.z + A[7] * Pb.w);
                        float db2 = w * (A[2] * Pb.y + A[5] * Pb.z + A[8] * Pb.w);
                        fxb[0] += -dx * db0 + wb * dw[0][o0] * s.w[1][o1] * s.w[2][o2];
                        fxb[1] += -dx * db1 + wb * s.w[0][o0] * dw[1][o1] * s.w[2][o2];
                        fxb[2] += -dx * db2 + wb * s.w[0][o0] * s.w[1][o1] * dw[2][o2];
                    }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float* px = a.xb + (size_t)c * N + q;
                gstore(px, gload(px) + e.inv_dx * fxb[c]);
                float* pv = a.vb + (size_t)c * N + q;
                gstore(pv, gload(pv) + vbp[c]);
            }
            float taub[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                float* pc = a.Cb + (size_t)c * N + q;
                gstore(pc, gload(pc) + m * Ab[c]);
                taub[c] = kf * Ab[c];
            }
            // tau = mu (F F^T - I) + lam ln J I
            float Fb[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    Fb[3 * r + c] = mu * ((taub[3 * r] + taub[r]) * F[c] + (taub[3 * r + 1] + taub[3 + r]) * F[3 + c] +
                                          (taub[3 * r + 2] + taub[6 + r]) * F[6 + c]);
            double trt = (double)taub[0] + taub[4] + taub[8];
            double jm1 = jm1_of(H);
            double lnJ = inverted ? log(J_MIN) : log1p(jm1);
            if (!inverted) {
                // F^-T = cof(F) / J, F = I + H exactly in FP64
                double f[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) f[c] = (double)H[c] + ((c & 3) == 0 ? 1.0 : 0.0);
                double ci[9] = {f[4] * f[8] - f[5] * f[7], -(f[3] * f[8] - f[5] * f[6]), f[3] * f[7] - f[4] * f[6],
                                -(f[1] * f[8] - f[2] * f[7]), f[0] * f[8] - f[2] * f[6], -(f[0] * f[7] - f[1] * f[6]),
                                f[1] * f[5] - f[2] * f[4], -(f[0] * f[5] - f[2] * f[3]), f[0] * f[4] - f[1] * f[3]};
                double sc = (double)lam * trt / (1.0 + jm1);
#pragma unroll
                for (int c = 0; c < 9; ++c) Fb[c] += (float)(sc * ci[c]);
            }
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                float* pf = a.Fb + (size_t)c * N + q;
                gstore(pf, gload(pf) + Fb[c]);
            }
            // dL/dmu = taubar : (F F^T - I) = taubar : (H + H^T + H H^T),  dL/dlambda = tr(taubar) ln J
            double ff = 0.0;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double G = (double)H[3 * r + c] + H[3 * c + r] + (double)H[3 * r] * H[3 * c] +
                               (double)H[3 * r + 1] * H[3 * c + 1] + (double)H[3 * r + 2] * H[3 * c + 2];
                    ff += (double)taub[3 * r + c] * G;
                }
            mub = ff;
            lamb = trt * lnJ;
        }
    }
    wave_env_add(a.mubar, env, mub, active);
    wave_env_add(a.lambar, env, lamb, active);
}

// Chain the per-substep tool gradients through T_{s+1} = T_s + dt u_s and
// the Lame parameters through (E, nu).  One thread per (env, tool).
__global__ __launch_bounds__(256) void k_adj_finish(Dev d, AdjBuf a, int n, double *gE, double *gnu, double *gu, double *gT)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int nt = d.max_tools > 0 ? d.max_tools : 1;
    if (t >= d.n_envs * nt) return;
    int env = t / nt, tool = t % nt;
    if (d.max_tools > 0) {
        // dL/du_j = ubar_j + dt (Tbar_{j+1} + ... + Tbar_{n-1}), summed from the last
        // substep down; K substeps' terms are loaded together before they are used
        constexpr int K = 16;
        const size_t ib = ((size_t)env * d.max_tools + tool) * a.max_tape * 3;
        const size_t ob = ((size_t)env * d.max_tools + tool) * (size_t)n * 3;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int j1 = n; j1 > 0; j1 -= K) {
            double ub[K][3], tb[K][3];
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int j = j1 - 1 - q;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ub[q][c] = j >= 0 && gu ? gload(a.ubar + ib + (size_t)j * 3 + c) : 0.0;
                    tb[q][c] = j >= 0 ? gload(a.Tbar + ib + (size_t)j * 3 + c) : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int j = j1 - 1 - q;   // j < 0: past the first substep, its terms are zero
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (gu && j >= 0) gstore(gu + ob + (size_t)j * 3 + c, ub[q][c] + (double)d.dt * acc[c]);
                    acc[c] += tb[q][c];
                }
            }
        }
        if (gT)
            for (int c = 0; c < 3; ++c) gstore(gT + ((size_t)env * d.max_tools + tool) * 3 + c, acc[c]);
    }
    if (tool == 0) {
        double E = gload(d.material + 4 * env), nu = gload(d.material + 4 * env + 1);
        double mub = gload(a.mubar + env), lamb = gload(a.lambar + env);
        double dmu_dE = 1.0 / (2.0 * (1.0 + nu)), dmu_dnu = -E / (2.0 * (1.0 + nu) * (1.0 + nu));
        double dlam_dE = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        double dlam_dnu = E * (1.0 + 2.0 * nu * nu) / ((1.0 + nu) * (1.0 + nu) * (1.0 - 2.0 * nu) * (1.0 - 2.0 * nu));
        if (gE) gstore(gE + env, mub * dmu_dE + lamb * dlam_dE);
        if (gnu) gstore(gnu + env, mub * dmu_dnu + lamb * dlam_dnu);
    }
}

// dst[c][pid[q]] = src[c][q]  (slot order -> original order)
// Component c of element `from` of src to element `to` of dst, c < comps, in
// groups of eight whose loads are all issued before the group's stores (the
// arrays may alias as far as the compiler knows: a store between two loads
// would wait for the first load's round trip).
__device__ __forceinline__ void move_components(const float *src, size_t from, float *dst, size_t to, size_t n,
                                                int comps)
{
    for (int c0 = 0; c0 < comps; c0 += 8) {
        float t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (c0 + k < comps) t[k] = gload(src + (size_t)(c0 + k) * n + from);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (c0 + k < comps) gstore(dst + (size_t)(c0 + k) * n + to, t[k]);
    }
}

__global__ void k_unpermute(const float *src, const int32_t *pid, int ntot, int comps, float *dst)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ntot) return;
    int o = gload(pid + q);
    move_components(src, q, dst, o, ntot, comps);
}

__global__ void k_copy_words(uint32_t *dst, const uint32_t *src, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        gstore(dst + i, gload(src + i));
}

// Up to COPY_JOBS word copies in one launch: job blockIdx.y.
__global__ void k_copy_jobs(CopyJobs j)
{
    const int q = blockIdx.y;
    uint32_t *dst = j.dst[q];
    const uint32_t *src = j.src[q];
    const size_t n = j.words[q];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        gstore(dst + i, gload(src + i));
}

__global__ void k_fill_f64(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        gstore(p + i, 0.0);
}

// ---------------------------------------------------------------------------
// Tiled reverse kernels: particles in brick-sorted slots (the order a tape
// segment was recomputed in), one work item per (brick, slot range).

struct AdjTiledArgs {
    const int4 *items;  // (brick, first slot, count, environment)
    const int2 *totals;
    int slots;          // node pass: particles per half-wave step (1 or 3)
    ActiveBuf act;      // unused by the reverse kernels (no marking)
};

// Reverse of G2P + advection + F update for one particle whose stencil s
// lies in the grid (state H at the start of the substep, node velocities
// through Vat(a0, a1, a2)).  In: the adjoints xb, vb, Cb, Fb of the state
// after the substep; out: those of the state before it (vb and Cb become
// zero: v and C enter the substep only through P2G), and the payload of the
// node-velocity adjoint w (vbt + Bb q).
//
// Separable form of the stencil sums.  Per node only wb = V . g(a)
// (g(a) = vbar_t + Bbar (a - f), linear in the node offset a) and the
// weighted node velocity are formed; the sums then run over the third axis,
// the second and the first:
//   B[i][j] = sum w V_i a_j - f_j S_i,  fxb[k] = sum (dw/dx_k) wb - (Bbar^T S)_k,
//   S = sum w V.
template <class VTile, class VGlobal>
__device__ __forceinline__ void adj_g2p_particle(const Dev &d, const EnvDev &e, const Stencil &s, const float H[9],
                                                 float xb[3], float vb[3], float Cb[9], float Fb[9], bool in_tile,
                                                 VTile vtile, VGlobal vglobal, float vbt[3], float Bb[9])
{
    float dw[3][3];
    weight_grads(s, dw);
    // the particle's adjoint state first: Bbar and vbar_t do not depend on the
    // recomputed C, so one pass over the stencil serves C and the x adjoint
    const float cs = 4.0f * e.inv_dx;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float cbt = Cb[3 * r + c] + d.dt * (Fb[3 * r + c] + Fb[3 * r] * H[3 * c] + Fb[3 * r + 1] * H[3 * c + 1] +
                                                      Fb[3 * r + 2] * H[3 * c + 2]);
            Bb[3 * r + c] = cs * cbt;
        }
#pragma unroll
    for (int i = 0; i < 3; ++i) vbt[i] = vb[i] + d.dt * xb[i];
    float gf[3];   // vbar_t - Bbar f
#pragma unroll
    for (int i = 0; i < 3; ++i)
        gf[i] = vbt[i] - (Bb[3 * i] * s.fx[0] + Bb[3 * i + 1] * s.fx[1] + Bb[3 * i + 2] * s.fx[2]);
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;   // sum of (dw/dx_k) wb
    float S[3] = {0.f, 0.f, 0.f}, Mo[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    auto sums = [&](auto Vat) {
#pragma unroll
    for (int a0 = 0; a0 < 3; ++a0) {
        float X1 = 0.f, X1d = 0.f, Y1 = 0.f;
        float E1[3] = {0.f, 0.f, 0.f}, E2[3] = {0.f, 0.f, 0.f}, E3[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a1 = 0; a1 < 3; ++a1) {
            float X = 0.f, Y = 0.f, AV[3] = {0.f, 0.f, 0.f}, BV[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int a2 = 0; a2 < 3; ++a2) {
                const float4 V4 = Vat(a0, a1, a2);
                const float V[3] = {V4.x, V4.y, V4.z};
                const float w2 = s.w[2][a2];
                float wb = 0.f;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    wb = fmaf(V[i], gf[i] + Bb[3 * i] * a0 + Bb[3 * i + 1] * a1 + Bb[3 * i + 2] * a2, wb);
                X = fmaf(w2, wb, X);
                Y = fmaf(dw[2][a2], wb, Y);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    AV[i] = fmaf(w2, V[i], AV[i]);
                    BV[i] = fmaf(w2 * a2, V[i], BV[i]);
                }
            }
            const float w1 = s.w[1][a1], d1 = dw[1][a1];
            X1 = fmaf(w1, X, X1);
            X1d = fmaf(d1, X, X1d);
            Y1 = fmaf(w1, Y, Y1);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                E1[i] = fmaf(w1, AV[i], E1[i]);
                E2[i] = fmaf(w1 * a1, AV[i], E2[i]);
                E3[i] = fmaf(w1, BV[i], E3[i]);
            }
        }
        const float w0 = s.w[0][a0], d0 = dw[0][a0];
        g0 = fmaf(d0, X1, g0);
        g1 = fmaf(w0, X1d, g1);
        g2 = fmaf(w0, Y1, g2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            S[i] = fmaf(w0, E1[i], S[i]);
            Mo[i][0] = fmaf(w0 * a0, E1[i], Mo[i][0]);
            Mo[i][1] = fmaf(w0, E2[i], Mo[i][1]);
            Mo[i][2] = fmaf(w0, E3[i], Mo[i][2]);
        }
    }
    };
    if (in_tile) sums(vtile); else sums(vglobal);
    float B[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B[3 * i + j] = Mo[i][j] - s.fx[j] * S[i];
    const float fxb[3] = {g0 - (Bb[0] * S[0] + Bb[3] * S[1] + Bb[6] * S[2]),
                          g1 - (Bb[1] * S[0] + Bb[4] * S[1] + Bb[7] * S[2]),
                          g2 - (Bb[2] * S[0] + Bb[5] * S[1] + Bb[8] * S[2])};
    // F' = (I + dt C') F with C' = cs B:  Fbar <- (I + dt C')^T Fbar'
    float Fbn[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Fbn[3 * r + c] = Fb[3 * r + c] + d.dt * cs * (B[r] * Fb[c] + B[3 + r] * Fb[3 + c] + B[6 + r] * Fb[6 + c]);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        Fb[c] = Fbn[c];
        Cb[c] = 0.0f;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xb[c] += e.inv_dx * fxb[c];
        vb[c] = 0.0f;
    }
}

// Reverse of P2G and of the stress for one particle whose stencil s lies in
// the grid (state v, C, H; node adjoints (m, mv)bar through Pat(a0, a1, a2)).
// Adds its terms to the adjoints xb, vb, Cb, Fb of the state before the
// substep and returns the particle's dL/dmu, dL/dlambda terms.
//
// Separable form of the stencil sums.  Per node only the momentum weight
// wb = m pm + q . c(a) (c(a) = m v + A (a - f) dx, the affine momentum at
// node offset a) and the node's weighted values are formed; the sums then run
// over the third axis, the second and the first:
//   vbp = m S,  Ab[i][j] = dx (sum w q_i a_j - f_j S_i),
//   fxb[k] = sum (dw/dx_k) wb - dx (A^T S)_k,  S = sum w q.
template <class PTile, class PGlobal>
__device__ __forceinline__ void adj_p2g_particle(const Dev &d, const EnvDev &e, const Stencil &s, const float H[9],
                                                 const float C[9], const float v[3], float mu, float lamda, float m,
                                                 float kf, bool in_tile, PTile ptile, PGlobal pglobal, float xb[3],
                                                 float vb[3], float Cb[9], float Fb[9], double &mub, double &lamb)
{
    float F[9], tau[9], A[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) F[c] = H[c] + ((c & 3) == 0 ? 1.0f : 0.0f);
    // the forward's FP32 stress (same formulas, same inversion decision)
    const float jm1 = jm1_f(H);
    const bool inverted = inverted_f(H, jm1);
    kirchhoff_f(H, jm1, inverted, mu, lamda, tau);
#pragma unroll
    for (int c = 0; c < 9; ++c) A[c] = kf * tau[c] + m * C[c];
    float dw[3][3];
    weight_grads(s, dw);
    const float dx = e.dx;
    float lam[3][3], cf[3];   // lam[j][i] = dx A[i][j]; cf = m v - dx A f
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) lam[j][i] = dx * A[3 * i + j];
        cf[i] = m * v[i] - (lam[0][i] * s.fx[0] + lam[1][i] * s.fx[1] + lam[2][i] * s.fx[2]);
    }
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;   // sum of (dw/dx_k) wb
    float S[3] = {0.f, 0.f, 0.f}, Mo[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    auto sums = [&](auto Pat) {
#pragma unroll
    for (int a0 = 0; a0 < 3; ++a0) {
        float X1 = 0.f, X1d = 0.f, Y1 = 0.f;
        float E1[3] = {0.f, 0.f, 0.f}, E2[3] = {0.f, 0.f, 0.f}, E3[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a1 = 0; a1 < 3; ++a1) {
            float X = 0.f, Y = 0.f, AQ[3] = {0.f, 0.f, 0.f}, BQ[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int a2 = 0; a2 < 3; ++a2) {
                const float4 Pb = Pat(a0, a1, a2);
                const float q[3] = {Pb.y, Pb.z, Pb.w};
                const float w2 = s.w[2][a2];
                float wb = m * Pb.x;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    wb = fmaf(q[i], cf[i] + lam[0][i] * a0 + lam[1][i] * a1 + lam[2][i] * a2, wb);
                X = fmaf(w2, wb, X);
                Y = fmaf(dw[2][a2], wb, Y);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    AQ[i] = fmaf(w2, q[i], AQ[i]);
                    BQ[i] = fmaf(w2 * a2, q[i], BQ[i]);
                }
            }
            const float w1 = s.w[1][a1], d1 = dw[1][a1];
            X1 = fmaf(w1, X, X1);
            X1d = fmaf(d1, X, X1d);
            Y1 = fmaf(w1, Y, Y1);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                E1[i] = fmaf(w1, AQ[i], E1[i]);
                E2[i] = fmaf(w1 * a1, AQ[i], E2[i]);
                E3[i] = fmaf(w1, BQ[i], E3[i]);
            }
        }
        const float w0 = s.w[0][a0], d0 = dw[0][a0];
        g0 = fmaf(d0, X1, g0);
        g1 = fmaf(w0, X1d, g1);
        g2 = fmaf(w0, Y1, g2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            S[i] = fmaf(w0, E1[i], S[i]);
            Mo[i][0] = fmaf(w0 * a0, E1[i], Mo[i][0]);
            Mo[i][1] = fmaf(w0, E2[i], Mo[i][1]);
            Mo[i][2] = fmaf(w0, E3[i], Mo[i][2]);
        }
    }
    };
    if (in_tile) sums(ptile); else sums(pglobal);
    float Ab[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        vb[i] += m * S[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) Ab[3 * i + j] = dx * (Mo[i][j] - s.fx[j] * S[i]);
    }
    const float fxb[3] = {g0 - dx * (A[0] * S[0] + A[3] * S[1] + A[6] * S[2]),
                          g1 - dx * (A[1] * S[0] + A[4] * S[1] + A[7] * S[2]),
                          g2 - dx * (A[2] * S[0] + A[5] * S[1] + A[8] * S[2])};
#pragma unroll
    for (int c = 0; c < 3; ++c) xb[c] += e.inv_dx * fxb[c];
    float taub[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        Cb[c] += m * Ab[c];
        taub[c] = kf * Ab[c];
    }
    // tau-bar -> F-bar: mu (tau-bar + tau-bar^T) F + lam tr(tau-bar) cof(F) / J
    float Fs[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Fs[3 * r + c] = mu * ((taub[3 * r] + taub[r]) * F[c] + (taub[3 * r + 1] + taub[3 + r]) * F[3 + c] +
                                  (taub[3 * r + 2] + taub[6 + r]) * F[6 + c]);
    const float trt = taub[0] + taub[4] + taub[8];
    const float lnJ = inverted ? -13.815510557964274f : log1pf(jm1);
    if (!inverted) {
        const float ci[9] = {F[4] * F[8] - F[5] * F[7], -(F[3] * F[8] - F[5] * F[6]), F[3] * F[7] - F[4] * F[6],
                             -(F[1] * F[8] - F[2] * F[7]), F[0] * F[8] - F[2] * F[6], -(F[0] * F[7] - F[1] * F[6]),
                             F[1] * F[5] - F[2] * F[4], -(F[0] * F[5] - F[2] * F[3]), F[0] * F[4] - F[1] * F[3]};
        const float sc = lamda * trt / (1.0f + jm1);
#pragma unroll
        for (int c = 0; c < 9; ++c) Fs[c] = fmaf(sc, ci[c], Fs[c]);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) Fb[c] += Fs[c];
    // dL/dmu and dL/dlam of this particle (summed per environment in FP64)
    float ff = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float G = H[3 * r + c] + H[3 * c + r] + H[3 * r] * H[3 * c] + H[3 * r + 1] * H[3 * c + 1] +
                            H[3 * r + 2] * H[3 * c + 2];
            ff = fmaf(taub[3 * r + c], G, ff);
        }
    mub = ff;
    lamb = (double)trt * lnJ;
}

// Adjoint state of particle slot q: load and store of xb, vb, Cb, Fb.
__device__ __forceinline__ void load_adj(const AdjBuf &a, int N, uint32_t q, float xb[3], float vb[3], float Cb[9],
                                         float Fb[9])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xb[c] = gload(a.xb + (size_t)c * N + q);
        vb[c] = gload(a.vb + (size_t)c * N + q);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        Cb[c] = gload(a.Cb + (size_t)c * N + q);
        Fb[c] = gload(a.Fb + (size_t)c * N + q);
    }
}

__device__ __forceinline__ void store_adj(const AdjBuf &a, int N, uint32_t q, const float xb[3], const float vb[3],
                                          const float Cb[9], const float Fb[9])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        gstore(a.xb + (size_t)c * N + q, xb[c]);
        gstore(a.vb + (size_t)c * N + q, vb[c]);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        gstore(a.Cb + (size_t)c * N + q, Cb[c]);
        gstore(a.Fb + (size_t)c * N + q, Fb[c]);
    }
}

// Shared memory of the tiled reverse kernels: node velocities (G2P reverse),
// node adjoints (m, mv)bar (P2G reverse), per-half-wave tiles of the
// node-velocity adjoint and the node pass's payloads.
template <int W, bool PB, bool GV>
struct AdjShared {
    float4 tb[PB ? TILE_NODES : 1];
    float4 tv[GV ? TILE_NODES : 1];
    float4 tp[GV ? 2 * W * TILE_NODES : 1];
    Payload pay[GV ? 64 * W : 1];
    float2 wz[1];   // the plain payload form has no side array
};

// Material of the tile's environment: mu, lambda, particle mass, stress factor.
__device__ __forceinline__ void adj_material(const Dev &d, const EnvDev &e, int env, float &mu, float &lam, float &m,
                                             float &kf)
{
    const float *mat = d.material + 4 * env;
    const float E = uload(mat), nu = uload(mat + 1), rho = uload(mat + 2), V0 = uload(mat + 3);
    lame(E, nu, mu, lam);
    m = rho * V0;
    kf = -d.dt * V0 * 4.0f * e.inv_dx * e.inv_dx;
}

// The tiled reverse pass over one item's particles.  PB: reverse of P2G of
// substep j (state dp = slot j, node adjoints a.gPb); GV: then reverse of G2P
// of the substep before, j - 1 with PB (state dg = slot j - 1, node velocities
// dg.gV), scattering its node-velocity adjoint into a.gVb.  PB alone is the
// reverse P2G of one substep, GV alone its reverse G2P; both at once walk two
// reverse stages with one load and store of the particle adjoints.
template <int W, bool PB, bool GV>
__device__ __forceinline__ void adj_tiled_body(const Dev &dp, const Dev &dg, const AdjBuf &a, const AdjTiledArgs &ta,
                                               AdjShared<W, PB, GV> &sh)
{
    constexpr int T = 64 * W;
    const Dev &d = GV ? dg : dp;   // environment tables (shared by both)
    const int N = d.ntot, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int hw = 2 * wave + (lane >> 5);
    const int nitems = uload(ta.totals).y;
    int first, stride, end;
    item_range(nitems, first, stride, end);
    int4 next = first < end ? uload(ta.items + first) : make_int4(0, 0, 0, 0);
    for (int it = first; it < end; it += stride) {
        const int4 item = next;   // loaded one iteration ahead
        if (it + stride < end) next = uload(ta.items + it + stride);
        const int item_end = item.y + item.z;
        EnvDev e;
        const Tile t = make_tile(d, item, e);
        for (int n = tid; n < TILE_NODES; n += T) {
            const int i = t.o[0] + n / 36, j = t.o[1] + (n / 6) % 6, k = t.o[2] + n % 6;
            const bool in = i < e.n && j < e.n && k < e.n;
            if (PB) sh.tb[n] = in ? gload(a.gPb + node_id(e, i, j, k)) : make_float4(0.f, 0.f, 0.f, 0.f);
            if (GV) {
                for (int w = 0; w < 2 * W; ++w) sh.tp[w * TILE_NODES + n] = make_float4(0.f, 0.f, 0.f, 0.f);
                sh.tv[n] = in ? gload(dg.gV + node_id(e, i, j, k)) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        __syncthreads();
        float mu = 0.f, lam = 0.f, m = 0.f, kf = 0.f;
        if (PB) adj_material(d, e, t.env, mu, lam, m, kf);
        for (int chunk = item.y; chunk < item_end; chunk += T) {
            const int q = chunk + tid;
            const bool active = q < item_end;
            const uint32_t uq = (uint32_t)q;
            double mub = 0.0, lamb = 0.0;
            int key = KEY_NONE;
            if (active) {
                // reverse P2G terms first, into zeroed sums; the particle's adjoint
                // state is loaded after them, so it is not held across the stencil sums.
                // The recorded states of both substeps are loaded up front, together
                float xb[3] = {0.f, 0.f, 0.f}, vb[3] = {0.f, 0.f, 0.f};
                float Cb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float Fb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float px[3], pH[9], pC[9], pv[3], gx[3], gH[9];
                if (PB) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) px[c] = gload(dp.x + (size_t)c * N + uq);
#pragma unroll
                    for (int c = 0; c < 9; ++c) {
                        pH[c] = gload(dp.H + (size_t)c * N + uq);
                        pC[c] = gload(dp.C + (size_t)c * N + uq);
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) pv[c] = gload(dp.v + (size_t)c * N + uq);
                }
                if (GV) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) gx[c] = gload(dg.x + (size_t)c * N + uq);
#pragma unroll
                    for (int c = 0; c < 9; ++c) gH[c] = gload(dg.H + (size_t)c * N + uq);
                }
                if (PB) {
                    Stencil s;
                    make_stencil(px[0], px[1], px[2], e.inv_dx, e.n, s);
                    if (!s.outside) {
                        float H[9], C[9], v[3];
#pragma unroll
                        for (int c = 0; c < 9; ++c) {
                            H[c] = pH[c];
                            C[c] = pC[c];
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) v[c] = pv[c];
                        int l0, l1, l2;
                        const bool in_tile = stencil_in_tile(t, s, l0, l1, l2);
                        adj_p2g_particle(
                            dp, e, s, H, C, v, mu, lam, m, kf, in_tile,
                            [&](int a0, int a1, int a2) { return sh.tb[((l0 + a0) * TILE + l1 + a1) * TILE + l2 + a2]; },
                            [&](int a0, int a1, int a2) {
                                return gload(a.gPb + node_id(e, s.b[0] + a0, s.b[1] + a1, s.b[2] + a2));
                            },
                            xb, vb, Cb, Fb, mub, lamb);
                    }
                }
                {
                    float axb[3], avb[3], aCb[9], aFb[9];
                    load_adj(a, N, uq, axb, avb, aCb, aFb);
#pragma unroll
                    for (int c = 0; c < 3; ++c) { xb[c] += axb[c]; vb[c] += avb[c]; }
#pragma unroll
                    for (int c = 0; c < 9; ++c) { Cb[c] += aCb[c]; Fb[c] += aFb[c]; }
                }
                if (GV) {
                    Stencil s;
                    make_stencil(gx[0], gx[1], gx[2], e.inv_dx, e.n, s);
                    if (!s.outside) {   // a frozen particle's adjoints pass through
                        float H[9];
#pragma unroll
                        for (int c = 0; c < 9; ++c) H[c] = gH[c];
                        int l0, l1, l2;
                        const bool in_tile = stencil_in_tile(t, s, l0, l1, l2);
                        float vbt[3], Bb[9];
                        adj_g2p_particle(
                            dg, e, s, H, xb, vb, Cb, Fb, in_tile,
                            [&](int a0, int a1, int a2) { return sh.tv[((l0 + a0) * TILE + l1 + a1) * TILE + l2 + a2]; },
                            [&](int a0, int a1, int a2) {
                                return gload(dg.gV + node_id(e, s.b[0] + a0, s.b[1] + a1, s.b[2] + a2));
                            },
                            vbt, Bb);
                        // node contributions w (vbar_t + Bbar q): the form of P2G's w (m v + A q),
                        // in the plain payload form: the pair kernel then fits two wavefronts per
                        // SIMD without a register cap (capped, with the forward's form, it ran 10%
                        // longer)
                        key = in_tile ? key_in_tile(l0, l1, l2) : key_global(s.b);
                        store_payload<false>(sh.pay[tid], sh.wz[tid], s.fx, s.w[2], key, vbt, Bb);
                    }
                }
                store_adj(a, N, uq, xb, vb, Cb, Fb);
            }
            if (PB) {
                // every particle of an item belongs to the tile's environment
                wave_env_add(a.mubar, t.env, mub, active);
                wave_env_add(a.lambar, t.env, lamb, active);
            }
            if (GV) {
                if (key == KEY_NONE) payload_none(sh.pay[tid]);
                __syncthreads();
                int r0, r1;
                half_wave_run<W>(hw, min(T, item_end - chunk), r0, r1);
                // .x sums the weights (the flush skips nodes no particle reached)
                node_pass<false>(ta.slots, sh.pay, sh.wz, r0, r1, sh.tp + hw * TILE_NODES, lane, 1.0f,
                          [&](const float4 &c4, int i, int j, int k) {
                              float *g = reinterpret_cast<float *>(a.gVb + node_id(e, i, j, k));
                              gatomic_add(g + 0, c4.y);
                              gatomic_add(g + 1, c4.z);
                              gatomic_add(g + 2, c4.w);
                          });
                __syncthreads();
            }
        }
        if (GV) {
            // a node's 2W tile entries are read together, whole
            for (int n = tid; n < TILE_NODES; n += T) {
                float4 q4[2 * W];
#pragma unroll
                for (int w = 0; w < 2 * W; ++w) q4[w] = sh.tp[w * TILE_NODES + n];
                float4 sum = q4[0];
#pragma unroll
                for (int w = 1; w < 2 * W; ++w) {
                    sum.x += q4[w].x; sum.y += q4[w].y; sum.z += q4[w].z; sum.w += q4[w].w;
                }
                // keeps the adjoint sums from being sunk under the weight test
                asm volatile("" : "+v"(sum.x), "+v"(sum.y), "+v"(sum.z), "+v"(sum.w));
                if (sum.x != 0.f) {
                    const int i = t.o[0] + n / 36, j = t.o[1] + (n / 6) % 6, k = t.o[2] + n % 6;
                    float *g = reinterpret_cast<float *>(a.gVb + node_id(e, i, j, k));
                    gatomic_add(g + 0, sum.y);
                    gatomic_add(g + 1, sum.z);
                    gatomic_add(g + 2, sum.w);
                }
            }
        }
        __syncthreads();
    }
}

// Reverse of G2P + advection + F update (pass 1, lane = particle: C' from
// the tape's node velocities in an LDS tile, the particle adjoints and the
// weight-gradient terms; pass 2, lane = stencil node: w (vbar_t + Bbar q)
// into per-half-wave tiles, flushed to the node-velocity adjoint with one
// float atomic per component).
template <int W>
__global__ __launch_bounds__(64 * W) void k_adj_g2p_tiled(Dev d, AdjBuf a, AdjTiledArgs ta)
{
    __shared__ AdjShared<W, false, true> sh;
    adj_tiled_body<W, false, true>(d, d, a, ta, sh);
}

// Reverse of P2G and of the stress, gathering the node adjoints (m, mv)bar
// of the item's tile from LDS.
template <int W>
__global__ __launch_bounds__(64 * W) void k_adj_p2g_tiled(Dev d, AdjBuf a, AdjTiledArgs ta)
{
    __shared__ AdjShared<W, true, false> sh;
    adj_tiled_body<W, true, false>(d, d, a, ta, sh);
}

// Reverse P2G of substep j (dp: slot j) and reverse G2P of substep j - 1
// (dg: slot j - 1) in one pass over the particles.
template <int W>
__global__ __launch_bounds__(64 * W) void k_adj_pair_tiled(Dev dp, Dev dg, AdjBuf a, AdjTiledArgs ta)
{
    __shared__ AdjShared<W, true, true> sh;
    adj_tiled_body<W, true, true>(dp, dg, a, ta, sh);
}


// dst[c][q] = src[c][perm[q]] (gather into slot order) or the reverse scatter.
__global__ void k_permute(const float *src, const int32_t *perm, int ntot, int comps, float *dst, int scatter)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ntot) return;
    int o = gload(perm + q);
    if (scatter) move_components(src, q, dst, o, ntot, comps);
    else move_components(src, o, dst, q, ntot, comps);
}

static unsigned blocks_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

// enough workgroups for a node per thread up to 2M nodes, grid-stride beyond
static unsigned tape_blocks(int64_t total_nodes)
{
    const int64_t b = (total_nodes + 255) / 256;
    return (unsigned)(b < 8 ? 8 : (b > 8192 ? 8192 : b));
}

void launch_grid_tape(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, ContactCode *dec, ToolDev *snap,
                      int slots, const TapeList &tl, hipStream_t st)
{
    launch_k(k_grid_tape, dim3(tape_blocks(total_nodes)), dim3(256), 0, st, d, env_gofs, total_nodes, dec, snap, slots,
             tl);
}

void launch_adj_g2p(const Dev &d, const AdjBuf &a, hipStream_t st)
{
    launch_k(k_adj_g2p, dim3((d.ntot + 255) / 256), dim3(256), 0, st, d, a);
}

__global__ __launch_bounds__(256) void k_tape_clear(Dev d, const int64_t *env_gofs, int64_t total_nodes, TapeList tl)
{
    tape_nodes<false>(d, env_gofs, total_nodes, tl, nullptr,
                      [&](int, const EnvDev &, const ToolDev *, int64_t g, int64_t) {
                          gstore(d.gP + g, make_float4(0.f, 0.f, 0.f, 0.f));
                      });
}

void launch_tape_clear(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, const TapeList &tl,
                       hipStream_t st)
{
    launch_k(k_tape_clear, dim3(tape_blocks(total_nodes)), dim3(256), 0, st, d, env_gofs, total_nodes, tl);
}

void launch_adj_grid(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, const ContactCode *dec,
                     const AdjBuf &a, const TapeList &tl, hipStream_t st)
{
    launch_k(k_adj_grid, dim3(tape_blocks(total_nodes)), dim3(256), 0, st, d, env_gofs, total_nodes, dec, a, tl);
}

void launch_adj_p2g(const Dev &d, const AdjBuf &a, hipStream_t st)
{
    launch_k(k_adj_p2g, dim3((d.ntot + 255) / 256), dim3(256), 0, st, d, a);
}

void launch_adj_finish(const Dev &d, const AdjBuf &a, int n, double *gE, double *gnu, double *gu, double *gT,
                       hipStream_t st)
{
    int nt = d.n_envs * (d.max_tools > 0 ? d.max_tools : 1);
    launch_k(k_adj_finish, dim3((nt + 255) / 256), dim3(256), 0, st, d, a, n, gE, gnu, gu, gT);
}

void launch_adj_g2p_tiled(const Dev &d, const AdjBuf &a, const int4 *items, const int2 *totals, int slots,
                          const ActiveBuf &act, int block, int nblocks, hipStream_t st)
{
    AdjTiledArgs ta{items, totals, slots, act};
    if (block == 64) launch_k((k_adj_g2p_tiled<1>), dim3(nblocks), dim3(64), 0, st, d, a, ta);
    else if (block == 128) launch_k((k_adj_g2p_tiled<2>), dim3(nblocks), dim3(128), 0, st, d, a, ta);
    else launch_k((k_adj_g2p_tiled<4>), dim3(nblocks), dim3(256), 0, st, d, a, ta);
}

void launch_adj_p2g_tiled(const Dev &d, const AdjBuf &a, const int4 *items, const int2 *totals,
                          const ActiveBuf &act, int block, int nblocks, hipStream_t st)
{
    AdjTiledArgs ta{items, totals, 1, act};
    if (block == 64) launch_k((k_adj_p2g_tiled<1>), dim3(nblocks), dim3(64), 0, st, d, a, ta);
    else if (block == 128) launch_k((k_adj_p2g_tiled<2>), dim3(nblocks), dim3(128), 0, st, d, a, ta);
    else launch_k((k_adj_p2g_tiled<4>), dim3(nblocks), dim3(256), 0, st, d, a, ta);
}

void launch_adj_pair_tiled(const Dev &dp, const Dev &dg, const AdjBuf &a, const int4 *items, const int2 *totals,
                           int slots, const ActiveBuf &act, int block, int nblocks, hipStream_t st)
{
    AdjTiledArgs ta{items, totals, slots, act};
    if (block == 64) launch_k((k_adj_pair_tiled<1>), dim3(nblocks), dim3(64), 0, st, dp, dg, a, ta);
    else if (block == 128) launch_k((k_adj_pair_tiled<2>), dim3(nblocks), dim3(128), 0, st, dp, dg, a, ta);
    else launch_k((k_adj_pair_tiled<4>), dim3(nblocks), dim3(256), 0, st, dp, dg, a, ta);
}

void launch_permute(const float *src, const int32_t *perm, int ntot, int comps, float *dst, int scatter,
                    hipStream_t st)
{
    launch_k(k_permute, dim3((ntot + 255) / 256), dim3(256), 0, st, src, perm, ntot, comps, dst, scatter);
}

void launch_unpermute(const float *src, const int32_t *pid, int ntot, int comps, float *dst, hipStream_t st)
{
    launch_k(k_unpermute, dim3((ntot + 255) / 256), dim3(256), 0, st, src, pid, ntot, comps, dst);
}

void launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    size_t n = bytes / 4;
    launch_k(k_copy_words, dim3(blocks_for((int64_t)n)), dim3(256), 0, st, static_cast<uint32_t *>(dst),
                       static_cast<const uint32_t *>(src), n);
}

void launch_copies(std::initializer_list<CopySpec> jobs, hipStream_t st)
{
    if (jobs.size() == 0 || jobs.size() > (size_t)COPY_JOBS) throw std::logic_error("launch_copies: 1 to 4 jobs");
    CopyJobs j{};
    size_t most = 0;
    int q = 0;
    for (const CopySpec &c : jobs) {
        j.dst[q] = static_cast<uint32_t *>(c.dst);
        j.src[q] = static_cast<const uint32_t *>(c.src);
        j.words[q] = c.bytes / 4;
        most = j.words[q] > most ? j.words[q] : most;
        ++q;
    }
    launch_k(k_copy_jobs, dim3(blocks_for((int64_t)most), q), dim3(256), 0, st, j);
}

void launch_fill_f64(double *p, int64_t n, hipStream_t st)
{
    launch_k(k_fill_f64, dim3(blocks_for(n)), dim3(256), 0, st, p, n);
}

}  // namespace mpm
