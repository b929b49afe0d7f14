// Tiled scheme kernels.
//
// Particles are sorted by the cell of their stencil base, brick-major; a work
// item is (brick, slot range, environment).  For each item a workgroup stages
// the 6^3 nodes the brick's stencils reach in LDS:
//   - G2P reads node velocities from the tile,
//   - P2G accumulates mass/momentum into per-half-wave tiles and flushes each
//     non-empty tile node to the global grid with one float atomic per
//     component,
// so global atomics scale with tile nodes, not with particles x 27.  A
// particle whose stencil has drifted out of its sort-time brick uses global
// memory directly (rare between sorts; correct either way).
//
// Workgroups are persistent over the item list; workgroup w runs on XCD
// w % 8 and walks a contiguous eighth of the (spatially ordered) items, so
// neighbouring tiles, which share halo nodes, stay in one XCD's L2.
#include <algorithm>

#include "mpm_tile_util.h"

namespace mpm {

__device__ __forceinline__ void advance_end_of_substep(const Dev &d)
{
    if (blockIdx.x != 0) return;
    for (int t = threadIdx.x; t < d.n_envs; t += blockDim.x) d.step[t] += 1;
    for (int t = threadIdx.x; t < d.n_envs * d.max_tools; t += blockDim.x) {
        ToolDev &T = d.tools[t];
        if (T.active) {
            advance_tool(T, d.dt);
        }
    }
}

// G2P of one particle whose stencil is outside the item's tile (drift since
// the sort): velocity and C = (4/dx) sum w v (o - fx)^T from global memory.
template <bool COH>
__device__ __forceinline__ void g2p_global(const Dev &d, const EnvDev &e, const Stencil &s, float vp[3], float Cn[9])
{
    float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    vp[0] = vp[1] = vp[2] = 0.f;
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                const float4 *q = d.gV + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2);
                const float4 V = COH ? cload(q) : gload(q);
                const float d0 = o0 - s.fx[0], d1 = o1 - s.fx[1], d2 = o2 - s.fx[2];
                const float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                const float wx = w * V.x, wy = w * V.y, wz = w * V.z;
                vp[0] += wx; vp[1] += wy; vp[2] += wz;
                B[0] += wx * d0; B[1] += wx * d1; B[2] += wx * d2;
                B[3] += wy * d0; B[4] += wy * d1; B[5] += wy * d2;
                B[6] += wz * d0; B[7] += wz * d1; B[8] += wz * d2;
            }
    const float cs = 4.0f * e.inv_dx;
#pragma unroll
    for (int c = 0; c < 9; ++c) Cn[c] = cs * B[c];
}

// Component c of a [comp][N] particle array: a uniform base pointer, so a
// particle access is that base plus a 32-bit lane offset (one address form,
// no per-lane 64-bit arithmetic).
template <class T>
__device__ __forceinline__ T *comp(T *base, int c, int N) { return base + (size_t)c * N; }

// A = -dt V0 (4/dx^2) tau(F) + m C (the MLS force folded into the affine term).
__device__ __forceinline__ void affine_stress_f(const Dev &d, const EnvDev &e, const float H[9], float jm1,
                                                bool inv, const float C[9], float mu, float lam, float m, float V0,
                                                float A[9])
{
    float tau[9];
    kirchhoff_f(H, jm1, inv, mu, lam, tau);
    const float k = -d.dt * V0 * 4.0f * e.inv_dx * e.inv_dx;
#pragma unroll
    for (int c = 0; c < 9; ++c) A[c] = fmaf(m, C[c], k * tau[c]);
}

// MODE 0: P2G only (head of a call; reads x, v, C, H).
// MODE 1: fused G2P(s) + F update + advection + P2G(s+1) (reads/writes x, H).
// MODE 2: G2P only (tail of a call; writes x, v, C, H).
// MODE 3: as MODE 1, also writing v and C (tape recompute: every substep's
//         full state is kept).
//
// W wavefronts per workgroup.  Pass 1 (lane = particle): G2P from the LDS
// velocity tile, F update, advection, stress and the P2G payload.  Pass 2
// (lane = stencil node): the chunk's payloads are split into 2W contiguous
// runs, one per half-wave; lanes 0-26 of a half-wave take one particle's 27
// nodes per step, sum the contributions of consecutive particles with the
// same stencil (the sort groups particles by cell) in registers, and add
// each sum to the half-wave's own LDS tile with plain read-modify-write
// (27 lanes, 27 distinct nodes).  LDS float atomics run at about 1/3 lane
// per clock per CU on this chip, far below plain LDS traffic.  The 2W tiles
// are summed and flushed to the global grid with one float atomic per
// component per non-empty node.
template <int W, bool GAS = false, bool P2G = true>
struct TiledShared {
    float4 tv[GAS ? GTILE_NODES : TILE_NODES];   // node velocities (GAS: the 8^3 tile)
    float4 tp[P2G ? 2 * W * TILE_NODES : 1];     // per-half-wave (m, mv) tiles
    Payload pay[P2G ? 64 * W : 1];
    float2 wz[P2G ? 64 * W : 1];                 // the payloads' side array
    ToolDev tl[GAS ? MAX_TOOLS : 1];             // GAS: the item environment's tools at this substep
};

// Grid operation at staging: the momentum buffer of two substeps ago is
// zeroed over the static brick list (one wavefront per brick), or over the
// whole grid after a sort or a P2G that reached a far brick.  The loads that
// decide it are issued at kernel start (gas_clear_issue) and the stores made
// once the first tile is staged (gas_clear_finish), so their latency overlaps
// the item's own loads.
struct GasClear {
    int stamp;   // far_stamp[clear_slot]
    int ns;      // static list length
    int sl;      // this wavefront's first listed brick
};

template <int T>
__device__ __forceinline__ GasClear gas_clear_issue(const TiledArgs &a)
{
    GasClear c;
    c.stamp = uload(a.far_stamp + a.clear_slot);
    c.ns = uload(a.act.scount);
    const int i0 = blockIdx.x * (T >> 6) + (threadIdx.x >> 6);
    c.sl = i0 < a.act.nbricks ? uload(a.act.slist + i0) : 0;
    return c;
}

// COH: device-coherent stores (workgroups of the same launch add to the buffer later).
template <int T, bool COH = false>
__device__ __forceinline__ void gas_clear_finish(const TiledArgs &a, const GasClear &c)
{
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    auto put = [&](float4 *q) {
        if (COH) cstore(q, zero);
        else gstore(q, zero);
    };
    if (a.full_clear || c.stamp == a.clear_stamp) {
        const int64_t stride = (int64_t)gridDim.x * T;
        for (int64_t g = (int64_t)blockIdx.x * T + threadIdx.x; g < a.total_nodes; g += stride) put(a.gP_clear + g);
        return;
    }
    const int nw = T >> 6, i0 = blockIdx.x * nw + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int i = i0; i < c.ns; i += gridDim.x * nw)
        put(a.gP_clear + (int64_t)(i == i0 ? c.sl : gload(a.act.slist + i)) * BRICK_NODES + lane);
}

// Tool poses of the grid-at-staging kernels, written by one workgroup at its
// start (nothing in the launch reads what it writes: the kernels take T and k
// from a.pose_in).  Head (MODE 0): this call's first poses from the tool table.
// Otherwise the next substep's poses (T <- T + dt u, as advance_tool) and the
// step counters; the tail of a call also writes the poses back into the table.
template <int MODE, int T>
__device__ __forceinline__ void gas_poses(const Dev &d, const TiledArgs &a)
{
    const int nt = d.n_envs * d.max_tools;
    if (MODE == 0) {
        for (int q = threadIdx.x; q < nt; q += T) {
            const ToolDev &Tq = d.tools[q];
            a.pose_out[q] = ToolPose{{Tq.T[0], Tq.T[1], Tq.T[2]}, Tq.k, 0};
        }
        return;
    }
    for (int t = threadIdx.x; t < d.n_envs; t += T) d.step[t] += 1;
    for (int t = threadIdx.x; t < nt; t += T) {
        ToolDev Tt = d.tools[t];
        const ToolPose q = a.pose_in[t];
        Tt.T[0] = q.T[0]; Tt.T[1] = q.T[1]; Tt.T[2] = q.T[2];
        Tt.k = q.k;
        if (Tt.active) advance_tool(Tt, d.dt);
        a.pose_out[t] = ToolPose{{Tt.T[0], Tt.T[1], Tt.T[2]}, Tt.k, 0};
        if (MODE == 2) {
            d.tools[t].T[0] = Tt.T[0]; d.tools[t].T[1] = Tt.T[1]; d.tools[t].T[2] = Tt.T[2];
            d.tools[t].k = Tt.k;
        }
    }
}

// Word w of environment env's tool slots as the grid-at-staging kernels see
// them: the pose fields (T, k) from the substep's pose table, the rest from the
// tool table.
__device__ __forceinline__ const int *tool_word(const Dev &d, const ToolPose *pose, int env, int w)
{
    constexpr int WPT = (int)(sizeof(ToolDev) / 4);
    constexpr int KW = (int)(offsetof(ToolDev, k) / 4), TW = (int)(offsetof(ToolDev, T) / 4);
    const int slot = w / WPT, off = w - slot * WPT;
    const size_t s = (size_t)env * d.max_tools + slot;
    const int *pw = reinterpret_cast<const int *>(pose + s);
    if (off == KW) return pw + offsetof(ToolPose, k) / 4;
    if (off >= TW && off < TW + 6) return pw + offsetof(ToolPose, T) / 4 + (off - TW);
    return reinterpret_cast<const int *>(d.tools + s) + off;
}

// G2P of one particle whose stencil is outside the 8^3 tile (grid operation
// at staging): each node's velocity is the grid operation of its momentum.
template <bool COH>
__device__ __forceinline__ void g2p_global_gas(const Dev &d, const EnvDev &e, const ToolDev *tl, const float4 *gP,
                                               const Stencil &s, float vp[3], float Cn[9])
{
    float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    vp[0] = vp[1] = vp[2] = 0.f;
    // the loop stays rolled (its body holds a whole grid operation), so the
    // weights are selected by offset rather than indexed: an indexed stencil
    // would live in scratch memory
    auto wsel = [&](int a, int o) { return o == 0 ? s.w[a][0] : (o == 1 ? s.w[a][1] : s.w[a][2]); };
    for (int o0 = 0; o0 < 3; ++o0)
        for (int o1 = 0; o1 < 3; ++o1)
            for (int o2 = 0; o2 < 3; ++o2) {
                const int i = s.b[0] + o0, j = s.b[1] + o1, k = s.b[2] + o2;
                const float4 *q = gP + node_id(e, i, j, k);
                const float3 V = grid_node_velocity_tl<false>(d, e, tl, COH ? cload(q) : gload(q), i, j, k, nullptr);
                const float d0 = o0 - s.fx[0], d1 = o1 - s.fx[1], d2 = o2 - s.fx[2];
                const float w = wsel(0, o0) * wsel(1, o1) * wsel(2, o2);
                const float wx = w * V.x, wy = w * V.y, wz = w * V.z;
                vp[0] += wx; vp[1] += wy; vp[2] += wz;
                B[0] += wx * d0; B[1] += wx * d1; B[2] += wx * d2;
                B[3] += wy * d0; B[4] += wy * d1; B[5] += wy * d2;
                B[6] += wz * d0; B[7] += wz * d1; B[8] += wz * d2;
            }
    const float cs = 4.0f * e.inv_dx;
#pragma unroll
    for (int c = 0; c < 9; ++c) Cn[c] = cs * B[c];
}

// State of the grid-at-staging kernels that outlives one pass over the
// items: a single environment's entry, an environment's tool slots (with the
// substep's poses) on their way through registers (tw, environment tw_env)
// into LDS (environment tl_env), and the momentum clear's prefetched values.
template <int T>
struct GasState {
    static constexpr int WPT = (int)(sizeof(ToolDev) / 4);
    static constexpr int NTW = (MAX_TOOLS * WPT + T - 1) / T;
    int tw[NTW];
    int tw_env = -1, tl_env = -1;
    bool one_env = false;
    EnvDev e0;
    GasClear clr;
    bool clr_pending = false;
};

template <int T>
__device__ __forceinline__ void gas_tools_issue(const Dev &d, const ToolPose *pose, GasState<T> &gs, int env)
{
    const int words = d.max_tools * GasState<T>::WPT;
#pragma unroll
    for (int q = 0; q < GasState<T>::NTW; ++q)
        if (threadIdx.x + q * T < words) gs.tw[q] = gload(tool_word(d, pose, env, threadIdx.x + q * T));
    gs.tw_env = env;
}

// The issued tool slots into LDS; tl must be unused (after a barrier).
template <int T>
__device__ __forceinline__ void gas_tools_commit(const Dev &d, ToolDev *tl, GasState<T> &gs)
{
    const int words = d.max_tools * GasState<T>::WPT;
#pragma unroll
    for (int q = 0; q < GasState<T>::NTW; ++q)
        if (threadIdx.x + q * T < words) reinterpret_cast<int *>(tl)[threadIdx.x + q * T] = gs.tw[q];
    gs.tl_env = gs.tw_env;
}

// Items first, first + stride, ... below end.  COH (persistent kernels): grid
// data that other workgroups of the same launch wrote is read with
// device-coherent loads (node velocities; with GAS, the momentum), and GAS
// clears and stamps are stored device-coherently.  GAS (grid operation at
// staging, MODE 0-2): no grid kernel runs between particle passes; the G2P
// stages the 8^3 node velocities of its tile by applying the grid operation
// to this substep's momentum (a.gP_read) with the tool slots gs carries into
// LDS, and P2G writes the next substep's momentum to d.gP.
template <int MODE, int W, bool COH, bool GAS, class SH>
__device__ __forceinline__ void tiled_items(const Dev &d, const TiledArgs &a, SH &sh, int first,
                                            int stride, int end, GasState<64 * W> &gs)
{
    constexpr bool G2P = MODE >= 1, P2G = MODE <= 1 || MODE == 3;
    constexpr int T = 64 * W;
    constexpr int TS = GAS ? GTILE : TILE;   // velocity tile edge
    float4 *tv = sh.tv, *tp = sh.tp;
    Payload *pay = sh.pay;

    const int N = d.ntot, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int hw = 2 * wave + (lane >> 5);   // half-wave index

    int4 next = first < end ? uload(a.items + first) : make_int4(0, 0, 0, 0);
    for (int it = first; it < end; it += stride) {
        const int4 item = next;   // loaded one iteration ahead
        if (it + stride < end) next = uload(a.items + it + stride);
        if (GAS && G2P && item.w != gs.tw_env) gas_tools_issue(d, a.pose_in, gs, item.w);
        EnvDev e;
        Tile t;
        if (gs.one_env) {
            e = gs.e0;
            t = tile_of(item, e);
        } else {
            t = make_tile(d, item, e);
        }
        const int item_end = item.y + item.z;
        // position and deformation of this lane's particle in the next chunk, loaded
        // ahead so the loads overlap the tile set-up (first chunk) or the node pass
        float px[3], pH[9];
        auto prefetch = [&](int chunk) {
            const int p = chunk + tid;
            if (p < item_end) {
#pragma unroll
                for (int c = 0; c < 3; ++c) px[c] = gload(comp(a.xin, c, N) + (uint32_t)p);
#pragma unroll
                for (int c = 0; c < 9; ++c) pH[c] = gload(comp(a.Hin, c, N) + (uint32_t)p);
            }
        };
        prefetch(item.y);
        float mu = 0.f, lam = 0.f, m = 0.f, V0 = 0.f;
        if (P2G) {
            const float *mat = d.material + 4 * t.env;
            const float E = uload(mat), nu = uload(mat + 1), rho = uload(mat + 2);
            V0 = uload(mat + 3);
            lame(E, nu, mu, lam);
            m = rho * V0;
        }
        for (int n = tid; n < TILE_NODES; n += T) {
            int la = n / 36, lb = (n / 6) % 6, lc = n % 6;
            if (P2G)
                for (int w = 0; w < 2 * W; ++w) tp[w * TILE_NODES + n] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (G2P && !GAS) {
                int i = t.o[0] + la, j = t.o[1] + lb, k = t.o[2] + lc;
                float4 V = make_float4(0.f, 0.f, 0.f, 0.f);
                if (i < e.n && j < e.n && k < e.n) V = COH ? cload(d.gV + node_id(e, i, j, k)) : gload(d.gV + node_id(e, i, j, k));
                tv[n] = V;
            }
        }
        if (GAS && G2P) {
            // a thread's momentum loads (up to four) are all issued before its first grid operation
            constexpr int NS = GTILE_NODES / T, NG = NS < 4 ? NS : 4;
#pragma unroll
            for (int g0 = 0; g0 < NS; g0 += NG) {
                float4 P[NG];
                int64_t gid[NG];
                bool in[NG];
#pragma unroll
                for (int q = 0; q < NG; ++q) {
                    const int n = tid + (g0 + q) * T;
                    const int i = t.o[0] - 1 + (n >> 6), j = t.o[1] - 1 + ((n >> 3) & 7), k = t.o[2] - 1 + (n & 7);
                    in[q] = i >= 0 && j >= 0 && k >= 0 && i < e.n && j < e.n && k < e.n;
                    gid[q] = in[q] ? node_id(e, i, j, k) : 0;
                    P[q] = in[q] ? (COH ? cload(a.gP_read + gid[q]) : gload(a.gP_read + gid[q])) : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                if (g0 == 0 && t.env != gs.tl_env) {
                    gas_tools_commit(d, sh.tl, gs);
                    __syncthreads();
                }
                // every lane takes the grid operation (a node outside the grid has no mass and
                // leaves it at once), so each load is consumed on every path
#pragma unroll
                for (int q = 0; q < NG; ++q) {
                    const int n = tid + (g0 + q) * T;
                    const int la = n >> 6, lb = (n >> 3) & 7, lc = n & 7;
                    const float3 v = grid_node_velocity_tl<false>(d, e, sh.tl, P[q], t.o[0] - 1 + la,
                                                                  t.o[1] - 1 + lb, t.o[2] - 1 + lc, nullptr);
                    const float4 V = make_float4(v.x, v.y, v.z, 0.f);
                    // the tail leaves the velocities of the item's own brick readable
                    if (MODE == 2 && in[q] && la >= 1 && la <= 4 && lb >= 1 && lb <= 4 && lc >= 1 && lc <= 4)
                        gstore(d.gV + gid[q], V);
                    tv[n] = V;
                }
            }
        }
        __syncthreads();
        // persistent run: the loads its substep issued before this item (tool velocities, stamp)
        // were older than the staging loads just consumed, so they are complete; saying so here
        // spares the flush a wait for every memory operation in flight
        if (COH && GAS) __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
        if (GAS && gs.clr_pending) {
            gas_clear_finish<T, COH>(a, gs.clr);
            gs.clr_pending = false;
        }

        for (int chunk = item.y; chunk < item_end; chunk += T) {
            // ---- pass 1: lane = particle
            const int p = chunk + tid;
            int key = KEY_NONE;
            if (p < item_end) {
                float x[3] = {px[0], px[1], px[2]};
                float H[9], v[3], C[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) H[c] = pH[c];
                Stencil s;
                make_stencil(x[0], x[1], x[2], e.inv_dx, e.n, s);
                if (s.outside) {
                    // out of the domain: state unchanged, no transfers
                    set_flag(d.status, t.env, MPM_FLAG_OUT_OF_DOMAIN);
                    if (a.xout != a.xin) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            gstore(comp(a.xout, c, N) + (uint32_t)p, x[c]);
                            gstore(comp(a.vout, c, N) + (uint32_t)p, gload(comp(a.vin, c, N) + (uint32_t)p));
                        }
#pragma unroll
                        for (int c = 0; c < 9; ++c) {
                            gstore(comp(a.Hout, c, N) + (uint32_t)p, H[c]);
                            gstore(comp(a.Cout, c, N) + (uint32_t)p, gload(comp(a.Cin, c, N) + (uint32_t)p));
                        }
                    }
                    if (a.pidout != a.pidin) gstore(a.pidout + (uint32_t)p, gload(a.pidin + (uint32_t)p));
                } else {
                    float jm1 = 0.f;
                    bool inv = false;
                    if (G2P) {
                        int l0, l1, l2;
                        if (GAS ? stencil_in_gtile(t, s, l0, l1, l2) : stencil_in_tile(t, s, l0, l1, l2)) {
                            // v = sum w V, B = sum w V (o - fx)^T, summed over o2 first
                            float q[3][3], w2q[3];
#pragma unroll
                            for (int k = 0; k < 3; ++k) {
                                q[0][k] = k - s.fx[0]; q[1][k] = k - s.fx[1]; q[2][k] = k - s.fx[2];
                                w2q[k] = s.w[2][k] * q[2][k];
                            }
                            float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                            v[0] = v[1] = v[2] = 0.f;
                            const float4 *tb = tv + (l0 * TS + l1) * TS + l2;
#pragma unroll
                            for (int a0 = 0; a0 < 3; ++a0) {
                                // a plane's nine reads are issued together (the barrier keeps
                                // them ahead of the sums), so their latencies overlap
                                float3 Vp[3][3];
#pragma unroll
                                for (int a1 = 0; a1 < 3; ++a1)
#pragma unroll
                                    for (int a2 = 0; a2 < 3; ++a2) {
                                        const float4 V = tb[(a0 * TS + a1) * TS + a2];
                                        Vp[a1][a2] = make_float3(V.x, V.y, V.z);
                                    }
                                asm volatile("" ::: "memory");
#pragma unroll
                                for (int a1 = 0; a1 < 3; ++a1) {
                                    float sx = 0.f, sy = 0.f, sz = 0.f, ux = 0.f, uy = 0.f, uz = 0.f;
#pragma unroll
                                    for (int a2 = 0; a2 < 3; ++a2) {
                                        const float3 V = Vp[a1][a2];
                                        const float w2 = s.w[2][a2];
                                        sx = fmaf(w2, V.x, sx); sy = fmaf(w2, V.y, sy); sz = fmaf(w2, V.z, sz);
                                        ux = fmaf(w2q[a2], V.x, ux); uy = fmaf(w2q[a2], V.y, uy);
                                        uz = fmaf(w2q[a2], V.z, uz);
                                    }
                                    const float ww = s.w[0][a0] * s.w[1][a1];
                                    const float w0q = ww * q[0][a0], w1q = ww * q[1][a1];
                                    v[0] = fmaf(ww, sx, v[0]); v[1] = fmaf(ww, sy, v[1]); v[2] = fmaf(ww, sz, v[2]);
                                    B[0] = fmaf(w0q, sx, B[0]); B[1] = fmaf(w1q, sx, B[1]); B[2] = fmaf(ww, ux, B[2]);
                                    B[3] = fmaf(w0q, sy, B[3]); B[4] = fmaf(w1q, sy, B[4]); B[5] = fmaf(ww, uy, B[5]);
                                    B[6] = fmaf(w0q, sz, B[6]); B[7] = fmaf(w1q, sz, B[7]); B[8] = fmaf(ww, uz, B[8]);
                                }
                            }
                            const float cs = 4.0f * e.inv_dx;
#pragma unroll
                            for (int c = 0; c < 9; ++c) C[c] = cs * B[c];
                        } else if (GAS) {
                            g2p_global_gas<COH>(d, e, sh.tl, a.gP_read, s, v, C);
                        } else {
                            g2p_global<COH>(d, e, s, v, C);
                        }
                        x[0] += d.dt * v[0];
                        x[1] += d.dt * v[1];
                        x[2] += d.dt * v[2];
                        update_h(H, C, d.dt);
                        jm1 = jm1_f(H);
                        inv = inverted_f(H, jm1);
                        if (inv) set_flag(d.status, t.env, MPM_FLAG_INVERTED);
                        if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(v[0]) &&
                              isfinite(v[1]) && isfinite(v[2])))
                            set_flag(d.status, t.env, MPM_FLAG_NONFINITE);
                    } else {
#pragma unroll
                        for (int c = 0; c < 3; ++c) v[c] = gload(comp(a.vin, c, N) + (uint32_t)p);
#pragma unroll
                        for (int c = 0; c < 9; ++c) C[c] = gload(comp(a.Cin, c, N) + (uint32_t)p);
                        jm1 = jm1_f(H);
                        inv = inverted_f(H, jm1);
                        if (inv) set_flag(d.status, t.env, MPM_FLAG_INVERTED);
                    }
                    bool write_vc = MODE >= 2;
                    if (P2G) {
                        Stencil s2;
                        if (G2P) make_stencil(x[0], x[1], x[2], e.inv_dx, e.n, s2); else s2 = s;
                        if (s2.outside) {
                            // leaves the domain now: freeze with this G2P's v, C
                            set_flag(d.status, t.env, MPM_FLAG_OUT_OF_DOMAIN);
                            write_vc = true;
                        } else {
                            float A[9];
                            affine_stress_f(d, e, H, jm1, inv, C, mu, lam, m, V0, A);
                            int l0, l1, l2;
                            key = stencil_in_tile(t, s2, l0, l1, l2) ? key_in_tile(l0, l1, l2) : key_global(s2.b);
                            const float mv[3] = {m * v[0], m * v[1], m * v[2]};
#pragma unroll
                            for (int c = 0; c < 9; ++c) A[c] *= e.dx;
                            store_payload(pay[tid], sh.wz[tid], s2.fx, s2.w[2], key, mv, A);
                        }
                    }
                    if (G2P) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) gstore(comp(a.xout, c, N) + (uint32_t)p, x[c]);
#pragma unroll
                        for (int c = 0; c < 9; ++c) gstore(comp(a.Hout, c, N) + (uint32_t)p, H[c]);
                        if (write_vc) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) gstore(comp(a.vout, c, N) + (uint32_t)p, v[c]);
#pragma unroll
                            for (int c = 0; c < 9; ++c) gstore(comp(a.Cout, c, N) + (uint32_t)p, C[c]);
                        }
                        if (a.pidout != a.pidin) gstore(a.pidout + (uint32_t)p, gload(a.pidin + (uint32_t)p));
                    }
                }
            }
            if (chunk + T < item_end) prefetch(chunk + T);
            if (P2G) {
                if (key == KEY_NONE) payload_none(pay[tid]);
                __syncthreads();
                // ---- pass 2: lane = stencil node, the chunk split into 2W contiguous runs
                int r0, r1;
                half_wave_run<W>(hw, min(T, item_end - chunk), r0, r1);
                node_pass(a.slots, pay, sh.wz, r0, r1, tp + hw * TILE_NODES, lane, m, [&](const float4 &c4, int i, int j, int k) {
                    // stencil outside the tile: straight to the global grid
                    float *g = reinterpret_cast<float *>(d.gP + node_id(e, i, j, k));
                    gatomic_add(g + 0, c4.x);
                    gatomic_add(g + 1, c4.y);
                    gatomic_add(g + 2, c4.z);
                    gatomic_add(g + 3, c4.w);
                    const int di = (i >> 2) - t.bi, dj = (j >> 2) - t.bj, dk = (k >> 2) - t.bk;
                    if (di < -1 || di > 1 || dj < -1 || dj > 1 || dk < -1 || dk > 1) {
                        // grid at staging and tape recompute: a stamp (that grid is then cleared or
                        // swept whole); otherwise the brick goes to a list
                        if (GAS || a.far_stamp) {   // (grid-at-staging kernels always stamp)
                            if (COH) cstore(a.far_stamp + a.write_slot, a.write_stamp);
                            else gstore(a.far_stamp + a.write_slot, a.write_stamp);
                        } else {
                            mark_far_brick(a.act, a.par, e.bofs + ((i >> 2) * e.nb + (j >> 2)) * e.nb + (k >> 2),
                                           t.env, e.bofs);
                        }
                    }
                });
            }
            if (P2G) __syncthreads();   // payload slots are rewritten by the next chunk
        }

        if (P2G) {
            // sum the wave tiles and flush the non-empty nodes (their bricks are in the static list);
            // a node's 2W tile entries are read together, whole
            for (int n = tid; n < TILE_NODES; n += T) {
                float4 q[2 * W];
#pragma unroll
                for (int w = 0; w < 2 * W; ++w) q[w] = tp[w * TILE_NODES + n];
                float4 sum = q[0];
#pragma unroll
                for (int w = 1; w < 2 * W; ++w) {
                    sum.x += q[w].x; sum.y += q[w].y; sum.z += q[w].z; sum.w += q[w].w;
                }
                // keeps the momentum sums from being sunk under the mass test
                asm volatile("" : "+v"(sum.x), "+v"(sum.y), "+v"(sum.z), "+v"(sum.w));
                if (sum.x != 0.f) {
                    int la = n / 36, lb = (n / 6) % 6, lc = n % 6;
                    int i = t.o[0] + la, j = t.o[1] + lb, k = t.o[2] + lc;
                    float *g = reinterpret_cast<float *>(d.gP + node_id(e, i, j, k));
                    gatomic_add(g + 0, sum.x);
                    gatomic_add(g + 1, sum.y);
                    gatomic_add(g + 2, sum.z);
                    gatomic_add(g + 3, sum.w);
                }
            }
        }
        __syncthreads();
    }
}

// One pass of a tiled kernel over its items.  COH (persistent kernel): the
// tool poses and step counters are left to the caller.  GAS kernels take their
// item range from a.totals (first, stride and end are ignored), after issuing
// the loads that do not depend on it: the momentum clear's, and a single
// environment's entry and tool slots.
template <int MODE, int W, bool COH = false, bool GAS = false, class SH>
__device__ __forceinline__ void tiled_body(const Dev &d, const TiledArgs &a, SH &sh, int first,
                                           int stride, int end)
{
    constexpr bool G2P = MODE >= 1;
    constexpr int T = 64 * W;
    GasState<T> gs;
    if constexpr (GAS) {
        gs.one_env = d.n_envs == 1;
        if (G2P && gs.one_env) gas_tools_issue(d, a.pose_in, gs, 0);
        if (gs.one_env) gs.e0 = load_env(d.env);
        if (a.gP_clear) {
            gs.clr = gas_clear_issue<T>(a);
            gs.clr_pending = true;
        }
        // the last workgroup in launch order has the fewest items
        if (blockIdx.x == gridDim.x - 1) gas_poses<MODE, T>(d, a);
        item_range(uload(a.totals).y, first, stride, end);
    }
    tiled_items<MODE, W, COH, GAS>(d, a, sh, first, stride, end, gs);
    if (GAS && gs.clr_pending) gas_clear_finish<T, COH>(a, gs.clr);   // a workgroup without items
    if (COH || GAS) return;
    if (G2P) advance_end_of_substep(d);
    // the tail ends a call: both dynamic lists start empty at the next head
    if (MODE == 2 && blockIdx.x == 0 && threadIdx.x < 2 && a.act.dcount) gstore(a.act.dcount + threadIdx.x, 0);
}

template <int MODE, int W>
__global__ __launch_bounds__(64 * W) void k_tiled(Dev d, TiledArgs a)
{
    __shared__ TiledShared<W, false, MODE != 2> sh;
    int first, stride, end;
    item_range(uload(a.totals).y, first, stride, end);
    tiled_body<MODE, W>(d, a, sh, first, stride, end);
}

// The grid-at-staging forms; two wavefronts per SIMD (up to 256 VGPRs): with
// the loads issued ahead of the item range, three (168 VGPRs) spill to scratch.
template <int MODE, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2))) void k_tiled_gas(Dev d, TiledArgs a)
{
    __shared__ TiledShared<W, true, MODE != 2> sh;
    tiled_body<MODE, W, false, true>(d, a, sh, 0, 0, 0);   // item range from a.totals
}

// A persistent run of the grid-at-staging form (GasRun): the fused substeps
// between two sorts of a single environment in one launch, with every
// workgroup resident (the launch uses the occupancy-derived count).  Between
// substeps the workgroups meet at run_barrier; grid data crosses workgroups
// only through device-scope atomics and device-coherent loads and stores.
// Every workgroup keeps the tool slots in LDS and advances them itself after
// each substep (the same FP64 arithmetic as the per-substep form); the item
// list and static brick list stay those of the last sort.
template <int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2))) void k_gas_run(Dev d, TiledArgs a, GasRun r)
{
    __shared__ TiledShared<W, true> sh;
    __shared__ int ok;
    constexpr int T = 64 * W;
    GasState<T> gs;
    gs.one_env = true;
    gas_tools_issue(d, r.pose_in, gs, 0);
    gs.e0 = load_env(d.env);
    const GasClear c0 = gas_clear_issue<T>(a);   // static list length and first entry (fixed for the run)
    int first, stride, end;
    item_range(uload(a.totals).y, first, stride, end);
    gas_tools_commit(d, sh.tl, gs);
    __syncthreads();
    const int mt = d.max_tools;
    int done = 0;
    for (int s = 0; s < r.m; ++s) {
        const int i = r.i0 + s;
        TiledArgs as = a;
        if (s > 0) {   // the first substep reads the call's input (a sort's output); later ones update in place
            as.xin = a.xout; as.vin = a.vout; as.Cin = a.Cout; as.Hin = a.Hout; as.pidin = a.pidout;
        }
        Dev ds = d;
        ds.gP = r.buf[(i + 1) % 3];
        as.gP_read = r.buf[i % 3];
        as.gP_clear = i >= 1 ? r.buf[(i + 2) % 3] : nullptr;
        as.full_clear = (r.sorted_at == i || r.sorted_at == i - 1) ? 1 : 0;
        as.clear_slot = (r.m0 + i - 1) & 3;
        as.clear_stamp = r.m0 + i - 1;
        as.write_slot = (r.m0 + i + 1) & 3;
        as.write_stamp = r.m0 + i + 1;
        if (as.gP_clear) {
            gs.clr = c0;
            gs.clr.stamp = cload(a.far_stamp + as.clear_slot);
            gs.clr_pending = true;
        }
        // this substep's tool velocities (read now, applied after the substep)
        float3 u = make_float3(0.f, 0.f, 0.f);
        if (threadIdx.x < mt && sh.tl[threadIdx.x].active) u = tool_velocity(sh.tl[threadIdx.x]);
        tiled_items<1, W, true, true>(ds, as, sh, first, stride, end, gs);
        if (gs.clr_pending) {   // a workgroup without items
            gas_clear_finish<T, true>(as, gs.clr);
            gs.clr_pending = false;
        }
        if (threadIdx.x < mt && sh.tl[threadIdx.x].active) advance_tool_u(sh.tl[threadIdx.x], d.dt, u);
        done = s + 1;
        if (s + 1 < r.m && !run_barrier(d, r.bar, s + 1, r.spin_limit, ok)) break;
    }
    __syncthreads();
    if (blockIdx.x == gridDim.x - 1) {
        if (threadIdx.x < mt) {
            const ToolDev &Tt = sh.tl[threadIdx.x];
            r.pose_out[threadIdx.x] = ToolPose{{Tt.T[0], Tt.T[1], Tt.T[2]}, Tt.k, 0};
        }
        if (threadIdx.x == 0) d.step[0] += done;
    }
    run_exit(r.bar);
}

// Grid operation at staging: the clear of one momentum buffer on its own.
__global__ __launch_bounds__(256) void k_gas_clear(TiledArgs a)
{
    gas_clear_finish<256>(a, gas_clear_issue<256>(a));
}

// Grid operation over the static brick list and dynamic list `par`: one
// wavefront per 4^3 brick.  Writes V and clears P of every brick that
// received mass; clears the flags of the dynamic bricks, and the other
// dynamic list's count for the next P2G.
template <bool SDF>
__device__ __forceinline__ void grid_active_body(const Dev &d, const ActiveBuf &a, int par)
{
    // 256 threads (k_grid_active's launch): the wavefront count is a constant, so the
    // first list entry's address does not wait for the launch's size
    constexpr int nw = 256 >> 6;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int stride = gridDim.x * nw;
    int i = blockIdx.x * nw + wave;
    // the first static entry is loaded together with the counts (used only if i < ns)
    int bs = i < a.nbricks ? uload(a.slist + i) : 0;
    const int ns = uload(a.scount), nd = gload(a.dcount + par);
    const int32_t *dl = a.dlist + (size_t)par * a.nbricks;
    // one environment: its entry is loaded once, before the loop; several: each
    // brick's environment is looked up beside its P (not after the emptiness test),
    // so a listed brick waits for two dependent loads after its id, not three
    const bool one_env = d.n_envs == 1;
    EnvDev e1{};
    if (one_env) e1 = load_env(d.env);
    for (; i < ns + nd; i += stride) {
        const bool dyn = i >= ns;
        const int b = dyn ? gload(dl + (i - ns)) : bs;
        if (i + stride < a.nbricks) bs = gload(a.slist + i + stride);
        // a sort between the listing P2G and this pass moved the brick to the static list
        if (dyn && gload(a.flag + b) == 1) continue;
        // environments' grids are consecutive brick-major slices, so node l of brick b is
        // node 64 b + l of the whole grid: P is loaded without waiting for the environment
        const int64_t g = (int64_t)b * BRICK_NODES + lane;
        float4 P = gload(d.gP + g);
        int env = 0;
        if (!one_env) {
            env = gload(a.brick_env + b);
            asm volatile("" :: "v"(env));   // keeps the load here, issued with P's
        }
        if (!__any(P.x != 0.f)) {
            // no mass reached the brick this substep: P is already clear and no
            // particle's G2P reads its velocities, so there is nothing to write
            if (dyn && lane == 0) gstore(a.flag + b, 0);
            continue;
        }
        EnvDev e = e1;
        if (!one_env) e = load_env(d.env + env);
        int lb = b - e.bofs;
        int gi, gj, gk;
        brick_local_to_ijk(e, lb, lane, gi, gj, gk);
        float3 v = grid_node_velocity<SDF>(d, e, env, P, gi, gj, gk, nullptr);
        gstore(d.gV + g, make_float4(v.x, v.y, v.z, 0.f));
        gstore(d.gP + g, make_float4(0.f, 0.f, 0.f, 0.f));
        if (dyn && lane == 0) gstore(a.flag + b, 0);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) gstore(a.dcount + (par ^ 1), 0);
}

template <bool SDF>
__global__ __launch_bounds__(256) void k_grid_active(Dev d, ActiveBuf a, int par)
{
    grid_active_body<SDF>(d, a, par);
}

// ---------------------------------------------------------------------------
// Persistent form: one launch runs m substeps (a run between two sorts) of
// every environment.  Each environment has its own group of workgroups and
// its own completion counter; the group alternates the grid operation over
// the environment's flagged bricks and the particle pass over its items,
// with a group barrier after each, so environments never wait for each
// other.  The grid data that crosses workgroups inside the launch (momentum
// P, velocity V, brick flags) moves only through device-coherent accesses
// (float atomics, cload / cstore), so a barrier needs no cache write-back or
// invalidation: a workgroup waits until its own memory operations have
// completed, then adds one to the counter; the others wait for the count.
// A workgroup keeps the particles of the same items through the run, so
// particle state never crosses workgroups.

// Barrier k (1, 2, ...) of a group of gsize workgroups on counter ctr.
// Returns false, after setting MPM_FLAG_BARRIER_TIMEOUT, if the spin limit
// ran out (some workgroup of the group is not resident).
__device__ __forceinline__ bool group_barrier(const Dev &d, int env, unsigned *ctr, unsigned target, int spin_limit,
                                              int &ok_shared)
{
    __builtin_amdgcn_s_waitcnt(0);   // this wave's loads, stores and atomics have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __hip_atomic_fetch_add(gptr(ctr), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1, spins = 0;
        while (__hip_atomic_load(gptr(ctr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > spin_limit) { ok = 0; break; }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (!ok) set_flag(d.status, env, MPM_FLAG_BARRIER_TIMEOUT);
        ok_shared = ok;
    }
    __syncthreads();
    return ok_shared != 0;
}

// List the environment's flagged bricks (static neighbourhood 1, far-drift
// 2) for a run: the wavefronts of the group sweep the flags 64 at a time and
// append to the environment's run list.  Bricks a particle reaches later in
// the run are appended by mark_far_brick, so the list only grows.
__device__ __forceinline__ void list_env_bricks(const EnvDev &e, int env, const ActiveBuf &a, int rank, int gsize)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int nbe = e.nb * e.nb * e.nb;
    for (int c0 = (rank * nw + wave) * 64; c0 < nbe; c0 += gsize * nw * 64) {
        const int f = c0 + lane < nbe ? cload(a.flag + e.bofs + c0 + lane) : 0;
        const unsigned long long listed = __ballot(f != 0);
        if (!listed) continue;
        int base = 0;
        if (lane == 0) base = gatomic_add(a.ecount + env, (int)__popcll(listed));
        base = __shfl(base, 0);
        if (f != 0) cstore(a.elist + e.bofs + base + (int)__popcll(listed & ((1ull << lane) - 1ull)), e.bofs + c0 + lane);
    }
}

// Grid operation of one environment by workgroup `rank` of a group of
// `gsize`: the group's wavefronts take the run list's bricks in turn, one
// node per lane.  last: the final grid operation of the call, which returns
// far-drift flags to 0 (the G2P tail after it lists nothing).
template <bool SDF>
__device__ __forceinline__ void grid_env_phase(const Dev &d, const EnvDev &e, int env, const ToolDev *tl,
                                               const ActiveBuf &a, int rank, int gsize, bool last)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int n = cload(a.ecount + env);
    for (int j = rank * nw + wave; j < n; j += gsize * nw) {
        const int b = cload(a.elist + e.bofs + j), lb = b - e.bofs;
        float4 *gp = d.gP + (int64_t)b * BRICK_NODES + lane;
        const float4 P = cload(gp);
        if (__any(P.x != 0.f)) {
            int gi, gj, gk;
            brick_local_to_ijk(e, lb, lane, gi, gj, gk);
            const float3 v = grid_node_velocity_tl<SDF>(d, e, tl, P, gi, gj, gk, nullptr);
            cstore(d.gV + (int64_t)b * BRICK_NODES + lane, make_float4(v.x, v.y, v.z, 0.f));
            cstore(gp, make_float4(0.f, 0.f, 0.f, 0.f));
        }
        if (last && lane == 0 && cload(a.flag + b) == 2) cstore(a.flag + b, 0);
    }
}

// The contiguous items [i0, i1) of group member `rank` of `gsize` among an
// environment's items [ie0, ie1): the items are cut where the running sum of
// their weights crosses multiples of 1/gsize of the total (a block-wide
// scan in chunks of the workgroup's size; `scratch` holds blockDim.x / 64 + 3
// ints of LDS).  Every member computes the same cuts.
__device__ __forceinline__ void member_items(const int4 *items, int ie0, int ie1, int rank, int gsize, int *scratch,
                                             int &i0, int &i1)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    int *wsum = scratch, *lo = scratch + nw, *hi = scratch + nw + 1, *tot = scratch + nw + 2;
    // total weight
    int part = 0;
    for (int i = ie0 + tid; i < ie1; i += blockDim.x) part += gload(items + i).z + ITEM_FIXED_COST;
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (tid == 0) { *lo = ie1; *hi = ie0; *tot = 0; }
    __syncthreads();
    if (lane == 0) atomicAdd(tot, part);
    __syncthreads();
    const long long W = *tot;
    if (W == 0) {   // no items
        i0 = i1 = ie0;
        __syncthreads();
        return;
    }
    int carry = 0;
    for (int c0 = ie0; c0 < ie1; c0 += blockDim.x) {
        const int i = c0 + tid;
        const int w = i < ie1 ? gload(items + i).z + ITEM_FIXED_COST : 0;
        int incl = w;   // inclusive scan within the wavefront
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int before = carry;
        for (int q = 0; q < wave; ++q) before += wsum[q];
        int chunk_total = 0;
        for (int q = 0; q < nw; ++q) chunk_total += wsum[q];
        // the member owning an item is the one whose share holds the item's start
        const long long start = before + incl - w;
        if (i < ie1 && (int)((start * gsize) / W) == rank) {
            atomicMin(lo, i);
            atomicMax(hi, i + 1);
        }
        carry += chunk_total;
        __syncthreads();
    }
    i0 = *lo;
    i1 = *hi;
    if (i1 < i0) i1 = i0;
    __syncthreads();
}

// First work item of the bricks from brick k on (the sort's per-brick item
// prefix; the total past the last brick).
__device__ __forceinline__ int item_prefix(const SortBuf &s, int k, int nbricks)
{
    if (k >= nbricks) return gload(s.totals).y;
    return gload(s.brick_offset + k).y + gload(s.chunk_sum + k / SORT_SCAN_CHUNK).y;
}

template <int W, bool SDF>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3))) void k_persistent(Dev d, TiledArgs first, TiledArgs rest, EnvGroups g, int m,
                                                       int tail_last, int spin_limit)
{
    __shared__ TiledShared<W> sh;
    __shared__ ToolDev tl[MAX_TOOLS];
    __shared__ int ok;
    const int4 me = gload(g.wg + blockIdx.x);   // (first env, env count, rank, group size)
    const int mt = d.max_tools;
    for (int ei = 0; ei < me.y; ++ei) {
        const int env = me.x + ei;
        const EnvDev e = load_env(d.env + env);
        // the environment's tool slots, advanced here substep by substep (every
        // workgroup of the group does the same FP64 arithmetic)
        for (int w = threadIdx.x; w < mt * (int)(sizeof(ToolDev) / 4); w += blockDim.x)
            reinterpret_cast<int *>(tl)[w] = gload(reinterpret_cast<const int *>(d.tools + (size_t)env * mt) + w);
        const int ie0 = item_prefix(g.sort, e.bofs, g.nbricks), ie1 = item_prefix(g.sort, e.bofs + e.nb * e.nb * e.nb, g.nbricks);
        int i0, i1;
        member_items(first.items, ie0, ie1, me.z, me.w, reinterpret_cast<int *>(sh.pay), i0, i1);
        unsigned *ctr = g.arrive + env;
        unsigned k = 0;
        if (threadIdx.x == 0) ok = 1;
        __syncthreads();
        list_env_bricks(e, env, first.act, me.z, me.w);
        for (int i = 0; i < m && group_barrier(d, env, ctr, ++k * me.w, spin_limit, ok); ++i) {
            grid_env_phase<SDF>(d, e, env, tl, first.act, me.z, me.w, i == m - 1 && tail_last);
            if (!group_barrier(d, env, ctr, ++k * me.w, spin_limit, ok)) break;
            const TiledArgs &a = i == 0 ? first : rest;
            if (i == m - 1 && tail_last) tiled_body<2, W, true>(d, a, sh, i0, 1, i1);
            else tiled_body<1, W, true>(d, a, sh, i0, 1, i1);
            if (threadIdx.x < mt && tl[threadIdx.x].active) advance_tool(tl[threadIdx.x], d.dt);
            __syncthreads();
        }
        if (me.z == 0) {
            for (int w = threadIdx.x; w < mt * (int)(sizeof(ToolDev) / 4); w += blockDim.x)
                gstore(reinterpret_cast<int *>(d.tools + (size_t)env * mt) + w, reinterpret_cast<const int *>(tl)[w]);
            if (threadIdx.x == 0) gstore(d.step + env, gload(d.step + env) + m);
        }
        __syncthreads();
    }
}

template <int MODE, bool GAS = false>
static void launch_mode(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    if constexpr (GAS) {
        if (block == 64) launch_k((k_tiled_gas<MODE, 1>), dim3(nblocks), dim3(64), 0, st, d, a);
        else if (block == 128) launch_k((k_tiled_gas<MODE, 2>), dim3(nblocks), dim3(128), 0, st, d, a);
        else launch_k((k_tiled_gas<MODE, 4>), dim3(nblocks), dim3(256), 0, st, d, a);
    } else if (block == 64) launch_k((k_tiled<MODE, 1>), dim3(nblocks), dim3(64), 0, st, d, a);
    else if (block == 128) launch_k((k_tiled<MODE, 2>), dim3(nblocks), dim3(128), 0, st, d, a);
    else launch_k((k_tiled<MODE, 4>), dim3(nblocks), dim3(256), 0, st, d, a);
}

void launch_gas_head(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    launch_mode<0, true>(d, a, block, nblocks, st);
}

void launch_gas_fused(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    launch_mode<1, true>(d, a, block, nblocks, st);
}

void launch_gas_tail(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    launch_mode<2, true>(d, a, block, nblocks, st);
}

void launch_gas_clear(const Dev &, const TiledArgs &a, hipStream_t st)
{
    launch_k(k_gas_clear, dim3(256), dim3(256), 0, st, a);
}

void launch_gas_run(const Dev &d, const TiledArgs &a, const GasRun &r, int block, int nblocks, hipStream_t st)
{
    if (block == 64) launch_k(k_gas_run<1>, dim3(nblocks), dim3(64), 0, st, d, a, r);
    else if (block == 128) launch_k(k_gas_run<2>, dim3(nblocks), dim3(128), 0, st, d, a, r);
    else launch_k(k_gas_run<4>, dim3(nblocks), dim3(256), 0, st, d, a, r);
}

void launch_p2g_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    launch_mode<0>(d, a, block, nblocks, st);
}

void launch_fused_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    launch_mode<1>(d, a, block, nblocks, st);
}

void launch_g2p_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    launch_mode<2>(d, a, block, nblocks, st);
}

void launch_fused_full_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    launch_mode<3>(d, a, block, nblocks, st);
}

template <bool SDF>
static void launch_persistent_sdf(const Dev &d, const TiledArgs &first, const TiledArgs &rest, const EnvGroups &g,
                                  int m, int tail_last, int spin_limit, int block, int nblocks, hipStream_t st)
{
    if (block == 64)
        launch_k((k_persistent<1, SDF>), dim3(nblocks), dim3(64), 0, st, d, first, rest, g, m, tail_last, spin_limit);
    else if (block == 128)
        launch_k((k_persistent<2, SDF>), dim3(nblocks), dim3(128), 0, st, d, first, rest, g, m, tail_last, spin_limit);
    else
        launch_k((k_persistent<4, SDF>), dim3(nblocks), dim3(256), 0, st, d, first, rest, g, m, tail_last, spin_limit);
}

void launch_persistent(const Dev &d, const TiledArgs &first, const TiledArgs &rest, const EnvGroups &g, int m,
                       int tail_last, int spin_limit, bool sdf, int block, int nblocks, hipStream_t st)
{
    if (sdf) launch_persistent_sdf<true>(d, first, rest, g, m, tail_last, spin_limit, block, nblocks, st);
    else launch_persistent_sdf<false>(d, first, rest, g, m, tail_last, spin_limit, block, nblocks, st);
}

int persistent_workgroups(int block)
{
    int dev = 0, cus = 256, per = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0) cus = p.multiProcessorCount;
    }
    // the SDF instance uses the more registers; its occupancy holds for both
    hipError_t e;
    if (block == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<1, true>, 64, 0);
    else if (block == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<2, true>, 128, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<4, true>, 256, 0);
    int per2 = 0;
    hipError_t e2;
    if (block == 64) e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, k_persistent<1, false>, 64, 0);
    else if (block == 128) e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, k_persistent<2, false>, 128, 0);
    else e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, k_persistent<4, false>, 256, 0);
    if (e != hipSuccess || e2 != hipSuccess || per < 1 || per2 < 1) return 0;
    int g = std::min(per, per2) * cus;
    g -= g % NXCD;
    return g;
}

int tiled_workgroups(int block, bool gas)
{
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0) cus = p.multiProcessorCount;
    }
    hipError_t e;
    if (gas) {
        if (block == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tiled_gas<1, 1>, 64, 0);
        else if (block == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tiled_gas<1, 2>, 128, 0);
        else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tiled_gas<1, 4>, 256, 0);
    } else if (block == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tiled<1, 1>, 64, 0);
    else if (block == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tiled<1, 2>, 128, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tiled<1, 4>, 256, 0);
    if (e != hipSuccess || per < 1) per = 1;
    int g = per * cus;
    g -= g % NXCD;
    return g < NXCD ? NXCD : g;
}

// Workgroups of a persistent grid-at-staging run: as many as are resident at
// once (the run's barrier needs every one of them running).
int gas_run_workgroups(int block)
{
    int dev = 0, cus = 256, per = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0) cus = p.multiProcessorCount;
    }
    hipError_t e;
    if (block == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_gas_run<1>, 64, 0);
    else if (block == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_gas_run<2>, 128, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_gas_run<4>, 256, 0);
    if (e != hipSuccess || per < 1) return 0;
    const int g = per * cus;
    return g - g % NXCD;
}

__global__ __launch_bounds__(256) void k_brick_env(const int32_t *env_bofs, int n_envs, int nbricks, int32_t *out)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nbricks; b += gridDim.x * blockDim.x)
        out[b] = env_of_brick(env_bofs, n_envs, b);
}

void launch_brick_env(const int32_t *env_bofs, int n_envs, int nbricks, int32_t *brick_env, hipStream_t st)
{
    const int nblk = (nbricks + 255) / 256;
    launch_k(k_brick_env, dim3(nblk < 4096 ? nblk : 4096), dim3(256), 0, st, env_bofs, n_envs, nbricks, brick_env);
}

void launch_grid_active(const Dev &d, const ActiveBuf &a, int par, int nblocks, bool sdf, hipStream_t st)
{
    if (sdf) launch_k(k_grid_active<true>, dim3(nblocks), dim3(256), 0, st, d, a, par);
    else launch_k(k_grid_active<false>, dim3(nblocks), dim3(256), 0, st, d, a, par);
}

}  // namespace mpm
