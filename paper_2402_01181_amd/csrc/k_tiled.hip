// Tiled scheme kernels.
//
// Particles are sorted by the 4x4x4-cell brick of their stencil base; a work
// item is (brick, slot range).  For each item a workgroup stages an 8^3 node
// tile (the brick's 6^3 stencil reach plus one cell of drift margin on each
// side) in LDS:
//   - G2P reads node velocities from the tile,
//   - P2G accumulates mass/momentum into the tile with LDS float atomics and
//     flushes each non-empty tile node to the global grid with one float
//     atomic per component,
// so global atomics scale with tile nodes, not with particles x 27.  A
// particle whose stencil has drifted out of the tile since the last sort
// uses global memory directly (rare; correct either way).
//
// Workgroups are persistent over the item list; workgroup w runs on XCD
// w % 8 and walks a contiguous eighth of the (spatially ordered) items, so
// neighbouring tiles, which share halo nodes, stay in one XCD's L2.
#include "mpm_tiled.h"

namespace mpm {

constexpr int NXCD = 8;
// Padded LDS strides for the 8^3 tile: node (a,b,c) -> a*73 + b*9 + c
// spreads the i-, j- and k-neighbours over different banks.
constexpr int LS_I = 73, LS_J = 9, TILE_LDS = 7 * LS_I + 7 * LS_J + 7 + 1;

__device__ __forceinline__ int lds_index(int a, int b, int c) { return a * LS_I + b * LS_J + c; }

struct Tile {
    int env;
    int bi, bj, bk;   // brick coordinates
    int o[3];         // node coordinates of tile corner (0,0,0) = 4*brick - 1
};

__device__ __forceinline__ int env_of_brick(const int32_t *env_bofs, int n_envs, int b)
{
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (gload(env_bofs + mid) <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ Tile make_tile(const Dev &d, const ActiveBuf &act, int brick, EnvDev &e)
{
    Tile t;
    t.env = env_of_brick(act.env_bofs, d.n_envs, brick);
    e = load_env(d.env + t.env);
    int lb = brick - e.bofs;
    t.bk = lb % e.nb;
    int r = lb / e.nb;
    t.bj = r % e.nb;
    t.bi = r / e.nb;
    t.o[0] = 4 * t.bi - 1;
    t.o[1] = 4 * t.bj - 1;
    t.o[2] = 4 * t.bk - 1;
    return t;
}

// Item walk: contiguous eighth of the list per XCD.
__device__ __forceinline__ void item_range(int nitems, int &first, int &stride, int &end)
{
    int G = gridDim.x;               // multiple of NXCD
    int x = blockIdx.x % NXCD, r = blockIdx.x / NXCD;
    int per = (nitems + NXCD - 1) / NXCD;
    first = x * per + r;
    end = min(nitems, (x + 1) * per);
    stride = G / NXCD;
}

__device__ __forceinline__ void mark_brick(const ActiveBuf &act, int par, int b)
{
    if (gatomic_cas(act.flag + b, 0, 1)) {
        int slot = gatomic_add(act.count + par, 1);
        gstore(act.list + (size_t)par * act.stride + slot, b);
    }
}

// Mark every node brick a stencil with base b touches (global fallback path).
__device__ __forceinline__ void mark_stencil_bricks(const ActiveBuf &act, int par, const EnvDev &e, const int b[3])
{
    int lo0 = b[0] >> 2, hi0 = (b[0] + 2) >> 2, lo1 = b[1] >> 2, hi1 = (b[1] + 2) >> 2;
    int lo2 = b[2] >> 2, hi2 = (b[2] + 2) >> 2;
    for (int i = lo0; i <= hi0; ++i)
        for (int j = lo1; j <= hi1; ++j)
            for (int k = lo2; k <= hi2; ++k) mark_brick(act, par, e.bofs + (i * e.nb + j) * e.nb + k);
}

__device__ __forceinline__ void advance_end_of_substep(const Dev &d)
{
    if (blockIdx.x != 0) return;
    for (int t = threadIdx.x; t < d.n_envs; t += blockDim.x) d.step[t] += 1;
    for (int t = threadIdx.x; t < d.n_envs * d.max_tools; t += blockDim.x) {
        ToolDev &T = d.tools[t];
        if (T.active) {
            float3 u = tool_velocity(T);
            T.T[0] += (double)d.dt * u.x;
            T.T[1] += (double)d.dt * u.y;
            T.T[2] += (double)d.dt * u.z;
            T.k += 1;
        }
    }
}

// G2P of one particle: velocity and the affine matrix
// C = (4/dx) sum w v (o - fx), from the LDS tile or, when the stencil is
// outside the tile, from global memory.
template <bool FROM_TILE>
__device__ __forceinline__ void g2p_accumulate(const Dev &d, const EnvDev &e, const Stencil &s, int l0, int l1,
                                               int l2, const float *tvx, const float *tvy, const float *tvz,
                                               float vp[3], float Cn[9])
{
    float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    vp[0] = vp[1] = vp[2] = 0.f;
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                float V0, V1, V2;
                if (FROM_TILE) {
                    int li = lds_index(l0 + o0, l1 + o1, l2 + o2);
                    V0 = tvx[li]; V1 = tvy[li]; V2 = tvz[li];
                } else {
                    float4 V = gload(d.gV + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2));
                    V0 = V.x; V1 = V.y; V2 = V.z;
                }
                float d0 = o0 - s.fx[0], d1 = o1 - s.fx[1], d2 = o2 - s.fx[2];
                float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                float wx = w * V0, wy = w * V1, wz = w * V2;
                vp[0] += wx; vp[1] += wy; vp[2] += wz;
                B[0] += wx * d0; B[1] += wx * d1; B[2] += wx * d2;
                B[3] += wy * d0; B[4] += wy * d1; B[5] += wy * d2;
                B[6] += wz * d0; B[7] += wz * d1; B[8] += wz * d2;
            }
    const float cs = 4.0f * e.inv_dx;
#pragma unroll
    for (int c = 0; c < 9; ++c) Cn[c] = cs * B[c];
}

// P2G of one particle into the tile (LDS atomics) or, when its stencil is
// outside the tile, into the global grid.  The two paths are separate loops
// so every atomic has a fixed address space.
__device__ __forceinline__ void p2g_weights(const EnvDev &e, const Stencil &s, float m, const float A[9],
                                            const float v[3], int o0, int o1, int o2, float &pm, float &p0,
                                            float &p1, float &p2)
{
    float d0 = (o0 - s.fx[0]) * e.dx, d1 = (o1 - s.fx[1]) * e.dx, d2 = (o2 - s.fx[2]) * e.dx;
    float w = s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
    p0 = w * (m * v[0] + A[0] * d0 + A[1] * d1 + A[2] * d2);
    p1 = w * (m * v[1] + A[3] * d0 + A[4] * d1 + A[5] * d2);
    p2 = w * (m * v[2] + A[6] * d0 + A[7] * d1 + A[8] * d2);
    pm = w * m;
}

__device__ __forceinline__ bool stencil_in_tile(const Tile &t, const Stencil &s, int &l0, int &l1, int &l2)
{
    l0 = s.b[0] - t.o[0];
    l1 = s.b[1] - t.o[1];
    l2 = s.b[2] - t.o[2];
    return l0 >= 0 && l1 >= 0 && l2 >= 0 && l0 <= TILE - 3 && l1 <= TILE - 3 && l2 <= TILE - 3;
}

__device__ __noinline__ void p2g_particle_global(const Dev &d, const ActiveBuf &act, int par, const EnvDev &e,
                                                 const Stencil &s, float m, const float A[9], const float v[3])
{
    for (int o0 = 0; o0 < 3; ++o0)
        for (int o1 = 0; o1 < 3; ++o1)
            for (int o2 = 0; o2 < 3; ++o2) {
                float pm, p0, p1, p2;
                p2g_weights(e, s, m, A, v, o0, o1, o2, pm, p0, p1, p2);
                float *g = reinterpret_cast<float *>(d.gP + node_id(e, s.b[0] + o0, s.b[1] + o1, s.b[2] + o2));
                gatomic_add(g + 0, pm);
                gatomic_add(g + 1, p0);
                gatomic_add(g + 2, p1);
                gatomic_add(g + 3, p2);
            }
    mark_stencil_bricks(act, par, e, s.b);
}

// A = -dt V0 (4/dx^2) tau(F) + m C   (MLS force folded into the affine term)
__device__ __forceinline__ void affine_with_stress(const Dev &d, const EnvDev &e, int env, const float H[9],
                                                   const float C[9], float A[9], float &m)
{
    const float *mat = d.material + 4 * env;
    float E = gload(mat), nu = gload(mat + 1), rho = gload(mat + 2), V0 = gload(mat + 3);
    float mu, lam;
    lame(E, nu, mu, lam);
    m = rho * V0;
    float tau[9];
    if (kirchhoff(H, mu, lam, tau)) set_flag(d.status, env, MPM_FLAG_INVERTED);
    const float k = -d.dt * V0 * 4.0f * e.inv_dx * e.inv_dx;
#pragma unroll
    for (int c = 0; c < 9; ++c) A[c] = k * tau[c] + m * C[c];
}

// MODE 0: P2G only (head of a call; reads x, v, C, H).
// MODE 1: fused G2P(s) + F update + advection + P2G(s+1) (reads/writes x, H).
// MODE 2: G2P only (tail of a call; writes x, v, C, H).
template <int MODE>
__global__ __launch_bounds__(256) void k_tiled(Dev d, TiledArgs a)
{
    constexpr bool G2P = MODE >= 1, P2G = MODE <= 1;
    __shared__ float tm[P2G ? TILE_LDS : 1], tpx[P2G ? TILE_LDS : 1], tpy[P2G ? TILE_LDS : 1],
        tpz[P2G ? TILE_LDS : 1];
    __shared__ float tvx[G2P ? TILE_LDS : 1], tvy[G2P ? TILE_LDS : 1], tvz[G2P ? TILE_LDS : 1];
    __shared__ int touched;

    const int N = d.ntot, T = blockDim.x, tid = threadIdx.x;
    const int nitems = gload(a.totals).y;
    int first, stride, end;
    item_range(nitems, first, stride, end);
    for (int it = first; it < end; it += stride) {
        const int4 item = gload(a.items + it);
        EnvDev e;
        const Tile t = make_tile(d, a.act, item.x, e);
        // stage the tile
        for (int n = tid; n < TILE_NODES; n += T) {
            int la = n >> 6, lb = (n >> 3) & 7, lc = n & 7;
            int li = lds_index(la, lb, lc);
            if (P2G) { tm[li] = 0.f; tpx[li] = 0.f; tpy[li] = 0.f; tpz[li] = 0.f; }
            if (G2P) {
                int i = t.o[0] + la, j = t.o[1] + lb, k = t.o[2] + lc;
                float4 V = make_float4(0.f, 0.f, 0.f, 0.f);
                if (i >= 0 && j >= 0 && k >= 0 && i < e.n && j < e.n && k < e.n) V = gload(d.gV + node_id(e, i, j, k));
                tvx[li] = V.x; tvy[li] = V.y; tvz[li] = V.z;
            }
        }
        if (tid == 0) touched = 0;
        __syncthreads();

        for (int p = item.y + tid; p < item.y + item.z; p += T) {
            float x[3] = {gload(a.xin + p), gload(a.xin + N + p), gload(a.xin + 2 * N + p)};
            float H[9], v[3], C[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) H[c] = gload(a.Hin + (size_t)c * N + p);
            Stencil s;
            make_stencil(x[0], x[1], x[2], e.inv_dx, e.n, s);
            bool frozen = stencil_outside(s, e.n);
            if (frozen) {
                // out of the domain: state unchanged, no transfers
                set_flag(d.status, t.env, MPM_FLAG_OUT_OF_DOMAIN);
                if (a.xout != a.xin) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        gstore(a.xout + (size_t)c * N + p, x[c]);
                        gstore(a.vout + (size_t)c * N + p, gload(a.vin + (size_t)c * N + p));
                    }
#pragma unroll
                    for (int c = 0; c < 9; ++c) {
                        gstore(a.Hout + (size_t)c * N + p, H[c]);
                        gstore(a.Cout + (size_t)c * N + p, gload(a.Cin + (size_t)c * N + p));
                    }
                }
                if (a.pidout != a.pidin) gstore(a.pidout + p, gload(a.pidin + p));
                continue;
            }
            if (G2P) {
                int l0, l1, l2;
                if (stencil_in_tile(t, s, l0, l1, l2))
                    g2p_accumulate<true>(d, e, s, l0, l1, l2, tvx, tvy, tvz, v, C);
                else
                    g2p_accumulate<false>(d, e, s, 0, 0, 0, tvx, tvy, tvz, v, C);
                x[0] += d.dt * v[0];
                x[1] += d.dt * v[1];
                x[2] += d.dt * v[2];
                update_h(H, C, d.dt);
                if (inverted_h(H)) set_flag(d.status, t.env, MPM_FLAG_INVERTED);
                if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2])))
                    set_flag(d.status, t.env, MPM_FLAG_NONFINITE);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = gload(a.vin + (size_t)c * N + p);
#pragma unroll
                for (int c = 0; c < 9; ++c) C[c] = gload(a.Cin + (size_t)c * N + p);
            }
            bool write_vc = MODE == 2;
            if (P2G) {
                Stencil s2;
                if (G2P) make_stencil(x[0], x[1], x[2], e.inv_dx, e.n, s2); else s2 = s;
                if (stencil_outside(s2, e.n)) {
                    // leaves the domain now: freeze with this G2P's v, C
                    set_flag(d.status, t.env, MPM_FLAG_OUT_OF_DOMAIN);
                    write_vc = true;
                } else {
                    float A[9], m;
                    affine_with_stress(d, e, t.env, H, C, A, m);
                    int l0, l1, l2;
                    if (stencil_in_tile(t, s2, l0, l1, l2)) {
#pragma unroll
                        for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
                            for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
                                for (int o2 = 0; o2 < 3; ++o2) {
                                    float pm, p0, p1, p2;
                                    p2g_weights(e, s2, m, A, v, o0, o1, o2, pm, p0, p1, p2);
                                    int li = lds_index(l0 + o0, l1 + o1, l2 + o2);
                                    atomicAdd(&tm[li], pm);
                                    atomicAdd(&tpx[li], p0);
                                    atomicAdd(&tpy[li], p1);
                                    atomicAdd(&tpz[li], p2);
                                }
                    } else {
                        p2g_particle_global(d, a.act, a.par, e, s2, m, A, v);
                    }
                }
            }
            if (G2P) {
#pragma unroll
                for (int c = 0; c < 3; ++c) gstore(a.xout + (size_t)c * N + p, x[c]);
#pragma unroll
                for (int c = 0; c < 9; ++c) gstore(a.Hout + (size_t)c * N + p, H[c]);
                if (write_vc) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) gstore(a.vout + (size_t)c * N + p, v[c]);
#pragma unroll
                    for (int c = 0; c < 9; ++c) gstore(a.Cout + (size_t)c * N + p, C[c]);
                }
                if (a.pidout != a.pidin) gstore(a.pidout + p, gload(a.pidin + p));
            }
        }

        if (P2G) {
            __syncthreads();
            // flush non-empty tile nodes; remember which node bricks were hit
            for (int n = tid; n < TILE_NODES; n += T) {
                int la = n >> 6, lb = (n >> 3) & 7, lc = n & 7;
                int li = lds_index(la, lb, lc);
                float pm = tm[li];
                if (pm != 0.f) {
                    int i = t.o[0] + la, j = t.o[1] + lb, k = t.o[2] + lc;
                    float *g = reinterpret_cast<float *>(d.gP + node_id(e, i, j, k));
                    float q0 = tpx[li], q1 = tpy[li], q2 = tpz[li];
                    gatomic_add(g + 0, pm);
                    gatomic_add(g + 1, q0);
                    gatomic_add(g + 2, q1);
                    gatomic_add(g + 3, q2);
                    int bit = (((i >> 2) - t.bi + 1) * 3 + ((j >> 2) - t.bj + 1)) * 3 + ((k >> 2) - t.bk + 1);
                    atomicOr(&touched, 1 << bit);
                }
            }
            __syncthreads();
            if (tid < 27 && ((touched >> tid) & 1)) {
                int bi = t.bi - 1 + tid / 9, bj = t.bj - 1 + (tid / 3) % 3, bk = t.bk - 1 + tid % 3;
                mark_brick(a.act, a.par, e.bofs + (bi * e.nb + bj) * e.nb + bk);
            }
        }
        __syncthreads();
    }
    if (G2P) advance_end_of_substep(d);
    // the tail ends a call: both active lists start empty at the next head
    if (MODE == 2 && blockIdx.x == 0 && tid < 2) gstore(a.act.count + tid, 0);
}

// Grid operation over the active node bricks of list `par`: one wavefront
// per 4^3 brick.  Writes V, clears P and the brick's flag; clears the other
// list's count for the next P2G.
__global__ __launch_bounds__(256) void k_grid_active(Dev d, ActiveBuf a, int par)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int cnt = gload(a.count + par);
    const int32_t *list = a.list + (size_t)par * a.stride;
    for (int i = blockIdx.x * nw + wave; i < cnt; i += gridDim.x * nw) {
        int b = gload(list + i);
        int env = env_of_brick(a.env_bofs, d.n_envs, b);
        const EnvDev e = load_env(d.env + env);
        int lb = b - e.bofs;
        int gi, gj, gk;
        brick_local_to_ijk(e, lb, lane, gi, gj, gk);
        int64_t g = e.gofs + (int64_t)lb * 64 + lane;
        float4 P = gload(d.gP + g);
        float3 v = grid_node_velocity(d, e, env, P, gi, gj, gk, nullptr);
        gstore(d.gV + g, make_float4(v.x, v.y, v.z, 0.f));
        gstore(d.gP + g, make_float4(0.f, 0.f, 0.f, 0.f));
        if (lane == 0) gstore(a.flag + b, 0);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) gstore(a.count + (par ^ 1), 0);
}

void launch_p2g_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_tiled<0>, dim3(nblocks), dim3(block), 0, st, d, a);
}

void launch_fused_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_tiled<1>, dim3(nblocks), dim3(block), 0, st, d, a);
}

void launch_g2p_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_tiled<2>, dim3(nblocks), dim3(block), 0, st, d, a);
}

int tiled_workgroups(int block)
{
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0) cus = p.multiProcessorCount;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tiled<1>, block, 0) != hipSuccess || per < 1) per = 1;
    int g = per * cus;
    g -= g % NXCD;
    return g < NXCD ? NXCD : g;
}

void launch_grid_active(const Dev &d, const ActiveBuf &a, int par, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_grid_active, dim3(nblocks), dim3(256), 0, st, d, a, par);
}

}  // namespace mpm
