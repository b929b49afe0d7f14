// Device helpers shared by the tiled forward and adjoint kernels: brick
// tiles, the XCD-aware item walk, listing of far bricks, and the node pass
// (a particle pass hands each particle's payload to lanes = stencil nodes).
#pragma once
#include "mpm_tiled.h"

namespace mpm {

constexpr int NXCD = 8;

struct Tile {
    int env;
    int bi, bj, bk;   // brick coordinates
    int o[3];         // node coordinates of tile corner (0,0,0) = 4*brick
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

// Tile of work item (brick, first slot, count, environment) whose
// environment entry e is at hand.
__device__ __forceinline__ Tile tile_of(const int4 &item, const EnvDev &e)
{
    Tile t;
    t.env = item.w;
    int lb = item.x - e.bofs;
    t.bk = lb % e.nb;
    int r = lb / e.nb;
    t.bj = r % e.nb;
    t.bi = r / e.nb;
    t.o[0] = 4 * t.bi;
    t.o[1] = 4 * t.bj;
    t.o[2] = 4 * t.bk;
    return t;
}

// Tile of a work item, loading its environment's entry into e.
__device__ __forceinline__ Tile make_tile(const Dev &d, const int4 &item, EnvDev &e)
{
    e = load_env(d.env + item.w);
    return tile_of(item, e);
}

// Item walk: workgroup x + NXCD r runs on XCD x (workgroups are dealt to the
// XCDs round-robin) and takes every (G / NXCD)-th item, from its r-th on, of
// the contiguous eighth of the (spatially ordered) item list that belongs to
// XCD x, so neighbouring tiles, which share halo nodes, meet in one L2.
__device__ __forceinline__ void item_range(int nitems, int &first, int &stride, int &end)
{
    const int G = gridDim.x;         // multiple of NXCD
    const int x = blockIdx.x % NXCD, r = blockIdx.x / NXCD;
    const int per = (nitems + NXCD - 1) / NXCD;
    first = x * per + r;
    end = min(nitems, (x + 1) * per);
    stride = G / NXCD;
}

// A stencil reached brick b (of environment env, whose bricks start at
// bofs) outside the static neighbourhood of the particle's sort-time brick:
// list b once for the next grid operation (flag 2, and an entry in dynamic
// list `par`, or in the environment's run list in the persistent kernel).
__device__ __forceinline__ void mark_far_brick(const ActiveBuf &act, int par, int b, int env, int bofs)
{
    if (!act.flag) return;   // no bookkeeping (tape recompute)
    if (!gatomic_cas(act.flag + b, 0, 2)) return;
    if (act.elist) {
        const int slot = gatomic_add(act.ecount + env, 1);
        cstore(act.elist + bofs + slot, b);
    } else {
        const int slot = gatomic_add(act.dcount + par, 1);
        gstore(act.dlist + (size_t)par * act.nbricks + slot, b);
    }
}

// Grid barrier of a persistent run.  Every wavefront's loads, stores and
// atomics have completed before its workgroup arrives; a workgroup counts
// itself on its XCD's counter, the last of an XCD counts the XCD on the global
// counter, and the last XCD writes gen into every XCD's release word; each
// workgroup waits for its XCD's (bounded spin: a timeout sets
// MPM_FLAG_BARRIER_TIMEOUT and returns false).  Arrivals and polls never share
// a line, and each release word has one XCD's workgroups polling it.
__device__ __forceinline__ bool run_barrier(const Dev &d, unsigned *ctr, unsigned gen, int spin_limit, int &ok_shared)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        unsigned *g = ctr + NXCD * RUN_BARRIER_LINE;
        unsigned *rel = ctr + (NXCD + 2) * RUN_BARRIER_LINE;
        const unsigned per = gridDim.x / NXCD, x = blockIdx.x % NXCD;
        if (__hip_atomic_fetch_add(gptr(ctr + x * RUN_BARRIER_LINE), 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) + 1 == gen * per)
            if (__hip_atomic_fetch_add(gptr(g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == gen * NXCD)
                for (int q = 0; q < NXCD; ++q)
                    __hip_atomic_store(gptr(rel + q * RUN_BARRIER_LINE), gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1, spins = 0;
        while (__hip_atomic_load(gptr(rel + x * RUN_BARRIER_LINE), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
            if (++spins > spin_limit) { ok = 0; break; }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (!ok) set_flag(d.status, 0, MPM_FLAG_BARRIER_TIMEOUT);
        ok_shared = ok;
    }
    __syncthreads();
    return ok_shared != 0;
}

// End of a persistent run: the last workgroup out zeroes the barrier's
// counters for the next run (every other workgroup has left its last wait).
__device__ __forceinline__ void run_exit(unsigned *bar)
{
    if (threadIdx.x != 0) return;
    unsigned *ex = bar + (NXCD + 1) * RUN_BARRIER_LINE;
    if (__hip_atomic_fetch_add(gptr(ex), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == gridDim.x)
        for (int q = 0; q < 2 * NXCD + 2; ++q)
            __hip_atomic_store(gptr(bar + q * RUN_BARRIER_LINE), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool stencil_in_tile(const Tile &t, const Stencil &s, int &l0, int &l1, int &l2)
{
    l0 = s.b[0] - t.o[0];
    l1 = s.b[1] - t.o[1];
    l2 = s.b[2] - t.o[2];
    return l0 >= 0 && l1 >= 0 && l2 >= 0 && l0 <= TILE - 3 && l1 <= TILE - 3 && l2 <= TILE - 3;
}

// The stencil's base relative to the 8^3 velocity tile of the grid-at-staging
// kernels (origin one node below the brick's), and whether the stencil lies in it.
__device__ __forceinline__ bool stencil_in_gtile(const Tile &t, const Stencil &s, int &l0, int &l1, int &l2)
{
    l0 = s.b[0] - t.o[0] + 1;
    l1 = s.b[1] - t.o[1] + 1;
    l2 = s.b[2] - t.o[2] + 1;
    return l0 >= 0 && l1 >= 0 && l2 >= 0 && l0 <= GTILE - 3 && l1 <= GTILE - 3 && l2 <= GTILE - 3;
}

// Per-particle inputs handed from a particle pass (lane = particle) to the
// node pass of the same workgroup (lane = stencil node), 72 bytes = four LDS
// vector reads of the payload and one of its side array.  Node o (integer
// offsets from the stencil base) receives w(o) (s, g + M (o - fx)); s is the
// particle mass in P2G and 1 (a touch count) in the G2P adjoint.  The
// particle pass stores g0 = g - M fx, so a node lane forms g0 + M o from
// integer offsets, and the third axis's three B-spline weights, which are
// the same for every lane of a particle.
struct Payload {
    float4 fk;   // fx0, fx1, third-axis weight at offset 0, key (an int, see below)
    float4 q1;   // g0, M00
    float4 q2;   // M01, M02, M10, M11
    float4 q3;   // M12, M20, M21, M22
};
// The side array holds the third-axis weights at offsets 1 and 2 (a float2 per
// payload: the payload stays 64 bytes, the LDS of the smaller workgroups
// within what six of them may hold per CU).
//
// key: >= 0: the stencil is inside the tile and the key is the tile index of
// its base; KEY_NONE: no particle; otherwise the stencil leaves the tile and
// bits 0-9, 10-19, 20-29 hold its absolute base (grids are at most 512 nodes
// per axis), bit 31 set.
constexpr int KEY_NONE = -1;

__device__ __forceinline__ int key_in_tile(int l0, int l1, int l2) { return (l0 * TILE + l1) * TILE + l2; }
__device__ __forceinline__ int key_global(const int b[3])
{
    return (int)(0x80000000u | (unsigned)b[0] | ((unsigned)b[1] << 10) | ((unsigned)b[2] << 20));
}

// w2: the third axis's weights at offsets 0, 1, 2 (the particle pass has them
// from its stencil).  G0 false (the plain form): the payload holds fx2 and g
// itself, the side array is not used, and the node pass forms g + M (o - fx)
// and the third-axis weights per lane.
template <bool G0 = true>
__device__ __forceinline__ void store_payload(Payload &P, float2 &wz, const float fx[3], const float w2[3], int key,
                                              const float g[3], const float M[9])
{
    if constexpr (G0) {
        float g0[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            g0[r] = fmaf(-M[3 * r], fx[0], fmaf(-M[3 * r + 1], fx[1], fmaf(-M[3 * r + 2], fx[2], g[r])));
        P.fk = make_float4(fx[0], fx[1], w2[0], __int_as_float(key));
        P.q1 = make_float4(g0[0], g0[1], g0[2], M[0]);
        wz = make_float2(w2[1], w2[2]);
    } else {
        P.fk = make_float4(fx[0], fx[1], fx[2], __int_as_float(key));
        P.q1 = make_float4(g[0], g[1], g[2], M[0]);
    }
    P.q2 = make_float4(M[1], M[2], M[3], M[4]);
    P.q3 = make_float4(M[5], M[6], M[7], M[8]);
}


// A payload slot without a particle.
__device__ __forceinline__ void payload_none(Payload &P) { P.fk.w = __int_as_float(KEY_NONE); }

// The absolute node of a stencil that leaves the tile: key's base + (o0, o1, o2).
__device__ __forceinline__ void key_node(int key, int o0, int o1, int o2, int &i, int &j, int &k)
{
    i = (key & 1023) + o0;
    j = ((key >> 10) & 1023) + o1;
    k = ((key >> 20) & 1023) + o2;
}

// One particle per half-wave step (node_pass1).  Lane o < 27 of each
// half-wave takes stencil node (o0, o1, o2); the quadratic B-spline of the
// first two offsets is alpha (fx - c)^2 + gamma (fx in [0.5, 1.5)), three
// constants instead of a branch; the third comes with the payload.
struct NodeLane1 {
    bool on;
    int o0, o1, o2, lo;   // lo: tile offset of the node from the stencil base
    float of[3];          // the offsets as floats
    float wc[2], wa[2], wg[2];
};

// An opaque copy of a value: the out-of-tile path of the node pass is rare, and
// taking its key through this keeps the compiler from hoisting that path's
// node-index arithmetic into the common (in-tile) path of every step.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ NodeLane1 node_lane1(int lane)
{
    NodeLane1 L;
    const int o = lane & 31;
    L.on = o < 27;
    L.o0 = o / 9; L.o1 = (o / 3) % 3; L.o2 = o % 3;
    L.lo = (L.o0 * TILE + L.o1) * TILE + L.o2;
    const int oo[3] = {L.o0, L.o1, L.o2};
#pragma unroll
    for (int k = 0; k < 3; ++k) L.of[k] = (float)oo[k];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        L.wc[k] = 1.5f - 0.5f * oo[k];
        L.wa[k] = oo[k] == 1 ? -1.0f : 0.5f;
        L.wg[k] = oo[k] == 1 ? 0.75f : 0.0f;
    }
    return L;
}

// node_pass1: the node pass of one half-wave over payloads [r0, r1), one
// particle per step.  Consecutive particles with the same stencil (the sort
// groups particles by cell) are summed in registers and the sum is added to
// the half-wave's own LDS tile with a plain read-modify-write when the
// stencil changes: the 27 lanes touch 27 distinct nodes and no other
// half-wave writes the tile, so no atomic is needed.  A stencil outside the
// tile goes to `outside(c4, i, j, k)` (node indices).
template <bool G0, class Outside>
__device__ __forceinline__ void node_pass1(const Payload *pay, const float2 *wzs, int r0, int r1, float4 *tile,
                                           int lane, float s, Outside &&outside)
{
    const NodeLane1 L = node_lane1(lane);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int cur = -1;
    for (int r = r0; L.on && r < r1; ++r) {
        const Payload &P = pay[r];
        const float4 fk = P.fk, q1 = P.q1, q2 = P.q2, q3 = P.q3;
        const int key = __float_as_int(fk.w);
        if (key == KEY_NONE) continue;
        const float t0 = fk.x - L.wc[0], t1 = fk.y - L.wc[1];
        float w2, o[3];
        if constexpr (G0) {
            const float2 wz = wzs[r];
            w2 = L.o2 == 0 ? fk.z : (L.o2 == 1 ? wz.x : wz.y);
            o[0] = L.of[0]; o[1] = L.of[1]; o[2] = L.of[2];
        } else {
            const float t2 = fk.z - (1.5f - 0.5f * L.o2);
            w2 = L.o2 == 1 ? 0.75f - t2 * t2 : 0.5f * t2 * t2;
            o[0] = L.of[0] - fk.x; o[1] = L.of[1] - fk.y; o[2] = L.of[2] - fk.z;
        }
        const float w = fmaf(L.wa[0], t0 * t0, L.wg[0]) * fmaf(L.wa[1], t1 * t1, L.wg[1]) * w2;
        // the momentum term at this node before the weight
        const float gx = fmaf(q1.w, o[0], fmaf(q2.x, o[1], fmaf(q2.y, o[2], q1.x)));
        const float gy = fmaf(q2.z, o[0], fmaf(q2.w, o[1], fmaf(q3.x, o[2], q1.y)));
        const float gz = fmaf(q3.y, o[0], fmaf(q3.z, o[1], fmaf(q3.w, o[2], q1.z)));
        if (key >= 0) {
            const int l = key + L.lo;
            if (l != cur) {
                if (cur >= 0) {
                    float4 old = tile[cur];
                    tile[cur] = make_float4(old.x + acc.x, old.y + acc.y, old.z + acc.z, old.w + acc.w);
                }
                acc = make_float4(0.f, 0.f, 0.f, 0.f);
                cur = l;
            }
            acc.x = fmaf(w, s, acc.x); acc.y = fmaf(w, gx, acc.y); acc.z = fmaf(w, gy, acc.z); acc.w = fmaf(w, gz, acc.w);
        } else {
            int i, j, k;
            key_node(opaque(key), L.o0, L.o1, L.o2, i, j, k);
            outside(make_float4(w * s, w * gx, w * gy, w * gz), i, j, k);
        }
    }
    if (cur >= 0) {
        float4 old = tile[cur];
        tile[cur] = make_float4(old.x + acc.x, old.y + acc.y, old.z + acc.z, old.w + acc.w);
    }
}

// Three particles per half-wave step (node_pass3).  Lane o < 27 of a
// half-wave belongs to slot k = o / 9 (three particles are in flight per
// half-wave) and takes the stencil column (o0, o1) = ((o % 9) / 3, o % 3),
// i.e. the three nodes (o0, o1, 0..2).
struct NodeLane3 {
    bool on;
    int slot, o0, o1, lo;   // lo: tile offset of node (o0, o1, 0) from the stencil base
    float of0, of1;         // o0, o1 as floats
    float wc[2], wa[2], wg[2];
};

__device__ __forceinline__ NodeLane3 node_lane3(int lane)
{
    NodeLane3 L;
    const int o = lane & 31;
    L.on = o < 27;
    L.slot = o / 9;
    L.o0 = (o % 9) / 3;
    L.o1 = o % 3;
    L.lo = (L.o0 * TILE + L.o1) * TILE;
    L.of0 = (float)L.o0;
    L.of1 = (float)L.o1;
    const int oo[2] = {L.o0, L.o1};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        L.wc[k] = 1.5f - 0.5f * oo[k];
        L.wa[k] = oo[k] == 1 ? -1.0f : 0.5f;
        L.wg[k] = oo[k] == 1 ? 0.75f : 0.0f;
    }
    return L;
}

// node_pass3: the node pass of one half-wave over payloads [r0, r1): the
// run is cut into three contiguous parts, one per slot, processed side by
// side (one particle per slot per step).  Consecutive particles of a slot with the same stencil
// (the sort groups particles by cell) are summed in registers, three nodes
// per lane; when a slot's stencil changes its sums are added to the
// half-wave's LDS tile with plain read-modify-writes, one slot after the
// other (a slot's 9 lanes x 3 nodes are 27 distinct nodes, and no other
// half-wave writes the tile), so no atomic is needed.  A stencil outside the
// tile goes to `outside(c4, i, j, k)` (node indices), node by node.
template <bool G0, class Outside>
__device__ __forceinline__ void node_pass3(const Payload *pay, const float2 *wzs, int r0, int r1, float4 *tile,
                                           int lane, float s, Outside &&outside)
{
    const NodeLane3 L = node_lane3(lane);
    const int per = (r1 - r0 + 2) / 3;
    const int my0 = r0 + L.slot * per, my1 = min(r1, my0 + per);
    float4 acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    int cur = -1;
    // add a slot's sums to the tile, slot by slot (only lanes with `go` write).
    // Per lane the three rounds are exclusive, so the compiler could merge them
    // into one; the memory barriers between them keep three separate LDS
    // read-modify-writes, executed in order by the wavefront, so slots that
    // share nodes never write them in the same instruction.
    auto flush = [&](bool go) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (go && L.slot == k) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float4 old = tile[cur + c];
                    tile[cur + c] = make_float4(old.x + acc[c].x, old.y + acc[c].y, old.z + acc[c].z, old.w + acc[c].w);
                }
            }
            asm volatile("" ::: "memory");
        }
    };
    for (int i = 0; i < per; ++i) {
        const int r = my0 + i;
        const bool live = L.on && r < my1;
        const int rr = live ? r : r0;
        const Payload &P = pay[rr];
        const float4 fk = P.fk, q1 = P.q1, q2 = P.q2, q3 = P.q3;
        // its own shift, not an offset from the payload's address
        const float2 wz = G0 ? wzs[opaque(rr)] : make_float2(0.f, 0.f);
        const int key = live ? __float_as_int(fk.w) : KEY_NONE;
        const bool in_tile = key >= 0;
        const int l = key + L.lo;
        const bool change = in_tile && l != cur;
        if (__ballot(change && cur >= 0)) flush(change && cur >= 0);
        if (change) {
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
            cur = l;
        }
        const float t0 = fk.x - L.wc[0], t1 = fk.y - L.wc[1];
        const float w01 = fmaf(L.wa[0], t0 * t0, L.wg[0]) * fmaf(L.wa[1], t1 * t1, L.wg[1]);
        float w[3], g[3][3];
        if constexpr (G0) {
            w[0] = w01 * fk.z; w[1] = w01 * wz.x; w[2] = w01 * wz.y;
            // g0 + M (o0, o1, c): the column's base term, then the third axis node by node
            g[0][0] = fmaf(q1.w, L.of0, fmaf(q2.x, L.of1, q1.x));
            g[0][1] = fmaf(q2.z, L.of0, fmaf(q2.w, L.of1, q1.y));
            g[0][2] = fmaf(q3.y, L.of0, fmaf(q3.z, L.of1, q1.z));
            g[1][0] = g[0][0] + q2.y; g[1][1] = g[0][1] + q3.x; g[1][2] = g[0][2] + q3.w;
            g[2][0] = g[1][0] + q2.y; g[2][1] = g[1][1] + q3.x; g[2][2] = g[1][2] + q3.w;
        } else {
            const float f2 = fk.z;
            w[0] = w01 * (0.5f * (1.5f - f2) * (1.5f - f2));
            w[1] = w01 * (0.75f - (f2 - 1.0f) * (f2 - 1.0f));
            w[2] = w01 * (0.5f * (f2 - 0.5f) * (f2 - 0.5f));
            // g + M (o - fx): the column's part, then the third axis node by node
            const float d0 = L.of0 - fk.x, d1 = L.of1 - fk.y;
            const float bx = fmaf(q1.w, d0, fmaf(q2.x, d1, q1.x));
            const float by = fmaf(q2.z, d0, fmaf(q2.w, d1, q1.y));
            const float bz = fmaf(q3.y, d0, fmaf(q3.z, d1, q1.z));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float d2 = c - f2;
                g[c][0] = fmaf(q2.y, d2, bx); g[c][1] = fmaf(q3.x, d2, by); g[c][2] = fmaf(q3.w, d2, bz);
            }
        }
        if (in_tile) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[c].x = fmaf(w[c], s, acc[c].x); acc[c].y = fmaf(w[c], g[c][0], acc[c].y);
                acc[c].z = fmaf(w[c], g[c][1], acc[c].z); acc[c].w = fmaf(w[c], g[c][2], acc[c].w);
            }
        } else if (key != KEY_NONE) {
            const int k = opaque(key);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int ni, nj, nk;
                key_node(k, L.o0, L.o1, c, ni, nj, nk);
                outside(make_float4(w[c] * s, w[c] * g[c][0], w[c] * g[c][1], w[c] * g[c][2]), ni, nj, nk);
            }
        }
    }
    flush(cur >= 0);
}

// Node pass with `slots` (1 or 3) particles in flight per half-wave: one
// particle per step keeps runs long at few particles per cell; three per step
// need a third of the arithmetic per node when cells hold many particles.
template <bool G0 = true, class Outside>
__device__ __forceinline__ void node_pass(int slots, const Payload *pay, const float2 *wz, int r0, int r1,
                                          float4 *tile, int lane, float s, Outside &&outside)
{
    if (slots == 3) node_pass3<G0>(pay, wz, r0, r1, tile, lane, s, outside);
    else node_pass1<G0>(pay, wz, r0, r1, tile, lane, s, outside);
}

// Half-wave hw of 2W takes the contiguous run [r0, r1) of a chunk of n payloads.
template <int W>
__device__ __forceinline__ void half_wave_run(int hw, int n, int &r0, int &r1)
{
    const int per = (n + 2 * W - 1) / (2 * W);
    r0 = hw * per;
    r1 = min(n, r0 + per);
}

}  // namespace mpm
