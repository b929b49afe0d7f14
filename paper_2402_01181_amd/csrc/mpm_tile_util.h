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

// Tile of work item (brick, first slot, count, environment).
__device__ __forceinline__ Tile make_tile(const Dev &d, const int4 &item, EnvDev &e)
{
    Tile t;
    t.env = item.w;
    e = load_env(d.env + t.env);
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

// A stencil reached brick b outside the static neighbourhood of the
// particle's sort-time brick: list b once for the next grid operation.
__device__ __forceinline__ void mark_far_brick(const ActiveBuf &act, int par, int b)
{
    if (!act.flag) return;   // no bookkeeping (tape recompute)
    if (gatomic_cas(act.flag + b, 0, 2)) {
        int slot = gatomic_add(act.dcount + par, 1);
        gstore(act.dlist + (size_t)par * act.nbricks + slot, b);
    }
}

__device__ __forceinline__ bool stencil_in_tile(const Tile &t, const Stencil &s, int &l0, int &l1, int &l2)
{
    l0 = s.b[0] - t.o[0];
    l1 = s.b[1] - t.o[1];
    l2 = s.b[2] - t.o[2];
    return l0 >= 0 && l1 >= 0 && l2 >= 0 && l0 <= TILE - 3 && l1 <= TILE - 3 && l2 <= TILE - 3;
}

// Per-particle inputs handed from a particle pass (lane = particle) to the
// node pass of the same workgroup (lane = stencil node), 64 bytes = four LDS
// vector reads: fx and a packed key, a 3-vector g, and a 3x3 matrix M row by
// row.  Node o of the stencil receives w(o) (s, g + M (o - fx)); s is the
// particle mass in P2G and 1 (a touch count) in the G2P adjoint.
struct Payload4 {
    float4 fk;         // fx0, fx1, fx2, key
    float4 q1;         // g, M00
    float4 q2;         // M01, M02, M10, M11
    float4 q3;         // M12, M20, M21, M22
};
// key: bit 0 valid; bit 1 stencil inside the tile, then bits 2.. hold the
// tile index of the stencil base; otherwise bits 2-11, 12-21, 22-31 hold the
// absolute base (grids are at most 512 nodes per axis).
constexpr int KEY_VALID = 1, KEY_IN_TILE = 2;

__device__ __forceinline__ int key_in_tile(int l0, int l1, int l2)
{
    return KEY_VALID | KEY_IN_TILE | (((l0 * TILE + l1) * TILE + l2) << 2);
}
__device__ __forceinline__ int key_global(const int b[3])
{
    return KEY_VALID | (b[0] << 2) | (b[1] << 12) | (b[2] << 22);
}

__device__ __forceinline__ void store_payload(Payload4 &P, const float fx[3], int key, const float g[3],
                                              const float M[9])
{
    P.fk = make_float4(fx[0], fx[1], fx[2], __int_as_float(key));
    P.q1 = make_float4(g[0], g[1], g[2], M[0]);
    P.q2 = make_float4(M[1], M[2], M[3], M[4]);
    P.q3 = make_float4(M[5], M[6], M[7], M[8]);
}

// Node-pass role of a lane: lane o < 27 of each half-wave takes stencil node
// (o0, o1, o2); the quadratic B-spline of that offset is alpha (fx - c)^2 +
// gamma per axis (fx in [0.5, 1.5)), three constants instead of a branch.
struct NodeLane {
    bool on;
    int o0, o1, o2, lo;   // lo: tile offset of the node from the stencil base
    float wc[3], wa[3], wg[3];
};

__device__ __forceinline__ NodeLane node_lane_of(int lane)
{
    NodeLane L;
    const int o = lane & 31;
    L.on = o < 27;
    L.o0 = o / 9; L.o1 = (o / 3) % 3; L.o2 = o % 3;
    L.lo = (L.o0 * TILE + L.o1) * TILE + L.o2;
    const int oo[3] = {L.o0, L.o1, L.o2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        L.wc[k] = 1.5f - 0.5f * oo[k];
        L.wa[k] = oo[k] == 1 ? -1.0f : 0.5f;
        L.wg[k] = oo[k] == 1 ? 0.75f : 0.0f;
    }
    return L;
}

// Node pass of one half-wave over payloads [r0, r1).  Consecutive particles
// with the same stencil (the sort groups particles by cell) are summed in
// registers and the sum is added to the half-wave's own LDS tile with a plain
// read-modify-write when the stencil changes: the 27 lanes touch 27 distinct
// nodes and no other half-wave writes the tile, so no atomic is needed.  A
// stencil outside the tile goes to `outside(c4, i, j, k)` (node indices).
template <class Outside>
__device__ __forceinline__ void node_pass(const Payload4 *pay, int r0, int r1, float4 *tile, const NodeLane &L,
                                          float s, Outside &&outside)
{
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int cur = -1;
    for (int r = r0; L.on && r < r1; ++r) {
        const Payload4 &P = pay[r];
        const float4 fk = P.fk, q1 = P.q1, q2 = P.q2, q3 = P.q3;
        const int pk = __float_as_int(fk.w);
        const float t0 = fk.x - L.wc[0], t1 = fk.y - L.wc[1], t2 = fk.z - L.wc[2];
        const float w = fmaf(L.wa[0], t0 * t0, L.wg[0]) * fmaf(L.wa[1], t1 * t1, L.wg[1]) *
                        fmaf(L.wa[2], t2 * t2, L.wg[2]);
        const float d0 = L.o0 - fk.x, d1 = L.o1 - fk.y, d2 = L.o2 - fk.z;
        float4 c4;
        c4.x = w * s;
        c4.y = w * fmaf(q1.w, d0, fmaf(q2.x, d1, fmaf(q2.y, d2, q1.x)));
        c4.z = w * fmaf(q2.z, d0, fmaf(q2.w, d1, fmaf(q3.x, d2, q1.y)));
        c4.w = w * fmaf(q3.y, d0, fmaf(q3.z, d1, fmaf(q3.w, d2, q1.z)));
        if (!(pk & KEY_VALID)) continue;
        if (pk & KEY_IN_TILE) {
            const int l = (pk >> 2) + L.lo;
            if (l != cur) {
                if (cur >= 0) {
                    float4 old = tile[cur];
                    tile[cur] = make_float4(old.x + acc.x, old.y + acc.y, old.z + acc.z, old.w + acc.w);
                }
                acc = make_float4(0.f, 0.f, 0.f, 0.f);
                cur = l;
            }
            acc.x += c4.x; acc.y += c4.y; acc.z += c4.z; acc.w += c4.w;
        } else {
            outside(c4, ((pk >> 2) & 1023) + L.o0, ((pk >> 12) & 1023) + L.o1, ((pk >> 22) & 1023) + L.o2);
        }
    }
    if (cur >= 0) {
        float4 old = tile[cur];
        tile[cur] = make_float4(old.x + acc.x, old.y + acc.y, old.z + acc.z, old.w + acc.w);
    }
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
