// Device helpers shared by the tiled forward and adjoint kernels: brick
// tiles, the XCD-aware item walk, active-brick marking and the per-particle
// payload handed from a particle pass to a node pass.
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
    t.o[0] = 4 * t.bi;
    t.o[1] = 4 * t.bj;
    t.o[2] = 4 * t.bk;
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

// Per-particle P2G inputs handed from the particle pass to the node pass of
// the same wavefront: fx and m, m v with the packed flags, and the affine
// matrix A dx with the absolute stencil base.
struct Payload {
    float4 f_m;        // fx0, fx1, fx2, m
    float4 mv_bits;    // m v, bits (1: valid, 2: stencil inside the tile)
    float4 a0, a1, a2; // rows of A dx, .w = stencil base b0, b1, b2
};
constexpr int PAY_VALID = 1, PAY_IN_TILE = 2;

// Quadratic B-spline of u = fx - o (|u| < 1.5).
__device__ __forceinline__ float bspline2(float u)
{
    float a = fabsf(u);
    return a < 0.5f ? 0.75f - a * a : 0.5f * (1.5f - a) * (1.5f - a);
}

}  // namespace mpm
