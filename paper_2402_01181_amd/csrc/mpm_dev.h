// Device-side data structures and per-particle / per-node math of the HIP
// path.  gfx950 only; FP32 arithmetic with FP64 for det F and ln J.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpm.h"

namespace mpm {

constexpr int BRICK = 4;            // grid bricks are 4x4x4 nodes = 64 nodes = one wavefront
constexpr int BRICK_NODES = 64;
constexpr int MAX_TOOLS = 8;
constexpr double J_MIN = 1e-6;

// One environment: its particle range, its grid slice and constants.
struct EnvDev {
    int32_t n;        // nodes per axis
    int32_t nb;       // bricks per axis = n / 4
    int32_t pofs;     // first particle (global index)
    int32_t np;       // particle count
    int64_t gofs;     // first node of this environment's grid slice (multiple of 64)
    int32_t bofs;     // first brick (global brick id)
    int32_t bound;
    float dx, inv_dx;
    int32_t pad[2];
};

// One tool slot; T and k advance on the device once per substep.
struct ToolDev {
    int32_t active, shape, contact, n_traj;
    float radius, half_len, friction, theta;
    float R[9];
    int32_t k;              // substeps taken since the slot was set
    const float *u;         // caller-owned [n_traj][3]
    double T[3];            // FP64 position of the tool origin
};

// Everything a kernel needs, passed by value.
struct Dev {
    int32_t n_envs, max_tools, ntot, pad0;
    float dt, gx, gy, gz;
    const EnvDev *env;        // [n_envs]
    const int32_t *env_pofs;  // [n_envs + 1] particle offsets
    const float *material;    // [n_envs][4] E, nu, rho, V0
    ToolDev *tools;           // [n_envs][max_tools]
    uint32_t *status;         // [n_envs]
    int32_t *step;            // [n_envs] substeps taken
    // particle state, SoA component-major [comp][ntot]
    float *x, *v, *C, *F;
    int32_t *pid;             // original index of the particle held in each slot
    // grid: P = (m, mv) and V = (v, 0) as float4 over all environments
    float4 *gP, *gV;
};

__device__ __forceinline__ int env_of_particle(const Dev &d, int q)
{
    int lo = 0, hi = d.n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d.env_pofs[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Node (i,j,k) of an environment -> global node index (brick-major layout).
__device__ __forceinline__ int64_t node_id(const EnvDev &e, int i, int j, int k)
{
    int b = ((i >> 2) * e.nb + (j >> 2)) * e.nb + (k >> 2);
    return e.gofs + (int64_t)b * BRICK_NODES + ((i & 3) << 4) + ((j & 3) << 2) + (k & 3);
}

__device__ __forceinline__ void brick_local_to_ijk(const EnvDev &e, int b, int l, int &i, int &j, int &k)
{
    int bk = b % e.nb, t = b / e.nb;
    int bj = t % e.nb, bi = t / e.nb;
    i = bi * 4 + (l >> 4);
    j = bj * 4 + ((l >> 2) & 3);
    k = bk * 4 + (l & 3);
}

// Quadratic B-spline stencil of a particle: base node and per-axis weights.
// `outside` is decided in floating point before any index is formed: the
// 3x3x3 stencil fits the n^3 grid iff 0 <= x/dx - 0.5 < n - 2 on every axis
// (false for NaN and infinities, so no index is built from them).
struct Stencil {
    int b[3];
    float fx[3];
    float w[3][3];
    bool outside;
};

__device__ __forceinline__ void make_stencil(float x0, float x1, float x2, float inv_dx, int n, Stencil &s)
{
    float xs[3] = {x0, x1, x2};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float t = xs[a] * inv_dx;
        float tb = t - 0.5f;
        ok = ok && (tb >= 0.0f) && (tb < (float)(n - 2));
        float bf = floorf(fminf(fmaxf(tb, 0.0f), (float)(n - 3)));
        s.b[a] = (int)bf;
        float f = t - bf;
        s.fx[a] = f;
        s.w[a][0] = 0.5f * (1.5f - f) * (1.5f - f);
        s.w[a][1] = 0.75f - (f - 1.0f) * (f - 1.0f);
        s.w[a][2] = 0.5f * (f - 0.5f) * (f - 0.5f);
    }
    s.outside = !ok;
}

__device__ __forceinline__ bool stencil_outside(const Stencil &s, int) { return s.outside; }

// Lame parameters from (E, nu).
__device__ __forceinline__ void lame(float E, float nu, float &mu, float &lam)
{
    mu = E / (2.0f * (1.0f + nu));
    lam = E * nu / ((1.0f + nu) * (1.0f - 2.0f * nu));
}

// Neo-Hookean Kirchhoff stress tau = mu (F F^T - I) + lam ln J I, with
// F F^T - I formed from G = F - I as G + G^T + G G^T to avoid cancellation.
// J and ln J in FP64.  Returns true if J <= J_MIN (then ln J_MIN is used).
__device__ __forceinline__ bool kirchhoff(const float F[9], float mu, float lam, float tau[9])
{
    double J = (double)F[0] * ((double)F[4] * F[8] - (double)F[5] * F[7]) -
               (double)F[1] * ((double)F[3] * F[8] - (double)F[5] * F[6]) +
               (double)F[2] * ((double)F[3] * F[7] - (double)F[4] * F[6]);
    bool inv = !(J > J_MIN);
    double lnJ = log(inv ? J_MIN : J);
    float G[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) G[3 * a + b] = F[3 * a + b] - (a == b ? 1.0f : 0.0f);
    float p = (float)((double)lam * lnJ);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            float s = G[3 * a + b] + G[3 * b + a];
#pragma unroll
            for (int c = 0; c < 3; ++c) s = fmaf(G[3 * a + c], G[3 * b + c], s);
            float t = mu * s + (a == b ? p : 0.0f);
            tau[3 * a + b] = t;
            tau[3 * b + a] = t;
        }
    return inv;
}

__device__ __forceinline__ double det3d(const float F[9])
{
    return (double)F[0] * ((double)F[4] * F[8] - (double)F[5] * F[7]) -
           (double)F[1] * ((double)F[3] * F[8] - (double)F[5] * F[6]) +
           (double)F[2] * ((double)F[3] * F[7] - (double)F[4] * F[6]);
}

// Grid operation of one node with mass (Sec. III-B item 2, Sec. III-C):
// normalise + gravity, z-buffer over the environment's tools (nearest
// capsule, ties to the lowest slot), contact projection, boundary band.
// Writes the contact record used by the adjoint when rec != nullptr.
struct ContactRec {
    int tool;     // -1: no contact
    int branch;   // 0 unchanged, 1 friction, 2 tool velocity
};

__device__ __forceinline__ float3 tool_velocity(const ToolDev &t)
{
    int k = t.k < t.n_traj ? t.k : t.n_traj - 1;
    return make_float3(t.u[3 * k], t.u[3 * k + 1], t.u[3 * k + 2]);
}

// Capsule distance in the tool frame and world-frame unit normal.
__device__ __forceinline__ float capsule_phi(const ToolDev &t, float px, float py, float pz, float3 &nrm)
{
    float dx0 = (float)(px - t.T[0]), dx1 = (float)(py - t.T[1]), dx2 = (float)(pz - t.T[2]);
    // x_ref = R^T (x - T)
    float r0 = t.R[0] * dx0 + t.R[3] * dx1 + t.R[6] * dx2;
    float r1 = t.R[1] * dx0 + t.R[4] * dx1 + t.R[7] * dx2;
    float r2 = t.R[2] * dx0 + t.R[5] * dx1 + t.R[8] * dx2;
    float c = fminf(fmaxf(r0, -t.half_len), t.half_len);
    float q0 = r0 - c;
    float len = sqrtf(q0 * q0 + r1 * r1 + r2 * r2);
    float l0, l1, l2;
    if (len < 1e-12f) { l0 = 0.f; l1 = 1.f; l2 = 0.f; }
    else { float il = 1.0f / len; l0 = q0 * il; l1 = r1 * il; l2 = r2 * il; }
    nrm.x = t.R[0] * l0 + t.R[1] * l1 + t.R[2] * l2;
    nrm.y = t.R[3] * l0 + t.R[4] * l1 + t.R[5] * l2;
    nrm.z = t.R[6] * l0 + t.R[7] * l1 + t.R[8] * l2;
    return len - t.radius;
}

__device__ __forceinline__ float3 grid_node_velocity(const Dev &d, const EnvDev &e, int env, float4 P, int i,
                                                     int j, int k, ContactRec *rec)
{
    float3 v = make_float3(0.f, 0.f, 0.f);
    if (rec) { rec->tool = -1; rec->branch = 0; }
    if (!(P.x > 0.0f)) return v;
    v.x = P.y / P.x + d.dt * d.gx;
    v.y = P.z / P.x + d.dt * d.gy;
    v.z = P.w / P.x + d.dt * d.gz;
    bool wall = i < e.bound || j < e.bound || k < e.bound || i >= e.n - e.bound || j >= e.n - e.bound ||
                k >= e.n - e.bound;
    if (wall) return make_float3(0.f, 0.f, 0.f);
    if (d.max_tools > 0) {
        float px = i * e.dx, py = j * e.dx, pz = k * e.dx;
        const ToolDev *tl = d.tools + (size_t)env * d.max_tools;
        float best = INFINITY;
        int bt = -1;
        float3 bn = make_float3(0.f, 1.f, 0.f);
        for (int t = 0; t < d.max_tools; ++t) {
            if (!tl[t].active) continue;
            float3 nrm;
            float phi = capsule_phi(tl[t], px, py, pz, nrm);
            if (phi < best) { best = phi; bt = t; bn = nrm; }
        }
        if (bt >= 0 && best < tl[bt].theta) {
            const ToolDev &T = tl[bt];
            float3 u = tool_velocity(T);
            if (rec) rec->tool = bt;
            if (T.contact == MPM_CONTACT_STICKY) {
                v = u;
                if (rec) rec->branch = 2;
            } else {
                float r0 = v.x - u.x, r1 = v.y - u.y, r2 = v.z - u.z;
                float vn = r0 * bn.x + r1 * bn.y + r2 * bn.z;
                if (vn < 0.0f) {
                    float t0 = r0 - vn * bn.x, t1 = r1 - vn * bn.y, t2 = r2 - vn * bn.z;
                    float nt = sqrtf(t0 * t0 + t1 * t1 + t2 * t2);
                    float s = 0.0f;
                    if (nt > 0.0f) s = fmaxf(0.0f, 1.0f + T.friction * vn / nt);
                    if (rec) rec->branch = s > 0.0f ? 1 : 2;
                    v.x = s * t0 + u.x;
                    v.y = s * t1 + u.y;
                    v.z = s * t2 + u.z;
                }
            }
        }
    }
    return v;
}

__device__ __forceinline__ void set_flag(uint32_t *status, int env, uint32_t f)
{
    atomicOr(status + env, f);
}

}  // namespace mpm
