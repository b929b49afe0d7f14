/*
 * FP64 CPU oracle for the MLS-MPM Neo-Hookean tissue substep of
 * arXiv 2402.01181 (Sec. III-B "Material Point Method", Sec. III-C
 * "Collision Detection and Handling").
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg.  Plain serial loops, no blocking, fusion or
 * reordering beyond what the equations state.  Shares no code with the HIP
 * library.
 *
 * Readings of the paper (where it is silent, ambiguous or garbled):
 *  R1  Stress: the printed P = mu (F - F^T) + lambda log J F^-T is read as the
 *      compressible Neo-Hookean P = mu (F - F^-T) + lambda ln J F^-T (the
 *      printed F - F^T is antisymmetric and would give no stress under any
 *      stretch).  P F^T = mu (F F^T - I) + lambda ln J I is used directly.
 *  R2  The stress in the MLS force uses the current F; F is updated at the end
 *      of G2P as F <- (I + dt C_new) F.  ("1 + dt C" of the paper is I + dt C.)
 *  R3  Weights: quadratic B-spline, base = floor(x/dx - 0.5).
 *  R4  The 4/dx^2 factor is the inverse of the quadratic-B-spline inertia
 *      D_p = dx^2/4 I.
 *  R5  Gravity is added after normalisation: v_i = (mv)_i/m_i + dt g.
 *  R6  Domain boundary: sticky, v_i = 0 on nodes with any index < bound or
 *      >= n - bound; applied last in the grid operation.
 *  R7  Empty nodes (m_i == 0 exactly) get v_i = 0.
 *  R8  Grid-operation order: normalise, gravity, tool projection, boundary.
 *  R9  Contact iff the merged distance is < theta (per tool).
 *  R10 Tool distance, three shapes.  Capsule: analytic SDF (segment on the
 *      tool-frame x axis) with its analytic gradient as the normal.  Box (the
 *      gripper-jaw bounding box): analytic signed distance to a box of half
 *      extents b, optionally rounded by r.  Sampled SDF: a lattice of
 *      res^3 samples, sample (i,j,k) at lo + (i,j,k) h in the tool frame;
 *      "nearest" reads the sample of the lattice cell the node falls in,
 *      s = (x_ref - lo)/h, index floor(s) (the paper's SDF[x_ref/dx]), and
 *      takes the central-difference gradient of that sample as the normal;
 *      "trilinear" interpolates the samples and their central-difference
 *      gradients over the cell.  A node whose lattice cell has no complete
 *      central differences (index outside [1, res-2]) is outside the tool's
 *      field: no contact with that tool.  The lattice coordinate s is formed
 *      in FP64 (the kernels do the same), so both take the same cell.
 *  R11 Normal n = R grad/|grad|; on the capsule axis, or where the gradient
 *      vanishes (|grad| < 1e-12), n = R e_y.
 *  R12 Friction: Coulomb projection v_rel' = max(0, 1 + mu_f v_n/|v_t|) v_t,
 *      and 0 when |v_t| = 0 (the printed formula has no static clamp).
 *  R13 Slip contact projects only when v_n < 0; sticky contact sets the node
 *      velocity to the tool velocity whenever in contact.
 *  R14 Tool velocity field v_co = u (no rotation); pose advances every
 *      substep, T_{s+1} = T_s + dt u_s.
 *  R15 z-buffer over tools: strict < scanning ids upward, so ties go to the
 *      lowest id.
 *  R16 J <= 1e-6 flags INVERTED and the stress uses ln(1e-6).
 *  R17 A particle whose stencil leaves the grid (base < 0 or base + 2 > n - 1)
 *      flags OUT_OF_DOMAIN and takes no part in the transfers; its state is
 *      left unchanged.
 */
#include "mpm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(n, i, j, k) ((((size_t)(i)) * (size_t)(n) + (size_t)(j)) * (size_t)(n) + (size_t)(k))

static double det3(const double A[9])
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* Inverse-transpose via the cofactor matrix: F^-T = cof(F) / det F. */
static void inv_transpose3(const double A[9], double out[9])
{
    double d = det3(A);
    out[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    out[1] = -(A[3] * A[8] - A[5] * A[6]) / d;
    out[2] = (A[3] * A[7] - A[4] * A[6]) / d;
    out[3] = -(A[1] * A[8] - A[2] * A[7]) / d;
    out[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    out[5] = -(A[0] * A[7] - A[1] * A[6]) / d;
    out[6] = (A[1] * A[5] - A[2] * A[4]) / d;
    out[7] = -(A[0] * A[5] - A[2] * A[3]) / d;
    out[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

/* Lame parameters from Young's modulus and Poisson's ratio (Sec. III-B, the
 * mu / lambda equation). */
void orc_lame(double E, double nu, double *mu, double *lam)
{
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* Quadratic B-spline weights per axis (R3) and their derivatives with
 * respect to fx.  w[d][o] is the weight of node base[d] + o along axis d. */
void orc_weights(const double x[3], double inv_dx, int base[3], double fx[3], double w[3][3],
                 double dw[3][3])
{
    for (int d = 0; d < 3; ++d) {
        double s = x[d] * inv_dx;
        base[d] = (int)floor(s - 0.5);
        fx[d] = s - base[d];
        double f = fx[d];
        w[d][0] = 0.5 * (1.5 - f) * (1.5 - f);
        w[d][1] = 0.75 - (f - 1.0) * (f - 1.0);
        w[d][2] = 0.5 * (f - 0.5) * (f - 0.5);
        if (dw) {
            dw[d][0] = -(1.5 - f);
            dw[d][1] = -2.0 * (f - 1.0);
            dw[d][2] = f - 0.5;
        }
    }
}

/* Kirchhoff stress tau = P F^T of the Neo-Hookean model (R1, R16). */
uint32_t orc_kirchhoff(const double F[9], double mu, double lam, double tau[9])
{
    uint32_t flags = 0;
    double J = det3(F);
    if (!(J > ORC_J_MIN)) {
        flags |= ORC_FLAG_INVERTED;
        J = ORC_J_MIN;
    }
    double lnJ = log(J);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double FFt = 0.0;
            for (int c = 0; c < 3; ++c) FFt += F[3 * a + c] * F[3 * b + c];
            tau[3 * a + b] = mu * (FFt - (a == b ? 1.0 : 0.0)) + (a == b ? lam * lnJ : 0.0);
        }
    return flags;
}

/* Capsule signed distance in the tool frame (R10): distance from the segment
 * [-h, h] x e_x minus the radius.  q receives the offset from the closest
 * segment point; *interior tells whether the closest point is strictly inside
 * the segment. */
double orc_capsule_sdf(const double xref[3], double radius, double half_len, double q[3], int *interior)
{
    double c = xref[0];
    int in = 1;
    if (c < -half_len) { c = -half_len; in = 0; }
    if (c > half_len) { c = half_len; in = 0; }
    q[0] = xref[0] - c;
    q[1] = xref[1];
    q[2] = xref[2];
    if (interior) *interior = in;
    return sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) - radius;
}

/* Box of half extents b rounded by r (R10): outside the core box the offset
 * q = x_ref - clamp(x_ref, -b, b) gives phi = |q| - r and l = q/|q|; inside,
 * phi = max_a(|x_a| - b_a) - r with l = sign(x_k) e_k on the first axis k
 * reaching the maximum.  Jl = dl/dx_ref: (I - l l^T) D / |q| outside, with
 * D_aa = 1 on the axes the clamp is active on, and 0 inside. */
double orc_box_sdf(const double xref[3], const double half[3], double radius, double l[3], double Jl[9])
{
    double q[3];
    int outside = 0;
    for (int a = 0; a < 3; ++a) {
        double c = xref[a];
        if (c < -half[a]) c = -half[a];
        if (c > half[a]) c = half[a];
        q[a] = xref[a] - c;
        if (xref[a] < -half[a] || xref[a] > half[a]) outside = 1;
    }
    if (Jl) memset(Jl, 0, 9 * sizeof(double));
    if (outside) {
        double len = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        if (len < 1e-12) {
            l[0] = 0.0; l[1] = 1.0; l[2] = 0.0;
            return len - radius;
        }
        for (int a = 0; a < 3; ++a) l[a] = q[a] / len;
        if (Jl)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    int act = xref[b] < -half[b] || xref[b] > half[b];
                    Jl[3 * a + b] = act ? ((a == b ? 1.0 : 0.0) - l[a] * l[b]) / len : 0.0;
                }
        return len - radius;
    }
    int k = 0;
    double best = fabs(xref[0]) - half[0];
    for (int a = 1; a < 3; ++a)
        if (fabs(xref[a]) - half[a] > best) { best = fabs(xref[a]) - half[a]; k = a; }
    l[0] = l[1] = l[2] = 0.0;
    l[k] = xref[k] >= 0.0 ? 1.0 : -1.0;
    return best - radius;
}

static double sdf_at(const orc_tool *tl, int i, int j, int k)
{
    return (double)tl->sdf[((size_t)i * tl->sdf_res + j) * tl->sdf_res + k];
}

/* Central-difference gradient of the samples at lattice point (i,j,k)
 * (Sec. III-C, normal equation). */
static void sdf_grad(const orc_tool *tl, int i, int j, int k, double g[3])
{
    double h2 = 2.0 * tl->sdf_h;
    g[0] = (sdf_at(tl, i + 1, j, k) - sdf_at(tl, i - 1, j, k)) / h2;
    g[1] = (sdf_at(tl, i, j + 1, k) - sdf_at(tl, i, j - 1, k)) / h2;
    g[2] = (sdf_at(tl, i, j, k + 1) - sdf_at(tl, i, j, k - 1)) / h2;
}

/* Sampled SDF (R10).  Returns phi (INFINITY outside the field) with the
 * tool-frame unit normal l and Jl = dl/dx_ref. */
double orc_sampled_sdf(const orc_tool *tl, const double xref[3], double l[3], double Jl[9])
{
    const int tri = tl->sdf_interp == ORC_SDF_TRILINEAR;
    const double lim = tri ? tl->sdf_res - 2 : tl->sdf_res - 1;
    double s[3];
    int i0[3];
    if (Jl) memset(Jl, 0, 9 * sizeof(double));
    l[0] = 0.0; l[1] = 1.0; l[2] = 0.0;
    for (int a = 0; a < 3; ++a) {
        s[a] = (xref[a] - tl->sdf_lo[a]) / tl->sdf_h;
        if (!(s[a] >= 1.0 && s[a] < lim)) return INFINITY;
        i0[a] = (int)floor(s[a]);
    }
    double phi, g[3], dg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (!tri) {
        phi = sdf_at(tl, i0[0], i0[1], i0[2]);
        sdf_grad(tl, i0[0], i0[1], i0[2], g);
    } else {
        double f[3] = {s[0] - i0[0], s[1] - i0[1], s[2] - i0[2]};
        phi = 0.0;
        g[0] = g[1] = g[2] = 0.0;
        for (int c = 0; c < 8; ++c) {
            int o[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
            double wa[3], w = 1.0, gw[3];
            for (int a = 0; a < 3; ++a) {
                wa[a] = o[a] ? f[a] : 1.0 - f[a];
                w *= wa[a];
            }
            /* d w / d s_b */
            for (int b = 0; b < 3; ++b) {
                gw[b] = o[b] ? 1.0 : -1.0;
                for (int a = 0; a < 3; ++a)
                    if (a != b) gw[b] *= wa[a];
            }
            double Gc[3];
            sdf_grad(tl, i0[0] + o[0], i0[1] + o[1], i0[2] + o[2], Gc);
            phi += w * sdf_at(tl, i0[0] + o[0], i0[1] + o[1], i0[2] + o[2]);
            for (int a = 0; a < 3; ++a) {
                g[a] += w * Gc[a];
                for (int b = 0; b < 3; ++b) dg[3 * a + b] += Gc[a] * gw[b] / tl->sdf_h;
            }
        }
    }
    double gl = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (gl < 1e-12) return phi;
    for (int a = 0; a < 3; ++a) l[a] = g[a] / gl;
    if (Jl && tri)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0.0;
                for (int c = 0; c < 3; ++c) v += ((a == c ? 1.0 : 0.0) - l[a] * l[c]) * dg[3 * c + b];
                Jl[3 * a + b] = v / gl;
            }
    return phi;
}

static int out_of_domain(const int base[3], int n)
{
    for (int d = 0; d < 3; ++d)
        if (base[d] < 0 || base[d] + 2 > n - 1) return 1;
    return 0;
}

/* P2G (Sec. III-B item 1, Eq. P2G and Eq. fip) onto the node planes
 * i0 <= i < i1 of the grid (all of it: 0, n):
 *   m_i    = sum_p w_ip m_p
 *   (mv)_i = sum_p w_ip [ m_p v_p + m_p C_p (x_i - x_p) + f_ip dt ]
 *   f_ip dt = -dt V0 (4/dx^2) tau_p (x_i - x_p)
 * Every node receives its terms in particle order, whatever the planes.    */
static uint32_t p2g_planes(const orc_params *P, int32_t N, const double *x, const double *v, const double *C,
                           const double *F, double *gm, double *gmv, int i0, int i1)
{
    const int n = P->n;
    const double dx = 1.0 / n, inv_dx = (double)n, D = 4.0 * inv_dx * inv_dx;
    const double m = P->rho * P->V0;
    const size_t plane = (size_t)n * n;
    double mu, lam;
    uint32_t flags = 0;
    orc_lame(P->E, P->nu, &mu, &lam);
    memset(gm + (size_t)i0 * plane, 0, sizeof(double) * (size_t)(i1 - i0) * plane);
    memset(gmv + 3 * (size_t)i0 * plane, 0, sizeof(double) * 3 * (size_t)(i1 - i0) * plane);
    for (int p = 0; p < N; ++p) {
        int base[3];
        double fx[3], w[3][3], tau[9], A[9];
        orc_weights(x + 3 * p, inv_dx, base, fx, w, NULL);
        if (out_of_domain(base, n)) {
            flags |= ORC_FLAG_OUT_OF_DOMAIN;
            continue;
        }
        if (base[0] + 2 < i0 || base[0] >= i1) continue;   /* no node on these planes */
        flags |= orc_kirchhoff(F + 9 * p, mu, lam, tau);
        for (int k = 0; k < 9; ++k) A[k] = -P->dt * P->V0 * D * tau[k] + m * C[9 * p + k];
        for (int o0 = 0; o0 < 3; ++o0) {
            if (base[0] + o0 < i0 || base[0] + o0 >= i1) continue;
            for (int o1 = 0; o1 < 3; ++o1)
                for (int o2 = 0; o2 < 3; ++o2) {
                    double dpos[3] = {(o0 - fx[0]) * dx, (o1 - fx[1]) * dx, (o2 - fx[2]) * dx};
                    double wt = w[0][o0] * w[1][o1] * w[2][o2];
                    size_t i = IDX(n, base[0] + o0, base[1] + o1, base[2] + o2);
                    gm[i] += wt * m;
                    for (int a = 0; a < 3; ++a) {
                        double Ad = A[3 * a + 0] * dpos[0] + A[3 * a + 1] * dpos[1] + A[3 * a + 2] * dpos[2];
                        gmv[3 * i + a] += wt * (m * v[3 * p + a] + Ad);
                    }
                }
        }
    }
    return flags;
}

uint32_t orc_p2g(const orc_params *P, int32_t N, const double *x, const double *v, const double *C,
                 const double *F, double *gm, double *gmv)
{
    return p2g_planes(P, N, x, v, C, F, gm, gmv, 0, P->n);
}

/* World-frame contact normal of tool t at tool-frame offset q (R11). */
static void capsule_normal(const orc_tool *tl, const double q[3], double nrm[3])
{
    double len = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    double nl[3];
    if (len < 1e-12) {
        nl[0] = 0.0; nl[1] = 1.0; nl[2] = 0.0;
    } else {
        nl[0] = q[0] / len; nl[1] = q[1] / len; nl[2] = q[2] / len;
    }
    for (int a = 0; a < 3; ++a) nrm[a] = tl->R[3 * a + 0] * nl[0] + tl->R[3 * a + 1] * nl[1] + tl->R[3 * a + 2] * nl[2];
}

/* Grid operation (Sec. III-B item 2, Sec. III-C) for every node of the
 * planes i0 <= i < i1, with the tool poses T[t][3] and velocities u[t][3] of
 * this substep. */
static void grid_update_planes(const orc_params *P, const orc_tool *tools, const double *T, const double *u,
                               const double *gm, const double *gmv, double *gv, orc_node_rec *rec, int i0, int i1)
{
    const int n = P->n;
    const double dx = 1.0 / n;
    for (int i = i0; i < i1; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                size_t id = IDX(n, i, j, k);
                orc_node_rec r;
                memset(&r, 0, sizeof r);
                r.tool = -1;
                double vv[3] = {0.0, 0.0, 0.0};
                int wall = (i < P->bound || j < P->bound || k < P->bound || i >= n - P->bound ||
                            j >= n - P->bound || k >= n - P->bound);
                r.wall = wall;
                if (gm[id] > 0.0) {
                    for (int a = 0; a < 3; ++a) vv[a] = gmv[3 * id + a] / gm[id] + P->dt * P->g[a];
                    memcpy(r.vhat, vv, sizeof vv);
                    /* z-buffer: nearest tool, ties to the lowest id (R15) */
                    double xi[3] = {i * dx, j * dx, k * dx};
                    double best = INFINITY, bq[3] = {0, 0, 0}, bl[3] = {0, 1, 0}, bxr[3] = {0, 0, 0};
                    int bt = -1, bin = 0;
                    for (int t = 0; t < P->n_tools; ++t) {
                        const orc_tool *tl = &tools[t];
                        double d[3] = {xi[0] - T[3 * t + 0], xi[1] - T[3 * t + 1], xi[2] - T[3 * t + 2]};
                        double xr[3], q[3] = {0, 0, 0}, l[3] = {0, 1, 0}, phi;
                        int in = 0;
                        for (int a = 0; a < 3; ++a) xr[a] = tl->R[0 + a] * d[0] + tl->R[3 + a] * d[1] + tl->R[6 + a] * d[2];
                        if (tl->shape == ORC_TOOL_BOX) phi = orc_box_sdf(xr, tl->half, tl->radius, l, NULL);
                        else if (tl->shape == ORC_TOOL_SDF) phi = orc_sampled_sdf(tl, xr, l, NULL);
                        else phi = orc_capsule_sdf(xr, tl->radius, tl->half_len, q, &in);
                        if (phi < best) {
                            best = phi; bt = t; bin = in;
                            memcpy(bq, q, sizeof q); memcpy(bl, l, sizeof l); memcpy(bxr, xr, sizeof xr);
                        }
                    }
                    if (bt >= 0 && best < tools[bt].theta) {
                        const orc_tool *tl = &tools[bt];
                        const double *uc = u + 3 * bt;
                        double nrm[3];
                        if (tl->shape == ORC_TOOL_CAPSULE) capsule_normal(tl, bq, nrm);
                        else
                            for (int a = 0; a < 3; ++a)
                                nrm[a] = tl->R[3 * a + 0] * bl[0] + tl->R[3 * a + 1] * bl[1] + tl->R[3 * a + 2] * bl[2];
                        r.tool = bt;
                        memcpy(r.n, nrm, sizeof nrm);
                        memcpy(r.q, bq, sizeof bq);
                        memcpy(r.xr, bxr, sizeof bxr);
                        r.interior = bin;
                        if (tl->contact == ORC_CONTACT_STICKY) {
                            for (int a = 0; a < 3; ++a) vv[a] = uc[a];
                            r.branch = 2;
                        } else {
                            double vr[3] = {vv[0] - uc[0], vv[1] - uc[1], vv[2] - uc[2]};
                            double vn = vr[0] * nrm[0] + vr[1] * nrm[1] + vr[2] * nrm[2];
                            if (vn < 0.0) {
                                double vt[3] = {vr[0] - vn * nrm[0], vr[1] - vn * nrm[1], vr[2] - vn * nrm[2]};
                                double nt = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
                                double s = 0.0;
                                if (nt > 0.0) {
                                    s = 1.0 + tl->friction * vn / nt;
                                    if (s < 0.0) s = 0.0;
                                }
                                r.branch = (s > 0.0) ? 1 : 2;
                                for (int a = 0; a < 3; ++a) vv[a] = s * vt[a] + uc[a];
                            }
                        }
                    }
                    if (wall) vv[0] = vv[1] = vv[2] = 0.0;
                }
                for (int a = 0; a < 3; ++a) gv[3 * id + a] = vv[a];
                if (rec) rec[id] = r;
            }
}

void orc_grid_update(const orc_params *P, const orc_tool *tools, const double *T, const double *u,
                     const double *gm, const double *gmv, double *gv, orc_node_rec *rec)
{
    grid_update_planes(P, tools, T, u, gm, gmv, gv, rec, 0, P->n);
}

/* G2P and advection (Sec. III-B item 3) followed by the F update (R2) for
 * particles p0 <= p < p1:
 *   v_p = sum_i w_ip v_i,  C_p = (4/dx^2) sum_i w_ip v_i (x_i - x_p)^T,
 *   x_p += dt v_p,  F_p <- (I + dt C_p) F_p.                              */
static uint32_t g2p_range(const orc_params *P, int32_t p0, int32_t p1, double *x, double *v, double *C, double *F,
                          const double *gv)
{
    const int n = P->n;
    const double dx = 1.0 / n, inv_dx = (double)n, D = 4.0 * inv_dx * inv_dx;
    uint32_t flags = 0;
    for (int p = p0; p < p1; ++p) {
        int base[3];
        double fx[3], w[3][3];
        orc_weights(x + 3 * p, inv_dx, base, fx, w, NULL);
        if (out_of_domain(base, n)) {
            flags |= ORC_FLAG_OUT_OF_DOMAIN;
            continue;
        }
        double vp[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int o0 = 0; o0 < 3; ++o0)
            for (int o1 = 0; o1 < 3; ++o1)
                for (int o2 = 0; o2 < 3; ++o2) {
                    double dpos[3] = {(o0 - fx[0]) * dx, (o1 - fx[1]) * dx, (o2 - fx[2]) * dx};
                    double wt = w[0][o0] * w[1][o1] * w[2][o2];
                    const double *vi = gv + 3 * IDX(n, base[0] + o0, base[1] + o1, base[2] + o2);
                    for (int a = 0; a < 3; ++a) {
                        vp[a] += wt * vi[a];
                        for (int b = 0; b < 3; ++b) B[3 * a + b] += wt * vi[a] * dpos[b];
                    }
                }
        double Fn[9];
        for (int a = 0; a < 3; ++a) {
            v[3 * p + a] = vp[a];
            x[3 * p + a] += P->dt * vp[a];
            for (int b = 0; b < 3; ++b) C[9 * p + 3 * a + b] = D * B[3 * a + b];
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c)
                    s += ((a == c ? 1.0 : 0.0) + P->dt * C[9 * p + 3 * a + c]) * F[9 * p + 3 * c + b];
                Fn[3 * a + b] = s;
            }
        memcpy(F + 9 * p, Fn, sizeof Fn);
        if (!(det3(Fn) > ORC_J_MIN)) flags |= ORC_FLAG_INVERTED;
        for (int a = 0; a < 3; ++a)
            if (!isfinite(x[3 * p + a]) || !isfinite(v[3 * p + a])) flags |= ORC_FLAG_NONFINITE;
    }
    return flags;
}

uint32_t orc_g2p(const orc_params *P, int32_t N, double *x, double *v, double *C, double *F,
                 const double *gv)
{
    return g2p_range(P, 0, N, x, v, C, F, gv);
}

/* One substep with tool poses T (advanced in place, R14) and velocities u. */
uint32_t orc_substep(const orc_params *P, const orc_tool *tools, double *T, const double *u,
                     int32_t N, double *x, double *v, double *C, double *F,
                     double *gm, double *gmv, double *gv)
{
    uint32_t flags = orc_p2g(P, N, x, v, C, F, gm, gmv);
    orc_grid_update(P, tools, T, u, gm, gmv, gv, NULL);
    flags |= orc_g2p(P, N, x, v, C, F, gv);
    for (int t = 0; t < P->n_tools; ++t)
        for (int a = 0; a < 3; ++a) T[3 * t + a] += P->dt * u[3 * t + a];
    return flags;
}

/* Velocities of every tool at absolute substep s; traj is [n_tools][n_traj][3]
 * and the last entry is held beyond the end. */
static void traj_at(const orc_params *P, const double *traj, int32_t n_traj, int32_t s, double *u)
{
    int k = s < n_traj ? s : n_traj - 1;
    for (int t = 0; t < P->n_tools; ++t)
        for (int a = 0; a < 3; ++a) u[3 * t + a] = traj[((size_t)t * n_traj + k) * 3 + a];
}

uint32_t orc_run(const orc_params *P, const orc_tool *tools, const double *traj, int32_t n_traj,
                 int32_t s0, int32_t S, double *T, int32_t N, double *x, double *v, double *C,
                 double *F)
{
    size_t nn = (size_t)P->n * P->n * P->n;
    double *gm = malloc(sizeof(double) * nn), *gmv = malloc(sizeof(double) * 3 * nn),
           *gv = malloc(sizeof(double) * 3 * nn);
    double u[3 * 64];
    uint32_t flags = 0;
    for (int s = s0; s < s0 + S; ++s) {
        if (P->n_tools > 0) traj_at(P, traj, n_traj, s, u);
        flags |= orc_substep(P, tools, T, u, N, x, v, C, F, gm, gmv, gv);
    }
    free(gm); free(gmv); free(gv);
    return flags;
}

/* The substep of orc_run spread over threads (OpenMP), for timing the oracle
 * on a many-core host.  P2G: each thread owns a slab of node planes,
 * i in [cut[t], cut[t+1]), balanced by the particles whose stencils reach it,
 * and runs the plain P2G loop over all particles for its own nodes only; every
 * node still receives its terms in particle order, so the grid is the serial
 * one bit for bit (no private copies, nothing to reduce).  The grid operation
 * is split over planes and G2P over particles, both without shared writes.
 * The result equals orc_run's exactly. */
uint32_t orc_run_threads(const orc_params *P, const orc_tool *tools, const double *traj, int32_t n_traj,
                         int32_t s0, int32_t S, double *T, int32_t N, double *x, double *v, double *C,
                         double *F, int32_t nthreads)
{
    const int n = P->n;
    const size_t nn = (size_t)n * n * n;
    double *gm = malloc(sizeof(double) * nn), *gmv = malloc(sizeof(double) * 3 * nn),
           *gv = malloc(sizeof(double) * 3 * nn);
    int *hist = malloc(sizeof(int) * (size_t)(n + 1)), *cut = malloc(sizeof(int) * (size_t)(nthreads + 1));
    double u[3 * 64];
    uint32_t flags = 0;
    if (nthreads < 1) nthreads = 1;
    for (int s = s0; s < s0 + S; ++s) {
        if (P->n_tools > 0) traj_at(P, traj, n_traj, s, u);
        /* plane slabs with about equal numbers of (particle, plane) pairs */
        memset(hist, 0, sizeof(int) * (size_t)(n + 1));
        long long pairs = 0;
        for (int p = 0; p < N; ++p) {
            int b = (int)floor(x[3 * p] * n - 0.5);
            if (b < 0 || b + 2 > n - 1) continue;
            hist[b] += 1; hist[b + 1] += 1; hist[b + 2] += 1;
            pairs += 3;
        }
        cut[0] = 0;
        long long acc = 0;
        int t = 1;
        for (int i = 0; i < n && t < nthreads; ++i) {
            acc += hist[i];
            while (t < nthreads && acc * nthreads >= pairs * t) cut[t++] = i + 1;
        }
        while (t <= nthreads) cut[t++] = n;
        uint32_t f = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1) reduction(| : f)
        for (int k = 0; k < nthreads; ++k)
            if (cut[k] < cut[k + 1]) f |= p2g_planes(P, N, x, v, C, F, gm, gmv, cut[k], cut[k + 1]);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
        for (int i = 0; i < n; ++i) grid_update_planes(P, tools, T, u, gm, gmv, gv, NULL, i, i + 1);
        const int chunk = (N + nthreads - 1) / nthreads;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1) reduction(| : f)
        for (int k = 0; k < nthreads; ++k) {
            int p0 = k * chunk, p1 = p0 + chunk < N ? p0 + chunk : N;
            if (p0 < p1) f |= g2p_range(P, p0, p1, x, v, C, F, gv);
        }
        for (int tl = 0; tl < P->n_tools; ++tl)
            for (int a = 0; a < 3; ++a) T[3 * tl + a] += P->dt * u[3 * tl + a];
        flags |= f;
    }
    free(gm); free(gmv); free(gv); free(hist); free(cut);
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Adjoint: exact transpose of the substep recurrence above, with a full tape
 * (the state at the start of every substep) and the grid of each substep
 * recomputed in reverse.                                                    */

/* Reverse of the grid operation at one node.  vbar_out is the adjoint of the
 * node's final velocity; returns the adjoint of vhat in vhbar and adds the
 * tool-velocity and tool-position adjoints of the colliding tool. */
static void grid_node_adjoint(const orc_tool *tools, const double *u, const orc_node_rec *r,
                              const double vbar_out[3], double vhbar[3], double *ubar, double *Tbar)
{
    vhbar[0] = vhbar[1] = vhbar[2] = 0.0;
    if (r->wall) return;
    if (r->tool < 0 || r->branch == 0) {
        memcpy(vhbar, vbar_out, 3 * sizeof(double));
        return;
    }
    int t = r->tool;
    const orc_tool *tl = &tools[t];
    const double *uc = u + 3 * t;
    for (int a = 0; a < 3; ++a) ubar[3 * t + a] += vbar_out[a];
    if (r->branch == 2) return;
    /* friction branch: v = s v_t + u, s = 1 + mu vn/|vt| */
    const double *nrm = r->n;
    double vr[3] = {r->vhat[0] - uc[0], r->vhat[1] - uc[1], r->vhat[2] - uc[2]};
    double vn = vr[0] * nrm[0] + vr[1] * nrm[1] + vr[2] * nrm[2];
    double vt[3] = {vr[0] - vn * nrm[0], vr[1] - vn * nrm[1], vr[2] - vn * nrm[2]};
    double nt = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
    double s = 1.0 + tl->friction * vn / nt;
    const double *a_ = vbar_out;
    double sbar = a_[0] * vt[0] + a_[1] * vt[1] + a_[2] * vt[2];
    double vtbar[3] = {s * a_[0], s * a_[1], s * a_[2]};
    double vnbar = sbar * tl->friction / nt;
    double ntbar = -sbar * tl->friction * vn / (nt * nt);
    for (int k = 0; k < 3; ++k) vtbar[k] += ntbar * vt[k] / nt;
    double vrbar[3], nbar[3];
    double vtn = vtbar[0] * nrm[0] + vtbar[1] * nrm[1] + vtbar[2] * nrm[2];
    vnbar -= vtn;
    for (int k = 0; k < 3; ++k) {
        vrbar[k] = vtbar[k] + vnbar * nrm[k];
        nbar[k] = -vn * vtbar[k] + vnbar * vr[k];
    }
    for (int k = 0; k < 3; ++k) {
        vhbar[k] = vrbar[k];
        ubar[3 * t + k] -= vrbar[k];
    }
    if (tl->shape != ORC_TOOL_CAPSULE) {
        /* n = R l(x_ref), x_ref = R^T (x_i - T):  x_ref_bar = Jl^T R^T n_bar */
        double l[3], Jl[9], nlbar[3], xrbar[3];
        if (tl->shape == ORC_TOOL_BOX) orc_box_sdf(r->xr, tl->half, tl->radius, l, Jl);
        else orc_sampled_sdf(tl, r->xr, l, Jl);
        for (int b = 0; b < 3; ++b) nlbar[b] = tl->R[0 + b] * nbar[0] + tl->R[3 + b] * nbar[1] + tl->R[6 + b] * nbar[2];
        for (int b = 0; b < 3; ++b) xrbar[b] = Jl[0 + b] * nlbar[0] + Jl[3 + b] * nlbar[1] + Jl[6 + b] * nlbar[2];
        for (int a = 0; a < 3; ++a)
            Tbar[3 * t + a] -= tl->R[3 * a + 0] * xrbar[0] + tl->R[3 * a + 1] * xrbar[1] + tl->R[3 * a + 2] * xrbar[2];
        return;
    }
    /* n = R q/|q|, q = q(x_ref), x_ref = R^T (x_i - T) */
    double ql = sqrt(r->q[0] * r->q[0] + r->q[1] * r->q[1] + r->q[2] * r->q[2]);
    if (ql < 1e-12) return;
    double nl[3] = {r->q[0] / ql, r->q[1] / ql, r->q[2] / ql};
    double nlbar[3];
    for (int b = 0; b < 3; ++b) nlbar[b] = tl->R[0 + b] * nbar[0] + tl->R[3 + b] * nbar[1] + tl->R[6 + b] * nbar[2];
    double dotn = nlbar[0] * nl[0] + nlbar[1] * nl[1] + nlbar[2] * nl[2];
    double qbar[3];
    for (int b = 0; b < 3; ++b) qbar[b] = (nlbar[b] - dotn * nl[b]) / ql;
    double xrbar[3] = {r->interior ? 0.0 : qbar[0], qbar[1], qbar[2]};
    for (int a = 0; a < 3; ++a)
        Tbar[3 * t + a] -= tl->R[3 * a + 0] * xrbar[0] + tl->R[3 * a + 1] * xrbar[1] + tl->R[3 * a + 2] * xrbar[2];
}

/* Reverse of G2P, advection and the F update (Sec. III-B item 3, the F'
 * relation) for every particle, from the substep-start x, F and the node
 * velocities gv.  On entry xbar, vbar, Cbar, Fbar hold the adjoints of the
 * state after the stage; on exit xbar and Fbar hold those of x and F before
 * it and vbar, Cbar are zero (the stage overwrites v and C); gvbar receives
 * the adjoint of the node velocities. */
void orc_g2p_adjoint(const orc_params *P, int32_t N, const double *x, const double *F, const double *gv,
                     double *xbar, double *vbar, double *Cbar, double *Fbar, double *gvbar)
{
    const int n = P->n;
    const size_t nn = (size_t)n * n * n;
    const double dx = 1.0 / n, inv_dx = (double)n, D = 4.0 * inv_dx * inv_dx, dt = P->dt;
    memset(gvbar, 0, sizeof(double) * 3 * nn);
    for (int p = 0; p < N; ++p) {
        int base[3];
        double fx[3], w[3][3], dw[3][3];
        orc_weights(x + 3 * p, inv_dx, base, fx, w, dw);
        if (out_of_domain(base, n)) continue;  /* state passes through unchanged */
        /* forward values of this particle's G2P */
        double vp[3] = {0, 0, 0}, B[9] = {0};
        for (int o0 = 0; o0 < 3; ++o0) for (int o1 = 0; o1 < 3; ++o1) for (int o2 = 0; o2 < 3; ++o2) {
            double dpos[3] = {(o0 - fx[0]) * dx, (o1 - fx[1]) * dx, (o2 - fx[2]) * dx};
            double wt = w[0][o0] * w[1][o1] * w[2][o2];
            const double *vi = gv + 3 * IDX(n, base[0] + o0, base[1] + o1, base[2] + o2);
            for (int a = 0; a < 3; ++a) {
                vp[a] += wt * vi[a];
                for (int b = 0; b < 3; ++b) B[3 * a + b] += wt * vi[a] * dpos[b];
            }
        }
        double Cn[9];
        for (int k = 0; k < 9; ++k) Cn[k] = D * B[k];
        const double *Fp = F + 9 * p;
        double *Fb = Fbar + 9 * p, *Cb = Cbar + 9 * p, *vb = vbar + 3 * p, *xb = xbar + 3 * p;
        /* F' = (I + dt C') F */
        double Fbn[9], Cbt[9];
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) {
            double s1 = 0.0, s2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                s1 += ((c == a ? 1.0 : 0.0) + dt * Cn[3 * c + a]) * Fb[3 * c + b];
                s2 += Fb[3 * a + c] * Fp[3 * b + c];
            }
            Fbn[3 * a + b] = s1;
            Cbt[3 * a + b] = Cb[3 * a + b] + dt * s2;
        }
        /* x' = x + dt v' */
        double vbt[3] = {vb[0] + dt * xb[0], vb[1] + dt * xb[1], vb[2] + dt * xb[2]};
        double fxbar[3] = {0, 0, 0};
        for (int o0 = 0; o0 < 3; ++o0) for (int o1 = 0; o1 < 3; ++o1) for (int o2 = 0; o2 < 3; ++o2) {
            int o[3] = {o0, o1, o2};
            double dpos[3] = {(o0 - fx[0]) * dx, (o1 - fx[1]) * dx, (o2 - fx[2]) * dx};
            double wt = w[0][o0] * w[1][o1] * w[2][o2];
            size_t id = IDX(n, base[0] + o0, base[1] + o1, base[2] + o2);
            const double *vi = gv + 3 * id;
            double g[3];
            for (int a = 0; a < 3; ++a)
                g[a] = vbt[a] + D * (Cbt[3 * a + 0] * dpos[0] + Cbt[3 * a + 1] * dpos[1] + Cbt[3 * a + 2] * dpos[2]);
            for (int a = 0; a < 3; ++a) gvbar[3 * id + a] += wt * g[a];
            double wbar = vi[0] * g[0] + vi[1] * g[1] + vi[2] * g[2];
            for (int b = 0; b < 3; ++b) {
                double dposbar = wt * D * (Cbt[0 + b] * vi[0] + Cbt[3 + b] * vi[1] + Cbt[6 + b] * vi[2]);
                double dwd = dw[b][o[b]];
                for (int e = 0; e < 3; ++e) if (e != b) dwd *= w[e][o[e]];
                fxbar[b] += -dx * dposbar + wbar * dwd;
            }
        }
        for (int a = 0; a < 3; ++a) xb[a] += inv_dx * fxbar[a];
        memcpy(Fb, Fbn, sizeof Fbn);
        for (int k = 0; k < 9; ++k) Cb[k] = 0.0;
        vb[0] = vb[1] = vb[2] = 0.0;
    }

}

/* Reverse of the grid operation (Sec. III-B item 2, Sec. III-C) at every
 * node with mass, using the forward's node records (tool, contact branch,
 * normal): gvbar is the adjoint of the node velocities; gmbar, gmvbar receive
 * those of the node mass and momentum, and the tool-velocity and tool-position
 * adjoints of this substep are added to ubar[t][3], Tbar[t][3]. */
void orc_grid_adjoint(const orc_params *P, const orc_tool *tools, const double *u, const double *gm,
                      const double *gmv, const orc_node_rec *rec, const double *gvbar, double *gmbar, double *gmvbar,
                      double *ubar, double *Tbar)
{
    const size_t nn = (size_t)P->n * P->n * P->n;
    for (size_t id = 0; id < nn; ++id) {
        gmbar[id] = 0.0;
        gmvbar[3 * id] = gmvbar[3 * id + 1] = gmvbar[3 * id + 2] = 0.0;
        if (!(gm[id] > 0.0)) continue;
        double vhbar[3];
        grid_node_adjoint(tools, u, &rec[id], gvbar + 3 * id, vhbar,
                          ubar, Tbar);
        double pv[3];
        for (int a = 0; a < 3; ++a) {
            gmvbar[3 * id + a] = vhbar[a] / gm[id];
            pv[a] = gmv[3 * id + a] / gm[id];
        }
        gmbar[id] = -(vhbar[0] * pv[0] + vhbar[1] * pv[1] + vhbar[2] * pv[2]) / gm[id];
    }

}

/* Reverse of P2G and of the Neo-Hookean stress (Sec. III-B item 1, Eq. P2G,
 * Eq. fip) for every particle, from the substep-start state: adds to xbar,
 * vbar, Cbar, Fbar the adjoints through the node mass and momentum (adjoints
 * gmbar, gmvbar) and to mubar, lambar those of the Lame parameters. */
void orc_p2g_adjoint(const orc_params *P, int32_t N, const double *x, const double *v, const double *C,
                     const double *F, const double *gmbar, const double *gmvbar, double *xbar, double *vbar,
                     double *Cbar, double *Fbar, double *mubar, double *lambar)
{
    const int n = P->n;
    const double dx = 1.0 / n, inv_dx = (double)n, D = 4.0 * inv_dx * inv_dx, dt = P->dt;
    const double m = P->rho * P->V0;
    double mu, lam;
    orc_lame(P->E, P->nu, &mu, &lam);
    for (int p = 0; p < N; ++p) {
        int base[3];
        double fx[3], w[3][3], dw[3][3], tau[9], A[9];
        orc_weights(x + 3 * p, inv_dx, base, fx, w, dw);
        if (out_of_domain(base, n)) continue;
        const double *Fp = F + 9 * p;
        orc_kirchhoff(Fp, mu, lam, tau);
        for (int k = 0; k < 9; ++k) A[k] = -dt * P->V0 * D * tau[k] + m * C[9 * p + k];
        double vbp[3] = {0, 0, 0}, Abar[9] = {0}, fxbar[3] = {0, 0, 0};
        for (int o0 = 0; o0 < 3; ++o0) for (int o1 = 0; o1 < 3; ++o1) for (int o2 = 0; o2 < 3; ++o2) {
            int o[3] = {o0, o1, o2};
            double dpos[3] = {(o0 - fx[0]) * dx, (o1 - fx[1]) * dx, (o2 - fx[2]) * dx};
            double wt = w[0][o0] * w[1][o1] * w[2][o2];
            size_t id = IDX(n, base[0] + o0, base[1] + o1, base[2] + o2);
            const double *Pb = gmvbar + 3 * id;
            double contrib[3];
            for (int a = 0; a < 3; ++a) {
                vbp[a] += m * wt * Pb[a];
                for (int b = 0; b < 3; ++b) Abar[3 * a + b] += wt * Pb[a] * dpos[b];
                contrib[a] = m * v[3 * p + a] + A[3 * a + 0] * dpos[0] + A[3 * a + 1] * dpos[1] + A[3 * a + 2] * dpos[2];
            }
            double wbar = m * gmbar[id] + Pb[0] * contrib[0] + Pb[1] * contrib[1] + Pb[2] * contrib[2];
            for (int b = 0; b < 3; ++b) {
                double dposbar = wt * (A[0 + b] * Pb[0] + A[3 + b] * Pb[1] + A[6 + b] * Pb[2]);
                double dwd = dw[b][o[b]];
                for (int e = 0; e < 3; ++e) if (e != b) dwd *= w[e][o[e]];
                fxbar[b] += -dx * dposbar + wbar * dwd;
            }
        }
        double *xb = xbar + 3 * p;
        for (int a = 0; a < 3; ++a) {
            xb[a] += inv_dx * fxbar[a];
            vbar[3 * p + a] += vbp[a];
        }
        for (int k = 0; k < 9; ++k) Cbar[9 * p + k] += m * Abar[k];
        double taub[9];
        for (int k = 0; k < 9; ++k) taub[k] = -dt * P->V0 * D * Abar[k];
        double J = det3(Fp);
        double trt = taub[0] + taub[4] + taub[8];
        double FFt_I = 0.0;
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) {
            double FFt = 0.0;
            for (int c = 0; c < 3; ++c) FFt += Fp[3 * a + c] * Fp[3 * b + c];
            FFt_I += taub[3 * a + b] * (FFt - (a == b ? 1.0 : 0.0));
        }
        *mubar += FFt_I;
        double *Fb = Fbar + 9 * p;
        if (J > ORC_J_MIN) {
            double Fit[9];
            inv_transpose3(Fp, Fit);
            *lambar += trt * log(J);
            for (int k = 0; k < 9; ++k) Fb[k] += lam * trt * Fit[k];
        } else {
            *lambar += trt * log(ORC_J_MIN);
        }
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) {
            double s1 = 0.0;
            for (int c = 0; c < 3; ++c) s1 += (taub[3 * a + c] + taub[3 * c + a]) * Fp[3 * c + b];
            Fb[3 * a + b] += mu * s1;
        }
    }
}

uint32_t orc_adjoint(const orc_params *P, const orc_tool *tools, const double *traj, int32_t n_traj,
                     int32_t S, const double *T0, int32_t N, const double *x0, const double *v0,
                     const double *C0, const double *F0, double *xbar, double *vbar, double *Cbar,
                     double *Fbar, double *gE, double *gnu, double *gu, double *gT0)
{
    const int n = P->n, nt = P->n_tools;
    const size_t nn = (size_t)n * n * n;
    const double dt = P->dt;
    uint32_t flags = 0;

    /* forward with a full tape of substep-start states and tool poses */
    double *tx = malloc(sizeof(double) * 3 * N * (size_t)S), *tv = malloc(sizeof(double) * 3 * N * (size_t)S);
    double *tC = malloc(sizeof(double) * 9 * N * (size_t)S), *tF = malloc(sizeof(double) * 9 * N * (size_t)S);
    double *tT = malloc(sizeof(double) * 3 * (nt > 0 ? nt : 1) * (size_t)(S + 1));
    double *tu = malloc(sizeof(double) * 3 * (nt > 0 ? nt : 1) * (size_t)S);
    double *x = malloc(sizeof(double) * 3 * N), *v = malloc(sizeof(double) * 3 * N);
    double *C = malloc(sizeof(double) * 9 * N), *F = malloc(sizeof(double) * 9 * N);
    double *gm = malloc(sizeof(double) * nn), *gmv = malloc(sizeof(double) * 3 * nn), *gv = malloc(sizeof(double) * 3 * nn);
    double *gvbar = malloc(sizeof(double) * 3 * nn), *gmbar = malloc(sizeof(double) * nn), *gmvbar = malloc(sizeof(double) * 3 * nn);
    orc_node_rec *rec = malloc(sizeof(orc_node_rec) * nn);
    double *Tbar = calloc(3 * (nt > 0 ? nt : 1) * (size_t)S, sizeof(double));
    double *T = malloc(sizeof(double) * 3 * (nt > 0 ? nt : 1));

    memcpy(x, x0, sizeof(double) * 3 * N); memcpy(v, v0, sizeof(double) * 3 * N);
    memcpy(C, C0, sizeof(double) * 9 * N); memcpy(F, F0, sizeof(double) * 9 * N);
    if (nt > 0) memcpy(T, T0, sizeof(double) * 3 * nt);
    for (int s = 0; s < S; ++s) {
        memcpy(tx + 3 * (size_t)N * s, x, sizeof(double) * 3 * N);
        memcpy(tv + 3 * (size_t)N * s, v, sizeof(double) * 3 * N);
        memcpy(tC + 9 * (size_t)N * s, C, sizeof(double) * 9 * N);
        memcpy(tF + 9 * (size_t)N * s, F, sizeof(double) * 9 * N);
        if (nt > 0) {
            memcpy(tT + 3 * (size_t)nt * s, T, sizeof(double) * 3 * nt);
            traj_at(P, traj, n_traj, s, tu + 3 * (size_t)nt * s);
        }
        flags |= orc_substep(P, tools, T, nt > 0 ? tu + 3 * (size_t)nt * s : NULL, N, x, v, C, F, gm, gmv, gv);
    }

    double mubar = 0.0, lambar = 0.0;
    if (nt > 0) memset(gu, 0, sizeof(double) * 3 * nt * (size_t)S);
    for (int s = S - 1; s >= 0; --s) {
        /* restore the substep-start state and recompute the substep's grid */
        memcpy(x, tx + 3 * (size_t)N * s, sizeof(double) * 3 * N);
        memcpy(v, tv + 3 * (size_t)N * s, sizeof(double) * 3 * N);
        memcpy(C, tC + 9 * (size_t)N * s, sizeof(double) * 9 * N);
        memcpy(F, tF + 9 * (size_t)N * s, sizeof(double) * 9 * N);
        const double *Ts = tT + 3 * (size_t)nt * s, *us = tu + 3 * (size_t)nt * s;
        orc_p2g(P, N, x, v, C, F, gm, gmv);
        orc_grid_update(P, tools, Ts, us, gm, gmv, gv, rec);

        /* reverse of F update, advection and G2P, of the grid operation, of P2G and the stress */
        orc_g2p_adjoint(P, N, x, F, gv, xbar, vbar, Cbar, Fbar, gvbar);
        orc_grid_adjoint(P, tools, us, gm, gmv, rec, gvbar, gmbar, gmvbar, nt > 0 ? gu + 3 * (size_t)nt * s : NULL,
                         Tbar + 3 * (size_t)nt * s);
        orc_p2g_adjoint(P, N, x, v, C, F, gmbar, gmvbar, xbar, vbar, Cbar, Fbar, &mubar, &lambar);
    }

    /* tool pose T_s = T_0 + dt sum_{s'<s} u_{s'} */
    if (nt > 0) {
        for (int t = 0; t < nt; ++t) {
            double acc[3] = {0, 0, 0};
            for (int s = S - 1; s >= 0; --s) {
                for (int a = 0; a < 3; ++a) gu[3 * ((size_t)nt * s + t) + a] += dt * acc[a];
                for (int a = 0; a < 3; ++a) acc[a] += Tbar[3 * ((size_t)nt * s + t) + a];
            }
            if (gT0) for (int a = 0; a < 3; ++a) gT0[3 * t + a] = acc[a];
        }
    }
    /* chain rule through the Lame parameters */
    double nu = P->nu, E = P->E;
    double dmu_dE = 1.0 / (2.0 * (1.0 + nu)), dmu_dnu = -E / (2.0 * (1.0 + nu) * (1.0 + nu));
    double dlam_dE = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double dlam_dnu = E * (1.0 + 2.0 * nu * nu) / ((1.0 + nu) * (1.0 + nu) * (1.0 - 2.0 * nu) * (1.0 - 2.0 * nu));
    *gE = mubar * dmu_dE + lambar * dlam_dE;
    *gnu = mubar * dmu_dnu + lambar * dlam_dnu;

    free(tx); free(tv); free(tC); free(tF); free(tT); free(tu);
    free(x); free(v); free(C); free(F); free(gm); free(gmv); free(gv);
    free(gvbar); free(gmbar); free(gmvbar); free(rec); free(Tbar); free(T);
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Surface extraction: marching cubes over the mass volume (Sec. III-A, the
 * post-processing that turns the particles into a triangle mesh; Lorensen and
 * Cline's method as cited there).
 *
 * Readings (R18): the mass volume is the P2G mass on the simulation grid,
 * density rho_i = m_i / dx^3 at node i, and the surface is rho = iso.  A cell
 * corner is inside when rho >= iso.  Per cell the surface is made of closed
 * polygons found by walking the six faces: on a face, the edges whose two
 * corners differ are crossed once; two crossings are joined by one segment;
 * four crossings (diagonally opposite inside corners) by two segments, each
 * cutting off one inside corner.  Each segment runs so that, seen from
 * outside the cell, the inside corners it cuts off lie on its left; a
 * crossing point is then the end of one segment and the start of the next,
 * which chains the segments into polygons.  A polygon is split into a fan of
 * triangles from its lowest-numbered edge, and polygons are taken in order of
 * their lowest-numbered edge.  Crossing points are the linear interpolation
 * of rho along the edge.  Triangles are wound so that their right-hand normal
 * points out of the dense region.
 *
 * Numbering: corner c = 4 dx + 2 dy + dz at (i+dx, j+dy, k+dz) h; edge
 * e = 4 a + p along axis a, p = the two other corner bits in axis order.
 * Cells (i, j, k) in [0, n-1)^3, row-major. */

static int mc_edge(int ca, int cb)
{
    int diff = ca ^ cb, a = diff == 4 ? 0 : diff == 2 ? 1 : 2;
    int lo = ca & ~diff;
    int bx = (lo >> 2) & 1, by = (lo >> 1) & 1, bz = lo & 1;
    int p = a == 0 ? 2 * by + bz : a == 1 ? 2 * bx + bz : 2 * bx + by;
    return 4 * a + p;
}

static void mc_edge_corners(int e, int *ca, int *cb)
{
    int a = e / 4, p = e % 4, hi = (p >> 1) & 1, lo = p & 1;
    int bits[3];
    if (a == 0) { bits[1] = hi; bits[2] = lo; }
    else if (a == 1) { bits[0] = hi; bits[2] = lo; }
    else { bits[0] = hi; bits[1] = lo; }
    bits[a] = 0;
    *ca = 4 * bits[0] + 2 * bits[1] + bits[2];
    bits[a] = 1;
    *cb = 4 * bits[0] + 2 * bits[1] + bits[2];
}

static void mc_corner_pos(int c, double p[3])
{
    p[0] = (c >> 2) & 1; p[1] = (c >> 1) & 1; p[2] = c & 1;
}

static void mc_edge_mid(int e, double m[3])
{
    int ca, cb;
    double pa[3], pb[3];
    mc_edge_corners(e, &ca, &cb);
    mc_corner_pos(ca, pa);
    mc_corner_pos(cb, pb);
    for (int d = 0; d < 3; ++d) m[d] = 0.5 * (pa[d] + pb[d]);
}

/* Orientation test for a segment p -> q on the face with outward normal N
 * cutting off inside corner K: K lies on the left, seen from outside. */
static int mc_left(int p, int q, const double N[3], int K)
{
    double mp[3], mq[3], ck[3], d[3], l[3];
    mc_edge_mid(p, mp);
    mc_edge_mid(q, mq);
    mc_corner_pos(K, ck);
    for (int a = 0; a < 3; ++a) d[a] = mq[a] - mp[a];
    l[0] = N[1] * d[2] - N[2] * d[1];
    l[1] = N[2] * d[0] - N[0] * d[2];
    l[2] = N[0] * d[1] - N[1] * d[0];
    return l[0] * (ck[0] - mp[0]) + l[1] * (ck[1] - mp[1]) + l[2] * (ck[2] - mp[2]) > 0.0;
}

/* Triangles (as edge triples) of one cell case; returns their number, or -1
 * if the face segments do not chain into closed polygons. */
int orc_mc_case(int mask, int32_t tri[][3])
{
    int next[12];
    for (int e = 0; e < 12; ++e) next[e] = -1;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) {
            int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
            int ring[4];
            const int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            for (int r = 0; r < 4; ++r) {
                int bits[3];
                bits[a] = s;
                bits[u] = uv[r][0];
                bits[v] = uv[r][1];
                ring[r] = 4 * bits[0] + 2 * bits[1] + bits[2];
            }
            double N[3] = {0.0, 0.0, 0.0};
            N[a] = s ? 1.0 : -1.0;
            int in[4], ncross = 0;
            for (int r = 0; r < 4; ++r) in[r] = (mask >> ring[r]) & 1;
            for (int r = 0; r < 4; ++r) ncross += in[r] != in[(r + 1) % 4];
            if (ncross == 0) continue;
            /* segments as (edge, edge, inside corner they cut off or bound) */
            int segs[2][3], nseg = 0;
            if (ncross == 2) {
                int ends[2], ne = 0, K = -1;
                for (int r = 0; r < 4; ++r) {
                    if (in[r] != in[(r + 1) % 4]) ends[ne++] = mc_edge(ring[r], ring[(r + 1) % 4]);
                    if (in[r] && K < 0) K = ring[r];
                }
                segs[0][0] = ends[0]; segs[0][1] = ends[1]; segs[0][2] = K;
                nseg = 1;
            } else {
                for (int r = 0; r < 4; ++r)
                    if (in[r]) {
                        segs[nseg][0] = mc_edge(ring[(r + 3) % 4], ring[r]);
                        segs[nseg][1] = mc_edge(ring[r], ring[(r + 1) % 4]);
                        segs[nseg][2] = ring[r];
                        ++nseg;
                    }
            }
            for (int g = 0; g < nseg; ++g) {
                int p = segs[g][0], q = segs[g][1];
                if (!mc_left(p, q, N, segs[g][2])) { int t = p; p = q; q = t; }
                if (next[p] >= 0) return -1;
                next[p] = q;
            }
        }
    int used[12] = {0}, nt = 0;
    for (int e0 = 0; e0 < 12; ++e0) {
        if (next[e0] < 0 || used[e0]) continue;
        int loop[12], k = 0, e = e0;
        do {
            if (e < 0 || used[e] || k >= 12) return -1;
            used[e] = 1;
            loop[k++] = e;
            e = next[e];
        } while (e != e0);
        for (int t = 1; t + 1 < k; ++t) {
            tri[nt][0] = loop[0];
            tri[nt][1] = loop[t + 1];
            tri[nt][2] = loop[t];
            ++nt;
        }
    }
    for (int e = 0; e < 12; ++e)
        if ((next[e] >= 0) != used[e]) return -1;
    return nt;
}

int64_t orc_surface(int32_t n, double h, const double *rho, double iso, int32_t *cell_ntri, int32_t *tri_edges,
                    double *tris, int64_t max_tris)
{
    const int nc = n - 1;
    int64_t total = 0;
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j)
            for (int k = 0; k < nc; ++k) {
                double val[8];
                int mask = 0;
                for (int c = 0; c < 8; ++c) {
                    val[c] = rho[IDX(n, i + ((c >> 2) & 1), j + ((c >> 1) & 1), k + (c & 1))];
                    if (val[c] >= iso) mask |= 1 << c;
                }
                int32_t tri[12][3];
                int nt = orc_mc_case(mask, tri);
                if (nt < 0) return -1;
                if (cell_ntri) cell_ntri[((size_t)i * nc + j) * nc + k] = nt;
                for (int t = 0; t < nt; ++t, ++total) {
                    if (total >= max_tris) continue;
                    for (int v = 0; v < 3; ++v) {
                        int ca, cb;
                        double pa[3], pb[3];
                        mc_edge_corners(tri[t][v], &ca, &cb);
                        mc_corner_pos(ca, pa);
                        mc_corner_pos(cb, pb);
                        double f = (iso - val[ca]) / (val[cb] - val[ca]);
                        const int cell[3] = {i, j, k};
                        for (int d = 0; d < 3; ++d)
                            tris[9 * total + 3 * v + d] = (cell[d] + pa[d] + f * (pb[d] - pa[d])) * h;
                        if (tri_edges) tri_edges[3 * total + v] = tri[t][v];
                    }
                }
            }
    return total;
}
