/*
 * FP64 CPU oracle for the MLS-MPM Neo-Hookean tissue substep.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference that the
 * HIP path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product path never does.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * What it computes (section / equation of arXiv 2402.01181):
 *   P2G       Sec. III-B item 1, Eq. P2G (APIC momentum + mass), Eq. fip
 *             (MLS stress force), Neo-Hookean stress, Lame parameters.
 *   Grid op   Sec. III-B item 2 (normalisation, boundary nodes), Sec. III-C
 *             (tool frame transform, SDF threshold, normal, Coulomb
 *             friction, z-buffer over tools).
 *   G2P       Sec. III-B item 3 (velocity, affine matrix, advection).
 *   F update  Sec. III-B item 1, the F' = (I + dt C) F relation.
 *   Surface   Sec. III-A post-processing: marching cubes over the mass
 *             volume (orc_surface, orc_mc_case).
 * Readings where the paper is silent or garbled are listed beside each
 * function in mpm_oracle.c.
 *
 * Layout: particles are AoS double arrays, x[N][3], v[N][3], C[N][3][3],
 * F[N][3][3] (row-major matrices).  Grids are dense, node (i,j,k) at index
 * (i*n + j)*n + k, node position (i,j,k)*dx with dx = 1/n; gm[n^3],
 * gmv[n^3][3], gv[n^3][3].
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H
#include <stdint.h>

#define ORC_FLAG_OUT_OF_DOMAIN 1u
#define ORC_FLAG_INVERTED 2u
#define ORC_FLAG_NONFINITE 4u
#define ORC_J_MIN 1e-6

#define ORC_CONTACT_SLIP 0
#define ORC_CONTACT_STICKY 1

#define ORC_TOOL_CAPSULE 0   /* analytic capsule (segment on the tool-frame x axis) */
#define ORC_TOOL_BOX 1       /* box of half extents `half`, corners rounded by `radius` */
#define ORC_TOOL_SDF 2       /* signed distances sampled on a regular tool-frame lattice */

#define ORC_SDF_NEAREST 0    /* the sample of the cell the point falls in (index truncation) */
#define ORC_SDF_TRILINEAR 1  /* trilinear in the samples and in their central-difference gradients */

typedef struct {
    int32_t n;          /* grid nodes per axis */
    int32_t bound;      /* boundary band width in nodes */
    int32_t n_tools;
    int32_t pad;
    double dt;
    double g[3];
    double E, nu, rho, V0;  /* particle mass m = rho * V0 */
} orc_params;

typedef struct {
    int32_t contact;    /* ORC_CONTACT_SLIP or ORC_CONTACT_STICKY */
    int32_t shape;      /* ORC_TOOL_* */
    double radius, half_len, friction, theta;
    double R[9];        /* world-from-tool rotation, row-major */
    double half[3];     /* box half extents (tool frame) */
    double sdf_h;       /* sampled SDF: lattice spacing */
    double sdf_lo[3];   /* sampled SDF: tool-frame position of sample (0,0,0) */
    int32_t sdf_res;    /* sampled SDF: samples per axis */
    int32_t sdf_interp; /* ORC_SDF_NEAREST or ORC_SDF_TRILINEAR */
    const float *sdf;   /* sampled SDF: [res][res][res], sample (i,j,k) at lo + (i,j,k) h */
} orc_tool;

/* Per-node record of the grid operation, kept so the adjoint can replay the
 * discrete decisions (contact, branch) without re-deriving them. */
typedef struct {
    double vhat[3];     /* velocity after normalisation and gravity */
    double n[3];        /* contact normal (world) */
    double q[3];        /* tool-frame offset from the capsule axis */
    int32_t tool;       /* colliding tool id, -1 if none */
    int32_t branch;     /* 0 none/separating, 1 friction, 2 set to tool velocity */
    int32_t wall;
    int32_t interior;   /* tool-frame axial coordinate strictly inside the segment */
    double xr[3];       /* node position in the colliding tool's frame */
} orc_node_rec;

void orc_lame(double E, double nu, double *mu, double *lam);
void orc_weights(const double x[3], double inv_dx, int base[3], double fx[3], double w[3][3],
                 double dw[3][3]);
uint32_t orc_kirchhoff(const double F[9], double mu, double lam, double tau[9]);
double orc_capsule_sdf(const double xref[3], double radius, double half_len, double q[3], int *interior);
double orc_box_sdf(const double xref[3], const double half[3], double radius, double l[3], double Jl[9]);
double orc_sampled_sdf(const orc_tool *tl, const double xref[3], double l[3], double Jl[9]);

uint32_t orc_p2g(const orc_params *P, int32_t N, const double *x, const double *v, const double *C,
                 const double *F, double *gm, double *gmv);
void orc_grid_update(const orc_params *P, const orc_tool *tools, const double *T, const double *u,
                     const double *gm, const double *gmv, double *gv, orc_node_rec *rec);
uint32_t orc_g2p(const orc_params *P, int32_t N, double *x, double *v, double *C, double *F,
                 const double *gv);
uint32_t orc_substep(const orc_params *P, const orc_tool *tools, double *T, const double *u,
                     int32_t N, double *x, double *v, double *C, double *F,
                     double *gm, double *gmv, double *gv);
uint32_t orc_run(const orc_params *P, const orc_tool *tools, const double *traj, int32_t n_traj,
                 int32_t s0, int32_t S, double *T, int32_t N, double *x, double *v, double *C,
                 double *F);
void orc_g2p_adjoint(const orc_params *P, int32_t N, const double *x, const double *F, const double *gv,
                     double *xbar, double *vbar, double *Cbar, double *Fbar, double *gvbar);
void orc_grid_adjoint(const orc_params *P, const orc_tool *tools, const double *u, const double *gm,
                      const double *gmv, const orc_node_rec *rec, const double *gvbar, double *gmbar, double *gmvbar,
                      double *ubar, double *Tbar);
void orc_p2g_adjoint(const orc_params *P, int32_t N, const double *x, const double *v, const double *C,
                     const double *F, const double *gmbar, const double *gmvbar, double *xbar, double *vbar,
                     double *Cbar, double *Fbar, double *mubar, double *lambar);
uint32_t orc_run_threads(const orc_params *P, const orc_tool *tools, const double *traj, int32_t n_traj,
                         int32_t s0, int32_t S, double *T, int32_t N, double *x, double *v, double *C,
                         double *F, int32_t nthreads);
int orc_mc_case(int mask, int32_t tri[][3]);
int64_t orc_surface(int32_t n, double h, const double *rho, double iso, int32_t *cell_ntri, int32_t *tri_edges,
                    double *tris, int64_t max_tris);
uint32_t orc_adjoint(const orc_params *P, const orc_tool *tools, const double *traj, int32_t n_traj,
                     int32_t S, const double *T0, int32_t N, const double *x0, const double *v0,
                     const double *C0, const double *F0, double *xbar, double *vbar, double *Cbar,
                     double *Fbar, double *gE, double *gnu, double *gu, double *gT0);
#endif
