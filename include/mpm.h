/*
 * mpm.h -- C ABI of the MI355X (gfx950) MLS-MPM tissue library.
 *
 * The library steps the MLS-MPM substep of arXiv 2402.01181 for Neo-Hookean
 * tissue touched by rigid tools (capsules, boxes, sampled SDFs): P2G
 * (Sec. III-B item 1, Eq. P2G and Eq. fip), the grid operation with boundary
 * nodes and tool contact (Sec. III-B item 2, Sec. III-C), G2P with advection
 * (Sec. III-B item 3) and the deformation-gradient update, for one or many
 * independent environments at once, plus the reverse (adjoint) of those
 * substeps and the surface mesh of the tissue (Sec. III-A post-processing).
 *
 * Conventions shared by every entry point:
 *  - Device memory is owned by the CALLER: initial state, material table,
 *    tool trajectories, gradient outputs and the single workspace the
 *    library carves all its device buffers from (mpm_create_static takes the
 *    workspace from a device array inside the library instead).  The library
 *    owns only the host-side context object.  It never calls hipMalloc/hipFree.
 *  - Streams are hipStream_t passed as void*; NULL means the null stream.
 *    A context is used from one stream at a time and is not thread-safe.
 *  - Particle arrays are FP32, structure-of-arrays, component-major and
 *    environment-concatenated: x[3][Ntot], v[3][Ntot], C[9][Ntot],
 *    F[9][Ntot] (matrix entry (a,b) is component 3a+b), Ntot = sum of the
 *    per-environment particle counts in environment order.
 *  - Environment e has a cubic grid of grid_n[e]^3 nodes on the unit cube,
 *    dx = 1/grid_n[e]; node (i,j,k) sits at (i,j,k)*dx.
 *  - No exceptions cross the ABI.  Every call returns MPM_OK or a negative
 *    code; argument errors return MPM_E_ARG and change nothing; HIP runtime
 *    failures return MPM_E_HIP; mpm_last_error() describes the last error.
 *  - Conditions met inside kernels set sticky per-environment status bits
 *    (MPM_FLAG_*), read with mpm_read_state(..., MPM_F_STATUS, ...).
 *    mpm_substep and mpm_substep_adjoint never synchronise with the host and
 *    issue only kernel launches, so a caller may capture them in a hipGraph.
 *    A captured call replays the launches it recorded (a counting sort
 *    included if one fell in it); the context's host-side bookkeeping (the
 *    substeps since the last sort) advances once, at capture, so a caller
 *    mixing replays with direct calls should capture calls that sort.
 */
#ifndef MPM355_MPM_H
#define MPM355_MPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_ctx mpm_ctx;
typedef int32_t mpm_status;

enum {
    MPM_OK = 0,
    MPM_E_ARG = -1,          /* invalid argument; nothing changed */
    MPM_E_HIP = -2,          /* a HIP runtime call failed */
    MPM_E_STATE = -3,        /* call not valid in the current state (e.g. no tape) */
    MPM_E_UNSUPPORTED = -4,  /* valid request this build does not implement */
    MPM_E_WORKSPACE = -5     /* workspace missing, misaligned or too small */
};

/* Sticky per-environment status bits. */
enum {
    MPM_FLAG_OUT_OF_DOMAIN = 1u,    /* a particle's 3x3x3 stencil left the grid; it was frozen */
    MPM_FLAG_INVERTED = 2u,         /* det F <= 1e-6 (FP64); the stress used ln(1e-6) */
    MPM_FLAG_NONFINITE = 4u,        /* a particle position or velocity became non-finite */
    MPM_FLAG_BARRIER_TIMEOUT = 8u   /* persistent kernels: a barrier exceeded its spin limit */
};

/* Fields for mpm_read_state. */
enum {
    MPM_F_X = 0,        /* float [3][N_env], original particle order */
    MPM_F_V = 1,        /* float [3][N_env] */
    MPM_F_C = 2,        /* float [9][N_env] */
    MPM_F_F = 3,        /* float [9][N_env] */
    MPM_F_GRID_M = 4,   /* float [n^3], node (i,j,k) at (i*n+j)*n+k: mass (Eq. P2G, Sec. III-B item 1) held
                           in the momentum buffer: the last P2G after MPM_STAGE_P2G, MPM_STAGE_TILED_P2G or a
                           fused tiled stage.  The tiled grid operation consumes and clears it, so after
                           mpm_substep in MPM_SCHEME_TILED (or MPM_STAGE_TILED_GRID) it reads zeros */
    MPM_F_GRID_MV = 5,  /* float [3][n^3]: momentum held in the momentum buffer, as MPM_F_GRID_M */
    MPM_F_GRID_V = 6,   /* float [3][n^3]: velocity after the last grid operation (Sec. III-B item 2); the
                           tiled grid operation writes only nodes that received mass, the others keep
                           older values (no particle's stencil reads them); with MPM_OPT_GRID_AT_STAGING
                           the last substep of a call writes the nodes of bricks that hold particles */
    MPM_F_STATUS = 7,   /* uint32 [1]: sticky MPM_FLAG_* bits of the environment */
    MPM_F_TOOL_T = 8,   /* double [max_tools][3]: current tool positions */
    MPM_F_STEP = 9,     /* int32 [1]: substeps taken by the environment */
    MPM_F_DENSITY = 10  /* float [n^3]: density volume (kg/m^3) of the last mpm_extract_surface, which must
                           have been for this environment (else MPM_E_STATE) */
};

/* Tool shapes (Sec. III-C: simple objects such as the gripper jaws by
 * bounding boxes, objects with complex geometry by a precomputed SDF in the
 * tool's frame; the analytic capsule is the SDF of a rod-like tool). */
enum { MPM_TOOL_CAPSULE = 0, MPM_TOOL_BOX = 1, MPM_TOOL_SDF = 2 };
/* Sampled-SDF lookup.  NEAREST: the sample of the lattice cell a node falls
 * in (the index of x_ref/h truncated, as in the paper's SDF[x_ref/dx]) with
 * the central-difference gradient there as the normal.  TRILINEAR: samples
 * and central-difference gradients interpolated trilinearly over the cell. */
enum { MPM_SDF_NEAREST = 0, MPM_SDF_TRILINEAR = 1 };
enum { MPM_CONTACT_SLIP = 0, MPM_CONTACT_STICKY = 1 };
/* Stages for mpm_run_stage.  The first three are the direct scheme's kernels;
 * the TILED ones are mpm_substep's tiled-scheme kernels, launched one at a
 * time in the order a call of mpm_substep launches them. */
enum {
    MPM_STAGE_P2G = 0,             /* direct: P2G of the current state into a cleared grid */
    MPM_STAGE_GRID = 1,            /* direct: grid operation over every node */
    MPM_STAGE_G2P = 2,             /* direct: G2P, advection and F update */
    MPM_STAGE_TILED_P2G = 3,       /* opens a tiled sequence: the counting sort if one is due, then the
                                      tiled P2G of the current state (MPM_F_GRID_M/MV read it) */
    MPM_STAGE_TILED_GRID = 4,      /* grid operation over the listed bricks: writes MPM_F_GRID_V where mass
                                      arrived and clears the momentum buffer; follows a P2G stage */
    MPM_STAGE_TILED_FUSED = 5,     /* fused particle pass: G2P, F update, advection of this substep and the
                                      P2G of the next one; writes x and F (v and C stay in registers, so
                                      MPM_F_V / MPM_F_C are not current until a later TILED_FUSED_FULL or
                                      TILED_G2P), MPM_F_GRID_M/MV read the new P2G; follows TILED_GRID */
    MPM_STAGE_TILED_FUSED_FULL = 6,/* as TILED_FUSED, also writing v and C (the adjoint's recompute kernel) */
    MPM_STAGE_TILED_G2P = 7        /* G2P, F update and advection only; closes the sequence; follows
                                      TILED_GRID */
};

/* Tunables (mpm_set_option).  Every setting gives the same results up to
 * the order of floating-point accumulation. */
enum {
    MPM_OPT_SCHEME = 0,       /* MPM_SCHEME_* */
    MPM_OPT_SORT_EVERY = 1,   /* counting-sort particles by grid brick every k substeps (>= 1); setting it
                                 (to any value, the current one included) restarts the schedule: the
                                 next substep call opens with a sort */
    MPM_OPT_BLOCK = 2,        /* threads per workgroup of the tiled particle kernels: 64, 128, 256 */
    MPM_OPT_GRAPH = 3,        /* 1: mpm_substep replays an internally captured hipGraph */
    MPM_OPT_PERSISTENT = 4,   /* tiled scheme, 1: each run of up to sort_every substeps is one persistent
                                 kernel.  Every environment gets its own group of workgroups (in
                                 proportion to its particles; small environments share one) and steps
                                 through the run alone: grid operation, then particle pass, separated by
                                 barriers of that group only (a counter per environment, bounded spin; a
                                 timeout sets MPM_FLAG_BARRIER_TIMEOUT).  With MPM_OPT_GRID_AT_STAGING and
                                 one environment the runs take that form instead (see there).  Setting it
                                 (or the block or item size while it is on) builds the group table with a
                                 synchronous copy, so set it outside stream capture */
    MPM_OPT_SPIN_LIMIT = 5,   /* persistent kernel: barrier spin limit (iterations), > 0 */
    MPM_OPT_ITEM = 6,         /* tiled scheme: max particles per work item, multiple of 16 in [16, 4096] */
    MPM_OPT_NODE_SLOTS = 7,   /* tiled scheme: particles per half-wavefront step of the P2G node pass, 1 or 3
                                 (3: a third of the arithmetic per node, better at many particles per cell) */
    MPM_OPT_GRID_AT_STAGING = 8 /* tiled scheme, 1: one launch per substep.  The particle pass applies
                                 the grid operation (Sec. III-B item 2) to each node of its 8^3 velocity
                                 tile as it stages it, from the momentum of the substep, so no grid
                                 kernel runs in between; momentum grids rotate over three buffers.
                                 Pays where work items are few and full (one slab).  With
                                 MPM_OPT_PERSISTENT and one environment, the substeps between two sorts
                                 are one persistent launch: every workgroup resident, a grid barrier
                                 between substeps (bounded spin; a timeout sets
                                 MPM_FLAG_BARRIER_TIMEOUT); with several environments
                                 MPM_OPT_PERSISTENT takes precedence.  With a sampled-SDF tool active the
                                 form does not apply and substeps take the per-phase launches.  0
                                 (default): a grid kernel over the listed bricks between particle
                                 passes */
};
enum {
    MPM_SCHEME_DIRECT = 0,    /* one thread per particle, global float atomics, dense grid pass */
    MPM_SCHEME_TILED = 1      /* brick-sorted particles, LDS tiles, fused G2P+P2G, active bricks */
};

typedef struct {
    int32_t n_envs;              /* >= 1 */
    const int32_t *n_particles;  /* host [n_envs], each >= 1 */
    const int32_t *grid_n;       /* host [n_envs], multiple of 4, 8 <= n <= 512; at most 2^30 nodes and
                                    2^30 particles over all environments */
    float dt;                    /* substep length (s), > 0 */
    float gravity[3];            /* m/s^2 */
    int32_t bound;               /* boundary band width in nodes (sticky), >= 0 */
    int32_t max_tools;           /* tool slots per environment, 0..8 */
    int32_t checkpoint_every;    /* adjoint: state checkpoint interval (substeps), >= 1 */
    int32_t max_tape_substeps;   /* adjoint: longest recordable tape; 0 disables the adjoint */
    const float *x0, *v0, *C0, *F0;  /* device SoA as above; copied by mpm_create */
    const float *material;       /* device [n_envs][4] = {E, nu, rho, V0}; read at every substep,
                                    so the caller may change it between calls (graph-safe) */
    int32_t hold_tape;           /* adjoint, 0 or 1.  1: the workspace holds the recomputed tape of every
                                    segment of the longest recording (ceil(max_tape_substeps /
                                    checkpoint_every) segments; at 30K particles on 64^3 and 20-substep
                                    segments, about 11.5 MB per substep).  mpm_substep with record_tape then
                                    computes each segment's tape itself (the tiled recompute passes, sorted
                                    at each segment start) instead of running the forward form, and the next
                                    mpm_substep_adjoint reverses the held tapes without recomputing them.  It
                                    consumes them: a second adjoint of the same recording recomputes from the
                                    checkpoints.  Any sequence of recordings, substeps and adjoint windows
                                    is valid: tapes a reverse did not consume (an adjoint window shorter
                                    than the recording, a recording never reversed) are cleared by the next
                                    recompute into them.  With the direct scheme a recording keeps
                                    checkpoints only.
                                    0: checkpoints only (every adjoint recomputes) */
} mpm_desc;

typedef struct {
    int32_t shape;      /* MPM_TOOL_CAPSULE: segment [-half_len, half_len] on the tool-frame x axis, radius `radius`;
                           MPM_TOOL_BOX: the box [-half, half] of the tool frame, edges rounded by `radius`;
                           MPM_TOOL_SDF: signed distances sampled on a tool-frame lattice (sdf_* fields) */
    int32_t contact;    /* MPM_CONTACT_SLIP (Coulomb friction) or MPM_CONTACT_STICKY */
    float radius;       /* capsule radius (m), > 0; box rounding radius, >= 0; unused for MPM_TOOL_SDF */
    float half_len;     /* capsule half segment length (m), >= 0 */
    float friction;     /* Coulomb coefficient, >= 0 (slip only) */
    float theta;        /* contact threshold: contact iff distance < theta (Sec. III-C) */
    float R[9];         /* world-from-tool rotation, row-major */
    float T0[3];        /* world position of the tool origin now */
    float half[3];      /* MPM_TOOL_BOX: half extents (m), each >= 0 */
    int32_t sdf_res;    /* MPM_TOOL_SDF: samples per axis, 4..2048 */
    int32_t sdf_interp; /* MPM_TOOL_SDF: MPM_SDF_NEAREST or MPM_SDF_TRILINEAR */
    float sdf_h;        /* MPM_TOOL_SDF: lattice spacing (m), > 0 */
    float sdf_lo[3];    /* MPM_TOOL_SDF: tool-frame position of sample (0,0,0) */
    const float *sdf;   /* MPM_TOOL_SDF: device array [res][res][res] of float32 signed distances (m), sample
                           (i,j,k) at sdf_lo + (i,j,k) sdf_h (i along the tool-frame x axis), index
                           (i*res + j)*res + k.  Caller-owned, read at every substep, must stay valid while
                           the slot holds this tool.  A node whose lattice coordinate s = (x_ref - sdf_lo)/sdf_h
                           (formed in FP64) has floor(s) outside [1, res-2] on any axis (trilinear: floor(s)+1
                           too) has no complete central differences and is out of this tool's reach. */
} mpm_tool;

/* Adjoint inputs and outputs.  All pointers are device memory; particle
 * arrays use the original particle order and the SoA layout above. */
typedef struct {
    const float *xbar, *vbar, *Cbar, *Fbar;  /* adjoints of the final state (NULL = 0) */
    float *xbar0, *vbar0, *Cbar0, *Fbar0;    /* out: adjoints of the state n substeps earlier (NULL = skip) */
    double *gE, *gnu;                        /* out [n_envs]: dL/dE, dL/dnu (NULL = skip) */
    double *gu;                              /* out [n_envs][max_tools][n][3]: dL/du of each substep's tool velocity */
    double *gT;                              /* out [n_envs][max_tools][3]: dL/dT of the tool positions n substeps earlier */
} mpm_adjoint_io;

/* Bytes of device workspace a context with this description needs.  Returns 0
 * for an invalid description (mpm_create then reports why). */
size_t mpm_workspace_size(const mpm_desc *desc);

/* Create a context holding the material points of Sec. III-B (position x,
 * velocity v, affine velocity C and deformation gradient F per particle,
 * with mass and volume from rho and V0, and Lame parameters from E and nu
 * by the relation of Sec. III-B) and the background grid of each
 * environment.  Validates desc (MPM_E_ARG for a bad field, e.g. E <= 0, nu
 * outside (-1, 0.5) or not finite), carves the caller's workspace (device
 * memory of at least mpm_workspace_size(desc) bytes, 256-byte aligned, owned
 * by the caller and kept alive until mpm_destroy), copies the initial state
 * and clears the grids on `stream`.  Tools start unset.  On success *out owns
 * a host object released by mpm_destroy. */
mpm_status mpm_create(const mpm_desc *desc, void *workspace, size_t workspace_bytes, void *stream,
                      mpm_ctx **out);

/* Size of the workspace mpm_create_static uses (64 MiB per device). */
#define MPM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, serving loops and harnesses that forbid hipMalloc): mpm_create
 * with the workspace taken from a device array inside the library instead of
 * a caller allocation.  The array holds MPM_STATIC_WORKSPACE_BYTES; each GPU
 * the library runs on keeps its own copy until the process ends.  The context
 * lives on the current device; desc, stream and out as for mpm_create, and
 * the context is used and released exactly like one from mpm_create.
 *  - A description needing more than MPM_STATIC_WORKSPACE_BYTES
 *    (mpm_workspace_size) returns MPM_E_WORKSPACE and creates nothing.
 *  - A device's array serves one context at a time: while a context made by
 *    this call is alive on the device, another call on it returns
 *    MPM_E_STATE.  Work of two contexts sharing one array would race, and
 *    this keeps them apart.  mpm_destroy frees the array for the next call.
 *  - The array keeps what the previous context left there; creation clears
 *    everything that must start at zero, as mpm_create does for a fresh
 *    caller workspace.
 *  - Calls no hipMalloc/hipFree or other allocating routine.  The first call
 *    on a device looks up the array's device address (hipGetSymbolAddress). */
mpm_status mpm_create_static(const mpm_desc *desc, void *stream, mpm_ctx **out);

/* Release the host object.  NULL is a no-op.  Does not touch the workspace
 * (of a mpm_create_static context: frees the device's static workspace for
 * the next mpm_create_static). */
void mpm_destroy(mpm_ctx *ctx);

/* Set tool slot `tool` of environment `env` (Sec. III-C): shape, contact
 * mode, pose.  u is a caller-owned device array [n_traj][3] of tool
 * velocities; substep k after this call uses u[min(k, n_traj-1)] as the tool
 * velocity v_co and then advances the position, T <- T + dt u (FP64).  u is
 * read at every substep, so the caller may rewrite it between calls.
 * n_traj >= 1.  Passing tool == NULL clears the slot.  The nearest tool of
 * any shape with distance < theta takes a node (the z-buffer / collision
 * objects table of Sec. III-C; equal distances go to the lower slot).
 * Returns MPM_E_ARG for a shape parameter out of range (see mpm_tool). */
mpm_status mpm_set_tool(mpm_ctx *ctx, int32_t env, int32_t tool, const mpm_tool *desc,
                        const float *u, int32_t n_traj);

/* Triangle mesh of one environment's tissue surface, made on the device: the
 * paper's post-processing (Sec. III-A) extracts the surface from the mass
 * volume by marching cubes.  Density rho_i = sum_p w_ip m_p / dx^3 at every
 * node of the environment's grid (the P2G mass, quadratic B-spline weights),
 * then the surface rho = iso over the grid cells: a corner is inside when
 * rho >= iso; on each cell face the edges whose corners differ are crossed
 * (four crossings: two segments, each cutting off one inside corner); the
 * crossings chain into polygons, each a fan of triangles from its lowest
 * edge; crossing points interpolate rho linearly along the edge.  Triangles
 * are wound with their normal pointing out of the tissue and come out in
 * cell order (cell (i,j,k) of (n-1)^3, row-major); positions carry the
 * rounding of the density's float atomic sums, which can differ per call.  The surface is open where the tissue touches the grid's
 * outer faces.
 *   tris   float [max_tris][3][3]: vertex positions (m); device memory, or
 *          host memory from hipHostMalloc (the kernels then write it directly,
 *          with no separate copy).  Only the first max_tris are written.
 *   n_tris int64 [1], device or hipHostMalloc'd host memory: the number of
 *          triangles of the whole surface (may exceed max_tris).
 *   iso    density threshold (kg/m^3), > 0; half the material density puts
 *          the surface near the tissue boundary.
 * Stream-ordered, never synchronises; uses scratch sized for the largest
 * environment, so calls on one context must not overlap.  Afterwards
 * MPM_F_DENSITY reads the density volume. */
mpm_status mpm_extract_surface(mpm_ctx *ctx, int32_t env, float iso, float *tris, int64_t max_tris, int64_t *n_tris,
                               void *stream);

/* Set a tunable (MPM_OPT_*).  Takes effect at the next substep call. */
mpm_status mpm_set_option(mpm_ctx *ctx, int32_t option, int32_t value);

/* Advance every environment by n_substeps >= 1 substeps on `stream`.  One
 * substep is the MLS-MPM step of Sec. III-B: P2G of mass and APIC momentum
 * with the Neo-Hookean stress force (item 1, Eq. P2G and Eq. fip), the grid
 * operation with gravity, boundary nodes and tool contact (item 2, Sec.
 * III-C), and G2P with advection and the update of F (item 3).
 * record_tape != 0 starts a new adjoint tape at the current state and
 * records these substeps (n_substeps <= max_tape_substeps).  Never
 * synchronises. */
mpm_status mpm_substep(mpm_ctx *ctx, int32_t n_substeps, int32_t record_tape, void *stream);

/* Run one stage of a substep in isolation (Sec. III-B items 1-3), for
 * inspection and per-stage checking; not for throughput.  Direct stages:
 * P2G, then GRID, then G2P make one substep.  Tiled stages: TILED_P2G,
 * then TILED_GRID, then either TILED_G2P (one substep) or a fused stage
 * followed by TILED_GRID again (one more substep per fused stage), ending
 * with TILED_G2P.  A stage out of that order returns MPM_E_STATE and
 * launches nothing; so do mpm_substep, mpm_substep_adjoint,
 * mpm_extract_surface and the direct stages while a tiled sequence is open
 * (mpm_read_state may be called at any point).  A tiled sequence sorts only
 * at its start and advances the step counters and tool poses like the
 * mpm_substep calls it mirrors. */
mpm_status mpm_run_stage(mpm_ctx *ctx, int32_t stage, void *stream);

/* Reverse the last n_substeps recorded substeps (1 <= n <= tape length):
 * given adjoints of the current state, produce adjoints of the state n
 * substeps earlier and the parameter / tool gradients.  Restores tape
 * checkpoints and recomputes forward segments internally; the forward state
 * of the context is left as it was.  Returns MPM_E_STATE without a tape of
 * at least n substeps.  Never synchronises. */
mpm_status mpm_substep_adjoint(mpm_ctx *ctx, int32_t n_substeps, const mpm_adjoint_io *io,
                               void *stream);

/* Copy one field of environment env into dst (dst_bytes must equal the
 * field's size, else MPM_E_ARG; env out of range: MPM_E_ARG): the particle
 * state the simulator hands on each step (Sec. III-A: particle positions go
 * to surface extraction and rendering), the grid fields of Sec. III-B, the
 * status bits, tool positions and step counters.  dst_on_device != 0: dst is
 * device memory and the copy is asynchronous on `stream`; otherwise dst is
 * host memory and the call waits for `stream`.  Particle fields come back in
 * the original particle order. */
mpm_status mpm_read_state(mpm_ctx *ctx, int32_t env, int32_t field, void *dst, size_t dst_bytes,
                          int32_t dst_on_device, void *stream);

/* Built-in kernel timer.  enable != 0 starts recording: every kernel the
 * library launches on a context is bracketed by two hipEvents on its own
 * stream (adds a little host overhead; not available with MPM_OPT_GRAPH).
 * enable == 0 stops and keeps the totals.  Starting again clears them. */
mpm_status mpm_profile(mpm_ctx *ctx, int32_t enable);

/* Totals of kernel kind `kind` (0 <= kind < number of kinds; MPM_E_ARG past
 * the end): its name, summed event time in ms and launch count.  Waits for
 * the recorded events. */
mpm_status mpm_profile_read(mpm_ctx *ctx, int32_t kind, const char **name, double *total_ms,
                            int64_t *launches);

/* Message of the last failed call on ctx (or of the last failed mpm_create /
 * mpm_workspace_size when ctx is NULL). Never NULL. */
const char *mpm_last_error(const mpm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
