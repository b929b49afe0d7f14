// Tiled scheme: brick-sorted particles, LDS node tiles, fused G2P + P2G,
// node-brick work lists for the grid operation.
#pragma once
#include "mpm_kernels.h"

namespace mpm {

// Sort scratch and the resulting work items.
// Counting sort by cell of the stencil base, cells numbered brick-major
// (brick * 64 + cell within the 4^3-cell brick): particles of one brick are
// contiguous, and within it grouped by cell.
struct SortBuf {
    int32_t *count;        // [total_bricks * 64] particles per cell (zero between sorts)
    int32_t *brick_count;  // [total_bricks] particles per brick (zero between sorts)
    int32_t *offset;       // [total_bricks * 64] first slot of each cell (occupied bricks only)
    int2 *brick_offset;    // [total_bricks] (first slot, first item) before the chunk prefix
    int2 *chunk_sum;       // [chunks] exclusive prefix of each scan chunk of bricks
    int2 *totals;          // [1] (particles, items)
    int32_t *key;          // [ntot] cell of each particle
    int32_t *rank;         // [ntot] rank within the cell
    int4 *items;           // [max_items] (brick, first slot, count, environment)
};

struct ParticleBuf {
    float *x, *v, *C, *H;   // H = F - I
    int32_t *pid;
};

// Active node bricks: flag per brick and two compact lists used alternately
// (substep parity): P2G appends to list p, the grid operation of that
// substep consumes list p and clears the count of list p^1, which the next
// P2G fills.  A call's G2P-only tail clears both counts.
// Node bricks the grid operation visits.  The static list, rebuilt at every
// sort, holds the 27-brick neighbourhood of every occupied particle brick: all
// nodes a particle can reach while its stencil base stays within one cell of
// its sort-time brick.  A particle that has drifted further lists the bricks
// it reaches in a dynamic list (two, alternating with substep parity) that
// the next grid operation consumes and clears.
struct ActiveBuf {
    int32_t *flag;            // [nbricks] 0 unlisted, 1 static, 2 dynamic; nullptr: no bookkeeping
    int32_t *slist;           // [nbricks] static list
    int32_t *scount;          // [1]
    int32_t *dlist;           // [2][nbricks] dynamic lists
    int32_t *dcount;          // [2]
    const int32_t *env_bofs;  // [n_envs + 1] first brick of each environment
    const int32_t *brick_env; // [nbricks] environment of each brick
    int32_t nbricks;          // total bricks over all environments
    // persistent kernel: per-environment brick lists of a run (environment e's
    // entries at elist[env_bofs[e]..], ecount[e] of them); far bricks are
    // appended there instead of to the dynamic lists.  Null otherwise.
    int32_t *elist;
    int32_t *ecount;
};

// Tile geometry: the nodes reached by the stencils of a brick of 4^3 cells
// (bases 4B..4B+3, offsets 0..2): 6 nodes per axis.
constexpr int TILE = 6;
constexpr int TILE_NODES = TILE * TILE * TILE;

struct TiledArgs {
    const float *xin, *vin, *Cin, *Hin;   // particle input (sorted slots); H = F - I
    const int32_t *pidin;
    float *xout, *vout, *Cout, *Hout;     // particle output (tail: all; fused: x, H)
    int32_t *pidout;                      // copied when pidin != pidout
    const int4 *items;                    // (brick, first slot, count, environment)
    const int2 *totals;                   // .y = number of items
    int slots;                            // node pass: particles per half-wave step (1 or 3)
    ActiveBuf act;
    int par;                              // dynamic list this kernel's P2G appends to
    // Grid operation at tile staging (one launch per substep): the kernel reads
    // this substep's momentum gP_read and computes node velocities where it stages
    // them, writes the next substep's momentum to the Dev's gP, and clears gP_clear
    // (two substeps old) over the static brick list, or over the whole grid when
    // full_clear is set or its P2G reached a far brick (far_stamp[clear_slot] ==
    // clear_stamp; a P2G that reaches one stores write_stamp at write_slot).
    const float4 *gP_read;
    float4 *gP_clear;
    int64_t total_nodes;
    int full_clear;
    int *far_stamp;                       // [4]; null: far bricks go to the dynamic lists
    int write_slot, write_stamp, clear_slot, clear_stamp;
    const ToolPose *pose_in;              // [n_envs][max_tools] this substep's tool poses
    ToolPose *pose_out;                   // the next substep's (written by workgroup 0)
};

// Velocity tile of the grid-at-staging kernels: 8^3 nodes from the brick
// origin minus one, so a stencil base that has drifted one cell either way
// since the sort still reads the tile.
constexpr int GTILE = 8;
constexpr int GTILE_NODES = GTILE * GTILE * GTILE;

// Bricks per chunk of the sort's brick scan (brick_offset is a prefix within
// its chunk, chunk_sum the prefix of the chunks).
constexpr int SORT_SCAN_CHUNK = 1024;

// Most workgroups the persistent kernel launches (its group table's size).
constexpr int MAX_PERSISTENT_WG = 8192;
// Cost weight of a work item of z particles in the persistent kernel's work
// split: z + ITEM_FIXED_COST (the tile's staging and flush, in particles).
constexpr int ITEM_FIXED_COST = 96;

// Environment groups of the persistent kernel: workgroup b serves
// environments wg[b].x .. wg[b].x + wg[b].y - 1 as member wg[b].z of a group
// of wg[b].w workgroups (a group with several environments has one member).
struct EnvGroups {
    const int4 *wg;        // [launched workgroups]
    unsigned *arrive;      // [n_envs] barrier counters, zero at each launch
    SortBuf sort;          // the last sort: items per brick
    int nbricks;
};

// A persistent run of the grid-at-staging form (one environment): the call's
// fused substeps i0 .. i0 + m - 1 in one launch.  Substep i reads momentum
// buffer buf[i % 3], adds the next substep's into buf[(i + 1) % 3] and clears
// buf[(i + 2) % 3] for the substep after; its momentum carries stamp m0 + i.
struct GasRun {
    float4 *buf[3];
    const ToolPose *pose_in;   // tool poses at substep i0
    ToolPose *pose_out;        // at substep i0 + m (written by the last workgroup)
    unsigned *bar;             // RUN_BARRIER_WORDS counters, zero between launches
    int i0, m;
    int m0;
    int sorted_at;             // the call's substep before which a sort ran (-10: none)
    int spin_limit;
};
// The run's grid barrier: a counter per XCD, a global one, an exit count and
// a release word per XCD, each on its own 128-byte line.
constexpr int RUN_BARRIER_LINE = 32;
constexpr int RUN_BARRIER_WORDS = 18 * RUN_BARRIER_LINE;

// act.flag == nullptr: the static brick list is left as it is (act.brick_env is always used).
void launch_sort(const Dev &d, const SortBuf &s, const ActiveBuf &act, int total_bricks, int P,
                 const ParticleBuf &dst, int full, hipStream_t st);
size_t sort_chunk_count(int64_t n);   // scan chunks over n bricks

void launch_p2g_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st);
void launch_fused_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st);
void launch_g2p_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st);
// fused G2P + P2G that also writes v and C (d.gV: this substep's grid, d.gP: the next one's)
void launch_fused_full_tiled(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st);
void launch_grid_active(const Dev &d, const ActiveBuf &a, int par, int nblocks, bool sdf, hipStream_t st);
// Grid operation at staging: head P2G (initialises a.pose_out from the tool
// table), fused substep (grid operation of this substep in the staging, G2P,
// F update, advection, P2G of the next), tail (grid operation in the staging,
// G2P; writes v, C and the node velocities of the items' bricks, and the
// final tool poses into the table), and the clear of one momentum buffer.
void launch_gas_head(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st);
void launch_gas_fused(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st);
void launch_gas_tail(const Dev &d, const TiledArgs &a, int block, int nblocks, hipStream_t st);
void launch_gas_clear(const Dev &d, const TiledArgs &a, hipStream_t st);
void launch_gas_run(const Dev &d, const TiledArgs &a, const GasRun &r, int block, int nblocks, hipStream_t st);
// brick_env[b] = environment of brick b (once, at create)
void launch_brick_env(const int32_t *env_bofs, int n_envs, int nbricks, int32_t *brick_env, hipStream_t st);
// Persistent workgroup count for the tiled particle kernels at this block
// size: co-resident blocks per CU x CUs, a multiple of the 8 XCDs.
int tiled_workgroups(int block, bool gas = false);
int gas_run_workgroups(int block);   // 0: occupancy unknown
// Persistent kernel: m substeps of (grid operation, fused particle pass) per
// environment group, the last one a G2P-only tail if tail_last; groups
// synchronise through their own counters.  nblocks must not exceed
// persistent_workgroups(block) (all workgroups co-resident; 0 if unknown).
void launch_persistent(const Dev &d, const TiledArgs &first, const TiledArgs &rest, const EnvGroups &g, int m,
                       int tail_last, int spin_limit, bool sdf, int block, int nblocks, hipStream_t st);
int persistent_workgroups(int block);

}  // namespace mpm
