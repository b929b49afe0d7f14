// Host-side context of the C ABI: configuration, the carved workspace and
// the sequencing state.  Internal to the library.
#pragma once
#include <string>
#include <vector>

#include "mpm_adjoint.h"
#include "mpm_surface.h"

// Kernel kinds timed by the built-in profiler (mpm_profile_*).
enum ProfKind {
    PK_FILL = 0, PK_P2G_DIRECT, PK_GRID_DENSE, PK_G2P_DIRECT, PK_SORT, PK_P2G_TILED, PK_FUSED_TILED,
    PK_G2P_TILED, PK_GRID_ACTIVE, PK_ADJ_G2P, PK_ADJ_GRID, PK_ADJ_P2G, PK_ADJ_MISC, PK_PERSISTENT,
    PK_COUNT
};
static const char *const PROF_NAMES[PK_COUNT] = {
    "fill", "p2g_direct", "grid_dense", "g2p_direct", "sort", "p2g_tiled", "fused_g2p_p2g_tiled",
    "g2p_tiled", "grid_active", "adj_g2p", "adj_grid", "adj_p2g", "adj_misc",
    "persistent_tiled"};
// Kinds launched as one kernel: timed by the kernel's own start/end events;
// the others by events recorded around their launches.
static const bool PROF_SINGLE_KERNEL[PK_COUNT] = {
    true, true, true, true, false, true, true,
    true, true, true, true, true, false,
    true};

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;      // reusable events
    size_t used = 0;
    std::vector<std::pair<int, size_t>> marks;   // (kind, index of start event; stop = +1)
    double total_ms[PK_COUNT] = {};
    long long launches[PK_COUNT] = {};
};

// One captured call of n substeps (MPM_OPT_GRAPH) and the host-side
// sequencing state that call leaves behind.
struct GraphEntry {
    int n = 0, scheme = 0, block = 0, item = 0, sort_every = 0, persistent = 0, node_slots = 0, gas = 0;
    bool sdf = false;
    hipGraphExec_t exec = nullptr;
    int since_sort_after = 0;
};

struct mpm_ctx {
    std::string err;
    int static_dev = -1;             // device whose static workspace holds the buffers (mpm_create_static)
    // configuration
    int n_envs = 0, max_tools = 0, ntot = 0, bound = 0;
    float dt = 0.f, g[3] = {0.f, 0.f, 0.f};
    int checkpoint_every = 1, max_tape = 0;
    std::vector<int32_t> np, gn, pofs, bofs;
    std::vector<int64_t> gofs;
    int64_t total_nodes = 0;
    int32_t total_bricks = 0;
    const float *material = nullptr;
    hipStream_t stream0 = nullptr;
    // options
    int scheme = MPM_SCHEME_TILED, sort_every = 16, block = 256, item = 512, use_graph = 0, persistent = 0;
    int node_slots = 3;                // particles per half-wave step in the P2G node pass (1 or 3)
    int grid_at_staging = 0;           // one launch per substep (MPM_OPT_GRID_AT_STAGING)
    int spin_limit = 1 << 22;
    // device buffers carved from the caller's workspace
    mpm::EnvDev *env = nullptr;
    int32_t *env_pofs = nullptr;
    int64_t *env_gofs = nullptr;
    mpm::ToolDev *tools = nullptr;
    uint32_t *status = nullptr;
    int32_t *step = nullptr;
    float *x = nullptr, *v = nullptr, *C = nullptr, *H = nullptr;   // H = F - I
    int32_t *pid = nullptr;
    float4 *gP = nullptr, *gV = nullptr;
    // grid operation at staging: the other two momentum buffers of the rotation
    // (gP is the first), tool poses of two substeps, far-reach stamps, and the
    // number of momentum grids produced so far (stamp values)
    float4 *gP1 = nullptr, *gP2 = nullptr;
    mpm::ToolPose *poses = nullptr;   // [2][n_envs * max_tools]
    int32_t *far_stamp = nullptr;     // [4]
    int gas_count = 0;
    unsigned *run_bar = nullptr;      // [RUN_BARRIER_WORDS] barrier of the persistent grid-at-staging runs
    // tiled scheme
    mpm::ParticleBuf alt{};          // sort destination
    mpm::SortBuf sort{};
    mpm::ActiveBuf act{};
    int32_t *brick_env = nullptr;      // [total_bricks] environment of each brick
    int32_t *env_bofs = nullptr;
    int64_t max_items = 0;
    // sequencing state
    bool grid_clean = true;          // momentum buffer all zero, no active bricks
    bool has_sdf = false;            // some active tool is a sampled SDF (grid kernel instantiation)
    mpm::SurfBuf surf{};             // surface extraction scratch, sized for the largest environment
    int surf_env = -1;               // environment whose density the scratch holds
    bool items_valid = false;        // sort items match the current slot order and item size
    int items_P = 0;
    int since_sort = 0;
    int tiled_blocks = 0;            // persistent workgroups of the particle kernels
    int gas_blocks = 0;              // the same for the grid-at-staging kernels
    int run_blocks = 0;              // and for their persistent runs (all resident at once)
    // persistent kernel: environment groups (wg_tab) for groups_block threads and
    // groups_item particles per item, groups_n workgroups (0: not available)
    int groups_block = 0, groups_item = 0, groups_n = 0;
    // tiled stage sequence of mpm_run_stage: 0 none open, 1 a P2G awaits its grid
    // operation, 2 a grid operation awaits its particle pass
    int tstage = 0;
    int tstage_i = 0;                // substeps the open sequence has taken (dynamic-list parity)
    mpm::ParticleBuf tstage_in{};    // particle input of the sequence's next particle pass
    int4 *wg_tab = nullptr;          // [MAX_PERSISTENT_WG] workgroup -> (first env, env count, rank, group size)
    unsigned *arrive = nullptr;      // [2 n_envs] group barrier counters, then the run-list counts (ecount)
    int32_t *ecount = nullptr;       // = arrive + n_envs
    int32_t *elist = nullptr;        // [total_bricks] per-environment run lists of the persistent kernel
    // host mirror of the tool slots
    std::vector<mpm::ToolDev> tools_h;
    Profiler prof;
    // adjoint tape (carved only when max_tape > 0)
    struct Tape {
        int n_ckpt = 0;
        float *ckpt_state = nullptr;        // [n_ckpt][24][ntot], original order
        mpm::ToolDev *ckpt_tools = nullptr; // [n_ckpt][slots]
        int32_t *ckpt_step = nullptr;       // [n_ckpt][n_envs]
        float *seg_state = nullptr;         // [k + 1][24][ntot] state at each substep start
        mpm::ToolDev *seg_tools = nullptr;  // [k][slots]
        float4 *seg_P = nullptr, *seg_V = nullptr;   // [k][total_nodes]
        mpm::ContactCode *seg_dec = nullptr;         // [k][total_nodes]
        float *work = nullptr;              // [24][ntot] recompute state
        mpm::ToolDev *work_tools = nullptr;
        int32_t *work_step = nullptr;
        uint32_t *work_status = nullptr;
        mpm::AdjBuf adj{};
        float *adj_state = nullptr;         // [24][ntot] (xb, vb, Cb, Fb), original order
        float *adj_slot = nullptr;          // [24][ntot] the same in a segment's sorted slot order
        int32_t *perm = nullptr;            // [ntot] sorted slot -> original index of the current segment
        int32_t *iota = nullptr;            // [ntot] identity
        // the recompute's own static brick list (built by its sort) and far-reach
        // stamps per tape slot; tape grids are zero outside listed bricks between uses
        int32_t *tflag = nullptr, *tslist = nullptr, *tscount = nullptr;
        int32_t *tfar = nullptr;            // [k + 1]
        int stamp = 0;                      // stamp of the selected segment tape's recompute
        int stamp_top = 0;                  // largest stamp given out (stamps never repeat)
        int len = 0;                        // recorded substeps
        // Segment tapes: one, or (held tape) one per segment of the longest recording.  The
        // fields above point into the selected one; items and totals are its sort's work
        // items (with one segment tape, the live state's arrays).
        struct Seg {
            float *state = nullptr;
            mpm::ToolDev *tools = nullptr;
            float4 *P = nullptr, *V = nullptr;
            mpm::ContactCode *dec = nullptr;
            int32_t *perm = nullptr, *tflag = nullptr, *tslist = nullptr, *tscount = nullptr, *tfar = nullptr;
            int4 *items = nullptr;
            int2 *totals = nullptr;
            int stamp = 0;
            int dirty = 0;                  // slots whose tape grid P a recompute filled and no reverse cleared
        };
        std::vector<Seg> segs;
        int sel = 0;                        // the selected segment tape
        int held = 0;                       // segment tapes of the current recording already computed
        int4 *live_items = nullptr;         // the live state's work items (restored after a held tape)
        int2 *live_totals = nullptr;
    } tape;
    size_t tool_slots() const { return (size_t)n_envs * (max_tools > 0 ? max_tools : 1); }

    std::vector<GraphEntry> graphs;
    hipStream_t capture_stream = nullptr;

    ~mpm_ctx()
    {
        for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
        for (auto &g : graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
    }

    mpm::Dev dev() const
    {
        mpm::Dev d{};
        d.n_envs = n_envs;
        d.max_tools = max_tools;
        d.ntot = ntot;
        d.dt = dt;
        d.gx = g[0]; d.gy = g[1]; d.gz = g[2];
        d.env = env;
        d.env_pofs = env_pofs;
        d.material = material;
        d.tools = tools;
        d.status = status;
        d.step = step;
        d.x = x; d.v = v; d.C = C; d.H = H;
        d.pid = pid;
        d.gP = gP; d.gV = gV;
        return d;
    }
};
