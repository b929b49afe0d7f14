// C ABI of the MLS-MPM library: validation, workspace carving, sequencing of
// the kernels.  Every entry point catches everything and returns a status.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "mpm_ctx.h"

using namespace mpm;

static thread_local std::string g_last_error = "no error";

// Workspace of mpm_create_static: a device array of MPM_STATIC_WORKSPACE_BYTES
// in the library's code object, so each GPU the library runs on holds its own
// copy until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.  One context at a time may use a device's copy.
static __device__ __align__(256) unsigned char scratch[MPM_STATIC_WORKSPACE_BYTES];

namespace {

struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct Shape {
    int n_envs, max_tools, ntot;
    int64_t total_nodes, max_env_nodes, max_env_cells;
    int32_t total_bricks;
    int max_tape, ck;
    int hold;   // segment tapes kept for a whole recording
};

// One description of the workspace layout, used both to size and to carve it.
void carve(mpm_ctx &c, const Shape &s, Carver &cv)
{
    c.env = cv.take<EnvDev>(s.n_envs);
    c.env_pofs = cv.take<int32_t>(s.n_envs + 1);
    c.env_gofs = cv.take<int64_t>(s.n_envs + 1);
    c.tools = cv.take<ToolDev>((size_t)s.n_envs * std::max(1, s.max_tools));
    c.status = cv.take<uint32_t>(s.n_envs);
    c.step = cv.take<int32_t>(s.n_envs);
    c.x = cv.take<float>((size_t)3 * s.ntot);
    c.v = cv.take<float>((size_t)3 * s.ntot);
    c.C = cv.take<float>((size_t)9 * s.ntot);
    c.H = cv.take<float>((size_t)9 * s.ntot);
    c.pid = cv.take<int32_t>(s.ntot);
    c.gP = cv.take<float4>(s.total_nodes);
    c.gV = cv.take<float4>(s.total_nodes);
    c.gP1 = cv.take<float4>(s.total_nodes);
    c.gP2 = cv.take<float4>(s.total_nodes);
    c.poses = cv.take<ToolPose>((size_t)2 * s.n_envs * std::max(1, s.max_tools));
    c.far_stamp = cv.take<int32_t>(4);
    c.run_bar = cv.take<unsigned>(RUN_BARRIER_WORDS);
    // surface extraction
    c.surf.rho = cv.take<float>(s.max_env_nodes);
    c.surf.ofs = cv.take<int32_t>(s.max_env_cells);
    c.surf.chunk = cv.take<int32_t>(surf_chunk_count(s.max_env_cells));
    c.surf.table = cv.take<McTable>(1);
    // tiled scheme
    c.alt.x = cv.take<float>((size_t)3 * s.ntot);
    c.alt.v = cv.take<float>((size_t)3 * s.ntot);
    c.alt.C = cv.take<float>((size_t)9 * s.ntot);
    c.alt.H = cv.take<float>((size_t)9 * s.ntot);
    c.alt.pid = cv.take<int32_t>(s.ntot);
    c.sort.count = cv.take<int32_t>((size_t)s.total_bricks * 64);
    c.sort.brick_count = cv.take<int32_t>(s.total_bricks);
    c.sort.offset = cv.take<int32_t>((size_t)s.total_bricks * 64);
    c.sort.brick_offset = cv.take<int2>(s.total_bricks);
    c.sort.chunk_sum = cv.take<int2>(sort_chunk_count(s.total_bricks));
    c.sort.totals = cv.take<int2>(1);
    c.sort.key = cv.take<int32_t>(s.ntot);
    c.sort.rank = cv.take<int32_t>(s.ntot);
    c.max_items = (int64_t)s.total_bricks + s.ntot / 16 + 1;   // items of >= 16 particles
    c.sort.items = cv.take<int4>(c.max_items);
    c.act.flag = cv.take<int32_t>(s.total_bricks);
    c.act.slist = cv.take<int32_t>(s.total_bricks);
    c.act.scount = cv.take<int32_t>(1);
    c.act.dlist = cv.take<int32_t>((size_t)2 * s.total_bricks);
    c.act.dcount = cv.take<int32_t>(2);
    c.act.nbricks = s.total_bricks;
    c.brick_env = cv.take<int32_t>(s.total_bricks);
    c.act.brick_env = c.brick_env;
    c.env_bofs = cv.take<int32_t>(s.n_envs + 1);
    c.act.env_bofs = c.env_bofs;
    c.wg_tab = cv.take<int4>(MAX_PERSISTENT_WG);
    c.arrive = cv.take<unsigned>((size_t)2 * s.n_envs);
    c.ecount = c.arrive ? reinterpret_cast<int32_t *>(c.arrive + s.n_envs) : nullptr;
    c.elist = cv.take<int32_t>(s.total_bricks);
    // adjoint tape
    if (s.max_tape > 0) {
        const size_t st24 = (size_t)24 * s.ntot;
        const size_t slots = (size_t)s.n_envs * std::max(1, s.max_tools);
        const int k = s.ck;
        auto &T = c.tape;
        T.n_ckpt = (s.max_tape + k - 1) / k + 1;
        T.ckpt_state = cv.take<float>(st24 * T.n_ckpt);
        T.ckpt_tools = cv.take<ToolDev>(slots * T.n_ckpt);
        T.ckpt_step = cv.take<int32_t>((size_t)s.n_envs * T.n_ckpt);
        // segment tapes: one, or one per segment of the longest recording (held tape)
        const int nseg = s.hold ? (s.max_tape + k - 1) / k : 1;
        T.segs.assign(nseg, {});
        for (auto &g : T.segs) {
            g.state = cv.take<float>(st24 * (k + 1));
            g.tools = cv.take<ToolDev>(slots * k);
            g.P = cv.take<float4>((size_t)s.total_nodes * k);
            g.V = cv.take<float4>((size_t)s.total_nodes * k);
            g.dec = cv.take<ContactCode>((size_t)s.total_nodes * k);
            g.perm = cv.take<int32_t>(s.ntot);
            g.tflag = cv.take<int32_t>(s.total_bricks);
            g.tslist = cv.take<int32_t>(s.total_bricks);
            g.tscount = cv.take<int32_t>(1);
            g.tfar = cv.take<int32_t>(k + 1);
            g.items = s.hold ? cv.take<int4>(c.max_items) : c.sort.items;
            g.totals = s.hold ? cv.take<int2>(1) : c.sort.totals;
        }
        T.work = cv.take<float>(st24);
        T.work_tools = cv.take<ToolDev>(slots);
        T.work_step = cv.take<int32_t>(s.n_envs);
        T.work_status = cv.take<uint32_t>(s.n_envs);
        T.adj_state = cv.take<float>(st24);
        T.adj_slot = cv.take<float>(st24);
        T.iota = cv.take<int32_t>(s.ntot);
        T.live_items = c.sort.items;
        T.live_totals = c.sort.totals;
        const auto &g0 = T.segs[0];
        T.seg_state = g0.state; T.seg_tools = g0.tools; T.seg_P = g0.P; T.seg_V = g0.V; T.seg_dec = g0.dec;
        T.perm = g0.perm; T.tflag = g0.tflag; T.tslist = g0.tslist; T.tscount = g0.tscount; T.tfar = g0.tfar;
        T.adj.xb = T.adj_state;
        T.adj.vb = T.adj_state ? T.adj_state + (size_t)3 * s.ntot : nullptr;
        T.adj.Cb = T.adj_state ? T.adj_state + (size_t)6 * s.ntot : nullptr;
        T.adj.Fb = T.adj_state ? T.adj_state + (size_t)15 * s.ntot : nullptr;
        T.adj.gVb = cv.take<float4>(s.total_nodes);
        T.adj.gPb = cv.take<float4>(s.total_nodes);
        const size_t ng = slots * s.max_tape * 3;
        T.adj.ubar = cv.take<double>(ng);
        T.adj.Tbar = cv.take<double>(ng);
        T.adj.mubar = cv.take<double>(s.n_envs);
        T.adj.lambar = cv.take<double>(s.n_envs);
        T.adj.max_tape = s.max_tape;
    }
}

// Every device buffer the kernels use must have been carved.
bool all_carved(const mpm_ctx &c)
{
    const void *p[] = {c.env, c.env_pofs, c.env_gofs, c.tools, c.status, c.step, c.x, c.v, c.C, c.H, c.pid,
                       c.gP, c.gV, c.gP1, c.gP2, c.poses, c.far_stamp, c.run_bar, c.alt.x, c.alt.v, c.alt.C, c.alt.H, c.alt.pid, c.sort.count, c.sort.brick_count, c.sort.offset, c.sort.brick_offset,
                       c.sort.chunk_sum, c.sort.totals, c.sort.key, c.sort.rank, c.sort.items, c.act.flag,
                       c.act.slist, c.act.scount, c.act.dlist, c.act.dcount, c.brick_env, c.env_bofs, c.wg_tab, c.arrive, c.elist, c.act.env_bofs,
                       c.surf.rho, c.surf.ofs, c.surf.chunk, c.surf.table};
    for (const void *q : p)
        if (!q) return false;
    if (c.max_tape > 0) {
        const auto &T = c.tape;
        const void *t[] = {T.ckpt_state, T.ckpt_tools, T.ckpt_step, T.seg_state, T.seg_tools, T.seg_P, T.seg_V,
                           T.seg_dec, T.work, T.work_tools, T.work_step, T.work_status, T.adj_state, T.adj.gVb,
                           T.adj.gPb, T.adj.ubar, T.adj.Tbar, T.adj.mubar, T.adj.lambar, T.adj_slot, T.perm, T.iota,
                           T.tflag, T.tslist, T.tscount, T.tfar};
        for (const void *q : t)
            if (!q) return false;
        for (const auto &g : T.segs) {
            const void *u[] = {g.state, g.tools, g.P, g.V, g.dec, g.perm, g.tflag, g.tslist, g.tscount, g.tfar,
                               g.items, g.totals};
            for (const void *q : u)
                if (!q) return false;
        }
    }
    return true;
}

bool validate(const mpm_desc *d, std::string &why, Shape &s)
{
    if (!d) { why = "desc is NULL"; return false; }
    if (d->n_envs < 1 || d->n_envs > (1 << 20)) { why = "n_envs must be in [1, 2^20]"; return false; }
    if (!d->n_particles || !d->grid_n) { why = "n_particles and grid_n must be host arrays"; return false; }
    if (!(d->dt > 0.f) || !std::isfinite(d->dt)) { why = "dt must be finite and > 0"; return false; }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->gravity[a])) { why = "gravity must be finite"; return false; }
    if (d->bound < 0) { why = "bound must be >= 0"; return false; }
    if (d->max_tools < 0 || d->max_tools > MAX_TOOLS) { why = "max_tools must be in [0, 8]"; return false; }
    if (d->max_tape_substeps < 0) { why = "max_tape_substeps must be >= 0"; return false; }
    if (d->max_tape_substeps > 0 && d->checkpoint_every < 1) { why = "checkpoint_every must be >= 1"; return false; }
    if (d->hold_tape != 0 && d->hold_tape != 1) { why = "hold_tape must be 0 or 1"; return false; }
    if (!d->x0 || !d->v0 || !d->C0 || !d->F0 || !d->material) { why = "x0, v0, C0, F0 and material must be device pointers"; return false; }
    int64_t ntot = 0, nodes = 0, bricks = 0, max_nodes = 0, max_cells = 0;
    for (int e = 0; e < d->n_envs; ++e) {
        int n = d->grid_n[e];
        max_nodes = std::max(max_nodes, (int64_t)n * n * n);
        max_cells = std::max(max_cells, (int64_t)(n - 1) * (n - 1) * (n - 1));
        if (n < 8 || n > 512 || n % 4) { why = "grid_n[" + std::to_string(e) + "] must be a multiple of 4 in [8, 512]"; return false; }
        if (2 * d->bound >= n) { why = "bound leaves no interior nodes"; return false; }
        if (d->n_particles[e] < 1) { why = "n_particles[" + std::to_string(e) + "] must be >= 1"; return false; }
        ntot += d->n_particles[e];
        nodes += (int64_t)n * n * n;
        bricks += (int64_t)(n / 4) * (n / 4) * (n / 4);
    }
    if (ntot > (1ll << 30)) { why = "too many particles (max 2^30)"; return false; }
    if (nodes > (1ll << 30)) { why = "too many grid nodes (max 2^30 over all environments)"; return false; }
    s.n_envs = d->n_envs;
    s.max_tools = d->max_tools;
    s.max_tape = d->max_tape_substeps;
    s.ck = d->max_tape_substeps > 0 ? std::min(d->checkpoint_every, d->max_tape_substeps) : 1;
    s.hold = d->max_tape_substeps > 0 && d->hold_tape != 0;
    s.ntot = (int)ntot;
    s.total_nodes = nodes;
    s.max_env_nodes = max_nodes;
    s.max_env_cells = max_cells;
    s.total_bricks = (int32_t)bricks;
    return true;
}

mpm_status fail(mpm_ctx *c, mpm_status code, const std::string &msg)
{
    if (c) c->err = msg;
    g_last_error = msg;
    return code;
}

#define HIP_TRY(ctx, call)                                                                      \
    do {                                                                                        \
        hipError_t _e = (call);                                                                 \
        if (_e != hipSuccess)                                                                   \
            return fail(ctx, MPM_E_HIP, std::string(#call) + ": " + hipGetErrorString(_e));     \
    } while (0)

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

mpm_status check_launch(mpm_ctx *c, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, MPM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return MPM_OK;
}

// Built-in profiler: when on, each launch is bracketed by two events on its
// stream; mpm_profile_read() resolves them.
hipEvent_t prof_event(mpm_ctx *c)
{
    Profiler &P = c->prof;
    if (P.used == P.pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        P.pool.push_back(e);
    }
    return P.pool[P.used++];
}

template <class F>
void timed(mpm_ctx *c, hipStream_t st, int kind, F &&launch)
{
    if (!c->prof.on) { launch(); return; }
    size_t i0 = c->prof.used;
    hipEvent_t a = prof_event(c), b = prof_event(c);
    if (!a || !b) { launch(); return; }
    if (PROF_SINGLE_KERNEL[kind]) {
        // the kernel itself records its start and end
        launch_timer = LaunchTimer{a, b, false};
        launch();
        const bool used = launch_timer.used;
        launch_timer = LaunchTimer{};
        if (used) c->prof.marks.emplace_back(kind, i0);
        return;
    }
    (void)hipEventRecord(a, st);
    launch();
    (void)hipEventRecord(b, st);
    c->prof.marks.emplace_back(kind, i0);
}

void prof_resolve(mpm_ctx *c)
{
    Profiler &P = c->prof;
    for (auto &m : P.marks) {
        float ms = 0.f;
        if (hipEventSynchronize(P.pool[m.second + 1]) == hipSuccess &&
            hipEventElapsedTime(&ms, P.pool[m.second], P.pool[m.second + 1]) == hipSuccess) {
            P.total_ms[m.first] += ms;
            P.launches[m.first] += 1;
        }
    }
    P.marks.clear();
    P.used = 0;
}

// One substep of the direct scheme.  Leaves the last P2G in the momentum
// buffer (readable), so the grid is not clean afterwards.
void substep_direct(mpm_ctx *c, hipStream_t st)
{
    Dev d = c->dev();
    timed(c, st, PK_FILL, [&] { launch_fill_f4(c->gP, c->total_nodes, st); });
    timed(c, st, PK_P2G_DIRECT, [&] { launch_p2g_direct(d, st); });
    timed(c, st, PK_GRID_DENSE, [&] { launch_grid_dense(d, c->env_gofs, c->total_nodes, 0, st); });
    timed(c, st, PK_G2P_DIRECT, [&] { launch_g2p_direct(d, st); });
    c->grid_clean = false;
}

ParticleBuf live(const mpm_ctx *c) { return ParticleBuf{c->x, c->v, c->C, c->H, c->pid}; }

TiledArgs tiled_args(const mpm_ctx *c, const ParticleBuf &in, const ParticleBuf &out, int par)
{
    TiledArgs a{};
    a.xin = in.x; a.vin = in.v; a.Cin = in.C; a.Hin = in.H; a.pidin = in.pid;
    a.xout = out.x; a.vout = out.v; a.Cout = out.C; a.Hout = out.H; a.pidout = out.pid;
    a.items = c->sort.items;
    a.totals = c->sort.totals;
    a.slots = c->node_slots;
    a.act = c->act;
    a.par = par;
    return a;
}

// Sort live particles into the alternate buffers and rebuild the items.
// mid_call: between the fused substeps of a call, where v and C are carried
// by frozen particles only (the sort moves them for particles near the
// domain edge); otherwise the whole state moves.
void sort_into_alt(mpm_ctx *c, hipStream_t st, bool mid_call = false)
{
    timed(c, st, PK_SORT, [&] {
        launch_sort(c->dev(), c->sort, c->act, c->total_bricks, c->item, c->alt, mid_call ? 0 : 1, st);
    });
    c->items_valid = true;
    c->items_P = c->item;
    c->since_sort = 0;
}

int grid_blocks(const mpm_ctx *c)
{
    // one wavefront per brick up to 64K listed bricks; beyond that waves take several
    int64_t b = ((int64_t)c->total_bricks + 3) / 4;
    return (int)std::max<int64_t>(8, std::min<int64_t>(b, 16384));
}

// Work of each environment in one substep of the persistent kernel, in
// particle-equivalents, from the current positions (counted on the host):
// its particles, a fixed cost per work item (bricks it occupies, at most
// `item` particles per item) and per brick of the static neighbourhood the
// grid operation visits.  The kernel's own per-item split uses the same
// fixed cost.
mpm_status work_estimate(mpm_ctx *c, std::vector<int64_t> &work)
{
    std::vector<float> x((size_t)3 * c->ntot);
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(x.data(), c->x, x.size() * sizeof(float), hipMemcpyDeviceToHost));
    const size_t N = c->ntot;
    work.assign(c->n_envs, 0);
    std::vector<int32_t> cnt;
    std::vector<uint8_t> near;
    for (int e = 0; e < c->n_envs; ++e) {
        const int n = c->gn[e], nb = n / 4;
        cnt.assign((size_t)nb * nb * nb, 0);
        for (int p = c->pofs[e]; p < c->pofs[e + 1]; ++p) {
            int t[3];
            for (int a = 0; a < 3; ++a) {
                const float v = x[a * N + p] * n - 0.5f;
                t[a] = std::isfinite(v) ? (int)std::floor(std::min(std::max(v, 0.0f), (float)(n - 3))) : 0;
            }
            ++cnt[((size_t)(t[0] >> 2) * nb + (t[1] >> 2)) * nb + (t[2] >> 2)];
        }
        near.assign(cnt.size(), 0);
        int64_t items = 0, bricks = 0;
        for (int bi = 0; bi < nb; ++bi)
            for (int bj = 0; bj < nb; ++bj)
                for (int bk = 0; bk < nb; ++bk) {
                    const int k = cnt[((size_t)bi * nb + bj) * nb + bk];
                    if (!k) continue;
                    items += (k + c->item - 1) / c->item;
                    for (int a = std::max(bi - 1, 0); a <= std::min(bi + 1, nb - 1); ++a)
                        for (int b = std::max(bj - 1, 0); b <= std::min(bj + 1, nb - 1); ++b)
                            for (int q = std::max(bk - 1, 0); q <= std::min(bk + 1, nb - 1); ++q)
                                near[((size_t)a * nb + b) * nb + q] = 1;
                }
        for (uint8_t f : near) bricks += f;
        work[e] = c->np[e] + (int64_t)ITEM_FIXED_COST * items + 16 * bricks;
    }
    return MPM_OK;
}

// Environment groups of the persistent kernel for the current block and item
// sizes.  Each environment gets workgroups in proportion to the work items of
// its particles (at least one, at most one per item); when there are more
// environments than workgroups, consecutive environments share one workgroup
// (a group of one member, which never waits).  Host computation and
// synchronous copies: called from mpm_set_option, never under stream capture.
mpm_status build_groups(mpm_ctx *c)
{
    c->groups_n = 0;
    c->groups_block = c->block;
    c->groups_item = c->item;
    const int G = std::min(persistent_workgroups(c->block), MAX_PERSISTENT_WG);
    if (G <= 0) return MPM_OK;   // occupancy unknown: the persistent option falls back to per-phase launches
    const int E = c->n_envs;
    std::vector<int4> tab;
    std::vector<int64_t> work;
    if (mpm_status r = work_estimate(c, work)) return r;
    int64_t total = 0;
    for (int e = 0; e < E; ++e) total += work[e];
    if (E > G) {
        // consecutive environments per workgroup, each filled to about the
        // particles left over the workgroups left; the last takes the rest
        double left = (double)total;
        int e = 0;
        for (int b = 0; b < G && e < E; ++b) {
            const double target = left / (G - b);
            const int first = e;
            double w = 0.0;
            do {
                w += work[e];
                ++e;
            } while (e < E && (b == G - 1 || w + 0.5 * work[e] <= target));
            left -= w;
            tab.push_back(make_int4(first, e - first, 0, 1));
        }
    } else {
        std::vector<int> g(E);
        int used = 0;
        for (int e = 0; e < E; ++e) {
            const int cap = std::max(1, (int)(work[e] / (c->item + ITEM_FIXED_COST)) + 1);
            g[e] = std::min(cap, std::max(1, (int)((double)G * work[e] / total)));
            used += g[e];
        }
        while (used > G) {   // at least one each: take back from the largest groups
            int big = 0;
            for (int e = 1; e < E; ++e) if (g[e] > g[big]) big = e;
            --g[big]; --used;
        }
        for (bool grew = true; used < G && grew;) {   // spare workgroups to the most loaded groups
            grew = false;
            int best = -1;
            double load = 0.0;
            for (int e = 0; e < E; ++e) {
                const int cap = std::max(1, (int)(work[e] / (c->item + ITEM_FIXED_COST)) + 1);
                if (g[e] >= cap) continue;
                const double l = (double)work[e] / g[e];
                if (l > load) { load = l; best = e; }
            }
            if (best >= 0) { ++g[best]; ++used; grew = true; }
        }
        for (int e = 0; e < E; ++e)
            for (int r = 0; r < g[e]; ++r) tab.push_back(make_int4(e, 1, r, g[e]));
    }
    const int n = (int)tab.size();
    HIP_TRY(c, hipMemcpy(c->wg_tab, tab.data(), sizeof(int4) * n, hipMemcpyHostToDevice));
    c->groups_n = n;
    return MPM_OK;
}

// n substeps with the grid operation at tile staging, one launch per substep.
// Momentum grids rotate over three buffers: substep i (0-based) reads
// buf[i % 3], its P2G writes buf[(i + 1) % 3], and it clears buf[(i + 2) % 3],
// which held the momentum of substep i - 1 (read by the launch before).  A
// clear covers the static brick list, or the whole grid when that momentum was
// written before the last sort (a different static list) or reached a brick
// outside its neighbourhood (a stamp).  The call ends with the clear of the
// buffer the tail read, so every call starts and ends with all three zero.
// Tool poses alternate between two pose arrays.  Particles enter from `in`
// (the sort destination right after a sort).
void substeps_gas(mpm_ctx *c, int n, ParticleBuf in, hipStream_t st)
{
    float4 *buf[3] = {c->gP, c->gP1, c->gP2};
    const size_t slots = c->tool_slots();
    ToolPose *pose[2] = {c->poses, c->poses + slots};
    if (c->gas_blocks == 0) c->gas_blocks = tiled_workgroups(c->block, true);
    const int nb = c->gas_blocks;
    const ParticleBuf A = live(c);
    const int m0 = c->gas_count;   // stamp of substep i's momentum: m0 + i
    int sorted_at = -10;   // substep before which a sort ran mid-call (a sort before the head needs nothing)
    auto args = [&](const ParticleBuf &i_, const ParticleBuf &o_) {
        TiledArgs a = tiled_args(c, i_, o_, 0);
        a.total_nodes = c->total_nodes;
        a.far_stamp = c->far_stamp;
        return a;
    };
    {
        Dev d = c->dev();
        d.gP = buf[0];
        TiledArgs a = args(in, in);
        a.write_slot = m0 & 3;
        a.write_stamp = m0;
        a.pose_out = pose[0];
        timed(c, st, PK_P2G_TILED, [&] { launch_gas_head(d, a, c->block, nb, st); });
    }
    // persistent runs (one environment): the fused substeps between sorts, one launch each
    if (c->persistent && c->n_envs == 1 && c->run_blocks == 0) c->run_blocks = gas_run_workgroups(c->block);
    const bool runs = c->persistent && c->n_envs == 1 && c->run_blocks > 0;
    for (int i = 0; runs && i < n - 1;) {
        if (i > 0 && c->since_sort >= c->sort_every && in.x == A.x) {
            sort_into_alt(c, st, true);
            in = c->alt;
            sorted_at = i;
        }
        const int m = std::max(1, std::min(n - 1 - i, c->sort_every - c->since_sort));
        GasRun r{};
        r.buf[0] = buf[0]; r.buf[1] = buf[1]; r.buf[2] = buf[2];
        r.pose_in = pose[i & 1];
        r.pose_out = pose[(i + m) & 1];
        r.bar = c->run_bar;
        r.i0 = i;
        r.m = m;
        r.m0 = m0;
        r.sorted_at = sorted_at;
        r.spin_limit = c->spin_limit;
        const TiledArgs a = args(in, A);
        timed(c, st, PK_PERSISTENT, [&] { launch_gas_run(c->dev(), a, r, c->block, c->run_blocks, st); });
        in = A;
        i += m;
        c->since_sort += m;
    }
    for (int i = runs ? n - 1 : 0; i < n; ++i) {
        if (i > 0 && i < n - 1 && c->since_sort >= c->sort_every && in.x == A.x) {
            sort_into_alt(c, st, true);
            in = c->alt;
            sorted_at = i;
        }
        const bool tail = i == n - 1;
        Dev d = c->dev();
        d.gP = tail ? nullptr : buf[(i + 1) % 3];
        TiledArgs a = args(in, A);
        a.gP_read = buf[i % 3];
        a.gP_clear = i >= 1 ? buf[(i + 2) % 3] : nullptr;
        // the momentum of substep i - 1 was written under the old static list if a sort ran before i or i - 1
        a.full_clear = (sorted_at == i || sorted_at == i - 1) ? 1 : 0;
        a.clear_slot = (m0 + i - 1) & 3;
        a.clear_stamp = m0 + i - 1;
        a.write_slot = (m0 + i + 1) & 3;
        a.write_stamp = m0 + i + 1;
        a.pose_in = pose[i & 1];
        a.pose_out = pose[(i + 1) & 1];
        if (tail) timed(c, st, PK_G2P_TILED, [&] { launch_gas_tail(d, a, c->block, nb, st); });
        else timed(c, st, PK_FUSED_TILED, [&] { launch_gas_fused(d, a, c->block, nb, st); });
        in = A;
        c->since_sort += 1;
    }
    // the tail read buf[(n - 1) % 3]: clear it for the next call
    TiledArgs a = args(A, A);
    a.gP_clear = buf[(n - 1) % 3];
    a.full_clear = sorted_at == n - 1 ? 1 : 0;
    a.clear_slot = (m0 + n - 1) & 3;
    a.clear_stamp = m0 + n - 1;
    timed(c, st, PK_FILL, [&] { launch_gas_clear(c->dev(), a, st); });
    c->gas_count = m0 + n;
}

// n substeps of the tiled scheme:
//   [sort] head P2G, then n x (grid op, fused G2P+P2G) with the last fused
//   step replaced by a G2P-only tail that materialises v and C.
void substeps_tiled(mpm_ctx *c, int n, hipStream_t st)
{
    Dev d = c->dev();
    if (!c->grid_clean) {
        timed(c, st, PK_FILL, [&] { launch_fill_f4(c->gP, c->total_nodes, st); });
        c->grid_clean = true;
    }
    if (c->tiled_blocks == 0) c->tiled_blocks = tiled_workgroups(c->block);
    const int nb = c->tiled_blocks;
    ParticleBuf A = live(c), in = A;
    if (!c->items_valid || c->items_P != c->item || c->since_sort >= c->sort_every) {
        sort_into_alt(c, st);
        in = c->alt;
    }
    // grid at staging: per-substep launches, or persistent runs for one environment; where
    // the form does not apply (a sampled-SDF tool) the substeps take the per-phase launches
    const bool gas = c->grid_at_staging && (!c->persistent || c->n_envs == 1);
    if (gas && !c->has_sdf) {
        substeps_gas(c, n, in, st);
        return;
    }
    const bool pers = !gas && c->persistent && c->groups_n > 0 && c->groups_block == c->block &&
                      c->groups_item == c->item;
    if (pers) {
        // runs of up to sort_every substeps, one persistent launch each, sorts in
        // between; the kernel finds far-drift bricks by their flags (no dynamic lists)
        auto args = [&](const ParticleBuf &i, const ParticleBuf &o) {
            TiledArgs a = tiled_args(c, i, o, 0);
            a.act.elist = c->elist;
            a.act.ecount = c->ecount;
            return a;
        };
        timed(c, st, PK_P2G_TILED, [&] { launch_p2g_tiled(d, args(in, in), c->block, nb, st); });
        const EnvGroups g{c->wg_tab, c->arrive, c->sort, c->total_bricks};
        for (int done = 0; done < n;) {
            if (done > 0) {
                sort_into_alt(c, st, true);
                in = c->alt;
            }
            const int m = std::min(n - done, c->sort_every);
            const int tail = done + m == n;
            timed(c, st, PK_FILL, [&] { launch_fill_u32(c->arrive, 2 * c->n_envs, 0u, st); });
            timed(c, st, PK_PERSISTENT, [&] {
                launch_persistent(d, args(in, A), args(A, A), g, m, tail, c->spin_limit, c->has_sdf, c->block,
                                  c->groups_n, st);
            });
            in = A;
            done += m;
            c->since_sort = m;
        }
        return;
    }
    // substep i: P2G lists far bricks in dynamic list i&1, its grid operation consumes it
    timed(c, st, PK_P2G_TILED, [&] { launch_p2g_tiled(d, tiled_args(c, in, in, 0), c->block, nb, st); });
    for (int i = 0; i < n; ++i) {
        timed(c, st, PK_GRID_ACTIVE, [&] { launch_grid_active(d, c->act, i & 1, grid_blocks(c), c->has_sdf, st); });
        if (i == n - 1) {
            timed(c, st, PK_G2P_TILED, [&] { launch_g2p_tiled(d, tiled_args(c, in, A, 0), c->block, nb, st); });
        } else {
            if (c->since_sort >= c->sort_every && in.x == A.x) {
                sort_into_alt(c, st, true);
                in = c->alt;
            }
            timed(c, st, PK_FUSED_TILED, [&] { launch_fused_tiled(d, tiled_args(c, in, A, (i + 1) & 1), c->block, nb, st); });
            in = A;
        }
        c->since_sort += 1;
    }
}


void run_substeps(mpm_ctx *c, int n, hipStream_t st)
{
    if (c->scheme == MPM_SCHEME_TILED) substeps_tiled(c, n, st);
    else for (int i = 0; i < n; ++i) substep_direct(c, st);
}

// MPM_OPT_GRAPH: replay a captured call of n substeps.  The captured
// sequence sorts at the start of the call and every sort_every substeps, so it
// depends only on (n, options); fills needed before it run outside the graph.
mpm_status run_substeps_graph(mpm_ctx *c, int n, hipStream_t st)
{
    if (!c->grid_clean) {
        launch_fill_f4(c->gP, c->total_nodes, st);
        c->grid_clean = true;
    }
    GraphEntry *ge = nullptr;
    for (auto &g : c->graphs)
        if (g.n == n && g.scheme == c->scheme && g.block == c->block && g.item == c->item &&
            g.sort_every == c->sort_every && g.persistent == c->persistent && g.node_slots == c->node_slots &&
            g.sdf == c->has_sdf && g.gas == c->grid_at_staging)
            ge = &g;
    if (!ge) {
        if (c->scheme == MPM_SCHEME_TILED && c->tiled_blocks == 0) c->tiled_blocks = tiled_workgroups(c->block);
        if (!c->capture_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
        c->items_valid = false;               // force the sort at the start of the captured call
        hipGraph_t graph = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
        run_substeps(c, n, c->capture_stream);
        hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
        if (e != hipSuccess) return fail(c, MPM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        GraphEntry g;
        g.n = n; g.scheme = c->scheme; g.block = c->block; g.item = c->item; g.sort_every = c->sort_every;
        g.persistent = c->persistent;
        g.node_slots = c->node_slots;
        g.sdf = c->has_sdf;
        g.gas = c->grid_at_staging;
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(c, MPM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        g.since_sort_after = c->since_sort;
        c->graphs.push_back(g);
        ge = &c->graphs.back();
    }
    HIP_TRY(c, hipGraphLaunch(ge->exec, st));
    if (c->scheme == MPM_SCHEME_TILED) {
        c->items_valid = true;
        c->items_P = c->item;
        c->since_sort = ge->since_sort_after;
    } else {
        c->grid_clean = false;
    }
    return MPM_OK;
}

// Kernel view of a [24][ntot] particle block: x(3) v(3) C(9) F(9).
Dev state_view(const mpm_ctx *c, float *blk)
{
    Dev d = c->dev();
    const size_t N = c->ntot;
    d.x = blk;
    d.v = blk + 3 * N;
    d.C = blk + 6 * N;
    d.H = blk + 15 * N;
    d.pid = nullptr;
    return d;
}

// Checkpoint k of the tape: live state in original order, tool table, steps.
void save_checkpoint(mpm_ctx *c, int k, hipStream_t st)
{
    auto &T = c->tape;
    const size_t N = c->ntot;
    float *dst = T.ckpt_state + (size_t)k * 24 * N;
    timed(c, st, PK_ADJ_MISC, [&] {
        launch_unpermute(c->x, c->pid, c->ntot, 3, dst, st);
        launch_unpermute(c->v, c->pid, c->ntot, 3, dst + 3 * N, st);
        launch_unpermute(c->C, c->pid, c->ntot, 9, dst + 6 * N, st);
        launch_unpermute(c->H, c->pid, c->ntot, 9, dst + 15 * N, st);
        launch_copies({{T.ckpt_tools + (size_t)k * c->tool_slots(), c->tools, sizeof(ToolDev) * c->tool_slots()},
                       {T.ckpt_step + (size_t)k * c->n_envs, c->step, sizeof(int32_t) * c->n_envs}},
                      st);
    });
}

// The recompute's brick bookkeeping: its own static list (built by the
// segment's sort, so the forward's lists are left as they were); far reaches
// are stamped, not listed.
// Point the tape's segment fields and the sort's work items at segment tape b
// (with one segment tape the items are the live state's, as before).
void select_seg(mpm_ctx *c, int b)
{
    auto &T = c->tape;
    const auto &g = T.segs[b];
    T.seg_state = g.state; T.seg_tools = g.tools; T.seg_P = g.P; T.seg_V = g.V; T.seg_dec = g.dec;
    T.perm = g.perm; T.tflag = g.tflag; T.tslist = g.tslist; T.tscount = g.tscount; T.tfar = g.tfar;
    c->sort.items = g.items;
    c->sort.totals = g.totals;
    T.stamp = g.stamp;
    T.sel = b;
}

// Back to the live state's work items after using held segment tapes.
void select_live_items(mpm_ctx *c)
{
    c->sort.items = c->tape.live_items;
    c->sort.totals = c->tape.live_totals;
}

ActiveBuf tape_act(const mpm_ctx *c)
{
    ActiveBuf a = c->act;
    a.flag = c->tape.tflag;
    a.slist = c->tape.tslist;
    a.scount = c->tape.tscount;
    a.dlist = nullptr;
    a.dcount = nullptr;
    a.elist = nullptr;
    a.ecount = nullptr;
    return a;
}

// Nodes a tape grid pass of slot `slot` visits (the tape's static list, or all
// of them if that slot's P2G reached beyond it).
TapeList tape_list(const mpm_ctx *c, int slot)
{
    const auto &T = c->tape;
    return TapeList{T.tslist, T.tscount, c->brick_env, T.tfar, slot, T.stamp, 0};
}

TapeList dense_list(const mpm_ctx *c)
{
    const auto &T = c->tape;
    return TapeList{T.tslist, T.tscount, c->brick_env, T.tfar, 0, 0, 1};
}

// Recompute substeps [s_begin, s_end) from checkpoint `seg`, keeping each
// substep's starting state, tool table, grid (m, vhat), node velocities and
// contact decisions in the segment tape.  Uses the direct-scheme kernels on
// the tape's own buffers; the live state is not touched.
void recompute_segment(mpm_ctx *c, int seg, int s_begin, int s_end, hipStream_t st)
{
    auto &T = c->tape;
    const size_t N = c->ntot, slots = c->tool_slots();
    timed(c, st, PK_ADJ_MISC, [&] {
        launch_copies({{T.work, T.ckpt_state + (size_t)seg * 24 * N, sizeof(float) * 24 * N},
                       {T.work_tools, T.ckpt_tools + (size_t)seg * slots, sizeof(ToolDev) * slots},
                       {T.work_step, T.ckpt_step + (size_t)seg * c->n_envs, sizeof(int32_t) * c->n_envs}},
                      st);
    });
    for (int j = s_begin; j < s_end; ++j) {
        const int slot = j - s_begin;
        Dev d = state_view(c, T.work);
        d.tools = T.work_tools;
        d.step = T.work_step;
        d.status = T.work_status;
        d.gP = T.seg_P + (size_t)slot * c->total_nodes;
        d.gV = T.seg_V + (size_t)slot * c->total_nodes;
        timed(c, st, PK_ADJ_MISC, [&] {
            launch_copies({{T.seg_state + (size_t)slot * 24 * N, T.work, sizeof(float) * 24 * N},
                           {T.seg_tools + (size_t)slot * slots, T.work_tools, sizeof(ToolDev) * slots}},
                          st);
            launch_fill_f4(d.gP, c->total_nodes, st);
        });
        timed(c, st, PK_P2G_DIRECT, [&] { launch_p2g_direct(d, st); });
        timed(c, st, PK_GRID_DENSE, [&] {
            launch_grid_tape(d, c->env_gofs, c->total_nodes, T.seg_dec + (size_t)slot * c->total_nodes, nullptr, 0,
                             dense_list(c), st);
        });
        timed(c, st, PK_G2P_DIRECT, [&] { launch_g2p_direct(d, st); });
    }
}

// Tape bookkeeping without active-brick flags (the tape's grid passes are dense).
ParticleBuf seg_view(const mpm_ctx *c, int slot)
{
    const size_t N = c->ntot;
    float *b = c->tape.seg_state + (size_t)slot * 24 * N;
    return ParticleBuf{b, b + 3 * N, b + 6 * N, b + 15 * N, c->tape.perm};
}

// Tiled recompute of substeps [s_begin, s_end) from checkpoint `seg`: the
// checkpoint is counting-sorted by brick into tape slot 0 (its permutation
// kept), then each substep runs the tiled P2G head into its own tape grid,
// the dense tape grid pass, and the tiled G2P tail writing the next slot.
void recompute_segment_tiled(mpm_ctx *c, int seg, int s_begin, int s_end, hipStream_t st, const Dev *src = nullptr)
{
    auto &T = c->tape;
    const size_t N = c->ntot, slots = c->tool_slots();
    // a held recording that was not reversed (or only partly) left its grids in this
    // segment tape: clear them, over the bricks its recompute listed, before the sort
    // below replaces that list
    for (int slot = 0; slot < T.segs[T.sel].dirty; ++slot) {
        Dev d = c->dev();
        d.gP = T.seg_P + (size_t)slot * c->total_nodes;
        timed(c, st, PK_ADJ_MISC, [&] { launch_tape_clear(d, c->env_gofs, c->total_nodes, tape_list(c, slot), st); });
    }
    // the sort's input: the checkpoint (original order), or src, the same state held
    // elsewhere with its particle index
    Dev dc = state_view(c, T.ckpt_state + (size_t)seg * 24 * N);
    dc.pid = T.iota;
    if (src) dc = *src;
    timed(c, st, PK_SORT, [&] { launch_sort(dc, c->sort, tape_act(c), c->total_bricks, c->item, seg_view(c, 0), 1, st); });
    c->items_valid = false;   // the live state's work items were overwritten
    if (c->tiled_blocks == 0) c->tiled_blocks = tiled_workgroups(c->block);
    timed(c, st, PK_ADJ_MISC, [&] {
        launch_copies({{T.work_tools, T.ckpt_tools + (size_t)seg * slots, sizeof(ToolDev) * slots},
                       {T.work_step, T.ckpt_step + (size_t)seg * c->n_envs, sizeof(int32_t) * c->n_envs}},
                      st);
    });
    const ActiveBuf ta = tape_act(c);
    // substep j: grid pass on slot j's P, then G2P(j) into slot j + 1 fused with P2G(j + 1)
    // into slot j + 1's P (the last substep: G2P only)
    auto slot_dev = [&](int slot) {
        Dev d = c->dev();
        d.tools = T.work_tools;
        d.step = T.work_step;
        d.status = T.work_status;
        d.gP = T.seg_P + (size_t)slot * c->total_nodes;
        d.gV = T.seg_V + (size_t)slot * c->total_nodes;
        return d;
    };
    // tape grids are zero outside the listed bricks (the reverse grid pass clears what it
    // visits), so no P needs clearing here; a P2G that reaches beyond the list stamps its slot
    // with a stamp no earlier recompute used
    T.stamp = ++T.stamp_top;
    T.segs[T.sel].stamp = T.stamp;
    // P2G fills the grids of slots 0 .. s_end - s_begin - 1; the reverse, or the clears of
    // the substeps before its window, zero them again
    T.segs[T.sel].dirty = s_end - s_begin;
    auto stamped = [&](TiledArgs a, int slot) {
        a.act = ta;
        a.far_stamp = T.tfar;
        a.write_slot = slot;
        a.write_stamp = T.stamp;
        return a;
    };
    {
        Dev d = slot_dev(0);
        ParticleBuf in = seg_view(c, 0);
        const TiledArgs head = stamped(tiled_args(c, in, in, 0), 0);
        timed(c, st, PK_P2G_TILED, [&] { launch_p2g_tiled(d, head, c->block, c->tiled_blocks, st); });
    }
    for (int j = s_begin; j < s_end; ++j) {
        const int slot = j - s_begin;
        const bool last = j + 1 == s_end;
        Dev d = slot_dev(slot);
        // the grid pass also snapshots the tool table
        float4 *next_P = last ? nullptr : T.seg_P + (size_t)(slot + 1) * c->total_nodes;
        timed(c, st, PK_GRID_DENSE, [&] {
            launch_grid_tape(d, c->env_gofs, c->total_nodes, T.seg_dec + (size_t)slot * c->total_nodes,
                             T.seg_tools + (size_t)slot * slots, (int)slots, tape_list(c, slot), st);
        });
        const TiledArgs step = stamped(tiled_args(c, seg_view(c, slot), seg_view(c, slot + 1), 0), slot + 1);
        if (last) {
            timed(c, st, PK_G2P_TILED, [&] { launch_g2p_tiled(d, step, c->block, c->tiled_blocks, st); });
        } else {
            d.gP = next_P;
            timed(c, st, PK_FUSED_TILED, [&] { launch_fused_full_tiled(d, step, c->block, c->tiled_blocks, st); });
        }
    }
}

// A recording kept whole (held tape): the tiled recompute passes run as the
// forward, segment by segment, each into its own segment tape.  The last slot
// of a segment is the next segment's checkpoint (in original order) and, at
// the end, the live state (original order, identity particle index); tool
// table, step counters and status flags continue from the recompute's.
void record_held(mpm_ctx *c, int n, hipStream_t st)
{
    auto &T = c->tape;
    const int k = c->checkpoint_every;
    const size_t N = c->ntot, slots = c->tool_slots();
    const int nseg = (n + k - 1) / k;
    timed(c, st, PK_ADJ_MISC, [&] { launch_copy_bytes(T.work_status, c->status, sizeof(uint32_t) * c->n_envs, st); });
    for (int seg = 0; seg < nseg; ++seg) {
        const int sb = seg * k, se = std::min(sb + k, n);
        // the segment's sort reads particles already in cell order (the live state, then the
        // previous segment's last slot), not the checkpoint: its histogram atomics then
        // aggregate per wavefront
        Dev src = c->dev();
        if (seg > 0) {
            const auto &p = T.segs[seg - 1];
            src = state_view(c, p.state + (size_t)k * 24 * N);
            src.pid = p.perm;
        }
        select_seg(c, seg);
        recompute_segment_tiled(c, seg, sb, se, st, &src);
        const float *last = T.seg_state + (size_t)(se - sb) * 24 * N;
        timed(c, st, PK_ADJ_MISC, [&] {
            if (seg + 1 < nseg) {
                launch_unpermute(last, T.perm, c->ntot, 24, T.ckpt_state + (size_t)(seg + 1) * 24 * N, st);
                launch_copies({{T.ckpt_tools + (size_t)(seg + 1) * slots, T.work_tools, sizeof(ToolDev) * slots},
                               {T.ckpt_step + (size_t)(seg + 1) * c->n_envs, T.work_step,
                                sizeof(int32_t) * c->n_envs}},
                              st);
            } else {
                launch_unpermute(last, T.perm, c->ntot, 3, c->x, st);
                launch_unpermute(last + 3 * N, T.perm, c->ntot, 3, c->v, st);
                launch_unpermute(last + 6 * N, T.perm, c->ntot, 9, c->C, st);
                launch_unpermute(last + 15 * N, T.perm, c->ntot, 9, c->H, st);
                launch_copies({{c->pid, T.iota, sizeof(int32_t) * N},
                               {c->tools, T.work_tools, sizeof(ToolDev) * slots},
                               {c->step, T.work_step, sizeof(int32_t) * c->n_envs},
                               {c->status, T.work_status, sizeof(uint32_t) * c->n_envs}},
                              st);
            }
        });
    }
    select_live_items(c);
    c->items_valid = false;
    T.held = nseg;
}

// Reverse the recomputed segment's substeps [lo, s_end) in its sorted slot
// order; adjoints are gathered from / scattered back to original order.
void reverse_segment_tiled(mpm_ctx *c, int s_begin, int lo, int s_end, int s0, hipStream_t st)
{
    auto &T = c->tape;
    const size_t N = c->ntot;
    timed(c, st, PK_ADJ_MISC, [&] { launch_permute(T.adj_state, T.perm, c->ntot, 24, T.adj_slot, 0, st); });
    AdjBuf a = T.adj;
    a.xb = T.adj_slot;
    a.vb = T.adj_slot + 3 * N;
    a.Cb = T.adj_slot + 6 * N;
    a.Fb = T.adj_slot + 15 * N;
    const ActiveBuf ta = tape_act(c);
    // recorded state of tape slot `slot` (substep s_begin + slot)
    auto slot_dev = [&](int slot) {
        ParticleBuf sv = seg_view(c, slot);
        Dev d = c->dev();
        d.x = sv.x; d.v = sv.v; d.C = sv.C; d.H = sv.H; d.pid = nullptr;
        d.gP = T.seg_P + (size_t)slot * c->total_nodes;
        d.gV = T.seg_V + (size_t)slot * c->total_nodes;
        d.tools = T.seg_tools + (size_t)slot * c->tool_slots();
        return d;
    };
    // reverse G2P of the last substep; then per substep j the reverse grid
    // operation, and the reverse P2G of j fused with the reverse G2P of j - 1
    // (one pass over the particles), the last reverse P2G on its own
    timed(c, st, PK_ADJ_G2P, [&] {
        launch_adj_g2p_tiled(slot_dev(s_end - 1 - s_begin), a, c->sort.items, c->sort.totals, c->node_slots, ta,
                             c->block, c->tiled_blocks, st);
    });
    for (int j = s_end - 1; j >= lo; --j) {
        const int slot = j - s_begin;
        const Dev d = slot_dev(slot);
        a.j = j - s0;
        timed(c, st, PK_ADJ_GRID, [&] {
            launch_adj_grid(d, c->env_gofs, c->total_nodes, T.seg_dec + (size_t)slot * c->total_nodes, a,
                            tape_list(c, slot), st);
        });
        if (j > lo) {
            timed(c, st, PK_ADJ_P2G, [&] {
                launch_adj_pair_tiled(d, slot_dev(slot - 1), a, c->sort.items, c->sort.totals, c->node_slots, ta,
                                      c->block, c->tiled_blocks, st);
            });
        } else {
            timed(c, st, PK_ADJ_P2G, [&] {
                launch_adj_p2g_tiled(d, a, c->sort.items, c->sort.totals, ta, c->block, c->tiled_blocks, st);
            });
        }
    }
    timed(c, st, PK_ADJ_MISC, [&] { launch_permute(T.adj_slot, T.perm, c->ntot, 24, T.adj_state, 1, st); });
}

// Reverse substep j (tape slot `slot`); window index j - s0.
void reverse_substep(mpm_ctx *c, int slot, int jw, hipStream_t st)
{
    auto &T = c->tape;
    const size_t N = c->ntot;
    Dev d = state_view(c, T.seg_state + (size_t)slot * 24 * N);
    d.gP = T.seg_P + (size_t)slot * c->total_nodes;
    d.gV = T.seg_V + (size_t)slot * c->total_nodes;
    d.tools = T.seg_tools + (size_t)slot * c->tool_slots();
    AdjBuf a = T.adj;
    a.j = jw;
    timed(c, st, PK_ADJ_G2P, [&] { launch_adj_g2p(d, a, st); });
    timed(c, st, PK_ADJ_GRID, [&] {
        launch_adj_grid(d, c->env_gofs, c->total_nodes, T.seg_dec + (size_t)slot * c->total_nodes, a, dense_list(c),
                        st);
    });
    timed(c, st, PK_ADJ_P2G, [&] { launch_adj_p2g(d, a, st); });
}

// Checks shared by the surface entry points; device addresses of the outputs.
mpm_status surface_args(mpm_ctx *c, int32_t env, float iso, float *tris, int64_t max_tris, int64_t *n_tris,
                               void **tris_d, void **count_d)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    if (env < 0 || env >= c->n_envs) return fail(c, MPM_E_ARG, "env out of range");
    if (!(iso > 0.f) || !std::isfinite(iso)) return fail(c, MPM_E_ARG, "iso must be finite and > 0");
    if (max_tris < 0 || (max_tris > 0 && !tris)) return fail(c, MPM_E_ARG, "tris must hold max_tris >= 0 triangles");
    if (!n_tris) return fail(c, MPM_E_ARG, "n_tris is NULL");
    if (c->tstage) return fail(c, MPM_E_STATE, "a tiled stage sequence is open: end it with MPM_STAGE_TILED_G2P");
    // device memory, or pinned host memory written through its device alias;
    // anything else (pageable host memory) is refused rather than faulted on
    auto device_alias = [&](void *p, void **out) -> bool {
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, p) != hipSuccess) { (void)hipGetLastError(); return false; }
        if (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged) { *out = p; return true; }
        unsigned int hflags = 0;
        if (at.type == hipMemoryTypeHost && at.devicePointer && hipHostGetFlags(&hflags, p) == hipSuccess) {
            *out = static_cast<char *>(at.devicePointer) +
                   (static_cast<char *>(p) - static_cast<char *>(at.hostPointer ? at.hostPointer : p));
            return true;
        }
        return false;
    };
    *tris_d = nullptr;
    *count_d = nullptr;
    if (max_tris > 0 && !device_alias(tris, tris_d))
        return fail(c, MPM_E_ARG, "tris must be device memory or pinned (hipHostMalloc) host memory");
    if (!device_alias(n_tris, count_d))
        return fail(c, MPM_E_ARG, "n_tris must be device memory or pinned (hipHostMalloc) host memory");
    return MPM_OK;
}

// The sorted work items are usable while the live state sits in their slots.
SurfItems surface_items(const mpm_ctx *c)
{
    if (c->scheme == MPM_SCHEME_TILED && c->items_valid) return SurfItems{c->sort.items, c->sort.totals, c->max_items};
    return SurfItems{nullptr, nullptr, 0};
}

}  // namespace

extern "C" {

size_t mpm_workspace_size(const mpm_desc *desc)
{
    try {
        Shape s;
        std::string why;
        if (!validate(desc, why, s)) { g_last_error = why; return 0; }
        mpm_ctx tmp;
        Carver cv(nullptr);
        carve(tmp, s, cv);
        return (cv.off + 255) & ~size_t(255);
    } catch (...) {
        g_last_error = "internal error in mpm_workspace_size";
        return 0;
    }
}

}  // extern "C"

namespace {

mpm_status create_in(const mpm_desc *desc, void *workspace, size_t workspace_bytes, void *stream, mpm_ctx **out)
{
    try {
        if (!out) return fail(nullptr, MPM_E_ARG, "out is NULL");
        *out = nullptr;
        Shape s;
        std::string why;
        if (!validate(desc, why, s)) return fail(nullptr, MPM_E_ARG, why);
        size_t need = mpm_workspace_size(desc);
        if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
            return fail(nullptr, MPM_E_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
        if (workspace_bytes < need)
            return fail(nullptr, MPM_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
        hipStream_t st = as_stream(stream);

        // material sanity (read once here; kernels read it every substep)
        std::vector<float> mat((size_t)4 * desc->n_envs);
        hipError_t he = hipMemcpyAsync(mat.data(), desc->material, mat.size() * sizeof(float), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return fail(nullptr, MPM_E_HIP, std::string("reading material: ") + hipGetErrorString(he));
        for (int e = 0; e < desc->n_envs; ++e) {
            float E = mat[4 * e], nu = mat[4 * e + 1], rho = mat[4 * e + 2], V0 = mat[4 * e + 3];
            if (!(E > 0.f) || !(nu > -1.f && nu < 0.5f) || !(rho > 0.f) || !(V0 > 0.f) || !std::isfinite(E) ||
                !std::isfinite(rho) || !std::isfinite(V0))
                return fail(nullptr, MPM_E_ARG, "material of env " + std::to_string(e) +
                                                    " must have E > 0, -1 < nu < 0.5, rho > 0, V0 > 0");
        }

        mpm_ctx *c = new (std::nothrow) mpm_ctx();
        if (!c) return fail(nullptr, MPM_E_ARG, "out of host memory");
        c->n_envs = s.n_envs;
        c->max_tools = s.max_tools;
        c->ntot = s.ntot;
        c->bound = desc->bound;
        c->dt = desc->dt;
        for (int a = 0; a < 3; ++a) c->g[a] = desc->gravity[a];
        c->max_tape = desc->max_tape_substeps;
        c->checkpoint_every = s.ck;
        c->material = desc->material;
        c->stream0 = st;
        c->total_nodes = s.total_nodes;
        c->total_bricks = s.total_bricks;
        Carver cv(workspace);
        carve(*c, s, cv);
        if (!all_carved(*c) || cv.off > workspace_bytes) {
            delete c;
            return fail(nullptr, MPM_E_WORKSPACE, "internal: workspace layout incomplete");
        }

        std::vector<EnvDev> envh(s.n_envs);
        c->np.resize(s.n_envs);
        c->gn.resize(s.n_envs);
        c->pofs.assign(s.n_envs + 1, 0);
        c->gofs.assign(s.n_envs + 1, 0);
        c->bofs.assign(s.n_envs + 1, 0);
        for (int e = 0; e < s.n_envs; ++e) {
            int n = desc->grid_n[e];
            c->np[e] = desc->n_particles[e];
            c->gn[e] = n;
            c->pofs[e + 1] = c->pofs[e] + c->np[e];
            c->gofs[e + 1] = c->gofs[e] + (int64_t)n * n * n;
            c->bofs[e + 1] = c->bofs[e] + (n / 4) * (n / 4) * (n / 4);
            // n = 4 nb, so gofs = 64 bofs for every environment (the grid kernel relies on it)
            EnvDev &E = envh[e];
            memset(&E, 0, sizeof E);
            E.n = n;
            E.nb = n / 4;
            E.pofs = c->pofs[e];
            E.np = c->np[e];
            E.gofs = c->gofs[e];
            E.bofs = c->bofs[e];
            E.bound = desc->bound;
            E.dx = 1.0f / n;
            E.inv_dx = (float)n;
        }
        c->tools_h.assign((size_t)s.n_envs * std::max(1, s.max_tools), ToolDev{});
        auto cleanup_fail = [&](hipError_t e2, const char *what) {
            std::string m = std::string(what) + ": " + hipGetErrorString(e2);
            delete c;
            return fail(nullptr, MPM_E_HIP, m);
        };
        hipError_t e2;
        if ((e2 = hipMemcpyAsync(c->env, envh.data(), sizeof(EnvDev) * s.n_envs, hipMemcpyHostToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy env table");
        if ((e2 = hipMemcpyAsync(c->env_pofs, c->pofs.data(), sizeof(int32_t) * (s.n_envs + 1), hipMemcpyHostToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy particle offsets");
        if ((e2 = hipMemcpyAsync(c->env_gofs, c->gofs.data(), sizeof(int64_t) * (s.n_envs + 1), hipMemcpyHostToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy grid offsets");
        if ((e2 = hipMemcpyAsync(c->env_bofs, c->bofs.data(), sizeof(int32_t) * (s.n_envs + 1), hipMemcpyHostToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy brick offsets");
        if ((e2 = hipMemcpyAsync(c->tools, c->tools_h.data(), sizeof(ToolDev) * c->tools_h.size(), hipMemcpyHostToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy tools");
        static McTable mc_table;
        static const bool mc_ok = build_mc_table(mc_table);
        if (!mc_ok) return cleanup_fail(hipErrorInvalidValue, "marching-cubes case table does not close");
        if ((e2 = hipMemcpyAsync(const_cast<McTable *>(c->surf.table), &mc_table, sizeof(McTable), hipMemcpyHostToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy case table");
        size_t N = s.ntot;
        if ((e2 = hipMemcpyAsync(c->x, desc->x0, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e2 = hipMemcpyAsync(c->v, desc->v0, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e2 = hipMemcpyAsync(c->C, desc->C0, 9 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e2 = hipMemcpyAsync(c->H, desc->F0, 9 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy initial state");
        launch_add_identity(c->H, s.ntot, s.ntot, -1.0f, st);    // stored as H = F - I
        launch_iota(c->pid, s.ntot, st);
        if (c->max_tape > 0) {
            launch_iota(c->tape.iota, s.ntot, st);
            // tape grids start zero and are left zero by every reverse pass
            for (const auto &g : c->tape.segs) {
                launch_fill_f4(g.P, (int64_t)s.total_nodes * s.ck, st);
                launch_fill_u32(reinterpret_cast<uint32_t *>(g.tflag), s.total_bricks, 0u, st);
                launch_fill_u32(reinterpret_cast<uint32_t *>(g.tscount), 1, 0u, st);
                launch_fill_u32(reinterpret_cast<uint32_t *>(g.tfar), s.ck + 1, 0xffffffffu, st);
            }
        }
        launch_fill_u32(c->status, s.n_envs, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->step), s.n_envs, 0u, st);
        launch_fill_f4(c->gP, s.total_nodes, st);
        launch_fill_f4(c->gV, s.total_nodes, st);
        launch_fill_f4(c->gP1, s.total_nodes, st);
        launch_fill_f4(c->gP2, s.total_nodes, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->far_stamp), 4, 0xffffffffu, st);
        launch_fill_u32(c->run_bar, RUN_BARRIER_WORDS, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->act.flag), s.total_bricks, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->sort.count), (int64_t)s.total_bricks * 64, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->sort.brick_count), s.total_bricks, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->act.scount), 1, 0u, st);
        launch_brick_env(c->env_bofs, s.n_envs, s.total_bricks, c->brick_env, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->act.dcount), 2, 0u, st);
        launch_fill_u32(c->arrive, 2 * s.n_envs, 0u, st);
        if ((e2 = hipGetLastError()) != hipSuccess) return cleanup_fail(e2, "init kernels");
        if ((e2 = hipStreamSynchronize(st)) != hipSuccess) return cleanup_fail(e2, "create sync");
        *out = c;
        return MPM_OK;
    } catch (...) {
        return fail(nullptr, MPM_E_ARG, "internal error in mpm_create");
    }
}

constexpr int MAX_STATIC_DEVICES = 64;
struct StaticWorkspace {
    void *ptr = nullptr;   // device address of this device's `scratch`
    bool in_use = false;   // a live context was created in it
};
std::mutex g_static_mu;
StaticWorkspace g_static[MAX_STATIC_DEVICES];

}  // namespace

extern "C" {

mpm_status mpm_create(const mpm_desc *desc, void *workspace, size_t workspace_bytes, void *stream, mpm_ctx **out)
{
    return create_in(desc, workspace, workspace_bytes, stream, out);
}

mpm_status mpm_create_static(const mpm_desc *desc, void *stream, mpm_ctx **out)
{
    try {
        if (!out) return fail(nullptr, MPM_E_ARG, "out is NULL");
        *out = nullptr;
        const size_t need = mpm_workspace_size(desc);
        if (need == 0) return fail(nullptr, MPM_E_ARG, g_last_error);
        if (need > MPM_STATIC_WORKSPACE_BYTES)
            return fail(nullptr, MPM_E_WORKSPACE,
                        "this description needs " + std::to_string(need) + " bytes of workspace; the static "
                        "workspace holds " + std::to_string((size_t)MPM_STATIC_WORKSPACE_BYTES) +
                        " (use mpm_create with a caller-allocated workspace)");
        int dev = 0;
        HIP_TRY(nullptr, hipGetDevice(&dev));
        if (dev < 0 || dev >= MAX_STATIC_DEVICES)
            return fail(nullptr, MPM_E_UNSUPPORTED, "static workspace: device index beyond " +
                                                        std::to_string(MAX_STATIC_DEVICES - 1));
        std::lock_guard<std::mutex> lock(g_static_mu);
        StaticWorkspace &w = g_static[dev];
        if (!w.ptr) {
            void *p = nullptr;
            HIP_TRY(nullptr, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p || (reinterpret_cast<uintptr_t>(p) & 255))
                return fail(nullptr, MPM_E_HIP, "static workspace: no 256-byte aligned device address");
            w.ptr = p;
        }
        if (w.in_use)
            return fail(nullptr, MPM_E_STATE, "the static workspace of device " + std::to_string(dev) +
                                                  " is held by a live context; destroy it first");
        mpm_status r = create_in(desc, w.ptr, MPM_STATIC_WORKSPACE_BYTES, stream, out);
        if (r != MPM_OK) return r;
        w.in_use = true;
        (*out)->static_dev = dev;
        return MPM_OK;
    } catch (...) {
        return fail(nullptr, MPM_E_ARG, "internal error in mpm_create_static");
    }
}

void mpm_destroy(mpm_ctx *ctx)
{
    if (ctx && ctx->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static[ctx->static_dev].in_use = false;
    }
    delete ctx;
}

mpm_status mpm_set_tool(mpm_ctx *c, int32_t env, int32_t tool, const mpm_tool *t, const float *u, int32_t n_traj)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    try {
        if (env < 0 || env >= c->n_envs) return fail(c, MPM_E_ARG, "env out of range");
        if (tool < 0 || tool >= c->max_tools) return fail(c, MPM_E_ARG, "tool slot out of range");
        ToolDev td{};
        if (t) {
            if (t->contact != MPM_CONTACT_SLIP && t->contact != MPM_CONTACT_STICKY) return fail(c, MPM_E_ARG, "bad contact mode");
            if (!(t->friction >= 0.f) || !std::isfinite(t->friction) || !std::isfinite(t->theta))
                return fail(c, MPM_E_ARG, "tool needs friction >= 0 and a finite theta");
            if (t->shape == MPM_TOOL_CAPSULE) {
                if (!(t->radius > 0.f) || !(t->half_len >= 0.f) || !std::isfinite(t->radius) || !std::isfinite(t->half_len))
                    return fail(c, MPM_E_ARG, "capsule needs radius > 0 and half_len >= 0");
            } else if (t->shape == MPM_TOOL_BOX) {
                if (!(t->radius >= 0.f) || !std::isfinite(t->radius)) return fail(c, MPM_E_ARG, "box needs radius >= 0");
                for (int i = 0; i < 3; ++i)
                    if (!(t->half[i] >= 0.f) || !std::isfinite(t->half[i])) return fail(c, MPM_E_ARG, "box needs half extents >= 0");
            } else if (t->shape == MPM_TOOL_SDF) {
                if (!t->sdf) return fail(c, MPM_E_ARG, "sampled SDF tool needs a device sample array");
                if (t->sdf_res < 4 || t->sdf_res > 2048) return fail(c, MPM_E_ARG, "sdf_res must be in [4, 2048]");
                if (t->sdf_interp != MPM_SDF_NEAREST && t->sdf_interp != MPM_SDF_TRILINEAR)
                    return fail(c, MPM_E_ARG, "sdf_interp must be MPM_SDF_NEAREST or MPM_SDF_TRILINEAR");
                if (!(t->sdf_h > 0.f) || !std::isfinite(t->sdf_h)) return fail(c, MPM_E_ARG, "sdf_h must be > 0");
                for (int i = 0; i < 3; ++i)
                    if (!std::isfinite(t->sdf_lo[i])) return fail(c, MPM_E_ARG, "sdf_lo must be finite");
            } else {
                return fail(c, MPM_E_ARG, "unknown tool shape");
            }
            for (int i = 0; i < 9; ++i) if (!std::isfinite(t->R[i])) return fail(c, MPM_E_ARG, "R must be finite");
            for (int i = 0; i < 3; ++i) if (!std::isfinite(t->T0[i])) return fail(c, MPM_E_ARG, "T0 must be finite");
            if (!u || n_traj < 1) return fail(c, MPM_E_ARG, "u must be a device array with n_traj >= 1");
            td.active = 1;
            td.shape = t->shape;
            td.contact = t->contact;
            td.n_traj = n_traj;
            td.radius = t->radius;
            td.half_len = t->half_len;
            td.friction = t->friction;
            td.theta = t->theta;
            memcpy(td.R, t->R, sizeof td.R);
            for (int i = 0; i < 3; ++i) td.half[i] = t->half[i];
            td.sdf_res = t->sdf_res;
            td.sdf_interp = t->sdf_interp;
            td.sdf_h = t->sdf_h;
            for (int i = 0; i < 3; ++i) td.sdf_lo[i] = t->sdf_lo[i];
            td.sdf = t->shape == MPM_TOOL_SDF ? t->sdf : nullptr;
            td.k = 0;
            td.u = u;
            for (int i = 0; i < 3; ++i) td.T[i] = (double)t->T0[i];
        }
        size_t slot = (size_t)env * c->max_tools + tool;
        c->tools_h[slot] = td;
        c->has_sdf = false;
        for (const ToolDev &h : c->tools_h) c->has_sdf |= h.active && h.shape == MPM_TOOL_SDF;
        HIP_TRY(c, hipMemcpyAsync(c->tools + slot, &c->tools_h[slot], sizeof(ToolDev), hipMemcpyHostToDevice, c->stream0));
        HIP_TRY(c, hipStreamSynchronize(c->stream0));
        return MPM_OK;
    } catch (...) {
        return fail(c, MPM_E_ARG, "internal error in mpm_set_tool");
    }
}

mpm_status mpm_set_option(mpm_ctx *c, int32_t option, int32_t value)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    switch (option) {
    case MPM_OPT_SCHEME:
        if (value != MPM_SCHEME_DIRECT && value != MPM_SCHEME_TILED) return fail(c, MPM_E_ARG, "unknown scheme");
        c->scheme = value;
        return MPM_OK;
    case MPM_OPT_SORT_EVERY:
        if (value < 1) return fail(c, MPM_E_ARG, "sort_every must be >= 1");
        c->sort_every = value;
        c->since_sort = value;   // the schedule restarts: the next substep call opens with a sort
        return MPM_OK;
    case MPM_OPT_BLOCK:
        if (value != 64 && value != 128 && value != 256) return fail(c, MPM_E_ARG, "block must be 64, 128 or 256");
        c->block = value;
        c->tiled_blocks = 0;
        c->gas_blocks = 0;
        c->run_blocks = 0;
        return c->persistent ? build_groups(c) : MPM_OK;
    case MPM_OPT_ITEM:
        if (value < 16 || value > 4096 || value % 16) return fail(c, MPM_E_ARG, "item size must be a multiple of 16 in [16, 4096]");
        c->item = value;
        return c->persistent ? build_groups(c) : MPM_OK;
    case MPM_OPT_NODE_SLOTS:
        if (value != 1 && value != 3) return fail(c, MPM_E_ARG, "node slots must be 1 or 3");
        c->node_slots = value;
        return MPM_OK;
    case MPM_OPT_GRAPH:
        c->use_graph = value != 0;
        return MPM_OK;
    case MPM_OPT_PERSISTENT:
        c->persistent = value != 0;
        return c->persistent ? build_groups(c) : MPM_OK;
    case MPM_OPT_GRID_AT_STAGING:
        c->grid_at_staging = value != 0;
        return MPM_OK;
    case MPM_OPT_SPIN_LIMIT:
        if (value < 1) return fail(c, MPM_E_ARG, "spin limit must be > 0");
        c->spin_limit = value;
        return MPM_OK;
    default:
        return fail(c, MPM_E_ARG, "unknown option");
    }
}

mpm_status mpm_substep(mpm_ctx *c, int32_t n_substeps, int32_t record_tape, void *stream)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    if (n_substeps < 1) return fail(c, MPM_E_ARG, "n_substeps must be >= 1");
    if (c->tstage) return fail(c, MPM_E_STATE, "a tiled stage sequence is open: end it with MPM_STAGE_TILED_G2P");
    hipStream_t st = as_stream(stream);
    if (!record_tape) {
        c->tape.len = 0;   // the tape no longer ends at the current state
        if (c->use_graph && !c->prof.on) {
            mpm_status r = run_substeps_graph(c, n_substeps, st);
            if (r != MPM_OK) return r;
        } else {
            run_substeps(c, n_substeps, st);
        }
        return check_launch(c, "mpm_substep");
    }
    if (c->max_tape == 0) return fail(c, MPM_E_STATE, "context was created without a tape (max_tape_substeps = 0)");
    if (n_substeps > c->max_tape) return fail(c, MPM_E_ARG, "n_substeps exceeds max_tape_substeps");
    const int k = c->checkpoint_every;
    c->tape.len = 0;
    c->tape.held = 0;
    save_checkpoint(c, 0, st);
    if (c->tape.segs.size() > 1 && c->scheme == MPM_SCHEME_TILED) {
        record_held(c, n_substeps, st);
    } else {
        for (int done = 0; done < n_substeps;) {
            int m = std::min(k, n_substeps - done);
            run_substeps(c, m, st);
            done += m;
            if (done < n_substeps) save_checkpoint(c, done / k, st);
        }
    }
    c->tape.len = n_substeps;
    return check_launch(c, "mpm_substep");
}

mpm_status mpm_run_stage(mpm_ctx *c, int32_t stage, void *stream)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    hipStream_t st = as_stream(stream);
    Dev d = c->dev();
    const bool tiled_stage = stage >= MPM_STAGE_TILED_P2G && stage <= MPM_STAGE_TILED_G2P;
    if (c->tstage && !tiled_stage)
        return fail(c, MPM_E_STATE, "a tiled stage sequence is open: end it with MPM_STAGE_TILED_G2P");
    if (tiled_stage && c->tiled_blocks == 0) c->tiled_blocks = tiled_workgroups(c->block);
    switch (stage) {
    case MPM_STAGE_P2G:
        launch_fill_f4(c->gP, c->total_nodes, st);
        launch_p2g_direct(d, st);
        c->grid_clean = false;
        break;
    case MPM_STAGE_GRID:
        launch_grid_dense(d, c->env_gofs, c->total_nodes, 0, st);
        break;
    case MPM_STAGE_G2P:
        launch_g2p_direct(d, st);
        break;
    case MPM_STAGE_TILED_P2G: {
        // the head of mpm_substep's tiled scheme: sort when due, then P2G of the current state
        if (c->tstage) return fail(c, MPM_E_STATE, "a tiled stage sequence is open: end it with MPM_STAGE_TILED_G2P");
        if (!c->grid_clean) {
            launch_fill_f4(c->gP, c->total_nodes, st);
            c->grid_clean = true;
        }
        ParticleBuf in = live(c);
        if (!c->items_valid || c->items_P != c->item || c->since_sort >= c->sort_every) {
            sort_into_alt(c, st);
            in = c->alt;
        }
        launch_p2g_tiled(d, tiled_args(c, in, in, 0), c->block, c->tiled_blocks, st);
        c->tstage = 1;
        c->tstage_i = 0;
        c->tstage_in = in;
        break;
    }
    case MPM_STAGE_TILED_GRID:
        if (c->tstage != 1) return fail(c, MPM_E_STATE, "MPM_STAGE_TILED_GRID needs a tiled P2G before it");
        launch_grid_active(d, c->act, c->tstage_i & 1, grid_blocks(c), c->has_sdf, st);
        c->tstage = 2;
        c->since_sort += 1;
        break;
    case MPM_STAGE_TILED_FUSED:
    case MPM_STAGE_TILED_FUSED_FULL: {
        if (c->tstage != 2) return fail(c, MPM_E_STATE, "a fused tiled stage needs MPM_STAGE_TILED_GRID before it");
        const TiledArgs a = tiled_args(c, c->tstage_in, live(c), (c->tstage_i + 1) & 1);
        if (stage == MPM_STAGE_TILED_FUSED) launch_fused_tiled(d, a, c->block, c->tiled_blocks, st);
        else launch_fused_full_tiled(d, a, c->block, c->tiled_blocks, st);
        c->tstage = 1;
        c->tstage_i += 1;
        c->tstage_in = live(c);
        break;
    }
    case MPM_STAGE_TILED_G2P:
        if (c->tstage != 2) return fail(c, MPM_E_STATE, "MPM_STAGE_TILED_G2P needs MPM_STAGE_TILED_GRID before it");
        launch_g2p_tiled(d, tiled_args(c, c->tstage_in, live(c), 0), c->block, c->tiled_blocks, st);
        c->tstage = 0;
        break;
    default:
        return fail(c, MPM_E_ARG, "unknown stage");
    }
    return check_launch(c, "mpm_run_stage");
}

mpm_status mpm_substep_adjoint(mpm_ctx *c, int32_t n_substeps, const mpm_adjoint_io *io, void *stream)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    if (!io) return fail(c, MPM_E_ARG, "io is NULL");
    if (n_substeps < 1) return fail(c, MPM_E_ARG, "n_substeps must be >= 1");
    if (c->tstage) return fail(c, MPM_E_STATE, "a tiled stage sequence is open: end it with MPM_STAGE_TILED_G2P");
    if (c->max_tape == 0 || c->tape.len < n_substeps)
        return fail(c, MPM_E_STATE, "no recorded tape of at least n_substeps substeps ending at the current state");
    hipStream_t st = as_stream(stream);
    auto &T = c->tape;
    const size_t N = c->ntot;
    const int k = c->checkpoint_every, len = T.len, s0 = len - n_substeps;
    // seeds (original order) or zero
    const float *seeds[4] = {io->xbar, io->vbar, io->Cbar, io->Fbar};
    float *adj[4] = {T.adj.xb, T.adj.vb, T.adj.Cb, T.adj.Fb};
    const int comps[4] = {3, 3, 9, 9};
    timed(c, st, PK_ADJ_MISC, [&] {
        for (int f = 0; f < 4; ++f) {
            if (seeds[f]) launch_copy_bytes(adj[f], seeds[f], sizeof(float) * comps[f] * N, st);
            else launch_fill_u32(reinterpret_cast<uint32_t *>(adj[f]), (int64_t)comps[f] * N, 0u, st);
        }
        launch_fill_f4(T.adj.gVb, c->total_nodes, st);
        launch_fill_f4(T.adj.gPb, c->total_nodes, st);   // bricks without mass are never written
        const int64_t ng = (int64_t)c->tool_slots() * c->max_tape * 3;
        launch_fill_f64(T.adj.ubar, ng, st);
        launch_fill_f64(T.adj.Tbar, ng, st);
        launch_fill_f64(T.adj.mubar, c->n_envs, st);
        launch_fill_f64(T.adj.lambar, c->n_envs, st);
    });
    // held segment tapes (a recording kept whole) are reversed as they are, once
    const bool held = T.held > 0 && c->scheme == MPM_SCHEME_TILED;
    const bool multi = T.segs.size() > 1;
    for (int seg = (len - 1) / k; seg >= s0 / k; --seg) {
        const int sb = seg * k, se = std::min(sb + k, len), lo = std::max(sb, s0);
        const bool tiled = c->scheme == MPM_SCHEME_TILED;
        select_seg(c, multi ? seg : 0);
        if (tiled) {
            if (!held) recompute_segment_tiled(c, seg, sb, se, st);
            reverse_segment_tiled(c, sb, lo, se, s0, st);
        } else {
            recompute_segment(c, seg, sb, se, st);
            for (int j = se - 1; j >= lo; --j) reverse_substep(c, j - sb, j - s0, st);
        }
        // the reverse grid pass leaves each tape grid it visits zero; those of recomputed
        // substeps before the window are cleared here
        for (int j = sb; j < lo; ++j) {
            Dev d = c->dev();
            d.gP = T.seg_P + (size_t)(j - sb) * c->total_nodes;
            timed(c, st, PK_ADJ_MISC, [&] {
                launch_tape_clear(d, c->env_gofs, c->total_nodes, tiled ? tape_list(c, j - sb) : dense_list(c), st);
            });
        }
        T.segs[T.sel].dirty = 0;
    }
    T.held = 0;
    if (multi) {
        select_seg(c, 0);
        select_live_items(c);
    }
    timed(c, st, PK_ADJ_MISC, [&] {
        launch_adj_finish(c->dev(), T.adj, n_substeps, io->gE, io->gnu, io->gu, io->gT, st);
        float *outs[4] = {io->xbar0, io->vbar0, io->Cbar0, io->Fbar0};
        for (int f = 0; f < 4; ++f)
            if (outs[f]) launch_copy_bytes(outs[f], adj[f], sizeof(float) * comps[f] * N, st);
    });
    return check_launch(c, "mpm_substep_adjoint");
}

mpm_status mpm_read_state(mpm_ctx *c, int32_t env, int32_t field, void *dst, size_t dst_bytes, int32_t dst_on_device,
                          void *stream)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    if (env < 0 || env >= c->n_envs) return fail(c, MPM_E_ARG, "env out of range");
    if (!dst) return fail(c, MPM_E_ARG, "dst is NULL");
    hipStream_t st = as_stream(stream);
    int np = c->np[env], n = c->gn[env];
    int64_t nn = (int64_t)n * n * n;
    size_t need = 0;
    int comps = 0;
    const float *src = nullptr;
    switch (field) {
    case MPM_F_X: comps = 3; src = c->x; break;
    case MPM_F_V: comps = 3; src = c->v; break;
    case MPM_F_C: comps = 9; src = c->C; break;
    case MPM_F_F: comps = 9; src = c->H; break;   // returned as F = I + H
    case MPM_F_GRID_M: comps = 1; break;
    case MPM_F_GRID_MV: comps = 3; break;
    case MPM_F_GRID_V: comps = 3; break;
    case MPM_F_STATUS: need = sizeof(uint32_t); break;
    case MPM_F_TOOL_T: need = sizeof(double) * 3 * std::max(1, c->max_tools); break;
    case MPM_F_STEP: need = sizeof(int32_t); break;
    case MPM_F_DENSITY:
        if (c->surf_env != env) return fail(c, MPM_E_STATE, "no surface extracted for this environment since the last one");
        need = sizeof(float) * (size_t)nn;
        break;
    default: return fail(c, MPM_E_ARG, "unknown field");
    }
    if (field <= MPM_F_F) need = sizeof(float) * comps * (size_t)np;
    else if (field <= MPM_F_GRID_V) need = sizeof(float) * comps * (size_t)nn;
    if (dst_bytes != need) return fail(c, MPM_E_ARG, "dst_bytes must be " + std::to_string(need));

    // Device destinations are filled by a conversion kernel; host destinations
    // get a raw copy that is reordered on the host.
    if (field <= MPM_F_F) {
        if (dst_on_device) {
            launch_read_particles(src, c->pid, c->ntot, c->pofs[env], np, comps, static_cast<float *>(dst), st);
            if (field == MPM_F_F) launch_add_identity(static_cast<float *>(dst), np, np, 1.0f, st);
            return check_launch(c, "read particles");
        }
        std::vector<float> raw((size_t)comps * np);
        std::vector<int32_t> pid(np);
        for (int k = 0; k < comps; ++k)
            HIP_TRY(c, hipMemcpyAsync(raw.data() + (size_t)k * np, src + (size_t)k * c->ntot + c->pofs[env],
                                      sizeof(float) * np, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipMemcpyAsync(pid.data(), c->pid + c->pofs[env], sizeof(int32_t) * np, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        float *out = static_cast<float *>(dst);
        for (int i = 0; i < np; ++i) {
            int o = pid[i] - c->pofs[env];
            for (int k = 0; k < comps; ++k) out[(size_t)k * np + o] = raw[(size_t)k * np + i];
        }
        if (field == MPM_F_F)
            for (int i = 0; i < np; ++i) {
                out[i] += 1.0f;
                out[(size_t)4 * np + i] += 1.0f;
                out[(size_t)8 * np + i] += 1.0f;
            }
        return MPM_OK;
    }
    if (field <= MPM_F_GRID_V) {
        const float4 *g = field == MPM_F_GRID_V ? c->gV : c->gP;
        int comp0 = field == MPM_F_GRID_MV ? 1 : 0;
        if (dst_on_device) {
            launch_read_grid(g, c->gofs[env], n, comp0, comps, static_cast<float *>(dst), st);
            return check_launch(c, "read grid");
        }
        std::vector<float4> raw(nn);
        HIP_TRY(c, hipMemcpyAsync(raw.data(), g + c->gofs[env], sizeof(float4) * nn, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        float *out = static_cast<float *>(dst);
        int nb = n / 4;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    int b = ((i >> 2) * nb + (j >> 2)) * nb + (k >> 2);
                    const float *s = reinterpret_cast<const float *>(&raw[(size_t)b * 64 + ((i & 3) << 4) + ((j & 3) << 2) + (k & 3)]);
                    size_t id = ((size_t)i * n + j) * n + k;
                    for (int q = 0; q < comps; ++q) out[(size_t)q * nn + id] = s[comp0 + q];
                }
        return MPM_OK;
    }
    if (field == MPM_F_DENSITY) {
        HIP_TRY(c, hipMemcpyAsync(dst, c->surf.rho, need, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        if (!dst_on_device) HIP_TRY(c, hipStreamSynchronize(st));
        return MPM_OK;
    }
    if (field == MPM_F_STATUS) {
        HIP_TRY(c, hipMemcpyAsync(dst, c->status + env, sizeof(uint32_t),
                                  dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        if (!dst_on_device) HIP_TRY(c, hipStreamSynchronize(st));
        return MPM_OK;
    }
    if (field == MPM_F_STEP) {
        HIP_TRY(c, hipMemcpyAsync(dst, c->step + env, sizeof(int32_t),
                                  dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        if (!dst_on_device) HIP_TRY(c, hipStreamSynchronize(st));
        return MPM_OK;
    }
    // tool positions come from the device tool table
    int nt = std::max(1, c->max_tools);
    std::vector<ToolDev> tl(nt);
    HIP_TRY(c, hipMemcpyAsync(tl.data(), c->tools + (size_t)env * c->max_tools, sizeof(ToolDev) * (c->max_tools ? nt : 0),
                              hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (field == MPM_F_TOOL_T) {
        std::vector<double> T(3 * nt, 0.0);
        for (int t = 0; t < c->max_tools; ++t)
            for (int a = 0; a < 3; ++a) T[3 * t + a] = tl[t].T[a];
        if (dst_on_device) HIP_TRY(c, hipMemcpyAsync(dst, T.data(), need, hipMemcpyHostToDevice, st));
        else memcpy(dst, T.data(), need);
        if (dst_on_device) HIP_TRY(c, hipStreamSynchronize(st));
        return MPM_OK;
    }
    return fail(c, MPM_E_ARG, "unknown field");
}

mpm_status mpm_extract_surface(mpm_ctx *c, int32_t env, float iso, float *tris, int64_t max_tris, int64_t *n_tris,
                               void *stream)
{
    void *tris_d = nullptr, *count_d = nullptr;
    mpm_status r = surface_args(c, env, iso, tris, max_tris, n_tris, &tris_d, &count_d);
    if (r != MPM_OK) return r;
    const int n = c->gn[env];
    launch_surface(c->dev(), env, c->np[env], n, 1.0f / (float)n, iso, c->surf, surface_items(c),
                   static_cast<float *>(tris_d), max_tris, static_cast<int64_t *>(count_d), as_stream(stream));
    c->surf_env = env;
    return check_launch(c, "mpm_extract_surface");
}

mpm_status mpm_profile(mpm_ctx *c, int32_t enable)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    if (enable && c->use_graph) return fail(c, MPM_E_STATE, "profiling is not available with the graph option");
    if (!enable && c->prof.on) prof_resolve(c);
    if (enable && !c->prof.on) {
        for (int k = 0; k < PK_COUNT; ++k) { c->prof.total_ms[k] = 0.0; c->prof.launches[k] = 0; }
        c->prof.marks.clear();
        c->prof.used = 0;
    }
    c->prof.on = enable != 0;
    return MPM_OK;
}

mpm_status mpm_profile_read(mpm_ctx *c, int32_t kind, const char **name, double *total_ms, int64_t *launches)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    if (kind < 0 || kind >= PK_COUNT) return fail(c, MPM_E_ARG, "kind out of range");
    if (c->prof.on) prof_resolve(c);
    if (name) *name = PROF_NAMES[kind];
    if (total_ms) *total_ms = c->prof.total_ms[kind];
    if (launches) *launches = c->prof.launches[kind];
    return MPM_OK;
}

const char *mpm_last_error(const mpm_ctx *c)
{
    if (c) return c->err.empty() ? "no error" : c->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"
