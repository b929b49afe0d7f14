// C ABI of the MLS-MPM library: validation, workspace carving, sequencing of
// the kernels.  Every entry point catches everything and returns a status.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "mpm_ctx.h"

using namespace mpm;

static thread_local std::string g_last_error = "no error";

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
    int64_t total_nodes;
    int32_t total_bricks;
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
    c.F = cv.take<float>((size_t)9 * s.ntot);
    c.pid = cv.take<int32_t>(s.ntot);
    c.gP = cv.take<float4>(s.total_nodes);
    c.gV = cv.take<float4>(s.total_nodes);
    // tiled scheme
    c.alt.x = cv.take<float>((size_t)3 * s.ntot);
    c.alt.v = cv.take<float>((size_t)3 * s.ntot);
    c.alt.C = cv.take<float>((size_t)9 * s.ntot);
    c.alt.F = cv.take<float>((size_t)9 * s.ntot);
    c.alt.pid = cv.take<int32_t>(s.ntot);
    c.sort.count = cv.take<int2>(s.total_bricks);
    c.sort.offset = cv.take<int2>(s.total_bricks);
    c.sort.chunk_sum = cv.take<int2>(sort_chunk_count(s.total_bricks));
    c.sort.totals = cv.take<int2>(1);
    c.sort.key = cv.take<int32_t>(s.ntot);
    c.sort.rank = cv.take<int32_t>(s.ntot);
    c.max_items = (int64_t)s.total_bricks + s.ntot / 64 + 1;
    c.sort.items = cv.take<int4>(c.max_items);
    c.act.flag = cv.take<int32_t>(s.total_bricks);
    c.act.list = cv.take<int32_t>(s.total_bricks);
    c.act.count = cv.take<int32_t>(1);
    c.act.done = cv.take<int32_t>(1);
    c.env_bofs = cv.take<int32_t>(s.n_envs + 1);
    c.act.env_bofs = c.env_bofs;
}

// Every device buffer the kernels use must have been carved.
bool all_carved(const mpm_ctx &c)
{
    const void *p[] = {c.env, c.env_pofs, c.env_gofs, c.tools, c.status, c.step, c.x, c.v, c.C, c.F, c.pid,
                       c.gP, c.gV, c.alt.x, c.alt.v, c.alt.C, c.alt.F, c.alt.pid, c.sort.count, c.sort.offset,
                       c.sort.chunk_sum, c.sort.totals, c.sort.key, c.sort.rank, c.sort.items, c.act.flag,
                       c.act.list, c.act.count, c.act.done, c.env_bofs, c.act.env_bofs};
    for (const void *q : p)
        if (!q) return false;
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
    if (!d->x0 || !d->v0 || !d->C0 || !d->F0 || !d->material) { why = "x0, v0, C0, F0 and material must be device pointers"; return false; }
    int64_t ntot = 0, nodes = 0, bricks = 0;
    for (int e = 0; e < d->n_envs; ++e) {
        int n = d->grid_n[e];
        if (n < 8 || n > 512 || n % 4) { why = "grid_n[" + std::to_string(e) + "] must be a multiple of 4 in [8, 512]"; return false; }
        if (2 * d->bound >= n) { why = "bound leaves no interior nodes"; return false; }
        if (d->n_particles[e] < 1) { why = "n_particles[" + std::to_string(e) + "] must be >= 1"; return false; }
        ntot += d->n_particles[e];
        nodes += (int64_t)n * n * n;
        bricks += (int64_t)(n / 4) * (n / 4) * (n / 4);
    }
    if (ntot > (1ll << 30)) { why = "too many particles (max 2^30)"; return false; }
    if (bricks > (1ll << 30)) { why = "too many grid bricks"; return false; }
    s.n_envs = d->n_envs;
    s.max_tools = d->max_tools;
    s.ntot = (int)ntot;
    s.total_nodes = nodes;
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

// One substep of the direct scheme.  Leaves the last P2G in the momentum
// buffer (readable), so the grid is not clean afterwards.
void substep_direct(mpm_ctx *c, hipStream_t st)
{
    Dev d = c->dev();
    launch_fill_f4(c->gP, c->total_nodes, st);
    launch_p2g_direct(d, st);
    launch_grid_dense(d, c->env_gofs, c->total_nodes, 0, st);
    launch_g2p_direct(d, st);
    c->grid_clean = false;
}

ParticleBuf live(const mpm_ctx *c) { return ParticleBuf{c->x, c->v, c->C, c->F, c->pid}; }

TiledArgs tiled_args(const mpm_ctx *c, const ParticleBuf &in, const ParticleBuf &out)
{
    TiledArgs a{};
    a.xin = in.x; a.vin = in.v; a.Cin = in.C; a.Fin = in.F; a.pidin = in.pid;
    a.xout = out.x; a.vout = out.v; a.Cout = out.C; a.Fout = out.F; a.pidout = out.pid;
    a.items = c->sort.items;
    a.totals = c->sort.totals;
    a.act = c->act;
    return a;
}

// Sort live particles into the alternate buffers and rebuild the items.
void sort_into_alt(mpm_ctx *c, hipStream_t st)
{
    launch_sort(c->dev(), c->sort, c->total_bricks, c->item, c->alt, 1, st);
    c->items_valid = true;
    c->items_P = c->item;
    c->since_sort = 0;
}

int grid_blocks(const mpm_ctx *c)
{
    int64_t b = ((int64_t)c->total_bricks + 3) / 4;
    return (int)std::max<int64_t>(8, std::min<int64_t>(b, 2048));
}

// n substeps of the tiled scheme:
//   [sort] head P2G, then n x (grid op, fused G2P+P2G) with the last fused
//   step replaced by a G2P-only tail that materialises v and C.
void substeps_tiled(mpm_ctx *c, int n, hipStream_t st)
{
    Dev d = c->dev();
    if (!c->grid_clean) {
        launch_fill_f4(c->gP, c->total_nodes, st);
        c->grid_clean = true;
    }
    if (c->tiled_blocks == 0) c->tiled_blocks = tiled_workgroups(c->block);
    const int nb = c->tiled_blocks;
    ParticleBuf A = live(c), in = A;
    if (!c->items_valid || c->items_P != c->item || c->since_sort >= c->sort_every) {
        sort_into_alt(c, st);
        in = c->alt;
    }
    launch_p2g_tiled(d, tiled_args(c, in, in), c->block, nb, st);
    for (int i = 0; i < n; ++i) {
        launch_grid_active(d, c->act, grid_blocks(c), st);
        if (i == n - 1) {
            launch_g2p_tiled(d, tiled_args(c, in, A), c->block, nb, st);
        } else {
            if (c->since_sort >= c->sort_every && in.x == A.x) {
                sort_into_alt(c, st);
                in = c->alt;
            }
            launch_fused_tiled(d, tiled_args(c, in, A), c->block, nb, st);
            in = A;
        }
        c->since_sort += 1;
    }
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

mpm_status mpm_create(const mpm_desc *desc, void *workspace, size_t workspace_bytes, void *stream, mpm_ctx **out)
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
        c->checkpoint_every = std::max(1, desc->checkpoint_every);
        c->max_tape = desc->max_tape_substeps;
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
        size_t N = s.ntot;
        if ((e2 = hipMemcpyAsync(c->x, desc->x0, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e2 = hipMemcpyAsync(c->v, desc->v0, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e2 = hipMemcpyAsync(c->C, desc->C0, 9 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e2 = hipMemcpyAsync(c->F, desc->F0, 9 * N * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return cleanup_fail(e2, "copy initial state");
        launch_iota(c->pid, s.ntot, st);
        launch_fill_u32(c->status, s.n_envs, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->step), s.n_envs, 0u, st);
        launch_fill_f4(c->gP, s.total_nodes, st);
        launch_fill_f4(c->gV, s.total_nodes, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->act.flag), s.total_bricks, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->act.count), 1, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->act.done), 1, 0u, st);
        if ((e2 = hipGetLastError()) != hipSuccess) return cleanup_fail(e2, "init kernels");
        if ((e2 = hipStreamSynchronize(st)) != hipSuccess) return cleanup_fail(e2, "create sync");
        *out = c;
        return MPM_OK;
    } catch (...) {
        return fail(nullptr, MPM_E_ARG, "internal error in mpm_create");
    }
}

void mpm_destroy(mpm_ctx *ctx)
{
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
            if (t->shape != MPM_TOOL_CAPSULE) return fail(c, MPM_E_UNSUPPORTED, "only MPM_TOOL_CAPSULE is implemented");
            if (t->contact != MPM_CONTACT_SLIP && t->contact != MPM_CONTACT_STICKY) return fail(c, MPM_E_ARG, "bad contact mode");
            if (!(t->radius > 0.f) || !(t->half_len >= 0.f) || !(t->friction >= 0.f) || !std::isfinite(t->theta) ||
                !std::isfinite(t->radius) || !std::isfinite(t->half_len) || !std::isfinite(t->friction))
                return fail(c, MPM_E_ARG, "tool needs radius > 0, half_len >= 0, friction >= 0, finite theta");
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
            td.k = 0;
            td.u = u;
            for (int i = 0; i < 3; ++i) td.T[i] = (double)t->T0[i];
        }
        size_t slot = (size_t)env * c->max_tools + tool;
        c->tools_h[slot] = td;
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
        return MPM_OK;
    case MPM_OPT_BLOCK:
        if (value != 64 && value != 128 && value != 256) return fail(c, MPM_E_ARG, "block must be 64, 128 or 256");
        c->block = value;
        c->tiled_blocks = 0;
        return MPM_OK;
    case MPM_OPT_ITEM:
        if (value < 64 || value > 4096 || value % 64) return fail(c, MPM_E_ARG, "item size must be a multiple of 64 in [64, 4096]");
        c->item = value;
        return MPM_OK;
    case MPM_OPT_GRAPH:
        c->use_graph = value != 0;
        return MPM_OK;
    case MPM_OPT_PERSISTENT:
        if (value) return fail(c, MPM_E_UNSUPPORTED, "persistent kernel not available");
        c->persistent = 0;
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
    if (record_tape) return fail(c, MPM_E_UNSUPPORTED, "adjoint tape not available");
    hipStream_t st = as_stream(stream);
    if (c->scheme == MPM_SCHEME_TILED) substeps_tiled(c, n_substeps, st);
    else for (int i = 0; i < n_substeps; ++i) substep_direct(c, st);
    return check_launch(c, "mpm_substep");
}

mpm_status mpm_run_stage(mpm_ctx *c, int32_t stage, void *stream)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    hipStream_t st = as_stream(stream);
    Dev d = c->dev();
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
    default:
        return fail(c, MPM_E_ARG, "unknown stage");
    }
    return check_launch(c, "mpm_run_stage");
}

mpm_status mpm_substep_adjoint(mpm_ctx *c, int32_t n_substeps, const mpm_adjoint_io *io, void *stream)
{
    if (!c) return fail(nullptr, MPM_E_ARG, "ctx is NULL");
    (void)n_substeps; (void)io; (void)stream;
    return fail(c, MPM_E_STATE, "no adjoint tape recorded");
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
    case MPM_F_F: comps = 9; src = c->F; break;
    case MPM_F_GRID_M: comps = 1; break;
    case MPM_F_GRID_MV: comps = 3; break;
    case MPM_F_GRID_V: comps = 3; break;
    case MPM_F_STATUS: need = sizeof(uint32_t); break;
    case MPM_F_TOOL_T: need = sizeof(double) * 3 * std::max(1, c->max_tools); break;
    case MPM_F_STEP: need = sizeof(int32_t); break;
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

const char *mpm_last_error(const mpm_ctx *c)
{
    if (c) return c->err.empty() ? "no error" : c->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"
