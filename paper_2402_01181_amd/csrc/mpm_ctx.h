// Host-side context of the C ABI: configuration, the carved workspace and
// the sequencing state.  Internal to the library.
#pragma once
#include <string>
#include <vector>

#include "mpm_tiled.h"

struct mpm_ctx {
    std::string err;
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
    int spin_limit = 1 << 26;
    // device buffers carved from the caller's workspace
    mpm::EnvDev *env = nullptr;
    int32_t *env_pofs = nullptr;
    int64_t *env_gofs = nullptr;
    mpm::ToolDev *tools = nullptr;
    uint32_t *status = nullptr;
    int32_t *step = nullptr;
    float *x = nullptr, *v = nullptr, *C = nullptr, *F = nullptr;
    int32_t *pid = nullptr;
    float4 *gP = nullptr, *gV = nullptr;
    // tiled scheme
    mpm::ParticleBuf alt{};          // sort destination
    mpm::SortBuf sort{};
    mpm::ActiveBuf act{};
    int32_t *env_bofs = nullptr;
    int64_t max_items = 0;
    // sequencing state
    bool grid_clean = true;          // momentum buffer all zero, no active bricks
    bool items_valid = false;        // sort items match the current slot order and item size
    int items_P = 0;
    int since_sort = 0;
    int tiled_blocks = 0;            // persistent workgroups of the particle kernels
    // host mirror of the tool slots
    std::vector<mpm::ToolDev> tools_h;

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
        d.x = x; d.v = v; d.C = C; d.F = F;
        d.pid = pid;
        d.gP = gP; d.gV = gV;
        return d;
    }
};
