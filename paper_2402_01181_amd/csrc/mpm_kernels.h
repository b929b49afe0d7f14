// Kernel launchers of the HIP path (host-callable), grouped by scheme.
#pragma once
#include "mpm_dev.h"

namespace mpm {

// direct scheme (k_direct.hip)
void launch_p2g_direct(const Dev &d, hipStream_t st);
void launch_grid_dense(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, int zero_P, hipStream_t st);
void launch_g2p_direct(const Dev &d, hipStream_t st);

// utilities (k_util.hip)
void launch_fill_f4(float4 *p, int64_t n, hipStream_t st);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t st);
void launch_iota(int32_t *p, int n, hipStream_t st);
void launch_read_particles(const float *src, const int32_t *pid, int ntot, int pofs, int np, int comps,
                           float *dst, hipStream_t st);
void launch_write_particles(float *dst, const int32_t *pid, int ntot, int pofs, int np, int comps,
                            const float *src, hipStream_t st);
// p[c][i] += sign for the diagonal components c = 0, 4, 8 of a [9][stride] array, i < n.
void launch_add_identity(float *p, int64_t n, int64_t stride, float sign, hipStream_t st);
void launch_read_grid(const float4 *g, int64_t gofs, int n, int comp0, int comps, float *dst, hipStream_t st);

}  // namespace mpm
