// Small utility kernels: fills, copies and layout conversion for reads.
// Fills are kernels (not hipMemsetAsync) so callers may capture them.
#include "mpm_kernels.h"

namespace mpm {

thread_local LaunchTimer launch_timer;

__global__ void k_fill_f4(float4 *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_iota(int32_t *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

// Particle slot q of environment [pofs, pofs+np) holds original particle
// pid[q]; write it to dst[c][pid[q] - pofs].
__global__ void k_read_particles(const float *src, const int32_t *pid, int ntot, int pofs, int np, int comps,
                                 float *dst)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int q = pofs + i;
    int o = pid[q] - pofs;
    for (int c = 0; c < comps; ++c) dst[(size_t)c * np + o] = src[(size_t)c * ntot + q];
}

__global__ void k_write_particles(float *dst, const int32_t *pid, int ntot, int pofs, int np, int comps,
                                  const float *src)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int q = pofs + i;
    int o = pid[q] - pofs;
    for (int c = 0; c < comps; ++c) dst[(size_t)c * ntot + q] = src[(size_t)c * np + o];
}

// Brick-major grid slice -> dense [comp][n^3] with node (i,j,k) at (i*n+j)*n+k.
__global__ void k_read_grid(const float4 *g, int64_t gofs, int n, int comp0, int comps, float *dst)
{
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nn = (int64_t)n * n * n;
    if (id >= nn) return;
    int k = (int)(id % n), j = (int)((id / n) % n), i = (int)(id / ((int64_t)n * n));
    int nb = n / 4;
    int b = ((i >> 2) * nb + (j >> 2)) * nb + (k >> 2);
    const float *src = reinterpret_cast<const float *>(g + gofs + (int64_t)b * 64 + ((i & 3) << 4) + ((j & 3) << 2) + (k & 3));
    for (int c = 0; c < comps; ++c) dst[(size_t)c * nn + id] = src[comp0 + c];
}

__global__ void k_add_identity(float *p, int64_t n, int64_t stride, float sign)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        p[i] += sign;
        p[4 * stride + i] += sign;
        p[8 * stride + i] += sign;
    }
}

static unsigned grid_for(int64_t n, int block = 256)
{
    int64_t b = (n + block - 1) / block;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_fill_f4(float4 *p, int64_t n, hipStream_t st)
{
    launch_k(k_fill_f4, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t st)
{
    launch_k(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, st, p, n, value);
}

void launch_iota(int32_t *p, int n, hipStream_t st)
{
    launch_k(k_iota, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}

void launch_read_particles(const float *src, const int32_t *pid, int ntot, int pofs, int np, int comps,
                           float *dst, hipStream_t st)
{
    launch_k(k_read_particles, dim3((np + 255) / 256), dim3(256), 0, st, src, pid, ntot, pofs, np,
                       comps, dst);
}

void launch_write_particles(float *dst, const int32_t *pid, int ntot, int pofs, int np, int comps,
                            const float *src, hipStream_t st)
{
    launch_k(k_write_particles, dim3((np + 255) / 256), dim3(256), 0, st, dst, pid, ntot, pofs, np,
                       comps, src);
}

void launch_add_identity(float *p, int64_t n, int64_t stride, float sign, hipStream_t st)
{
    launch_k(k_add_identity, dim3(grid_for(n)), dim3(256), 0, st, p, n, stride, sign);
}

void launch_read_grid(const float4 *g, int64_t gofs, int n, int comp0, int comps, float *dst, hipStream_t st)
{
    int64_t nn = (int64_t)n * n * n;
    launch_k(k_read_grid, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, g, gofs, n, comp0,
                       comps, dst);
}

}  // namespace mpm
