// Surface extraction on the device: the paper's post-processing turns the
// particles into a triangle mesh by marching cubes over the mass volume
// (Sec. III-A; Lorensen and Cline's method as cited there).  Done here
// without leaving the GPU:
//
//   k_surf_density  particle mass splatted with the quadratic B-spline onto a
//                   dense n^3 node volume, density = m w / dx^3 (the P2G mass);
//                   k_surf_density_tiled does it per sorted work item through
//                   an LDS tile when the last sort's items are valid
//   k_surf_count    per cell: inside mask of the 8 corners (rho >= iso),
//                   triangles from the case table, exclusive scan in chunks
//   k_surf_top      scan of the chunk totals, total triangle count
//   k_surf_emit     per cell: crossing points by linear interpolation, the
//                   case's triangles written at the cell's offset
//
// Triangles come out in cell order (the order is fixed; vertex positions carry
// the rounding of the density's float atomic sums).  The case
// table is built on the host at context creation from the face-walk rule:
// on each cell face, the edges whose corners differ are crossed; two
// crossings make one segment, four (diagonal inside corners) make two, each
// cutting off one inside corner; every segment runs with the inside corners
// it bounds on its left seen from outside the cell, so the segments chain
// into closed polygons, each split into a fan from its lowest-numbered edge
// (polygons in order of their lowest edge), wound with the normal pointing
// out of the dense region.  Corner c = 4 dx + 2 dy + dz; edge e = 4 a + p
// along axis a, p = the other two corner bits in axis order.
#include "mpm_surface.h"
#include "mpm_tile_util.h"

#include <cstring>

namespace mpm {

namespace {

constexpr int SURF_T = 256;
constexpr int SURF_E = 8;
constexpr int SURF_CHUNK = SURF_T * SURF_E;

// the two corners of edge e (low end first)
__host__ __device__ inline void edge_corners(int e, int &c0, int &c1)
{
    const int a = e >> 2, hi = (e >> 1) & 1, lo = e & 1;
    int b[3];
    b[a] = 0;
    b[a == 0 ? 1 : 0] = hi;
    b[a == 2 ? 1 : 2] = lo;
    c0 = (b[0] << 2) | (b[1] << 1) | b[2];
    c1 = c0 | (4 >> a);
}

}  // namespace

// ---------------------------------------------------------------- case table (host)

static int edge_between(int c0, int c1)
{
    const int d = c0 ^ c1;
    const int a = d == 4 ? 0 : (d == 2 ? 1 : 2);
    const int lo = c0 & ~d;
    const int bx = (lo >> 2) & 1, by = (lo >> 1) & 1, bz = lo & 1;
    const int p = a == 0 ? (by << 1) | bz : (a == 1 ? (bx << 1) | bz : (bx << 1) | by);
    return (a << 2) | p;
}

// doubled integer coordinates of a corner and of an edge midpoint
static void corner2(int c, int v[3])
{
    v[0] = ((c >> 2) & 1) * 2; v[1] = ((c >> 1) & 1) * 2; v[2] = (c & 1) * 2;
}

static void mid2(int e, int v[3])
{
    int c0, c1, a[3], b[3];
    edge_corners(e, c0, c1);
    corner2(c0, a);
    corner2(c1, b);
    for (int k = 0; k < 3; ++k) v[k] = (a[k] + b[k]) / 2;
}

bool build_mc_table(McTable &t)
{
    memset(&t, 0, sizeof t);
    for (int mask = 0; mask < 256; ++mask) {
        int succ[12];
        for (int &s : succ) s = -1;
        for (int face = 0; face < 6; ++face) {
            const int a = face >> 1, side = face & 1;
            const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
            int ring[4];
            static const int RU[4] = {0, 1, 1, 0}, RV[4] = {0, 0, 1, 1};
            for (int r = 0; r < 4; ++r) {
                int bits[3];
                bits[a] = side; bits[u] = RU[r]; bits[v] = RV[r];
                ring[r] = (bits[0] << 2) | (bits[1] << 1) | bits[2];
            }
            bool in[4];
            int ncross = 0;
            for (int r = 0; r < 4; ++r) in[r] = (mask >> ring[r]) & 1;
            for (int r = 0; r < 4; ++r) ncross += in[r] != in[(r + 1) & 3];
            // segments (edge, edge, the inside corner on their left)
            int seg[2][3], ns = 0;
            if (ncross == 2) {
                int k = 0;
                seg[0][2] = -1;
                for (int r = 0; r < 4; ++r) {
                    if (in[r] != in[(r + 1) & 3]) seg[0][k++] = edge_between(ring[r], ring[(r + 1) & 3]);
                    if (in[r] && seg[0][2] < 0) seg[0][2] = ring[r];
                }
                ns = 1;
            } else if (ncross == 4) {
                for (int r = 0; r < 4; ++r)
                    if (in[r]) {
                        seg[ns][0] = edge_between(ring[(r + 3) & 3], ring[r]);
                        seg[ns][1] = edge_between(ring[r], ring[(r + 1) & 3]);
                        seg[ns][2] = ring[r];
                        ++ns;
                    }
            }
            int N[3] = {0, 0, 0};
            N[a] = side ? 1 : -1;
            for (int g = 0; g < ns; ++g) {
                int p = seg[g][0], q = seg[g][1], mp[3], mq[3], ck[3];
                mid2(p, mp);
                mid2(q, mq);
                corner2(seg[g][2], ck);
                const int d[3] = {mq[0] - mp[0], mq[1] - mp[1], mq[2] - mp[2]};
                const int l[3] = {N[1] * d[2] - N[2] * d[1], N[2] * d[0] - N[0] * d[2], N[0] * d[1] - N[1] * d[0]};
                const int side_k = l[0] * (ck[0] - mp[0]) + l[1] * (ck[1] - mp[1]) + l[2] * (ck[2] - mp[2]);
                if (side_k < 0) std::swap(p, q);
                if (side_k == 0 || succ[p] >= 0) return false;
                succ[p] = q;
            }
        }
        bool done[12] = {};
        int nt = 0;
        for (int start = 0; start < 12; ++start) {
            if (succ[start] < 0 || done[start]) continue;
            int poly[12], k = 0;
            for (int e = start; !done[e]; e = succ[e]) {
                if (succ[e] < 0 || k == 12) return false;
                done[e] = true;
                poly[k++] = e;
            }
            if (poly[0] != start || succ[poly[k - 1]] != start) return false;
            for (int i = 1; i + 1 < k; ++i) {
                if (nt == MC_MAX_TRI) return false;
                t.edge[mask][3 * nt + 0] = (int8_t)poly[0];
                t.edge[mask][3 * nt + 1] = (int8_t)poly[i + 1];
                t.edge[mask][3 * nt + 2] = (int8_t)poly[i];
                ++nt;
            }
        }
        t.ntri[mask] = (uint8_t)nt;
    }
    return true;
}

// ---------------------------------------------------------------- kernels

__global__ __launch_bounds__(256) void k_surf_clear(float *rho, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        rho[i] = 0.0f;
}

// Mass of each particle of the environment, spread with the P2G weights.
__global__ __launch_bounds__(256) void k_surf_density(Dev d, int env, float *rho)
{
    const EnvDev e = load_env(d.env + env);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= e.np) return;
    const int g = e.pofs + q;
    const int N = d.ntot;
    Stencil s;
    make_stencil(gload(d.x + g), gload(d.x + N + g), gload(d.x + 2 * N + g), e.inv_dx, e.n, s);
    if (s.outside) return;
    const float *mat = d.material + 4 * env;
    const float md = gload(mat + 2) * gload(mat + 3) * e.inv_dx * e.inv_dx * e.inv_dx;   // m / dx^3
    const int n = e.n;
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                const size_t id = ((size_t)(s.b[0] + o0) * n + (s.b[1] + o1)) * n + (s.b[2] + o2);
                gatomic_add(rho + id, md * s.w[0][o0] * s.w[1][o1] * s.w[2][o2]);
            }
}

// The same with the work items of the last sort: each workgroup takes an item
// (one brick's particles, in sorted slots) and sums its mass in a 6^3 LDS
// tile, which it then adds to the volume node by node; particles that have
// left the brick's tile since the sort add to the volume directly.  Cuts the
// global atomics on the densely shared nodes by the particles per node.
__global__ __launch_bounds__(256) void k_surf_density_tiled(Dev d, const int4 *items, const int2 *totals, int env,
                                                            float *rho)
{
    __shared__ float tile[TILE * TILE * TILE];
    const int nitems = gload(&totals->y);
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 item = gload(items + it);
        if (item.w != env) continue;
        EnvDev e;
        const Tile t = make_tile(d, item, e);
        for (int i = threadIdx.x; i < TILE * TILE * TILE; i += blockDim.x) tile[i] = 0.0f;
        __syncthreads();
        const float *mat = d.material + 4 * env;
        const float md = gload(mat + 2) * gload(mat + 3) * e.inv_dx * e.inv_dx * e.inv_dx;
        const int N = d.ntot, n = e.n;
        for (int q = threadIdx.x; q < item.z; q += blockDim.x) {
            const int g = item.y + q;
            Stencil s;
            make_stencil(gload(d.x + g), gload(d.x + N + g), gload(d.x + 2 * N + g), e.inv_dx, n, s);
            if (s.outside) continue;
            int l0, l1, l2;
            const bool in = stencil_in_tile(t, s, l0, l1, l2);
#pragma unroll
            for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
                for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
                    for (int o2 = 0; o2 < 3; ++o2) {
                        const float w = md * s.w[0][o0] * s.w[1][o1] * s.w[2][o2];
                        if (in) atomicAdd(&tile[((l0 + o0) * TILE + (l1 + o1)) * TILE + (l2 + o2)], w);
                        else gatomic_add(rho + ((size_t)(s.b[0] + o0) * n + (s.b[1] + o1)) * n + (s.b[2] + o2), w);
                    }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < TILE * TILE * TILE; i += blockDim.x) {
            const float v = tile[i];
            const int a = t.o[0] + i / (TILE * TILE), b = t.o[1] + (i / TILE) % TILE, c = t.o[2] + i % TILE;
            if (v != 0.0f && a < n && b < n && c < n) gatomic_add(rho + ((size_t)a * n + b) * n + c, v);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int cell_mask(const float *rho, int n, int i, int j, int k, float iso, float val[8])
{
    int m = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        val[c] = gload(rho + ((size_t)(i + ((c >> 2) & 1)) * n + (j + ((c >> 1) & 1))) * n + (k + (c & 1)));
        m |= (val[c] >= iso ? 1 : 0) << c;
    }
    return m;
}

__device__ __forceinline__ void cell_ijk(int64_t cell, int nc, int &i, int &j, int &k)
{
    k = (int)(cell % nc);
    const int64_t r = cell / nc;
    j = (int)(r % nc);
    i = (int)(r / nc);
}

// Triangles per cell and their exclusive prefix within chunks of SURF_CHUNK cells.
__global__ __launch_bounds__(SURF_T) void k_surf_count(const float *rho, int n, float iso, const McTable *tab,
                                                       int32_t *ofs, int32_t *chunk)
{
    __shared__ int sh[SURF_T];
    const int nc = n - 1;
    const int64_t ncell = (int64_t)nc * nc * nc;
    const int64_t base = (int64_t)blockIdx.x * SURF_CHUNK + (int64_t)threadIdx.x * SURF_E;
    int cnt[SURF_E], sum = 0;
#pragma unroll
    for (int q = 0; q < SURF_E; ++q) {
        cnt[q] = 0;
        const int64_t cell = base + q;
        if (cell < ncell) {
            int i, j, k;
            float val[8];
            cell_ijk(cell, nc, i, j, k);
            cnt[q] = tab->ntri[cell_mask(rho, n, i, j, k, iso, val)];
        }
        sum += cnt[q];
    }
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < SURF_T; off <<= 1) {      // inclusive Hillis-Steele scan
        const int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - sum;
#pragma unroll
    for (int q = 0; q < SURF_E; ++q) {
        const int64_t cell = base + q;
        if (cell < ncell) ofs[cell] = run;
        run += cnt[q];
    }
    if (threadIdx.x == SURF_T - 1) chunk[blockIdx.x] = sh[SURF_T - 1];
}

// Exclusive scan of the chunk totals (one workgroup) and the total count.
__global__ __launch_bounds__(SURF_T) void k_surf_top(int32_t *chunk, int nchunk, int64_t *total)
{
    __shared__ int64_t sh[SURF_T];
    int64_t carry = 0;
    for (int base = 0; base < nchunk; base += SURF_T) {
        const int i = base + threadIdx.x;
        const int64_t v = i < nchunk ? chunk[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < SURF_T; off <<= 1) {
            const int64_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nchunk) chunk[i] = (int32_t)(carry + sh[threadIdx.x] - v);
        carry += sh[SURF_T - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) gstore(total, carry);
}

__global__ __launch_bounds__(256) void k_surf_emit(const float *rho, int n, float dx, float iso, const McTable *tab,
                                                   const int32_t *ofs, const int32_t *chunk, float *tris,
                                                   int64_t max_tris)
{
    const int nc = n - 1;
    const int64_t ncell = (int64_t)nc * nc * nc;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncell) return;
    int i, j, k;
    float val[8];
    cell_ijk(cell, nc, i, j, k);
    const int mask = cell_mask(rho, n, i, j, k, iso, val);
    const int nt = tab->ntri[mask];
    if (nt == 0) return;
    const int64_t first = (int64_t)gload(ofs + cell) + gload(chunk + cell / SURF_CHUNK);
    const float org[3] = {(float)i, (float)j, (float)k};
    for (int t = 0; t < nt; ++t) {
        const int64_t slot = first + t;
        if (slot >= max_tris) return;
        float *out = tris + 9 * slot;
        for (int vtx = 0; vtx < 3; ++vtx) {
            int c0, c1;
            edge_corners(tab->edge[mask][3 * t + vtx], c0, c1);
            const float f = (iso - val[c0]) / (val[c1] - val[c0]);
            const int a = (c0 ^ c1) == 4 ? 0 : ((c0 ^ c1) == 2 ? 1 : 2);
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
                float p = org[dd] + (float)((c0 >> (2 - dd)) & 1);
                if (dd == a) p += f;
                gstore(out + 3 * vtx + dd, p * dx);
            }
        }
    }
}

void launch_surface(const Dev &d, int env, int np, int n, float dx, float iso, const SurfBuf &b,
                    const SurfItems &items, float *tris, int64_t max_tris, int64_t *n_tris, hipStream_t st)
{
    const int64_t nodes = (int64_t)n * n * n;
    const int64_t cells = (int64_t)(n - 1) * (n - 1) * (n - 1);
    const int nchunk = (int)((cells + SURF_CHUNK - 1) / SURF_CHUNK);
    launch_k(k_surf_clear, dim3((unsigned)std::min<int64_t>((nodes + 255) / 256, 8192)), dim3(256), 0, st, b.rho, nodes);
    if (items.items)
        launch_k(k_surf_density_tiled, dim3((unsigned)std::min<int64_t>(items.max_items, 4096)), dim3(256), 0, st, d,
                 items.items, items.totals, env, b.rho);
    else if (np > 0)
        launch_k(k_surf_density, dim3((np + 255) / 256), dim3(256), 0, st, d, env, b.rho);
    launch_k(k_surf_count, dim3(nchunk), dim3(SURF_T), 0, st, b.rho, n, iso, b.table, b.ofs, b.chunk);
    launch_k(k_surf_top, dim3(1), dim3(SURF_T), 0, st, b.chunk, nchunk, n_tris);
    launch_k(k_surf_emit, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, b.rho, n, dx, iso, b.table,
             b.ofs, b.chunk, tris, max_tris);
}

size_t surf_chunk_count(int64_t cells) { return (size_t)((cells + SURF_CHUNK - 1) / SURF_CHUNK); }

}  // namespace mpm
