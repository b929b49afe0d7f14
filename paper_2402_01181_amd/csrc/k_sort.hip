// Counting sort of particles by the cell of their stencil base, cells
// numbered brick-major (so each 4x4x4-cell brick is contiguous and grouped
// by cell inside), and the work-item list of the tiled scheme.  All kernels,
// no host sync.
//
//   1. k_cell_count: cell of each particle; rank within the cell by an
//      atomic counter (histogram), and particles per brick.
//   2. scan of (particles, items) per brick, items = ceil(count / P).
//   3. k_make_items: per occupied brick, the first slot of each of its 64
//      cells (a wavefront scan) and its items (brick, first slot, count,
//      environment); the counters are cleared for the next sort.
//   4. k_sort_scatter: move particle state into its sorted slot.
// Cell counts are only touched where particles are, so nothing proportional
// to the grid is cleared or scanned.
#include "mpm_tile_util.h"

namespace mpm {

// Cell key of a particle: brick-major number of the cell holding its
// stencil base, clamped in floating point (NaN -> 0) so frozen particles go
// to an edge cell.
__device__ __forceinline__ int particle_cell(const EnvDev &e, float x0, float x1, float x2)
{
    int t[3];
    float xs[3] = {x0, x1, x2};
#pragma unroll
    for (int a = 0; a < 3; ++a) t[a] = (int)floorf(fminf(fmaxf(xs[a] * e.inv_dx - 0.5f, 0.0f), (float)(e.n - 3)));
    const int brick = e.bofs + ((t[0] >> 2) * e.nb + (t[1] >> 2)) * e.nb + (t[2] >> 2);
    return brick * 64 + ((t[0] & 3) * 4 + (t[1] & 3)) * 4 + (t[2] & 3);
}

// Whether a particle may be frozen out of the domain, with half a cell to
// spare: its stencil base within half a cell of where the particle kernels
// freeze it (or a non-finite position).  Between the fused substeps of a
// call only such particles carry v and C (the others' are recomputed from
// the grid), so a sort there moves those two fields for them alone.  The
// margin keeps the decision independent of how either side rounds the test.
__device__ __forceinline__ bool near_domain_edge(const EnvDev &e, float x0, float x1, float x2)
{
    const float xs[3] = {x0, x1, x2};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float tb = xs[a] * e.inv_dx - 0.5f;
        in = in && tb >= 0.5f && tb < (float)(e.n - 2) - 0.5f;
    }
    return !in;
}

// Bit of a particle's rank that marks it near the domain edge.
constexpr int RANK_EDGE = (int)0x80000000u;

// Cell key and rank of each particle, and the particle count of every cell
// and brick.  Particles arrive mostly in cell order (from the previous sort),
// so a wavefront holds few distinct cells and bricks.  The lanes of one cell
// are grouped first (ballots, no memory traffic); then the lowest lane of
// every group adds the group's size to its cell's counter, all groups in one
// atomic instruction, and each lane's rank is that base plus its position in
// the group.
__global__ __launch_bounds__(256) void k_cell_count(Dev d, SortBuf s, ActiveBuf act)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x & 63;
    if (act.flag && q == 0) gstore(act.scount, 0);   // the static list is rebuilt next
    const bool valid = q < d.ntot;
    const int N = d.ntot;
    int key = -1;
    bool edge = false;
    if (valid) {
        const EnvDev e = load_env(d.env + env_of_particle(d, q));
        const float x0 = gload(d.x + q), x1 = gload(d.x + N + q), x2 = gload(d.x + 2 * N + q);
        key = particle_cell(e, x0, x1, x2);
        edge = near_domain_edge(e, x0, x1, x2);
        gstore(s.key + q, key);
    }
    const unsigned long long lower = (1ull << lane) - 1ull;
    const int brick = key >> 6;
    int leader = lane, pos = 0, size = 0;        // cell group
    int bleader = lane, bsize = 0;               // brick group
    unsigned long long pending = __ballot(valid);
    while (pending) {
        const int l = __builtin_ctzll(pending);
        const int kc = __builtin_amdgcn_readlane(key, l);   // l is the same on every lane
        const unsigned long long same = __ballot(valid && key == kc);
        if ((same >> lane) & 1ull) {
            leader = l;
            pos = (int)__popcll(same & lower);
        }
        if (lane == l) size = (int)__popcll(same);
        pending &= ~same;
    }
    pending = __ballot(valid);
    while (pending) {
        const int l = __builtin_ctzll(pending);
        const int kb = __builtin_amdgcn_readlane(brick, l);
        const unsigned long long same = __ballot(valid && brick == kb);
        if ((same >> lane) & 1ull) bleader = l;
        if (lane == l) bsize = (int)__popcll(same);
        pending &= ~same;
    }
    int base = 0;
    if (valid && lane == leader) base = gatomic_add(s.count + key, size);
    if (valid && lane == bleader) gatomic_add(s.brick_count + brick, bsize);
    base = __shfl(base, leader);
    if (valid) gstore(s.rank + q, (base + pos) | (edge ? RANK_EDGE : 0));
}

// Block-wide exclusive scan of int2 over 256 threads x 4 elements.
constexpr int SCAN_T = 256, SCAN_E = 4, SCAN_CHUNK = SCAN_T * SCAN_E;
static_assert(SCAN_CHUNK == SORT_SCAN_CHUNK, "brick scan chunk");

__device__ __forceinline__ int2 add2(int2 a, int2 b) { return make_int2(a.x + b.x, a.y + b.y); }

__device__ int2 block_exclusive_scan(int2 v, int2 *sh, int2 &total)
{
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int2 a = t >= off ? sh[t - off] : make_int2(0, 0);
        __syncthreads();
        sh[t] = add2(sh[t], a);
        __syncthreads();
    }
    int2 incl = sh[t];
    total = sh[SCAN_T - 1];
    __syncthreads();
    return make_int2(incl.x - v.x, incl.y - v.y);
}

// Per brick: (particles, items = ceil(count / P)); local exclusive scan per
// chunk of bricks.
__global__ __launch_bounds__(SCAN_T) void k_scan_local(SortBuf s, int nb, int P)
{
    __shared__ int2 sh[SCAN_T];
    int base = blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_E;
    int2 v[SCAN_E], sum = make_int2(0, 0);
#pragma unroll
    for (int i = 0; i < SCAN_E; ++i) {
        int k = base + i;
        int c = k < nb ? gload(s.brick_count + k) : 0;
        v[i] = make_int2(c, (c + P - 1) / P);
        sum = add2(sum, v[i]);
    }
    int2 total;
    int2 ex = block_exclusive_scan(sum, sh, total);
#pragma unroll
    for (int i = 0; i < SCAN_E; ++i) {
        int k = base + i;
        if (k < nb) s.brick_offset[k] = ex;
        ex = add2(ex, v[i]);
    }
    if (threadIdx.x == 0) s.chunk_sum[blockIdx.x] = total;
}

// Scan of the chunk sums in one block; writes totals (particles, items).
__global__ __launch_bounds__(SCAN_T) void k_scan_chunks(SortBuf s, int nchunks)
{
    __shared__ int2 sh[SCAN_T];
    int2 carry = make_int2(0, 0);
    for (int c0 = 0; c0 < nchunks; c0 += SCAN_T) {
        int k = c0 + threadIdx.x;
        int2 v = k < nchunks ? s.chunk_sum[k] : make_int2(0, 0);
        int2 total;
        int2 ex = block_exclusive_scan(v, sh, total);
        if (k < nchunks) s.chunk_sum[k] = add2(ex, carry);
        carry = add2(carry, total);
    }
    if (threadIdx.x == 0) *s.totals = carry;
}

// One wavefront per brick: an occupied brick gets the first slot of each of
// its 64 cells (exclusive scan of the cell counts across the lanes) and its
// items; its counters are cleared for the next sort.
__global__ __launch_bounds__(256) void k_make_items(SortBuf s, const int32_t *brick_env, int nb, int P)
{
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (k >= nb) return;
    const int c = gload(s.brick_count + k);
    if (c == 0) return;
    const int2 o = add2(s.brick_offset[k], s.chunk_sum[k / SCAN_CHUNK]);
    const int64_t cell = (int64_t)k * 64 + lane;
    const int n = gload(s.count + cell);
    int incl = n;                       // inclusive scan over the 64 lanes
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    gstore(s.offset + cell, o.x + incl - n);
    gstore(s.count + cell, 0);
    const int env = gload(brick_env + k);
    for (int j = lane, first = o.x + lane * P; first < o.x + c; j += 64, first += 64 * P) {
        const int cnt = o.x + c - first;
        s.items[o.y + j] = make_int4(k, first, cnt < P ? cnt : P, env);
    }
    if (lane == 0) gstore(s.brick_count + k, 0);
}

// Move each particle to its slot: x, H and the particle index, and v and C
// too for every particle (full = 1: the state at the start of a call) or for
// the particles near the domain edge only (full = 0: between fused substeps,
// where only frozen particles carry v and C).  All of a particle's loads are
// issued before its first store: the destination may alias a source as far
// as the compiler knows, so stores placed between the loads would each wait
// for the memory round trip of the load before them.
__global__ __launch_bounds__(256) void k_sort_scatter(Dev d, SortBuf s, ParticleBuf dst, int full)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.ntot) return;
    const size_t N = d.ntot;
    float x[3], H[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = gload(d.x + c * N + q);
#pragma unroll
    for (int c = 0; c < 9; ++c) H[c] = gload(d.H + c * N + q);
    const int pid = gload(d.pid + q);
    const int rank = gload(s.rank + q);
    const size_t to = gload(s.offset + gload(s.key + q)) + (rank & ~RANK_EDGE);
    if (full || (rank & RANK_EDGE)) {
        float v[3], C[9];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = gload(d.v + c * N + q);
#pragma unroll
        for (int c = 0; c < 9; ++c) C[c] = gload(d.C + c * N + q);
#pragma unroll
        for (int c = 0; c < 3; ++c) gstore(dst.v + c * N + to, v[c]);
#pragma unroll
        for (int c = 0; c < 9; ++c) gstore(dst.C + c * N + to, C[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) gstore(dst.x + c * N + to, x[c]);
#pragma unroll
    for (int c = 0; c < 9; ++c) gstore(dst.H + c * N + to, H[c]);
    gstore(dst.pid + to, pid);
}

// Drop the previous static brick list (its flags).
__global__ void k_static_clear(ActiveBuf act)
{
    const int n = gload(act.scount);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        gstore(act.flag + gload(act.slist + i), 0);
}

// New static brick list: the 27-brick neighbourhood (within its environment's
// grid) of every occupied particle brick; one lane per (brick, neighbour).  A
// brick a P2G listed as far (flag 2) before this sort, whose dynamic entry
// the next grid operation has not consumed yet, moves to the static list
// too (2 -> 1): later P2Gs add to it without listing it, so the static list
// must hold it; the grid operation then skips its dynamic entry.
__global__ __launch_bounds__(256) void k_static_build(Dev d, SortBuf s, ActiveBuf act)
{
    const int b = blockIdx.x * 8 + (threadIdx.x >> 5), o = threadIdx.x & 31;
    if (b >= act.nbricks || o >= 27 || gload(s.brick_count + b) == 0) return;
    const EnvDev e = load_env(d.env + gload(act.brick_env + b));
    const int lb = b - e.bofs;
    const int bi = lb / (e.nb * e.nb) + o / 9 - 1, bj = (lb / e.nb) % e.nb + (o / 3) % 3 - 1,
              bk = lb % e.nb + o % 3 - 1;
    if (bi < 0 || bj < 0 || bk < 0 || bi >= e.nb || bj >= e.nb || bk >= e.nb) return;
    const int x = e.bofs + (bi * e.nb + bj) * e.nb + bk;
    if (gatomic_cas(act.flag + x, 0, 1) || gatomic_cas(act.flag + x, 2, 1))
        gstore(act.slist + gatomic_add(act.scount, 1), x);
}

void launch_sort(const Dev &d, const SortBuf &s, const ActiveBuf &act, int total_bricks, int P,
                 const ParticleBuf &dst, int full, hipStream_t st)
{
    // cell and brick counters are zero here: set at create, cleared by k_make_items
    const int nblk = (total_bricks + 255) / 256;
    if (act.flag) launch_k(k_static_clear, dim3(nblk < 1024 ? nblk : 1024), dim3(256), 0, st, act);
    launch_k(k_cell_count, dim3((d.ntot + 255) / 256), dim3(256), 0, st, d, s, act);
    if (act.flag) launch_k(k_static_build, dim3((total_bricks + 7) / 8), dim3(256), 0, st, d, s, act);
    int nchunks = (total_bricks + SCAN_CHUNK - 1) / SCAN_CHUNK;
    launch_k(k_scan_local, dim3(nchunks), dim3(SCAN_T), 0, st, s, total_bricks, P);
    launch_k(k_scan_chunks, dim3(1), dim3(SCAN_T), 0, st, s, nchunks);
    launch_k(k_make_items, dim3((total_bricks + 3) / 4), dim3(256), 0, st, s, act.brick_env, total_bricks, P);
    launch_k(k_sort_scatter, dim3((d.ntot + 255) / 256), dim3(256), 0, st, d, s, dst, full);
}

size_t sort_chunk_count(int64_t n) { return (size_t)((n + SCAN_CHUNK - 1) / SCAN_CHUNK); }

}  // namespace mpm
