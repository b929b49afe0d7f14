// Surface extraction (marching cubes over the mass volume): case table,
// scratch buffers and the launcher.
#pragma once
#include "mpm_dev.h"

namespace mpm {

constexpr int MC_MAX_TRI = 5;      // the face-walk rule never needs more per cell

// Triangles of each of the 256 corner cases as edge triples (4 KB).
struct McTable {
    uint8_t ntri[256];
    int8_t edge[256][3 * MC_MAX_TRI];
};

static_assert(sizeof(McTable) == 4096, "McTable layout");

struct SurfBuf {
    float *rho;             // [n^3] density of the environment being extracted
    int32_t *ofs;           // [(n-1)^3] triangle offset of each cell within its scan chunk
    int32_t *chunk;         // [chunks] exclusive prefix of the chunk totals
    const McTable *table;   // device copy of the case table
};

// Work items of the last sort, when the particle buffers are in their sorted
// slots (items == nullptr: no valid items, one atomic per weight instead).
struct SurfItems {
    const int4 *items;
    const int2 *totals;
    int64_t max_items;
};

// Builds the table from the face-walk rule; false if a case does not close.
bool build_mc_table(McTable &t);
void launch_surface(const Dev &d, int env, int np, int n, float dx, float iso, const SurfBuf &b,
                    const SurfItems &items, float *tris, int64_t max_tris, int64_t *n_tris, hipStream_t st);
size_t surf_chunk_count(int64_t cells);

}  // namespace mpm
