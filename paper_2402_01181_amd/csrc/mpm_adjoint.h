// Reverse-mode (adjoint) substep: tape layout and kernel launchers.
#pragma once
#include <initializer_list>

#include "mpm_tiled.h"

namespace mpm {

// Adjoint state of one reverse pass.  Particle arrays use the original
// particle order, [comp][ntot].
struct AdjBuf {
    float *xb, *vb, *Cb, *Fb;
    float4 *gVb;        // [total_nodes] adjoint of the node velocity (xyz); kept zero between substeps
    float4 *gPb;        // [total_nodes] adjoint of (m, mv)
    double *ubar;       // [n_envs][max_tools][max_tape][3] direct dL/du per substep
    double *Tbar;       // [n_envs][max_tools][max_tape][3] dL/dT per substep
    double *mubar;      // [n_envs]
    double *lambar;     // [n_envs]
    int max_tape;
    int j;              // window-relative substep index of the current reverse step
};

// Contact decision of a node, recorded by the tape's grid pass:
// -1 no contact / unchanged, else tool * 4 + branch (branch as in ContactRec).
typedef int8_t ContactCode;

// The nodes a tape grid pass visits: the tape's static brick list (one
// wavefront per brick), or every node when `dense` is set or the P2G that
// wrote this grid reached a brick outside the list (far[far_slot] ==
// far_stamp).
struct TapeList {
    const int32_t *slist;
    const int32_t *scount;
    const int32_t *brick_env;
    const int32_t *far;
    int far_slot, far_stamp;
    int dense;
};

// Grid pass of the tape: V, (m, v-hat) and the contact decision of the
// visited nodes.  With snap != nullptr the tool table (slots entries) is
// copied there.
void launch_grid_tape(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, ContactCode *dec, ToolDev *snap,
                      int slots, const TapeList &tl, hipStream_t st);
void launch_adj_g2p(const Dev &d, const AdjBuf &a, hipStream_t st);
// Reverse grid operation over the visited nodes; clears the node-velocity
// adjoint and the tape's (m, v-hat) of every node it visits, so tape grids and
// adjoints are zero outside the visited nodes between uses.
void launch_adj_grid(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, const ContactCode *dec,
                     const AdjBuf &a, const TapeList &tl, hipStream_t st);
void launch_adj_p2g(const Dev &d, const AdjBuf &a, hipStream_t st);
// Zero the tape grid d.gP over the nodes tl visits (a recomputed substep the
// reverse pass did not reach).
void launch_tape_clear(const Dev &d, const int64_t *env_gofs, int64_t total_nodes, const TapeList &tl,
                       hipStream_t st);
void launch_adj_finish(const Dev &d, const AdjBuf &a, int n, double *gE, double *gnu, double *gu, double *gT,
                       hipStream_t st);
void launch_adj_g2p_tiled(const Dev &d, const AdjBuf &a, const int4 *items, const int2 *totals, int slots,
                          const ActiveBuf &act, int block, int nblocks, hipStream_t st);
void launch_adj_p2g_tiled(const Dev &d, const AdjBuf &a, const int4 *items, const int2 *totals,
                          const ActiveBuf &act, int block, int nblocks, hipStream_t st);
// reverse P2G of substep j (dp: its recorded state) and reverse G2P of substep
// j - 1 (dg: its recorded state, node velocities dg.gV) in one kernel
void launch_adj_pair_tiled(const Dev &dp, const Dev &dg, const AdjBuf &a, const int4 *items, const int2 *totals,
                           int slots, const ActiveBuf &act, int block, int nblocks, hipStream_t st);
// scatter == 0: dst[c][q] = src[c][perm[q]]; scatter != 0: dst[c][perm[q]] = src[c][q]
void launch_permute(const float *src, const int32_t *perm, int ntot, int comps, float *dst, int scatter,
                    hipStream_t st);
void launch_unpermute(const float *src, const int32_t *pid, int ntot, int comps, float *dst, hipStream_t st);
void launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st);
// Several copies (bytes a multiple of 4, regions disjoint) in one launch.
constexpr int COPY_JOBS = 4;
struct CopySpec {
    void *dst;
    const void *src;
    size_t bytes;
};
struct CopyJobs {
    uint32_t *dst[COPY_JOBS];
    const uint32_t *src[COPY_JOBS];
    size_t words[COPY_JOBS];
};
void launch_copies(std::initializer_list<CopySpec> jobs, hipStream_t st);
void launch_fill_f64(double *p, int64_t n, hipStream_t st);

}  // namespace mpm
