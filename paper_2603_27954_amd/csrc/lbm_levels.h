// Block grid of every level and the coarse/fine coupling plan.  Internal.
#pragma once
#include <functional>
#include <string>
#include <vector>

#include "../../include/lbmtree.h"
#include "lbm_internal.h"

namespace lbm {

// Coupling between level l (coarse) and l + 1 (fine).
struct AmrPair {
    // coarse cells whose (rho, u, S) feed the fine ghost interpolation
    std::vector<uint2> h_src;
    // fine ghost cells and, per ghost, 8 indices into the source list
    // (trilinear stencil, weights 3/4 and 1/4 per axis)
    std::vector<uint2> h_ghost;
    std::vector<int32_t> h_ghost_src;
    std::vector<uint8_t> h_ghost_par;  // bit a: fine index odd along axis a
    // coarse band cells (covered, within two cells of the coarse leaf region)
    // and their eight fine children (cell addresses on level l + 1)
    std::vector<uint2> h_band;
    std::vector<uint32_t> h_band_child;
    // device copies
    uint2 *d_src = nullptr, *d_ghost = nullptr, *d_band = nullptr;
    int32_t *d_ghost_src = nullptr;
    uint8_t *d_ghost_par = nullptr;
    uint32_t *d_band_child = nullptr;
    float *d_mom[2] = {nullptr, nullptr};  // 10 floats per source cell at T and T+1
};

struct AmrPlan {
    std::vector<AmrPair> pairs;  // pairs[l] couples l and l + 1
};

using Alloc = std::function<lbm_status(void **, size_t)>;

lbm_status build_levels(const lbm_grid_desc &d, int B, int L, const lbm_branch *b, int n_b,
                        const lbm_refine_desc *refine, const std::vector<uint8_t> &solid,
                        std::vector<DevLevel> &lv, AmrPlan &plan, std::string *msg);

// element address (block * B^3 + local) of level cell (x, y, z), wrapping y
// and z periodically; -1 when the level does not hold the cell
int64_t level_cell_address(const DevLevel &v, int B, int x, int y, int z);

lbm_status amr_upload(AmrPlan &plan, std::vector<DevLevel> &lv, int B, const Alloc &alloc, hipStream_t s,
                      std::string *msg);
// coarse moments of pair l at slot (0: time T, 1: time T + 1)
lbm_status amr_moments(AmrPlan &plan, std::vector<DevLevel> &lv, int l, int slot, int storage, int B,
                       hipStream_t s, std::string *msg);
// fine ghost populations of pair l for fine sub-step sub (0: from T, 1: mean of T and T+1)
lbm_status amr_prolong(AmrPlan &plan, std::vector<DevLevel> &lv, int l, int sub, int storage, int B,
                       uint32_t flags, hipStream_t s, std::string *msg);
// coarse band populations of pair l from the fine level
lbm_status amr_restrict(AmrPlan &plan, std::vector<DevLevel> &lv, int l, int storage, int B, uint32_t flags,
                        hipStream_t s, std::string *msg);

}  // namespace lbm
