// Block grid of every level and the coarse/fine coupling plan.  Internal.
#pragma once
#include <functional>
#include <string>
#include <vector>

#include "../../include/lbmtree.h"
#include "lbm_geometry.h"
#include "lbm_internal.h"

namespace lbm {

// Coupling between level l (coarse) and l + 1 (fine).
struct AmrPair {
    // coarse cells (element addresses) whose (rho, u, strain rate) feed the
    // fine ghost interpolation
    std::vector<uint32_t> h_src;
    // fine ghost cells and, per ghost, 8 indices into the source list; entry
    // q = (ox + 2 oy + 4 oz) is the coarse cell P + o*s of the trilinear
    // stencil (weights 3/4 for o = 0, 1/4 for o = 1 per axis)
    std::vector<uint32_t> h_ghost;
    std::vector<int32_t> h_ghost_src;
    // per ghost, bit k set when its post-collision population k streams into
    // a collided cell (active or band) of level l + 1; only those are stored
    std::vector<uint32_t> h_ghost_mask;
    // coarse band cells (covered, within two cells of the coarse leaf region)
    // and their eight fine children (cell addresses on level l + 1)
    std::vector<uint32_t> h_band;
    std::vector<uint32_t> h_band_child;
    // device copies
    uint32_t *d_src = nullptr, *d_ghost = nullptr, *d_ghost_mask = nullptr, *d_band = nullptr;
    int32_t *d_ghost_src = nullptr;
    uint32_t *d_band_child = nullptr;
    float *d_mom[2] = {nullptr, nullptr};  // MOM_REC floats per source cell at T and T+1
    int32_t *d_mom_idx = nullptr;          // per cell address of level l: source index or -1
};

struct AmrPlan {
    std::vector<AmrPair> pairs;  // pairs[l] couples l and l + 1
};

using Alloc = std::function<lbm_status(void **, size_t)>;

lbm_status build_levels(const lbm_grid_desc &d, int B, int L, const lbm_branch *b, int n_b,
                        const lbm_refine_desc *refine, const SolidMask &solid,
                        std::vector<DevLevel> &lv, AmrPlan &plan, std::string *msg);

// element address of level cell (x, y, z) (dense: x + nx (y + ny z); blocks:
// block * B^3 + local), wrapping y and z periodically; -1 when the level does
// not hold the cell
int64_t level_cell_address(const DevLevel &v, int B, int x, int y, int z);

lbm_status amr_upload(AmrPlan &plan, std::vector<DevLevel> &lv, int B, const Alloc &alloc, hipStream_t s,
                      std::string *msg);

}  // namespace lbm
