// Block grid construction (paper Sec. 2.2: LBM on the cubic leaf blocks of
// an octree, finest near the tree surface, coarser away from it; blocks in
// space-filling-curve order) and the coarse/fine coupling plan.
#include "lbm_levels.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

namespace lbm {

static uint64_t spread3(uint64_t v)
{
    v &= 0x1FFFFF;
    v = (v | v << 32) & 0x1F00000000FFFFULL;
    v = (v | v << 16) & 0x1F0000FF0000FFULL;
    v = (v | v << 8) & 0x100F00F00F00F00FULL;
    v = (v | v << 4) & 0x10C30C30C30C30C3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}
static uint64_t morton(int x, int y, int z) { return spread3(x) | spread3(y) << 1 | spread3(z) << 2; }

int64_t level_cell_address(const DevLevel &v, int B, int x, int y, int z)
{
    if (x < 0 || x >= v.nx)
        return -1;
    y = (y % v.ny + v.ny) % v.ny;
    z = (z % v.nz + v.nz) % v.nz;
    if (v.dense)
        return (int64_t)x + (int64_t)v.nx * ((int64_t)y + (int64_t)v.ny * z);
    const int bi = v.h_lattice_to_block[(size_t)(x / B) + (size_t)v.nbx * ((size_t)(y / B) + (size_t)v.nby * (z / B))];
    if (bi < 0)
        return -1;
    return (int64_t)bi * B * B * B + (x % B) + B * ((y % B) + B * (z % B));
}

// Fills the block list (Morton order), lattice index, neighbour table and
// block coordinates of level v from its block map.  Level 0 wraps y and z and
// marks x faces; finer levels send absent neighbours to the sink block.
static void index_level(DevLevel &v, int level)
{
    std::vector<std::array<int, 3>> coords;
    for (int z = 0; z < v.nbz; ++z)
        for (int y = 0; y < v.nby; ++y)
            for (int x = 0; x < v.nbx; ++x)
                if (v.h_map[(size_t)x + (size_t)v.nbx * ((size_t)y + (size_t)v.nby * z)] != 0)
                    coords.push_back({x, y, z});
    std::sort(coords.begin(), coords.end(), [](const std::array<int, 3> &a, const std::array<int, 3> &b) {
        return morton(a[0], a[1], a[2]) < morton(b[0], b[1], b[2]);
    });
    v.nb = (int)coords.size();
    v.h_lattice_to_block.assign((size_t)v.nbx * v.nby * v.nbz, -1);
    v.h_bxyz.assign(3 * (size_t)(v.nb + 1), -1000000);
    for (int i = 0; i < v.nb; ++i) {
        const auto &c = coords[i];
        v.h_lattice_to_block[(size_t)c[0] + (size_t)v.nbx * ((size_t)c[1] + (size_t)v.nby * c[2])] = i;
        v.h_bxyz[3 * i] = c[0];
        v.h_bxyz[3 * i + 1] = c[1];
        v.h_bxyz[3 * i + 2] = c[2];
    }
    v.h_nbr.assign(27 * (size_t)(v.nb + 1), v.nb);
    for (int i = 0; i < v.nb; ++i) {
        const auto &c = coords[i];
        for (int k = 0; k < 27; ++k) {
            const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
            int x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
            int val;
            if (level == 0 && x < 0)
                val = NB_INLET;
            else if (level == 0 && x >= v.nbx)
                val = NB_OUTLET;
            else {
                if (level == 0) {
                    y = (y + v.nby) % v.nby;
                    z = (z + v.nbz) % v.nbz;
                }
                if (x < 0 || y < 0 || z < 0 || x >= v.nbx || y >= v.nby || z >= v.nbz)
                    val = v.nb;
                else {
                    const int bi = v.h_lattice_to_block[(size_t)x + (size_t)v.nbx * ((size_t)y + (size_t)v.nby * z)];
                    val = bi < 0 ? v.nb : bi;
                }
            }
            v.h_nbr[27 * (size_t)i + k] = val;
        }
    }
}

// Work list of a dense level: 256-cell tiles in element order holding at
// least one selected cell; partly selected tiles carry a bit mask.
static void dense_tiles(DevLevel &v, const std::function<bool(int64_t)> &sel, std::vector<uint2> &work,
                        int64_t *count)
{
    const int64_t N = (int64_t)v.nx * v.ny * v.nz;
    const int64_t ntile = N / DENSE_TILE;
    work.clear();
    *count = 0;
    std::vector<uint32_t> m(DENSE_TILE / 32);
    for (int64_t t = 0; t < ntile; ++t) {
        std::fill(m.begin(), m.end(), 0u);
        int n = 0;
        for (int c = 0; c < DENSE_TILE; ++c)
            if (sel(t * DENSE_TILE + c)) {
                m[c >> 5] |= 1u << (c & 31);
                ++n;
            }
        *count += n;
        if (n == 0)
            continue;
        uint32_t mid = FULL_MASK;
        if (n != DENSE_TILE) {
            mid = (uint32_t)(v.h_masks.size() / (DENSE_TILE / 32));
            v.h_masks.insert(v.h_masks.end(), m.begin(), m.end());
        }
        work.push_back(make_uint2((unsigned)t, mid));
    }
}

lbm_status build_levels(const lbm_grid_desc &d, int B, int L, const lbm_branch *b, int n_b,
                        const lbm_refine_desc *refine, const std::vector<uint8_t> &solid,
                        std::vector<DevLevel> &lv, AmrPlan &plan, std::string *msg)
{
    (void)b;
    (void)n_b;
    (void)refine;
    plan.pairs.clear();
    lv.assign(L, DevLevel{});
    if (L != 1) {
        *msg = "multi-level grids are built by build_levels_amr";
        return LBM_E_INVALID;
    }
    DevLevel &v = lv[0];
    v.level = 0;
    v.dense = true;
    v.nx = d.nx;
    v.ny = d.ny;
    v.nz = d.nz;
    v.nbx = d.nx / B;
    v.nby = d.ny / B;
    v.nbz = d.nz / B;
    v.h_map.assign((size_t)v.nbx * v.nby * v.nbz, 1);
    v.leaf_cells = (int64_t)d.nx * d.ny * d.nz;
    dense_tiles(v, [&](int64_t c) { return solid[(size_t)c] == 0; }, v.h_work, &v.updated_cells);
    v.h_leaf = v.h_work;
    return LBM_OK;
}

lbm_status amr_upload(AmrPlan &plan, std::vector<DevLevel> &lv, int B, const Alloc &alloc, hipStream_t s,
                      std::string *msg)
{
    (void)lv;
    (void)B;
    (void)alloc;
    (void)s;
    (void)msg;
    if (!plan.pairs.empty()) {
        *msg = "coarse/fine coupling not available";
        return LBM_E_INVALID;
    }
    return LBM_OK;
}

lbm_status amr_moments(AmrPlan &, std::vector<DevLevel> &, int, int, int, int, hipStream_t, std::string *msg)
{
    *msg = "coarse/fine coupling not available";
    return LBM_E_INVALID;
}

lbm_status amr_prolong(AmrPlan &, std::vector<DevLevel> &, int, int, int, int, uint32_t, hipStream_t,
                       std::string *msg)
{
    *msg = "coarse/fine coupling not available";
    return LBM_E_INVALID;
}

lbm_status amr_restrict(AmrPlan &, std::vector<DevLevel> &, int, int, int, uint32_t, hipStream_t,
                        std::string *msg)
{
    *msg = "coarse/fine coupling not available";
    return LBM_E_INVALID;
}

}  // namespace lbm
