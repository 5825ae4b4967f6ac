// Block grid construction (paper Sec. 2.2: LBM on the cubic leaf blocks of
// an octree, finest near the tree surface, coarser away from it; blocks in
// space-filling-curve order) and the coarse/fine coupling plan.
#include "lbm_levels.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <unordered_map>
#include <array>

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
    const int64_t slot = v.block_slot(x / B, y / B, z / B);
    if (slot < 0)
        return -1;
    const int bi = v.h_lattice_to_block[(size_t)slot];
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
    for (int z = v.box_o[2]; z < v.box_o[2] + v.box_n[2]; ++z)
        for (int y = v.box_o[1]; y < v.box_o[1] + v.box_n[1]; ++y)
            for (int x = v.box_o[0]; x < v.box_o[0] + v.box_n[0]; ++x)
                if (v.block_kind(x, y, z) != 0)
                    coords.push_back({x, y, z});
    std::sort(coords.begin(), coords.end(), [](const std::array<int, 3> &a, const std::array<int, 3> &b) {
        return morton(a[0], a[1], a[2]) < morton(b[0], b[1], b[2]);
    });
    v.nb = (int)coords.size();
    v.h_lattice_to_block.assign(v.h_map.size(), -1);
    v.h_bxyz.assign(3 * (size_t)(v.nb + 1), -1000000);
    for (int i = 0; i < v.nb; ++i) {
        const auto &c = coords[i];
        v.h_lattice_to_block[(size_t)v.block_slot(c[0], c[1], c[2])] = i;
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
                const int64_t slot = v.block_slot(x, y, z);
                if (x < 0 || y < 0 || z < 0 || x >= v.nbx || y >= v.nby || z >= v.nbz || slot < 0)
                    val = v.nb;
                else {
                    const int bi = v.h_lattice_to_block[(size_t)slot];
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

namespace {

// Refinement rule, computed on block lattices.  A level-(l-1) block that
// exists is refined when a branch axis segment meets its box grown by
// R + band[l] on every side, or when its box overlaps the wake box.
struct RefineRule {
    const lbm_branch *b;
    int n;
    const lbm_refine_desc *r;
    double tree_lo[3], tree_hi[3];

    RefineRule(const lbm_branch *b_, int n_, const lbm_refine_desc *r_) : b(b_), n(n_), r(r_)
    {
        for (int k = 0; k < 3; ++k) {
            tree_lo[k] = 1e300;
            tree_hi[k] = -1e300;
        }
        for (int i = 0; i < n; ++i) {
            const double rad = 0.5 * b[i].diameter;
            for (int k = 0; k < 3; ++k) {
                tree_lo[k] = std::min(tree_lo[k], std::min(b[i].p0[k], b[i].p1[k]) - rad);
                tree_hi[k] = std::max(tree_hi[k], std::max(b[i].p0[k], b[i].p1[k]) + rad);
            }
        }
    }

    // closed-box slab test of the axis segment of branch br against [lo, hi]
    static bool axis_hits(const lbm_branch &br, const double lo[3], const double hi[3])
    {
        double enter = 0.0, leave = 1.0;
        for (int k = 0; k < 3; ++k) {
            const double d = br.p1[k] - br.p0[k];
            if (d == 0.0) {
                if (br.p0[k] < lo[k] || br.p0[k] > hi[k])
                    return false;
                continue;
            }
            const double a = (lo[k] - br.p0[k]) / d, c = (hi[k] - br.p0[k]) / d;
            enter = std::max(enter, std::min(a, c));
            leave = std::min(leave, std::max(a, c));
            if (enter > leave)
                return false;
        }
        return true;
    }

    // block (bx, by, bz) of edge bf finest cells, refined towards level l?
    bool wants(int l, int bx, int by, int bz, double bf) const
    {
        for (int i = 0; i < n; ++i) {
            const double e = 0.5 * b[i].diameter + r->band[l];
            const double lo[3] = {bx * bf - e, by * bf - e, bz * bf - e};
            const double hi[3] = {(bx + 1) * bf + e, (by + 1) * bf + e, (bz + 1) * bf + e};
            if (axis_hits(b[i], lo, hi))
                return true;
        }
        if (r->wake[l] > 0) {
            const double lo[3] = {bx * bf, by * bf, bz * bf};
            const double w0[3] = {tree_lo[0], tree_lo[1] - r->band[l], tree_lo[2] - r->band[l]};
            const double w1[3] = {tree_hi[0] + r->wake[l], tree_hi[1] + r->band[l], tree_hi[2] + r->band[l]};
            for (int k = 0; k < 3; ++k)
                if (!(lo[k] < w1[k] && lo[k] + bf > w0[k]))
                    return false;
            return true;
        }
        return false;
    }
};

// Block map of one level over a stored box of its lattice (whole lattice
// NX x NY x NZ; stored box from o, extent n), grown on demand: finer levels
// store only the blocks around the refined region.
struct Lattice {
    int NX = 0, NY = 0, NZ = 0;
    int o[3] = {0, 0, 0}, n[3] = {0, 0, 0};
    std::vector<int8_t> m;  // 0 none, 1 leaf, 2 refined, 3 ghost storage
    int64_t slot(int x, int y, int z) const
    {
        x -= o[0];
        y -= o[1];
        z -= o[2];
        if ((unsigned)x >= (unsigned)n[0] || (unsigned)y >= (unsigned)n[1] || (unsigned)z >= (unsigned)n[2])
            return -1;
        return (int64_t)x + (int64_t)n[0] * ((int64_t)y + (int64_t)n[1] * z);
    }
    bool in_lattice(int x, int y, int z) const { return x >= 0 && y >= 0 && z >= 0 && x < NX && y < NY && z < NZ; }
    // -1 outside the lattice, 0 for blocks outside the stored box
    int8_t get(int x, int y, int z) const
    {
        if (!in_lattice(x, y, z))
            return -1;
        const int64_t s = slot(x, y, z);
        return s < 0 ? (int8_t)0 : m[(size_t)s];
    }
    // (x, y, z) must lie in the lattice; the stored box grows to hold it
    int8_t &at(int x, int y, int z)
    {
        int64_t s = slot(x, y, z);
        if (s < 0) {
            const int lo[3] = {x, y, z}, hi[3] = {x, y, z};
            reshape(lo, hi, 8);
            s = slot(x, y, z);
        }
        return m[(size_t)s];
    }
    // stored box = the current one joined with [lo, hi] grown by margin,
    // clipped to the lattice; entries keep their values
    void reshape(const int lo_in[3], const int hi_in[3], int margin)
    {
        const int N[3] = {NX, NY, NZ};
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::max(0, lo_in[a] - margin);
            hi[a] = std::min(N[a] - 1, hi_in[a] + margin);
            if (n[a] > 0) {
                lo[a] = std::min(lo[a], o[a]);
                hi[a] = std::max(hi[a], o[a] + n[a] - 1);
            }
        }
        Lattice t;
        t.NX = NX;
        t.NY = NY;
        t.NZ = NZ;
        for (int a = 0; a < 3; ++a) {
            t.o[a] = lo[a];
            t.n[a] = hi[a] - lo[a] + 1;
        }
        t.m.assign((size_t)t.n[0] * t.n[1] * t.n[2], 0);
        for (int z = 0; z < n[2]; ++z)
            for (int y = 0; y < n[1]; ++y)
                for (int x = 0; x < n[0]; ++x)
                    t.m[(size_t)t.slot(o[0] + x, o[1] + y, o[2] + z)] =
                        m[(size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z)];
        *this = std::move(t);
    }
    // stored box = the blocks present grown by margin (clipped)
    void fit(int margin)
    {
        int lo[3] = {NX, NY, NZ}, hi[3] = {-1, -1, -1};
        for (int z = 0; z < n[2]; ++z)
            for (int y = 0; y < n[1]; ++y)
                for (int x = 0; x < n[0]; ++x)
                    if (m[(size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z)] != 0) {
                        const int c[3] = {o[0] + x, o[1] + y, o[2] + z};
                        for (int a = 0; a < 3; ++a) {
                            lo[a] = std::min(lo[a], c[a]);
                            hi[a] = std::max(hi[a], c[a]);
                        }
                    }
        if (hi[0] < 0)
            return;
        Lattice t;
        t.NX = NX;
        t.NY = NY;
        t.NZ = NZ;
        t.reshape(lo, hi, margin);
        for (int z = 0; z < n[2]; ++z)
            for (int y = 0; y < n[1]; ++y)
                for (int x = 0; x < n[0]; ++x) {
                    const int8_t v = m[(size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z)];
                    if (v != 0)
                        t.m[(size_t)t.slot(o[0] + x, o[1] + y, o[2] + z)] = v;
                }
        *this = std::move(t);
    }
};

// refine (bx,by,bz) at level l, bringing it (and its ancestors) into existence
bool make_refined(std::vector<Lattice> &lat, int l, int bx, int by, int bz)
{
    if (lat[l].get(bx, by, bz) < 0)
        return false;
    if (lat[l].at(bx, by, bz) == 0) {
        if (l == 0 || !make_refined(lat, l - 1, bx >> 1, by >> 1, bz >> 1))
            return false;
    }
    lat[l].at(bx, by, bz) = 2;
    for (int s = 0; s < 8; ++s) {
        int8_t &c = lat[l + 1].at(2 * bx + (s & 1), 2 * by + ((s >> 1) & 1), 2 * bz + (s >> 2));
        if (c == 0)
            c = 1;
    }
    return true;
}

}  // namespace

lbm_status build_levels(const lbm_grid_desc &d, int B, int L, const lbm_branch *b, int n_b,
                        const lbm_refine_desc *refine, const SolidMask &solid,
                        std::vector<DevLevel> &lv, AmrPlan &plan, std::string *msg)
{
    plan.pairs.clear();
    lv.assign(L, DevLevel{});
    for (int l = 0; l < L; ++l) {
        DevLevel &v = lv[l];
        const int h = 1 << (L - 1 - l);
        v.level = l;
        v.dense = l == 0;
        v.nx = d.nx / h;
        v.ny = d.ny / h;
        v.nz = d.nz / h;
        v.nbx = v.nx / B;
        v.nby = v.ny / B;
        v.nbz = v.nz / B;
    }
    if (L == 1) {
        DevLevel &v = lv[0];
        v.h_map.assign((size_t)v.nbx * v.nby * v.nbz, 1);
        v.box_n[0] = v.nbx;
        v.box_n[1] = v.nby;
        v.box_n[2] = v.nbz;
        v.leaf_cells = (int64_t)d.nx * d.ny * d.nz;
        dense_tiles(v, [&](int64_t c) { return !solid.cell(c); }, v.h_work, &v.updated_cells);
        v.collided_cells = v.updated_cells;
        v.h_leaf = v.h_work;
        return LBM_OK;
    }

    // ---- block maps ----------------------------------------------------------
    // level 0 stores its whole lattice; finer levels store a box around their
    // blocks that grows as blocks appear
    std::vector<Lattice> lat(L);
    for (int l = 0; l < L; ++l) {
        lat[l].NX = lv[l].nbx;
        lat[l].NY = lv[l].nby;
        lat[l].NZ = lv[l].nbz;
    }
    {
        const int lo[3] = {0, 0, 0}, hi[3] = {lv[0].nbx - 1, lv[0].nby - 1, lv[0].nbz - 1};
        lat[0].reshape(lo, hi, 0);
        std::fill(lat[0].m.begin(), lat[0].m.end(), (int8_t)1);
    }
    RefineRule rule(b, n_b, refine);
    for (int l = 1; l < L; ++l) {
        Lattice &P = lat[l - 1];
        const double bf = (double)B * (double)(1 << (L - l));
        const int o[3] = {P.o[0], P.o[1], P.o[2]}, e[3] = {P.n[0], P.n[1], P.n[2]};
        for (int z = o[2]; z < o[2] + e[2]; ++z)
            for (int y = o[1]; y < o[1] + e[1]; ++y)
                for (int x = o[0]; x < o[0] + e[0]; ++x)
                    if (P.get(x, y, z) > 0 && rule.wants(l, x, y, z, bf)) {
                        P.at(x, y, z) = 2;
                        for (int s = 0; s < 8; ++s)
                            lat[l].at(2 * x + (s & 1), 2 * y + ((s >> 1) & 1), 2 * z + (s >> 2)) = 1;
                    }
    }
    for (bool changed = true; changed;) {
        changed = false;
        for (int l = L - 2; l >= 1; --l) {
            Lattice &T = lat[l];
            const int o[3] = {T.o[0], T.o[1], T.o[2]}, e[3] = {T.n[0], T.n[1], T.n[2]};
            for (int z = o[2]; z < o[2] + e[2]; ++z)
                for (int y = o[1]; y < o[1] + e[1]; ++y)
                    for (int x = o[0]; x < o[0] + e[0]; ++x) {
                        if (T.get(x, y, z) != 2)
                            continue;
                        for (int k = 0; k < 27; ++k) {
                            const int X = x + k % 3 - 1, Y = y + (k / 3) % 3 - 1, Z = z + k / 9 - 1;
                            const int8_t v = T.get(X, Y, Z);
                            if (v < 0) {
                                *msg = "a refined region reaches the box faces";
                                return LBM_E_INVALID;
                            }
                            if (v == 0) {
                                if (!make_refined(lat, l - 1, X >> 1, Y >> 1, Z >> 1)) {
                                    *msg = "refinement closure failed";
                                    return LBM_E_INVALID;
                                }
                                changed = true;
                            }
                        }
                    }
        }
    }
    for (int l = 0; l < L - 1; ++l) {
        const Lattice &T = lat[l];
        for (int z = T.o[2]; z < T.o[2] + T.n[2]; ++z)
            for (int y = T.o[1]; y < T.o[1] + T.n[1]; ++y)
                for (int x = T.o[0]; x < T.o[0] + T.n[0]; ++x)
                    if (T.get(x, y, z) == 2 &&
                        (x < 1 || y < 1 || z < 1 || x > T.NX - 2 || y > T.NY - 2 || z > T.NZ - 2)) {
                        *msg = "a refined region comes within one block of the box faces";
                        return LBM_E_INVALID;
                    }
    }
    for (int l = 1; l < L; ++l) {
        Lattice &T = lat[l];
        T.fit(1);  // room for the ghost-storage blocks around the present ones
        std::vector<int8_t> add(T.m.size(), 0);
        for (int z = T.o[2]; z < T.o[2] + T.n[2]; ++z)
            for (int y = T.o[1]; y < T.o[1] + T.n[1]; ++y)
                for (int x = T.o[0]; x < T.o[0] + T.n[0]; ++x) {
                    if (T.get(x, y, z) != 0)
                        continue;
                    for (int k = 0; k < 27; ++k) {
                        const int8_t v = T.get(x + k % 3 - 1, y + (k / 3) % 3 - 1, z + k / 9 - 1);
                        if (v == 1 || v == 2) {
                            add[(size_t)T.slot(x, y, z)] = 1;
                            break;
                        }
                    }
                }
        for (size_t i = 0; i < T.m.size(); ++i)
            if (add[i])
                T.m[i] = 3;
    }
    for (int l = 0; l < L; ++l) {
        lv[l].h_map = lat[l].m;
        for (int a = 0; a < 3; ++a) {
            lv[l].box_o[a] = lat[l].o[a];
            lv[l].box_n[a] = lat[l].n[a];
        }
        if (l > 0)
            index_level(lv[l], l);
    }

    // ---- cell classes ------------------------------------------------------
    // 1 active, 2 band (refined, <= 2 cells from active), 3 deep, 4 ghost, 0 none
    auto block_of = [&](int l, int x, int y, int z) -> int8_t {
        if (x < 0 || y < 0 || z < 0 || x >= lv[l].nx || y >= lv[l].ny || z >= lv[l].nz)
            return -1;
        return lat[l].get(x / B, y / B, z / B);
    };
    // the kinds of the blocks that the cell window [x - r, x + r]^3 meets
    // (every block of that range holds a cell of the window): 1 when one of
    // them is a leaf (or, with refined_too, refined)
    auto fdiv = [&](int v) { return v >= 0 ? v / B : -((-v + B - 1) / B); };
    auto window_meets = [&](int l, int x, int y, int z, int r, bool refined_too) -> bool {
        const int x0 = fdiv(x - r), x1 = fdiv(x + r), y0 = fdiv(y - r), y1 = fdiv(y + r);
        const int z0 = fdiv(z - r), z1 = fdiv(z + r);
        for (int bz = z0; bz <= z1; ++bz)
            for (int by = y0; by <= y1; ++by)
                for (int bx = x0; bx <= x1; ++bx) {
                    const int8_t v = lat[l].get(bx, by, bz);
                    if (v == 1 || (refined_too && v == 2))
                        return true;
                }
        return false;
    };
    auto cell_class = [&](int l, int x, int y, int z) -> int {
        const int8_t m = block_of(l, x, y, z);
        if (m == 1)
            return 1;
        if (m == 2)  // band: a leaf cell within Chebyshev distance 2
            return window_meets(l, x, y, z, 2, false) ? 2 : 3;
        if (m == 3)  // ghost: a leaf or refined cell among the 26 neighbours
            return window_meets(l, x, y, z, 1, true) ? 4 : 0;
        return 0;
    };
    const int cells = B * B * B;
    auto finest_solid = [&](int x, int y, int z) { return solid(x, y, z); };
    for (int l = 0; l < L; ++l) {
        DevLevel &v = lv[l];
        const bool finest = l == L - 1;
        v.leaf_cells = 0;
        v.updated_cells = 0;
        v.collided_cells = 0;
        if (v.dense) {
            // level 0: collide active and band cells; leaf = active
            std::vector<uint8_t> cls((size_t)v.nx * v.ny * v.nz);
            for (int z = 0; z < v.nz; ++z)
                for (int y = 0; y < v.ny; ++y)
                    for (int x = 0; x < v.nx; ++x)
                        cls[(size_t)x + (size_t)v.nx * ((size_t)y + (size_t)v.ny * z)] = (uint8_t)cell_class(l, x, y, z);
            dense_tiles(v, [&](int64_t c) { return cls[c] == 1 || cls[c] == 2; }, v.h_work, &v.collided_cells);
            dense_tiles(v, [&](int64_t c) { return cls[c] == 1; }, v.h_leaf, &v.updated_cells);
            v.leaf_cells = v.updated_cells;
            continue;
        }
        for (int bi = 0; bi < v.nb; ++bi) {
            const int bx = v.h_bxyz[3 * bi], by = v.h_bxyz[3 * bi + 1], bz = v.h_bxyz[3 * bi + 2];
            std::vector<uint32_t> mw(cells / 32, 0u), ml(cells / 32, 0u);
            int nw = 0, nl = 0;
            for (int c = 0; c < cells; ++c) {
                const int x = bx * B + c % B, y = by * B + (c / B) % B, z = bz * B + c / (B * B);
                const int k = cell_class(l, x, y, z);
                const bool sol = finest && (k == 1 || k == 2) && finest_solid(x, y, z);
                if (k == 1 || k == 2)
                    v.leaf_cells += k == 1;
                // ghost cells (4) are collided by the prolongation itself
                if ((k == 1 || k == 2) && !sol) {
                    mw[c >> 5] |= 1u << (c & 31);
                    ++nw;
                }
                if (k == 1 && !sol) {
                    ml[c >> 5] |= 1u << (c & 31);
                    ++nl;
                }
            }
            v.updated_cells += nl;
            v.collided_cells += nw;
            auto push = [&](std::vector<uint2> &list, const std::vector<uint32_t> &m, int cnt) {
                if (cnt == 0)
                    return;
                uint32_t mid = FULL_MASK;
                if (cnt != cells) {
                    mid = (uint32_t)(v.h_masks.size() / (cells / 32));
                    v.h_masks.insert(v.h_masks.end(), m.begin(), m.end());
                }
                list.push_back(make_uint2((unsigned)bi, mid));
            };
            push(v.h_work, mw, nw);
            push(v.h_leaf, ml, nl);
        }
        // The odd step reads one element of the next block's row at each x
        // face.  Running blocks that share an x face close together lets the
        // L2 serve that line to both; the even step keeps memory order.
        v.h_work_odd = v.h_work;
        std::stable_sort(v.h_work_odd.begin(), v.h_work_odd.end(), [&](const uint2 &p, const uint2 &q) {
            const int *u = &v.h_bxyz[3 * (size_t)p.x], *w = &v.h_bxyz[3 * (size_t)q.x];
            if (u[2] != w[2]) return u[2] < w[2];
            if (u[1] != w[1]) return u[1] < w[1];
            return u[0] < w[0];
        });
    }

    // ---- coarse/fine plans -------------------------------------------------
    plan.pairs.resize(L - 1);
    for (int l = 0; l < L - 1; ++l) {
        AmrPair &pr = plan.pairs[l];
        const DevLevel &C = lv[l], &F = lv[l + 1];
        std::unordered_map<uint32_t, int32_t> src_index;
        bool bad = false;
        auto addr_of = [&](const DevLevel &v, int x, int y, int z) -> uint32_t {
            const int64_t e = level_cell_address(v, B, x, y, z);
            if (e < 0)
                bad = true;
            return (uint32_t)std::max<int64_t>(e, 0);
        };
        // prolongation sources hold the coarse level's pre-collision state:
        // active or band cells, never ghosts (which hold post-collision data)
        bool bad_src = false;
        auto src_of = [&](int x, int y, int z) -> int32_t {
            const int k = cell_class(l, x, y, z);
            if (k != 1 && k != 2)
                bad_src = true;
            const uint32_t e = addr_of(C, x, y, z);
            auto it = src_index.find(e);
            if (it != src_index.end())
                return it->second;
            const int32_t id = (int32_t)pr.h_src.size();
            src_index.emplace(e, id);
            pr.h_src.push_back(e);
            return id;
        };
        // fine ghost cells, in block order
        for (int bi = 0; bi < F.nb; ++bi) {
            if (lat[l + 1].get(F.h_bxyz[3 * bi], F.h_bxyz[3 * bi + 1], F.h_bxyz[3 * bi + 2]) != 3)
                continue;
            const int bx = F.h_bxyz[3 * bi], by = F.h_bxyz[3 * bi + 1], bz = F.h_bxyz[3 * bi + 2];
            for (int c = 0; c < cells; ++c) {
                const int x = bx * B + c % B, y = by * B + (c / B) % B, z = bz * B + c / (B * B);
                if (cell_class(l + 1, x, y, z) != 4)
                    continue;
                pr.h_ghost.push_back((uint32_t)bi * cells + c);
                uint32_t gm = 0;
                for (int k = 0; k < 27; ++k) {
                    const int t = cell_class(l + 1, x + k % 3 - 1, y + (k / 3) % 3 - 1, z + k / 9 - 1);
                    if (t == 1 || t == 2)
                        gm |= 1u << k;
                }
                pr.h_ghost_mask.push_back(gm);
                const int P[3] = {x >> 1, y >> 1, z >> 1};
                const int s[3] = {(x & 1) ? 1 : -1, (y & 1) ? 1 : -1, (z & 1) ? 1 : -1};
                for (int q = 0; q < 8; ++q)
                    pr.h_ghost_src.push_back(src_of(P[0] + (q & 1) * s[0], P[1] + ((q >> 1) & 1) * s[1],
                                                    P[2] + ((q >> 2) & 1) * s[2]));
            }
        }
        // source cells in address order (coalesced moment loads); the ghost
        // stencils follow the renumbering
        {
            std::vector<int32_t> order(pr.h_src.size()), rank(pr.h_src.size());
            for (size_t i = 0; i < order.size(); ++i)
                order[i] = (int32_t)i;
            std::sort(order.begin(), order.end(),
                      [&](int32_t a, int32_t b) { return pr.h_src[a] < pr.h_src[b]; });
            std::vector<uint32_t> sorted(order.size());
            for (size_t i = 0; i < order.size(); ++i) {
                sorted[i] = pr.h_src[order[i]];
                rank[order[i]] = (int32_t)i;
            }
            pr.h_src.swap(sorted);
            for (int32_t &v : pr.h_ghost_src)
                v = rank[v];
        }
        // coarse band cells and their children
        auto band_cell = [&](int x, int y, int z) {
            pr.h_band.push_back(addr_of(C, x, y, z));
            for (int q = 0; q < 8; ++q) {
                const int fx = 2 * x + (q & 1), fy = 2 * y + ((q >> 1) & 1), fz = 2 * z + ((q >> 2) & 1);
                const bool sol = (l + 1 == L - 1) && finest_solid(fx, fy, fz);
                pr.h_band_child.push_back(sol ? FULL_MASK : addr_of(F, fx, fy, fz));
            }
        };
        for (int bz = C.box_o[2]; bz < C.box_o[2] + C.box_n[2]; ++bz)
            for (int by = C.box_o[1]; by < C.box_o[1] + C.box_n[1]; ++by)
                for (int bx = C.box_o[0]; bx < C.box_o[0] + C.box_n[0]; ++bx) {
                    if (lat[l].get(bx, by, bz) != 2)
                        continue;
                    for (int c = 0; c < cells; ++c) {
                        const int x = bx * B + c % B, y = by * B + (c / B) % B, z = bz * B + c / (B * B);
                        if (cell_class(l, x, y, z) == 2)
                            band_cell(x, y, z);
                    }
                }
        if (bad) {
            *msg = "internal: a coarse/fine stencil cell is not held by its level";
            return LBM_E_INVALID;
        }
        if (bad_src) {
            *msg = "internal: a prolongation source is not an active or band cell of the coarse level";
            return LBM_E_INVALID;
        }
    }
    return LBM_OK;
}

lbm_status amr_upload(AmrPlan &plan, std::vector<DevLevel> &lv, int B, const Alloc &alloc, hipStream_t s,
                      std::string *msg)
{
    (void)B;
    for (AmrPair &pr : plan.pairs) {
        auto put = [&](void **dst, const void *src, size_t bytes) -> lbm_status {
            lbm_status st = alloc(dst, std::max<size_t>(bytes, 16));
            if (st != LBM_OK)
                return st;
            if (bytes && hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) {
                *msg = "hipMemcpyAsync of the coupling plan failed";
                return LBM_E_DEVICE;
            }
            return LBM_OK;
        };
        lbm_status st;
        if ((st = put((void **)&pr.d_src, pr.h_src.data(), pr.h_src.size() * 4)) != LBM_OK ||
            (st = put((void **)&pr.d_ghost, pr.h_ghost.data(), pr.h_ghost.size() * 4)) != LBM_OK ||
            (st = put((void **)&pr.d_ghost_src, pr.h_ghost_src.data(), pr.h_ghost_src.size() * 4)) != LBM_OK ||
            (st = put((void **)&pr.d_ghost_mask, pr.h_ghost_mask.data(), pr.h_ghost_mask.size() * 4)) != LBM_OK ||
            (st = put((void **)&pr.d_band, pr.h_band.data(), pr.h_band.size() * 4)) != LBM_OK ||
            (st = put((void **)&pr.d_band_child, pr.h_band_child.data(), pr.h_band_child.size() * 4)) != LBM_OK)
            return st;
        for (int k = 0; k < 2; ++k)
            if ((st = alloc((void **)&pr.d_mom[k], std::max<size_t>(pr.h_src.size() * MOM_REC * sizeof(float), 16))) != LBM_OK)
                return st;
        {
            const size_t li = (size_t)(&pr - plan.pairs.data());
            std::vector<int32_t> idx(lv[li].dir_elems, -1);
            for (size_t i = 0; i < pr.h_src.size(); ++i)
                idx[pr.h_src[i]] = (int32_t)i;
            if ((st = put((void **)&pr.d_mom_idx, idx.data(), idx.size() * 4)) != LBM_OK)
                return st;
            // the staging vector dies here: the copy must finish first
            if (hipStreamSynchronize(s) != hipSuccess) {
                *msg = "hipStreamSynchronize after the source map upload failed";
                return LBM_E_DEVICE;
            }
        }
    }
    return LBM_OK;
}

}  // namespace lbm
