// Internal structures shared by the host runtime and the HIP kernels of
// liblbmtree.so.  Not part of the public ABI.
#pragma once
#include <algorithm>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace lbm {

// neighbour-table codes for block offsets that leave the box at level 0
constexpr int NB_INLET = -2;   // x < 0: equilibrium ghost plane
constexpr int NB_OUTLET = -3;  // x >= nx: zero-gradient ghost plane
constexpr uint32_t FULL_MASK = 0xFFFFFFFFu;
// force samples kept on the device (ring of total-force triples)
constexpr int RING = 65536;
// coarse/fine transfer record of one source cell: drho, ux, uy, uz, D (6), two pad floats
constexpr int MOM_REC = 12;
// coarse band cells per work-group item of the restriction in the persistent
// launch (one per thread of its 256-thread work-groups)
constexpr int RESTRICT_CELLS = 256;
// links per piece of the force reduction (one work-group each)
constexpr int LINK_PIECE = 8192;
// seconds after which one wait of the persistent launch gives up (a phase of
// the largest grids takes milliseconds)
constexpr double PERSIST_WAIT_S = 1.0;

// Arguments of the collide-and-stream kernel of one level.
constexpr int DENSE_TILE = 256;  // cells per work item of a dense level
// spare elements after a dense level's cells in every direction array: the
// odd step's populations that leave through a face land at row index mod
// DENSE_SINK, so concurrent rows write different elements
constexpr int DENSE_SINK = 4096;
constexpr size_t DENSE_ALIGN = (size_t)1 << 19;  // elements

struct CollideArgs {
    void *pop[27];            // per-direction arrays (storage type)
    const int *nbr;           // 27 neighbour block ids per block
    const int *bxyz;          // block coordinates (3 per block)
    const uint2 *work;        // (block, mask id or FULL_MASK)
    const uint32_t *masks;    // B^3/32 words per masked block
    int n_work;
    int parts;                // work-groups per block (block layout)
    int xcd_group;            // consecutive tiles per XCD run (1 = plain order)
    int dense;                // 1: level stored as x-pencils over its whole box
    int nx;                   // level box along x (cells)
    float om1, om2;
    int galilean;
    int faces;                // 1: this level owns the inlet/outlet planes
    int lateral;              // 1: its y and z faces are inflow faces (ghosts f_eq(1, u_in e_x)); 0: periodic
    int nbx;                  // blocks along x (face detection)
    int ny, nz;               // level box (transverse) in cells
    float u_in;
    const float *in_prev;     // inlet fluctuation plane used at t-1 (3*ny*nz) or null
    const float *in_cur;      // inlet fluctuation plane used at t, or null
    float *gbuf;              // outlet ghost copies, 27*ny*nz
    // coarse/fine transfer records of the level's prolongation sources, taken
    // from the pre-collision state inside the collide launch: mom_idx[cell] is
    // the source index (or -1), the record goes to mom_out[MOM_REC * index];
    // mom_idx null: no records
    const int32_t *mom_idx;
    float *mom_out;
    float mom_dt;             // level step in finest time units
};

// Arguments of the interpolated bounce-back kernel (finest level).
struct LinkArgs {
    char *pop;                // base of the direction arrays
    size_t dir_bytes;         // bytes per direction array
    const uint32_t *af, *ap, *am;  // cell addresses of x_f, x_f + c_j, x_f - c_j
    const uint8_t *dir;       // j | 0x80 when x_f - c_j is fluid
    const float *q;
    int n;
    float *lforce;            // 3 per link when sampling, else null
};

// Arguments of the wall-friction kernel (finest level): one surface element
// per axis face between a fluid cell and a solid neighbour.
struct FricArgs {
    const uint32_t *a0;       // element address of the fluid cell x_f
    const uint32_t *a1;       // element address of x_f - e_k (FRIC_NO_UP: none)
    const float *q;           // wall distance along e_k
    const float4 *nw;         // outward body normal at the wall point (x, y, z) and the weight |n_k|
    int n;
    float om1;                // shear rate of the finest level
    float *force;             // 3 per element: the element's friction force
};
constexpr uint32_t FRIC_NO_UP = 0xFFFFFFFFu;

// One phase of a coarse step run as a single persistent launch: the work
// items of what would otherwise be one kernel launch, followed by a grid-wide
// barrier.  The host records the phases in the order the per-phase launches
// would run, so both forms execute the same bodies in the same order.
enum PhaseKind : int {
    PH_COLLIDE = 0,       // a; items = collide work items (dense tiles or block tiles)
    PH_LINKS = 1,         // la, odd = parity just completed; items = ceil(la.n / 256)
    PH_BRANCH_SUM = 2,    // items = nseg
    PH_BRANCH_TOTAL = 3,  // items = 1
    PH_AMR_MOMENTS = 4,   // a = coarse level, cells = sources; items = ceil(n / 256)
    PH_AMR_PROLONG = 5,   // a = fine level, cells = ghosts, src = stencils
    PH_AMR_RESTRICT = 6,  // a = coarse, b = fine, cells = band, child = children
};

struct Phase {
    int kind;
    int odd, odd2;            // A-A parity (restriction: coarse, fine)
    int rowwave;              // dense odd collide: row-per-wave variant
    int items;                // work items (one work-group each)
    int chunk, chunks;        // items per claim, number of claims
    int n, nsrc;
    float om1, dt, om2, dt2;
    CollideArgs a, b;
    LinkArgs la;
    const uint32_t *cells;
    const int32_t *src;
    const uint32_t *gmask;  // prolongation: stored directions per ghost
    const uint32_t *child;
    const float *m0, *m1;
    float *out;
    const float *lforce;
    const int *pstart, *segp;
    int npieces, nseg;
    double *piece_sum;
    double *sample, *acc_branch, *acc_total, *ring;
    unsigned long long *ring_pos;
};

// launcher of the persistent coarse step (lbm_persist.hip).  ctr: 2 n_phases
// + 1 counters, zero before the first launch (each launch leaves them zero);
// abort_flag: set by the launch when a wait gave up after wait_ticks of the
// device's constant real-time counter.  Any grid size is correct;
// persistent_max_grid gives the number of resident work-groups.
hipError_t launch_persistent(int B, int storage, const Phase *phases, int n_phases, unsigned *ctr,
                             unsigned *abort_flag, unsigned long long wait_ticks, int grid, hipStream_t s);
hipError_t persistent_max_grid(int B, int storage, int device, int *grid, int *cus);

struct DevLevel {
    int level;
    bool dense = false;       // x-pencil layout over the whole box (no blocks)
    int nb = 0;               // blocks (sink block has index nb)
    int nbx = 0, nby = 0, nbz = 0;
    int nx = 0, ny = 0, nz = 0;
    size_t dir_elems = 0;     // dense: nx*ny*nz; blocks: (nb+1) * B^3
    void *pop = nullptr;
    int *nbr = nullptr;
    int *bxyz = nullptr;
    uint2 *work = nullptr;    // collide work list (unit, mask id): dense tiles or blocks, in memory order
    uint2 *work_odd = nullptr;  // the same items for odd steps of a block level, x fastest (null: use work)
    int n_work = 0;
    uint2 *leaf = nullptr;    // leaf-cell work list (mass, fields)
    int n_leaf = 0;
    uint32_t *masks = nullptr;
    float *gbuf = nullptr;
    double om1 = 1.0;
    int64_t steps = 0;
    int64_t updated_cells = 0;   // leaf fluid cells (the updates a level sub-step counts)
    int64_t collided_cells = 0;  // cells collided per sub-step (leaf + band + ghost, solid excluded)
    int64_t leaf_cells = 0;
    // host mirrors.  The block map and the block index cover the stored block
    // box (first block box_o, extent box_n) of the level's lattice: the whole
    // lattice for level 0, the blocks around the refined region for finer
    // levels, so that a level's host tables scale with its blocks, not with
    // its box.
    int box_o[3] = {0, 0, 0}, box_n[3] = {0, 0, 0};
    std::vector<int> h_bxyz;          // 3 per block
    std::vector<int> h_nbr;           // 27 per block
    std::vector<int8_t> h_map;        // block map over the stored box (0 none, 1 leaf, 2 refined, 3 ghost)
    std::vector<int> h_lattice_to_block;  // over the stored box, -1 when absent
    std::vector<uint2> h_work, h_work_odd, h_leaf;
    std::vector<uint32_t> h_masks;

    // index of block (bx, by, bz) in the stored box, -1 outside it
    int64_t block_slot(int bx, int by, int bz) const
    {
        bx -= box_o[0];
        by -= box_o[1];
        bz -= box_o[2];
        if ((unsigned)bx >= (unsigned)box_n[0] || (unsigned)by >= (unsigned)box_n[1] || (unsigned)bz >= (unsigned)box_n[2])
            return -1;
        return (int64_t)bx + (int64_t)box_n[0] * ((int64_t)by + (int64_t)box_n[1] * bz);
    }
    // kind of block (bx, by, bz): 0 none (also outside the stored box)
    int8_t block_kind(int bx, int by, int bz) const
    {
        const int64_t s = block_slot(bx, by, bz);
        return s < 0 ? (int8_t)0 : h_map[(size_t)s];
    }
    // the block map over the whole lattice, x fastest (nbx * nby * nbz bytes)
    void expand_map(int8_t *dense) const
    {
        std::fill(dense, dense + (size_t)nbx * nby * nbz, (int8_t)0);
        for (int z = 0; z < box_n[2]; ++z)
            for (int y = 0; y < box_n[1]; ++y)
                for (int x = 0; x < box_n[0]; ++x)
                    dense[(size_t)(box_o[0] + x) + (size_t)nbx * ((size_t)(box_o[1] + y) + (size_t)nby * (box_o[2] + z))] =
                        h_map[(size_t)x + (size_t)box_n[0] * ((size_t)y + (size_t)box_n[1] * z)];
    }
};

// launchers (lbm_kernels.hip)
// lds_bytes: dynamic LDS reserved per work-group to cap the number of
// resident work-groups per CU (160 KiB of LDS per CU on gfx950)
hipError_t launch_collide(int B, int storage, int odd, const CollideArgs &a, int threads, int lds_bytes,
                          hipStream_t s);
constexpr int LDS_PER_CU = 160 * 1024;
// dynamic LDS that limits a 256-thread work-group kernel to occ waves per SIMD
inline int lds_for_occupancy(int occ) { return occ <= 0 ? 0 : LDS_PER_CU / occ - 1024; }
hipError_t launch_links(int storage, int odd_done, const LinkArgs &a, hipStream_t s);
hipError_t launch_init(int unit, int storage, void *pop, size_t dir_elems, const uint2 *work,
                       int n, const uint32_t *masks, float u_in, hipStream_t s);
hipError_t launch_fill_sink_and_all(int storage, void *pop, size_t dir_elems, hipStream_t s);
// force sums of one sample: link pieces (pstart, npieces + 1 offsets) summed by
// one work-group each, then per branch (pieces segp[s] .. segp[s + 1]) and in total
hipError_t launch_branch_reduce(const float *lforce, const int *pstart, int npieces, const int *segp, int nseg,
                                double *piece_sum, double *sample, double *acc_branch, double *acc_total,
                                double *ring, unsigned long long *ring_pos, unsigned *counter, hipStream_t s);
// friction force of every surface element from the level's pre-collision
// state for its next step (odd: that step's parity)
hipError_t launch_friction(int B, int storage, int odd, const CollideArgs &a, const FricArgs &f, hipStream_t s);
// element addresses (dense: x + nx (y + ny z); blocks: block * B^3 + local)
hipError_t launch_gather(int B, int storage, int odd, const CollideArgs &a, const uint32_t *cells,
                         int n, double *out_f, size_t out_stride, hipStream_t s);
hipError_t launch_scatter(int storage, void *pop, size_t dir_elems, const uint32_t *cells,
                          int n, const double *in_f, size_t in_stride, hipStream_t s);
hipError_t launch_mass(int B, int storage, int odd, const CollideArgs &a, const uint2 *leaf,
                       int n_leaf, double cell_volume, double *out4, hipStream_t s);

// coarse/fine transfer (lbm_amr_kernels.hip); moments are written SoA
// (10 arrays of n floats), stencils hold 8 source indices per ghost and
// 8 child addresses per band cell (FULL_MASK = skip)
hipError_t launch_amr_moments(int B, int storage, int odd, const CollideArgs &a, const uint32_t *cells, int n,
                              float om1, float dt, float *out, hipStream_t s);
hipError_t launch_amr_prolong(int B, int storage, int odd, const CollideArgs &fine, const uint32_t *ghosts,
                              const uint32_t *gmask, const int32_t *src, int n, int nsrc, const float *m0, const float *m1, float om1,
                              float dt, hipStream_t s);
hipError_t launch_amr_restrict(int B, int storage, int odd_c, int odd_f, const CollideArgs &coarse,
                               const CollideArgs &fine, const uint32_t *band, const uint32_t *child, int n,
                               float om_c, float dt_c, float om_f, float dt_f, hipStream_t s);

}  // namespace lbm
