// Host runtime and C ABI of liblbmtree (declared in include/lbmtree.h).
//
// Owns the grid description, the finest-level geometry (solid mask, links),
// the block grid of every level, the device buffers and the step schedule.
// Every device operation runs on the grid's stream; synchronising calls
// (drag, state access) wait on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/lbmtree.h"
#include "lbm_geometry.h"
#include "lbm_internal.h"
#include "lbm_levels.h"
#include "lbm_grid.h"
#include "lbm_inflow.h"
#include "lbm_persist_protocol.h"

using namespace lbm;

static thread_local std::string g_thread_error;


static lbm_status fail(lbm_grid *g, lbm_status st, const std::string &msg)
{
    if (g)
        g->err = msg;
    else
        g_thread_error = msg;
    return st;
}

#define HIPX(g, call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((g), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
static lbm_status dalloc(lbm_grid *g, T **p, size_t count)
{
    void *q = nullptr;
    if (count == 0)
        count = 1;
    const hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess)
        return fail(g, LBM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    g->allocs.push_back(q);
    g->device_bytes += count * sizeof(T);
    *p = (T *)q;
    return LBM_OK;
}

template <typename T>
static lbm_status upload(lbm_grid *g, T **p, const std::vector<T> &h)
{
    lbm_status st = dalloc(g, p, h.size());
    if (st != LBM_OK)
        return st;
    if (!h.empty())
        HIPX(g, hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, g->stream));
    return LBM_OK;
}

static size_t storage_bytes(int storage) { return storage == LBM_FP32 ? 4 : 2; }

// Elements per direction array of a level.  A dense level's arrays end in
// DENSE_SINK spare elements, where the odd step stores the populations that
// leave through the box faces.  The distance between the direction arrays
// changes how the 27 streams of a step spread over the HBM channels; measured
// on the uniform 512x256x256 grid, FP32 runs fastest with a power-of-two
// distance and FP16/BF16 with a multiple of DENSE_ALIGN elements.
static size_t level_dir_elems(const DevLevel &v, int B, int storage)
{
    if (!v.dense)
        return (size_t)(v.nb + 1) * B * B * B;
    const size_t need = (size_t)v.nx * v.ny * v.nz + DENSE_SINK;
    size_t p2 = 1;
    while (p2 < need)
        p2 <<= 1;
    if (storage == 0 && p2 <= (size_t)UINT32_MAX / 2)
        return p2;
    return (need + DENSE_ALIGN - 1) / DENSE_ALIGN * DENSE_ALIGN;
}

// bytes one level's populations take in bound memory (256-byte aligned)
static size_t bound_share(size_t bytes) { return (bytes + 255) / 256 * 256; }

static int nu_to_level_omega(double nu_f, int L, int l, double *om)
{
    const double nu = nu_f / double(1 << (L - 1 - l));
    *om = 1.0 / (3.0 * nu + 0.5);
    return 0;
}

// kernel arguments of level l for the current state
static CollideArgs collide_args(lbm_grid *g, int l)
{
    DevLevel &v = g->lv[l];
    CollideArgs a{};
    const size_t eb = storage_bytes(g->d.storage);
    for (int k = 0; k < 27; ++k)
        a.pop[k] = (char *)v.pop + (size_t)k * v.dir_elems * eb;
    a.nbr = v.nbr;
    a.bxyz = v.bxyz;
    a.work = v.work;
    a.masks = v.masks;
    a.n_work = v.n_work;
    a.dense = v.dense ? 1 : 0;
    a.nx = v.nx;
    const int cells = g->B * g->B * g->B;
    a.parts = std::max(1, cells / std::max(1, g->tile));
    a.xcd_group = std::max(1, g->xcd_group);
    a.om1 = (float)v.om1;
    a.om2 = 1.0f;
    a.galilean = (g->d.flags & LBM_F_NO_GALILEAN) ? 0 : 1;
    a.faces = l == 0 ? 1 : 0;
    a.lateral = (l == 0 && g->d.periodic_yz == 0) ? 1 : 0;
    a.nbx = v.nbx;
    a.ny = v.ny;
    a.nz = v.nz;
    a.u_in = (float)g->d.u_in;
    a.in_prev = (l == 0 && g->turb) ? g->d_in_prev : nullptr;
    a.in_cur = (l == 0 && g->turb) ? g->d_in_cur : nullptr;
    a.gbuf = v.gbuf;
    return a;
}

static LinkArgs link_args(lbm_grid *g, bool sample)
{
    DevLevel &v = g->lv[g->L - 1];
    LinkArgs a{};
    a.pop = (char *)v.pop;
    a.dir_bytes = v.dir_elems * storage_bytes(g->d.storage);
    a.af = g->d_af;
    a.ap = g->d_ap;
    a.am = g->d_am;
    a.dir = g->d_dir;
    a.q = g->d_q;
    a.n = g->n_links;
    a.lforce = sample ? g->d_lforce : nullptr;
    return a;
}

// ---------------------------------------------------------------------------
// step schedule
// ---------------------------------------------------------------------------

static int timing_mark(lbm_grid *g)
{
    if (!g->timing)
        return -1;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess)
        return -1;
    g->ev_pool.push_back(e);
    (void)hipEventRecord(e, g->stream);
    return (int)g->ev_pool.size() - 1;
}

static Phase new_phase(PhaseKind k)
{
    Phase p;
    std::memset(&p, 0, sizeof p);
    p.kind = k;
    return p;
}

// inlet planes of the coming odd level-0 step (times 2m and 2m + 1, m = tick)
static lbm_status inflow_planes(lbm_grid *g)
{
    const double d0 = (double)(1 << (g->L - 1));
    const DevLevel &v = g->lv[0];
    HIPX(g, launch_inflow(g->d_modes, g->n_modes, g->d_tick, g->d.u_in, d0, d0, v.ny, v.nz, g->d_in_prev,
                          g->d_in_cur, g->stream));
    return LBM_OK;
}

// level step in finest time units
static float level_dt(const lbm_grid *g, int l) { return (float)(1 << (g->L - 1 - l)); }

// One step of level l.  A level with a finer neighbour also writes the
// transfer records of its prolongation sources at time T from the
// pre-collision state it reads anyway (records slot 0).
static lbm_status level_collide(lbm_grid *g, int l)
{
    DevLevel &v = g->lv[l];
    const int odd = (int)(v.steps & 1);
    CollideArgs a = collide_args(g, l);
    if (odd && v.work_odd)
        a.work = v.work_odd;
    if (l < g->L - 1) {
        AmrPair &pr = g->amr.pairs[l];
        a.mom_idx = pr.d_mom_idx;
        a.mom_out = pr.d_mom[0];
        a.mom_dt = level_dt(g, l);
    }
    const bool inflow = l == 0 && g->turb && odd;
    if (g->rec && inflow)
        return fail(g, LBM_E_INVALID, "turbulent inflow is not available in the persistent form");
    if (g->rec) {
        Phase p = new_phase(PH_COLLIDE);
        p.odd = odd;
        p.a = a;
        p.rowwave = a.dense && a.nx % 64 == 0;
        p.items = a.dense ? a.n_work : a.n_work * a.parts;
        if (p.items > 0)
            g->rec->push_back(p);
        return LBM_OK;
    }
    if (inflow) {
        lbm_status st = inflow_planes(g);
        if (st != LBM_OK)
            return st;
    }
    const int e0 = timing_mark(g);
    HIPX(g, launch_collide(g->B, g->d.storage, odd, a, g->threads,
                           lds_for_occupancy(odd ? g->occ_odd : g->occ_even), g->stream));
    const int e1 = timing_mark(g);
    if (e0 >= 0 && e1 >= 0)
        g->ev_pairs.push_back({e0, 0});
    if (inflow)
        HIPX(g, launch_tick(g->d_tick, g->stream));
    return LBM_OK;
}

static lbm_status finest_links(lbm_grid *g, int odd_done)
{
    const bool sample = (g->finest_steps % g->d.drag_every) == 0;
    if (g->n_links > 0) {
        LinkArgs a = link_args(g, sample);
        if (g->rec) {
            Phase p = new_phase(PH_LINKS);
            p.odd = odd_done;
            p.la = a;
            p.items = (a.n + 255) / 256;
            g->rec->push_back(p);
        } else {
            const int e0 = timing_mark(g);
            HIPX(g, launch_links(g->d.storage, odd_done, a, g->stream));
            const int e1 = timing_mark(g);
            if (e0 >= 0 && e1 >= 0)
                g->ev_pairs.push_back({e0, 1});
        }
    }
    if (sample) {
        // the device ring position advances exactly when the reduction runs
        if (g->n_links > 0 && g->npieces > 0) {
            if (g->rec) {
                Phase p = new_phase(PH_BRANCH_SUM);
                p.lforce = g->d_lforce;
                p.pstart = g->d_pstart;
                p.npieces = g->npieces;
                p.piece_sum = g->d_piece_sum;
                p.items = g->npieces;
                g->rec->push_back(p);
                Phase t = new_phase(PH_BRANCH_TOTAL);
                t.piece_sum = g->d_piece_sum;
                t.segp = g->d_segp;
                t.nseg = g->nseg;
                t.sample = g->d_sample;
                t.acc_branch = g->d_acc_branch;
                t.acc_total = g->d_acc_total;
                t.ring = g->d_ring;
                t.ring_pos = g->d_ring_pos;
                t.items = 1;
                g->rec->push_back(t);
            } else {
                HIPX(g, launch_branch_reduce(g->d_lforce, g->d_pstart, g->npieces, g->d_segp, g->nseg,
                                             g->d_piece_sum, g->d_sample, g->d_acc_branch, g->d_acc_total,
                                             g->d_ring, g->d_ring_pos, g->d_counter, g->stream));
            }
            g->ring_count++;
        }
        if (g->n_fric > 0) {
            // wall friction from the state the links just completed: the
            // pre-collision populations of the finest level's next step
            if (g->rec)
                return fail(g, LBM_E_INVALID, "wall friction is not available in the persistent form");
            const int L1 = g->L - 1;
            FricArgs f{};
            f.a0 = g->d_fa0;
            f.a1 = g->d_fa1;
            f.q = g->d_fq;
            f.nw = g->d_fnw;
            f.n = g->n_fric;
            f.om1 = (float)g->lv[L1].om1;
            f.force = g->d_fforce;
            HIPX(g, launch_friction(g->B, g->d.storage, (int)(g->lv[L1].steps & 1), collide_args(g, L1), f,
                                    g->stream));
            HIPX(g, launch_branch_reduce(g->d_fforce, g->d_fpstart, g->fric_npieces, g->d_fsegp, g->nseg,
                                         g->d_fpiece_sum, nullptr, g->d_facc_branch, g->d_facc_total, nullptr,
                                         nullptr, g->d_fcounter, g->stream));
        }
        g->samples++;
    }
    return LBM_OK;
}

// Surface elements of the wall friction: every axis face between a fluid cell
// x_f and a solid neighbour x_f + e_k (the links in the six axis directions),
// with the wall point x_f + q e_k, the branch's outward normal there and the
// face's weight |n_k|, and x_f - e_k when it is a fluid cell of a leaf block of
// the finest level (else the stress of x_f alone is used).  Sorted by branch
// and cut into pieces of at most LINK_PIECE for the FP64 reduction.
static lbm_status build_friction(lbm_grid *g)
{
    const lbm_grid_desc &d = g->d;
    const DevLevel &fv = g->lv[g->L - 1];
    const int n_b = (int)g->branches.size();
    struct Face {
        uint32_t a0, a1;
        float q;
        float4 nw;
        int branch;
    };
    std::vector<Face> faces;
    auto leaf_fluid = [&](int x, int y, int z) -> int64_t {
        if (x < 0 || x >= d.nx || y < 0 || y >= d.ny || z < 0 || z >= d.nz)
            return -1;
        if (g->solid(x, y, z))
            return -1;
        if (!fv.dense && fv.block_kind(x / g->B, y / g->B, z / g->B) != 1)
            return -1;
        return level_cell_address(fv, g->B, x, y, z);
    };
    for (const HostLink &Lk : g->links) {
        const int i = Lk.dir, cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
        if (std::abs(cx) + std::abs(cy) + std::abs(cz) != 1 || Lk.branch < 0)
            continue;
        const int x = (int)(Lk.cell % d.nx), y = (int)((Lk.cell / d.nx) % d.ny),
                  z = (int)(Lk.cell / ((int64_t)d.nx * d.ny));
        const int64_t a0 = level_cell_address(fv, g->B, x, y, z);
        if (a0 < 0)
            return fail(g, LBM_E_INVALID, "friction surface cell outside the finest level");
        const int64_t a1 = leaf_fluid(x - cx, y - cy, z - cz);
        const double xw[3] = {x + 0.5 + Lk.q * cx, y + 0.5 + Lk.q * cy, z + 0.5 + Lk.q * cz};
        double n[3];
        branch_wall_normal(g->branches[(size_t)Lk.branch], xw, n);
        const double w = std::fabs(cx != 0 ? n[0] : cy != 0 ? n[1] : n[2]);
        faces.push_back({(uint32_t)a0, a1 < 0 ? FRIC_NO_UP : (uint32_t)a1, (float)Lk.q,
                         make_float4((float)n[0], (float)n[1], (float)n[2], (float)w), Lk.branch});
    }
    std::stable_sort(faces.begin(), faces.end(), [](const Face &a, const Face &b) { return a.branch < b.branch; });
    const int nf = (int)faces.size();
    std::vector<uint32_t> a0(nf), a1(nf);
    std::vector<float> q(nf);
    std::vector<float4> nw(nf);
    std::vector<int> seg(g->nseg + 1, 0);
    for (int t = 0; t < nf; ++t) {
        a0[t] = faces[t].a0;
        a1[t] = faces[t].a1;
        q[t] = faces[t].q;
        nw[t] = faces[t].nw;
        seg[faces[t].branch + 1]++;
    }
    for (int s2 = 0; s2 < g->nseg; ++s2)
        seg[s2 + 1] += seg[s2];
    std::vector<int> pstart(1, 0), segp(g->nseg + 1, 0);
    for (int s2 = 0; s2 < g->nseg; ++s2) {
        for (int l = seg[s2]; l < seg[s2 + 1]; l += LINK_PIECE)
            pstart.push_back(std::min(l + LINK_PIECE, seg[s2 + 1]));
        segp[s2 + 1] = (int)pstart.size() - 1;
    }
    (void)n_b;
    g->n_fric = nf;
    g->fric_npieces = (int)pstart.size() - 1;
    lbm_status st;
    if ((st = upload(g, &g->d_fa0, a0)) != LBM_OK || (st = upload(g, &g->d_fa1, a1)) != LBM_OK ||
        (st = upload(g, &g->d_fq, q)) != LBM_OK || (st = upload(g, &g->d_fnw, nw)) != LBM_OK ||
        (st = upload(g, &g->d_fpstart, pstart)) != LBM_OK || (st = upload(g, &g->d_fsegp, segp)) != LBM_OK ||
        (st = dalloc(g, &g->d_fforce, (size_t)3 * std::max(nf, 1))) != LBM_OK ||
        (st = dalloc(g, &g->d_fpiece_sum, (size_t)3 * std::max(g->fric_npieces, 1))) != LBM_OK ||
        (st = dalloc(g, &g->d_facc_branch, (size_t)3 * g->nseg)) != LBM_OK ||
        (st = dalloc(g, &g->d_facc_total, 3)) != LBM_OK || (st = dalloc(g, &g->d_fcounter, 1)) != LBM_OK)
        return st;
    HIPX(g, hipMemsetAsync(g->d_facc_branch, 0, sizeof(double) * 3 * g->nseg, g->stream));
    HIPX(g, hipMemsetAsync(g->d_facc_total, 0, sizeof(double) * 3, g->stream));
    HIPX(g, hipMemsetAsync(g->d_fcounter, 0, sizeof(unsigned), g->stream));
    return LBM_OK;
}

// transfer quantities of the coarse source cells of pair l into slot 0 (time
// T, before the coarse step) or 1 (T + 1, after it)
static lbm_status amr_moments(lbm_grid *g, int l, int slot)
{
    AmrPair &pr = g->amr.pairs[l];
    DevLevel &v = g->lv[l];
    CollideArgs a = collide_args(g, l);
    if (g->rec) {
        Phase p = new_phase(PH_AMR_MOMENTS);
        p.odd = (int)(v.steps & 1);
        p.a = a;
        p.cells = pr.d_src;
        p.n = (int)pr.h_src.size();
        p.om1 = (float)v.om1;
        p.dt = level_dt(g, l);
        p.out = pr.d_mom[slot];
        p.items = (p.n + 255) / 256;
        if (p.n > 0)
            g->rec->push_back(p);
        return LBM_OK;
    }
    HIPX(g, launch_amr_moments(g->B, g->d.storage, (int)(v.steps & 1), a, pr.d_src, (int)pr.h_src.size(),
                               (float)v.om1, level_dt(g, l), pr.d_mom[slot], g->stream));
    return LBM_OK;
}

// pre-collision state of the ghost cells of level l + 1 for its next sub-step
static lbm_status amr_prolong(lbm_grid *g, int l, int sub)
{
    AmrPair &pr = g->amr.pairs[l];
    DevLevel &f = g->lv[l + 1];
    CollideArgs a = collide_args(g, l + 1);
    if (g->rec) {
        Phase p = new_phase(PH_AMR_PROLONG);
        p.odd = (int)(f.steps & 1);
        p.a = a;
        p.cells = pr.d_ghost;
        p.src = pr.d_ghost_src;
        p.gmask = pr.d_ghost_mask;
        p.n = (int)pr.h_ghost.size();
        p.nsrc = (int)pr.h_src.size();
        p.m0 = pr.d_mom[0];
        p.m1 = sub ? pr.d_mom[1] : nullptr;
        p.om1 = (float)f.om1;
        p.dt = level_dt(g, l + 1);
        p.items = (p.n + 255) / 256;
        if (p.n > 0)
            g->rec->push_back(p);
        return LBM_OK;
    }
    HIPX(g, launch_amr_prolong(g->B, g->d.storage, (int)(f.steps & 1), a, pr.d_ghost, pr.d_ghost_mask, pr.d_ghost_src,
                               (int)pr.h_ghost.size(), (int)pr.h_src.size(), pr.d_mom[0],
                               sub ? pr.d_mom[1] : nullptr, (float)f.om1, level_dt(g, l + 1), g->stream));
    return LBM_OK;
}

// pre-collision state of the band cells of level l from level l + 1
static lbm_status amr_restrict(lbm_grid *g, int l)
{
    AmrPair &pr = g->amr.pairs[l];
    DevLevel &c = g->lv[l], &f = g->lv[l + 1];
    CollideArgs ac = collide_args(g, l), af = collide_args(g, l + 1);
    if (g->rec) {
        Phase p = new_phase(PH_AMR_RESTRICT);
        p.odd = (int)(c.steps & 1);
        p.odd2 = (int)(f.steps & 1);
        p.a = ac;
        p.b = af;
        p.cells = pr.d_band;
        p.child = pr.d_band_child;
        p.n = (int)pr.h_band.size();
        p.om1 = (float)c.om1;
        p.dt = level_dt(g, l);
        p.om2 = (float)f.om1;
        p.dt2 = level_dt(g, l + 1);
        p.items = (p.n + RESTRICT_CELLS - 1) / RESTRICT_CELLS;
        if (p.n > 0)
            g->rec->push_back(p);
        return LBM_OK;
    }
    HIPX(g, launch_amr_restrict(g->B, g->d.storage, (int)(c.steps & 1), (int)(f.steps & 1), ac, af, pr.d_band,
                                pr.d_band_child, (int)pr.h_band.size(), (float)c.om1, level_dt(g, l),
                                (float)f.om1, level_dt(g, l + 1), g->stream));
    return LBM_OK;
}

// One step of level l and, recursively, the two sub-steps of each finer
// level (coarse first): coarse step (with the transfer records at T), fine
// ghosts from T, fine sub-step, moments at T+1, fine ghosts from the mean,
// fine sub-step, restriction into the coarse band.
static lbm_status advance_level(lbm_grid *g, int l)
{
    lbm_status st;
    const bool finest = l == g->L - 1;
    DevLevel &v = g->lv[l];
    const int odd = (int)(v.steps & 1);
    if ((st = level_collide(g, l)) != LBM_OK)
        return st;
    v.steps++;
    if (finest) {
        g->finest_steps++;
        return finest_links(g, odd);
    }
    for (int sub = 0; sub < 2; ++sub) {
        if (sub == 1 && (st = amr_moments(g, l, 1)) != LBM_OK)
            return st;
        if ((st = amr_prolong(g, l, sub)) != LBM_OK)
            return st;
        if ((st = advance_level(g, l + 1)) != LBM_OK)
            return st;
    }
    return amr_restrict(g, l);
}

static lbm_status coarse_step(lbm_grid *g)
{
    lbm_status st = advance_level(g, 0);
    if (st == LBM_OK)
        g->coarse_steps++;
    return st;
}

// ---------------------------------------------------------------------------
// graph-captured coarse steps
// ---------------------------------------------------------------------------

static const size_t MAX_GRAPHS = 64;

// parity of every level, and which finest sub-steps of the coarse step
// sample the force (the finest step count after sub-step j is f0 + j + 1)
// A coarse step's launches depend on each level's A-A parity and on which of
// its finest sub-steps take force samples; the samples fall where
// (finest_steps + j + 1) is a multiple of drag_every, a pattern fixed by
// finest_steps mod drag_every.
static uint64_t step_key(const lbm_grid *g)
{
    uint64_t k = 0;
    for (int l = 0; l < g->L; ++l)
        k |= (uint64_t)(g->lv[l].steps & 1) << l;
    k |= (uint64_t)(g->finest_steps % g->d.drag_every) << LBM_MAX_LEVELS;
    return k;
}

static void graphs_clear(lbm_grid *g)
{
    for (lbm_grid::StepGraph &sg : g->graphs) {
        if (sg.exec)
            (void)hipGraphExecDestroy(sg.exec);
        if (sg.d_phases)
            (void)hipFree(sg.d_phases);
        if (sg.d_ctr)
            (void)hipFree(sg.d_ctr);
    }
    g->graphs.clear();
}

static void apply_deltas(lbm_grid *g, const lbm_grid::StepGraph &sg)
{
    for (int l = 0; l < g->L; ++l)
        g->lv[l].steps += sg.level_steps[l];
    g->coarse_steps += sg.coarse;
    g->finest_steps += sg.finest;
    g->samples += sg.samples;
    g->ring_count += sg.ring;
}

static lbm_status graph_step(lbm_grid *g)
{
    const uint64_t key = step_key(g);
    for (const lbm_grid::StepGraph &sg : g->graphs) {
        if (sg.key != key)
            continue;
        HIPX(g, hipGraphLaunch(sg.exec, g->stream));
        apply_deltas(g, sg);
        return LBM_OK;
    }
    if (g->graphs.size() >= MAX_GRAPHS)
        graphs_clear(g);
    // capture one coarse step; its host bookkeeping runs as in an eager step
    lbm_grid::StepGraph sg{};
    sg.key = key;
    int64_t steps0[LBM_MAX_LEVELS] = {0};
    for (int l = 0; l < g->L; ++l)
        steps0[l] = g->lv[l].steps;
    const int64_t c0 = g->coarse_steps, f0 = g->finest_steps, s0 = g->samples, r0 = g->ring_count;
    auto restore = [&]() {
        for (int l = 0; l < g->L; ++l)
            g->lv[l].steps = steps0[l];
        g->coarse_steps = c0, g->finest_steps = f0, g->samples = s0, g->ring_count = r0;
    };
    HIPX(g, hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    const lbm_status st = coarse_step(g);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->stream, &graph);
    if (st != LBM_OK || ec != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        restore();
        return st != LBM_OK ? st : fail(g, LBM_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    }
    const hipError_t ei = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        restore();
        return fail(g, LBM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    for (int l = 0; l < g->L; ++l)
        sg.level_steps[l] = g->lv[l].steps - steps0[l];
    sg.coarse = g->coarse_steps - c0;
    sg.finest = g->finest_steps - f0;
    sg.samples = g->samples - s0;
    sg.ring = g->ring_count - r0;
    g->graphs.push_back(sg);
    const hipError_t el = hipGraphLaunch(sg.exec, g->stream);
    if (el != hipSuccess) {
        restore();
        return fail(g, LBM_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(el));
    }
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// persistent coarse steps
// ---------------------------------------------------------------------------

static int persist_grid_size(const lbm_grid *g)
{
    return g->persist_grid > 0 ? std::min(g->persist_grid, g->persist_max) : g->persist_max;
}

static lbm_status persistent_step(lbm_grid *g)
{
    if (g->persist_failed)
        return fail(g, LBM_E_DEVICE, "an earlier persistent launch was abandoned (a bounded wait expired)");
    if (g->persist_max <= 0)
        return fail(g, LBM_E_DEVICE, "the persistent kernel cannot be resident on this device");
    const uint64_t key = step_key(g);
    const int grid = persist_grid_size(g);
    for (const lbm_grid::StepGraph &sg : g->graphs) {
        if (sg.key != key)
            continue;
        if (sg.exec)
            HIPX(g, hipGraphLaunch(sg.exec, g->stream));
        else
            HIPX(g, launch_persistent(g->B, g->d.storage, sg.d_phases, sg.n_phases, sg.d_ctr, g->d_abort,
                                      g->persist_wait_ticks, grid, g->stream));
        apply_deltas(g, sg);
        return LBM_OK;
    }
    if (g->graphs.size() >= MAX_GRAPHS)
        graphs_clear(g);
    // record the coarse step as phases; its host bookkeeping runs as in an
    // eager step
    lbm_grid::StepGraph sg{};
    sg.key = key;
    int64_t steps0[LBM_MAX_LEVELS] = {0};
    for (int l = 0; l < g->L; ++l)
        steps0[l] = g->lv[l].steps;
    const int64_t c0 = g->coarse_steps, f0 = g->finest_steps, s0 = g->samples, r0 = g->ring_count;
    auto restore = [&]() {
        for (int l = 0; l < g->L; ++l)
            g->lv[l].steps = steps0[l];
        g->coarse_steps = c0, g->finest_steps = f0, g->samples = s0, g->ring_count = r0;
    };
    std::vector<Phase> ph;
    g->rec = &ph;
    const lbm_status st = coarse_step(g);
    g->rec = nullptr;
    if (st != LBM_OK) {
        restore();
        return st;
    }
    for (Phase &p : ph) {
        p.chunk = persist_chunk(p.items, grid);
        p.chunks = (p.items + p.chunk - 1) / p.chunk;
    }
    sg.n_phases = (int)ph.size();
    const size_t nctr = 2 * ph.size() + 1;
    if (hipMalloc(&sg.d_phases, sizeof(Phase) * std::max<size_t>(ph.size(), 1)) != hipSuccess ||
        hipMalloc(&sg.d_ctr, sizeof(unsigned) * nctr) != hipSuccess) {
        if (sg.d_phases)
            (void)hipFree(sg.d_phases);
        restore();
        return fail(g, LBM_E_NOMEM, "hipMalloc of the phase list failed");
    }
    // the counters are cleared on the grid's stream, so the clear is ordered
    // before the first launch (the grid's own stream does not synchronise with
    // the null stream)
    if (hipMemcpy(sg.d_phases, ph.data(), sizeof(Phase) * ph.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(sg.d_ctr, 0, sizeof(unsigned) * nctr, g->stream) != hipSuccess) {
        (void)hipFree(sg.d_phases);
        (void)hipFree(sg.d_ctr);
        restore();
        return fail(g, LBM_E_DEVICE, "upload of the phase list failed");
    }
    if (g->d.flags & LBM_F_GRAPH) {
        // one graph node per coarse step
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const hipError_t el = launch_persistent(g->B, g->d.storage, sg.d_phases, sg.n_phases, sg.d_ctr,
                                                    g->d_abort, g->persist_wait_ticks, grid, g->stream);
            const hipError_t ee = hipStreamEndCapture(g->stream, &graph);
            ok = el == hipSuccess && ee == hipSuccess && graph &&
                 hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0) == hipSuccess;
        }
        if (graph)
            (void)hipGraphDestroy(graph);
        if (!ok) {
            (void)hipFree(sg.d_phases);
            (void)hipFree(sg.d_ctr);
            restore();
            return fail(g, LBM_E_DEVICE, "capture of the persistent launch failed");
        }
    }
    for (int l = 0; l < g->L; ++l)
        sg.level_steps[l] = g->lv[l].steps - steps0[l];
    sg.coarse = g->coarse_steps - c0;
    sg.finest = g->finest_steps - f0;
    sg.samples = g->samples - s0;
    sg.ring = g->ring_count - r0;
    g->graphs.push_back(sg);
    const hipError_t el = sg.exec ? hipGraphLaunch(sg.exec, g->stream)
                                  : launch_persistent(g->B, g->d.storage, sg.d_phases, sg.n_phases, sg.d_ctr,
                                                      g->d_abort, g->persist_wait_ticks, grid, g->stream);
    if (el != hipSuccess) {
        restore();
        return fail(g, LBM_E_DEVICE, std::string("persistent launch: ") + hipGetErrorString(el));
    }
    return LBM_OK;
}

// after persistent launches: fails when one of them was abandoned
static lbm_status check_persistent(lbm_grid *g)
{
    if (!(g->d.flags & LBM_F_PERSISTENT) || !g->d_abort)
        return LBM_OK;
    unsigned ab = 0;
    HIPX(g, hipStreamSynchronize(g->stream));
    HIPX(g, hipMemcpy(&ab, g->d_abort, sizeof ab, hipMemcpyDeviceToHost));
    if (ab) {
        g->persist_failed = true;
        return fail(g, LBM_E_DEVICE, "a persistent launch was abandoned (a bounded wait expired)");
    }
    return LBM_OK;
}

static lbm_status sync_device_counters(lbm_grid *g)
{
    HIPX(g, hipStreamSynchronize(g->stream));
    if (g->d_ring_pos) {
        const unsigned long long pos = (unsigned long long)g->ring_count;
        HIPX(g, hipMemcpy(g->d_ring_pos, &pos, sizeof pos, hipMemcpyHostToDevice));
    }
    if (g->d_tick) {
        const unsigned long long tick = (unsigned long long)(g->lv[0].steps / 2);
        HIPX(g, hipMemcpy(g->d_tick, &tick, sizeof tick, hipMemcpyHostToDevice));
    }
    return LBM_OK;
}

// before reading level-0 pre-collision states at odd parity: the inlet plane
// of the time the coming step reads
static lbm_status prepare_inlet(lbm_grid *g)
{
    if (g->turb && (g->lv[0].steps & 1))
        return inflow_planes(g);
    return LBM_OK;
}

namespace lbm {
lbm_status grid_fail(lbm_grid *g, lbm_status st, const std::string &msg) { return fail(g, st, msg); }
CollideArgs grid_collide_args(lbm_grid *g, int l) { return collide_args(g, l); }
lbm_status grid_coarse_step(lbm_grid *g) { return coarse_step(g); }
size_t grid_storage_bytes(int storage) { return storage_bytes(storage); }
int grid_timing_mark(lbm_grid *g) { return timing_mark(g); }
void grid_graphs_clear(lbm_grid *g) { graphs_clear(g); }
lbm_status grid_sync_device_counters(lbm_grid *g) { return sync_device_counters(g); }
}  // namespace lbm

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *lbm_last_error(const lbm_grid *g)
{
    if (g)
        return g->err.c_str();
    return g_thread_error.c_str();
}

// host validation of a grid description (shared by lbm_create_grid and
// lbm_plan_levels)
static lbm_status check_desc(const lbm_grid_desc *d, std::string *msg)
{
    const int B = d->block_edge;
    if (B != 8 && B != 16)
        return (*msg = "block_edge must be 8 or 16", LBM_E_INVALID);
    if (d->levels < 1 || d->levels > LBM_MAX_LEVELS)
        return (*msg = "levels must be 1..4", LBM_E_INVALID);
    const int unit = B << (d->levels - 1);
    if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0 || d->nx % unit || d->ny % unit || d->nz % unit)
        return (*msg = "nx, ny, nz must be positive multiples of block_edge << (levels-1)", LBM_E_INVALID);
    if ((int64_t)(d->nx / unit) * (d->ny / unit) * (d->nz / unit) > (1 << 24))
        return (*msg = "too many coarse blocks", LBM_E_INVALID);
    if (!(d->u_in >= 0.0) || std::sqrt(3.0) * d->u_in >= 0.3)
        return (*msg = "u_in must satisfy 0 <= sqrt(3) u_in < 0.3", LBM_E_INVALID);
    if (!(d->nu > 0.0) && !(d->re_h > 0.0))
        return (*msg = "need nu > 0 or re_h > 0", LBM_E_INVALID);
    if (d->storage < 0 || d->storage > 2)
        return (*msg = "storage must be LBM_FP32, LBM_FP16_DEV or LBM_BF16_DEV", LBM_E_INVALID);
    if (d->periodic_yz != 0 && d->periodic_yz != 1)
        return (*msg = "periodic_yz must be 1 (periodic lateral faces) or 0 (inflow faces)", LBM_E_INVALID);
    if (d->drag_every < 0)
        return (*msg = "drag_every must be >= 1", LBM_E_INVALID);
    if (d->flags & LBM_F_PERSISTENT)
        return (*msg = "LBM_F_PERSISTENT is disabled: the persistent coarse-step launch did not finish on the GPU "
                       "(its waits are bounded, so a cause outside them is still open); use LBM_F_GRAPH",
                LBM_E_INVALID);
    if (d->turb_intensity < 0.0 || d->turb_intensity > 0.5)
        return (*msg = "turb_intensity must be in [0, 0.5]", LBM_E_INVALID);
    if (d->turb_intensity > 0.0 && !(d->turb_length > 0.0))
        return (*msg = "turb_length must be > 0 with inflow turbulence", LBM_E_INVALID);
    return LBM_OK;
}

// host validation of a branch list (shared by lbm_set_geometry and
// lbm_plan_levels)
static lbm_status check_branches(const lbm_grid_desc &d, const lbm_branch *b, int32_t n_b, std::string *msg)
{
    if (!b || n_b <= 0)
        return (*msg = "need at least one branch", LBM_E_INVALID);
    for (int i = 0; i < n_b; ++i) {
        if (b[i].id != i)
            return (*msg = "branch ids must be 0 .. n_b-1 in order", LBM_E_INVALID);
        if (!(b[i].diameter > 0.0))
            return (*msg = "branch diameter must be > 0", LBM_E_INVALID);
        const double dx = b[i].p1[0] - b[i].p0[0], dy = b[i].p1[1] - b[i].p0[1], dz = b[i].p1[2] - b[i].p0[2];
        if (!(dx * dx + dy * dy + dz * dz > 0.0))
            return (*msg = "branch of zero length", LBM_E_INVALID);
    }
    const int margin = d.levels == 1 ? 2 : d.block_edge << (d.levels - 1);
    // one level with periodic y: a cylinder spanning y is allowed
    if (!tree_fits_box(b, n_b, d.nx, d.ny, d.nz, margin, d.levels == 1 && d.periodic_yz != 0))
        return (*msg = "tree comes too close to the box faces", LBM_E_INVALID);
    return LBM_OK;
}

lbm_status lbm_create_grid(const lbm_grid_desc *d, lbm_grid **out)
{
    if (!d || !out)
        return fail(nullptr, LBM_E_INVALID, "null argument");
    *out = nullptr;
    {
        std::string msg;
        if (check_desc(d, &msg) != LBM_OK)
            return fail(nullptr, LBM_E_INVALID, msg);
    }
    const int B = d->block_edge;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(nullptr, LBM_E_DEVICE, "no HIP device available");
    if (d->device < 0 || d->device >= ndev)
        return fail(nullptr, LBM_E_INVALID, "device ordinal out of range");
    lbm_grid *g = new (std::nothrow) lbm_grid();
    if (!g)
        return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    g->d = *d;
    if (g->d.drag_every == 0)
        g->d.drag_every = 1;
    if (g->d.turb_modes <= 0)
        g->d.turb_modes = 200;
    g->B = B;
    g->L = d->levels;
    g->tile = B * B;  // one z-slice of a block per work-group
    g->threads = std::min(256, g->tile);
    // measured defaults (uniform 512x256x256): streaming even steps run best
    // with 3 (FP32) or 4 (16-bit) waves per SIMD; odd steps are register-bound
    g->occ_even = d->storage == LBM_FP32 ? 3 : 4;
    g->occ_odd = 0;
    if (hipSetDevice(d->device) != hipSuccess) {
        delete g;
        return fail(nullptr, LBM_E_DEVICE, "hipSetDevice failed");
    }
    if (d->stream) {
        g->stream = (hipStream_t)d->stream;
    } else {
        if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
            delete g;
            return fail(nullptr, LBM_E_DEVICE, "hipStreamCreate failed");
        }
        g->own_stream = true;
    }
    *out = g;
    return LBM_OK;
}

void lbm_destroy_grid(lbm_grid *g)
{
    if (!g)
        return;
    if (g->stream)
        (void)hipStreamSynchronize(g->stream);
    delete g;
}

lbm_status lbm_tree_generate(const lbm_tree_params *p, lbm_branch *out, int32_t cap, int32_t *n)
{
    if (!p || !n)
        return fail(nullptr, LBM_E_INVALID, "null argument");
    if (p->m < 1 || p->m > 4 || p->order < 0 || p->order > 12 || !(p->s0 > 0) || !(p->w0 > 0))
        return fail(nullptr, LBM_E_INVALID, "tree parameters out of range");
    double total = 1, lvl = 1;
    for (int k = 0; k < p->order; ++k) {
        lvl *= p->m;
        total += lvl;
    }
    if (total > 4.0e6)
        return fail(nullptr, LBM_E_INVALID, "tree too large");
    std::vector<lbm_branch> v;
    tree_generate(*p, v);
    *n = (int32_t)v.size();
    if (out)
        std::memcpy(out, v.data(), sizeof(lbm_branch) * std::min<size_t>(v.size(), cap > 0 ? cap : 0));
    return LBM_OK;
}

lbm_status lbm_tree_place(lbm_branch *b, int32_t n, double target_h, const double com[3], double *height_out)
{
    if (!b || n <= 0 || !com)
        return fail(nullptr, LBM_E_INVALID, "null argument or empty tree");
    tree_place(b, n, target_h, com);
    if (height_out)
        *height_out = tree_height(b, n);
    return LBM_OK;
}

lbm_status lbm_set_geometry(lbm_grid *g, const lbm_branch *b, int32_t n_b, const lbm_refine_desc *refine,
                            size_t *device_bytes_out)
{
    if (!g)
        return fail(nullptr, LBM_E_INVALID, "null grid");
    if (g->state != 0)
        return fail(g, LBM_E_STATE, "geometry already set");
    const lbm_grid_desc &d = g->d;
    {
        std::string msg;
        if (check_branches(d, b, n_b, &msg) != LBM_OK)
            return fail(g, LBM_E_INVALID, msg);
    }
    if (g->L > 1 && !refine)
        return fail(g, LBM_E_INVALID, "refinement bands required when levels > 1");
    (void)hipSetDevice(d.device);
    g->branches.assign(b, b + n_b);
    g->H = tree_height(b, n_b);
    g->nu_f = d.nu > 0.0 ? d.nu : d.u_in * g->H / d.re_h;
    if (!(g->nu_f > 0.0) || !(g->nu_f < 10.0))
        return fail(g, LBM_E_INVALID, "finest viscosity out of range");

    voxelize(b, n_b, d.nx, d.ny, d.nz, g->solid);
    build_links(b, n_b, g->solid, g->links);
    g->area_x = (double)frontal_area(g->solid);

    // block grid of every level
    std::string msg;
    lbm_status st = build_levels(d, g->B, g->L, b, n_b, refine, g->solid, g->lv, g->amr, &msg);
    if (st != LBM_OK)
        return fail(g, st, msg);
    for (int l = 0; l < g->L; ++l)
        nu_to_level_omega(g->nu_f, g->L, l, &g->lv[l].om1);

    // device buffers of the levels
    const size_t eb = storage_bytes(d.storage);
    size_t need_bound = 0;
    for (int l = 0; l < g->L; ++l) {
        g->lv[l].dir_elems = level_dir_elems(g->lv[l], g->B, d.storage);
        need_bound += bound_share(g->lv[l].dir_elems * 27 * eb);
    }
    if (g->bound && need_bound > g->bound_bytes)
        return fail(g, LBM_E_INVALID, "bound memory too small: the populations need " + std::to_string(need_bound) +
                                          " bytes (lbm_plan_levels pop_bytes)");
    size_t bound_off = 0;
    for (int l = 0; l < g->L; ++l) {
        DevLevel &v = g->lv[l];
        if (v.dir_elems > (size_t)UINT32_MAX / 2)
            return fail(g, LBM_E_INVALID, "level too large for 32-bit cell addressing");
        char *pop = nullptr;
        if (g->bound) {
            // populations of every level carved from the caller's buffer
            pop = (char *)g->bound + bound_off;
            bound_off += bound_share(v.dir_elems * 27 * eb);
        } else if ((st = dalloc(g, &pop, v.dir_elems * 27 * eb)) != LBM_OK) {
            return st;
        }
        v.pop = pop;
        if (v.dense && v.h_nbr.empty())
            v.h_nbr.assign(27, 0);
        if ((st = upload(g, &v.nbr, v.h_nbr)) != LBM_OK || (st = upload(g, &v.bxyz, v.h_bxyz)) != LBM_OK ||
            (st = upload(g, &v.work, v.h_work)) != LBM_OK || (st = upload(g, &v.leaf, v.h_leaf)) != LBM_OK ||
            (st = upload(g, &v.masks, v.h_masks)) != LBM_OK)
            return st;
        if (!v.h_work_odd.empty() && (st = upload(g, &v.work_odd, v.h_work_odd)) != LBM_OK)
            return st;
        v.n_work = (int)v.h_work.size();
        v.n_leaf = (int)v.h_leaf.size();
        if (l == 0) {
            if ((st = dalloc(g, &v.gbuf, (size_t)27 * v.ny * v.nz)) != LBM_OK)
                return st;
            HIPX(g, hipMemsetAsync(v.gbuf, 0, sizeof(float) * 27 * (size_t)v.ny * v.nz, g->stream));
        }
        const int unit = v.dense ? DENSE_TILE : g->B * g->B * g->B;
        HIPX(g, launch_fill_sink_and_all(d.storage, v.pop, v.dir_elems, g->stream));
        HIPX(g, launch_init(unit, d.storage, v.pop, v.dir_elems, v.leaf, v.n_leaf, v.masks, (float)d.u_in,
                            g->stream));
        // ghost / band cells start from the same uniform state
        HIPX(g, launch_init(unit, d.storage, v.pop, v.dir_elems, v.work, v.n_work, v.masks, (float)d.u_in,
                            g->stream));
    }
    if ((st = amr_upload(g->amr, g->lv, g->B, [&](void **p, size_t bytes) -> lbm_status {
             char *q = nullptr;
             lbm_status s2 = dalloc(g, &q, bytes);
             *p = q;
             return s2;
         }, g->stream, &g->err)) != LBM_OK)
        return st;

    // links on the finest level, sorted by branch (segments for the reduction),
    // then by direction and cell address: neighbouring links of a wave then
    // touch the same population array at nearby addresses
    {
        const DevLevel &fv = g->lv[g->L - 1];
        const int nl = (int)g->links.size();
        std::vector<int32_t> perm(nl);
        std::iota(perm.begin(), perm.end(), 0);
        std::vector<int64_t> addr(nl);
        for (int t = 0; t < nl; ++t) {
            const int64_t c = g->links[t].cell;
            addr[t] = level_cell_address(fv, g->B, (int)(c % d.nx), (int)((c / d.nx) % d.ny),
                                         (int)(c / ((int64_t)d.nx * d.ny)));
        }
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) {
            const int ba = g->links[a].branch < 0 ? n_b : g->links[a].branch;
            const int bc = g->links[c].branch < 0 ? n_b : g->links[c].branch;
            if (ba != bc)
                return ba < bc;
            if (g->links[a].dir != g->links[c].dir)
                return g->links[a].dir < g->links[c].dir;
            return addr[a] < addr[c];
        });
        g->link_perm = perm;
        std::vector<uint32_t> af(nl), ap(nl), am(nl);
        std::vector<uint8_t> dr(nl);
        std::vector<float> q(nl);
        g->nseg = n_b + 1;
        std::vector<int> seg(g->nseg + 1, 0);
        const int fx = d.nx, fy = d.ny;
        for (int t = 0; t < nl; ++t) {
            const HostLink &Lk = g->links[perm[t]];
            const int x = (int)(Lk.cell % fx), y = (int)((Lk.cell / fx) % fy), z = (int)(Lk.cell / ((int64_t)fx * fy));
            const int i = Lk.dir, cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
            const int64_t a0 = level_cell_address(fv, g->B, x, y, z);
            const int64_t a1 = level_cell_address(fv, g->B, x + cx, y + cy, z + cz);
            const int64_t a2 = level_cell_address(fv, g->B, x - cx, y - cy, z - cz);
            if (a0 < 0 || a1 < 0 || a2 < 0)
                return fail(g, LBM_E_INVALID, "boundary link outside the finest level");
            af[t] = (uint32_t)a0;
            ap[t] = (uint32_t)a1;
            am[t] = (uint32_t)a2;
            dr[t] = (uint8_t)(i | (Lk.up_fluid ? 0x80 : 0));
            q[t] = (float)Lk.q;
            seg[(Lk.branch < 0 ? n_b : Lk.branch) + 1]++;
        }
        for (int s = 0; s < g->nseg; ++s)
            seg[s + 1] += seg[s];
        // pieces of at most LINK_PIECE links within each branch's run
        std::vector<int> pstart(1, 0), segp(g->nseg + 1, 0);
        for (int s = 0; s < g->nseg; ++s) {
            for (int l = seg[s]; l < seg[s + 1]; l += LINK_PIECE)
                pstart.push_back(std::min(l + LINK_PIECE, seg[s + 1]));
            segp[s + 1] = (int)pstart.size() - 1;
        }
        g->npieces = (int)pstart.size() - 1;
        g->n_links = nl;
        if ((st = upload(g, &g->d_af, af)) != LBM_OK || (st = upload(g, &g->d_ap, ap)) != LBM_OK ||
            (st = upload(g, &g->d_am, am)) != LBM_OK || (st = upload(g, &g->d_dir, dr)) != LBM_OK ||
            (st = upload(g, &g->d_q, q)) != LBM_OK || (st = upload(g, &g->d_pstart, pstart)) != LBM_OK ||
            (st = upload(g, &g->d_segp, segp)) != LBM_OK ||
            (st = dalloc(g, &g->d_piece_sum, (size_t)3 * std::max(g->npieces, 1))) != LBM_OK)
            return st;
        if ((st = dalloc(g, &g->d_lforce, (size_t)3 * std::max(nl, 1))) != LBM_OK ||
            (st = dalloc(g, &g->d_sample, (size_t)3 * g->nseg)) != LBM_OK ||
            (st = dalloc(g, &g->d_acc_branch, (size_t)3 * g->nseg)) != LBM_OK ||
            (st = dalloc(g, &g->d_acc_total, 3)) != LBM_OK || (st = dalloc(g, &g->d_ring, (size_t)3 * RING)) != LBM_OK ||
            (st = dalloc(g, &g->d_counter, 1)) != LBM_OK || (st = dalloc(g, &g->d_ring_pos, 1)) != LBM_OK ||
            (st = dalloc(g, &g->d_mass, 4 + 4 * 1024)) != LBM_OK)
            return st;
        HIPX(g, hipMemsetAsync(g->d_acc_branch, 0, sizeof(double) * 3 * g->nseg, g->stream));
        HIPX(g, hipMemsetAsync(g->d_acc_total, 0, sizeof(double) * 3, g->stream));
        HIPX(g, hipMemsetAsync(g->d_ring, 0, sizeof(double) * 3 * RING, g->stream));
        HIPX(g, hipMemsetAsync(g->d_counter, 0, sizeof(unsigned), g->stream));
        HIPX(g, hipMemsetAsync(g->d_ring_pos, 0, sizeof(unsigned long long), g->stream));
    }
    if (g->d.flags & LBM_F_FRICTION) {
        if ((st = build_friction(g)) != LBM_OK)
            return st;
    }
    if (g->d.turb_intensity > 0.0) {
        InflowModes m;
        const double d0 = (double)(1 << (g->L - 1));
        build_inflow_modes(g->d.turb_seed, g->d.turb_modes, g->d.turb_intensity, g->d.turb_length, d.u_in, d0, m);
        std::vector<double> packed;
        for (const std::vector<double> *v : {&m.kx, &m.ky, &m.kz, &m.sx, &m.sy, &m.sz, &m.psi, &m.amp})
            packed.insert(packed.end(), v->begin(), v->end());
        const size_t plane = (size_t)3 * g->lv[0].ny * g->lv[0].nz;
        if ((st = upload(g, &g->d_modes, packed)) != LBM_OK || (st = dalloc(g, &g->d_in_prev, plane)) != LBM_OK ||
            (st = dalloc(g, &g->d_in_cur, plane)) != LBM_OK || (st = dalloc(g, &g->d_tick, 1)) != LBM_OK)
            return st;
        HIPX(g, hipMemsetAsync(g->d_tick, 0, sizeof(unsigned long long), g->stream));
        g->n_modes = g->d.turb_modes;
        g->turb_ke = m.k_e;
        g->turb = true;
    }
    {
        lbm_status st2 = dalloc(g, &g->d_abort, 1);
        if (st2 != LBM_OK)
            return st2;
        HIPX(g, hipMemsetAsync(g->d_abort, 0, sizeof(unsigned), g->stream));
        if (persistent_max_grid(g->B, g->d.storage, g->d.device, &g->persist_max, &g->cus) != hipSuccess) {
            (void)hipGetLastError();
            g->persist_max = 0;
            g->cus = 0;
        }
        // one wait of the persistent launch gives up after PERSIST_WAIT_S
        // seconds of the device's constant real-time clock (kHz)
        int wall_khz = 0;
        if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, g->d.device) != hipSuccess ||
            wall_khz <= 0) {
            (void)hipGetLastError();
            g->persist_max = 0;  // no time bound, no persistent launch
        }
        g->persist_wait_ticks = (unsigned long long)(PERSIST_WAIT_S * 1000.0 * wall_khz);
        g->wall_khz = wall_khz;
    }
    HIPX(g, hipStreamSynchronize(g->stream));
    g->state = 1;
    if (device_bytes_out)
        *device_bytes_out = g->device_bytes;
    return LBM_OK;
}

lbm_status lbm_bind_memory(lbm_grid *g, void *device_ptr, size_t bytes)
{
    if (!g || !device_ptr || bytes == 0)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 0)
        return fail(g, LBM_E_STATE, "bind memory before lbm_set_geometry");
    if ((uintptr_t)device_ptr % 256 != 0)
        return fail(g, LBM_E_INVALID, "bound memory must be 256-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, device_ptr) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != g->d.device) {
        (void)hipGetLastError();
        return fail(g, LBM_E_INVALID, "bound memory must be device memory of the grid's device");
    }
    g->bound = device_ptr;
    g->bound_bytes = bytes;
    return LBM_OK;
}

lbm_status lbm_step(lbm_grid *g, int32_t n)
{
    if (!g)
        return fail(nullptr, LBM_E_INVALID, "null grid");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (n < 0)
        return fail(g, LBM_E_INVALID, "negative step count");
    const bool persistent = (g->d.flags & LBM_F_PERSISTENT) && !g->timing;
    const bool graph = (g->d.flags & LBM_F_GRAPH) && !g->timing;
    for (int s = 0; s < n; ++s) {
        lbm_status st = persistent ? persistent_step(g) : graph ? graph_step(g) : coarse_step(g);
        if (st != LBM_OK)
            return st;
    }
    return LBM_OK;
}

lbm_status lbm_mass(lbm_grid *g, double *mass)
{
    if (!g || !mass)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (lbm_status ps = check_persistent(g); ps != LBM_OK)
        return ps;
    if (lbm_status pi = prepare_inlet(g); pi != LBM_OK)
        return pi;
    double init[4] = {0.0, 1e300, -1e300, 0.0};
    HIPX(g, hipMemcpyAsync(g->d_mass, init, sizeof init, hipMemcpyHostToDevice, g->stream));
    for (int l = 0; l < g->L; ++l) {
        DevLevel &v = g->lv[l];
        CollideArgs a = collide_args(g, l);
        const double h = double(1 << (g->L - 1 - l));
        HIPX(g, launch_mass(g->B, g->d.storage, (int)(v.steps & 1), a, v.leaf, v.n_leaf, h * h * h, g->d_mass,
                            g->stream));
    }
    double out[4];
    HIPX(g, hipMemcpyAsync(out, g->d_mass, sizeof out, hipMemcpyDeviceToHost, g->stream));
    HIPX(g, hipStreamSynchronize(g->stream));
    *mass = out[0];
    if (out[3] > 0.0 || out[1] < 0.5 || out[2] > 1.5)
        return fail(g, LBM_E_UNSTABLE, "non-finite or out-of-range density detected");
    return LBM_OK;
}

lbm_status lbm_drag(lbm_grid *g, lbm_drag_result *out, double *per_branch)
{
    return lbm_drag_split(g, out, per_branch, nullptr);
}

lbm_status lbm_drag_split(lbm_grid *g, lbm_drag_result *out, double *per_branch, double *per_branch_friction)
{
    if (!g || !out)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (per_branch_friction && !(g->d.flags & LBM_F_FRICTION))
        return fail(g, LBM_E_STATE, "friction is sampled only with LBM_F_FRICTION");
    if (lbm_status ps = check_persistent(g); ps != LBM_OK)
        return ps;
    std::memset(out, 0, sizeof *out);
    const int nb = (int)g->branches.size();
    std::vector<double> acc(3 * g->nseg, 0.0);
    double tot[3] = {0, 0, 0};
    HIPX(g, hipMemcpyAsync(acc.data(), g->d_acc_branch, sizeof(double) * acc.size(), hipMemcpyDeviceToHost, g->stream));
    HIPX(g, hipMemcpyAsync(tot, g->d_acc_total, sizeof tot, hipMemcpyDeviceToHost, g->stream));
    HIPX(g, hipStreamSynchronize(g->stream));
    HIPX(g, hipMemsetAsync(g->d_acc_branch, 0, sizeof(double) * acc.size(), g->stream));
    HIPX(g, hipMemsetAsync(g->d_acc_total, 0, sizeof tot, g->stream));
    std::vector<double> facc;
    double ftot[3] = {0, 0, 0};
    if (g->d_facc_total) {
        facc.assign(3 * (size_t)g->nseg, 0.0);
        HIPX(g, hipMemcpyAsync(facc.data(), g->d_facc_branch, sizeof(double) * facc.size(), hipMemcpyDeviceToHost,
                               g->stream));
        HIPX(g, hipMemcpyAsync(ftot, g->d_facc_total, sizeof ftot, hipMemcpyDeviceToHost, g->stream));
        HIPX(g, hipStreamSynchronize(g->stream));
        HIPX(g, hipMemsetAsync(g->d_facc_branch, 0, sizeof(double) * facc.size(), g->stream));
        HIPX(g, hipMemsetAsync(g->d_facc_total, 0, sizeof ftot, g->stream));
    }
    const double ns = (double)std::max<int64_t>(g->samples, 1);
    for (int a = 0; a < 3; ++a) {
        out->force[a] = tot[a] / ns;
        out->friction[a] = ftot[a] / ns;
    }
    if (per_branch)
        for (int i = 0; i < nb; ++i)
            for (int a = 0; a < 3; ++a)
                per_branch[3 * i + a] = acc[3 * i + a] / ns;
    if (per_branch_friction)
        for (int i = 0; i < nb; ++i)
            for (int a = 0; a < 3; ++a)
                per_branch_friction[3 * i + a] = facc[3 * i + a] / ns;
    out->samples = g->samples;
    g->samples = 0;
    out->area_x = g->area_x;
    out->height = g->H;
    const double qa = 0.5 * g->d.u_in * g->d.u_in * g->area_x;
    out->cd = qa > 0.0 ? out->force[0] / qa : 0.0;
    out->cf = qa > 0.0 ? out->friction[0] / qa : 0.0;
    out->cp = out->cd - out->cf;
    out->step = g->coarse_steps;
    return lbm_mass(g, &out->mass);
}

lbm_status lbm_drag_series(lbm_grid *g, double *out, int64_t cap, int64_t *n)
{
    if (!g || !n || (!out && cap > 0))
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (lbm_status ps = check_persistent(g); ps != LBM_OK)
        return ps;
    std::vector<double> ring(3 * (size_t)RING);
    HIPX(g, hipMemcpyAsync(ring.data(), g->d_ring, sizeof(double) * ring.size(), hipMemcpyDeviceToHost, g->stream));
    HIPX(g, hipStreamSynchronize(g->stream));
    const int64_t have = std::min<int64_t>(g->ring_count, RING);
    const int64_t m = std::min(have, cap);
    const int64_t first = g->ring_count - m;
    for (int64_t s = 0; s < m; ++s)
        for (int a = 0; a < 3; ++a)
            out[3 * s + a] = ring[3 * ((first + s) % RING) + a];
    *n = m;
    return LBM_OK;
}

lbm_status lbm_timing_enable(lbm_grid *g, int32_t enable)
{
    if (!g)
        return fail(nullptr, LBM_E_INVALID, "null grid");
    HIPX(g, hipStreamSynchronize(g->stream));
    for (hipEvent_t e : g->ev_pool)
        (void)hipEventDestroy(e);
    g->ev_pool.clear();
    g->ev_pairs.clear();
    g->timing = enable != 0;
    return LBM_OK;
}

lbm_status lbm_timing_read(lbm_grid *g, double *collide_ms, int64_t *collide_n, double *links_ms, int64_t *links_n)
{
    if (!g)
        return fail(nullptr, LBM_E_INVALID, "null grid");
    HIPX(g, hipStreamSynchronize(g->stream));
    double t[2] = {0.0, 0.0};
    int64_t n[2] = {0, 0};
    for (const auto &pr : g->ev_pairs) {
        float ms = 0.0f;
        HIPX(g, hipEventElapsedTime(&ms, g->ev_pool[pr.first], g->ev_pool[pr.first + 1]));
        t[pr.second] += ms;
        n[pr.second]++;
    }
    if (collide_ms) *collide_ms = t[0];
    if (collide_n) *collide_n = n[0];
    if (links_ms) *links_ms = t[1];
    if (links_n) *links_n = n[1];
    return LBM_OK;
}

lbm_status lbm_get_info(const lbm_grid *g, lbm_info *out)
{
    if (!g || !out)
        return fail(const_cast<lbm_grid *>(g), LBM_E_INVALID, "null argument");
    std::memset(out, 0, sizeof *out);
    out->levels = g->L;
    out->block_edge = g->B;
    out->storage = g->d.storage;
    for (int l = 0; l < (int)g->lv.size(); ++l) {
        out->blocks[l] = g->lv[l].nb;
        out->active_cells[l] = g->lv[l].leaf_cells;
        out->updated_cells[l] = g->lv[l].updated_cells;
        out->collided_cells[l] = g->lv[l].collided_cells;
        out->omega1[l] = g->lv[l].om1;
    }
    out->links = g->n_links;
    out->branches = (int32_t)g->branches.size();
    out->height = g->H;
    out->area_x = g->area_x;
    out->nu_finest = g->nu_f;
    out->device_bytes = g->device_bytes;
    out->tile_cells = g->tile;
    out->threads = g->threads;
    out->occ_even = g->occ_even;
    out->occ_odd = g->occ_odd;
    out->persist_wgs = persist_grid_size(g);
    out->xcd_group = g->xcd_group;
    out->wall_clock_khz = g->wall_khz;
    out->persist_wait_ticks = g->persist_wait_ticks;
    bool pg = false;
    for (const lbm_grid::StepGraph &sg : g->graphs)
        pg = pg || (sg.d_phases && sg.exec);
    out->persist_graph = pg ? 1 : 0;
    return LBM_OK;
}

// element addresses of the cells a level holds (leaf and refined blocks), in
// box order, with their box positions, for state transfer
static void level_dense_cells(const lbm_grid *g, int l, std::vector<uint32_t> &cells, std::vector<int64_t> &pos)
{
    const DevLevel &v = g->lv[l];
    const int B = g->B;
    cells.clear();
    pos.clear();
    // only the stored block box can hold cells
    const int x0 = v.box_o[0] * B, y0 = v.box_o[1] * B, z0 = v.box_o[2] * B;
    const int x1 = x0 + v.box_n[0] * B, y1 = y0 + v.box_n[1] * B, z1 = z0 + v.box_n[2] * B;
    for (int z = z0; z < z1; ++z)
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) {
                const int8_t kind = v.block_kind(x / B, y / B, z / B);
                if (kind != 1 && kind != 2)
                    continue;
                cells.push_back((uint32_t)level_cell_address(v, B, x, y, z));
                pos.push_back((int64_t)x + (int64_t)v.nx * ((int64_t)y + (int64_t)v.ny * z));
            }
}

static lbm_status with_cells(lbm_grid *g, int l, std::vector<uint32_t> &cells, std::vector<int64_t> &pos,
                             uint32_t **d_cells)
{
    level_dense_cells(g, l, cells, pos);
    void *p = nullptr;
    HIPX(g, hipMalloc(&p, sizeof(uint32_t) * std::max<size_t>(cells.size(), 1)));
    *d_cells = (uint32_t *)p;
    HIPX(g, hipMemcpy(p, cells.data(), sizeof(uint32_t) * cells.size(), hipMemcpyHostToDevice));
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_grid *g, int32_t level, double *f)
{
    if (!g || !f)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (lbm_status ps = check_persistent(g); ps != LBM_OK)
        return ps;
    if (lbm_status pi = prepare_inlet(g); pi != LBM_OK)
        return pi;
    if (level < 0 || level >= g->L)
        return fail(g, LBM_E_INVALID, "level out of range");
    HIPX(g, hipStreamSynchronize(g->stream));
    std::vector<uint32_t> cells;
    std::vector<int64_t> pos;
    uint32_t *dc = nullptr;
    lbm_status st = with_cells(g, level, cells, pos, &dc);
    if (st != LBM_OK)
        return st;
    const size_t n = cells.size();
    double *dout = nullptr;
    HIPX(g, hipMalloc((void **)&dout, sizeof(double) * 27 * std::max<size_t>(n, 1)));
    DevLevel &v = g->lv[level];
    CollideArgs a = collide_args(g, level);
    HIPX(g, launch_gather(g->B, g->d.storage, (int)(v.steps & 1), a, dc, (int)n, dout, n, g->stream));
    std::vector<double> h(27 * n);
    HIPX(g, hipMemcpyAsync(h.data(), dout, sizeof(double) * h.size(), hipMemcpyDeviceToHost, g->stream));
    HIPX(g, hipStreamSynchronize(g->stream));
    (void)hipFree(dout);
    (void)hipFree(dc);
    const size_t N = (size_t)v.nx * v.ny * v.nz;
    for (size_t i = 0; i < 27 * N; ++i)
        f[i] = NAN;
    for (size_t t = 0; t < n; ++t)
        for (int i = 0; i < 27; ++i)
            f[i * N + pos[t]] = h[i * n + t];
    return LBM_OK;
}

lbm_status lbm_get_cells(lbm_grid *g, int32_t level, int64_t n, const int64_t *cells, double *f)
{
    if (!g || (n > 0 && (!cells || !f)) || n < 0)
        return fail(g, LBM_E_INVALID, "null argument or negative count");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (lbm_status ps = check_persistent(g); ps != LBM_OK)
        return ps;
    if (lbm_status pi = prepare_inlet(g); pi != LBM_OK)
        return pi;
    if (level < 0 || level >= g->L)
        return fail(g, LBM_E_INVALID, "level out of range");
    if (n > (int64_t)1 << 26)
        return fail(g, LBM_E_INVALID, "more than 2^26 cells in one call");
    const DevLevel &v = g->lv[level];
    const int B = g->B;
    const int64_t N = (int64_t)v.nx * v.ny * v.nz;
    std::vector<uint32_t> addr;
    std::vector<int64_t> pos;
    for (int64_t k = 0; k < n; ++k) {
        for (int i = 0; i < 27; ++i)
            f[i * n + k] = NAN;
        const int64_t c = cells[k];
        if (c < 0 || c >= N)
            continue;
        const int x = (int)(c % v.nx), y = (int)((c / v.nx) % v.ny), z = (int)(c / ((int64_t)v.nx * v.ny));
        const int8_t kind = v.block_kind(x / B, y / B, z / B);
        if (kind != 1 && kind != 2)
            continue;
        addr.push_back((uint32_t)level_cell_address(v, B, x, y, z));
        pos.push_back(k);
    }
    if (addr.empty())
        return LBM_OK;
    HIPX(g, hipStreamSynchronize(g->stream));
    const size_t m = addr.size();
    uint32_t *dc = nullptr;
    double *dout = nullptr;
    HIPX(g, hipMalloc((void **)&dc, sizeof(uint32_t) * m));
    if (hipMalloc((void **)&dout, sizeof(double) * 27 * m) != hipSuccess) {
        (void)hipFree(dc);
        return fail(g, LBM_E_DEVICE, "hipMalloc failed");
    }
    HIPX(g, hipMemcpyAsync(dc, addr.data(), sizeof(uint32_t) * m, hipMemcpyHostToDevice, g->stream));
    CollideArgs a = collide_args(g, level);
    HIPX(g, launch_gather(g->B, g->d.storage, (int)(v.steps & 1), a, dc, (int)m, dout, m, g->stream));
    std::vector<double> h(27 * m);
    HIPX(g, hipMemcpyAsync(h.data(), dout, sizeof(double) * h.size(), hipMemcpyDeviceToHost, g->stream));
    HIPX(g, hipStreamSynchronize(g->stream));
    (void)hipFree(dout);
    (void)hipFree(dc);
    for (size_t t = 0; t < m; ++t)
        for (int i = 0; i < 27; ++i)
            f[i * n + pos[t]] = h[i * m + t];
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_grid *g, int32_t level, const double *f)
{
    if (!g || !f)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (level < 0 || level >= g->L)
        return fail(g, LBM_E_INVALID, "level out of range");
    DevLevel &v = g->lv[level];
    if (v.steps & 1)
        return fail(g, LBM_E_STATE, "populations can be set only after an even number of level steps");
    HIPX(g, hipStreamSynchronize(g->stream));
    std::vector<uint32_t> cells;
    std::vector<int64_t> pos;
    uint32_t *dc = nullptr;
    lbm_status st = with_cells(g, level, cells, pos, &dc);
    if (st != LBM_OK)
        return st;
    const size_t n = cells.size();
    const size_t N = (size_t)v.nx * v.ny * v.nz;
    std::vector<double> h(27 * n);
    for (size_t t = 0; t < n; ++t)
        for (int i = 0; i < 27; ++i)
            h[i * n + t] = f[i * N + pos[t]];
    double *din = nullptr;
    HIPX(g, hipMalloc((void **)&din, sizeof(double) * std::max<size_t>(h.size(), 1)));
    HIPX(g, hipMemcpy(din, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
    HIPX(g, launch_scatter(g->d.storage, v.pop, v.dir_elems, dc, (int)n, din, n, g->stream));
    HIPX(g, hipStreamSynchronize(g->stream));
    (void)hipFree(din);
    (void)hipFree(dc);
    return LBM_OK;
}

lbm_status lbm_get_fields(lbm_grid *g, int32_t level, double *rho, double *u)
{
    if (!g || !rho || !u)
        return fail(g, LBM_E_INVALID, "null argument");
    if (level < 0 || level >= g->L)
        return fail(g, LBM_E_INVALID, "level out of range");
    const DevLevel &v = g->lv[level];
    const size_t N = (size_t)v.nx * v.ny * v.nz;
    std::vector<double> f(27 * N);
    lbm_status st = lbm_get_populations(g, level, f.data());
    if (st != LBM_OK)
        return st;
    for (size_t c = 0; c < N; ++c) {
        double r = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < 27; ++i) {
            const double val = f[i * N + c];
            r += val;
            j[0] += (i % 3 - 1) * val;
            j[1] += ((i / 3) % 3 - 1) * val;
            j[2] += (i / 9 - 1) * val;
        }
        rho[c] = r;
        for (int a = 0; a < 3; ++a)
            u[3 * c + a] = j[a] / r;
    }
    return LBM_OK;
}

lbm_status lbm_get_solid(lbm_grid *g, uint8_t *solid)
{
    if (!g || !solid)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    g->solid.expand(solid);
    return LBM_OK;
}

lbm_status lbm_get_links(lbm_grid *g, int64_t cap, int64_t *cell, int8_t *dir, double *q, int32_t *branch,
                         int64_t *n)
{
    if (!g || !n)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    *n = (int64_t)g->links.size();
    const int64_t m = std::min<int64_t>(cap, *n);
    for (int64_t t = 0; t < m; ++t) {
        if (cell) cell[t] = g->links[t].cell;
        if (dir) dir[t] = g->links[t].dir;
        if (q) q[t] = g->links[t].q;
        if (branch) branch[t] = g->links[t].branch;
    }
    return LBM_OK;
}

lbm_status lbm_inflow_modes(uint64_t seed, int32_t n_modes, double intensity, double length, double u_in,
                           double dx, double *out, double *k_e)
{
    if (!out || n_modes <= 0 || !(intensity > 0.0) || !(length > 0.0) || !(u_in > 0.0) || !(dx > 0.0))
        return fail(nullptr, LBM_E_INVALID, "bad inflow-mode arguments");
    InflowModes m;
    build_inflow_modes(seed, n_modes, intensity, length, u_in, dx, m);
    size_t o = 0;
    for (const std::vector<double> *v : {&m.kx, &m.ky, &m.kz, &m.sx, &m.sy, &m.sz, &m.psi, &m.amp})
        for (double x : *v)
            out[o++] = x;
    if (k_e)
        *k_e = m.k_e;
    return LBM_OK;
}

lbm_status lbm_plan_levels(const lbm_grid_desc *d, const lbm_branch *b, int32_t n_b, const lbm_refine_desc *refine,
                           lbm_plan *out, int8_t *const *maps)
{
    if (!d || !out)
        return fail(nullptr, LBM_E_INVALID, "null argument");
    std::string msg;
    if (check_desc(d, &msg) != LBM_OK || check_branches(*d, b, n_b, &msg) != LBM_OK)
        return fail(nullptr, LBM_E_INVALID, msg);
    if (d->levels > 1 && !refine)
        return fail(nullptr, LBM_E_INVALID, "refinement bands required when levels > 1");
    SolidMask solid;
    std::vector<HostLink> links;
    voxelize(b, n_b, d->nx, d->ny, d->nz, solid);
    build_links(b, n_b, solid, links);
    std::vector<DevLevel> lv;
    AmrPlan plan;
    const int B = d->block_edge;
    const lbm_status st = build_levels(*d, B, d->levels, b, n_b, refine, solid, lv, plan, &msg);
    if (st != LBM_OK)
        return fail(nullptr, st, msg);
    std::memset(out, 0, sizeof *out);
    out->levels = d->levels;
    out->block_edge = B;
    out->links = (int64_t)links.size();
    out->solid_cells = solid.count();
    const size_t eb = storage_bytes(d->storage);
    for (int l = 0; l < d->levels; ++l) {
        const DevLevel &v = lv[l];
        out->blocks[l] = v.nb;
        out->leaf_cells[l] = v.leaf_cells;
        out->collided_cells[l] = v.collided_cells;
        out->updated_cells[l] = v.updated_cells;
        out->work_blocks[l] = (int64_t)v.h_work.size();
        const int unit = v.dense ? DENSE_TILE : B * B * B, slice = v.dense ? DENSE_TILE : B * B;
        for (const uint2 &w : v.h_work) {
            for (int t = 0; t < unit / slice; ++t) {
                bool any = w.y == FULL_MASK;
                for (int c = t * slice; c < (t + 1) * slice && !any; ++c)
                    any = (v.h_masks[(size_t)w.y * (unit / 32) + (c >> 5)] >> (c & 31)) & 1u;
                out->work_tiles[l] += any;
            }
        }
        out->pop_bytes += (int64_t)bound_share(level_dir_elems(v, B, d->storage) * 27 * eb);
        out->lattice[l][0] = v.nbx;
        out->lattice[l][1] = v.nby;
        out->lattice[l][2] = v.nbz;
        if (maps && maps[l])
            v.expand_map(maps[l]);
    }
    return LBM_OK;
}

lbm_status lbm_plan_phases(const lbm_grid_desc *d, const lbm_branch *b, int32_t n_b, const lbm_refine_desc *refine,
                           int32_t groups, int32_t coarse_steps, lbm_phase_info *out, int32_t cap, int32_t *n)
{
    if (!d || !n || groups <= 0 || coarse_steps <= 0 || (!out && cap > 0))
        return fail(nullptr, LBM_E_INVALID, "bad arguments");
    std::string msg;
    lbm_grid_desc dd = *d;
    dd.flags &= ~LBM_F_PERSISTENT;
    if (check_desc(&dd, &msg) != LBM_OK || check_branches(dd, b, n_b, &msg) != LBM_OK)
        return fail(nullptr, LBM_E_INVALID, msg);
    if (dd.levels > 1 && !refine)
        return fail(nullptr, LBM_E_INVALID, "refinement bands required when levels > 1");
    if (dd.turb_intensity > 0.0)
        return fail(nullptr, LBM_E_INVALID, "turbulent inflow is not available in the persistent form");
    // the host state lbm_create_grid and lbm_set_geometry build, without
    // device memory: the recorded phases carry null device pointers
    lbm_grid g;
    g.d = dd;
    if (g.d.drag_every == 0)
        g.d.drag_every = 1;
    g.B = dd.block_edge;
    g.L = dd.levels;
    g.tile = g.B * g.B;
    g.branches.assign(b, b + n_b);
    g.H = tree_height(b, n_b);
    g.nu_f = dd.nu > 0.0 ? dd.nu : dd.u_in * g.H / dd.re_h;
    voxelize(b, n_b, dd.nx, dd.ny, dd.nz, g.solid);
    build_links(b, n_b, g.solid, g.links);
    lbm_status st = build_levels(dd, g.B, g.L, b, n_b, refine, g.solid, g.lv, g.amr, &msg);
    if (st != LBM_OK)
        return fail(nullptr, st, msg);
    for (int l = 0; l < g.L; ++l) {
        nu_to_level_omega(g.nu_f, g.L, l, &g.lv[l].om1);
        g.lv[l].n_work = (int)g.lv[l].h_work.size();
        g.lv[l].n_leaf = (int)g.lv[l].h_leaf.size();
    }
    g.n_links = (int)g.links.size();
    g.nseg = n_b + 1;
    std::vector<int> per_seg(g.nseg, 0);
    for (const HostLink &Lk : g.links)
        per_seg[Lk.branch < 0 ? n_b : Lk.branch]++;
    g.npieces = 0;
    for (int c : per_seg)
        g.npieces += (c + LINK_PIECE - 1) / LINK_PIECE;
    std::vector<Phase> ph;
    std::vector<int> step_of;
    g.rec = &ph;
    for (int s2 = 0; s2 < coarse_steps; ++s2) {
        if ((st = coarse_step(&g)) != LBM_OK) {
            g.rec = nullptr;
            return st;
        }
        step_of.resize(ph.size(), s2);
    }
    g.rec = nullptr;
    for (size_t i = 0; i < ph.size() && (int32_t)i < cap; ++i) {
        const Phase &p = ph[i];
        out[i].kind = p.kind;
        out[i].step = step_of[i];
        out[i].items = p.items;
        out[i].chunk = persist_chunk(p.items, groups);
        out[i].chunks = (p.items + out[i].chunk - 1) / out[i].chunk;
    }
    *n = (int32_t)ph.size();
    return LBM_OK;
}

lbm_status lbm_get_block_map(lbm_grid *g, int32_t level, int8_t *map)
{
    if (!g || !map)
        return fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return fail(g, LBM_E_STATE, "set_geometry first");
    if (level < 0 || level >= g->L)
        return fail(g, LBM_E_INVALID, "level out of range");
    g->lv[level].expand_map(map);
    return LBM_OK;
}

}  // extern "C"
