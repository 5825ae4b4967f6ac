// Grid handle of the C ABI (internal layout).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbmtree.h"
#include "lbm_geometry.h"
#include "lbm_internal.h"
#include "lbm_levels.h"

using lbm::AmrPlan;
using lbm::DevLevel;
using lbm::HostLink;


struct lbm_grid {
    lbm_grid_desc d{};
    std::string err;
    int state = 0;  // 0 created, 1 geometry set
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int B = 16, L = 1;
    double nu_f = 0.0, H = 0.0, area_x = 0.0;
    std::vector<lbm_branch> branches;
    lbm::SolidMask solid;
    std::vector<HostLink> links;  // (cell, dir) order
    std::vector<DevLevel> lv;
    AmrPlan amr;
    // device link table (sorted by branch)
    uint32_t *d_af = nullptr, *d_ap = nullptr, *d_am = nullptr;
    uint8_t *d_dir = nullptr;
    float *d_q = nullptr;
    int n_links = 0;
    int nseg = 0;                   // branches + 1 (links owned by no branch)
    int *d_pstart = nullptr;        // link pieces: npieces + 1 offsets
    int *d_segp = nullptr;          // pieces of segment s: segp[s] .. segp[s + 1]
    int npieces = 0;
    double *d_piece_sum = nullptr;  // 3 per piece
    float *d_lforce = nullptr;
    double *d_sample = nullptr, *d_acc_branch = nullptr, *d_acc_total = nullptr, *d_ring = nullptr;
    unsigned *d_counter = nullptr;
    double *d_mass = nullptr;
    std::vector<int32_t> link_perm;  // device order -> (cell, dir) order
    // wall friction (LBM_F_FRICTION): axis faces between fluid and solid cells,
    // sorted by branch and cut into pieces for the FP64 reduction
    int n_fric = 0, fric_npieces = 0;
    uint32_t *d_fa0 = nullptr, *d_fa1 = nullptr;
    float *d_fq = nullptr;
    float4 *d_fnw = nullptr;
    float *d_fforce = nullptr;
    int *d_fpstart = nullptr, *d_fsegp = nullptr;
    double *d_fpiece_sum = nullptr, *d_facc_branch = nullptr, *d_facc_total = nullptr;
    unsigned *d_fcounter = nullptr;
    int64_t samples = 0, ring_count = 0;
    int64_t coarse_steps = 0, finest_steps = 0;
    int threads = 256, tile = 0;
    int occ_even = 0, occ_odd = 0;  // waves per SIMD cap of the collide kernel (0 = none)
    int xcd_group = 1;              // tiles per XCD run of the collide kernels
    size_t device_bytes = 0;
    std::vector<void *> allocs;
    void *bound = nullptr;          // caller-owned memory holding the populations (lbm_bind_memory)
    size_t bound_bytes = 0;
    unsigned long long *d_ring_pos = nullptr;  // device copy of ring_count (slot of the next sample)
    // synthetic turbulent inflow (coarsest level's inlet)
    bool turb = false;
    int n_modes = 0;
    double turb_ke = 0.0;
    double *d_modes = nullptr;             // 8 n_modes doubles
    float *d_in_prev = nullptr, *d_in_cur = nullptr;  // 3 floats per inlet cell
    unsigned long long *d_tick = nullptr;  // odd level-0 steps done (= level-0 steps / 2)
    // Captured coarse steps.  A coarse step's launches depend on the host
    // state only through the A-A parity of every level and the phase of the
    // force sampling, so one graph per such key is replayed, and the host
    // counters advance by the deltas recorded at capture.
    // A persistent plan holds the coarse step's phase list on the device and
    // is launched directly or from a graph that captured that launch.
    struct StepGraph {
        uint64_t key;
        hipGraphExec_t exec;          // null: persistent plan launched directly
        lbm::Phase *d_phases;         // persistent plans only
        unsigned *d_ctr;              // claim / finish counters of the phases
        int n_phases;
        int64_t level_steps[LBM_MAX_LEVELS];
        int64_t coarse, finest, samples, ring;
    };
    std::vector<StepGraph> graphs;
    std::vector<lbm::Phase> *rec = nullptr;  // recording a coarse step as phases
    unsigned *d_abort = nullptr;   // set by a persistent launch whose bounded wait expired
    int persist_grid = 0;       // work-groups of the persistent launch (0 = all resident)
    int persist_max = 0, cus = 0;
    unsigned long long persist_wait_ticks = 0;  // time limit of one wait in the persistent launch
    int wall_khz = 0;                           // the device's constant real-time clock
    bool persist_failed = false;   // a wait expired: the state is undefined
    // per-kernel timing (event pairs, kind 0 collide, 1 links)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_pairs;  // (start index, kind)

    ~lbm_grid()
    {
        for (StepGraph &sg : graphs) {
            if (sg.exec)
                (void)hipGraphExecDestroy(sg.exec);
            if (sg.d_phases)
                (void)hipFree(sg.d_phases);
            if (sg.d_ctr)
                (void)hipFree(sg.d_ctr);
        }
        for (hipEvent_t e : ev_pool)
            (void)hipEventDestroy(e);
        for (void *p : allocs)
            (void)hipFree(p);
        if (own_stream && stream)
            (void)hipStreamDestroy(stream);
    }
};


namespace lbm {
lbm_status grid_fail(lbm_grid *g, lbm_status st, const std::string &msg);
CollideArgs grid_collide_args(lbm_grid *g, int l);
lbm_status grid_coarse_step(lbm_grid *g);
size_t grid_storage_bytes(int storage);
// records an event on the grid stream when timing is on; returns its index or -1
int grid_timing_mark(lbm_grid *g);
// drops every captured coarse step (launch shapes or state changed)
void grid_graphs_clear(lbm_grid *g);
// writes the host-held counters the kernels read from device memory (ring
// position, inflow time) after the host state was restored (synchronous)
lbm_status grid_sync_device_counters(lbm_grid *g);
}  // namespace lbm
