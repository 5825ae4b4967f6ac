// Autotuner of the collide kernel: times candidate launch shapes over whole
// coarse steps on the live grid -- work-group size and cells per work-group of
// the block levels, a cap on resident waves per SIMD (through reserved LDS)
// for the even and the odd step, and the run length of tiles per XCD -- keeps
// the fastest and restores the grid state afterwards.  Choices are cached in a text file keyed by the grid
// shape.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_grid.h"

using namespace lbm;

namespace {

std::string tune_key(const lbm_grid *g)
{
    char k[160];
    std::snprintf(k, sizeof k, "nx%d_ny%d_nz%d_B%d_L%d_S%d_links%d", g->d.nx, g->d.ny, g->d.nz, g->B, g->L,
                  g->d.storage, g->n_links);
    return k;
}

struct Choice {
    int threads, tile, occ_even, occ_odd, xcd;
};

bool cache_lookup(const char *path, const std::string &key, Choice *c)
{
    if (!path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char k[200];
    Choice v{};
    bool hit = false;
    while (std::fscanf(f, "%199s %d %d %d %d %d", k, &v.threads, &v.tile, &v.occ_even, &v.occ_odd, &v.xcd) == 6)
        if (key == k) {
            *c = v;
            hit = true;
        }
    std::fclose(f);
    return hit;
}

}  // namespace

extern "C" lbm_status lbm_autotune(lbm_grid *g, const char *cache_path)
{
    if (!g)
        return grid_fail(nullptr, LBM_E_INVALID, "null grid");
    if (g->state != 1)
        return grid_fail(g, LBM_E_STATE, "set_geometry first");
    const std::string key = tune_key(g);
    Choice cached{};
    if (cache_lookup(cache_path, key, &cached)) {
        // the entry must be a shape the search could have chosen: a tile
        // that divides a block into whole wavefronts, 64 to 256 threads
        const int cells = g->B * g->B * g->B;
        if (cached.threads < 64 || cached.threads > 256 || cached.threads % 64 != 0 || cached.tile < 64 ||
            cached.tile > cells || cells % cached.tile != 0)
            return grid_fail(g, LBM_E_INVALID, "tune cache entry for " + key + " has an invalid tile or work-group");
        grid_graphs_clear(g);
        g->threads = cached.threads;
        g->tile = cached.tile;
        g->occ_even = cached.occ_even;
        g->occ_odd = cached.occ_odd;
        g->xcd_group = cached.xcd;
        return LBM_OK;
    }
    const size_t eb = grid_storage_bytes(g->d.storage);
    // back up the evolving state
    std::vector<void *> backup(g->L, nullptr);
    auto free_backup = [&]() {
        for (void *p : backup)
            if (p) (void)hipFree(p);
    };
    hipError_t ce = hipSuccess;  // first failing copy
    auto keep = [&](hipError_t e) {
        if (ce == hipSuccess) ce = e;
    };
    for (int l = 0; l < g->L; ++l) {
        const size_t bytes = g->lv[l].dir_elems * 27 * eb;
        if (hipMalloc(&backup[l], bytes) != hipSuccess) {
            free_backup();
            return grid_fail(g, LBM_E_NOMEM, "autotune backup allocation failed");
        }
        keep(hipMemcpyAsync(backup[l], g->lv[l].pop, bytes, hipMemcpyDeviceToDevice, g->stream));
    }
    std::vector<double> acc(3 * (size_t)g->nseg + 3);
    keep(hipMemcpyAsync(acc.data(), g->d_acc_branch, sizeof(double) * 3 * g->nseg, hipMemcpyDeviceToHost, g->stream));
    keep(hipMemcpyAsync(acc.data() + 3 * g->nseg, g->d_acc_total, sizeof(double) * 3, hipMemcpyDeviceToHost,
                        g->stream));
    // the candidates' runs write force samples into the ring: keep its contents
    std::vector<double> ring(3 * (size_t)RING);
    keep(hipMemcpyAsync(ring.data(), g->d_ring, sizeof(double) * ring.size(), hipMemcpyDeviceToHost, g->stream));
    std::vector<double> facc(3 * (size_t)g->nseg + 3);
    if (g->d_facc_total) {
        keep(hipMemcpyAsync(facc.data(), g->d_facc_branch, sizeof(double) * 3 * g->nseg, hipMemcpyDeviceToHost,
                            g->stream));
        keep(hipMemcpyAsync(facc.data() + 3 * g->nseg, g->d_facc_total, sizeof(double) * 3, hipMemcpyDeviceToHost,
                            g->stream));
    }
    keep(hipStreamSynchronize(g->stream));
    if (ce != hipSuccess) {  // nothing has been run yet: the grid is unchanged
        free_backup();
        return grid_fail(g, LBM_E_DEVICE, std::string("autotune state backup: ") + hipGetErrorString(ce));
    }
    std::vector<int64_t> steps(g->L);
    for (int l = 0; l < g->L; ++l)
        steps[l] = g->lv[l].steps;
    const int64_t cs = g->coarse_steps, fs = g->finest_steps, sm = g->samples, rc = g->ring_count;
    const Choice old{g->threads, g->tile, g->occ_even, g->occ_odd, g->xcd_group};

    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    lbm_status st = LBM_OK;
    // times whole coarse steps (both parities) of candidate c: the fastest of
    // five runs of `reps` steps, so that one slow run (clock or power state)
    // does not decide the choice; `reps` makes each run last at least 25 ms
    int reps = 8;
    auto time_choice = [&](const Choice &c, float *ms) -> lbm_status {
        g->threads = c.threads;
        g->tile = c.tile;
        g->occ_even = c.occ_even;
        g->occ_odd = c.occ_odd;
        g->xcd_group = c.xcd;
        lbm_status s2 = grid_coarse_step(g);
        if (s2 == LBM_OK)
            s2 = grid_coarse_step(g);
        *ms = 1e30f;
        for (int rep = 0; rep < 5 && s2 == LBM_OK; ++rep) {
            (void)hipEventRecord(e0, g->stream);
            for (int r = 0; r < reps && s2 == LBM_OK; ++r)
                s2 = grid_coarse_step(g);
            (void)hipEventRecord(e1, g->stream);
            (void)hipEventSynchronize(e1);
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, e0, e1);
            *ms = std::min(*ms, t);
        }
        return s2;
    };
    Choice best = old;
    float best_ms = 1e30f;
    {
        float ms = 0.0f;
        st = time_choice(old, &ms);
        if (st == LBM_OK && ms > 0.0f)
            reps = std::min(64, std::max(8, (int)(25.0f * 8 / ms))) & ~1;  // even: both parities alike
    }
    // search in passes: block tiles (refined levels); the occupancy cap of the
    // even collide kernel; the odd kernel's cap jointly with the XCD run length
    // (the best cap depends on the tile order); the even cap again
    const int cells = g->B * g->B * g->B;
    std::vector<Choice> cand;
    if (g->L > 1)
        for (int threads : {64, 128, 256})
            for (int tile = cells; tile >= threads && tile >= cells / 16; tile /= 2)
                cand.push_back({threads, tile, best.occ_even, best.occ_odd, best.xcd});
    else
        cand.push_back(best);
    for (int pass = 0; pass < 4 && st == LBM_OK; ++pass) {
        if (pass == 1 || pass == 3) {
            cand.clear();
            for (int occ : {0, 2, 3, 4, 6})
                cand.push_back({best.threads, best.tile, occ, best.occ_odd, best.xcd});
        } else if (pass == 2) {
            cand.clear();
            for (int occ : {0, 2, 3, 4})
                for (int k : {1, 4, 16, 64, 256})
                    cand.push_back({best.threads, best.tile, best.occ_even, occ, k});
        }
        for (const Choice &c : cand) {
            float ms = 0.0f;
            st = time_choice(c, &ms);
            if (st != LBM_OK)
                break;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // restore
    for (int l = 0; l < g->L; ++l) {
        keep(hipMemcpyAsync(g->lv[l].pop, backup[l], g->lv[l].dir_elems * 27 * eb, hipMemcpyDeviceToDevice,
                            g->stream));
        g->lv[l].steps = steps[l];
    }
    keep(hipMemcpyAsync(g->d_acc_branch, acc.data(), sizeof(double) * 3 * g->nseg, hipMemcpyHostToDevice, g->stream));
    keep(hipMemcpyAsync(g->d_acc_total, acc.data() + 3 * g->nseg, sizeof(double) * 3, hipMemcpyHostToDevice,
                        g->stream));
    keep(hipMemcpyAsync(g->d_ring, ring.data(), sizeof(double) * ring.size(), hipMemcpyHostToDevice, g->stream));
    if (g->d_facc_total) {
        keep(hipMemcpyAsync(g->d_facc_branch, facc.data(), sizeof(double) * 3 * g->nseg, hipMemcpyHostToDevice,
                            g->stream));
        keep(hipMemcpyAsync(g->d_facc_total, facc.data() + 3 * g->nseg, sizeof(double) * 3, hipMemcpyHostToDevice,
                            g->stream));
    }
    keep(hipStreamSynchronize(g->stream));
    free_backup();
    if (ce != hipSuccess && st == LBM_OK)
        st = grid_fail(g, LBM_E_DEVICE, std::string("autotune state restore: ") + hipGetErrorString(ce));
    g->coarse_steps = cs;
    g->finest_steps = fs;
    g->samples = sm;
    g->ring_count = rc;
    grid_graphs_clear(g);
    if (st == LBM_OK)
        st = grid_sync_device_counters(g);
    const Choice use = st == LBM_OK ? best : old;
    g->threads = use.threads;
    g->tile = use.tile;
    g->occ_even = use.occ_even;
    g->occ_odd = use.occ_odd;
    g->xcd_group = use.xcd;
    if (st != LBM_OK)
        return st;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), use.threads, use.tile, use.occ_even, use.occ_odd,
                         use.xcd);
            std::fclose(f);
        }
    }
    return LBM_OK;
}
