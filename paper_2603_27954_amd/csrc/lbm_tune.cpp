// Tile autotuner of the collide kernel: times each (threads, cells per
// work-group) candidate over whole coarse steps on the live grid, keeps the
// fastest and restores the grid state afterwards.  Choices are cached in a
// text file keyed by the grid shape.
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

bool cache_lookup(const char *path, const std::string &key, int *threads, int *tile)
{
    if (!path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char k[200];
    int t, c;
    bool hit = false;
    while (std::fscanf(f, "%199s %d %d", k, &t, &c) == 3)
        if (key == k) {
            *threads = t;
            *tile = c;
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
    int bt = 0, bc = 0;
    if (cache_lookup(cache_path, key, &bt, &bc)) {
        g->threads = bt;
        g->tile = bc;
        return LBM_OK;
    }
    const size_t eb = grid_storage_bytes(g->d.storage);
    // back up the evolving state
    std::vector<void *> backup(g->L, nullptr);
    for (int l = 0; l < g->L; ++l) {
        const size_t bytes = g->lv[l].dir_elems * 27 * eb;
        if (hipMalloc(&backup[l], bytes) != hipSuccess) {
            for (void *p : backup)
                if (p) (void)hipFree(p);
            return grid_fail(g, LBM_E_NOMEM, "autotune backup allocation failed");
        }
        (void)hipMemcpyAsync(backup[l], g->lv[l].pop, bytes, hipMemcpyDeviceToDevice, g->stream);
    }
    std::vector<double> acc(3 * (size_t)g->nseg + 3);
    (void)hipMemcpyAsync(acc.data(), g->d_acc_branch, sizeof(double) * 3 * g->nseg, hipMemcpyDeviceToHost, g->stream);
    (void)hipMemcpyAsync(acc.data() + 3 * g->nseg, g->d_acc_total, sizeof(double) * 3, hipMemcpyDeviceToHost, g->stream);
    (void)hipStreamSynchronize(g->stream);
    std::vector<int64_t> steps(g->L);
    for (int l = 0; l < g->L; ++l)
        steps[l] = g->lv[l].steps;
    const int64_t cs = g->coarse_steps, fs = g->finest_steps, sm = g->samples, rc = g->ring_count;
    const int old_threads = g->threads, old_tile = g->tile;

    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int cells = g->B * g->B * g->B;
    float best = 1e30f;
    int best_t = old_threads, best_c = old_tile;
    lbm_status st = LBM_OK;
    for (int threads : {64, 128, 256}) {
        for (int tile = cells; tile >= threads && tile >= cells / 16; tile /= 2) {
            g->threads = threads;
            g->tile = tile;
            const int reps = 4;
            st = grid_coarse_step(g);  // warm-up (and even/odd balance with reps even)
            if (st == LBM_OK)
                st = grid_coarse_step(g);
            (void)hipEventRecord(e0, g->stream);
            for (int r = 0; r < reps && st == LBM_OK; ++r)
                st = grid_coarse_step(g);
            (void)hipEventRecord(e1, g->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (st != LBM_OK)
                break;
            if (ms < best) {
                best = ms;
                best_t = threads;
                best_c = tile;
            }
        }
        if (st != LBM_OK)
            break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // restore
    for (int l = 0; l < g->L; ++l) {
        (void)hipMemcpyAsync(g->lv[l].pop, backup[l], g->lv[l].dir_elems * 27 * eb, hipMemcpyDeviceToDevice, g->stream);
        g->lv[l].steps = steps[l];
    }
    (void)hipMemcpyAsync(g->d_acc_branch, acc.data(), sizeof(double) * 3 * g->nseg, hipMemcpyHostToDevice, g->stream);
    (void)hipMemcpyAsync(g->d_acc_total, acc.data() + 3 * g->nseg, sizeof(double) * 3, hipMemcpyHostToDevice, g->stream);
    (void)hipStreamSynchronize(g->stream);
    for (void *p : backup)
        (void)hipFree(p);
    g->coarse_steps = cs;
    g->finest_steps = fs;
    g->samples = sm;
    g->ring_count = rc;
    if (st != LBM_OK) {
        g->threads = old_threads;
        g->tile = old_tile;
        return st;
    }
    g->threads = best_t;
    g->tile = best_c;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%s %d %d\n", key.c_str(), best_t, best_c);
            std::fclose(f);
        }
    }
    return LBM_OK;
}
