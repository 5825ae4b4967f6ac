// Checkpoints, tile autotuning and the host-side collision probe of
// liblbmtree (C ABI in include/lbmtree.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_device.h"
#include "lbm_grid.h"

using namespace lbm;

namespace {

const uint64_t MAGIC = 0x34544B43544D424CULL;  // checkpoint tag (format 4: up to LBM_MAX_LEVELS levels)

struct CkptHeader {
    uint64_t magic;
    int32_t nx, ny, nz, B, L, storage;
    int64_t coarse_steps, finest_steps, samples, ring_count;
    int64_t steps[LBM_MAX_LEVELS];
    int64_t dir_elems[LBM_MAX_LEVELS];
    int32_t nseg;
};

bool wr(FILE *f, const void *p, size_t n) { return fwrite(p, 1, n, f) == n; }
bool rd(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

}  // namespace

extern "C" {

lbm_status lbm_save(lbm_grid *g, const char *path)
{
    if (!g || !path)
        return grid_fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return grid_fail(g, LBM_E_STATE, "set_geometry first");
    for (int l = 0; l < g->L; ++l)
        if (g->lv[l].steps & 1)
            return grid_fail(g, LBM_E_STATE, "checkpoints are taken after an even number of steps on every level");
    if (hipStreamSynchronize(g->stream) != hipSuccess)
        return grid_fail(g, LBM_E_DEVICE, "hipStreamSynchronize failed");
    CkptHeader h{};
    h.magic = MAGIC;
    h.nx = g->d.nx, h.ny = g->d.ny, h.nz = g->d.nz, h.B = g->B, h.L = g->L, h.storage = g->d.storage;
    h.coarse_steps = g->coarse_steps, h.finest_steps = g->finest_steps;
    h.samples = g->samples, h.ring_count = g->ring_count;
    for (int l = 0; l < g->L; ++l) {
        h.steps[l] = g->lv[l].steps;
        h.dir_elems[l] = (int64_t)g->lv[l].dir_elems;
    }
    h.nseg = g->nseg;
    FILE *f = fopen(path, "wb");
    if (!f)
        return grid_fail(g, LBM_E_INVALID, std::string("cannot open ") + path);
    bool ok = wr(f, &h, sizeof h);
    const size_t eb = grid_storage_bytes(g->d.storage);
    for (int l = 0; l < g->L && ok; ++l) {
        std::vector<char> buf(g->lv[l].dir_elems * 27 * eb);
        ok = hipMemcpy(buf.data(), g->lv[l].pop, buf.size(), hipMemcpyDeviceToHost) == hipSuccess &&
             wr(f, buf.data(), buf.size());
    }
    std::vector<double> acc(3 * (size_t)g->nseg + 3);
    if (ok)
        ok = hipMemcpy(acc.data(), g->d_acc_branch, sizeof(double) * 3 * g->nseg, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(acc.data() + 3 * g->nseg, g->d_acc_total, sizeof(double) * 3, hipMemcpyDeviceToHost) == hipSuccess &&
             wr(f, acc.data(), sizeof(double) * acc.size());
    // the force-sample ring, so that lbm_drag_series after a load returns the
    // samples taken before the checkpoint
    std::vector<double> ring(3 * (size_t)RING);
    if (ok)
        ok = hipMemcpy(ring.data(), g->d_ring, sizeof(double) * ring.size(), hipMemcpyDeviceToHost) == hipSuccess &&
             wr(f, ring.data(), sizeof(double) * ring.size());
    // the friction accumulators (zero when friction is not sampled)
    std::vector<double> facc(3 * (size_t)g->nseg + 3, 0.0);
    if (ok && g->d_facc_total)
        ok = hipMemcpy(facc.data(), g->d_facc_branch, sizeof(double) * 3 * g->nseg, hipMemcpyDeviceToHost) ==
                 hipSuccess &&
             hipMemcpy(facc.data() + 3 * g->nseg, g->d_facc_total, sizeof(double) * 3, hipMemcpyDeviceToHost) ==
                 hipSuccess;
    if (ok)
        ok = wr(f, facc.data(), sizeof(double) * facc.size());
    ok = (fclose(f) == 0) && ok;
    return ok ? LBM_OK : grid_fail(g, LBM_E_DEVICE, "checkpoint write failed");
}

lbm_status lbm_load(lbm_grid *g, const char *path)
{
    if (!g || !path)
        return grid_fail(g, LBM_E_INVALID, "null argument");
    if (g->state != 1)
        return grid_fail(g, LBM_E_STATE, "set_geometry first (same geometry as the checkpoint)");
    FILE *f = fopen(path, "rb");
    if (!f)
        return grid_fail(g, LBM_E_INVALID, std::string("cannot open ") + path);
    CkptHeader h{};
    bool ok = rd(f, &h, sizeof h) && h.magic == MAGIC && h.nx == g->d.nx && h.ny == g->d.ny && h.nz == g->d.nz &&
              h.B == g->B && h.L == g->L && h.storage == g->d.storage && h.nseg == g->nseg;
    for (int l = 0; l < g->L && ok; ++l)
        ok = h.dir_elems[l] == (int64_t)g->lv[l].dir_elems;
    if (!ok) {
        fclose(f);
        return grid_fail(g, LBM_E_INVALID, "checkpoint does not match this grid");
    }
    const size_t eb = grid_storage_bytes(g->d.storage);
    (void)hipStreamSynchronize(g->stream);
    for (int l = 0; l < g->L && ok; ++l) {
        std::vector<char> buf(g->lv[l].dir_elems * 27 * eb);
        ok = rd(f, buf.data(), buf.size()) &&
             hipMemcpy(g->lv[l].pop, buf.data(), buf.size(), hipMemcpyHostToDevice) == hipSuccess;
        g->lv[l].steps = h.steps[l];
    }
    std::vector<double> acc(3 * (size_t)g->nseg + 3);
    ok = ok && rd(f, acc.data(), sizeof(double) * acc.size()) &&
         hipMemcpy(g->d_acc_branch, acc.data(), sizeof(double) * 3 * g->nseg, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g->d_acc_total, acc.data() + 3 * g->nseg, sizeof(double) * 3, hipMemcpyHostToDevice) == hipSuccess;
    std::vector<double> ring(3 * (size_t)RING);
    ok = ok && rd(f, ring.data(), sizeof(double) * ring.size()) &&
         hipMemcpy(g->d_ring, ring.data(), sizeof(double) * ring.size(), hipMemcpyHostToDevice) == hipSuccess;
    std::vector<double> facc(3 * (size_t)g->nseg + 3, 0.0);
    ok = ok && rd(f, facc.data(), sizeof(double) * facc.size());
    if (ok && g->d_facc_total)
        ok = hipMemcpy(g->d_facc_branch, facc.data(), sizeof(double) * 3 * g->nseg, hipMemcpyHostToDevice) ==
                 hipSuccess &&
             hipMemcpy(g->d_facc_total, facc.data() + 3 * g->nseg, sizeof(double) * 3, hipMemcpyHostToDevice) ==
                 hipSuccess;
    fclose(f);
    if (!ok)
        return grid_fail(g, LBM_E_DEVICE, "checkpoint read failed");
    g->coarse_steps = h.coarse_steps;
    g->finest_steps = h.finest_steps;
    g->samples = h.samples;
    g->ring_count = h.ring_count;
    return grid_sync_device_counters(g);
}

// Host probe of the FP32 collision used by the kernels (one cell, FP64 in/out
// as full populations).
lbm_status lbm_collide_cell_host(const double *f_in, double *f_out, double omega1, double omega2, int galilean)
{
    if (!f_in || !f_out)
        return grid_fail(nullptr, LBM_E_INVALID, "null argument");
    float g[NQ];
    for (int i = 0; i < NQ; ++i)
        g[i] = (float)(f_in[i] - (double)qw(i));
    collide(g, (float)omega1, (float)omega2, galilean != 0);
    for (int i = 0; i < NQ; ++i)
        f_out[i] = (double)g[i] + (double)qw(i);
    return LBM_OK;
}

lbm_status lbm_geometry_build(const lbm_branch *b, int32_t n_b, int32_t nx, int32_t ny, int32_t nz,
                              uint8_t *solid, int64_t cap, int64_t *cell, int8_t *dir, double *q,
                              int32_t *branch, int64_t *n_links, double *area_x)
{
    if (!b || n_b <= 0 || nx <= 0 || ny <= 0 || nz <= 0)
        return grid_fail(nullptr, LBM_E_INVALID, "bad geometry arguments");
    SolidMask s;
    voxelize(b, n_b, nx, ny, nz, s);
    std::vector<HostLink> links;
    build_links(b, n_b, s, links);
    if (solid)
        s.expand(solid);
    const int64_t m = std::min<int64_t>(cap, (int64_t)links.size());
    for (int64_t t = 0; t < m; ++t) {
        if (cell) cell[t] = links[t].cell;
        if (dir) dir[t] = links[t].dir;
        if (q) q[t] = links[t].q;
        if (branch) branch[t] = links[t].branch;
    }
    if (n_links)
        *n_links = (int64_t)links.size();
    if (area_x)
        *area_x = (double)frontal_area(s);
    return LBM_OK;
}

}  // extern "C"
