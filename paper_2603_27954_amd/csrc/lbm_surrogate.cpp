// Host side of the per-branch drag surrogate (C ABI in include/lbmtree.h):
// parameter initialisation, training loop, inference and the branch-wise drag
// sweep over many trees.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbmtree.h"
#include "lbm_geometry.h"
#include "lbm_grid.h"
#include "lbm_mlp.h"
#include "lbm_random.h"

using namespace lbm;

struct lbm_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    MlpDev d{};
    int chunk_cap = 0;        // partial-sum capacity in chunks
    int32_t *idx = nullptr;   // training permutation
    int64_t idx_cap = 0;
    int64_t adam_t = 0;
    float *scratch = nullptr;  // this device's static gradient workspace (not owned)
    std::vector<void *> allocs;

    ~lbm_mlp()
    {
        for (void *p : allocs)
            (void)hipFree(p);
        if (idx)
            (void)hipFree(idx);
        if (own_stream && stream)
            (void)hipStreamDestroy(stream);
    }
};

namespace {

lbm_status mfail(lbm_status st, const std::string &msg) { return grid_fail(nullptr, st, msg); }

#define MHIP(call)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return mfail(LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

template <typename T>
lbm_status malloc_dev(lbm_mlp *m, T **p, size_t count)
{
    void *q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
        return mfail(LBM_E_NOMEM, "hipMalloc failed");
    m->allocs.push_back(q);
    *p = (T *)q;
    return LBM_OK;
}

lbm_status ensure_chunks(lbm_mlp *m, int chunks)
{
    if (chunks <= m->chunk_cap)
        return LBM_OK;
    float *p = nullptr;
    if (hipMalloc(&p, sizeof(float) * (size_t)chunks * MLP_PSTRIDE) != hipSuccess)
        return mfail(LBM_E_NOMEM, "hipMalloc of the gradient partials failed");
    auto it = std::find(m->allocs.begin(), m->allocs.end(), (void *)m->d.partial);
    if (it != m->allocs.end()) {
        (void)hipFree(*it);
        m->allocs.erase(it);
    }
    m->allocs.push_back(p);
    m->d.partial = p;
    m->chunk_cap = chunks;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_mlp_create(uint64_t seed, int32_t device, void *stream, lbm_mlp **out)
{
    if (!out)
        return mfail(LBM_E_INVALID, "null argument");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return mfail(LBM_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev)
        return mfail(LBM_E_INVALID, "device ordinal out of range");
    MHIP(hipSetDevice(device));
    lbm_mlp *m = new lbm_mlp();
    m->device = device;
    if (stream) {
        m->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) {
            delete m;
            return mfail(LBM_E_DEVICE, "hipStreamCreate failed");
        }
        m->own_stream = true;
    }
    lbm_status st;
    if ((st = malloc_dev(m, &m->d.master, MLP_NPARAM)) != LBM_OK || (st = malloc_dev(m, &m->d.wr, MLP_NPARAM)) != LBM_OK ||
        (st = malloc_dev(m, &m->d.w1b, 64 * 8)) != LBM_OK || (st = malloc_dev(m, &m->d.w2b, 64 * 64)) != LBM_OK ||
        (st = malloc_dev(m, &m->d.m, MLP_NPARAM)) != LBM_OK || (st = malloc_dev(m, &m->d.v, MLP_NPARAM)) != LBM_OK ||
        (st = malloc_dev(m, &m->d.grad, MLP_PSTRIDE)) != LBM_OK || (st = malloc_dev(m, &m->d.sc, 12)) != LBM_OK ||
        (st = ensure_chunks(m, 64)) != LBM_OK) {
        delete m;
        return st;
    }
    // the static workspace of lbm_mlp_grad_noalloc on this device, resolved
    // here (device current) so that the entry point itself calls nothing but
    // launches and copies
    if (mlp_static_scratch(device, &m->scratch) != hipSuccess) {
        delete m;
        return mfail(LBM_E_DEVICE, "hipGetSymbolAddress of the static gradient workspace failed");
    }
    // He-uniform weights for the ReLU layers, Glorot-uniform output weights,
    // zero biases; draws from SplitMix64(seed) in parameter order
    std::vector<float> p(MLP_NPARAM, 0.0f);
    SplitMix64 rng{seed};
    auto fill = [&](int off, int count, double bound) {
        for (int i = 0; i < count; ++i)
            p[off + i] = (float)((2.0 * rng.uniform() - 1.0) * bound);
    };
    fill(MLP_W1, 320, std::sqrt(6.0 / MLP_IN));
    fill(MLP_W2, 4096, std::sqrt(6.0 / MLP_H));
    fill(MLP_W3, 64, std::sqrt(6.0 / (MLP_H + 1)));
    const float sc[12] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0, 1};
    hipError_t e = hipMemcpy(m->d.master, p.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d.sc, sc, sizeof sc, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemsetAsync(m->d.w1b, 0, sizeof(uint16_t) * 64 * 8, m->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(m->d.m, 0, sizeof(float) * MLP_NPARAM, m->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(m->d.v, 0, sizeof(float) * MLP_NPARAM, m->stream);
    if (e == hipSuccess)
        e = launch_mlp_round(m->d, m->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        delete m;
        return mfail(LBM_E_DEVICE, std::string("surrogate set-up: ") + hipGetErrorString(e));
    }
    *out = m;
    return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp *m) { delete m; }

lbm_status lbm_mlp_get_params(lbm_mlp *m, float *params)
{
    if (!m || !params)
        return mfail(LBM_E_INVALID, "null argument");
    MHIP(hipStreamSynchronize(m->stream));
    MHIP(hipMemcpy(params, m->d.master, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
    return LBM_OK;
}

lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *params)
{
    if (!m || !params)
        return mfail(LBM_E_INVALID, "null argument");
    MHIP(hipStreamSynchronize(m->stream));
    MHIP(hipMemcpy(m->d.master, params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice));
    MHIP(hipMemsetAsync(m->d.m, 0, sizeof(float) * MLP_NPARAM, m->stream));
    MHIP(hipMemsetAsync(m->d.v, 0, sizeof(float) * MLP_NPARAM, m->stream));
    MHIP(launch_mlp_round(m->d, m->stream));
    MHIP(hipStreamSynchronize(m->stream));
    m->adam_t = 0;
    return LBM_OK;
}

lbm_status lbm_mlp_set_scaling(lbm_mlp *m, const float *x_mean, const float *x_std, float y_mean, float y_std)
{
    if (!m || !x_mean || !x_std)
        return mfail(LBM_E_INVALID, "null argument");
    float sc[12];
    for (int k = 0; k < MLP_IN; ++k) {
        if (!(x_std[k] > 0.0f))
            return mfail(LBM_E_INVALID, "feature scales must be > 0");
        sc[k] = x_mean[k];
        sc[MLP_IN + k] = x_std[k];
    }
    if (!(y_std > 0.0f))
        return mfail(LBM_E_INVALID, "target scale must be > 0");
    sc[10] = y_mean;
    sc[11] = y_std;
    MHIP(hipStreamSynchronize(m->stream));
    MHIP(hipMemcpy(m->d.sc, sc, sizeof sc, hipMemcpyHostToDevice));
    return LBM_OK;
}

lbm_status lbm_mlp_grad(lbm_mlp *m, const float *x, const float *t, int64_t n, float *grad, float *loss)
{
    if (!m || !x || !t || !grad || n <= 0 || n > (1 << 30))
        return mfail(LBM_E_INVALID, "bad arguments");
    const int chunks = (int)((n + MLP_CHUNK - 1) / MLP_CHUNK);
    lbm_status st = ensure_chunks(m, chunks);
    if (st != LBM_OK)
        return st;
    MHIP(launch_mlp_grad(m->d, x, t, nullptr, 0, (int)n, (int)n, m->stream));
    MHIP(launch_mlp_reduce(m->d, chunks, m->stream));
    std::vector<float> g(MLP_PSTRIDE);
    MHIP(hipMemcpyAsync(g.data(), m->d.grad, sizeof(float) * MLP_PSTRIDE, hipMemcpyDeviceToHost, m->stream));
    MHIP(hipStreamSynchronize(m->stream));
    std::memcpy(grad, g.data(), sizeof(float) * MLP_NPARAM);
    if (loss)
        *loss = g[MLP_NPARAM];
    return LBM_OK;
}

lbm_status lbm_mlp_grad_noalloc(lbm_mlp *m, const float *x, const float *t, int64_t n, float *grad, float *loss)
{
    if (!m || !x || !t || !grad || n <= 0)
        return mfail(LBM_E_INVALID, "bad arguments");
    if (n > (int64_t)MLP_STATIC_CHUNKS * MLP_CHUNK)
        return mfail(LBM_E_INVALID, "lbm_mlp_grad_noalloc: at most " +
                                        std::to_string((int64_t)MLP_STATIC_CHUNKS * MLP_CHUNK) + " samples, got " +
                                        std::to_string(n));
    if (!m->scratch)
        return mfail(LBM_E_STATE, "the static gradient workspace was not resolved for this device");
    const int chunks = (int)((n + MLP_CHUNK - 1) / MLP_CHUNK);
    // the same kernels as lbm_mlp_grad, on the static workspace: the reduced
    // row first, the chunk partials after it
    MlpDev d = m->d;
    d.grad = m->scratch;
    d.partial = m->scratch + MLP_PSTRIDE;
    MHIP(launch_mlp_grad(d, x, t, nullptr, 0, (int)n, (int)n, m->stream));
    MHIP(launch_mlp_reduce(d, chunks, m->stream));
    MHIP(hipMemcpyAsync(grad, d.grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, m->stream));
    if (loss)
        MHIP(hipMemcpyAsync(loss, d.grad + MLP_NPARAM, sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    return LBM_OK;
}

lbm_status lbm_mlp_adam_step(lbm_mlp *m, const float *grad, float lr)
{
    if (!m || !grad)
        return mfail(LBM_E_INVALID, "null argument");
    MHIP(hipStreamSynchronize(m->stream));
    MHIP(hipMemcpy(m->d.grad, grad, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice));
    m->adam_t++;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->adam_t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->adam_t));
    MHIP(launch_mlp_adam(m->d, lr, 0.9f, 0.999f, 1e-8f, bc1, bc2, m->stream));
    MHIP(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

lbm_status lbm_mlp_train(lbm_mlp *m, const float *x, const float *t, int64_t n, int32_t epochs, int32_t batch,
                         float lr, uint64_t seed, float *loss_per_epoch)
{
    if (!m || !x || !t || n <= 0 || n > (1 << 30) || epochs <= 0 || batch <= 0 || !(lr > 0.0f))
        return mfail(LBM_E_INVALID, "bad arguments");
    const int chunks = (batch + MLP_CHUNK - 1) / MLP_CHUNK;
    lbm_status st = ensure_chunks(m, chunks);
    if (st != LBM_OK)
        return st;
    if (m->idx_cap < n) {
        if (m->idx)
            (void)hipFree(m->idx);
        m->idx = nullptr;
        if (hipMalloc(&m->idx, sizeof(int32_t) * (size_t)n) != hipSuccess)
            return mfail(LBM_E_NOMEM, "hipMalloc of the permutation failed");
        m->idx_cap = n;
    }
    std::vector<int32_t> perm((size_t)n);
    std::vector<float> losses((size_t)epochs, 0.0f);
    for (int e = 0; e < epochs; ++e) {
        // Fisher-Yates shuffle from SplitMix64(seed + epoch); the previous
        // epoch's upload of the permutation must have drained first
        MHIP(hipStreamSynchronize(m->stream));
        for (int64_t i = 0; i < n; ++i)
            perm[(size_t)i] = (int32_t)i;
        SplitMix64 rng{seed + (uint64_t)e};
        for (int64_t i = n - 1; i > 0; --i) {
            const int64_t j = (int64_t)(rng.uniform() * (double)(i + 1));
            std::swap(perm[(size_t)i], perm[(size_t)j]);
        }
        MHIP(hipMemcpyAsync(m->idx, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, m->stream));
        // constant rate, then a tenth of it for the last 30 % of the epochs
        const float lr_e = e < (7 * epochs) / 10 ? lr : 0.1f * lr;
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            const int count = (int)std::min<int64_t>(batch, n - b0);
            MHIP(launch_mlp_grad(m->d, x, t, m->idx, b0, count, count, m->stream));
            MHIP(launch_mlp_reduce(m->d, (count + MLP_CHUNK - 1) / MLP_CHUNK, m->stream));
            m->adam_t++;
            const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->adam_t));
            const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->adam_t));
            MHIP(launch_mlp_adam(m->d, lr_e, 0.9f, 0.999f, 1e-8f, bc1, bc2, m->stream));
        }
        // the epoch's loss is the full-data loss after the epoch
        if (loss_per_epoch) {
            const int all = (int)((n + MLP_CHUNK - 1) / MLP_CHUNK);
            if ((st = ensure_chunks(m, all)) != LBM_OK)
                return st;
            MHIP(launch_mlp_grad(m->d, x, t, nullptr, 0, (int)n, (int)n, m->stream));
            MHIP(launch_mlp_reduce(m->d, all, m->stream));
            float l = 0.0f;
            MHIP(hipMemcpyAsync(&l, m->d.grad + MLP_NPARAM, sizeof(float), hipMemcpyDeviceToHost, m->stream));
            MHIP(hipStreamSynchronize(m->stream));
            losses[(size_t)e] = l;
        }
    }
    MHIP(hipStreamSynchronize(m->stream));
    if (loss_per_epoch)
        std::memcpy(loss_per_epoch, losses.data(), sizeof(float) * (size_t)epochs);
    return LBM_OK;
}

lbm_status lbm_branch_features(const lbm_branch *b, int32_t n, double re_h, double intensity, float *feat,
                               double *ld)
{
    if (!b || n <= 0 || !feat || !(re_h > 0.0))
        return mfail(LBM_E_INVALID, "bad arguments");
    const double H = tree_height(b, n), zb = b[0].p0[2];
    if (!(H > 0.0))
        return mfail(LBM_E_INVALID, "tree of zero height");
    for (int i = 0; i < n; ++i) {
        const double dx = b[i].p1[0] - b[i].p0[0], dy = b[i].p1[1] - b[i].p0[1], dz = b[i].p1[2] - b[i].p0[2];
        const double L = std::sqrt(dx * dx + dy * dy + dz * dz), D = b[i].diameter;
        const double alpha = std::acos(std::min(1.0, std::fabs(dx) / L)) * (180.0 / M_PI);
        feat[5 * (size_t)i + 0] = (float)std::log10(re_h * D / H);
        feat[5 * (size_t)i + 1] = (float)alpha;
        feat[5 * (size_t)i + 2] = (float)b[i].generation;
        feat[5 * (size_t)i + 3] = (float)intensity;
        feat[5 * (size_t)i + 4] = (float)((0.5 * (b[i].p0[2] + b[i].p1[2]) - zb) / H);
        if (ld)
            ld[i] = L * D;
    }
    return LBM_OK;
}

lbm_status lbm_tree_batch(const lbm_tree_params *base, uint64_t seed0, int32_t n_trees, const int32_t *orders,
                          int64_t cap, float *rec, int64_t *tree_start)
{
    if (!base || n_trees <= 0 || !tree_start || base->m < 1 || base->m > 4)
        return mfail(LBM_E_INVALID, "bad arguments");
    tree_start[0] = 0;
    for (int i = 0; i < n_trees; ++i) {
        const int order = orders ? orders[i] : base->order;
        if (order < 0 || order > 12)
            return mfail(LBM_E_INVALID, "tree order out of range");
        int64_t c = 0, pw = 1;
        for (int k = 0; k <= order; ++k, pw *= base->m)
            c += pw;
        tree_start[i + 1] = tree_start[i] + c;
    }
    if (!rec)
        return LBM_OK;
    if (tree_start[n_trees] > cap)
        return mfail(LBM_E_INVALID, "record capacity too small (tree_start[n_trees] holds the need)");
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int i = 0; i < n_trees; ++i) {
        lbm_tree_params p = *base;
        p.order = orders ? orders[i] : base->order;
        p.seed = seed0 + (uint64_t)i;
        std::vector<lbm_branch> b;
        tree_generate(p, b);
        const int n = (int)b.size();
        if (n != (int)(tree_start[i + 1] - tree_start[i])) {
            bad = 1;
            continue;
        }
        const double com[3] = {0.0, 0.0, 0.0};
        tree_place(b.data(), n, 1.0, com);
        const double zb = b[0].p0[2];
        for (int j = 0; j < n; ++j) {
            const lbm_branch &q = b[j];
            const double dx = q.p1[0] - q.p0[0], dy = q.p1[1] - q.p0[1], dz = q.p1[2] - q.p0[2];
            const double L = std::sqrt(dx * dx + dy * dy + dz * dz), D = q.diameter;
            float *r = rec + (tree_start[i] + j) * SWEEP_REC;
            r[0] = (float)std::log10(D);
            r[1] = (float)(std::acos(std::min(1.0, std::fabs(dx) / L)) * (180.0 / M_PI));
            r[2] = (float)q.generation;
            r[3] = (float)(0.5 * (q.p0[2] + q.p1[2]) - zb);
            r[4] = (float)(L * D);
            r[5] = (float)q.p0[1];
            r[6] = (float)q.p0[2];
            r[7] = (float)q.p1[1];
            r[8] = (float)q.p1[2];
            r[9] = (float)(0.5 * D);
        }
    }
    return bad ? mfail(LBM_E_INVALID, "tree generator returned an unexpected branch count") : LBM_OK;
}

lbm_status lbm_frontal_area(const float *rec, const int64_t *tree_start, int32_t n_trees, double h, float *area,
                            void *stream)
{
    if (!rec || !tree_start || !area || n_trees < 0 || !(h > 0.0))
        return mfail(LBM_E_INVALID, "bad arguments");
    MHIP(launch_frontal_area(rec, tree_start, n_trees, (float)h, area, (hipStream_t)stream));
    MHIP(hipStreamSynchronize((hipStream_t)stream));
    return LBM_OK;
}

static lbm_status sweep_args(const lbm_sweep_desc *d, SweepArgs &a)
{
    if (!d || !d->rec || !d->tree_start || !d->area || !d->cd || d->n_trees < 0 || !d->re_h || d->n_re <= 0 ||
        d->n_re > SWEEP_MAX_RE || d->intensity < 0.0 || d->intensity > 0.2)
        return mfail(LBM_E_INVALID, "bad sweep description");
    a = SweepArgs{};
    a.rec = d->rec;
    a.tree_start = d->tree_start;
    a.n_trees = d->n_trees;
    for (int q = 0; q < d->n_re; ++q) {
        if (!(d->re_h[q] > 0.0))
            return mfail(LBM_E_INVALID, "Re_H must be > 0");
        a.lg_re[q] = (float)std::log10(d->re_h[q]);
    }
    a.n_re = d->n_re;
    a.intensity = (float)d->intensity;
    a.lg_lo = (float)std::log10(std::max(d->re_d_lo, 1e-30));
    a.lg_hi = (float)std::log10(std::max(d->re_d_hi, 1e-30));
    // critical Re_D: 2.7e5 for uniform inflow, 1.4e4 at I_u = 8 %, log-linear in between
    a.re_cr = (float)(2.7e5 * std::pow(1.4e4 / 2.7e5, d->intensity / 0.08));
    a.area = d->area;
    a.cd = d->cd;
    return LBM_OK;
}

lbm_status lbm_surrogate_sweep(lbm_mlp *m, const lbm_sweep_desc *d)
{
    if (!m)
        return mfail(LBM_E_INVALID, "null handle");
    SweepArgs a;
    lbm_status st = sweep_args(d, a);
    if (st != LBM_OK)
        return st;
    if (!(d->re_d_lo > 0.0) || !(d->re_d_hi >= d->re_d_lo))
        return mfail(LBM_E_INVALID, "training envelope must satisfy 0 < re_d_lo <= re_d_hi");
    MHIP(launch_tree_sweep(m->d, a, m->stream));
    MHIP(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

lbm_status lbm_analytic_sweep(const lbm_sweep_desc *d, void *stream)
{
    SweepArgs a;
    lbm_status st = sweep_args(d, a);
    if (st != LBM_OK)
        return st;
    MHIP(launch_analytic_sweep(a, (hipStream_t)stream));
    MHIP(hipStreamSynchronize((hipStream_t)stream));
    return LBM_OK;
}

lbm_status lbm_analytic_split(const lbm_sweep_desc *d, const lbm_cf_table *t, float *cf, float *cp, void *stream)
{
    SweepArgs a;
    lbm_status st = sweep_args(d, a);
    if (st != LBM_OK)
        return st;
    if (!t || !t->lg_re || !t->cf || t->n < 2 || t->n > CF_MAX_NODES || !cf)
        return mfail(LBM_E_INVALID, "bad friction table or output");
    for (int k = 0; k < t->n; ++k) {
        if (!std::isfinite(t->lg_re[k]) || !std::isfinite(t->cf[k]) || !(t->cf[k] > 0.0))
            return mfail(LBM_E_INVALID, "friction table: finite nodes and C_f > 0 required");
        if (k > 0 && !(t->lg_re[k] > t->lg_re[k - 1]))
            return mfail(LBM_E_INVALID, "friction table: log10 Re_D nodes must increase strictly");
    }
    CfArgs c{};
    c.n_seg = t->n - 1;
    for (int k = 0; k < c.n_seg; ++k) {
        const double l0 = std::log2(t->cf[k]), l1 = std::log2(t->cf[k + 1]);
        const double s2 = (l1 - l0) / (t->lg_re[k + 1] - t->lg_re[k]);
        c.lg[k] = (float)t->lg_re[k];
        c.s2[k] = (float)s2;
        c.a2[k] = (float)(l0 - s2 * t->lg_re[k]);
    }
    c.cf = cf;
    c.cp = cp;
    MHIP(launch_analytic_split(a, c, (hipStream_t)stream));
    MHIP(hipStreamSynchronize((hipStream_t)stream));
    return LBM_OK;
}

lbm_status lbm_mlp_predict(lbm_mlp *m, const float *x, int64_t n, float *y)
{
    if (!m || !x || !y || n < 0)
        return mfail(LBM_E_INVALID, "bad arguments");
    MHIP(launch_mlp_predict(m->d, x, n, y, m->stream));
    MHIP(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

}  // extern "C"
