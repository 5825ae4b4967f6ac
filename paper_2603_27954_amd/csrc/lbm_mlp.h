// Per-branch drag surrogate network (5-64-64-1, ReLU) on the device.  Internal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int MLP_IN = 5, MLP_H = 64;
// packed parameter offsets: W1 (64 x 5), b1, W2 (64 x 64), b2, w3, b3
constexpr int MLP_W1 = 0, MLP_B1 = 320, MLP_W2 = 384, MLP_B2 = 4480, MLP_W3 = 4544, MLP_B3 = 4608;
constexpr int MLP_NPARAM = 4609;
constexpr int MLP_CHUNK = 32;           // samples per work-group of the gradient kernel
constexpr int MLP_PSTRIDE = MLP_NPARAM + 1;  // partial sums: parameters, then the loss

struct MlpDev {
    float *master;      // FP32 master parameters
    float *wr;          // parameters as the kernels use them (weights rounded to BF16)
    uint16_t *w1b;      // BF16 bits of W1, padded to 64 x 8
    uint16_t *w2b;      // BF16 bits of W2, 64 x 64
    float *m, *v;       // Adam moments
    float *grad;        // reduced gradient (+ loss at MLP_NPARAM)
    float *partial;     // per-chunk partial sums, MLP_PSTRIDE each
    float *sc;          // x_mean[5], x_std[5], y_mean, y_std
};

// Gradient of the mean-square loss over the batch samples idx[base ..
// base + count) (idx may be null: samples base ..), on targets standardised
// with y_mean / y_std, normalised by n_norm; per-chunk partial sums.
hipError_t launch_mlp_grad(const MlpDev &d, const float *x, const float *t, const int32_t *idx, int64_t base,
                           int count, int n_norm, hipStream_t s);
// grad = sum of the partial sums of nchunks chunks, in chunk order
hipError_t launch_mlp_reduce(const MlpDev &d, int nchunks, hipStream_t s);
// Static gradient workspace for callers that cannot allocate: per device, one
// reduced row and the partial sums of up to MLP_STATIC_CHUNKS chunks
// (MLP_PSTRIDE floats each) in a file-scope device array.
constexpr int MLP_STATIC_CHUNKS = 1024;  // 32768 samples
// Resolves the array's address on the current device (once per device) and
// returns it in *ptr; call with the device current.
hipError_t mlp_static_scratch(int device, float **ptr);

// one Adam step on grad; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t; refreshes wr, w1b, w2b
hipError_t launch_mlp_adam(const MlpDev &d, float lr, float beta1, float beta2, float eps, float bc1, float bc2,
                           hipStream_t s);
// refreshes wr, w1b, w2b from master (after parameters are set)
hipError_t launch_mlp_round(const MlpDev &d, hipStream_t s);
// y = network(x) for n rows of raw features, in output units (matrix cores, BF16 operands)
hipError_t launch_mlp_predict(const MlpDev &d, const float *x, int64_t n, float *y, hipStream_t s);

// Branch records of a batch of trees (lengths in units of the tree height
// H): log10(D/H), alpha (deg), generation, midpoint height / H, L D / H^2, and
// the branch axis projected on the (y, z) plane with the radius: y0, z0, y1,
// z1, D / 2.
constexpr int SWEEP_REC = 10;
constexpr int SWEEP_MAX_RE = 32;
constexpr int AREA_PIX = 640;  // frontal-area raster edge (pixels)

// Branch-wise drag sums of many trees at many Re_H.
struct SweepArgs {
    const float *rec;          // SWEEP_REC floats per branch
    const int64_t *tree_start; // n_trees + 1 branch offsets
    int n_trees;
    float lg_re[SWEEP_MAX_RE]; // log10 Re_H values
    int n_re;
    float intensity;
    float lg_lo, lg_hi;        // training envelope of log10 Re_D (surrogate only)
    float re_cr;               // critical Re_D of the cylinder curve for this intensity
    const float *area;         // per tree A_x / H^2
    float *cd;                 // n_trees x n_re
};
// Friction coefficient table of a cylinder normal to the flow: on segment k
// (log10 Re_D >= lg[k] for k >= 1; the first segment also below lg[1], the last
// also above the table) log2 C_f = a2[k] + s2[k] log10 Re_D.
constexpr int CF_MAX_NODES = 32;
struct CfArgs {
    int n_seg;                 // nodes - 1
    float lg[CF_MAX_NODES];    // segment start, log10 Re_D
    float a2[CF_MAX_NODES];    // intercept of log2 C_f
    float s2[CF_MAX_NODES];    // slope of log2 C_f over log10 Re_D
    float *cf;                 // n_trees x n_re friction estimates
    float *cp;                 // n_trees x n_re pressure estimates, or null
};
// surrogate: sum_b y_b L_b D_b / A_x with y_b from the network (extrapolated
// through the cylinder curve outside the envelope)
hipError_t launch_tree_sweep(const MlpDev &d, const SweepArgs &a, hipStream_t s);
// analytic model: sum_b C_d(Re_b) L_b D_b sin^3(alpha_b) / A_x
hipError_t launch_analytic_sweep(const SweepArgs &a, hipStream_t s);
// the same, and sum_b C_f(Re_b) L_b D_b sin^3(alpha_b) / A_x into c.cf, the
// difference of the two into c.cp
hipError_t launch_analytic_split(const SweepArgs &a, const CfArgs &c, hipStream_t s);
// frontal area of each tree (units of H^2): union of the branches' projected
// capsules rasterised with pixel edge h (units of H); -1 when the tree does
// not fit AREA_PIX pixels per side
hipError_t launch_frontal_area(const float *rec, const int64_t *tree_start, int n_trees, float h, float *area,
                               hipStream_t s);

}  // namespace lbm
