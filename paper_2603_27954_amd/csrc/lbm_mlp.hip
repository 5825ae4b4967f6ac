// Kernels of the per-branch drag surrogate (5-64-64-1 ReLU network).
//
// Precision: FP32 master parameters; the kernels use the weights rounded to
// BF16 (ties to even) and FP32 biases, and accumulate in FP32.  Training keeps
// activations in FP32.  Inference runs on the matrix cores with BF16 operands
// (scaled features and first-layer activations rounded to BF16) and FP32
// accumulators.
//
// Training is deterministic: each work-group sums the gradient of a fixed
// chunk of samples in a fixed order, and the chunks are added in chunk order.
//
// Inference maps 32 samples onto the N dimension of the 32x32x16 BF16 MFMA
// (gfx950), with neurons on M.  The 16 accumulator registers of lane l hold
// rows 8 (i / 4) + 4 (l / 32) + (i % 4) of column l % 32.  Taking the next
// layer's K-slots in the matching (permuted) neuron order makes those registers
// its B operands, so the hidden activations pass from layer to layer without
// leaving the lane.
#include "lbm_mlp.h"

#include <algorithm>
#include <mutex>

namespace lbm {

namespace {

__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(bf16_bits(x) << 16); }

__device__ __forceinline__ bool is_weight(int p)
{
    return (p >= MLP_W1 && p < MLP_B1) || (p >= MLP_W2 && p < MLP_B2) || (p >= MLP_W3 && p < MLP_B3);
}

// ---------------------------------------------------------------------------
// training: per-chunk gradient (32 samples, 8 threads per sample)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_mlp_grad(const float *wr, const float *sc, const float *x, const float *t,
                                                  const int32_t *idx, int64_t base, int count, int n_norm,
                                                  float *partial)
{
    constexpr int S = MLP_CHUNK, H = MLP_H;
    __shared__ float sW2[H * H];
    __shared__ float sH1[S * H], sH2[S * H], sD2[S * H], sD1[S * H];
    __shared__ float sX[S * MLP_IN], sY[S], sT[S], sDY[S], sYp[S * 8];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * S;
    const int ns = min(S, count - c0);
    for (int i = tid; i < H * H; i += 256)
        sW2[i] = wr[MLP_W2 + i];
    for (int i = tid; i < S * MLP_IN; i += 256) {
        const int s = i / MLP_IN, k = i - s * MLP_IN;
        float v = 0.0f;
        if (s < ns) {
            const int64_t row = idx ? (int64_t)idx[base + c0 + s] : base + c0 + s;
            v = (x[row * MLP_IN + k] - sc[k]) / sc[MLP_IN + k];
        }
        sX[i] = v;
    }
    if (tid < S) {
        float v = 0.0f;
        if (tid < ns) {
            const int64_t row = idx ? (int64_t)idx[base + c0 + tid] : base + c0 + tid;
            v = (t[row] - sc[10]) / sc[11];
        }
        sT[tid] = v;
    }
    __syncthreads();
    const int s = tid >> 3, part = tid & 7;  // sample, group of 8 hidden units
    const bool live = s < ns;
    // layer 1
    for (int u = part * 8; u < part * 8 + 8; ++u) {
        float z = wr[MLP_B1 + u];
        for (int k = 0; k < MLP_IN; ++k)
            z = fmaf(wr[MLP_W1 + u * MLP_IN + k], sX[s * MLP_IN + k], z);
        sH1[s * H + u] = z > 0.0f ? z : 0.0f;
    }
    __syncthreads();
    // layer 2 and the output
    float yp = 0.0f;
    for (int u = part * 8; u < part * 8 + 8; ++u) {
        float z = wr[MLP_B2 + u];
        for (int i = 0; i < H; ++i)
            z = fmaf(sW2[u * H + i], sH1[s * H + i], z);
        const float h = z > 0.0f ? z : 0.0f;
        sH2[s * H + u] = h;
        yp = fmaf(wr[MLP_W3 + u], h, yp);
    }
    sYp[s * 8 + part] = yp;
    __syncthreads();
    if (tid < S) {
        float y = wr[MLP_B3];
        for (int q = 0; q < 8; ++q)
            y += sYp[tid * 8 + q];
        sY[tid] = y;
        sDY[tid] = tid < ns ? 2.0f * (y - sT[tid]) / (float)n_norm : 0.0f;
    }
    __syncthreads();
    // backward through layer 2
    for (int u = part * 8; u < part * 8 + 8; ++u)
        sD2[s * H + u] = (live && sH2[s * H + u] > 0.0f) ? sDY[s] * wr[MLP_W3 + u] : 0.0f;
    __syncthreads();
    for (int i = part * 8; i < part * 8 + 8; ++i) {
        float d = 0.0f;
        for (int u = 0; u < H; ++u)
            d = fmaf(sW2[u * H + i], sD2[s * H + u], d);
        sD1[s * H + i] = sH1[s * H + i] > 0.0f ? d : 0.0f;
    }
    __syncthreads();
    // parameter gradients of this chunk (sums over samples in order)
    float *out = partial + (size_t)blockIdx.x * MLP_PSTRIDE;
    {
        const int u = tid >> 2, i0 = (tid & 3) * 16;
        for (int i = i0; i < i0 + 16; ++i) {
            float g = 0.0f;
            for (int q = 0; q < S; ++q)
                g = fmaf(sD2[q * H + u], sH1[q * H + i], g);
            out[MLP_W2 + u * H + i] = g;
        }
    }
    for (int p = tid; p < 320 + 64 + 64 + 64 + 1 + 1; p += 256) {
        float g = 0.0f;
        if (p < 320) {  // W1
            const int u = p / MLP_IN, k = p - u * MLP_IN;
            for (int q = 0; q < S; ++q)
                g = fmaf(sD1[q * H + u], sX[q * MLP_IN + k], g);
            out[MLP_W1 + p] = g;
        } else if (p < 384) {  // b1
            const int u = p - 320;
            for (int q = 0; q < S; ++q)
                g += sD1[q * H + u];
            out[MLP_B1 + u] = g;
        } else if (p < 448) {  // b2
            const int u = p - 384;
            for (int q = 0; q < S; ++q)
                g += sD2[q * H + u];
            out[MLP_B2 + u] = g;
        } else if (p < 512) {  // w3
            const int u = p - 448;
            for (int q = 0; q < S; ++q)
                g = fmaf(sDY[q], sH2[q * H + u], g);
            out[MLP_W3 + u] = g;
        } else if (p == 512) {  // b3
            for (int q = 0; q < S; ++q)
                g += sDY[q];
            out[MLP_B3] = g;
        } else {  // loss
            for (int q = 0; q < ns; ++q) {
                const float r = sY[q] - sT[q];
                g = fmaf(r, r, g);
            }
            out[MLP_NPARAM] = g / (float)n_norm;
        }
    }
}

__global__ void k_mlp_reduce(const float *partial, int nchunks, float *grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_PSTRIDE)
        return;
    float g = 0.0f;
    for (int c = 0; c < nchunks; ++c)
        g += partial[(size_t)c * MLP_PSTRIDE + p];
    grad[p] = g;
}

__device__ __forceinline__ void store_param(const MlpDev &d, int p, float v)
{
    d.master[p] = v;
    const float r = is_weight(p) ? bf16_round(v) : v;
    d.wr[p] = r;
    if (p >= MLP_W1 && p < MLP_B1) {
        const int u = (p - MLP_W1) / MLP_IN, k = (p - MLP_W1) - u * MLP_IN;
        d.w1b[u * 8 + k] = (uint16_t)bf16_bits(v);
    } else if (p >= MLP_W2 && p < MLP_B2) {
        d.w2b[p - MLP_W2] = (uint16_t)bf16_bits(v);
    }
}

__global__ void k_mlp_adam(MlpDev d, float lr, float beta1, float beta2, float eps, float bc1, float bc2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM)
        return;
    const float g = d.grad[p];
    const float m = beta1 * d.m[p] + (1.0f - beta1) * g;
    const float v = beta2 * d.v[p] + (1.0f - beta2) * g * g;
    d.m[p] = m;
    d.v[p] = v;
    const float mh = m / bc1, vh = v / bc2;
    store_param(d, p, d.master[p] - lr * mh / (sqrtf(vh) + eps));
}

__global__ void k_mlp_round(MlpDev d)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPARAM)
        store_param(d, p, d.master[p]);
    if (p < 64 * 3)  // padding columns 5..7 of W1
        d.w1b[(p / 3) * 8 + 5 + p % 3] = 0;
}

// ---------------------------------------------------------------------------
// inference on the matrix cores
// ---------------------------------------------------------------------------

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int acc_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

__device__ __forceinline__ __bf16 bf16_of(uint32_t bits) { return __builtin_bit_cast(__bf16, (uint16_t)bits); }

// Network weights held in registers by one wave (A operands of the
// 32x32x16 BF16 MFMA: lane l holds row l % 32 and the 8 K-slots
// 8 (l / 32) .. 8 (l / 32) + 7), and the biases and output weights in LDS.
// Layer 2's K-slot (s, h, j) of K-step s in 0..3 stands for input neuron
// 16 s + 4 h + (j < 4 ? j : j + 4).  These are the neurons that lane half h
// holds in accumulator registers 8 (s % 2) .. 8 (s % 2) + 7 of layer 1's tile
// s / 2, so the B operands are those registers as they are.
struct MlpRegs {
    bf16x8 a1[2], a2[2][4];
};

__device__ __forceinline__ int l2_neuron(int s, int h, int j) { return 16 * s + 4 * h + (j < 4 ? j : j + 4); }

__device__ __forceinline__ void load_regs(const MlpDev &d, MlpRegs &r, int lane)
{
    const int m = lane & 31, h = lane >> 5;
    for (int t = 0; t < 2; ++t) {
        for (int j = 0; j < 8; ++j)
            r.a1[t][j] = bf16_of(h == 0 ? d.w1b[(32 * t + m) * 8 + j] : 0u);
        for (int s = 0; s < 4; ++s)
            for (int j = 0; j < 8; ++j)
                r.a2[t][s][j] = bf16_of(d.w2b[(32 * t + m) * 64 + l2_neuron(s, h, j)]);
    }
}

// y (scaled output units, before b3) of the sample of column lane % 32, given
// its scaled features as the B operand of the first layer (lane half 0 holds
// features 0..4 and zeros, half 1 zeros); sb = b1[64], b2[64], w3[64] in LDS.
// Both lanes of a column return the same value.
// ReLU in one instruction: the median of (x, 0, FLT_MAX) is x for finite x >= 0
// and 0 for x < 0 (fmaxf on a matrix-core result costs a canonicalising max
// as well)
__device__ __forceinline__ float relu(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 3.402823466e38f); }

__device__ __forceinline__ float mlp_tile(const MlpRegs &r, bf16x8 b1, const float *sb, int lane)
{
    // an offset the compiler cannot see through: the 192 LDS values are read
    // per tile instead of being held in registers across a caller's loop
    int o = 0;
    asm volatile("" : "+s"(o));
    sb += o;
    f32x16 c1[2];
    for (int t = 0; t < 2; ++t) {
        for (int i = 0; i < 16; ++i)
            c1[t][i] = sb[32 * t + acc_row(i, lane)];
        c1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(r.a1[t], b1, c1[t], 0, 0, 0);
    }
    bf16x8 b2[4];
    for (int s = 0; s < 4; ++s)
        for (int j = 0; j < 8; ++j)
            b2[s][j] = (__bf16)relu(c1[s >> 1][8 * (s & 1) + j]);  // round to nearest even
    float y = 0.0f;
    for (int t = 0; t < 2; ++t) {
        f32x16 c2;
        for (int i = 0; i < 16; ++i)
            c2[i] = sb[64 + 32 * t + acc_row(i, lane)];
        for (int s = 0; s < 4; ++s)
            c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(r.a2[t][s], b2[s], c2, 0, 0, 0);
        for (int i = 0; i < 16; ++i)
            y = fmaf(sb[128 + 32 * t + acc_row(i, lane)], relu(c2[i]), y);
    }
    return y + __shfl_xor(y, 32, 64);
}

__device__ __forceinline__ void load_bias(const MlpDev &d, float *sb)
{
    for (int i = threadIdx.x; i < 192; i += blockDim.x)
        sb[i] = i < 64 ? d.wr[MLP_B1 + i] : (i < 128 ? d.wr[MLP_B2 + i - 64] : d.wr[MLP_W3 + i - 128]);
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_mlp_predict(MlpDev d, const float *x, int64_t n, float *y)
{
    __shared__ float sb[192];
    load_bias(d, sb);
    const int lane = threadIdx.x & 63;
    MlpRegs r;
    load_regs(d, r, lane);
    float mean[MLP_IN], inv[MLP_IN];
    for (int k = 0; k < MLP_IN; ++k) {
        mean[k] = d.sc[k];
        inv[k] = 1.0f / d.sc[MLP_IN + k];
    }
    const float b3 = d.wr[MLP_B3], ym = d.sc[10], ys = d.sc[11];
    const int64_t tiles = (n + 31) / 32;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t tile = wave; tile < tiles; tile += waves) {
        const int64_t row = tile * 32 + (lane & 31);
        bf16x8 b1;
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * (lane >> 5) + j;
            float v = 0.0f;
            if (k < MLP_IN && row < n)
                v = (x[row * MLP_IN + k] - mean[k]) * inv[k];
            b1[j] = (__bf16)v;
        }
        const float out = mlp_tile(r, b1, sb, lane);
        if (lane < 32 && row < n)
            y[row] = (out + b3) * ys + ym;
    }
}

// ---------------------------------------------------------------------------
// branch-wise drag sums over many trees
// ---------------------------------------------------------------------------

// Cylinder drag curve of the analytic model (a synthetic stand-in for the
// fitted measurements the paper does not print): a subcritical correlation
// 1 + 10 Re^(-2/3) blended into a post-critical branch
// 0.25 + 0.35 / (1 + exp(-(ln Re - ln(20 Re_cr)) / 0.8)) by the weight
// 1 / (1 + exp((ln Re - ln Re_cr) / 0.12)).
// Evaluated with the hardware exp2 and reciprocal (about 1 ulp each): the
// exponents are formed in log2 units, Re^(-2/3) = 2^(-(2/3) log2 Re).
__device__ __forceinline__ float cylinder_cd(float lg_re, float ln_rc)
{
    constexpr float LOG2_10 = 3.321928095f, LOG2_E = 1.442695041f;
    const float l2 = lg_re * LOG2_10;           // log2 Re
    const float l2c = ln_rc * LOG2_E;           // log2 Re_cr
    const float sub = 1.0f + 10.0f * __builtin_amdgcn_exp2f(-(2.0f / 3.0f) * l2);
    // ln(20) = 2.995732274; 1 / 0.8 and 1 / 0.12 as products
    const float post = 0.25f + 0.35f * __builtin_amdgcn_rcpf(
        1.0f + __builtin_amdgcn_exp2f(-(l2 - l2c - 2.995732274f * LOG2_E) * 1.25f));
    const float w = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f((l2 - l2c) * (1.0f / 0.12f)));
    return w * sub + (1.0f - w) * post;
}

__device__ __forceinline__ float wave_sum_f(float v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_down(v, o, 64);
    return v;
}

// One wave per tree.  Tiles of 32 branches run on the matrix cores; for each
// tile the four Re-independent features are scaled once and the Re_H values
// follow, each changing only the first feature.  Each lane keeps its sum per
// Re_H in LDS, adding tiles in order; a fixed shuffle tree ends each sum.
// Outside the training envelope the network's value at the envelope edge is
// carried along the cylinder curve: y C_d(Re_D) / C_d(edge).
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) k_tree_sweep(MlpDev d, SweepArgs a)
{
    __shared__ float sb[192];
    __shared__ float acc[SWEEP_MAX_RE][64];
    load_bias(d, sb);
    const int lane = threadIdx.x;
    MlpRegs r;
    load_regs(d, r, lane);
    const int tree = blockIdx.x;
    const int64_t b0 = a.tree_start[tree], b1 = a.tree_start[tree + 1];
    const float b3 = d.wr[MLP_B3], ym = d.sc[10], ys = d.sc[11];
    const float m0 = d.sc[0], s0 = d.sc[MLP_IN];
    const float ln_rc = logf(a.re_cr), inv = 1.0f / a.area[tree];
    const float inv_lo = 1.0f / cylinder_cd(a.lg_lo, ln_rc), inv_hi = 1.0f / cylinder_cd(a.lg_hi, ln_rc);
    const float inv_s0 = 1.0f / s0;
    const bool feat_lane = lane < 32;  // lane half 0 carries the features
    for (int q = 0; q < a.n_re; ++q)
        acc[q][lane] = 0.0f;
    for (int64_t t0 = b0; t0 < b1; t0 += 32) {
        const int64_t br = t0 + (lane & 31);
        const bool valid = br < b1;
        const float *rc = a.rec + (valid ? br : b0) * SWEEP_REC;
        const float lgd = rc[0], wgt = (feat_lane && valid) ? rc[4] : 0.0f;
        bf16x8 bop;
        bop[0] = (__bf16)0.0f;
        bop[1] = (__bf16)(feat_lane ? (rc[1] - d.sc[1]) / d.sc[MLP_IN + 1] : 0.0f);
        bop[2] = (__bf16)(feat_lane ? (rc[2] - d.sc[2]) / d.sc[MLP_IN + 2] : 0.0f);
        bop[3] = (__bf16)(feat_lane ? (a.intensity - d.sc[3]) / d.sc[MLP_IN + 3] : 0.0f);
        bop[4] = (__bf16)(feat_lane ? (rc[3] - d.sc[4]) / d.sc[MLP_IN + 4] : 0.0f);
        bop[5] = bop[6] = bop[7] = (__bf16)0.0f;
        for (int q = 0; q < a.n_re; ++q) {
            const float lre = a.lg_re[q] + lgd;
            const float lc = fminf(fmaxf(lre, a.lg_lo), a.lg_hi);
            bop[0] = (__bf16)(feat_lane ? (lc - m0) * inv_s0 : 0.0f);
            float y = (mlp_tile(r, bop, sb, lane) + b3) * ys + ym;
            if (lre != lc)
                y *= cylinder_cd(lre, ln_rc) * (lre > lc ? inv_hi : inv_lo);
            acc[q][lane] = fmaf(y, wgt, acc[q][lane]);
        }
    }
    for (int q = 0; q < a.n_re; ++q) {
        const float sum = wave_sum_f(acc[q][lane]);
        if (lane == 0)
            a.cd[(size_t)tree * a.n_re + q] = sum * inv;
    }
}

// C_f of the table at log10 Re_D = lg: the segment is picked by selects over
// the (wave-uniform) segment starts, so no lane indexes the table.
__device__ __forceinline__ float cylinder_cf(const CfArgs &c, float lg)
{
    float a2 = c.a2[0], s2 = c.s2[0];
    for (int k = 1; k < c.n_seg; ++k) {
        const bool up = lg >= c.lg[k];
        a2 = up ? c.a2[k] : a2;
        s2 = up ? c.s2[k] : s2;
    }
    return __builtin_amdgcn_exp2f(fmaf(s2, lg, a2));
}

template <bool SPLIT>
__global__ void __launch_bounds__(64) k_analytic_sweep(SweepArgs a, CfArgs c)
{
    const int lane = threadIdx.x, tree = blockIdx.x;
    const int64_t b0 = a.tree_start[tree], b1 = a.tree_start[tree + 1];
    const float ln_rc = logf(a.re_cr), inv = 1.0f / a.area[tree];
    for (int q = 0; q < a.n_re; ++q) {
        float acc = 0.0f, accf = 0.0f;
        for (int64_t br = b0 + lane; br < b1; br += 64) {
            const float *rc = a.rec + br * SWEEP_REC;
            const float sn = sinf(rc[1] * 0.01745329252f);
            const float lg = a.lg_re[q] + rc[0], w = rc[4] * sn * sn * sn;
            acc = fmaf(cylinder_cd(lg, ln_rc), w, acc);
            if constexpr (SPLIT)
                accf = fmaf(cylinder_cf(c, lg), w, accf);
        }
        const float sum = wave_sum_f(acc);
        const size_t o = (size_t)tree * a.n_re + q;
        if (lane == 0)
            a.cd[o] = sum * inv;
        if constexpr (SPLIT) {
            const float sumf = wave_sum_f(accf);
            if (lane == 0) {
                c.cf[o] = sumf * inv;
                if (c.cp)
                    c.cp[o] = (sum - sumf) * inv;
            }
        }
    }
}

// Union of the projected capsules (segment (y0, z0)-(y1, z1), radius r) on a
// pixel grid of edge h anchored at the tree's lower (y, z) bound; a pixel is
// covered when its centre lies within r of a segment.
__global__ void __launch_bounds__(256) k_frontal_area(const float *rec, const int64_t *tree_start, float h,
                                                      float *area)
{
    constexpr int WORDS = AREA_PIX * AREA_PIX / 32;
    __shared__ uint32_t bits[WORDS];
    __shared__ float red[4][256];
    __shared__ float box[256][6];
    __shared__ int boxi[256][2], pend[256], wsum[4];
    const int tid = threadIdx.x, tree = blockIdx.x;
    const int64_t b0 = tree_start[tree], b1 = tree_start[tree + 1];
    float ylo = 1e30f, yhi = -1e30f, zlo = 1e30f, zhi = -1e30f;
    for (int64_t b = b0 + tid; b < b1; b += 256) {
        const float *rc = rec + b * SWEEP_REC;
        const float rr = rc[9];
        ylo = fminf(ylo, fminf(rc[5], rc[7]) - rr);
        yhi = fmaxf(yhi, fmaxf(rc[5], rc[7]) + rr);
        zlo = fminf(zlo, fminf(rc[6], rc[8]) - rr);
        zhi = fmaxf(zhi, fmaxf(rc[6], rc[8]) + rr);
    }
    red[0][tid] = ylo, red[1][tid] = -yhi, red[2][tid] = zlo, red[3][tid] = -zhi;
    for (int i = tid; i < WORDS; i += 256)
        bits[i] = 0u;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o)
            for (int k = 0; k < 4; ++k)
                red[k][tid] = fminf(red[k][tid], red[k][tid + o]);
        __syncthreads();
    }
    ylo = red[0][0], yhi = -red[1][0], zlo = red[2][0], zhi = -red[3][0];
    const int ny = (int)ceilf((yhi - ylo) / h), nz = (int)ceilf((zhi - zlo) / h);
    __syncthreads();
    if (ny > AREA_PIX || nz > AREA_PIX || b1 <= b0) {
        if (tid == 0)
            area[tree] = -1.0f;
        return;
    }
    // Branches go in chunks of 256, one per thread: each thread puts its
    // branch's capsule and pixel-row range in LDS, a work-group scan of the
    // row counts lays the chunk's rows out in one index range, and the threads
    // take that range with stride 256 (a thread's row index only grows, so it
    // finds the owning branch by walking forward).  A capsule is convex, so
    // its pixels in one row form one span: the union of the spans of its two
    // end discs and of its straight part, which are solved in closed form.
    for (int64_t c0 = b0; c0 < b1; c0 += 256) {
        const int64_t b = c0 + tid;
        int nr = 0;
        if (b < b1) {
            const float *rc = rec + b * SWEEP_REC;
            const float y0 = rc[5], z0 = rc[6], y1 = rc[7], z1 = rc[8], rr = rc[9];
            const int pz0 = max(0, (int)floorf((fminf(z0, z1) - rr - zlo) / h));
            const int pz1 = min(nz - 1, (int)floorf((fmaxf(z0, z1) + rr - zlo) / h));
            nr = max(0, pz1 - pz0 + 1);
            const float dy = y1 - y0, dz = z1 - z0;
            box[tid][0] = y0;
            box[tid][1] = z0;
            box[tid][2] = dy;
            box[tid][3] = dz;
            box[tid][4] = rr;
            box[tid][5] = sqrtf(dy * dy + dz * dz);
            boxi[tid][0] = pz0;
        }
        // inclusive scan of the row counts over the work-group
        const int lane = tid & 63, wave = tid >> 6;
        int v = nr;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(v, o, 64);
            if (lane >= o)
                v += u;
        }
        if (lane == 63)
            wsum[wave] = v;
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w)
            off += wsum[w];
        pend[tid] = off + v;  // end of this branch's row range
        const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
        int j = 0;
        for (int p = tid; p < total; p += 256) {
            while (pend[j] <= p)
                ++j;
            const int pz = boxi[j][0] + p - (j ? pend[j - 1] : 0);
            const float y0 = box[j][0], dy = box[j][2], dz = box[j][3], r = box[j][4], len = box[j][5];
            const float c = zlo + (pz + 0.5f) * h - box[j][1];  // row height relative to the axis start
            float lo = 3.0e38f, hi = -3.0e38f;
            // end discs
            if (c * c <= r * r) {
                const float sd = sqrtf(r * r - c * c);
                lo = fminf(lo, -sd);
                hi = fmaxf(hi, sd);
            }
            const float e = c - dz;
            if (e * e <= r * r) {
                const float sd = sqrtf(r * r - e * e);
                lo = fminf(lo, dy - sd);
                hi = fmaxf(hi, dy + sd);
            }
            // straight part: 0 <= (u dy + c dz) <= L^2 and |u dz - c dy| <= r L
            if (len > 0.0f) {
                float ul = -3.0e38f, uh = 3.0e38f;
                bool ok = true;
                if (dy != 0.0f) {
                    const float a0 = -c * dz / dy, a1 = (len * len - c * dz) / dy;
                    ul = fmaxf(ul, fminf(a0, a1));
                    uh = fminf(uh, fmaxf(a0, a1));
                } else {
                    ok = c * dz >= 0.0f && c * dz <= len * len;
                }
                if (dz != 0.0f) {
                    const float a0 = (c * dy - r * len) / dz, a1 = (c * dy + r * len) / dz;
                    ul = fmaxf(ul, fminf(a0, a1));
                    uh = fminf(uh, fmaxf(a0, a1));
                } else {
                    ok = ok && fabsf(c * dy) <= r * len;
                }
                if (ok && ul <= uh) {
                    lo = fminf(lo, ul);
                    hi = fmaxf(hi, uh);
                }
            }
            if (lo > hi)
                continue;
            // pixel centres ylo + (py + 0.5) h inside [y0 + lo, y0 + hi]
            const int pa = max(0, (int)ceilf((y0 + lo - ylo) / h - 0.5f));
            const int pb = min(ny - 1, (int)floorf((y0 + hi - ylo) / h - 0.5f));
            if (pa > pb)
                continue;
            const int ba = pz * AREA_PIX + pa, bb = pz * AREA_PIX + pb;
            for (int w = ba >> 5; w <= (bb >> 5); ++w) {
                uint32_t m = 0xFFFFFFFFu;
                if (w == (ba >> 5))
                    m &= 0xFFFFFFFFu << (ba & 31);
                if (w == (bb >> 5))
                    m &= 0xFFFFFFFFu >> (31 - (bb & 31));
                atomicOr(&bits[w], m);
            }
        }
        __syncthreads();  // the boxes are refilled by the next chunk
    }
    __syncthreads();
    float cnt = 0.0f;
    for (int i = tid; i < WORDS; i += 256)
        cnt += (float)__popc(bits[i]);
    red[0][tid] = cnt;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o)
            red[0][tid] += red[0][tid + o];
        __syncthreads();
    }
    if (tid == 0)
        area[tree] = red[0][0] * h * h;
}

}  // namespace

hipError_t launch_mlp_grad(const MlpDev &d, const float *x, const float *t, const int32_t *idx, int64_t base,
                           int count, int n_norm, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    const int chunks = (count + MLP_CHUNK - 1) / MLP_CHUNK;
    hipLaunchKernelGGL(k_mlp_grad, dim3(chunks), dim3(256), 0, s, d.wr, d.sc, x, t, idx, base, count, n_norm,
                       d.partial);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const MlpDev &d, int nchunks, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_PSTRIDE + 255) / 256), dim3(256), 0, s, d.partial, nchunks, d.grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpDev &d, float lr, float beta1, float beta2, float eps, float bc1, float bc2,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, d, lr, beta1, beta2, eps, bc1,
                       bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_round(const MlpDev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_round, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(const MlpDev &d, const float *x, int64_t n, float *y, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t tiles = (n + 31) / 32;
    const int64_t blocks = std::min<int64_t>((tiles + 3) / 4, 8192);
    hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)blocks), dim3(256), 0, s, d, x, n, y);
    return hipGetLastError();
}

hipError_t launch_tree_sweep(const MlpDev &d, const SweepArgs &a, hipStream_t s)
{
    if (a.n_trees <= 0 || a.n_re <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_tree_sweep, dim3(a.n_trees), dim3(64), 0, s, d, a);
    return hipGetLastError();
}

hipError_t launch_analytic_sweep(const SweepArgs &a, hipStream_t s)
{
    if (a.n_trees <= 0 || a.n_re <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_analytic_sweep<false>, dim3(a.n_trees), dim3(64), 0, s, a, CfArgs{});
    return hipGetLastError();
}

hipError_t launch_analytic_split(const SweepArgs &a, const CfArgs &c, hipStream_t s)
{
    if (a.n_trees <= 0 || a.n_re <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_analytic_sweep<true>, dim3(a.n_trees), dim3(64), 0, s, a, c);
    return hipGetLastError();
}

hipError_t launch_frontal_area(const float *rec, const int64_t *tree_start, int n_trees, float h, float *area,
                               hipStream_t s)
{
    if (n_trees <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_frontal_area, dim3(n_trees), dim3(256), 0, s, rec, tree_start, h, area);
    return hipGetLastError();
}

// Gradient workspace of lbm_mlp_grad_noalloc: the reduced row, then the
// partial sums of MLP_STATIC_CHUNKS chunks (18.9 MB per device, held until the
// process ends).  Host code never passes the symbol itself to a kernel: the
// address hipGetSymbolAddress returns for each device is what the kernels take.
static __device__ __align__(256) float scratch[(size_t)(MLP_STATIC_CHUNKS + 1) * MLP_PSTRIDE];

hipError_t mlp_static_scratch(int device, float **ptr)
{
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static float *addr[MAX_DEV] = {};
    if (device < 0 || device >= MAX_DEV)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[device] = static_cast<float *>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace lbm
