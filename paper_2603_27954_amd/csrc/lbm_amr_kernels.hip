// Coarse/fine coupling kernels of the octree levels (paper Sec. 2.2: the LBM
// runs on leaf blocks of several resolutions).  Transfer runs in moment space:
//  - k_amr_moments: (density, velocity, strain rate) of listed cells of the
//    coarse level from their pre-collision populations;
//  - k_amr_prolong: each fine ghost cell interpolates those quantities
//    trilinearly (3/4 and 1/4 per axis) from its 2x2x2 coarse stencil, at the
//    fine time level (the coarse values at T, or the mean of T and T+1), and
//    its pre-collision populations are rebuilt with the fine rate and step
//    (all cumulants above the second order zero);
//  - k_amr_restrict: each coarse band cell averages its eight fine children
//    (mean density, mass-weighted velocity, mean strain rate) and is rebuilt
//    with the coarse rate and step.
// Rebuilt populations are written to the read positions of the level's next
// step (A-A parity aware).
#include "lbm_bodies.h"

namespace lbm {

template <int B, typename S, bool ODD>
__global__ void __launch_bounds__(256) k_amr_moments(const CollideArgs a, const uint32_t *cells, int n, float om1,
                                                     float dt, float *out)
{
    amr_moments_item<B, S, ODD>(a, cells, n, om1, dt, out, blockIdx.x * blockDim.x + threadIdx.x);
}

template <int B, typename S, bool ODD>
__global__ void __launch_bounds__(256) k_amr_prolong(const CollideArgs fine, const uint32_t *ghosts,
                                                     const uint32_t *gmask, const int32_t *src, int n, int nsrc,
                                                     const float *m0, const float *m1, float om1, float dt)
{
    amr_prolong_item<B, S, ODD>(fine, ghosts, gmask, src, n, nsrc, m0, m1, om1, dt,
                                blockIdx.x * blockDim.x + threadIdx.x);
}

// 64 band cells per 256-thread work-group: two passes of eight lanes per cell,
// then wave 0 rebuilds all 64
constexpr int RESTRICT_WG = 64;

template <int B, typename S, bool ODD_C, bool ODD_F>
__global__ void __launch_bounds__(256) k_amr_restrict(const CollideArgs coarse, const CollideArgs fine,
                                                      const uint32_t *band, const uint32_t *child, int n, float om_c,
                                                      float dt_c, float om_f, float dt_f)
{
    __shared__ float rec[11][RESTRICT_WG];
    amr_restrict_item<B, S, ODD_C, ODD_F, 256, RESTRICT_WG>(coarse, fine, band, child, n, om_c, dt_c, om_f, dt_f,
                                                            blockIdx.x, rec);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int B, typename S>
static void moments_t(int odd, const CollideArgs &a, const uint32_t *cells, int n, float om1, float dt, float *out,
                      hipStream_t s)
{
    const dim3 grid((n + 255) / 256), blk(256);
    if (odd)
        hipLaunchKernelGGL((k_amr_moments<B, S, true>), grid, blk, 0, s, a, cells, n, om1, dt, out);
    else
        hipLaunchKernelGGL((k_amr_moments<B, S, false>), grid, blk, 0, s, a, cells, n, om1, dt, out);
}

template <int B, typename S>
static void prolong_t(int odd, const CollideArgs &f, const uint32_t *ghosts, const uint32_t *gmask,
                      const int32_t *src, int n, int nsrc,
                      const float *m0, const float *m1, float om1, float dt, hipStream_t s)
{
    const dim3 grid((n + 255) / 256), blk(256);
    if (odd)
        hipLaunchKernelGGL((k_amr_prolong<B, S, true>), grid, blk, 0, s, f, ghosts, gmask, src, n, nsrc, m0, m1, om1, dt);
    else
        hipLaunchKernelGGL((k_amr_prolong<B, S, false>), grid, blk, 0, s, f, ghosts, gmask, src, n, nsrc, m0, m1, om1, dt);
}

template <int B, typename S>
static void restrict_t(int odd_c, int odd_f, const CollideArgs &c, const CollideArgs &f, const uint32_t *band,
                       const uint32_t *child, int n, float om_c, float dt_c, float om_f, float dt_f, hipStream_t s)
{
    const dim3 grid((n + RESTRICT_WG - 1) / RESTRICT_WG), blk(256);
#define LBM_RS(OC, OF) \
    hipLaunchKernelGGL((k_amr_restrict<B, S, OC, OF>), grid, blk, 0, s, c, f, band, child, n, om_c, dt_c, om_f, dt_f)
    if (odd_c && odd_f) LBM_RS(true, true);
    else if (odd_c) LBM_RS(true, false);
    else if (odd_f) LBM_RS(false, true);
    else LBM_RS(false, false);
#undef LBM_RS
}

#define LBM_DISPATCH(FN, ...)                                            \
    do {                                                                 \
        if (B == 16) {                                                   \
            if (storage == 0) FN<16, float>(__VA_ARGS__);                \
            else if (storage == 1) FN<16, __half>(__VA_ARGS__);          \
            else FN<16, __hip_bfloat16>(__VA_ARGS__);                    \
        } else {                                                         \
            if (storage == 0) FN<8, float>(__VA_ARGS__);                 \
            else if (storage == 1) FN<8, __half>(__VA_ARGS__);           \
            else FN<8, __hip_bfloat16>(__VA_ARGS__);                     \
        }                                                                \
    } while (0)

hipError_t launch_amr_moments(int B, int storage, int odd, const CollideArgs &a, const uint32_t *cells, int n,
                              float om1, float dt, float *out, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    LBM_DISPATCH(moments_t, odd, a, cells, n, om1, dt, out, s);
    return hipGetLastError();
}

hipError_t launch_amr_prolong(int B, int storage, int odd, const CollideArgs &fine, const uint32_t *ghosts,
                              const uint32_t *gmask, const int32_t *src, int n, int nsrc, const float *m0, const float *m1, float om1,
                              float dt, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    LBM_DISPATCH(prolong_t, odd, fine, ghosts, gmask, src, n, nsrc, m0, m1, om1, dt, s);
    return hipGetLastError();
}

hipError_t launch_amr_restrict(int B, int storage, int odd_c, int odd_f, const CollideArgs &coarse,
                               const CollideArgs &fine, const uint32_t *band, const uint32_t *child, int n,
                               float om_c, float dt_c, float om_f, float dt_f, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    LBM_DISPATCH(restrict_t, odd_c, odd_f, coarse, fine, band, child, n, om_c, dt_c, om_f, dt_f, s);
    return hipGetLastError();
}

}  // namespace lbm
