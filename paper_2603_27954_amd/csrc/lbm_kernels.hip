// HIP kernels for gfx950: collide-and-stream with in-place A-A streaming,
// interpolated bounce-back with momentum exchange, FP64 force and mass
// reductions, initialisation and state transfer (paper Sec. 2.2).
//
// Storage: per level, one array per direction i (structure of arrays).  A
// level that covers its whole box (the uniform grid, the coarsest level) is
// stored as x-pencils: cell (x, y, z) at element x + nx (y + ny z), so x
// neighbours stay contiguous across the whole row.  A sparse (refined) level
// holds (nb + 1) cubic blocks of B^3 cells, block nb being a sink for absent
// neighbours: cell c = x + B (y + B z) of block b at element b * B^3 + c.
// Values are deviations g = f - w.  Even steps use non-temporal loads and
// stores (pure streaming); odd steps keep the caches, which merge the
// neighbour-shifted partial lines.
//
// A-A pattern (one array, in place): an even step reads population i of cell
// x from slot i of x and writes the post-collision f*_i to slot opp(i) of x; an
// odd step reads population opp(k) of x from slot k of x + c_k and writes f*_k
// to the same slot k of x + c_k.  Each cell touches a set of slots no other
// cell touches, so a step needs no second array and no intra-step barrier.
// After an even number of steps population i of x sits in slot i of x.
#include "lbm_bodies.h"

namespace lbm {

// Work-groups are dispatched round-robin over the 8 XCDs (work-group b runs on
// XCD b % 8), and each XCD has its own L2.  With group size K (a.xcd_group),
// work-group b takes item s 8K + (b % 8) K + j, where s = b / 8K and
// j = (b % 8K) / 8.  Each XCD then walks runs of K consecutive tiles, so the
// cache line two neighbouring tiles of a run share (the x-shifted boundary of
// the odd step) is fetched into one L2 rather than two.  The runs interleave
// over the XCDs, which keeps the concurrently active addresses compact.  K = 1
// is the plain order.  The grid is a multiple of 8K; surplus work-groups exit.
__device__ __forceinline__ int xcd_item(int b, int k)
{
    const int span = 8 * k, s = b / span, r = b - s * span;
    return s * span + (r & 7) * k + (r >> 3);
}

template <typename S, bool ODD, bool ROWWAVE>
__global__ void __launch_bounds__(256) k_collide_dense(const CollideArgs a)
{
    collide_dense_item<S, ODD, ROWWAVE>(a, xcd_item(blockIdx.x, a.xcd_group));
}

template <int B, typename S, bool ODD>
__global__ void __launch_bounds__(256) k_collide_block(const CollideArgs a)
{
    __shared__ int nb[27];
    const int wg = xcd_item(blockIdx.x, a.xcd_group);
    if (wg < a.n_work * a.parts)
        collide_block_item<B, S, ODD>(a, wg, nb);
}

template <typename S>
static hipError_t launch_collide_s(int B, int odd, const CollideArgs &a, int threads, int lds, hipStream_t s)
{
    if (a.n_work == 0)
        return hipSuccess;
    // grids rounded up to a multiple of 8K (see xcd_item); surplus work-groups exit
    const int span = 8 * a.xcd_group;
    if (a.dense) {
        const dim3 grid((a.n_work + span - 1) / span * span);
        if (!odd)
            hipLaunchKernelGGL((k_collide_dense<S, false, false>), grid, dim3(DENSE_TILE), lds, s, a);
        else if (a.nx % 64 == 0)
            hipLaunchKernelGGL((k_collide_dense<S, true, true>), grid, dim3(DENSE_TILE), lds, s, a);
        else
            hipLaunchKernelGGL((k_collide_dense<S, true, false>), grid, dim3(DENSE_TILE), lds, s, a);
        return hipGetLastError();
    }
    const dim3 grid((a.n_work * a.parts + span - 1) / span * span), blk(threads);
    if (B == 16) {
        if (odd)
            hipLaunchKernelGGL((k_collide_block<16, S, true>), grid, blk, lds, s, a);
        else
            hipLaunchKernelGGL((k_collide_block<16, S, false>), grid, blk, lds, s, a);
    } else {
        if (odd)
            hipLaunchKernelGGL((k_collide_block<8, S, true>), grid, blk, lds, s, a);
        else
            hipLaunchKernelGGL((k_collide_block<8, S, false>), grid, blk, lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_collide(int B, int storage, int odd, const CollideArgs &a, int threads, int lds, hipStream_t s)
{
    if (storage == 0)
        return launch_collide_s<float>(B, odd, a, threads, lds, s);
    if (storage == 1)
        return launch_collide_s<__half>(B, odd, a, threads, lds, s);
    return launch_collide_s<__hip_bfloat16>(B, odd, a, threads, lds, s);
}

template <typename S, bool ODD_DONE>
__global__ void __launch_bounds__(256) k_links(const LinkArgs a)
{
    link_update<S, ODD_DONE>(a, blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_links(int storage, int odd_done, const LinkArgs &a, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const dim3 grid((a.n + 255) / 256), blk(256);
#define LBM_LINKS(T)                                                         \
    if (odd_done)                                                            \
        hipLaunchKernelGGL((k_links<T, true>), grid, blk, 0, s, a);          \
    else                                                                     \
        hipLaunchKernelGGL((k_links<T, false>), grid, blk, 0, s, a);
    if (storage == 0) {
        LBM_LINKS(float)
    } else if (storage == 1) {
        LBM_LINKS(__half)
    } else {
        LBM_LINKS(__hip_bfloat16)
    }
#undef LBM_LINKS
    return hipGetLastError();
}

// One work-group per link piece; the last work-group to finish forms the
// per-branch sums and the total and resets the arrival counter.
__global__ void __launch_bounds__(256) k_branch_reduce(const float *lforce, const int *pstart, int npieces,
                                                       const int *segp, int nseg, double *piece_sum,
                                                       double *sample, double *acc_branch, double *acc_total,
                                                       double *ring, unsigned long long *ring_pos,
                                                       unsigned *counter)
{
    __shared__ double sh[12];
    __shared__ bool last;
    link_piece_sum(lforce, pstart, blockIdx.x, piece_sum, sh);
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(counter, 1u) == (unsigned)npieces - 1;
    }
    __syncthreads();
    if (last) {
        if (threadIdx.x == 0)
            __threadfence();
        __syncthreads();
        branch_totals(piece_sum, segp, nseg, sample, acc_branch, acc_total, ring, ring_pos, sh);
        if (threadIdx.x == 0)
            *counter = 0u;
    }
}

hipError_t launch_branch_reduce(const float *lforce, const int *pstart, int npieces, const int *segp, int nseg,
                                double *piece_sum, double *sample, double *acc_branch, double *acc_total,
                                double *ring, unsigned long long *ring_pos, unsigned *counter, hipStream_t s)
{
    if (npieces == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_branch_reduce, dim3(npieces), dim3(256), 0, s, lforce, pstart, npieces, segp, nseg,
                       piece_sum, sample, acc_branch, acc_total, ring, ring_pos, counter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// wall friction (paper Sec. 3, Eq. (8)): shear stress integrated over the
// tree surface, one axis face between a fluid cell and a solid neighbour per
// thread
// ---------------------------------------------------------------------------

// deviatoric viscous stress -(1 - omega1/2) dev(N) of a cell's non-equilibrium
// second-order central moments N (xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ void cell_stress(const Moments &m, float om1, float (&s)[6])
{
    const float c = -(1.0f - 0.5f * om1);
    const float t3 = (m.nxx + m.nyy + m.nzz) * (1.0f / 3.0f);
    s[0] = c * (m.nxx - t3);
    s[1] = c * (m.nyy - t3);
    s[2] = c * (m.nzz - t3);
    s[3] = c * m.nxy;
    s[4] = c * m.nxz;
    s[5] = c * m.nyz;
}

// The stress at the wall point x_f + q e_k (linear along the axis from x_f
// and x_f - e_k, or that of x_f alone when x_f - e_k is not fluid), its
// traction on the body's outward normal n with the normal part removed (the
// wall shear stress), times the face's share |n_k| of the surface.
template <int B, typename S, bool ODD>
__global__ void __launch_bounds__(256) k_friction(const CollideArgs a, const FricArgs f)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= f.n)
        return;
    float g[NQ], s[6];
    load_pre<B, S, ODD>(a, f.a0[t], g);
    cell_stress(forward_moments(g), f.om1, s);
    const uint32_t a1 = f.a1[t];
    if (a1 != FRIC_NO_UP) {
        float s1[6];
        load_pre<B, S, ODD>(a, a1, g);
        cell_stress(forward_moments(g), f.om1, s1);
        const float q = f.q[t];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            s[k] = fmaf(q, s[k] - s1[k], s[k]);
    }
    const float4 nw = f.nw[t];
    const float tx = s[0] * nw.x + s[3] * nw.y + s[4] * nw.z;
    const float ty = s[3] * nw.x + s[1] * nw.y + s[5] * nw.z;
    const float tz = s[4] * nw.x + s[5] * nw.y + s[2] * nw.z;
    const float tn = tx * nw.x + ty * nw.y + tz * nw.z;
    f.force[3 * (size_t)t + 0] = nw.w * (tx - tn * nw.x);
    f.force[3 * (size_t)t + 1] = nw.w * (ty - tn * nw.y);
    f.force[3 * (size_t)t + 2] = nw.w * (tz - tn * nw.z);
}

template <int B, typename S>
static hipError_t launch_friction_t(int odd, const CollideArgs &a, const FricArgs &f, hipStream_t s)
{
    const dim3 grid((f.n + 255) / 256), blk(256);
    if (odd)
        hipLaunchKernelGGL((k_friction<B, S, true>), grid, blk, 0, s, a, f);
    else
        hipLaunchKernelGGL((k_friction<B, S, false>), grid, blk, 0, s, a, f);
    return hipGetLastError();
}

hipError_t launch_friction(int B, int storage, int odd, const CollideArgs &a, const FricArgs &f, hipStream_t s)
{
    if (f.n == 0)
        return hipSuccess;
    if (B == 16) {
        if (storage == 0) return launch_friction_t<16, float>(odd, a, f, s);
        if (storage == 1) return launch_friction_t<16, __half>(odd, a, f, s);
        return launch_friction_t<16, __hip_bfloat16>(odd, a, f, s);
    }
    if (storage == 0) return launch_friction_t<8, float>(odd, a, f, s);
    if (storage == 1) return launch_friction_t<8, __half>(odd, a, f, s);
    return launch_friction_t<8, __hip_bfloat16>(odd, a, f, s);
}

// ---------------------------------------------------------------------------
// state transfer: pre-collision populations of listed cells (FP64, full f)
// ---------------------------------------------------------------------------

template <int B, typename S, bool ODD>
__global__ void __launch_bounds__(256) k_gather(const CollideArgs a, const uint32_t *cells, int n, double *out,
                                                size_t stride)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n)
        return;
    float g[NQ];
    load_pre<B, S, ODD>(a, cells[t], g);
#pragma unroll
    for (int i = 0; i < NQ; ++i)
        out[i * stride + t] = (double)g[i] + (double)qw(i);
}

template <int B, typename S>
static hipError_t launch_gather_t(int odd, const CollideArgs &a, const uint32_t *cells, int n, double *out,
                                  size_t stride, hipStream_t s)
{
    const dim3 grid((n + 255) / 256), blk(256);
    if (odd)
        hipLaunchKernelGGL((k_gather<B, S, true>), grid, blk, 0, s, a, cells, n, out, stride);
    else
        hipLaunchKernelGGL((k_gather<B, S, false>), grid, blk, 0, s, a, cells, n, out, stride);
    return hipGetLastError();
}

hipError_t launch_gather(int B, int storage, int odd, const CollideArgs &a, const uint32_t *cells, int n,
                         double *out, size_t stride, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    if (B == 16) {
        if (storage == 0) return launch_gather_t<16, float>(odd, a, cells, n, out, stride, s);
        if (storage == 1) return launch_gather_t<16, __half>(odd, a, cells, n, out, stride, s);
        return launch_gather_t<16, __hip_bfloat16>(odd, a, cells, n, out, stride, s);
    }
    if (storage == 0) return launch_gather_t<8, float>(odd, a, cells, n, out, stride, s);
    if (storage == 1) return launch_gather_t<8, __half>(odd, a, cells, n, out, stride, s);
    return launch_gather_t<8, __hip_bfloat16>(odd, a, cells, n, out, stride, s);
}

// natural layout write (even parity): slot i of the cell holds population i
template <typename S>
__global__ void __launch_bounds__(256) k_scatter(void *pop, size_t dir_elems, const uint32_t *cells, int n,
                                                 const double *in, size_t stride)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n)
        return;
    const size_t e = cells[t];
    S *p = reinterpret_cast<S *>(pop);
#pragma unroll
    for (int i = 0; i < NQ; ++i)
        p[i * dir_elems + e] = Store<S>::st((float)(in[i * stride + t] - (double)qw(i)));
}

hipError_t launch_scatter(int storage, void *pop, size_t dir_elems, const uint32_t *cells, int n, const double *in,
                          size_t stride, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const dim3 grid((n + 255) / 256), blk(256);
    if (storage == 0) hipLaunchKernelGGL(k_scatter<float>, grid, blk, 0, s, pop, dir_elems, cells, n, in, stride);
    else if (storage == 1) hipLaunchKernelGGL(k_scatter<__half>, grid, blk, 0, s, pop, dir_elems, cells, n, in, stride);
    else hipLaunchKernelGGL(k_scatter<__hip_bfloat16>, grid, blk, 0, s, pop, dir_elems, cells, n, in, stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initial state: f = f_eq(1, (u_in, 0, 0)) on the listed cells, natural layout
// ---------------------------------------------------------------------------

template <typename S>
__global__ void __launch_bounds__(256) k_init(void *pop, size_t dir_elems, const uint2 *work, int n,
                                              const uint32_t *masks, int unit, float u_in)
{
    const int item = blockIdx.x;
    if (item >= n)
        return;
    const uint2 w = work[item];
    const uint32_t *mask = w.y == FULL_MASK ? nullptr : masks + (size_t)w.y * (unit / 32);
    S *p = reinterpret_cast<S *>(pop);
    for (int c = threadIdx.x; c < unit; c += blockDim.x) {
        const size_t e = (size_t)w.x * unit + c;
        const bool fluid = !mask || ((mask[c >> 5] >> (c & 31)) & 1u);
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            p[i * dir_elems + e] = Store<S>::st(fluid ? feq_dev(i, u_in, 0.0f, 0.0f) : 0.0f);
    }
}

hipError_t launch_init(int unit, int storage, void *pop, size_t dir_elems, const uint2 *work, int n,
                       const uint32_t *masks, float u_in, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    if (storage == 0) hipLaunchKernelGGL(k_init<float>, dim3(n), dim3(256), 0, s, pop, dir_elems, work, n, masks, unit, u_in);
    else if (storage == 1) hipLaunchKernelGGL(k_init<__half>, dim3(n), dim3(256), 0, s, pop, dir_elems, work, n, masks, unit, u_in);
    else hipLaunchKernelGGL(k_init<__hip_bfloat16>, dim3(n), dim3(256), 0, s, pop, dir_elems, work, n, masks, unit, u_in);
    return hipGetLastError();
}

// zero deviations everywhere (sink block included): weights = rest state
template <typename S>
__global__ void k_zero(S *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = Store<S>::st(0.0f);
}

hipError_t launch_fill_sink_and_all(int storage, void *pop, size_t dir_elems, hipStream_t s)
{
    const size_t n = dir_elems * NQ;
    const dim3 grid(2048), blk(256);
    if (storage == 0) hipLaunchKernelGGL(k_zero<float>, grid, blk, 0, s, (float *)pop, n);
    else if (storage == 1) hipLaunchKernelGGL(k_zero<__half>, grid, blk, 0, s, (__half *)pop, n);
    else hipLaunchKernelGGL(k_zero<__hip_bfloat16>, grid, blk, 0, s, (__hip_bfloat16 *)pop, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 mass and health check over leaf fluid cells:
// out4 = {sum rho * volume, min rho, max rho, count of non-finite}
// ---------------------------------------------------------------------------

template <int B, typename S, bool ODD>
__global__ void __launch_bounds__(256) k_mass(const CollideArgs a, const uint2 *leaf, int n_leaf,
                                              double vol, double *part)
{
    const int unit = a.dense ? DENSE_TILE : B * B * B;
    __shared__ double sh[4];
    double m = 0.0, mn = 1e300, mx = -1e300, bad = 0.0;
    for (int item = blockIdx.x; item < n_leaf; item += gridDim.x) {
        const uint2 w = leaf[item];
        const uint32_t *mask = w.y == FULL_MASK ? nullptr : a.masks + (size_t)w.y * (unit / 32);
        for (int c = threadIdx.x; c < unit; c += blockDim.x) {
            if (mask && !((mask[c >> 5] >> (c & 31)) & 1u))
                continue;
            float g[NQ];
            load_pre<B, S, ODD>(a, w.x * unit + c, g);
            double r = 1.0;
            for (int i = 0; i < NQ; ++i)
                r += (double)g[i];
            if (!(r == r) || r > 1e30 || r < -1e30) {
                bad += 1.0;
                continue;
            }
            m += r * vol;
            mn = r < mn ? r : mn;
            mx = r > mx ? r : mx;
        }
    }
    const double tm = block_sum<256>(m, sh);
    const double tb = block_sum<256>(bad, sh);
    // min / max through the same tree
    __shared__ double smn[256], smx[256];
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + o]);
            smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = tm;
        part[4 * blockIdx.x + 1] = smn[0];
        part[4 * blockIdx.x + 2] = smx[0];
        part[4 * blockIdx.x + 3] = tb;
    }
}

__global__ void k_mass_final(const double *part, int n, double *out4)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double m = 0.0, mn = 1e300, mx = -1e300, bad = 0.0;
    for (int i = 0; i < n; ++i) {
        m += part[4 * i];
        mn = fmin(mn, part[4 * i + 1]);
        mx = fmax(mx, part[4 * i + 2]);
        bad += part[4 * i + 3];
    }
    out4[0] += m;
    out4[1] = fmin(out4[1], mn);
    out4[2] = fmax(out4[2], mx);
    out4[3] += bad;
}

hipError_t launch_mass(int B, int storage, int odd, const CollideArgs &a, const uint2 *leaf, int n_leaf,
                       double vol, double *out4, hipStream_t s)
{
    if (n_leaf == 0)
        return hipSuccess;
    const int nblk = n_leaf < 1024 ? n_leaf : 1024;
    double *part = out4 + 4;  // caller provides 4 + 4*1024 doubles
#define LBM_MS(BB, T)                                                                              \
    if (odd)                                                                                       \
        hipLaunchKernelGGL((k_mass<BB, T, true>), dim3(nblk), dim3(256), 0, s, a, leaf, n_leaf, vol, part); \
    else                                                                                           \
        hipLaunchKernelGGL((k_mass<BB, T, false>), dim3(nblk), dim3(256), 0, s, a, leaf, n_leaf, vol, part);
    if (B == 16) {
        if (storage == 0) { LBM_MS(16, float) }
        else if (storage == 1) { LBM_MS(16, __half) }
        else { LBM_MS(16, __hip_bfloat16) }
    } else {
        if (storage == 0) { LBM_MS(8, float) }
        else if (storage == 1) { LBM_MS(8, __half) }
        else { LBM_MS(8, __hip_bfloat16) }
    }
#undef LBM_MS
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(64), 0, s, part, nblk, out4);
    return hipGetLastError();
}

}  // namespace lbm
