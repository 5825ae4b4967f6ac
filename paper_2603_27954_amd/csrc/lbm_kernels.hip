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
#include "lbm_access.h"

namespace lbm {

// ---------------------------------------------------------------------------
// collide and stream: dense (x-pencil) levels
// ---------------------------------------------------------------------------

// Odd step when every wavefront lies in one x-row (nx a multiple of 64): y and
// z are wave-uniform, so the eight neighbour-row offsets live in scalar
// registers and each direction addresses (scalar base + row offset) + one of
// three lane offsets (x-1, x, x+1; wrapped inside the row so every address
// stays in the level).
template <typename S>
__device__ __forceinline__ void dense_odd_rowwave(const CollideArgs &a, uint32_t own, int x, bool at_in,
                                                  bool at_out)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t first = __builtin_amdgcn_readfirstlane(own - (uint32_t)x);  // row start, uniform
    const uint32_t row = first / (uint32_t)nx;
    const int y = (int)(row % (uint32_t)ny), z = (int)(row / (uint32_t)ny);
    const int ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
    const int zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
    const uint32_t vx[3] = {x == 0 ? own + (uint32_t)nx - 1u : own - 1u, own,
                            x == nx - 1 ? own + 1u - (uint32_t)nx : own + 1u};
    float g[NQ];
    const S *bk[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int64_t roff = ((int64_t)ys[qcy(k) + 1] + (int64_t)ny * zs[qcz(k) + 1] - ((int64_t)y + (int64_t)ny * z)) * nx;
        bk[k] = reinterpret_cast<const S *>(a.pop[k]) + roff;
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        g[qopp(k)] = ldp<S>(bk[k], vx[qcx(k) + 1]);
    if (at_in || at_out) {
        const size_t pl = (size_t)ny * nz;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int ty = ys[qcy(k) + 1], tz = zs[qcz(k) + 1];
            if (at_in && qcx(k) == -1)
                g[qopp(k)] = inlet_dev(a, a.in_prev, qopp(k), ty, tz);
            if (at_out && qcx(k) == 1)
                g[qopp(k)] = a.gbuf[qopp(k) * pl + (size_t)tz * ny + ty];
        }
    }
    collide(g, a.om1, a.om2, a.galilean != 0);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const bool leaves = (at_in && qcx(k) == -1) || (at_out && qcx(k) == 1);
        if (!leaves)
            stp<S>(const_cast<S *>(bk[k]), vx[qcx(k) + 1], g[k]);
    }
    if (at_in) {
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (qcx(i) == 1)
                stp<S>(a.pop[i], own, inlet_dev(a, a.in_cur, i, ys[1 - qcy(i)], zs[1 - qcz(i)]));
    }
    if (at_out) {
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (qcx(i) == -1)
                stp<S>(a.pop[i], (uint32_t)x + (uint32_t)nx * ((uint32_t)ys[qcy(i) + 1] + (uint32_t)ny * zs[qcz(i) + 1]), g[i]);
    }
}

template <typename S, bool ODD, bool ROWWAVE>
__global__ void __launch_bounds__(256) k_collide_dense(const CollideArgs a)
{
    const int item = blockIdx.x;
    if (item >= a.n_work)
        return;
    const uint2 w = a.work[item];
    const int t = threadIdx.x;
    if (w.y != FULL_MASK) {
        const uint32_t *m = a.masks + (size_t)w.y * (DENSE_TILE / 32);
        if (!((m[t >> 5] >> (t & 31)) & 1u))
            return;
    }
    const uint32_t own = w.x * DENSE_TILE + t;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int x = (int)(own % (uint32_t)nx);
    const uint32_t yz = own / (uint32_t)nx;
    const int y = (int)(yz % (uint32_t)ny), z = (int)(yz / (uint32_t)ny);
    const bool at_in = a.faces && x == 0, at_out = a.faces && x == nx - 1;
    float g[NQ];

    if (!ODD) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            g[k] = ldp_nt<S>(a.pop[k], own);
        collide(g, a.om1, a.om2, a.galilean != 0);
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            stp_nt<S>(a.pop[qopp(k)], own, g[k]);
        if (at_out) {
            const size_t pl = (size_t)ny * nz;
#pragma unroll
            for (int i = 0; i < NQ; ++i)
                if (qcx(i) == -1)
                    a.gbuf[i * pl + (size_t)z * ny + y] = g[i];
        }
        return;
    }

    if (ROWWAVE) {
        dense_odd_rowwave<S>(a, own, x, at_in, at_out);
        return;
    }
    // odd: population opp(k) comes from slot k of x + c_k, f*_k goes back there
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ys[3] = {ym, y, yp}, zs[3] = {zm, z, zp}, xs[3] = {xm, x, xp};
    uint32_t addr[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        addr[k] = (uint32_t)xs[qcx(k) + 1] + (uint32_t)nx * ((uint32_t)ys[qcy(k) + 1] + (uint32_t)ny * zs[qcz(k) + 1]);
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        g[qopp(k)] = ldp<S>(a.pop[k], addr[k]);
    if (at_in || at_out) {
        const size_t pl = (size_t)ny * nz;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int ty = ys[qcy(k) + 1], tz = zs[qcz(k) + 1];
            if (at_in && qcx(k) == -1)  // enters from the inlet ghost at (y + cy_k, z + cz_k)
                g[qopp(k)] = inlet_dev(a, a.in_prev, qopp(k), ty, tz);
            if (at_out && qcx(k) == 1)  // enters from the outlet ghost, a copy of plane nx-1
                g[qopp(k)] = a.gbuf[qopp(k) * pl + (size_t)tz * ny + ty];
        }
    }
    collide(g, a.om1, a.om2, a.galilean != 0);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const bool leaves = (at_in && qcx(k) == -1) || (at_out && qcx(k) == 1);
        if (!leaves)
            stp<S>(a.pop[k], addr[k], g[k]);
    }
    if (at_in) {
        // populations entering from the inlet ghost for the next (even) step
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (qcx(i) == 1)
                stp<S>(a.pop[i], own, inlet_dev(a, a.in_cur, i, ys[1 - qcy(i)], zs[1 - qcz(i)]));
    }
    if (at_out) {
        // the outlet ghost (nx, y, z) copies this cell; its populations with
        // cx = -1 land on (nx - 1, y + cy, z + cz)
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (qcx(i) == -1)
                stp<S>(a.pop[i], (uint32_t)x + (uint32_t)nx * ((uint32_t)ys[qcy(i) + 1] + (uint32_t)ny * zs[qcz(i) + 1]), g[i]);
    }
}

// ---------------------------------------------------------------------------
// collide and stream: block levels (refined, sparse)
// ---------------------------------------------------------------------------

template <int B, typename S, bool ODD>
__device__ __forceinline__ void cell_update_block(const CollideArgs &a, int blk, int c, const int *nb)
{
    constexpr int CELLS = B * B * B;
    constexpr int LB = B == 16 ? 4 : 3;
    const int x = c & (B - 1), y = (c >> LB) & (B - 1), z = c >> (2 * LB);
    const uint32_t own = (uint32_t)blk * CELLS + c;
    float g[NQ];
    if (!ODD) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            g[k] = ldp_nt<S>(a.pop[k], own);
        collide(g, a.om1, a.om2, a.galilean != 0);
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            stp_nt<S>(a.pop[qopp(k)], own, g[k]);
        return;
    }
    const NbrLane<B> L(x, y, z);
    uint32_t addr[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int sx = qcx(k) + 1, sy = qcy(k) + 1, sz = qcz(k) + 1;
        addr[k] = (uint32_t)nb[L.code(sx, sy, sz)] * CELLS + L.local(sx, sy, sz);
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        g[qopp(k)] = ldp<S>(a.pop[k], addr[k]);
    collide(g, a.om1, a.om2, a.galilean != 0);
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        stp<S>(a.pop[k], addr[k], g[k]);
}

template <int B, typename S, bool ODD>
__global__ void __launch_bounds__(256) k_collide_block(const CollideArgs a)
{
    constexpr int CELLS = B * B * B;
    const int wg = blockIdx.x;
    const int item = wg / a.parts, part = wg - item * a.parts;
    if (item >= a.n_work)
        return;
    const uint2 w = a.work[item];
    const int blk = (int)w.x;
    __shared__ int nb[27];
    if (threadIdx.x < 27)
        nb[threadIdx.x] = a.nbr[(size_t)blk * 27 + threadIdx.x];
    __syncthreads();
    const int tile = CELLS / a.parts;
    const int c0 = part * tile;
    const uint32_t *mask = w.y == FULL_MASK ? nullptr : a.masks + (size_t)w.y * (CELLS / 32);
    for (int c = c0 + (int)threadIdx.x; c < c0 + tile; c += (int)blockDim.x) {
        if (mask && !((mask[c >> 5] >> (c & 31)) & 1u))
            continue;
        cell_update_block<B, S, ODD>(a, blk, c, nb);
    }
}

template <typename S>
static hipError_t launch_collide_s(int B, int odd, const CollideArgs &a, int threads, int lds, hipStream_t s)
{
    if (a.n_work == 0)
        return hipSuccess;
    if (a.dense) {
        if (!odd)
            hipLaunchKernelGGL((k_collide_dense<S, false, false>), dim3(a.n_work), dim3(DENSE_TILE), lds, s, a);
        else if (a.nx % 64 == 0)
            hipLaunchKernelGGL((k_collide_dense<S, true, true>), dim3(a.n_work), dim3(DENSE_TILE), lds, s, a);
        else
            hipLaunchKernelGGL((k_collide_dense<S, true, false>), dim3(a.n_work), dim3(DENSE_TILE), lds, s, a);
        return hipGetLastError();
    }
    const dim3 grid(a.n_work * a.parts), blk(threads);
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

// ---------------------------------------------------------------------------
// interpolated bounce-back (Bouzidi, linear) + momentum exchange
// ---------------------------------------------------------------------------

template <typename S, bool ODD_DONE>
__global__ void __launch_bounds__(256) k_links(const LinkArgs a)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.n)
        return;
    const uint8_t dj = a.dir[l];
    const int j = dj & 31, jb = 26 - j;
    const bool up = (dj & 0x80) != 0;
    const float q = a.q[l];
    const uint32_t af = a.af[l], ap = a.ap[l], am = a.am[l];
    const S *pj = reinterpret_cast<const S *>(a.pop + (size_t)j * a.dir_bytes);
    const S *pjb = reinterpret_cast<const S *>(a.pop + (size_t)jb * a.dir_bytes);
    float g1, g2, g3;  // f*_j(x_f), f*_j(x_f - c_j), f*_opp(j)(x_f)
    if (!ODD_DONE) {
        g1 = Store<S>::ld(pjb[af]);
        g3 = Store<S>::ld(pj[af]);
        g2 = up ? Store<S>::ld(pjb[am]) : 0.0f;
    } else {
        g1 = Store<S>::ld(pj[ap]);
        g3 = Store<S>::ld(pjb[am]);
        g2 = up ? Store<S>::ld(pj[af]) : 0.0f;
    }
    float gn;
    if (q < 0.5f)
        gn = up ? fmaf(2.0f * q, g1 - g2, g2) : g1;
    else {
        const float r = 0.5f / q;
        gn = fmaf(r, g1 - g3, g3);
    }
    S *dst = reinterpret_cast<S *>(a.pop + (size_t)(ODD_DONE ? jb : j) * a.dir_bytes);
    dst[ODD_DONE ? af : ap] = Store<S>::st(gn);
    if (a.lforce) {
        const float wj = w1d(qcx(j)) * w1d(qcy(j)) * w1d(qcz(j));
        const float mom = 2.0f * wj + g1 + gn;
        a.lforce[3 * (size_t)l + 0] = qcx(j) * mom;
        a.lforce[3 * (size_t)l + 1] = qcy(j) * mom;
        a.lforce[3 * (size_t)l + 2] = qcz(j) * mom;
    }
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

// ---------------------------------------------------------------------------
// FP64 reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_down(v, o, 64);
    return v;
}

// Sum of a work-group's values in a fixed order (lane tree per wave, then
// waves in order): the same inputs give the same bits on every run.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i)
            t += sh[i];
    __syncthreads();
    return t;
}

// One work-group per branch segment (links sorted by branch); the last
// work-group to finish adds the per-branch sums in branch order into the total,
// appends it to the sample ring at the device-held position ring_pos (so a
// captured graph replays with the right slot) and resets the counter.
__global__ void __launch_bounds__(256) k_branch_reduce(const float *lforce, const int *seg, int nseg,
                                                       double *sample, double *acc_branch,
                                                       double *acc_total, double *ring,
                                                       unsigned long long *ring_pos, unsigned *counter)
{
    __shared__ double sh[4];
    __shared__ bool last;
    const int b = blockIdx.x;
    const int s0 = seg[b], s1 = seg[b + 1];
    double v[3] = {0.0, 0.0, 0.0};
    for (int l = s0 + (int)threadIdx.x; l < s1; l += 256) {
        v[0] += (double)lforce[3 * (size_t)l];
        v[1] += (double)lforce[3 * (size_t)l + 1];
        v[2] += (double)lforce[3 * (size_t)l + 2];
    }
    for (int a = 0; a < 3; ++a) {
        const double t = block_sum<256>(v[a], sh);
        if (threadIdx.x == 0) {
            sample[3 * b + a] = t;
            acc_branch[3 * b + a] += t;
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(counter, 1u) == (unsigned)nseg - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        double t[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < nseg; ++i)
            for (int a = 0; a < 3; ++a)
                t[a] += __builtin_nontemporal_load(&sample[3 * i + a]);
        const unsigned long long slot = *ring_pos % RING;
        for (int a = 0; a < 3; ++a) {
            acc_total[a] += t[a];
            ring[3 * slot + a] = t[a];
        }
        *ring_pos += 1ull;
        *counter = 0u;
    }
}

hipError_t launch_branch_reduce(const float *lforce, const int *seg, int nseg, double *sample,
                                double *acc_branch, double *acc_total, double *ring,
                                unsigned long long *ring_pos, unsigned *counter, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_branch_reduce, dim3(nseg), dim3(256), 0, s, lforce, seg, nseg, sample,
                       acc_branch, acc_total, ring, ring_pos, counter);
    return hipGetLastError();
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
