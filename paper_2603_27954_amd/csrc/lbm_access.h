// Layout-aware access to the population arrays of a level (dense x-pencils
// or sparse blocks) for the HIP kernels: scalar-base accessors, per-lane
// neighbour addressing inside blocks, and the pre-collision read / write
// positions of a cell under the A-A pattern.
#pragma once
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// Accessors: a uniform (scalar) base pointer plus a 32-bit byte offset per
// lane, the form that lowers to global loads/stores with an SGPR base and a
// single VGPR offset (per-direction arrays stay below 4 GiB).
template <typename S>
__device__ __forceinline__ const S *at(const void *base, uint32_t elem)
{
    return reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + elem * (uint32_t)sizeof(S));
}
template <typename S>
__device__ __forceinline__ S *at(void *base, uint32_t elem)
{
    return reinterpret_cast<S *>(reinterpret_cast<char *>(base) + elem * (uint32_t)sizeof(S));
}
template <typename S>
__device__ __forceinline__ float ldp(const void *base, uint32_t elem)
{
    return Store<S>::ld(*at<S>(base, elem));
}
template <typename S>
__device__ __forceinline__ void stp(void *base, uint32_t elem, float v)
{
    *at<S>(base, elem) = Store<S>::st(v);
}
template <typename S>
__device__ __forceinline__ float ldp_nt(const void *base, uint32_t elem)
{
    if constexpr (sizeof(S) == 4) {
        return __builtin_nontemporal_load(reinterpret_cast<const float *>(at<S>(base, elem)));
    } else {
        const unsigned short bits = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(at<S>(base, elem)));
        return Store<S>::ld(__builtin_bit_cast(S, bits));
    }
}
template <typename S>
__device__ __forceinline__ void stp_nt(void *base, uint32_t elem, float v)
{
    if constexpr (sizeof(S) == 4) {
        __builtin_nontemporal_store(v, reinterpret_cast<float *>(at<S>(base, elem)));
    } else {
        const S h = Store<S>::st(v);
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, h), reinterpret_cast<unsigned short *>(at<S>(base, elem)));
    }
}

// equilibrium deviation of direction i in the inlet ghost cell at (ty, tz)
__device__ __forceinline__ float inlet_dev(const CollideArgs &a, const float *plane, int i, int ty, int tz)
{
    float ux = a.u_in, uy = 0.0f, uz = 0.0f;
    if (plane) {
        const float *p = plane + 3 * ((size_t)tz * a.ny + ty);
        ux += p[0];
        uy = p[1];
        uz = p[2];
    }
    return feq_dev(i, ux, uy, uz);
}

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Inflow-type lateral and vertical faces (Sec. 2.3): a population whose
// source cell lies outside the box in y or z comes from a ghost holding the
// undisturbed inflow f_eq(1, u_in e_x); these faces take precedence over the
// inlet and outlet ghosts at the box's edges.
__device__ __forceinline__ bool lateral_source(const CollideArgs &a, int ys, int zs)
{
    return a.lateral && (ys < 0 || ys >= a.ny || zs < 0 || zs >= a.nz);
}

// Per-lane neighbour addressing: for an offset s in {-1,0,1} along each axis
// the local part of the neighbour's cell index and its contribution to the
// 3x3x3 block-offset code.
template <int B>
struct NbrLane {
    static constexpr int LB = B == 16 ? 4 : 3;
    int lx[3], ly[3], lz[3], kx[3], ky[3], kz[3];
    __device__ __forceinline__ NbrLane(int x, int y, int z)
    {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int xs = x + s - 1, ys = y + s - 1, zs = z + s - 1;
            lx[s] = xs & (B - 1);
            ly[s] = (ys & (B - 1)) << LB;
            lz[s] = (zs & (B - 1)) << (2 * LB);
            kx[s] = xs < 0 ? 0 : (xs >= B ? 2 : 1);
            ky[s] = 3 * (ys < 0 ? 0 : (ys >= B ? 2 : 1));
            kz[s] = 9 * (zs < 0 ? 0 : (zs >= B ? 2 : 1));
        }
    }
    __device__ __forceinline__ int code(int sx, int sy, int sz) const { return kx[sx] + ky[sy] + kz[sz]; }
    __device__ __forceinline__ int local(int sx, int sy, int sz) const { return lx[sx] + ly[sy] + lz[sz]; }
};

template <int B>
__device__ __forceinline__ uint32_t block_neighbour(const CollideArgs &a, uint32_t elem, int dx, int dy, int dz)
{
    constexpr int CELLS = B * B * B;
    constexpr int LB = B == 16 ? 4 : 3;
    const int blk = (int)(elem / CELLS), c = (int)(elem % CELLS);
    const int x = (c & (B - 1)) + dx, y = ((c >> LB) & (B - 1)) + dy, z = (c >> (2 * LB)) + dz;
    const int code = (x < 0 ? 0 : (x >= B ? 2 : 1)) + 3 * (y < 0 ? 0 : (y >= B ? 2 : 1)) + 9 * (z < 0 ? 0 : (z >= B ? 2 : 1));
    const int n = a.nbr[(size_t)blk * 27 + code];
    return (uint32_t)n * CELLS + ((x & (B - 1)) | ((y & (B - 1)) << LB) | ((z & (B - 1)) << (2 * LB)));
}

// Pre-collision populations of the cell at element address elem for the next
// step of the level (its read positions, with the inlet and outlet ghosts).
template <int B, typename S, bool ODD>
__device__ __forceinline__ void load_pre(const CollideArgs &a, uint32_t elem, float (&g)[NQ])
{
    if (!ODD) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            g[k] = ldp<S>(a.pop[k], elem);
        return;
    }
    const size_t pl = (size_t)a.ny * a.nz;
    if (a.dense) {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const int x = (int)(elem % (uint32_t)nx);
        const uint32_t yz = elem / (uint32_t)nx;
        const int y = (int)(yz % (uint32_t)ny), z = (int)(yz / (uint32_t)ny);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            int xs = x + qcx(k);
            const int ys = wrapi(y + qcy(k), ny), zs = wrapi(z + qcz(k), nz);
            if (lateral_source(a, y + qcy(k), z + qcz(k))) {
                g[qopp(k)] = inlet_dev(a, nullptr, qopp(k), 0, 0);
            } else if (a.faces && xs < 0) {
                g[qopp(k)] = inlet_dev(a, a.in_prev, qopp(k), ys, zs);
            } else if (a.faces && xs >= nx) {
                g[qopp(k)] = a.gbuf[qopp(k) * pl + (size_t)zs * ny + ys];
            } else {
                xs = wrapi(xs, nx);
                g[qopp(k)] = ldp<S>(a.pop[k], (uint32_t)xs + (uint32_t)nx * ((uint32_t)ys + (uint32_t)ny * zs));
            }
        }
        return;
    }
    constexpr int CELLS = B * B * B;
    constexpr int LB = B == 16 ? 4 : 3;
    const int blk = (int)(elem / CELLS), c = (int)(elem % CELLS);
    const int x = c & (B - 1), y = (c >> LB) & (B - 1), z = c >> (2 * LB);
    const NbrLane<B> L(x, y, z);
    const int *nb = a.nbr + (size_t)blk * 27;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int sx = qcx(k) + 1, sy = qcy(k) + 1, sz = qcz(k) + 1;
        const int n = nb[L.code(sx, sy, sz)];
        g[qopp(k)] = ldp<S>(a.pop[k], (uint32_t)n * CELLS + L.local(sx, sy, sz));
    }
}

// Writes pre-collision populations g of the cell at elem into the positions
// the level's next step reads them from (even: slot i of the cell; odd:
// population opp(k) into slot k of x + c_k).  Used for cells whose state is
// rebuilt by the coarse/fine transfer; those never touch the box faces.
template <int B, typename S, bool ODD>
__device__ __forceinline__ void store_pre(const CollideArgs &a, uint32_t elem, const float (&g)[NQ])
{
    if (!ODD) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            stp<S>(a.pop[k], elem, g[k]);
        return;
    }
    if (a.dense) {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const int x = (int)(elem % (uint32_t)nx);
        const uint32_t yz = elem / (uint32_t)nx;
        const int y = (int)(yz % (uint32_t)ny), z = (int)(yz / (uint32_t)ny);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int xs = wrapi(x + qcx(k), nx), ys = wrapi(y + qcy(k), ny), zs = wrapi(z + qcz(k), nz);
            stp<S>(a.pop[k], (uint32_t)xs + (uint32_t)nx * ((uint32_t)ys + (uint32_t)ny * zs), g[qopp(k)]);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        stp<S>(a.pop[k], block_neighbour<B>(a, elem, qcx(k), qcy(k), qcz(k)), g[qopp(k)]);
}

// Post-collision populations of one cell stored where the collide kernel of
// the same A-A parity stores them (even: population k into slot opp(k) of the
// cell; odd: into slot k of x + c_k), for the directions k set in mask only.
template <int B, typename S, bool ODD>
__device__ __forceinline__ void store_post_masked(const CollideArgs &a, uint32_t elem, const float (&g)[NQ],
                                                  uint32_t mask)
{
    if (!ODD) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if ((mask >> k) & 1u)
                stp<S>(a.pop[qopp(k)], elem, g[k]);
        return;
    }
    if (a.dense) {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const int x = (int)(elem % (uint32_t)nx);
        const uint32_t yz = elem / (uint32_t)nx;
        const int y = (int)(yz % (uint32_t)ny), z = (int)(yz / (uint32_t)ny);
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if ((mask >> k) & 1u) {
                const int xs = wrapi(x + qcx(k), nx), ys = wrapi(y + qcy(k), ny), zs = wrapi(z + qcz(k), nz);
                stp<S>(a.pop[k], (uint32_t)xs + (uint32_t)nx * ((uint32_t)ys + (uint32_t)ny * zs), g[k]);
            }
        return;
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        if ((mask >> k) & 1u)
            stp<S>(a.pop[k], block_neighbour<B>(a, elem, qcx(k), qcy(k), qcz(k)), g[k]);
}

// store_pre for the populations k with k % parts == part only
template <int B, typename S, bool ODD>
__device__ __forceinline__ void store_pre_part(const CollideArgs &a, uint32_t elem, const float (&g)[NQ], int part,
                                               int parts)
{
    if (!ODD) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if (k % parts == part)
                stp<S>(a.pop[k], elem, g[k]);
        return;
    }
    if (a.dense) {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const int x = (int)(elem % (uint32_t)nx);
        const uint32_t yz = elem / (uint32_t)nx;
        const int y = (int)(yz % (uint32_t)ny), z = (int)(yz / (uint32_t)ny);
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if (k % parts == part) {
                const int xs = wrapi(x + qcx(k), nx), ys = wrapi(y + qcy(k), ny), zs = wrapi(z + qcz(k), nz);
                stp<S>(a.pop[k], (uint32_t)xs + (uint32_t)nx * ((uint32_t)ys + (uint32_t)ny * zs), g[qopp(k)]);
            }
        return;
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        if (k % parts == part)
            stp<S>(a.pop[k], block_neighbour<B>(a, elem, qcx(k), qcy(k), qcz(k)), g[qopp(k)]);
}

}  // namespace lbm
