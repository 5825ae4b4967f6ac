// Device bodies of the hot-path kernels, shared by the one-kernel-per-phase
// launches and by the persistent launch that runs a whole coarse step, so the
// two forms execute the same arithmetic (paper Sec. 2.2).  Each body handles
// one work item: a tile of a level (collide), one link (bounce-back), one
// branch segment (force sums) or one interface cell (coarse/fine transfer).
#pragma once
#include "lbm_access.h"

namespace lbm {

// ---------------------------------------------------------------------------
// collide and stream: dense (x-pencil) levels
// ---------------------------------------------------------------------------

// The collision of one cell (as collide()), writing first the coarse/fine
// transfer record of the cell's pre-collision state when the level keeps
// records and the cell is a prolongation source.
__device__ __forceinline__ void write_record(float *out, int r, const Transfer &tr)
{
    float4 *o = reinterpret_cast<float4 *>(out + (size_t)MOM_REC * r);
    o[0] = make_float4(tr.drho, tr.ux, tr.uy, tr.uz);
    o[1] = make_float4(tr.d[0], tr.d[1], tr.d[2], tr.d[3]);
    o[2] = make_float4(tr.d[4], tr.d[5], 0.0f, 0.0f);
}

// record index of cell own (-1: none); loaded before the populations so that
// its latency overlaps theirs
__device__ __forceinline__ int record_of(const CollideArgs &a, uint32_t own)
{
    return a.mom_idx ? a.mom_idx[own] : -1;
}

__device__ __forceinline__ void collide_rec(float (&g)[NQ], const CollideArgs &a, int r)
{
    Moments m = forward_moments(g);
    if (r >= 0)
        write_record(a.mom_out, r, to_transfer(m, a.om1, a.mom_dt));
    relax_second(m, a.om1, a.om2, a.galilean != 0);
    back_transform(m, g);
}

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
    const int rec = record_of(a, own);
    float g[NQ];
    const S *bk[NQ];
    uint32_t sink[NQ];  // offset of this row's spare element from bk[k] (wave-uniform)
    const int64_t ncell = (int64_t)nx * ny * nz + (int64_t)(row & (uint32_t)(DENSE_SINK - 1));
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int64_t roff = ((int64_t)ys[qcy(k) + 1] + (int64_t)ny * zs[qcz(k) + 1] - ((int64_t)y + (int64_t)ny * z)) * nx;
        bk[k] = reinterpret_cast<const S *>(a.pop[k]) + roff;
        sink[k] = (uint32_t)(ncell - roff);
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
    // inflow-type y and z faces (wave-uniform: the wave is one row)
    const bool ylo = a.lateral && y == 0, yhi = a.lateral && y == ny - 1;
    const bool zlo = a.lateral && z == 0, zhi = a.lateral && z == nz - 1;
    const bool lat = ylo || yhi || zlo || zhi;
    auto outside = [&](int k) {  // x + c_k leaves the box in y or z
        return (ylo && qcy(k) == -1) || (yhi && qcy(k) == 1) || (zlo && qcz(k) == -1) || (zhi && qcz(k) == 1);
    };
    if (lat) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if (outside(k))
                g[qopp(k)] = inlet_dev(a, nullptr, qopp(k), 0, 0);
    }
    collide_rec(g, a, rec);
    // every lane stores every direction (scalar base, 32-bit lane offset); a
    // population that leaves through a face goes to the spare elements, which
    // nothing reads
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const bool leaves = (at_in && qcx(k) == -1) || (at_out && qcx(k) == 1) || outside(k);
        stp<S>(const_cast<S *>(bk[k]), leaves ? sink[k] : vx[qcx(k) + 1], g[k]);
    }
    if (at_in) {
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (qcx(i) == 1)
                stp<S>(a.pop[i], own, inlet_dev(a, a.in_cur, i, ys[1 - qcy(i)], zs[1 - qcz(i)]));
    }
    if (at_out) {
        // the outlet ghost's populations land on (nx - 1, y + c_y, z + c_z),
        // unless that lies outside an inflow-type face
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (qcx(i) == -1 && !outside(i))
                stp<S>(a.pop[i], (uint32_t)x + (uint32_t)nx * ((uint32_t)ys[qcy(i) + 1] + (uint32_t)ny * zs[qcz(i) + 1]), g[i]);
    }
    if (lat) {
        // populations entering through an inflow-type face for the next
        // (even) step; last, so they take precedence at the inlet's edges
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (outside(qopp(i)))
                stp<S>(a.pop[i], own, inlet_dev(a, nullptr, i, 0, 0));
    }
}

template <typename S, bool ODD, bool ROWWAVE>
__device__ __forceinline__ void collide_dense_item(const CollideArgs &a, int item)
{
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
        const int rec = record_of(a, own);
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            g[k] = ldp_nt<S>(a.pop[k], own);
        collide_rec(g, a, rec);
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
    const int rec = record_of(a, own);
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
    // inflow-type y and z faces
    const bool ylo = a.lateral && y == 0, yhi = a.lateral && y == ny - 1;
    const bool zlo = a.lateral && z == 0, zhi = a.lateral && z == nz - 1;
    const bool lat = ylo || yhi || zlo || zhi;
    auto outside = [&](int k) {  // x + c_k leaves the box in y or z
        return (ylo && qcy(k) == -1) || (yhi && qcy(k) == 1) || (zlo && qcz(k) == -1) || (zhi && qcz(k) == 1);
    };
    if (lat) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if (outside(k))
                g[qopp(k)] = inlet_dev(a, nullptr, qopp(k), 0, 0);
    }
    collide_rec(g, a, rec);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const bool leaves = (at_in && qcx(k) == -1) || (at_out && qcx(k) == 1) || outside(k);
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
        // cx = -1 land on (nx - 1, y + cy, z + cz), unless that lies outside
        // an inflow-type face
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (qcx(i) == -1 && !outside(i))
                stp<S>(a.pop[i], (uint32_t)x + (uint32_t)nx * ((uint32_t)ys[qcy(i) + 1] + (uint32_t)ny * zs[qcz(i) + 1]), g[i]);
    }
    if (lat) {
        // populations entering through an inflow-type face for the next
        // (even) step; last, so they take precedence at the inlet's edges
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            if (outside(qopp(i)))
                stp<S>(a.pop[i], own, inlet_dev(a, nullptr, i, 0, 0));
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
    const int rec = record_of(a, own);
    float g[NQ];
    if (!ODD) {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            g[k] = ldp_nt<S>(a.pop[k], own);
        collide_rec(g, a, rec);
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
    collide_rec(g, a, rec);
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        stp<S>(a.pop[k], addr[k], g[k]);
}

// one tile (work-group item wg = block item * parts + part) of a block level;
// nb is the work-group's 27-entry neighbour table in LDS
template <int B, typename S, bool ODD>
__device__ __forceinline__ void collide_block_item(const CollideArgs &a, int wg, int *nb)
{
    constexpr int CELLS = B * B * B;
    const int item = wg / a.parts, part = wg - item * a.parts;
    if (item >= a.n_work)
        return;
    const uint2 w = a.work[item];
    const int blk = (int)w.x;
    if (ODD) {  // only the odd step reaches into neighbouring blocks
        if (threadIdx.x < 27)
            nb[threadIdx.x] = a.nbr[(size_t)blk * 27 + threadIdx.x];
        __syncthreads();
    }
    const int tile = CELLS / a.parts;
    const int c0 = part * tile;
    const uint32_t *mask = w.y == FULL_MASK ? nullptr : a.masks + (size_t)w.y * (CELLS / 32);
    for (int c = c0 + (int)threadIdx.x; c < c0 + tile; c += (int)blockDim.x) {
        if (mask && !((mask[c >> 5] >> (c & 31)) & 1u))
            continue;
        cell_update_block<B, S, ODD>(a, blk, c, nb);
    }
}


// ---------------------------------------------------------------------------
// interpolated bounce-back (Bouzidi, linear) + momentum exchange
// ---------------------------------------------------------------------------

template <typename S, bool ODD_DONE>
__device__ __forceinline__ void link_update(const LinkArgs &a, int l)
{
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
        // momentum exchange c_j (f*_j + f_opp(j)(t+1)) in gauge form: with
        // deviations g = f - w the resting state's 2 w_j, which sums to zero
        // over the closed tree, is already absent, so a branch (an open part of
        // the surface) carries gauge pressure
        const float mom = g1 + gn;
        a.lforce[3 * (size_t)l + 0] = qcx(j) * mom;
        a.lforce[3 * (size_t)l + 1] = qcy(j) * mom;
        a.lforce[3 * (size_t)l + 2] = qcz(j) * mom;
    }
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

// Work-group sums of three values at once (256 threads): lane tree within each
// wave, then the waves in order; the result is in thread 0.  sh holds 12 doubles.
__device__ __forceinline__ void block_sum3(double (&v)[3], double *sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v[a] = wave_sum(v[a]);
        if (lane == 0)
            sh[4 * a + wv] = v[a];
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            v[a] = ((sh[4 * a] + sh[4 * a + 1]) + sh[4 * a + 2]) + sh[4 * a + 3];
    __syncthreads();
}

// The links are sorted by branch and each branch's run of links is cut into
// pieces of at most LINK_PIECE links.  One work-group sums one piece in a
// fixed order (lane tree, then waves in order) and thread 0 stores the sum in
// piece_sum[3p .. 3p + 2].
__device__ __forceinline__ void link_piece_sum(const float *lforce, const int *pstart, int p, double *piece_sum,
                                               double *sh)
{
    const int s0 = pstart[p], s1 = pstart[p + 1];
    double v[3] = {0.0, 0.0, 0.0};
    for (int l0 = s0 + (int)threadIdx.x; l0 < s1; l0 += 8 * 256) {
        // eight links of this lane in flight at once, added in link order
        float buf[8][3];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int l = l0 + 256 * i;
            if (l < s1)
                for (int a = 0; a < 3; ++a)
                    buf[i][a] = lforce[3 * (size_t)l + a];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (l0 + 256 * i < s1)
                for (int a = 0; a < 3; ++a)
                    v[a] += (double)buf[i][a];
    }
    block_sum3(v, sh);
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a)
            piece_sum[3 * p + a] = v[a];
}

// Per-branch sums from the pieces of each branch, in piece order (the pieces of
// branch s are segp[s] .. segp[s + 1]), stored in sample and added to
// acc_branch; then the total over the branches (thread t adds branches t,
// t + 256, ... in order, then block_sum3) is added to acc_total and appended
// to the sample ring at the device-held position ring_pos, which a replayed
// graph advances itself (sample and ring null: the accumulators only).
// Called by the whole work-group (256 threads) after
// an acquire of the piece sums.
__device__ __forceinline__ void branch_totals(const double *piece_sum, const int *segp, int nseg, double *sample,
                                              double *acc_branch, double *acc_total, double *ring,
                                              unsigned long long *ring_pos, double *sh)
{
    double tot[3] = {0.0, 0.0, 0.0};
    for (int s = threadIdx.x; s < nseg; s += 256) {
        double t[3] = {0.0, 0.0, 0.0};
        const int q1 = segp[s + 1];
        for (int q = segp[s]; q < q1; q += 8) {
            // eight piece sums in flight at once, added in piece order
            double buf[8][3];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (q + i < q1)
                    for (int a = 0; a < 3; ++a)
                        buf[i][a] = piece_sum[3 * (q + i) + a];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (q + i < q1)
                    for (int a = 0; a < 3; ++a)
                        t[a] += buf[i][a];
        }
        for (int a = 0; a < 3; ++a) {
            if (sample)
                sample[3 * s + a] = t[a];
            acc_branch[3 * s + a] += t[a];
            tot[a] += t[a];
        }
    }
    block_sum3(tot, sh);
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a)
            acc_total[a] += tot[a];
        if (ring) {
            const unsigned long long slot = *ring_pos % RING;
            for (int a = 0; a < 3; ++a)
                ring[3 * slot + a] = tot[a];
            *ring_pos += 1ull;
        }
    }
}

// ---------------------------------------------------------------------------
// coarse/fine transfer in moment space
// ---------------------------------------------------------------------------

// one source cell per thread t; its record goes to out[MOM_REC t ..]
template <int B, typename S, bool ODD>
__device__ __forceinline__ void amr_moments_item(const CollideArgs &a, const uint32_t *cells, int n, float om1,
                                                 float dt, float *out, int t)
{
    if (t >= n)
        return;
    float g[NQ];
    load_pre<B, S, ODD>(a, cells[t], g);
    write_record(out, t, to_transfer(forward_moments(g), om1, dt));
}

__device__ __forceinline__ void mom_load(const float *m, int s, float (&x)[12])
{
    const float4 *r = reinterpret_cast<const float4 *>(m + (size_t)MOM_REC * s);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float4 v = r[k];
        x[4 * k] = v.x, x[4 * k + 1] = v.y, x[4 * k + 2] = v.z, x[4 * k + 3] = v.w;
    }
}

// One fine ghost cell per thread t.  The ghost's rebuilt pre-collision state
// is collided here as the level's own step would collide it (rates and
// Galilean flag of fine), and its post-collision populations are stored where
// that step stores them: the ghost cells are not in the level's work lists.
// Only the populations that stream into collided cells (bits of gmask[t]) are
// stored.  Run before or after the level's collide launch of the same step:
// the two touch disjoint slots.
template <int B, typename S, bool ODD>
__device__ __forceinline__ void amr_prolong_item(const CollideArgs &fine, const uint32_t *ghosts,
                                                 const uint32_t *gmask, const int32_t *src, int n, int nsrc,
                                                 const float *m0, const float *m1, float om1, float dt, int t)
{
    (void)nsrc;
    if (t >= n)
        return;
    float v[10];
#pragma unroll
    for (int k = 0; k < 10; ++k)
        v[k] = 0.0f;
    const int4 *sp = reinterpret_cast<const int4 *>(src + 8 * (size_t)t);
    const int4 s0 = sp[0], s1 = sp[1];
    const int sq[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float w = ((q & 1) ? 0.25f : 0.75f) * ((q & 2) ? 0.25f : 0.75f) * ((q & 4) ? 0.25f : 0.75f);
        float x[12];
        mom_load(m0, sq[q], x);
        if (m1) {
            float y[12];
            mom_load(m1, sq[q], y);
#pragma unroll
            for (int k = 0; k < 10; ++k)
                x[k] = 0.5f * (x[k] + y[k]);
        }
#pragma unroll
        for (int k = 0; k < 10; ++k)
            v[k] = fmaf(w, x[k], v[k]);
    }
    Transfer tr;
    tr.drho = v[0];
    tr.ux = v[1];
    tr.uy = v[2];
    tr.uz = v[3];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        tr.d[k] = v[4 + k];
    float g[NQ];
    back_transform(from_transfer(tr, om1, dt), g);
    collide(g, fine.om1, fine.om2, fine.galilean != 0);
    store_post_masked<B, S, ODD>(fine, ghosts[t], g, gmask[t]);
}

// One work-group item of NT threads covers the coarse band cells
// it * CELLS .. + CELLS - 1 (CELLS <= NT) in two stages.  Stage 1, passes of
// NT / 8 cells: eight lanes per cell, lane
// q = t & 7 holding child q; consecutive band cells run along x, so each
// population load of a wave covers whole rows of the fine level.  The
// children's sums meet over a butterfly of the eight lanes (fixed order) and
// go to the LDS record rec[.][cell].  Stage 2: threads 0 .. CELLS - 1, one per
// cell, rebuild the cells and store their populations.  Called by the whole
// work-group.
template <int B, typename S, bool ODD_C, bool ODD_F, int NT, int CELLS>
__device__ __forceinline__ void amr_restrict_item(const CollideArgs &coarse, const CollideArgs &fine,
                                                  const uint32_t *band, const uint32_t *child, int n, float om_c,
                                                  float dt_c, float om_f, float dt_f, int it, float (*rec)[CELLS])
{
    static_assert(CELLS <= NT && (8 * CELLS) % NT == 0, "whole passes of NT / 8 cells");
    const int tid = (int)threadIdx.x, q = tid & 7;
    const int base = it * CELLS;
    for (int pass = 0; pass < 8 * CELLS / NT; ++pass) {
        const int local = pass * (NT / 8) + (tid >> 3), cell = base + local;
        float v[11];
#pragma unroll
        for (int k = 0; k < 11; ++k)
            v[k] = 0.0f;
        const uint32_t c = cell < n ? child[8 * (size_t)cell + q] : FULL_MASK;
        if (c != FULL_MASK) {
            float g[NQ];
            load_pre<B, S, ODD_F>(fine, c, g);
            const Transfer tr = to_transfer(forward_moments(g), om_f, dt_f);
            const float rho = 1.0f + tr.drho;
            v[0] = tr.drho;
            v[1] = rho * tr.ux;
            v[2] = rho * tr.uy;
            v[3] = rho * tr.uz;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[4 + k] = tr.d[k];
            v[10] = 1.0f;
        }
#pragma unroll
        for (int m = 1; m < 8; m <<= 1)
#pragma unroll
            for (int k = 0; k < 11; ++k)
                v[k] += __shfl_xor(v[k], m, 8);
        if (q == 0)
#pragma unroll
            for (int k = 0; k < 11; ++k)
                rec[k][local] = v[k];
    }
    __syncthreads();
    const int cell = base + tid;
    if (tid < CELLS && cell < n) {
        // a band cell with no fluid child lies inside the wall: the fluid at
        // rest (all transfer quantities zero)
        Transfer tr;
        tr.drho = tr.ux = tr.uy = tr.uz = 0.0f;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            tr.d[k] = 0.0f;
        if (rec[10][tid] != 0.0f) {
            const float ic = 1.0f / rec[10][tid];
            tr.drho = rec[0][tid] * ic;
            const float irho = ic / (1.0f + tr.drho);
            tr.ux = rec[1][tid] * irho;
            tr.uy = rec[2][tid] * irho;
            tr.uz = rec[3][tid] * irho;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                tr.d[k] = rec[4 + k][tid] * ic;
        }
        float g[NQ];
        back_transform(from_transfer(tr, om_c, dt_c), g);
        store_pre<B, S, ODD_C>(coarse, band[cell], g);
    }
    __syncthreads();  // rec is refilled by the next item
}

}  // namespace lbm
