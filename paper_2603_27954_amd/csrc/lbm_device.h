// Device-side lattice arithmetic for gfx950: D3Q27 constants, storage
// conversions and the cumulant collision (paper Sec. 2.2) in FP32.
//
// Populations travel as deviations g_i = f_i - w_i from the lattice weights
// (FP32, FP16 or BF16 in memory, FP32 in registers).  The collision keeps every
// intermediate small:
//   forward: raw moments of g (three summation passes over the 3x3x3 lattice),
//            from which rho, u and the non-equilibrium second-order central
//            moments N = kappa_2 - rho/3 I follow without cancellation;
//   relax:   second-order cumulants (= central moments) relaxed with omega1 on
//            the deviatoric part and omega2 on the trace, with the Galilean
//            correction terms built from the velocity-gradient estimates that
//            N gives; every cumulant of order >= 3 relaxes to zero (rate 1);
//   back:    with all higher cumulants zero the post-collision central moments
//            are the Gaussian (Wick) products of the second-order ones; the
//            central moments of the weights about u factorise, so their
//            difference Delta is small and the inverse central-moment transform
//            of Delta yields g* directly.
// Population index i = (cx+1) + 3(cy+1) + 9(cz+1); moment index a + 3b + 9c.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace lbm {

constexpr int NQ = 27;

__host__ __device__ constexpr int qcx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int qcy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int qcz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int qopp(int i) { return 26 - i; }
__host__ __device__ constexpr float w1d(int c) { return c == 0 ? 2.0f / 3.0f : 1.0f / 6.0f; }
__host__ __device__ constexpr float qw(int i) { return w1d(qcx(i)) * w1d(qcy(i)) * w1d(qcz(i)); }

// ---- storage traits --------------------------------------------------------
template <typename S> struct Store;
template <> struct Store<float> {
    static __device__ __forceinline__ float ld(float v) { return v; }
    static __device__ __forceinline__ float st(float v) { return v; }
};
template <> struct Store<__half> {
    static __device__ __forceinline__ float ld(__half v) { return __half2float(v); }
    static __device__ __forceinline__ __half st(float v) { return __float2half(v); }
};
template <> struct Store<__hip_bfloat16> {
    static __device__ __forceinline__ float ld(__hip_bfloat16 v) { return __bfloat162float(v); }
    static __device__ __forceinline__ __hip_bfloat16 st(float v) { return __float2bfloat16(v); }
};

// ---- moments ------------------------------------------------------------------
// Second-order state of a cell: density deviation, velocity and the six
// non-equilibrium central moments (xx, yy, zz, xy, xz, yz).
struct Moments {
    float drho, ux, uy, uz;
    float nxx, nyy, nzz, nxy, nxz, nyz;
};

__host__ __device__ __forceinline__ Moments forward_moments(const float (&g)[NQ])
{
    // x pass over the nine (cy, cz) lines
    float a0[9], a1[9], a2[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        const float m = g[3 * l], o = g[3 * l + 1], p = g[3 * l + 2];
        const float s = p + m;
        a0[l] = s + o;
        a1[l] = p - m;
        a2[l] = s;
    }
    // y pass per cz group r (lines 3r .. 3r+2 are cy = -1, 0, 1)
    float b00[3], b01[3], b02[3], b10[3], b11[3], b20[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float s0 = a0[3 * r + 2] + a0[3 * r];
        b00[r] = s0 + a0[3 * r + 1];
        b01[r] = a0[3 * r + 2] - a0[3 * r];
        b02[r] = s0;
        b10[r] = (a1[3 * r] + a1[3 * r + 2]) + a1[3 * r + 1];
        b11[r] = a1[3 * r + 2] - a1[3 * r];
        b20[r] = (a2[3 * r] + a2[3 * r + 2]) + a2[3 * r + 1];
    }
    // z pass
    const float m000 = (b00[0] + b00[2]) + b00[1];
    const float m001 = b00[2] - b00[0];
    const float m002 = b00[2] + b00[0];
    const float m100 = (b10[0] + b10[2]) + b10[1];
    const float m101 = b10[2] - b10[0];
    const float m010 = (b01[0] + b01[2]) + b01[1];
    const float m011 = b01[2] - b01[0];
    const float m020 = (b02[0] + b02[2]) + b02[1];
    const float m110 = (b11[0] + b11[2]) + b11[1];
    const float m200 = (b20[0] + b20[2]) + b20[1];

    Moments m;
    m.drho = m000;
    const float inv = 1.0f / (1.0f + m000);
    m.ux = m100 * inv;
    m.uy = m010 * inv;
    m.uz = m001 * inv;
    const float d3 = m000 * (1.0f / 3.0f);
    m.nxx = m200 - d3 - m100 * m.ux;
    m.nyy = m020 - d3 - m010 * m.uy;
    m.nzz = m002 - d3 - m001 * m.uz;
    m.nxy = m110 - m100 * m.uy;
    m.nxz = m101 - m100 * m.uz;
    m.nyz = m011 - m010 * m.uz;
    return m;
}

// Relaxation of the second-order cumulants (in place on the N part).
__host__ __device__ __forceinline__ void relax_second(Moments &m, float om1, float om2, bool galilean)
{
    const float rho = 1.0f + m.drho;
    const float inv = 1.0f / rho;
    const float dxy = m.nxx - m.nyy, dxz = m.nxx - m.nzz;
    const float tr = m.nxx + m.nyy + m.nzz;
    float dxy_s = (1.0f - om1) * dxy, dxz_s = (1.0f - om1) * dxz, tr_s = (1.0f - om2) * tr;
    if (galilean) {
        const float dxu = -0.5f * inv * (om1 * (dxy + dxz) + om2 * tr);
        const float dyv = dxu + 1.5f * om1 * inv * dxy;
        const float dzw = dxu + 1.5f * om1 * inv * dxz;
        const float ux2 = m.ux * m.ux, uy2 = m.uy * m.uy, uz2 = m.uz * m.uz;
        const float c1 = 3.0f * rho * (1.0f - 0.5f * om1);
        const float c2 = 3.0f * rho * (1.0f - 0.5f * om2);
        const float xu = ux2 * dxu, yv = uy2 * dyv, zw = uz2 * dzw;
        dxy_s -= c1 * (xu - yv);
        dxz_s -= c1 * (xu - zw);
        tr_s -= c2 * ((xu + yv) + zw);
    }
    const float third = 1.0f / 3.0f;
    m.nxx = (dxy_s + dxz_s + tr_s) * third;
    m.nyy = (tr_s - 2.0f * dxy_s + dxz_s) * third;
    m.nzz = (tr_s + dxy_s - 2.0f * dxz_s) * third;
    m.nxy *= (1.0f - om1);
    m.nxz *= (1.0f - om1);
    m.nyz *= (1.0f - om1);
}

// One-dimensional inverse central-moment transform at velocity a:
// (k0, k1, k2) -> (f-, f0, f+).
__host__ __device__ __forceinline__ void inv1(float &p0, float &p1, float &p2, float a)
{
    const float k0 = p0, k1 = p1, k2 = p2;
    const float d = fmaf(a, k0, k1);      // f+ - f-
    const float s = fmaf(a, k1 + d, k2);  // f+ + f-
    const float fp = 0.5f * (s + d);
    p1 = k0 - s;
    p2 = fp;
    p0 = fp - d;
}

// Populations (as deviations from the weights) of the state with density
// 1 + drho, velocity u, non-equilibrium second-order central moments N and all
// higher cumulants zero.
__host__ __device__ __forceinline__ void back_transform(const Moments &m, float (&g)[NQ])
{
    const float rho = 1.0f + m.drho;
    const float inv = 1.0f / rho, inv2 = inv * inv;
    const float third = 1.0f / 3.0f, ninth = 1.0f / 9.0f;
    const float ux = m.ux, uy = m.uy, uz = m.uz;
    const float ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
    const float X = m.nxx, Y = m.nyy, Z = m.nzz, A = m.nxy, Bq = m.nxz, Cq = m.nyz;
    const float kxx = rho * third + X, kyy = rho * third + Y, kzz = rho * third + Z;
    // weights' central moments about u: mu0 = 1, mu1 = -u, mu2 = 1/3 + u^2
    const float mx2 = third + ux2, my2 = third + uy2, mz2 = third + uz2;

    float D[NQ];
    D[0] = m.drho;
    D[1] = ux;
    D[3] = uy;
    D[9] = uz;
    D[2] = m.drho * third + X - ux2;
    D[6] = m.drho * third + Y - uy2;
    D[18] = m.drho * third + Z - uz2;
    D[4] = A - ux * uy;
    D[10] = Bq - ux * uz;
    D[12] = Cq - uy * uz;
    D[13] = ux * uy * uz;
    D[5] = mx2 * uy;   // (2,1,0)
    D[11] = mx2 * uz;  // (2,0,1)
    D[7] = my2 * ux;   // (1,2,0)
    D[15] = my2 * uz;  // (0,2,1)
    D[19] = mz2 * ux;  // (1,0,2)
    D[21] = mz2 * uy;  // (0,1,2)
    // fourth order: Wick products kappa_aa kappa_bb + 2 kappa_ab^2 etc. minus
    // the weights' products, expanded so that only small terms remain
    D[8] = m.drho * ninth + (X + Y - ux2 - uy2) * third + (X * Y + 2.0f * A * A) * inv - ux2 * uy2;
    D[20] = m.drho * ninth + (X + Z - ux2 - uz2) * third + (X * Z + 2.0f * Bq * Bq) * inv - ux2 * uz2;
    D[24] = m.drho * ninth + (Y + Z - uy2 - uz2) * third + (Y * Z + 2.0f * Cq * Cq) * inv - uy2 * uz2;
    D[14] = (Cq - uy * uz) * third + (X * Cq + 2.0f * A * Bq) * inv - ux2 * uy * uz;  // (2,1,1)
    D[16] = (Bq - ux * uz) * third + (Y * Bq + 2.0f * A * Cq) * inv - uy2 * ux * uz;  // (1,2,1)
    D[22] = (A - ux * uy) * third + (Z * A + 2.0f * Bq * Cq) * inv - uz2 * ux * uy;   // (1,1,2)
    // fifth order: zero minus the weights' products mu2 mu2 mu1
    D[17] = mx2 * my2 * uz;  // (2,2,1)
    D[23] = mx2 * mz2 * uy;  // (2,1,2)
    D[25] = my2 * mz2 * ux;  // (1,2,2)
    // sixth order: kappa_222 = (kxx kyy kzz + 2 (kxx c^2 + kyy b^2 + kzz a^2) + 8 abc) / rho^2
    {
        const float lin = (X + Y + Z) * ninth;
        const float quad = (X * Y + X * Z + Y * Z) * third * inv;
        const float cub = X * Y * Z * inv2;
        const float mix = (2.0f * (kxx * Cq * Cq + kyy * Bq * Bq + kzz * A * A) + 8.0f * A * Bq * Cq) * inv2;
        const float wu = (ux2 + uy2 + uz2) * ninth + (ux2 * uy2 + ux2 * uz2 + uy2 * uz2) * third + ux2 * uy2 * uz2;
        D[26] = m.drho * (ninth * third) + lin + quad + cub + mix - wu;
    }
    // inverse transform: x pass, y pass, z pass
#pragma unroll
    for (int r = 0; r < 9; ++r)
        inv1(D[3 * r], D[3 * r + 1], D[3 * r + 2], ux);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            inv1(D[a + 9 * c], D[a + 3 + 9 * c], D[a + 6 + 9 * c], uy);
#pragma unroll
    for (int b = 0; b < 9; ++b)
        inv1(D[b], D[b + 9], D[b + 18], uz);
#pragma unroll
    for (int i = 0; i < NQ; ++i)
        g[i] = D[i];
}

// Coarse/fine transfer quantities of a cell: density deviation, velocity and
// the strain-rate tensor in finest time units (xx, yy, zz, xy, xz, yz).  From
// the pre-collision non-equilibrium moments N the lattice strain rate is
// S = -3/(2 rho) (omega1 dev N + omega2 tr(N)/3 I) per level step dt (finest
// steps); rebuilding at another level inverts this with that level's rate
// and step.  The bulk rate omega2 is 1 on every level.
struct Transfer {
    float drho, ux, uy, uz;
    float d[6];
};

__host__ __device__ __forceinline__ Transfer to_transfer(const Moments &m, float om1, float dt)
{
    Transfer t;
    const float rho = 1.0f + m.drho;
    const float c = -1.5f / (rho * dt);
    const float t3 = (m.nxx + m.nyy + m.nzz) * (1.0f / 3.0f);
    t.drho = m.drho;
    t.ux = m.ux;
    t.uy = m.uy;
    t.uz = m.uz;
    t.d[0] = c * (om1 * (m.nxx - t3) + t3);
    t.d[1] = c * (om1 * (m.nyy - t3) + t3);
    t.d[2] = c * (om1 * (m.nzz - t3) + t3);
    t.d[3] = c * om1 * m.nxy;
    t.d[4] = c * om1 * m.nxz;
    t.d[5] = c * om1 * m.nyz;
    return t;
}

__host__ __device__ __forceinline__ Moments from_transfer(const Transfer &t, float om1, float dt)
{
    Moments m;
    const float rho = 1.0f + t.drho;
    const float c = -2.0f * rho * dt / 3.0f;
    const float s3 = (t.d[0] + t.d[1] + t.d[2]) * (1.0f / 3.0f);
    const float iw = 1.0f / om1;
    m.drho = t.drho;
    m.ux = t.ux;
    m.uy = t.uy;
    m.uz = t.uz;
    m.nxx = c * ((t.d[0] - s3) * iw + s3);
    m.nyy = c * ((t.d[1] - s3) * iw + s3);
    m.nzz = c * ((t.d[2] - s3) * iw + s3);
    m.nxy = c * t.d[3] * iw;
    m.nxz = c * t.d[4] * iw;
    m.nyz = c * t.d[5] * iw;
    return m;
}

__host__ __device__ __forceinline__ void collide(float (&g)[NQ], float om1, float om2, bool galilean)
{
    Moments m = forward_moments(g);
    relax_second(m, om1, om2, galilean);
    back_transform(m, g);
}

// Equilibrium deviation f_eq_i(1, u) - w_i of direction i (product form,
// written as w_i ((1+ex)(1+ey)(1+ez) - 1) with small per-axis factors).
__host__ __device__ __forceinline__ float feq_dev(int i, float ux, float uy, float uz)
{
    const int cx = qcx(i), cy = qcy(i), cz = qcz(i);
    const float ex = cx == 0 ? -1.5f * ux * ux : 3.0f * ux * ux + 3.0f * cx * ux;
    const float ey = cy == 0 ? -1.5f * uy * uy : 3.0f * uy * uy + 3.0f * cy * uy;
    const float ez = cz == 0 ? -1.5f * uz * uz : 3.0f * uz * uz + 3.0f * cz * uz;
    const float axy = ex + ey + ex * ey;
    return qw(i) * (axy + ez + axy * ez);
}

} // namespace lbm
