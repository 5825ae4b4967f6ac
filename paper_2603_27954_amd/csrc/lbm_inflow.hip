// Inlet fluctuation planes of the synthetic turbulent inflow.  One thread per
// inlet cell of the coarsest level; the mode set (8 n doubles) is staged in
// LDS in chunks and the sum is taken in FP64 (phases reach k . U t ~ 1e3 rad
// over long runs, beyond what FP32 arguments resolve).  The time comes from a
// device counter, so captured graphs replay with the right time.
#include "lbm_inflow.h"

namespace lbm {

namespace {

constexpr int CHUNK = 128;

__global__ void __launch_bounds__(256) k_inflow(const double *modes, int n, const unsigned long long *tick,
                                                double u_in, double dx0, double dt0, int ny, int nz, float *prev,
                                                float *cur)
{
    __shared__ double sm[8 * CHUNK];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c < ny * nz;
    const int j = live ? c % ny : 0, k = live ? c / ny : 0;
    const double m2 = 2.0 * (double)(*tick);
    const double t0 = m2 * dt0, t1 = (m2 + 1.0) * dt0;
    const double x = -0.5 * dx0, y = (j + 0.5) * dx0, z = (k + 0.5) * dx0;
    double u0[3] = {0.0, 0.0, 0.0}, u1[3] = {0.0, 0.0, 0.0};
    for (int base = 0; base < n; base += CHUNK) {
        const int cnt = min(CHUNK, n - base);
        __syncthreads();
        for (int i = threadIdx.x; i < 8 * cnt; i += blockDim.x) {
            const int f = i / cnt, q = i - f * cnt;
            sm[f * CHUNK + q] = modes[(size_t)f * n + base + q];
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            const double kx = sm[q], ky = sm[CHUNK + q], kz = sm[2 * CHUNK + q];
            const double ph = kx * x + ky * y + kz * z + sm[6 * CHUNK + q];
            const double a2 = 2.0 * sm[7 * CHUNK + q];
            const double c0 = a2 * cos(ph - kx * u_in * t0), c1 = a2 * cos(ph - kx * u_in * t1);
            const double sx = sm[3 * CHUNK + q], sy = sm[4 * CHUNK + q], sz = sm[5 * CHUNK + q];
            u0[0] += c0 * sx, u0[1] += c0 * sy, u0[2] += c0 * sz;
            u1[0] += c1 * sx, u1[1] += c1 * sy, u1[2] += c1 * sz;
        }
    }
    if (live) {
        for (int a = 0; a < 3; ++a) {
            prev[3 * (size_t)c + a] = (float)u0[a];
            cur[3 * (size_t)c + a] = (float)u1[a];
        }
    }
}

__global__ void k_tick(unsigned long long *tick)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *tick += 1ull;
}

}  // namespace

hipError_t launch_inflow(const double *modes, int n, const unsigned long long *tick, double u_in, double dx0,
                         double dt0, int ny, int nz, float *prev, float *cur, hipStream_t s)
{
    const int cells = ny * nz;
    hipLaunchKernelGGL(k_inflow, dim3((cells + 255) / 256), dim3(256), 0, s, modes, n, tick, u_in, dx0, dt0, ny, nz,
                       prev, cur);
    return hipGetLastError();
}

hipError_t launch_tick(unsigned long long *tick, hipStream_t s)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, tick);
    return hipGetLastError();
}

}  // namespace lbm
