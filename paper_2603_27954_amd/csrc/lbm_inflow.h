// Synthetic turbulent inflow (random Fourier modes, von Karman spectrum).
// Internal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace lbm {

// Mode set of the inflow field u'(x, t) = 2 sum_n a_n sigma_n cos(k_n . (x -
// U t e_x) + psi_n), structure of arrays.
struct InflowModes {
    std::vector<double> kx, ky, kz, sx, sy, sz, psi, amp;
    double k_e = 0.0, A = 0.0;
};

void build_inflow_modes(uint64_t seed, int n_modes, double intensity, double length, double u_in, double dx,
                        InflowModes &m);

// Fills the inlet fluctuation planes (3 floats per cell, y fastest) of the
// coarsest level for the level-0 step pair (2m, 2m + 1), m = *tick: prev at
// time 2m dt0, cur at (2m + 1) dt0 (finest time units).  modes: 8 n doubles
// (kx, ky, kz, sx, sy, sz, psi, amp blocks).
hipError_t launch_inflow(const double *modes, int n_modes, const unsigned long long *tick, double u_in, double dx0,
                         double dt0, int ny, int nz, float *prev, float *cur, hipStream_t s);
// *tick += 1 (one thread)
hipError_t launch_tick(unsigned long long *tick, hipStream_t s);

}  // namespace lbm
