// Mode set of the synthetic turbulent inflow (host side).
//
// The paper characterises inflow turbulence by its streamwise intensity
// I_u = u'_rms / U_inf (Sec. 4.2) and gives no synthesis method.  The field
// used here is a sum of random Fourier modes frozen in the mean flow
// (Kraichnan 1970; inflow form of Smirnov, Shi and Celik 2001):
//   - N shells with log-spaced edges from 0.1 / L_t to the inlet Nyquist
//     wavenumber pi / dx, at geometric centres k_n with widths dk_n; the low
//     end sits below the von Karman peak (~1.2 / L_t), so the field carries
//     integral lengths larger than a narrow box's lateral period allows;
//   - amplitudes a_n = sqrt(E(k_n) dk_n), E = A s^4 / (1 + s^2)^(17/6),
//     s = k / k_e, with A and k_e solved on the discrete shells for a kinetic
//     energy of (3/2) u'^2 and a longitudinal integral length
//     (pi / (2 u'^2)) sum E / k dk = L_t (bisection in log k_e), then one
//     common factor making the realised streamwise rms sqrt(sum 2 a^2 sx^2)
//     equal to I_u U_inf;
//   - per mode, four SplitMix64 draws in order give an isotropic direction d
//     (cos theta = 2 xi - 1, phi = 2 pi xi), the angle alpha of sigma in the
//     plane normal to d (basis e1 = a x d / |a x d|, e2 = d x e1 with helper
//     axis a = e_z when |d_z| < 0.9, else e_x) and the phase psi = 2 pi xi.
#include <cmath>

#include "lbm_inflow.h"
#include "lbm_random.h"

namespace lbm {

namespace {

double vk_shape(double s) { return s * s * s * s / std::pow(1.0 + s * s, 17.0 / 6.0); }

}  // namespace

void build_inflow_modes(uint64_t seed, int n, double intensity, double length, double u_in, double dx,
                        InflowModes &m)
{
    const double kmin = 0.1 / length, kmax = M_PI / dx;
    std::vector<double> kc(n), dk(n);
    for (int i = 0; i < n; ++i) {
        const double e0 = kmin * std::pow(kmax / kmin, (double)i / n);
        const double e1 = kmin * std::pow(kmax / kmin, (double)(i + 1) / n);
        kc[i] = std::sqrt(e0 * e1);
        dk[i] = e1 - e0;
    }
    const double u2 = (intensity * u_in) * (intensity * u_in);
    auto energy = [&](double ke) {
        double e = 0.0;
        for (int i = 0; i < n; ++i)
            e += vk_shape(kc[i] / ke) * dk[i];
        return e;
    };
    auto integral_length = [&](double ke) {
        double e = 0.0, w = 0.0;
        for (int i = 0; i < n; ++i) {
            const double E = vk_shape(kc[i] / ke);
            e += E * dk[i];
            w += E / kc[i] * dk[i];
        }
        const double A = 1.5 * u2 / e;
        return M_PI / (2.0 * u2) * A * w;
    };
    double lo = std::log(kc[0] * 1e-3), hi = std::log(kc[n - 1] * 1e3);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (integral_length(std::exp(mid)) > length)
            lo = mid;
        else
            hi = mid;
    }
    m.k_e = std::exp(0.5 * (lo + hi));
    m.A = 1.5 * u2 / energy(m.k_e);
    m.kx.resize(n), m.ky.resize(n), m.kz.resize(n);
    m.sx.resize(n), m.sy.resize(n), m.sz.resize(n);
    m.psi.resize(n), m.amp.resize(n);
    SplitMix64 rng{seed};
    double sxx = 0.0;
    for (int i = 0; i < n; ++i) {
        const double ct = 2.0 * rng.uniform() - 1.0;
        const double phi = 2.0 * M_PI * rng.uniform();
        const double alpha = 2.0 * M_PI * rng.uniform();
        m.psi[i] = 2.0 * M_PI * rng.uniform();
        const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
        const double d[3] = {st * std::cos(phi), st * std::sin(phi), ct};
        const double a[3] = {std::fabs(d[2]) < 0.9 ? 0.0 : 1.0, 0.0, std::fabs(d[2]) < 0.9 ? 1.0 : 0.0};
        double e1[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2], a[0] * d[1] - a[1] * d[0]};
        const double nrm = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (double &v : e1)
            v /= nrm;
        const double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0]};
        const double ca = std::cos(alpha), sa = std::sin(alpha);
        m.sx[i] = ca * e1[0] + sa * e2[0];
        m.sy[i] = ca * e1[1] + sa * e2[1];
        m.sz[i] = ca * e1[2] + sa * e2[2];
        m.kx[i] = kc[i] * d[0];
        m.ky[i] = kc[i] * d[1];
        m.kz[i] = kc[i] * d[2];
        m.amp[i] = std::sqrt(m.A * vk_shape(kc[i] / m.k_e) * dk[i]);
        sxx += 2.0 * m.amp[i] * m.amp[i] * m.sx[i] * m.sx[i];
    }
    const double scale = intensity * u_in / std::sqrt(sxx);
    for (double &v : m.amp)
        v *= scale;
}

}  // namespace lbm
