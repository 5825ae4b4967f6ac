"""FP64 reference of the synthetic turbulent inflow.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark; the product library never loads it and the
two share no code.

The paper (Sec. 4.2) characterises inflow turbulence by its intensity
I_u = u'_rms / U_inf (about 8 % for near-neutral urban boundary layers) and
states no synthesis method.  The reading implemented here is a random-Fourier-
mode field (Kraichnan 1970; in the inflow form of Smirnov, Shi and Celik 2001
and Davidson 2007), frozen and advected with the mean flow:

    u'(x, t) = 2 sum_n a_n sigma_n cos(k_n . (x - U t e_x) + psi_n)

- N wavenumber shells with log-spaced edges from k_min = 0.1 / L_t to the
  Nyquist wavenumber pi / dx of the inlet grid.  Shell n has geometric centre
  k_n and width dk_n.
- Isotropic random directions d_n.  sigma_n is a unit vector perpendicular to
  d_n, so the field is divergence-free.  The phases psi_n are uniform in
  [0, 2 pi).
- Amplitudes a_n = sqrt(E(k_n) dk_n) with the von Karman shape
  E(k) = A s^4 / (1 + s^2)^(17/6), s = k / k_e.  A and k_e are solved
  numerically on the discrete shells, so that the shells carry
  (3/2) u'_rms^2 of kinetic energy and have the longitudinal integral length
  (pi / (2 u'_rms^2)) sum E / k dk = L_t.  A finite set of random directions
  splits the energy unevenly between the components, so the amplitudes are
  then scaled by one common factor that makes the realised streamwise rms,
  sqrt(sum 2 a_n^2 sigma_nx^2), equal I_u U_inf exactly (the paper's I_u is
  the streamwise intensity).  A common factor leaves the integral length
  unchanged.
- Draws come from SplitMix64 (Steele, Lea and Flood 2014) seeded with the seed,
  four per mode in mode order: cos(theta) = 2 xi1 - 1, phi = 2 pi xi2,
  alpha = 2 pi xi3, psi = 2 pi xi4.  Take d = (sin theta cos phi,
  sin theta sin phi, cos theta) and helper axis a = e_z when |d_z| < 0.9, else
  e_x.  Then e1 = (a x d) / |a x d|, e2 = d x e1 and
  sigma = cos(alpha) e1 + sin(alpha) e2.

The shells start below the energy peak rather than at the lateral period of
the box.  A -5/3 spectrum cut at k_min has an integral length of at most
about 0.94 / k_min, so a box 2H wide could not carry L_t = H / 2.  The field
is therefore not periodic across the lateral seam.

The inlet ghost plane of a level with cell size dx (finest units) sits at
x = -dx / 2 with cell centres y = (j + 1/2) dx, z = (k + 1/2) dx.  Time t is
in finest time units.
"""
import ctypes as C
import math
from dataclasses import dataclass

import numpy as np

from . import lib as _lib


@dataclass
class Modes:
    kvec: np.ndarray   # (N, 3) wavevectors, finest inverse length
    sigma: np.ndarray  # (N, 3) unit amplitude directions, sigma . kvec = 0
    psi: np.ndarray    # (N,) phases
    amp: np.ndarray    # (N,) amplitudes a_n
    k_e: float         # von Karman peak parameter
    A: float           # spectrum amplitude
    k: np.ndarray      # (N,) shell centres
    dk: np.ndarray     # (N,) shell widths


def von_karman_shape(s):
    return s ** 4 / (1.0 + s * s) ** (17.0 / 6.0)


def shells(n_modes, k_min, k_max):
    edges = k_min * (k_max / k_min) ** (np.arange(n_modes + 1) / n_modes)
    return np.sqrt(edges[:-1] * edges[1:]), np.diff(edges)


def calibrate(k, dk, urms, length):
    """(A, k_e) such that sum E dk = 1.5 urms^2 and the longitudinal integral
    length of the discrete spectrum equals `length` (bisection in log k_e)."""
    u2 = urms * urms

    def integral_length(ke):
        E = von_karman_shape(k / ke)
        A = 1.5 * u2 / np.sum(E * dk)
        return math.pi / (2.0 * u2) * A * np.sum(E / k * dk)

    lo, hi = math.log(k[0] * 1e-3), math.log(k[-1] * 1e3)  # integral length decreases with k_e
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if integral_length(math.exp(mid)) > length:
            lo = mid
        else:
            hi = mid
    ke = math.exp(0.5 * (lo + hi))
    A = 1.5 * u2 / np.sum(von_karman_shape(k / ke) * dk)
    return A, ke


def _uniform(state):
    return _lib().or_splitmix_uniform(C.byref(state))


def build_modes(seed, n_modes, intensity, length, u_in, dx):
    """Modes of the inflow field for an inlet grid of spacing dx (finest units)."""
    k, dk = shells(n_modes, 0.1 / length, math.pi / dx)
    A, ke = calibrate(k, dk, intensity * u_in, length)
    amp = np.sqrt(A * von_karman_shape(k / ke) * dk)
    state = C.c_uint64(seed)
    kvec = np.empty((n_modes, 3))
    sigma = np.empty((n_modes, 3))
    psi = np.empty(n_modes)
    for n in range(n_modes):
        ct = 2.0 * _uniform(state) - 1.0
        phi = 2.0 * math.pi * _uniform(state)
        alpha = 2.0 * math.pi * _uniform(state)
        psi[n] = 2.0 * math.pi * _uniform(state)
        st = math.sqrt(max(0.0, 1.0 - ct * ct))
        d = np.array([st * math.cos(phi), st * math.sin(phi), ct])
        a = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
        e1 = np.cross(a, d)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(d, e1)
        sigma[n] = math.cos(alpha) * e1 + math.sin(alpha) * e2
        kvec[n] = k[n] * d
    scale = intensity * u_in / math.sqrt(np.sum(2.0 * amp * amp * sigma[:, 0] ** 2))
    return Modes(kvec, sigma, psi, amp * scale, ke, A, k, dk)


def velocity(m: Modes, x, y, z, t, u_in):
    """u' at points (arrays broadcast together), shape (..., 3)."""
    x = np.asarray(x, dtype=np.float64) - u_in * t
    ph = (np.multiply.outer(x, m.kvec[:, 0]) + np.multiply.outer(np.asarray(y, np.float64), m.kvec[:, 1])
          + np.multiply.outer(np.asarray(z, np.float64), m.kvec[:, 2]) + m.psi)
    c = 2.0 * m.amp * np.cos(ph)
    return np.stack([c @ m.sigma[:, 0], c @ m.sigma[:, 1], c @ m.sigma[:, 2]], axis=-1)


def inlet_plane(m: Modes, ny, nz, dx, t, u_in):
    """u' of the inlet ghost plane of a level with ny x nz cells of size dx:
    array (nz, ny, 3), i.e. 3 values per cell in (y fastest, then z) order."""
    zz, yy = np.meshgrid((np.arange(nz) + 0.5) * dx, (np.arange(ny) + 0.5) * dx, indexing="ij")
    return velocity(m, np.full_like(yy, -0.5 * dx), yy, zz, t, u_in)
