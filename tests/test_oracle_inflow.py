"""Pins of the inflow-turbulence oracle (paper Sec. 4.2 defines I_u as the
streamwise rms over the mean speed; the random-Fourier-mode synthesis with a
von Karman spectrum is the reading implemented): the calibration against the
closed form of the von Karman integrals, the sampled intensity, the integral
length measured from the realised correlation, divergence-free fields and the
frozen advection."""
import math

import numpy as np
import pytest
from scipy.special import beta

from oracle import turb_oracle as T

U = 0.05


def test_calibration_reaches_the_closed_form_without_cutoffs():
    """Over [0, inf) the von Karman integrals are Beta functions:
    int s^4/(1+s^2)^(17/6) ds = B(5/2, 1/3)/2 and int s^3/(1+s^2)^(17/6) ds =
    B(2, 5/6)/2, so k_e L = (3 pi / 4) B(2, 5/6) / B(5/2, 1/3) (= 0.747).  The
    discrete calibration over a very wide shell range must reproduce it."""
    L = 10.0
    k, dk = T.shells(20000, 1e-5 / L, 1e5 / L)
    A, ke = T.calibrate(k, dk, 1.0, L)
    closed = 0.75 * math.pi * beta(2.0, 5.0 / 6.0) / beta(2.5, 1.0 / 3.0)
    assert abs(ke * L - closed) / closed < 2e-3
    # and the amplitude: (3/2) u^2 = A k_e B(5/2, 1/3) / 2
    assert abs(A * ke * beta(2.5, 1.0 / 3.0) / 2 - 1.5) / 1.5 < 2e-3


@pytest.mark.parametrize("seed", [1, 40, 977])
def test_sampled_streamwise_intensity(seed):
    """I_u from sampling the field on the inlet plane over many times (not
    from the amplitude formula)."""
    dx, ny = 4.0, 64
    m = T.build_modes(seed, 200, 0.08, 64.0, U, dx)
    planes = np.stack([T.inlet_plane(m, ny, ny, dx, t, U) for t in np.arange(0.0, 40000.0, 400.0)])
    iu = planes[..., 0].std() / U
    assert abs(iu - 0.08) < 0.005
    assert abs(planes[..., 0].mean()) < 0.2 * 0.08 * U


def test_components_are_isotropic_on_average():
    iv = []
    for seed in range(1, 33):
        m = T.build_modes(seed, 200, 0.08, 64.0, U, 4.0)
        e = 2.0 * m.amp ** 2
        iv.append([math.sqrt(np.sum(e * m.sigma[:, c] ** 2)) / U for c in range(3)])
    iv = np.array(iv)
    assert np.allclose(iv[:, 0], 0.08, rtol=1e-12)
    assert abs(iv[:, 1].mean() - 0.08) < 0.004 and abs(iv[:, 2].mean() - 0.08) < 0.004


def test_integral_length_from_the_realised_correlation():
    """Longitudinal correlation of the realised fields, R(r) = <u_x(x) u_x(x +
    r e_x)> / <u_x^2>, averaged over seeds; its integral is the longitudinal
    integral length, which the calibration sets to L_t (isotropic relation
    L = pi / (2 u^2) int E / k dk)."""
    L = 32.0
    r = np.linspace(0.0, 12.0 * L, 4001)
    R = np.zeros_like(r)
    for seed in range(1, 65):
        m = T.build_modes(seed, 400, 0.08, L, U, 0.5)
        w = 2.0 * m.amp ** 2 * m.sigma[:, 0] ** 2
        R += np.cos(np.multiply.outer(r, m.kvec[:, 0])) @ w / w.sum()
    R /= 64
    assert R[0] == pytest.approx(1.0)
    L_est = np.trapezoid(R, r)
    assert 0.8 * L < L_est < 1.2 * L


def test_field_is_divergence_free():
    m = T.build_modes(7, 200, 0.08, 16.0, U, 1.0)
    assert np.abs(np.sum(m.sigma * m.kvec, axis=1)).max() < 1e-15
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 100, (50, 3))
    h = 1e-3
    div = np.zeros(50)
    grad = np.zeros(50)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        up = T.velocity(m, *(p + e).T, 0.0, U)
        dn = T.velocity(m, *(p - e).T, 0.0, U)
        div += (up[:, a] - dn[:, a]) / (2 * h)
        grad += np.abs(up - dn).sum(1) / (2 * h)
    assert np.abs(div).max() < 1e-6 * grad.max()


def test_frozen_advection():
    m = T.build_modes(5, 64, 0.08, 16.0, U, 1.0)
    a = T.velocity(m, 3.0, 4.0, 5.0, 200.0, U)
    b = T.velocity(m, 3.0 - U * 200.0, 4.0, 5.0, 0.0, U)
    assert np.allclose(a, b, atol=1e-15)


def test_same_seed_same_modes_and_seeds_differ():
    a = T.build_modes(11, 50, 0.08, 16.0, U, 1.0)
    b = T.build_modes(11, 50, 0.08, 16.0, U, 1.0)
    c = T.build_modes(12, 50, 0.08, 16.0, U, 1.0)
    assert np.array_equal(a.kvec, b.kvec) and np.array_equal(a.psi, b.psi)
    assert not np.array_equal(a.kvec, c.kvec)
