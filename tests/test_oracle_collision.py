"""Pins of the FP64 oracle's single-cell collision against what the mathematics
fixes: the definition of central moments, the definition of cumulants (brute
force through the cumulant generating function), conservation, invariance of
the equilibrium and the closed form of the second-order relaxation.
Paper Sec. 2.2 (D3Q27 cumulant collision)."""
import math

import numpy as np
import pytest

import oracle as O


def _rand_state(rng, rho=1.0, scale=0.05):
    u = rng.uniform(-0.08, 0.08, 3)
    f = O.equilibrium(rho * rng.uniform(0.97, 1.03), u)
    return f * (1.0 + scale * rng.standard_normal(27))


def test_weights_and_isotropy():
    w = O.weights()
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    assert np.isclose(w[13], 8 / 27) and np.isclose(w[12], 2 / 27)
    assert np.isclose(w[1], 1 / 54) and np.isclose(w[0], 1 / 216)
    c = O.CVEC.astype(float)
    # second moment c_s^2 = 1/3, fourth-order isotropy of D3Q27
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(m2, np.eye(3) / 3, atol=1e-15)
    assert np.isclose(np.sum(w * c[:, 0] ** 2 * c[:, 1] ** 2), 1 / 9)
    assert np.isclose(np.sum(w * c[:, 0] ** 4), 1 / 3)


def test_equilibrium_moments():
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho, u = rng.uniform(0.9, 1.1), rng.uniform(-0.1, 0.1, 3)
        f = O.equilibrium(rho, u)
        assert np.isclose(f.sum(), rho, rtol=1e-14)
        assert np.allclose(f @ O.CVEC, rho * u, atol=1e-15)
        k = O.central_moments_direct(f, u)
        # factorised central moments: rho/3 on second-order diagonal, rho/9, rho/27
        assert np.isclose(k[2], rho / 3) and np.isclose(k[6], rho / 3) and np.isclose(k[18], rho / 3)
        assert np.isclose(k[2 + 6], rho / 9) and np.isclose(k[26], rho / 27)
        assert abs(k[1 + 3]) < 1e-15


def test_chimera_matches_definition_and_round_trips():
    """P3: the factorised transform equals the definition; inverse o forward = id."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        f = _rand_state(rng)
        u = rng.uniform(-0.1, 0.1, 3)
        k = O.chimera_forward(f, u)
        assert np.allclose(k, O.central_moments_direct(f, u), atol=1e-15, rtol=1e-13)
        assert np.allclose(O.chimera_inverse(k, u), f, atol=1e-15, rtol=1e-13)


def _series_mul(a, b):
    """Product of two power series in (tx, ty, tz) truncated to degree <= 2 per variable."""
    out = np.zeros((3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                if a[i, j, k] == 0.0:
                    continue
                out[i:, j:, k:] += a[i, j, k] * b[: 3 - i, : 3 - j, : 3 - k]
    return out


def _cumulants_brute(f):
    """rho * cumulants of f/rho from ln of its moment generating function about the mean."""
    rho = f.sum()
    u = (f @ O.CVEC) / rho
    p = f / rho
    M = np.zeros((3, 3, 3))  # M[a,b,g] = E[(c-u)^(a,b,g)] / (a! b! g!)
    for a in range(3):
        for b in range(3):
            for g in range(3):
                mom = np.sum(p * (O.CX - u[0]) ** a * (O.CY - u[1]) ** b * (O.CZ - u[2]) ** g)
                M[a, b, g] = mom / (math.factorial(a) * math.factorial(b) * math.factorial(g))
    X = M.copy()
    X[0, 0, 0] = 0.0
    logM = np.zeros((3, 3, 3))
    P = np.zeros((3, 3, 3))
    P[0, 0, 0] = 1.0
    for n in range(1, 8):
        P = _series_mul(P, X)
        logM += ((-1) ** (n + 1)) / n * P
    c = np.zeros(27)
    for a in range(3):
        for b in range(3):
            for g in range(3):
                c[a + 3 * b + 9 * g] = rho * logM[a, b, g] * math.factorial(a) * math.factorial(b) * math.factorial(g)
    c[0] = rho
    return c, u


def test_cumulants_match_generating_function():
    """Every order-4, 5 and 6 cumulant relation checked against ln(MGF)."""
    rng = np.random.default_rng(11)
    for _ in range(10):
        f = _rand_state(rng, scale=0.2)
        cb, u = _cumulants_brute(f)
        k = O.chimera_forward(f, u)
        c = O.cumulants_from_central(k)
        assert np.allclose(c[1:], cb[1:], atol=1e-14, rtol=1e-10)
        # and the inverse relations give the central moments back
        assert np.allclose(O.central_from_cumulants(c), k, atol=1e-15, rtol=1e-12)


@pytest.mark.parametrize("omega1", [0.7, 1.0, 1.5, 1.9, 1.999])
@pytest.mark.parametrize("galilean", [True, False])
def test_conservation(omega1, galilean):
    """P1: mass and momentum identical before and after the collision."""
    rng = np.random.default_rng(int(omega1 * 1000) + galilean)
    for _ in range(10):
        f = _rand_state(rng)
        g = O.collide(f, omega1, galilean=galilean)
        assert abs(g.sum() - f.sum()) < 1e-14
        assert np.allclose(g @ O.CVEC, f @ O.CVEC, atol=1e-15)


@pytest.mark.parametrize("rates", [(1.8, 1.0, 1.0), (1.2, 0.7, 1.3), (1.99, 1.5, 0.6)])
def test_equilibrium_is_fixed_point(rates):
    """P2: f_eq(rho, u) is unchanged by the collision for any rates."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        f = O.equilibrium(rng.uniform(0.9, 1.1), rng.uniform(-0.1, 0.1, 3))
        for gal in (True, False):
            g = O.collide(f, rates[0], omega2=rates[1], omega_high=rates[2], galilean=gal)
            assert np.allclose(g, f, atol=2e-16 * 8, rtol=1e-13)


def test_second_order_relaxation_closed_form():
    """At u = 0 the Galilean terms vanish: off-diagonal cumulants scale by (1-omega1),
    the deviatoric diagonal by (1-omega1), the trace relaxes to rho at omega2, and
    with omega_high = 1 every higher cumulant of the result is zero."""
    rng = np.random.default_rng(13)
    w1, w2 = 1.6, 0.8
    f = _rand_state(rng)
    rho = f.sum()
    mom = f @ O.CVEC
    # shift to zero velocity by mirroring: build a state with zero momentum
    f = 0.5 * (f + f[O.OPP])
    assert np.allclose(f @ O.CVEC, 0.0, atol=1e-16)
    rho = f.sum()
    u0 = np.zeros(3)
    c = O.cumulants_from_central(O.chimera_forward(f, u0))
    g = O.collide(f, w1, omega2=w2)
    cs = O.cumulants_from_central(O.chimera_forward(g, u0))
    for idx in (4, 10, 12):  # C110, C101, C011
        assert np.isclose(cs[idx], (1 - w1) * c[idx], atol=1e-16)
    tr, trs = c[2] + c[6] + c[18], cs[2] + cs[6] + cs[18]
    assert np.isclose(trs - rho, (1 - w2) * (tr - rho), atol=1e-15)
    assert np.isclose(cs[2] - cs[6], (1 - w1) * (c[2] - c[6]), atol=1e-16)
    for a in range(3):
        for b in range(3):
            for gg in range(3):
                if a + b + gg >= 3:
                    assert abs(cs[a + 3 * b + 9 * gg]) < 1e-15
    del mom


def test_body_force_adds_its_momentum():
    """With a body force the collision adds exactly F to the momentum and keeps
    the mass (velocity shifted by F/(2 rho), first-order central moments flipped)."""
    rng = np.random.default_rng(17)
    f = _rand_state(rng)
    F = np.array([1e-3, -2e-3, 5e-4])
    g = O.collide(f, 1.5, force=F)
    # correct forcing adds exactly F to the momentum
    assert np.allclose(g @ O.CVEC - f @ O.CVEC, F, atol=1e-15)
    assert abs(g.sum() - f.sum()) < 1e-14
