"""Pins of the oracle's multi-level (octree block) stepping (paper Sec. 2.2):
uniform flow stays uniform through every interface, a two-level grid without
refinement is the uniform coarse run bit for bit, the moment-space transfer
round-trips, the block maps obey nesting and the 26-neighbour closure, and a
partially refined run agrees with the uniform-finest run within the
discretisation tolerance."""
import numpy as np
import pytest

import oracle as O

NX, NY, NZ, B = 96, 96, 96, 8
U = 0.05


def _tree(com=(40.0, 48.0, 48.0)):
    return O.build_tree(O.cfg1_tree_params(), 0.0, list(com))


def _nu(b, re=100.0):
    return U * O.tree_height(b) / re


def test_transfer_round_trip():
    """Rebuilding a cell from its (rho, u, D) at the same level and step gives
    back rho, u and the second-order central moments; at another level the
    strain rate D is preserved."""
    rng = np.random.default_rng(4)
    for _ in range(10):
        u = rng.uniform(-0.05, 0.05, 3)
        f = O.equilibrium(rng.uniform(0.98, 1.02), u) * (1 + 0.01 * rng.standard_normal(27))
        w, dt = rng.uniform(1.2, 1.9), 2.0
        t = O.cell_transfer(f, w, dt)
        g = O.cell_rebuild(t, w, dt)
        assert np.isclose(g.sum(), f.sum(), rtol=1e-14)
        assert np.allclose(g @ O.CVEC, f @ O.CVEC, atol=1e-15)
        k_f = O.chimera_forward(f, t[1:4])
        k_g = O.chimera_forward(g, t[1:4])
        for idx in (2, 6, 18, 4, 10, 12):
            assert np.isclose(k_f[idx], k_g[idx], atol=1e-15)
        g2 = O.cell_rebuild(t, 1.5, 1.0)
        assert np.allclose(O.cell_transfer(g2, 1.5, 1.0), t, atol=1e-15)
    feq = O.equilibrium(1.01, [0.03, -0.01, 0.02])
    assert np.allclose(O.cell_transfer(feq, 1.7, 4.0)[4:], 0.0, atol=1e-16)


def test_block_maps_nesting_and_closure():
    b = _tree((96.0, 64.0, 64.0))
    sim = O.AmrSim(3, B, 256, 128, 128, U, _nu(b), b, band=[0, 2, 0], wake=[0, 0, 0])
    for l in range(3):
        s = sim.shape(l)
        m = sim.block_map(l).reshape(s[5], s[4], s[3])
        if l == 0:
            assert np.all((m == 1) | (m == 2))
        if l < 2:
            # every refined block has its 26 neighbours at its level
            for z, y, x in zip(*np.nonzero(m == 2)):
                nb = m[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2]
                assert nb.shape == (3, 3, 3) and np.all((nb == 1) | (nb == 2))
        if l >= 1:
            p = sim.block_map(l - 1).reshape(sim.shape(l - 1)[5], sim.shape(l - 1)[4], sim.shape(l - 1)[3])
            exists = (m == 1) | (m == 2)
            assert np.array_equal(exists, np.repeat(np.repeat(np.repeat(p == 2, 2, 0), 2, 1), 2, 2))
    # the finest level holds the whole tree
    s = sim.shape(2)
    m2 = sim.block_map(2).reshape(s[5], s[4], s[3])
    solid = O.voxelize(b, 256, 128, 128).reshape(128, 128, 256)
    zz, yy, xx = np.nonzero(solid)
    assert np.all((m2[zz // B, yy // B, xx // B] == 1))


def test_refinement_next_to_the_box_faces_is_rejected():
    b = _tree((40.0, 20.0, 32.0))
    with pytest.raises(ValueError):
        O.AmrSim(3, B, 256, 128, 128, U, _nu(b), b, band=[0, 24, 6], wake=[0, 40, 0])


def test_uniform_flow_stays_uniform():
    """Equilibrium at u_in everywhere is a fixed point of every level, of the
    prolongation and of the restriction (no body)."""
    b = _tree()
    sim = O.AmrSim(2, B, NX, NY, NZ, U, _nu(b), b, band=[0, 8], wake=[0, 0])
    sim.step(6)
    feq = O.equilibrium(1.0, [U, 0, 0])
    for l in range(2):
        f = sim.get_f(l)
        cls = sim.classes(l)
        act = (cls == O.CLS_ACTIVE)
        assert act.sum() > 0
        assert np.abs(f[:, act] - feq[:, None]).max() < 1e-14


def test_unrefined_two_level_grid_is_the_uniform_coarse_run():
    nu_f = 0.02
    sim = O.AmrSim(2, B, NX, NY, NZ, U, nu_f, np.zeros((0, 10)), band=[0, 0], wake=[0, 0])
    assert np.all(sim.block_map(1) == 0)
    rng = np.random.default_rng(9)
    N0 = (NX // 2) * (NY // 2) * (NZ // 2)
    f0 = np.empty((27, N0))
    for c in range(N0):
        f0[:, c] = O.equilibrium(1 + 0.01 * rng.standard_normal(), U + 0.01 * rng.standard_normal(3))
    sim.set_f(0, f0)
    ref = O.UniformSim(NX // 2, NY // 2, NZ // 2, O.omega_from_nu(nu_f / 2), u_in=U)
    ref.f[:] = f0
    sim.step(5)
    ref.step(5)
    assert np.array_equal(sim.get_f(0), ref.f)


@pytest.mark.slow
def test_refined_run_agrees_with_uniform_finest():
    """P9: order-1 tree refined to the finest level within 8 cells of its
    surface: C_D and the velocity near the tree within discretisation
    tolerance of the uniform-finest run (80 finest steps of the impulsive start)."""
    b = _tree()
    nu = _nu(b)
    solid = O.voxelize(b, NX, NY, NZ)
    lk = O.links(b, solid, NX, NY, NZ)
    amr = O.AmrSim(2, B, NX, NY, NZ, U, nu, b, band=[0, 8], wake=[0, 0], solid=solid, link=lk, n_branch=len(b))
    uni = O.UniformSim(NX, NY, NZ, O.omega_from_nu(nu), u_in=U, solid=solid, link=lk, n_branch=len(b))
    steps = 80
    amr.step(steps // 2)
    rec = []
    uni.step(steps, record=rec)
    ax = O.area_x(solid, NX, NY, NZ)
    cd = lambda F: F[0] / (0.5 * U * U * ax)
    fa = amr.force_log()
    assert len(fa) == steps
    cd_amr = np.mean([cd(F) for F in fa[-10:]])
    cd_uni = np.mean([cd(F) for F in rec[-10:]])
    assert abs(cd_amr - cd_uni) / abs(cd_uni) < 0.02
    _, ua = amr.fields(1)
    _, uu = uni.fields()
    cls = amr.classes(1)
    near = (cls == O.CLS_ACTIVE) & (solid == 0)
    assert np.abs(ua[near] - uu[near]).max() / U < 0.02


def _positions(shape, cells, h):
    """Cell centres (finest units) of level cells given as box indices."""
    nx, ny = shape[0], shape[1]
    ijk = np.stack([cells % nx, (cells // nx) % ny, cells // (nx * ny)], axis=1)
    return (ijk + 0.5) * h


def _linear_field(pos, rho_slope=True, u_slope=True):
    """(rho, u, D) affine in the finest-unit position; D in finest time units."""
    x, y, z = (pos / 96.0).T
    v = np.empty((len(pos), 10))
    v[:, 0] = 1.0 + (0.01 * x - 0.007 * y + 0.004 * z if rho_slope else 0.0)
    s = 1.0 if u_slope else 0.0
    v[:, 1] = 0.05 + s * (0.005 * x + 0.01 * y - 0.02 * z)
    v[:, 2] = -0.01 + s * (0.01 * x + 0.003 * z)
    v[:, 3] = 0.02 + s * (-0.01 * x + 0.01 * y)
    for k in range(6):
        v[:, 4 + k] = 1e-4 * ((k + 1) * x - (k - 2) * y + 0.5 * z - 0.3 * k)
    return v


def test_prolongation_reproduces_a_linear_field():
    """A fine ghost's parent P and the neighbours P + s (s = +1 for an odd fine
    index, -1 for an even one) carry weights 3/4 and 1/4 per axis, which puts
    the interpolation point at the ghost's own centre: (rho, u, D) affine in
    space come out exact at every ghost of the fine level."""
    b = _tree()
    nu = _nu(b)
    om = [O.omega_from_nu(nu / 2), O.omega_from_nu(nu)]
    sim = O.AmrSim(2, B, NX, NY, NZ, U, nu, b, band=[0, 8], wake=[0, 0])
    s0, s1 = sim.shape(0), sim.shape(1)
    n0 = s0[0] * s0[1] * s0[2]
    V = _linear_field(_positions(s0, np.arange(n0), 2.0))
    f0 = np.empty((27, n0))
    for c in range(n0):
        f0[:, c] = O.cell_rebuild(V[c], om[0], 2.0)
    sim.set_f(0, f0)
    sim.prolong_only(0)
    f1 = sim.get_f(1)
    gi = np.flatnonzero(sim.classes(1) == O.CLS_GHOST)
    assert len(gi) > 1000
    want = _linear_field(_positions(s1, gi, 1.0))
    got = np.array([O.cell_transfer(f1[:, c], om[1], 1.0) for c in gi])
    err = np.abs(got - want).max(axis=0)
    assert np.all(err < 1e-14)
    # the even/odd neighbour rule matters: the same field read at the parent
    # centres alone misses by the field's slope over a quarter coarse cell
    par = (_positions(s1, gi, 1.0) // 2.0 + 0.5) * 2.0
    assert np.abs(_linear_field(par)[:, 1] - want[:, 1]).max() > 1e-5


@pytest.mark.parametrize("rho_slope,u_slope", [(False, True), (True, False)])
def test_restriction_reproduces_a_linear_field(rho_slope, u_slope):
    """A coarse band cell gets the mean density, the mass-weighted velocity and
    the mean strain rate of its eight children, whose centres surround its own
    symmetrically: affine density (at constant velocity) or affine velocity (at
    constant density) and affine D come out exact at the band-cell centres."""
    b = _tree()
    nu = _nu(b)
    om = [O.omega_from_nu(nu / 2), O.omega_from_nu(nu)]
    sim = O.AmrSim(2, B, NX, NY, NZ, U, nu, b, band=[0, 8], wake=[0, 0])
    s0, s1 = sim.shape(0), sim.shape(1)
    bc = np.flatnonzero(sim.classes(0) == O.CLS_BAND)
    assert len(bc) > 500
    n1 = s1[0] * s1[1] * s1[2]
    f1 = np.tile(O.equilibrium(1.0, [U, 0.0, 0.0])[:, None], (1, n1))
    x0, y0, z0 = bc % s0[0], (bc // s0[0]) % s0[1], bc // (s0[0] * s0[1])
    for q in range(8):
        ch = (2 * x0 + (q & 1)) + s1[0] * ((2 * y0 + ((q >> 1) & 1)) + s1[1] * (2 * z0 + (q >> 2)))
        V = _linear_field(_positions(s1, ch, 1.0), rho_slope, u_slope)
        for k, c in enumerate(ch):
            f1[:, c] = O.cell_rebuild(V[k], om[1], 1.0)
    sim.set_f(1, f1)
    sim.restrict_only(0)
    f0 = sim.get_f(0)
    want = _linear_field(_positions(s0, bc, 2.0), rho_slope, u_slope)
    got = np.array([O.cell_transfer(f0[:, c], om[0], 2.0) for c in bc])
    err = np.abs(got - want).max(axis=0)
    assert np.all(err < 1e-14)


def test_restriction_of_a_band_cell_inside_the_wall_is_the_fluid_at_rest():
    """A band cell whose eight children are all solid lies inside the wall: it
    takes rho = 1, u = 0, D = 0 (the rest equilibrium), whatever its own and
    its children's populations held, while its neighbours keep the mean of
    their fluid children."""
    b = _tree()
    nu = _nu(b)
    om = [O.omega_from_nu(nu / 2), O.omega_from_nu(nu)]
    base = O.AmrSim(2, B, NX, NY, NZ, U, nu, b, band=[0, 8], wake=[0, 0])
    s0, s1 = base.shape(0), base.shape(1)
    bc = np.flatnonzero(base.classes(0) == O.CLS_BAND)
    inside = bc[::97][:6]
    solid = np.zeros(s1[0] * s1[1] * s1[2], np.uint8)
    x0, y0, z0 = inside % s0[0], (inside // s0[0]) % s0[1], inside // (s0[0] * s0[1])
    for q in range(8):
        solid[(2 * x0 + (q & 1)) + s1[0] * ((2 * y0 + ((q >> 1) & 1)) + s1[1] * (2 * z0 + (q >> 2)))] = 1
    sim = O.AmrSim(2, B, NX, NY, NZ, U, nu, b, band=[0, 8], wake=[0, 0], solid=solid)
    n0, n1 = s0[0] * s0[1] * s0[2], s1[0] * s1[1] * s1[2]
    moving = O.cell_rebuild(np.array([1.02, 0.04, -0.01, 0.02, 1e-4, 0, 0, 0, 0, 0]), om[1], 1.0)
    sim.set_f(1, np.tile(moving[:, None], (1, n1)))
    sim.set_f(0, np.full((27, n0), np.nan))
    sim.restrict_only(0)
    f0 = sim.get_f(0)
    rest = O.equilibrium(1.0, [0.0, 0.0, 0.0])
    assert np.abs(f0[:, inside] - rest[:, None]).max() < 1e-15
    others = np.setdiff1d(bc, inside)
    got = np.array([O.cell_transfer(f0[:, c], om[0], 2.0) for c in others[:50]])
    assert np.abs(got[:, :4] - np.array([1.02, 0.04, -0.01, 0.02])).max() < 1e-14


def _vertical_branch():
    """One branch on the axis x = 40, y = 32 from z = 20 to z = 44, diameter 4
    (finest cells): its box spans x 38..42, y 30..34, z 18..46."""
    return np.array([[40.0, 32.0, 20.0, 40.0, 32.0, 44.0, 4.0, 0.0, -1.0, 0.0]])


@pytest.mark.parametrize("wake,last_bx", [(0, 2), (64, 6), (70, 6), (71, 7)])
def test_wake_box_refines_exactly_the_blocks_it_overlaps(wake, last_bx):
    """Reading R17 worked by hand on two levels (no closure pass): level-0
    blocks are 16 finest cells wide.  With no band the branch refines block
    column x = 2 (cells 32..48) in rows y = 1, 2 and z = 1, 2.  The wake box
    runs from the branch box's upstream face x = 38 to 42 + wake over the same
    y and z, so it refines columns 2 .. last_bx: a block whose upstream face
    sits at or beyond the wake's end (112 for wake 70) stays coarse."""
    maps = O.amr_maps(2, 8, 256, 64, 64, _vertical_branch(), [0, 0], [0, wake])
    m0 = maps[0].reshape(4, 4, 16)
    want = np.ones_like(m0)
    want[1:3, 1:3, 2:last_bx + 1] = 2
    assert np.array_equal(m0, want)
    m1 = maps[1].reshape(8, 8, 32)
    exists = (m1 == 1) | (m1 == 2)
    assert np.array_equal(exists, np.repeat(np.repeat(np.repeat(want == 2, 2, 0), 2, 1), 2, 2))


def test_maps_only_entry_equals_the_full_state_maps():
    b = _tree((96.0, 64.0, 64.0))
    sim = O.AmrSim(3, B, 256, 128, 128, U, _nu(b), b, band=[0, 2, 0], wake=[0, 64, 0])
    maps = O.amr_maps(3, B, 256, 128, 128, b, [0, 2, 0], [0, 64, 0])
    for l in range(3):
        assert np.array_equal(maps[l], sim.block_map(l))
    # the wake refines level-0 blocks downstream of the tree
    assert (maps[0] == 2).sum() > (O.amr_maps(3, B, 256, 128, 128, b, [0, 2, 0], [0, 0, 0])[0] == 2).sum()
