"""Pins of the oracle's friction force (wall shear stress integrated over the
body surface, paper Sec. 3 Eqs. (8)-(9)) against closed forms: in steady plane
and pipe Poiseuille flow the walls carry the whole body force on the fluid as
friction (momentum balance, no pressure drag in a periodic channel); a fluid
at rest exerts none; the tree's friction drags downstream and stays below its
total drag."""
import numpy as np
import pytest

import oracle as O
from oracle import friction_oracle as F


def _plane(nu=0.1, g=1e-6, h=16, steps=6000):
    nx, ny, nz = 2, 2, h + 2
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[0] = solid[-1] = 1
    solid = solid.ravel()
    cells, dirs = [], []
    for cell in np.nonzero(solid == 0)[0]:
        zi = cell // (nx * ny)
        for i in range(27):
            if (zi == 1 and O.CZ[i] == -1) or (zi == nz - 2 and O.CZ[i] == 1):
                cells.append(cell)
                dirs.append(i)
    link = {"cell": np.array(cells, np.int64), "dir": np.array(dirs, np.int8), "q": np.full(len(cells), 0.5),
            "branch": np.zeros(len(cells), np.int32)}
    sim = O.UniformSim(nx, ny, nz, O.omega_from_nu(nu), solid=solid, link=link, periodic_x=True,
                       force=(g, 0, 0), n_branch=1)
    sim.step(steps)
    return sim, solid, link, (nx, ny, nz)


def _pipe(R, nu=1 / 6, g=1e-6):
    n = int(2 * R) + 4
    nx, ny, nz = 2, n, n
    c = n / 2.0
    z, y, x = np.meshgrid(np.arange(nz) + .5, np.arange(ny) + .5, np.arange(nx) + .5, indexing="ij")
    r2 = ((y - c) ** 2 + (z - c) ** 2).ravel()
    solid = (r2 >= R * R).astype(np.uint8)
    cells, dirs, qs = [], [], []
    for cell in np.nonzero(solid == 0)[0]:
        xi, yi, zi = cell % nx, (cell // nx) % ny, cell // (nx * ny)
        for i in range(27):
            sy, sz = yi + O.CY[i], zi + O.CZ[i]
            if i == 13 or not solid[(xi + O.CX[i]) % nx + nx * (sy + ny * sz)]:
                continue
            oy, oz, dy, dz = yi + .5 - c, zi + .5 - c, O.CY[i], O.CZ[i]
            A, B, Cc = dy * dy + dz * dz, 2 * (oy * dy + oz * dz), oy * oy + oz * oz - R * R
            cells.append(cell)
            dirs.append(i)
            qs.append((-B + np.sqrt(B * B - 4 * A * Cc)) / (2 * A))
    link = {"cell": np.array(cells, np.int64), "dir": np.array(dirs, np.int8), "q": np.array(qs),
            "branch": np.zeros(len(cells), np.int32)}
    sim = O.UniformSim(nx, ny, nz, O.omega_from_nu(nu), solid=solid, link=link, periodic_x=True,
                       force=(g, 0, 0), n_branch=1)
    ua = g / (4 * nu) * np.maximum(R * R - r2, 0)
    f = np.stack([O.equilibrium(1.0, [v, 0, 0]) for v in ua], 1)
    f[:, solid == 1] = O.weights()[:, None]
    sim.f[:] = f
    sim.step(int(25 * R * R))

    def normal(xw, k):  # the body is the solid outside the pipe: its normal points to the axis
        v = np.array([0.0, xw[1] - c, xw[2] - c])
        return -v / np.linalg.norm(v)
    return sim, solid, link, (nx, ny, nz), normal


def test_stress_of_a_linear_shear_equilibrium_is_zero_and_of_poiseuille_is_rho_nu_dudz():
    """At equilibrium the non-equilibrium stress vanishes; in plane Poiseuille
    flow the shear stress of every cell is rho nu du/dz of the parabola."""
    s = F.cell_stress(O.equilibrium(1.02, [0.03, -0.01, 0.02])[:, None], 1.7)
    assert np.abs(s).max() < 1e-16
    nu, g, h = 0.1, 1e-6, 16
    sim, solid, link, shape = _plane(nu, g, h)
    st = F.cell_stress(sim.f[:, solid == 0], O.omega_from_nu(nu))
    zc = (np.nonzero(solid == 0)[0] // 4) + 0.5 - 1.0
    want = g * (h / 2.0 - zc)  # rho nu du/dz with u = g z (h - z) / (2 nu)
    assert np.abs(st[:, 0, 2] - want).max() < 1e-3 * g * h / 2


def test_plane_channel_friction_equals_the_body_force():
    """Halfway walls, linear stress across the channel: the extrapolation to
    the walls is exact and the friction carries g rho V_fluid."""
    nu, g, h = 0.1, 1e-6, 16
    sim, solid, link, shape = _plane(nu, g, h)
    total, _ = F.friction_force(sim.f, O.omega_from_nu(nu), solid, link, shape,
                                lambda xw, k: np.array([0.0, 0.0, 1.0 if xw[2] < shape[2] / 2 else -1.0]))
    want = g * (solid == 0).sum()
    assert abs(total[0] / want - 1.0) < 2e-3
    assert abs(total[1]) < 1e-12 and abs(total[2]) < 1e-12


def test_pipe_friction_equals_the_body_force_and_converges():
    """Curved wall (interpolated bounce-back): the weighted face sum of the
    wall shear stress tends to the momentum balance g rho V_fluid, within 2 %
    at R = 16 and closer than at R = 8."""
    errs = []
    for R in (8.0, 16.0):
        sim, solid, link, shape, normal = _pipe(R)
        total, _ = F.friction_force(sim.f, O.omega_from_nu(1 / 6), solid, link, shape, normal)
        want = 1e-6 * (solid == 0).sum()
        errs.append(abs(total[0] / want - 1.0))
        assert abs(total[1]) < 1e-3 * want and abs(total[2]) < 1e-3 * want
    assert errs[1] < 0.02
    assert errs[1] < errs[0]


def test_branch_normals_of_the_cylinder_sphere_and_base():
    b = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 10.0, 4.0, 0, -1, 0])
    assert np.allclose(F.branch_normal(b, np.array([2.0, 0.0, 5.0])), [1.0, 0.0, 0.0])
    assert np.allclose(F.branch_normal(b, np.array([0.0, -2.0, 3.0])), [0.0, -1.0, 0.0])
    s = np.array([np.sqrt(2.0), 0.0, 10.0 + np.sqrt(2.0)])
    assert np.isclose(np.linalg.norm(s - [0, 0, 10]), 2.0)
    assert np.allclose(F.branch_normal(b, s), (s - [0, 0, 10.0]) / 2.0)
    assert np.allclose(F.branch_normal(b, np.array([0.5, 0.5, 0.0])), [0.0, 0.0, -1.0])


def test_tree_friction_drags_downstream_and_a_fluid_at_rest_exerts_none():
    nx, ny, nz = 64, 32, 32
    b = O.build_tree(O.cfg1_tree_params(), 0.0, [16.0, 16.0, 16.0])
    solid = O.voxelize(b, nx, ny, nz)
    lk = O.links(b, solid, nx, ny, nz)
    rest = O.UniformSim(nx, ny, nz, 1.8, u_in=0.0, solid=solid, link=lk, n_branch=len(b))
    rest.step(3)
    tot0, _ = F.tree_friction_force(rest.f, 1.8, solid, lk, (nx, ny, nz), b)
    assert np.abs(tot0).max() < 1e-15
    nu = 0.05 * O.tree_height(b) / 100.0
    om = O.omega_from_nu(nu)
    sim = O.UniformSim(nx, ny, nz, om, u_in=0.05, solid=solid, link=lk, n_branch=len(b))
    sim.step(300)
    tot, per = F.tree_friction_force(sim.f, om, solid, lk, (nx, ny, nz), b)
    assert np.abs(per.sum(0) - tot).max() <= 1e-12 * np.abs(tot).max()
    assert tot[0] > 0.0
    assert 0.0 < tot[0] < sim.last_force[0]
    # the tree is mirror-symmetric in y
    assert abs(tot[1]) < 1e-9 * tot[0]
