"""Pins of the oracle's geometry: the paper's printed tree features (Table 3),
the branch scaling laws of Sec. 2.1.2, branch counts, the SplitMix64 test
vector, voxel volumes against the analytic volume, link wall distances against
closed-form ray-circle roots, frontal area, and the unit conversions printed in
Sec. 4."""
import numpy as np
import pytest

import oracle as O


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows[key] = [float(v) for v in vals]
    return rows


@pytest.mark.parametrize("n", [4, 6, 8])
def test_paper_table3_features(n):
    """P10: D0/H and L0/H of the binary family (Table 2 parameters) within 1 % of
    Table 3 when the n rewrites draw n generations (trunk + n-1 child levels)."""
    t3 = _golden("table3_tree_features.txt")
    b = O.tree_generate(O.paper_tree_params(n - 1))
    H = O.tree_height(b)
    d0h, l0h = t3[f"n{n}"]
    assert abs((30.0 / H) / d0h - 1) < 0.01
    assert abs((100.0 / H) / l0h - 1) < 0.01
    assert len(b) == 2 ** n - 1


def test_paper_family_scaling_laws():
    """L_k = 0.8 L_{k-1}, D_k = 0.5^0.5 D_{k-1} (Sec. 2.1.2) and children start at
    the parent's end."""
    b = O.tree_generate(O.paper_tree_params(5))
    lens = np.linalg.norm(b[:, 3:6] - b[:, 0:3], axis=1)
    for i in range(1, len(b)):
        par = int(b[i, 8])
        assert np.isclose(lens[i], 0.8 * lens[par])
        assert np.isclose(b[i, 6], 0.5 ** 0.5 * b[par, 6])
        assert np.allclose(b[i, 0:3], b[par, 3:6])
        assert b[i, 7] == b[par, 7] + 1


@pytest.mark.parametrize("order,count", [(1, 4), (3, 40), (4, 121), (5, 364)])
def test_three_child_branch_counts_and_ratios(order, count):
    b = O.tree_generate(O.seeded3_tree_params(order, 2))
    assert len(b) == count == sum(3 ** k for k in range(order + 1))
    lens = np.linalg.norm(b[:, 3:6] - b[:, 0:3], axis=1)
    for i in range(1, len(b)):
        par = int(b[i, 8])
        assert np.isclose(lens[i], 0.7 * lens[par]) and np.isclose(b[i, 6], 0.7 * b[par, 6])
        # pitch angle between child and parent axes within 35 +- 5 degrees
        a = (b[i, 3:6] - b[i, 0:3]) / lens[i]
        p = (b[par, 3:6] - b[par, 0:3]) / lens[par]
        ang = np.degrees(np.arccos(np.clip(a @ p, -1, 1)))
        assert 30.0 - 1e-9 <= ang <= 40.0 + 1e-9
    assert np.isclose(b[0, 6] / lens[0], 0.3)


def test_seeded_tree_determinism():
    a = O.tree_generate(O.seeded3_tree_params(3, 7))
    b = O.tree_generate(O.seeded3_tree_params(3, 7))
    c = O.tree_generate(O.seeded3_tree_params(3, 8))
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_splitmix64_published_vector():
    """First outputs of SplitMix64 from state 0 (Vigna's reference generator)."""
    import ctypes as C
    st = C.c_uint64(0)
    L = O.lib()
    u = L.or_splitmix_uniform(C.byref(st))
    assert u == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53
    u2 = L.or_splitmix_uniform(C.byref(st))
    assert u2 == (0x6E789E6AA1B965F4 >> 11) * 2.0 ** -53


def test_cfg1_tree_height_and_placement():
    b = O.build_tree(O.cfg1_tree_params(), 0.0, [16.0, 16.0, 16.0])
    H = O.tree_height(b)
    assert abs(H - (16 + 11.2 * np.cos(np.radians(30)))) < 1e-12
    assert abs(b[0, 2] - 2.7717) < 1e-3
    # y-z plane children, symmetric about y = 16
    assert np.allclose(b[:, [0, 3]], 16.0)
    assert np.isclose(b[1, 4] - 16.0, -(b[2, 4] - 16.0))


def test_placed_tree_com_and_height():
    b = O.build_tree(O.seeded3_tree_params(3, 2), 128.0, [128.0, 128.0, 128.0])
    assert np.isclose(O.tree_height(b), 128.0)
    lens = np.linalg.norm(b[:, 3:6] - b[:, 0:3], axis=1)
    vol = np.pi * 0.25 * b[:, 6] ** 2 * lens
    com = (vol[:, None] * 0.5 * (b[:, 0:3] + b[:, 3:6])).sum(0) / vol.sum()
    assert np.allclose(com, 128.0)


def test_voxel_volume_matches_shapes():
    """Voxel count of one thick cylinder (trunk only) + end sphere vs analytic volume."""
    p = O.cfg1_tree_params()
    p.order = 0
    p.s0, p.w0 = 30.0, 16.0
    b = O.build_tree(p, 0.0, [32.0, 32.0, 32.0])
    n = 64
    s = O.voxelize(b, n, n, n)
    R, L = 8.0, 30.0
    vol = np.pi * R * R * L + 0.5 * 4 / 3 * np.pi * R ** 3
    assert abs(s.sum() / vol - 1) < 0.04  # lattice-point count of a radius-8 disc


def test_link_q_matches_ray_circle_roots():
    """Links of a vertical cylinder: for in-plane directions q is the first root
    of |o + t c - axis|^2 = R^2; the branch id is the only branch."""
    p = O.cfg1_tree_params()
    p.order = 0
    p.s0, p.w0 = 40.0, 9.0
    b = O.build_tree(p, 0.0, [16.3, 15.8, 30.0])
    nx, ny, nz = 32, 32, 64
    s = O.voxelize(b, nx, ny, nz)
    lk = O.links(b, s, nx, ny, nz)
    assert len(lk["cell"]) > 200
    ax = b[0, 0:2]
    R = b[0, 6] / 2
    z0, z1 = b[0, 2], b[0, 5]
    checked = 0
    for c, d, q, br in zip(lk["cell"], lk["dir"], lk["q"], lk["branch"]):
        assert 0 < q <= 1 and br == 0
        x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
        if O.CZ[d] != 0 or not (z0 + 2 < z + 0.5 < z1 - R - 2):
            continue
        o = np.array([x + .5, y + .5]) - ax
        dv = np.array([O.CX[d], O.CY[d]], float)
        A, B, Cc = dv @ dv, 2 * o @ dv, o @ o - R * R
        t = (-B - np.sqrt(B * B - 4 * A * Cc)) / (2 * A)
        assert abs(t - q) < 1e-12
        checked += 1
    assert checked > 50
    # every fluid cell next to a solid cell has exactly its links
    fl = np.nonzero(s == 0)[0]
    n_expected = 0
    for c in fl:
        x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
        for i in range(27):
            xs, ys, zs = x + O.CX[i], (y + O.CY[i]) % ny, (z + O.CZ[i]) % nz
            if 0 <= xs < nx and i != 13 and s[xs + nx * (ys + ny * zs)]:
                n_expected += 1
    assert n_expected == len(lk["cell"])


def test_frontal_area():
    p = O.cfg1_tree_params()
    p.order = 0
    p.s0, p.w0 = 20.0, 10.0
    b = O.build_tree(p, 0.0, [16.0, 16.0, 16.0])
    n = 32
    s = O.voxelize(b, n, n, n)
    ax = O.area_x(s, n, n, n)
    # projection of cylinder (20 x 10) plus the half-disc of the end sphere above it
    analytic = 20.0 * 10.0 + 0.5 * np.pi * 25.0
    assert abs(ax / analytic - 1) < 0.06


def test_unit_conversions_printed_in_paper():
    """P16: Re_H = U H / nu with nu = 1.5e-5: 1 m/s on 1.5 m and 60 m/s on 30 m
    span 1e5..1e8 (Sec. 4.1); Re_H,cr = 1.5e5 on a 10 m tree is U ~ 0.2 m/s (Sec. 4.2)."""
    nu = 1.5e-5
    assert 0.9e5 < 1.0 * 1.5 / nu < 1.1e5
    assert 1.0e8 < 60.0 * 30.0 / nu < 1.3e8
    assert abs(1.5e5 * nu / 10.0 - 0.225) < 1e-9
