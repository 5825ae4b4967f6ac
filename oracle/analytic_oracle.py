"""FP64 reference of the branch-wise analytic drag model.

TEST INFRASTRUCTURE ONLY (imported by the tests, the smoke check and the
benchmark's CPU leg; the product library never loads it).

Paper Sec. 2.4.  Each branch is a cylinder of length L and diameter D whose
axis makes the angle alpha with the flow direction.  Its drag is
F_d = C_d(Re_D) (rho U^2 / 2) L D sin^3(alpha) (Eq. (2)), and the tree's
estimate is C_D-est = sum F_d / ((rho U^2 / 2) A_x) (Eq. (4)).  The branch
Reynolds number is Re_D = Re_H D / H.

The paper fits C_d(Re) to published cylinder measurements that it does not
print.  The curve used here is SYNTHETIC, a documented stand-in and not the
paper's fit:

    C_sub(Re)  = 1 + 10 Re^(-2/3)      (subcritical correlation of White 1991)
    C_post(Re) = 0.25 + 0.35 / (1 + exp(-(ln Re - ln(20 Re_cr)) / 0.8))
    w(Re)      = 1 / (1 + exp((ln Re - ln Re_cr) / 0.12))
    C_d(Re)    = w C_sub + (1 - w) C_post

The critical Reynolds number is Re_cr = 2.7e5 for uniform inflow.  With the
trunk's D0 / H near 0.09, this places the tree's crisis near Re_H = 3e6.  For
an inflow turbulence intensity of 8 % it is Re_cr = 1.4e4, which places the
crisis near Re_H = 1.5e5.  The paper reports both onsets (Sec. 4.1, 4.2).
Between the two intensities Re_cr is interpolated log-linearly in I_u.

Friction split (Eqs. (3), (5), (6)).  A branch's friction drag is
F_f = C_f(Re_D) (rho U^2 / 2) L D sin^3(alpha) (Eq. (3)); C_F-est sums it over
the branches over (rho U^2 / 2) A_x (Eq. (5)) and C_P-est = C_D-est - C_F-est
(Eq. (6)).  The paper takes C_f of a cylinder normal to the flow from its own
LBM runs and prints no values, so C_f here is a table the caller passes: nodes
(log10 Re_D, C_f) joined by power laws (straight lines in log10 Re_D against
ln C_f), and the first and last segments' power laws continued below and above
the table.

Frontal area for the many-tree sweeps: the union of the branches' projected
capsules is rasterised on the (y, z) plane.  A capsule is the branch axis
swept by the branch radius; its projection along x is the 2D capsule of the
projected axis.  Pixels of edge h (units of H) are anchored at the tree's
lower (y, z) bound, and a pixel counts when its centre lies within a capsule.
"""
import math

import numpy as np


def re_critical(intensity):
    return 2.7e5 * (1.4e4 / 2.7e5) ** (intensity / 0.08)


def cylinder_cd(re, intensity=0.0):
    re = np.asarray(re, dtype=np.float64)
    rc = re_critical(intensity)
    lr = np.log(re)
    sub = 1.0 + 10.0 * re ** (-2.0 / 3.0)
    post = 0.25 + 0.35 / (1.0 + np.exp(-(lr - math.log(20.0 * rc)) / 0.8))
    w = 1.0 / (1.0 + np.exp((lr - math.log(rc)) / 0.12))
    return w * sub + (1.0 - w) * post


def branch_geometry(b):
    """Per branch: length L, diameter D, angle alpha to +x (radians), height of
    the midpoint.  b: (n, 10) branch records."""
    d = b[:, 3:6] - b[:, 0:3]
    L = np.linalg.norm(d, axis=1)
    cos_a = np.abs(d[:, 0]) / L
    alpha = np.arccos(np.clip(cos_a, 0.0, 1.0))
    zmid = 0.5 * (b[:, 2] + b[:, 5])
    return L, b[:, 6], alpha, zmid


def tree_cd_est(b, re_h, height, area_x, intensity=0.0):
    """C_D-est of Eq. (4) for one tree at each Re_H in re_h (array)."""
    L, D, alpha, _ = branch_geometry(b)
    w = L * D * np.sin(alpha) ** 3
    re_h = np.atleast_1d(np.asarray(re_h, dtype=np.float64))
    return np.array([np.sum(cylinder_cd(r * D / height, intensity) * w) for r in re_h]) / area_x


def projected_area(b, h):
    """Rasterised frontal area (units of the tree's length scale squared) of
    the branches b (n, 10), pixel edge h."""
    y0, z0, y1, z1, r = b[:, 1], b[:, 2], b[:, 4], b[:, 5], 0.5 * b[:, 6]
    ylo = np.min(np.minimum(y0, y1) - r)
    yhi = np.max(np.maximum(y0, y1) + r)
    zlo = np.min(np.minimum(z0, z1) - r)
    zhi = np.max(np.maximum(z0, z1) + r)
    ny, nz = int(math.ceil((yhi - ylo) / h)), int(math.ceil((zhi - zlo) / h))
    cy = ylo + (np.arange(ny) + 0.5) * h
    cz = zlo + (np.arange(nz) + 0.5) * h
    cover = np.zeros((nz, ny), dtype=bool)
    for k in range(len(b)):
        dy, dz = y1[k] - y0[k], z1[k] - z0[k]
        l2 = dy * dy + dz * dz
        jy = (cy >= min(y0[k], y1[k]) - r[k] - h) & (cy <= max(y0[k], y1[k]) + r[k] + h)
        jz = (cz >= min(z0[k], z1[k]) - r[k] - h) & (cz <= max(z0[k], z1[k]) + r[k] + h)
        if not jy.any() or not jz.any():
            continue
        Y, Z = np.meshgrid(cy[jy] - y0[k], cz[jz] - z0[k])
        t = np.clip((Y * dy + Z * dz) / l2, 0.0, 1.0) if l2 > 0 else np.zeros_like(Y)
        d2 = (Y - t * dy) ** 2 + (Z - t * dz) ** 2
        cover[np.ix_(jz, jy)] |= d2 <= r[k] ** 2
    return cover.sum() * h * h


def cylinder_cf(re, lg_nodes, cf_nodes):
    """C_f(Re_D) of a cylinder normal to the flow from the table (lg_nodes
    strictly increasing log10 Re_D, cf_nodes > 0): the power law through the
    two nodes of the segment that holds log10 Re_D, the end segments continued
    past the table."""
    lg_nodes = np.asarray(lg_nodes, dtype=np.float64)
    ln_cf = np.log(np.asarray(cf_nodes, dtype=np.float64))
    lg = np.log10(np.asarray(re, dtype=np.float64))
    i = np.clip(np.searchsorted(lg_nodes, lg, side="right") - 1, 0, len(lg_nodes) - 2)
    t = (lg - lg_nodes[i]) / (lg_nodes[i + 1] - lg_nodes[i])
    return np.exp((1.0 - t) * ln_cf[i] + t * ln_cf[i + 1])


def tree_cf_est(b, re_h, height, area_x, table):
    """C_F-est of Eq. (5) for one tree at each Re_H in re_h: the friction
    forces of Eq. (3) summed over the branches, with C_f from table =
    (lg_nodes, cf_nodes)."""
    L, D, alpha, _ = branch_geometry(b)
    w = L * D * np.sin(alpha) ** 3
    re_h = np.atleast_1d(np.asarray(re_h, dtype=np.float64))
    return np.array([np.sum(cylinder_cf(r * D / height, *table) * w) for r in re_h]) / area_x


def tree_cp_est(b, re_h, height, area_x, table, intensity=0.0):
    """C_P-est of Eq. (6): the total estimate less the friction estimate."""
    return tree_cd_est(b, re_h, height, area_x, intensity) - tree_cf_est(b, re_h, height, area_x, table)
