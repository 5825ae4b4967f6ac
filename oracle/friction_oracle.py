"""FP64 reference of the friction / pressure split of the drag.

TEST INFRASTRUCTURE ONLY (imported by the tests and the benchmark's CPU leg;
the product library never loads it).

Paper Sec. 3: the friction drag coefficient C_F comes from integrating the
wall shear stress over the whole tree surface into the friction force F_F,
C_F = F_F / (rho U^2 A_x / 2) (Eq. (8)), and the pressure drag coefficient is
the rest, C_P = C_D - C_F (Eq. (9)).  The paper does not say how the LBM
evaluates the wall shear stress.  Reading taken here (the product implements
it independently):

- Viscous stress of a cell, from its pre-collision populations f with density
  rho and velocity u: the second-order central moments
  Pi_ab = sum_i f_i (c_ia - u_a)(c_ib - u_b), their non-equilibrium part
  N = Pi - rho/3 I, and the deviatoric stress sigma = -(1 - omega1/2) dev(N)
  (dev A = A - tr(A)/3 I).  In the continuum limit this is
  rho nu (grad u + grad u^T) with nu = (1/omega1 - 1/2)/3.
- Surface elements: every face between a fluid cell x_f and a solid neighbour
  x_f + e_k along one of the six axis directions.  The wall point is
  x_w = x_f + q e_k with q the link's wall distance; the stress there is
  extrapolated linearly along the axis from x_f and x_f - e_k,
  sigma_w = sigma(x_f) + q (sigma(x_f) - sigma(x_f - e_k)), or taken as
  sigma(x_f) when x_f - e_k is not fluid.
- The face stands for the part of the true surface that projects onto it:
  it carries the weight |n_k|, with n the outward unit normal of the body at
  x_w (sum_k n_k^2 = 1 makes sum over faces of |n_k| g approach the surface
  integral of g).  For the tree, n is the analytic normal of the owning
  branch's shape at x_w: radial for the cylinder's side, radial from the end
  sphere's centre, minus the axis on the base disc, whichever surface lies
  nearest to x_w.
- Wall shear stress: the tangential part of the traction,
  tau_w = (I - n n^T) sigma_w n; the face adds |n_k| tau_w to the friction
  force on the body.
"""
import numpy as np

from . import CVEC, Q

AXES = {14: (0, 1), 12: (0, -1), 16: (1, 1), 10: (1, -1), 22: (2, 1), 4: (2, -1)}  # direction -> (axis, sign)


def cell_stress(f, omega1):
    """Deviatoric viscous stress (n, 3, 3) of pre-collision populations f (27, n)."""
    f = np.asarray(f, dtype=np.float64)
    rho = f.sum(0)
    u = (CVEC.T @ f) / rho
    d = CVEC[:, None, :] - u.T[None, :, :]            # (27, n, 3)
    pi = np.einsum("in,ina,inb->nab", f, d, d)
    N = pi - (rho / 3.0)[:, None, None] * np.eye(3)
    tr = np.trace(N, axis1=1, axis2=2)
    dev = N - (tr / 3.0)[:, None, None] * np.eye(3)
    return -(1.0 - 0.5 * omega1) * dev


def branch_normal(br, x):
    """Outward unit normal of one branch's solid (cylinder from p0 to p1 with
    a sphere of the same diameter at p1) at the surface point x."""
    p0, p1, R = br[0:3], br[3:6], 0.5 * br[6]
    a = p1 - p0
    la2 = a @ a
    t = (x - p0) @ a / la2
    cands = []
    radial = x - p0 - t * a
    r = np.linalg.norm(radial)
    if 0.0 <= t <= 1.0 and r > 0.0:
        cands.append((abs(r - R), radial / r))
    s = x - p1
    rs = np.linalg.norm(s)
    if rs > 0.0:
        cands.append((abs(rs - R), s / rs))
    if r <= R:
        cands.append((abs(t) * np.sqrt(la2), -a / np.sqrt(la2)))
    return min(cands, key=lambda c: c[0])[1]


def friction_force(f, omega1, solid, link, shape, normal, n_branch=1, usable=None):
    """Friction force on the body (3,) and per branch (n_branch, 3).

    f: pre-collision populations (27, N) of the box shape = (nx, ny, nz),
    cell = x + nx (y + ny z); solid: (N,) mask; link: dict of arrays cell,
    dir, q, branch (the boundary links); normal(x_w, branch) -> outward unit
    normal at the wall point (cell centres at integer + 1/2); usable: (N,)
    mask of the cells whose stress may serve as x_f - e_k (default: the fluid
    cells; on a refined grid, the fluid cells of the finest level's leaf
    blocks)."""
    nx, ny, nz = shape
    solid = np.asarray(solid).astype(bool)
    usable = ~solid if usable is None else np.asarray(usable).astype(bool)
    sel = np.isin(link["dir"], list(AXES))
    cells = link["cell"][sel].astype(np.int64)
    dirs = link["dir"][sel].astype(np.int64)
    qs = link["q"][sel]
    brs = link["branch"][sel]
    x = cells % nx
    y = (cells // nx) % ny
    z = cells // (nx * ny)
    ax = np.array([AXES[d][0] for d in dirs])
    sg = np.array([AXES[d][1] for d in dirs])
    back = np.stack([x, y, z], 1)
    back[np.arange(len(cells)), ax] -= sg
    inside = np.all((back >= 0) & (back < np.array([nx, ny, nz])), axis=1)
    bcell = back[:, 0] + nx * (back[:, 1] + ny * back[:, 2])
    bcell = np.where(inside, bcell, cells)
    up = inside & usable[bcell]
    s0 = cell_stress(f[:, cells], omega1)
    s1 = cell_stress(f[:, bcell], omega1)
    sw = np.where(up[:, None, None], s0 + qs[:, None, None] * (s0 - s1), s0)
    total = np.zeros(3)
    per = np.zeros((max(n_branch, 1), 3))
    for k in range(len(cells)):
        if brs[k] < 0:  # a wall point no branch claims has no normal
            continue
        xw = np.array([x[k] + 0.5, y[k] + 0.5, z[k] + 0.5])
        xw[ax[k]] += sg[k] * qs[k]
        n = normal(xw, brs[k])
        t = sw[k] @ n
        tau = t - (n @ t) * n
        df = abs(n[ax[k]]) * tau
        total += df
        if brs[k] < n_branch:
            per[brs[k]] += df
    return total, per


def tree_friction_force(f, omega1, solid, link, shape, branches, usable=None):
    """friction_force with the analytic normals of the tree's branches
    (rows of 10: p0, p1, diameter, generation, parent, id)."""
    b = np.asarray(branches, dtype=np.float64)
    return friction_force(f, omega1, solid, link, shape, lambda xw, k: branch_normal(b[k], xw), len(b), usable)
