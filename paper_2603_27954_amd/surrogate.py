"""Per-branch drag surrogate: training samples from LBM runs and tree-level
drag estimates.

This module only sequences calls into the library.  It grids a tree, steps the
flow, reads the per-branch momentum-exchange forces and evaluates the network,
and every computation runs inside the library.

A sample is one branch of one run.  Its features are those of
lbm_branch_features, and its target is the branch force coefficient
y_b = F_x,b / ((rho U^2 / 2) L_b D_b), with F_x,b averaged over the second
part of the run.  A tree's estimate is C_D = sum_b y_b L_b D_b / A_x
(paper Eqs. (2) and (4), with y_b in place of C_d sin^3(alpha)).
"""
import numpy as np

from . import Grid, LBM_F_GRAPH, branch_features, tree_generate, tree_params, tree_place

U_IN = 0.05


def seeded_tree(order, seed, height, com):
    """Three children per node, pitch 35 +- 5 deg, 90 deg phyllotaxis, length
    and width ratios 0.7, trunk width / length 0.3 (the seeded workloads)."""
    p = tree_params(3, order, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                    jitter=5.0, seed=seed)
    arr = tree_generate(p)
    tree_place(arr, height, list(com))
    return arr


def lbm_samples(order, seed, re_h, intensity=0.0, height=32.0, box=(128, 64, 64), steps=4000, average=3000,
                stream=None):
    """One LBM run of a seeded tree: per-branch features and force
    coefficients, the tree's LBM C_D and frontal area."""
    nx, ny, nz = box
    arr = seeded_tree(order, seed, height, (nx / 4.0, ny / 2.0, nz / 2.0))
    turb = {}
    if intensity > 0.0:
        turb = dict(turb_intensity=intensity, turb_length=height / 2.0, turb_seed=seed + 40, turb_modes=64)
    g = Grid(nx, ny, nz, u_in=U_IN, re_h=re_h, storage="fp32", drag_every=10, flags=LBM_F_GRAPH,
             stream=stream, **turb)
    g.set_geometry(arr)
    g.step(steps - average)
    g.drag()
    g.step(average)
    d = g.drag(per_branch=True)
    g.close()
    feat, ld = branch_features(arr, re_h, intensity)
    q = 0.5 * U_IN * U_IN
    y = (d["per_branch"][:, 0] / (q * ld)).astype(np.float32)
    return {"feat": feat, "y": y, "ld": ld, "cd": d["cd"], "area_x": d["area_x"], "branches": arr}


def tree_cd(mlp, feat, ld, area_x):
    """Surrogate C_D of one tree from its branch features."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(feat, dtype=np.float32)).cuda()
    y = torch.empty(len(feat), dtype=torch.float32, device="cuda")
    mlp.predict(x, y)
    return float(np.sum(y.cpu().numpy().astype(np.float64) * ld) / area_x)
