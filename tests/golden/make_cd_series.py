"""Writes the FP64 oracle's drag series that the GPU C_D parity tests read.

Calls only the oracle (oracle/); no value here comes from the GPU path.
Each series is the impulsive start of a seeded workload (paper Sec. 2.3:
f = f_eq(1, U) in the fluid at t = 0), sampled at every finest step: the
momentum-exchange force (Sec. 2.2) and C_D = F_x / (rho U^2 A_x / 2) of
Eq. (7).

  uniform   512x256x256 uniform box, order-3 seeded three-child tree (seed 2),
            H = 128, centre of mass (128, 128, 128), Re_H = 2500, U = 0.05,
            1000 steps                    -> cd_series_uniform512x256x256.txt
  octree3   three levels of 8^3-cell blocks, finest box 512x256x256, order-4
            seeded tree (seed 3), H = 128, centre of mass (136, 122.5, 141),
            bands 16 / 8 finest cells and a one-H wake on the middle level,
            Re_H = 2e4, 120 coarse steps  -> cd_series_octree3_512x256x256.txt

usage: python tests/golden/make_cd_series.py uniform|octree3
(OMP_NUM_THREADS sets the oracle's threads; the uniform series takes about
an hour on 8 cores and 15 GB of memory.)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

U = 0.05
WORKLOADS = {
    "uniform": dict(box=(512, 256, 256), order=3, seed=2, H=128.0, com=(128.0, 128.0, 128.0), re_h=2500.0,
                    steps=1000, levels=1, file="cd_series_uniform512x256x256.txt"),
    "octree3": dict(box=(512, 256, 256), order=4, seed=3, H=128.0, com=(136.0, 122.5, 141.0), re_h=2.0e4,
                    steps=120, levels=3, B=8, band=[0, 16, 8], wake=[0, 128, 0],
                    file="cd_series_octree3_512x256x256.txt"),
}


def tree(w):
    return O.build_tree(O.seeded3_tree_params(w["order"], w["seed"]), w["H"], list(w["com"]))


def run(name):
    w = WORKLOADS[name]
    nx, ny, nz = w["box"]
    b = tree(w)
    solid = O.voxelize(b, nx, ny, nz)
    lk = O.links(b, solid, nx, ny, nz)
    ax = O.area_x(solid, nx, ny, nz)
    nu = U * O.tree_height(b) / w["re_h"]
    t0 = time.time()
    if w["levels"] == 1:
        sim = O.UniformSim(nx, ny, nz, O.omega_from_nu(nu), u_in=U, solid=solid, link=lk, n_branch=len(b))
        rec = []
        for s in range(w["steps"]):
            sim.step(1, record=rec)
            if (s + 1) % 50 == 0:
                print(f"{name}: step {s + 1}/{w['steps']} C_D {rec[-1][0] / (0.5 * U * U * ax):.6f} "
                      f"({time.time() - t0:.0f} s)", flush=True)
        forces = np.array(rec)
    else:
        sim = O.AmrSim(w["levels"], w["B"], nx, ny, nz, U, nu, b, w["band"], w["wake"], solid=solid, link=lk,
                       n_branch=len(b))
        for s in range(w["steps"]):
            sim.step(1)
            if (s + 1) % 10 == 0:
                f = sim.force_log()
                print(f"{name}: coarse step {s + 1}/{w['steps']} C_D {f[-1, 0] / (0.5 * U * U * ax):.6f} "
                      f"({time.time() - t0:.0f} s)", flush=True)
        forces = sim.force_log()
    path = os.path.join(HERE, w["file"])
    with open(path, "w") as fh:
        fh.write(f"# FP64 oracle drag series, workload '{name}' of tests/golden/make_cd_series.py\n")
        fh.write(f"# box {nx}x{ny}x{nz}, levels {w['levels']}, Re_H {w['re_h']}, U {U}, A_x {ax}, "
                 f"H {O.tree_height(b):.6f}, branches {len(b)}\n")
        fh.write("# impulsive start (Sec. 2.3); per finest step: momentum-exchange force (Sec. 2.2) and "
                 "C_D of Eq. (7)\n")
        fh.write("# step  C_D  F_x  F_y  F_z\n")
        for s, f in enumerate(forces):
            fh.write(f"{s + 1} {f[0] / (0.5 * U * U * ax):.12e} {f[0]:.12e} {f[1]:.12e} {f[2]:.12e}\n")
    print(f"wrote {path} ({len(forces)} samples, {time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["uniform", "octree3"]:
        run(n)
