"""C_D parity where the stated targets apply: the GPU's drag series against the
FP64 oracle's, stored by tests/golden/make_cd_series.py (which calls only the
oracle), over the impulsive start of two seeded workloads at every finest
step (paper Sec. 2.2 momentum exchange, Eq. (7) C_D):

- the uniform 512x256x256 box (order-3 tree, H = 128, Re_H = 2500), 1000 steps;
- a three-level octree of 8^3 blocks (finest box 512x256x256, order-4 tree,
  H = 128, Re_H = 2e4, bands and a one-H wake), 120 coarse steps.

Targets: C_D within 1e-3 (FP32 storage) and 5e-3 (FP16 deviation storage) of
the oracle, read as: every sample's C_D within the tolerance times the mean
|C_D| of the series (the impulsive start passes near zero, where a pointwise
ratio means nothing), and the mean C_D over the second half within the
tolerance, relative."""
import os
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_cd_series as MK  # noqa: E402

TOL = {"fp32": 1e-3, "fp16": 5e-3}
# BF16 deviations keep 8 significant bits against FP16's 11, so their rounding
# error is 8x FP16's: 8 x 5e-3 allowed (a format bound, not a target)
TOL["bf16"] = 4e-2


def _golden(name):
    w = MK.WORKLOADS[name]
    path = os.path.join(HERE, "golden", w["file"])
    if not os.path.exists(path):
        pytest.skip(f"{w['file']} not written yet")
    ax = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("# box"):
                ax = float(line.split("A_x")[1].split(",")[0])
    data = np.loadtxt(path, comments="#")
    return w, data[:, 1], ax


def _compare(cd_gpu, cd_ref, storage, label):
    scale = np.abs(cd_ref).mean()
    dev = np.abs(cd_gpu - cd_ref).max() / scale
    half = len(cd_ref) // 2
    mean_rel = abs(cd_gpu[half:].mean() - cd_ref[half:].mean()) / abs(cd_ref[half:].mean())
    print(f"  {label} {storage}: max |dC_D| / mean|C_D| = {dev:.2e}, second-half mean C_D gpu "
          f"{cd_gpu[half:].mean():.6f} oracle {cd_ref[half:].mean():.6f} (rel {mean_rel:.2e})", flush=True)
    assert dev < TOL[storage]
    assert mean_rel < TOL[storage]


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_uniform_cd_series_matches_oracle(gpu, storage):
    print(f"[cd series] uniform 512x256x256 {storage}", flush=True)
    w, cd_ref, ax = _golden("uniform")
    b = MK.tree(w)
    g = gpu.Grid(*w["box"], u_in=MK.U, re_h=w["re_h"], storage=storage, drag_every=1)
    g.set_geometry(b)
    assert g.info()["area_x"] == ax
    g.step(w["steps"])
    f = g.drag_series(w["steps"])
    g.close()
    _compare(f[:, 0] / (0.5 * MK.U ** 2 * ax), cd_ref, storage, "uniform")


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_octree_cd_series_matches_oracle(gpu, storage):
    print(f"[cd series] three-level octree {storage}", flush=True)
    w, cd_ref, ax = _golden("octree3")
    b = MK.tree(w)
    g = gpu.Grid(*w["box"], u_in=MK.U, re_h=w["re_h"], block_edge=w["B"], levels=w["levels"], storage=storage,
                 drag_every=1, flags=gpu.LBM_F_GRAPH)
    g.set_geometry(b, refine={"band": w["band"], "wake": w["wake"]})
    assert g.info()["area_x"] == ax
    g.step(w["steps"])
    f = g.drag_series(w["steps"] << (w["levels"] - 1))
    g.close()
    _compare(f[:, 0] / (0.5 * MK.U ** 2 * ax), cd_ref, storage, "octree")
