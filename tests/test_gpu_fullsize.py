"""Parity at the full sizes of the benchmarked workloads, in the launch
configuration the benchmark times (autotuned shapes).

- Uniform 512x256x256 workload (order-3 seeded tree, H = 128, Re_H = 2500):
  every fluid cell's populations and the tree force after four steps against
  the FP64 oracle stepping the same box from the same start, FP32 and FP16
  storage (paper Sec. 2.2; Eq. (7)).
- Three-level octree (finest box 1024x512x512, about 2e8 effective cells) and
  the four-level FP16 octree with turbulent inflow (finest box
  2048x1024x1024): the FP64 oracle keeps every level as a dense box, about
  1e2 GB at these sizes, so these check properties that hold at any size --
  graph replay gives the eager bits, the per-branch forces add up to the tree
  force, the state stays finite, a box at rest stays at rest.  The same
  kernels meet the oracle element by element on the four-level box of
  test_gpu_amr.py and test_gpu_inflow.py.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

TOL_F = {"fp32": 2e-6, "fp16": 3e-5}       # per step, as on the small uniform boxes
TOL_FORCE = {"fp32": 2e-5, "fp16": 2e-3}   # relative to the largest force component


def _bench():
    import bench
    return bench


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_uniform_full_size_matches_oracle(gpu, storage):
    B = _bench()
    print(f"[full uniform] {storage}", flush=True)
    arr = B.build_tree(gpu)
    b = gpu.branches_to_numpy(arr)
    g = gpu.Grid(B.NX, B.NY, B.NZ, u_in=B.U_IN, re_h=B.RE_H, storage=storage, drag_every=1)
    g.set_geometry(arr)
    g.autotune()
    g.drag()  # restart the force mean after the tuner's steps
    solid = O.voxelize(b, B.NX, B.NY, B.NZ)
    lk = O.links(b, solid, B.NX, B.NY, B.NZ)
    nu = B.U_IN * O.tree_height(b) / B.RE_H
    sim = O.UniformSim(B.NX, B.NY, B.NZ, O.omega_from_nu(nu), u_in=B.U_IN, solid=solid, link=lk, n_branch=len(b))
    steps = 4
    sim.step(steps)
    g.step(steps - 1)
    g.drag()
    g.step(1)
    d = g.drag(per_branch=True)
    fg = g.get_populations(0)
    fluid = np.flatnonzero(solid == 0)
    err = max(float(np.abs(fg[i, fluid] - sim.f[i, fluid]).max()) for i in range(27))
    del fg
    fo = sim.last_force
    ferr = np.abs(d["force"] - fo).max() / np.abs(fo).max()
    berr = np.abs(d["per_branch"] - sim.last_branch_force[: len(b)]).max() / np.abs(fo).max()
    print(f"  {len(fluid)} fluid cells: max|df| {err:.2e}; force rel err {ferr:.2e}, per branch {berr:.2e}",
          flush=True)
    assert np.isfinite(err) and err < TOL_F[storage] * steps
    assert ferr < TOL_FORCE[storage] and berr < TOL_FORCE[storage]


def _sample(g, level, n, rng):
    """n seeded cell indices over the box of a level, among the cells it holds."""
    B = g.desc.block_edge
    nx, ny, nz = g.level_shape(level)
    m = g.block_map(level).reshape(nz // B, ny // B, nx // B)
    blocks = np.argwhere((m == 1) | (m == 2))
    pick = blocks[rng.integers(0, len(blocks), n)]
    off = rng.integers(0, B, (n, 3))
    z, y, x = (pick * B + off).T
    return x + nx * (y + ny * z)


def _amr_grid(gpu, box, tree, refine, flags, storage, cache, **kw):
    g = gpu.Grid(*box, block_edge=16, levels=len(refine["band"]), storage=storage, drag_every=1, flags=flags, **kw)
    g.set_geometry(tree, refine=refine)
    g.autotune(cache)
    return g


def test_three_level_full_size_properties(gpu):
    B = _bench()
    A = B.AMR
    print("[full amr3] eager and graph replay", flush=True)
    tree = B.amr_tree(gpu)
    refine = {"band": A["band"], "wake": A["wake"]}
    box = (A["nx"], A["ny"], A["nz"])
    cache = os.path.join(tempfile.mkdtemp(), "tune.txt")  # both grids run the same tuned shapes
    grids = [_amr_grid(gpu, box, tree, refine, flags, "fp32", cache, u_in=B.U_IN, re_h=A["re_h"])
             for flags in (0, gpu.LBM_F_GRAPH)]
    rng = np.random.default_rng(3)
    cells = [_sample(grids[0], l, 200000, rng) for l in range(3)]
    for g in grids:
        g.drag()
        g.step(3)
    for l in range(3):
        f0, f1 = grids[0].get_cells(cells[l], l), grids[1].get_cells(cells[l], l)
        assert np.isfinite(f0).all()
        assert np.array_equal(f0, f1)
    d = [g.drag(per_branch=True) for g in grids]
    assert np.array_equal(d[0]["force"], d[1]["force"]) and np.array_equal(d[0]["per_branch"], d[1]["per_branch"])
    tot, pb = d[0]["force"], d[0]["per_branch"]
    print(f"  C_D {d[0]['cd']:.4f}; per-branch sum - total {np.abs(pb.sum(0) - tot).max():.2e}", flush=True)
    assert np.isfinite(d[0]["cd"]) and d[0]["cd"] > 0.0
    assert np.abs(pb.sum(0) - tot).max() <= 1e-9 * np.abs(tot).max()
    for g in grids:
        g.close()


def test_three_level_full_size_rest_stays_at_rest(gpu):
    """No inflow: every level of the full-size octree keeps the rest state."""
    B = _bench()
    A = B.AMR
    print("[full amr3] at rest", flush=True)
    tree = B.amr_tree(gpu)
    g = gpu.Grid(A["nx"], A["ny"], A["nz"], u_in=0.0, nu=0.02, block_edge=16, levels=3, storage="fp32", drag_every=1)
    g.set_geometry(tree, refine={"band": A["band"], "wake": A["wake"]})
    g.step(2)
    rng = np.random.default_rng(4)
    w = O.weights()
    for l in range(3):
        f = g.get_cells(_sample(g, l, 100000, rng), l)
        held = np.isfinite(f[0])
        assert held.any()
        assert np.abs(f[:, held] - w[:, None]).max() < 1e-6
    d = g.drag()
    assert np.abs(d["force"]).max() < 1e-6
    g.close()


def test_four_level_fp16_turbulent_full_size(gpu):
    """The four-level production workload: order-5 seeded tree (364 branches),
    H = 384 finest cells in a 2048x1024x1024 finest box, Re_H = 1.2e5, FP16
    deviation storage, turbulent inflow I_u = 8 % with integral length H/2,
    replayed graphs and tuned shapes.  Over four coarse steps (32 finest
    sub-steps) C_D stays finite, the per-branch forces add up to the tree
    force, the inlet carries the fluctuations, and a sample of cells of every
    level stays finite."""
    import paper_2603_27954_amd as lt
    print("[full amr4] fp16, turbulent inflow", flush=True)
    H = 384.0
    p = lt.tree_params(3, 5, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                       jitter=5.0, seed=5)
    tree = lt.tree_generate(p)
    lt.tree_place(tree, H, [544.0, 495.5, 540.5])
    refine = {"band": [0, 48, 24, 12], "wake": [0, 768, 384, 0]}
    cache = os.path.join(tempfile.mkdtemp(), "tune.txt")
    g = _amr_grid(gpu, (2048, 1024, 1024), tree, refine, gpu.LBM_F_GRAPH, "fp16", cache, u_in=0.05, re_h=1.2e5,
                  turb_intensity=0.08, turb_length=H / 2, turb_seed=41, turb_modes=128)
    info = g.info()
    print(f"  blocks {info['blocks'][:4]}, links {info['links']}, device {info['device_bytes'] / 1e9:.1f} GB",
          flush=True)
    g.drag()
    cds = []
    for _ in range(4):
        g.step(1)
        cds.append(g.drag()["cd"])
    g.step(1)
    d = g.drag(per_branch=True)
    cds.append(d["cd"])
    print(f"  C_D per coarse step {np.round(cds, 4)}", flush=True)
    assert np.all(np.isfinite(cds))
    tot, pb = d["force"], d["per_branch"]
    assert np.abs(pb.sum(0) - tot).max() <= 1e-9 * np.abs(tot).max()
    rng = np.random.default_rng(5)
    for l in range(4):
        f = g.get_cells(_sample(g, l, 100000, rng), l)
        assert np.isfinite(f[:, np.isfinite(f[0])]).all()
    # the inlet column of the coarse level carries the turbulent fluctuations
    nx0, ny0, nz0 = g.level_shape(0)
    inlet = np.arange(ny0 * nz0) * nx0  # x = 0 of every (y, z)
    f = g.get_cells(inlet, 0)
    c = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)], dtype=np.float64)
    rho = f.sum(0)
    v = (c[:, 1:].T @ f) / rho
    rms = v.std(axis=1) / 0.05
    print(f"  inlet column transverse rms / U: {np.round(rms, 4)}", flush=True)
    assert np.all(rms > 0.01)
    g.close()
