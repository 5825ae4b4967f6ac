"""GPU parity of the multi-level (octree block) path against the FP64 oracle:
block maps (bit-exact), populations of every active cell of every level and
the per-finest-step tree force after a few coarse steps (both A-A parities,
prolongation from T and from the T/T+1 mean, restriction), and a longer run's
C_D (paper Sec. 2.2; Eq. (7))."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
U = 0.05

CONFIGS = {
    "two_level_b8": dict(L=2, B=8, box=(96, 96, 96), com=(40.0, 48.0, 48.0), band=[0, 8], wake=[0, 0]),
    "three_level_b8": dict(L=3, B=8, box=(256, 128, 128), com=(96.0, 64.0, 64.0), band=[0, 2, 0],
                           wake=[0, 0, 0]),
    "two_level_b16": dict(L=2, B=16, box=(128, 128, 128), com=(48.0, 64.0, 64.0), band=[0, 4], wake=[0, 0]),
    # wake-box refinement on both refined levels (the octree workloads refine
    # their wakes the same way)
    "three_level_b8_wake": dict(L=3, B=8, box=(256, 128, 128), com=(96.0, 64.0, 64.0), band=[0, 2, 0],
                                wake=[0, 48, 32]),
    # the paper's own tree (Table 2, n = 4 rewrites: trunk and three child
    # levels, 15 branches) at H = 64 on 8^3 blocks, with a wake
    "three_level_b8_paper_n4": dict(L=3, B=8, box=(512, 256, 256), com=(192.0, 128.0, 128.0), band=[0, 4, 0],
                                    wake=[0, 64, 0], tree="paper_n4", H=64.0),
    # four levels (the smallest box whose refined blocks keep one coarse block
    # from the faces): coarse 64x32x32, finest 512x256x256
    "four_level_b8": dict(L=4, B=8, box=(512, 256, 256), com=(192.0, 128.0, 128.0), band=[0, 4, 2, 0],
                          wake=[0, 0, 0, 0]),
}
# FP16 deviation storage: one rounding of deviations of O(0.05) to 11 bits per
# stored population and sub-step, 3e-5 (as on the uniform grid), summed over
# the finest sub-steps done
TOL_STEP = {"fp32": 4e-6, "fp16": 3e-5}


def _setup(gpu, name, storage="fp32", with_body=True):
    c = CONFIGS[name]
    nx, ny, nz = c["box"]
    if c.get("tree") == "paper_n4":
        b = O.build_tree(O.paper_tree_params(3), c["H"], list(c["com"]))
    else:
        b = O.build_tree(O.cfg1_tree_params(), 0.0, list(c["com"]))
    nu = U * O.tree_height(b) / 100.0
    g = gpu.Grid(nx, ny, nz, u_in=U, re_h=100.0, block_edge=c["B"], levels=c["L"], storage=storage, drag_every=1)
    g.set_geometry(b, refine={"band": c["band"], "wake": c["wake"]})
    solid = O.voxelize(b, nx, ny, nz)
    lk = O.links(b, solid, nx, ny, nz)
    sim = O.AmrSim(c["L"], c["B"], nx, ny, nz, U, nu, b, c["band"], c["wake"], solid=solid, link=lk,
                   n_branch=len(b))
    return g, sim, solid, b


@pytest.mark.parametrize("name", list(CONFIGS))
def test_block_maps_match_oracle(gpu, name):
    print(f"[amr maps] {name}", flush=True)
    g, sim, _, _ = _setup(gpu, name)
    for l in range(CONFIGS[name]["L"]):
        assert np.array_equal(g.block_map(l).astype(np.uint8), sim.block_map(l)), f"level {l}"


@pytest.mark.parametrize("name,storage", [("two_level_b8", "fp32"), ("three_level_b8", "fp32"),
                                          ("three_level_b8_wake", "fp32"), ("three_level_b8_wake", "fp16"),
                                          ("three_level_b8_paper_n4", "fp32"),
                                          ("two_level_b16", "fp32"), ("four_level_b8", "fp32"),
                                          ("three_level_b8", "fp16"), ("four_level_b8", "fp16")])
def test_coarse_steps_match_oracle(gpu, name, storage):
    print(f"[amr steps] {name} {storage}", flush=True)
    g, sim, solid, b = _setup(gpu, name, storage)
    L = CONFIGS[name]["L"]
    tol = TOL_STEP[storage] * (1 if storage == "fp32" else 1 << (L - 1))
    for step in range(3):
        g.step(1)
        sim.step(1)
        for l in range(L):
            cls = sim.classes(l)
            act = cls == O.CLS_ACTIVE
            if l == L - 1:
                act &= solid == 0
            idx = np.flatnonzero(act)
            err = np.abs(g.get_cells(idx, l) - sim.get_f(l)[:, idx]).max()
            print(f"  coarse step {step + 1} level {l}: {act.sum()} active cells, max |df| = {err:.3e}",
                  flush=True)
            assert np.isfinite(err) and err < tol * (step + 1)
    fo = sim.force_log()
    fgs = g.drag_series(len(fo))
    assert fgs.shape == fo.shape
    assert np.abs(fgs - fo).max() < (2e-5 if storage == "fp32" else 2e-3) * np.abs(fo).max()


def test_two_level_run_cd_matches_oracle(gpu):
    """40 coarse steps (80 finest) of the two-level grid: velocity of the
    finest active cells within 1e-4 U and C_D of the last coarse step within
    1e-3 of the oracle."""
    g, sim, solid, b = _setup(gpu, "two_level_b8")
    g.step(39)
    g.drag()
    g.step(1)
    d = g.drag()
    sim.step(40)
    fo = sim.force_log()
    ax = O.area_x(solid, *CONFIGS["two_level_b8"]["box"])
    cd_o = fo[-2:, 0].mean() / (0.5 * U * U * ax)
    rel = abs(d["cd"] - cd_o) / abs(cd_o)
    _, ug = g.fields(1)
    _, uo = sim.fields(1)
    act = (sim.classes(1) == O.CLS_ACTIVE) & (solid == 0)
    du = np.abs(ug[act] - uo[act]).max() / U
    print(f"  C_D gpu {d['cd']:.6f} oracle {cd_o:.6f} rel {rel:.2e}; max|du|/U {du:.2e}", flush=True)
    assert rel < 1e-3
    assert du < 1e-4
