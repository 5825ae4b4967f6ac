"""Host-side checks of liblbmtree (no GPU needed): every symbol the header
declares is exported, descriptions are validated before any device work, and
the host parts of the product path (tree generator, voxeliser, links, FP32
collision arithmetic) agree with the FP64 oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from tests.conftest import gpu_available

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lt():
    import paper_2603_27954_amd as lt
    lt.lib()
    return lt


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt))
    return names


def test_every_declared_symbol_is_exported(lt):
    names = _declared()
    assert len(names) >= 20
    L = C.CDLL(lt.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def _desc(**kw):
    d = dict(nx=64, ny=32, nz=32, u_in=0.05, re_h=100.0)
    d.update(kw)
    return d


@pytest.mark.parametrize("bad", [
    dict(block_edge=12), dict(levels=0), dict(levels=5), dict(nx=60), dict(ny=0),
    dict(u_in=0.2), dict(u_in=-0.01), dict(re_h=0.0, nu=0.0), dict(storage=7),
    dict(nx=64, levels=3, block_edge=16), dict(flags=4),
])
def test_invalid_descriptions_rejected_on_host(lt, bad):
    with pytest.raises(lt.LbmError) as e:
        lt.Grid(**_desc(**bad))
    assert e.value.status == lt.LBM_E_INVALID


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_valid_description_without_device_reports_device_error(lt):
    with pytest.raises(lt.LbmError) as e:
        lt.Grid(**_desc())
    assert e.value.status == lt.LBM_E_DEVICE


@pytest.mark.parametrize("lg, cf", [
    ([1.0], [0.5]),                      # one node
    ([1.0, 1.0], [0.5, 0.4]),            # nodes not increasing
    ([2.0, 1.0], [0.5, 0.4]),
    ([1.0, 2.0], [0.5, 0.0]),            # C_f must be > 0
    ([1.0, 2.0], [0.5, -0.1]),
    ([1.0, float("nan")], [0.5, 0.4]),
    ([1.0, 2.0], [0.5, float("inf")]),
    (list(range(33)), [0.1] * 33),       # more than 32 nodes
])
def test_friction_table_rejected_on_host(lt, lg, cf):
    """lbm_analytic_split validates the C_f table before any device work (the
    device pointers here are never dereferenced)."""
    fake = C.c_void_p(256)
    re_h = np.array([1e4, 1e5])
    d = lt.SweepDesc()
    d.rec, d.tree_start, d.n_trees = fake, fake, 1
    d.re_h, d.n_re = re_h.ctypes.data_as(C.POINTER(C.c_double)), 2
    d.area, d.cd = fake, fake
    lg, cf = np.array(lg, dtype=np.float64), np.array(cf, dtype=np.float64)
    t = lt.CfTable(lg.ctypes.data_as(C.POINTER(C.c_double)), cf.ctypes.data_as(C.POINTER(C.c_double)), len(lg))
    st = lt.lib().lbm_analytic_split(C.byref(d), C.byref(t), fake, None, None)
    assert st == lt.LBM_E_INVALID


def _lib_tree(lt, p: O.TreeParams, target_h, com):
    lp = lt.tree_params(p.m, p.order, p.s0, p.w0, p.len_ratio, p.wid_ratio, p.pre_roll, p.pitch,
                        p.post_roll, p.jitter, p.seed)
    arr = lt.tree_generate(lp)
    if target_h is not None:
        lt.tree_place(arr, target_h, com)
    return lt.branches_to_numpy(arr)


@pytest.mark.parametrize("case", ["cfg1", "seeded3_o3", "seeded3_o5", "paper_n6"])
def test_tree_generator_matches_oracle(lt, case):
    if case == "cfg1":
        p, h, com = O.cfg1_tree_params(), 0.0, [16.0, 16.0, 16.0]
    elif case == "seeded3_o3":
        p, h, com = O.seeded3_tree_params(3, 2), 128.0, [128.0, 128.0, 128.0]
    elif case == "seeded3_o5":
        p, h, com = O.seeded3_tree_params(5, 4), 512.0, [512.0, 512.0, 512.0]
    else:
        p, h, com = O.paper_tree_params(5), 1.0, [8.0, 8.0, 8.0]
    ref = O.build_tree(p, h, com)
    got = _lib_tree(lt, p, h, com)
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=0, atol=1e-9 * max(1.0, h))


@pytest.mark.parametrize("case", ["cfg1", "seeded3_small", "cylinder_spanning_y"])
def test_voxels_links_area_match_oracle(lt, case):
    """P11: accelerated voxeliser / link builder equal the brute-force oracle
    (with wrapped y and z neighbours, also for a cylinder that spans y)."""
    if case == "cfg1":
        nx, ny, nz = 64, 32, 32
        b = O.build_tree(O.cfg1_tree_params(), 0.0, [16.0, 16.0, 16.0])
    elif case == "cylinder_spanning_y":
        nx, ny, nz = 96, 16, 48
        b = np.array([[24.3, -16.0, 23.7, 24.3, 32.0, 23.7, 11.0, 0.0, -1.0, 0.0]])
    else:
        nx, ny, nz = 192, 96, 96
        b = O.build_tree(O.seeded3_tree_params(3, 2), 48.0, [48.0, 48.0, 48.0])
    solid_o = O.voxelize(b, nx, ny, nz)
    lk_o = O.links(b, solid_o, nx, ny, nz)
    solid_l, lk_l, ax_l = lt.geometry_build(b, nx, ny, nz)
    assert np.array_equal(solid_o, solid_l)
    assert ax_l == O.area_x(solid_o, nx, ny, nz)
    assert np.array_equal(lk_o["cell"], lk_l["cell"]) and np.array_equal(lk_o["dir"], lk_l["dir"])
    assert np.abs(lk_o["q"] - lk_l["q"]).max() < 1e-12
    assert np.array_equal(lk_o["branch"], lk_l["branch"])


def test_fp32_collision_matches_oracle(lt):
    """The kernels' FP32 collision arithmetic (run on the host) against the FP64
    oracle: populations within FP32 rounding, mass and momentum kept."""
    rng = np.random.default_rng(21)
    worst = 0.0
    for trial in range(200):
        u = rng.uniform(-0.1, 0.1, 3)
        f = O.equilibrium(rng.uniform(0.95, 1.05), u) * (1 + 0.05 * rng.standard_normal(27))
        w1 = rng.uniform(0.6, 1.999)
        gal = bool(trial % 2)
        ref = O.collide(f, w1, galilean=gal)
        got = lt.collide_cell_host(f, w1, galilean=gal)
        worst = max(worst, np.abs(got - ref).max())
        assert abs(got.sum() - ref.sum()) < 2e-7
        assert np.allclose(got @ O.CVEC, ref @ O.CVEC, atol=2e-7)
    assert worst < 5e-7


@pytest.mark.parametrize("case", [
    dict(L=2, B=8, box=(96, 96, 96), com=(40.0, 48.0, 48.0), band=[0, 8], wake=[0, 0]),
    dict(L=3, B=8, box=(256, 128, 128), com=(96.0, 64.0, 64.0), band=[0, 2, 0], wake=[0, 0, 0]),
    dict(L=2, B=16, box=(128, 128, 128), com=(48.0, 64.0, 64.0), band=[0, 4], wake=[0, 0]),
    dict(L=3, B=8, box=(256, 128, 128), com=(96.0, 64.0, 64.0), band=[0, 2, 0], wake=[0, 64, 0]),
    dict(L=3, B=8, box=(256, 128, 128), com=(96.0, 64.0, 64.0), band=[0, 2, 0], wake=[0, 48, 32]),
])
def test_planned_block_maps_match_oracle(lt, case):
    """The library's host-built block grid (lbm_plan_levels, the same builder
    lbm_set_geometry uses) equals the oracle's, level by level."""
    nx, ny, nz = case["box"]
    b = O.build_tree(O.cfg1_tree_params(), 0.0, list(case["com"]))
    refine = {"band": case["band"], "wake": case["wake"]}
    plan = lt.plan_levels(b, refine=refine, maps=True, nx=nx, ny=ny, nz=nz, u_in=0.05, re_h=100.0,
                          block_edge=case["B"], levels=case["L"])
    nu = 0.05 * O.tree_height(b) / 100.0
    sim = O.AmrSim(case["L"], case["B"], nx, ny, nz, 0.05, nu, b, case["band"], case["wake"])
    for l in range(case["L"]):
        assert np.array_equal(plan["maps"][l].astype(np.uint8), sim.block_map(l)), f"level {l}"
    solid = O.voxelize(b, nx, ny, nz)
    # cell classes: leaf cells (class active), and the cells each level
    # sub-step collides (active and band, minus the finest level's solid)
    for l in range(case["L"]):
        cls = sim.classes(l)
        sol = solid.astype(bool) if l == case["L"] - 1 else np.zeros(cls.shape, bool)
        assert plan["leaf_cells"][l] == int((cls == O.CLS_ACTIVE).sum()), f"level {l}"
        assert plan["updated_cells"][l] == int(((cls == O.CLS_ACTIVE) & ~sol).sum()), f"level {l}"
        assert plan["collided_cells"][l] == int((((cls == O.CLS_ACTIVE) | (cls == O.CLS_BAND)) & ~sol).sum()), \
            f"level {l}"
    assert plan["solid_cells"] == int(solid.sum())
    assert plan["links"] == len(O.links(b, solid, nx, ny, nz)["cell"])


# The octree workloads' own geometries: the three-level grid (order-4 seeded
# tree, seed 3, H = 256, finest box 1024x512x512, bands 32/16 and a one-H
# wake) and the four-level grid (order-5 tree, seed 5, H = 384, finest box
# 2048x1024x1024, bands 48/24/12, wakes 768/384)
OCTREES = {
    "three_level_1024x512x512": dict(order=4, seed=3, H=256.0, com=(272.0, 245.0, 282.0), box=(1024, 512, 512),
                                     band=[0, 32, 16], wake=[0, 256, 0]),
    "four_level_2048x1024x1024": dict(order=5, seed=5, H=384.0, com=(544.0, 495.5, 540.5),
                                      box=(2048, 1024, 1024), band=[0, 48, 24, 12], wake=[0, 768, 384, 0]),
}


@pytest.mark.parametrize("name", list(OCTREES))
def test_planned_block_maps_with_wake_match_oracle_at_full_size(lt, name):
    """Block maps of the wake-refined octree workloads, bit for bit against the
    oracle's refinement rule (maps only: the oracle's dense state would not fit
    at these sizes)."""
    c = OCTREES[name]
    L = len(c["band"])
    b = O.build_tree(O.seeded3_tree_params(c["order"], c["seed"]), c["H"], list(c["com"]))
    want = O.amr_maps(L, 16, *c["box"], b, c["band"], c["wake"])
    nx, ny, nz = c["box"]
    plan = lt.plan_levels(b, refine={"band": c["band"], "wake": c["wake"]}, maps=True, nx=nx, ny=ny, nz=nz,
                          u_in=0.05, re_h=2e4, block_edge=16, levels=L)
    for l in range(L):
        assert np.array_equal(plan["maps"][l].astype(np.uint8), want[l]), f"level {l}"
    # the wake refines blocks that the surface bands alone leave coarse
    bands_only = O.amr_maps(L, 16, *c["box"], b, c["band"], [0] * L)
    assert (want[0] == 2).sum() > (bands_only[0] == 2).sum()


# Five to seven levels (8^3 blocks) around the paper's n = 4 tree (Table 2)
# in the paper's 32H x 16H x 16H domain with the centre of mass at
# (8H, 8H, 8H): the surface refined to H/64 .. H/256 and the wake two levels
# above the finest
DEEP = {
    "five_level_H64": dict(L=5, H=64.0, band=[0, 64, 32, 16, 4], wake=[0, 0, 128, 0, 0]),
    "six_level_H128": dict(L=6, H=128.0, band=[0, 128, 64, 32, 16, 4], wake=[0, 0, 0, 256, 0, 0]),
    "seven_level_H256": dict(L=7, H=256.0, band=[0, 256, 128, 64, 32, 16, 8], wake=[0, 0, 0, 0, 512, 0, 0]),
}


def _paper_tree(lt, n, H, com):
    wq = 0.5 ** 0.5
    p = lt.tree_params(2, n - 1, 100.0, 30.0, [0.8, 0.8], [wq, wq], [0.0, 0.0], [30.0, -30.0], [137.0, 137.0])
    arr = lt.tree_generate(p)
    lt.tree_place(arr, H, list(com))
    return arr


@pytest.mark.parametrize("name", list(DEEP))
def test_planned_block_maps_of_deep_octrees_match_oracle(lt, name):
    """Grids of five to seven levels (the paper's surface resolution needs
    six or seven above a dense coarse level): block maps bit for bit against
    the oracle's refinement rule, although the library keeps each finer
    level's map over the blocks around its refined region only."""
    c = DEEP[name]
    H, L = c["H"], c["L"]
    nx, ny, nz = int(32 * H), int(16 * H), int(16 * H)
    arr = _paper_tree(lt, 4, H, (8 * H, 8 * H, 8 * H))
    b = lt.branches_to_numpy(arr)
    want = O.amr_maps(L, 8, nx, ny, nz, b, c["band"], c["wake"])
    plan = lt.plan_levels(arr, refine={"band": c["band"], "wake": c["wake"]}, maps=True, nx=nx, ny=ny, nz=nz,
                          u_in=0.05, re_h=2500.0, block_edge=8, levels=L)
    for l in range(L):
        assert np.array_equal(plan["maps"][l].astype(np.uint8), want[l]), f"level {l}"
        assert (want[l] == 1).any(), f"level {l} has leaf blocks"
    assert plan["levels"] == L


def test_plan_of_the_paper_tree_at_h512_stays_sparse(lt):
    """The n = 4 tree in the paper's 32H x 16H x 16H domain at H = 512 finest
    cells (six levels, coarse H/16): the finest lattice has 2.1e9 blocks and
    the finest box 1.1e12 cells, so dense host maps or masks could not be
    built; the plan holds the tree's own extent and finishes in seconds."""
    import time
    H = 512.0
    arr = _paper_tree(lt, 4, H, (8 * H, 8 * H, 8 * H))
    t0 = time.time()
    plan = lt.plan_levels(arr, refine={"band": [0, 256, 128, 64, 32, 16], "wake": [0, 0, 0, 1024, 0, 0]},
                          nx=int(32 * H), ny=int(16 * H), nz=int(16 * H), u_in=0.05, re_h=2500.0, block_edge=8,
                          levels=6, storage="fp16")
    dt = time.time() - t0
    assert plan["lattice"][5] == (2048, 1024, 1024)
    assert 0.99 * 512 * 256 * 256 < plan["leaf_cells"][0] < 512 * 256 * 256  # dense level 0, refined around the tree
    assert all(c > 0 for c in plan["leaf_cells"])
    assert plan["solid_cells"] > 1_000_000 and plan["links"] > plan["solid_cells"] // 10
    # 27 deviations of 2 bytes per stored cell (blocks + the spare block per level)
    cells = 512 * 256 * 256 + sum((b + 1) * 512 for b in plan["blocks"][1:])
    assert abs(plan["pop_bytes"] - 54 * cells) < 0.01 * plan["pop_bytes"] + 64 * 1024 * 6
    print(f"  H/512 plan: {dt:.1f} s, leaf cells {sum(plan['leaf_cells']):,}, {plan['pop_bytes'] / 1e9:.2f} GB")


def test_only_a_y_parallel_cylinder_may_cross_the_y_faces(lt):
    """On one level with periodic y a branch along y that runs past both y
    faces is accepted; one that ends inside the box near a y face, is tilted,
    or sits on a two-level grid is not."""
    def plan(b, levels=1):
        return lt.plan_levels(np.array(b, dtype=np.float64), refine={"band": [0, 8], "wake": [0, 0]} if levels > 1
                              else None, nx=128, ny=32, nz=128, u_in=0.05, nu=0.01, block_edge=16, levels=levels)
    ok = [[64.0, -8.0, 64.0, 64.0, 40.0, 64.0, 8.0, 0, -1, 0]]
    plan(ok)
    for bad, levels in (([[64.0, 1.0, 64.0, 64.0, 40.0, 64.0, 8.0, 0, -1, 0]], 1),
                        ([[64.0, -8.0, 64.0, 65.0, 40.0, 64.0, 8.0, 0, -1, 0]], 1),
                        (ok, 2)):
        with pytest.raises(lt.LbmError) as e:
            plan(bad, levels)
        assert e.value.status == lt.LBM_E_INVALID


def test_plan_rejects_refinement_at_the_faces(lt):
    b = O.build_tree(O.cfg1_tree_params(), 0.0, [40.0, 20.0, 32.0])
    with pytest.raises(lt.LbmError) as e:
        lt.plan_levels(b, refine={"band": [0, 24, 6], "wake": [0, 40, 0]}, nx=256, ny=128, nz=128, u_in=0.05,
                       re_h=100.0, block_edge=8, levels=3)
    assert e.value.status == lt.LBM_E_INVALID


@pytest.mark.parametrize("seed,n,dx,length", [(40, 200, 4.0, 128.0), (7, 64, 1.0, 8.0)])
def test_inflow_modes_match_oracle(lt, seed, n, dx, length):
    """The library's host-built inflow mode set (its own generator, shells and
    calibration) equals the oracle's built from the same seed."""
    from oracle import turb_oracle as T
    m = lt.inflow_modes(seed, n, 0.08, length, 0.05, dx)
    o = T.build_modes(seed, n, 0.08, length, 0.05, dx)
    assert abs(m["k_e"] - o.k_e) < 1e-12 * o.k_e
    assert np.allclose(m["kvec"], o.kvec, rtol=1e-13, atol=1e-16)
    assert np.allclose(m["sigma"], o.sigma, rtol=1e-13, atol=1e-15)
    assert np.allclose(m["psi"], o.psi, rtol=1e-15, atol=0)
    assert np.allclose(m["amp"], o.amp, rtol=1e-11, atol=0)


def test_tree_batch_records_match_oracle(lt):
    """Branch records of the many-tree sweep (seeded three-child trees at unit
    height) against the oracle's own trees and geometry."""
    from oracle import analytic_oracle as A
    params = lt.tree_params(3, 3, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                            jitter=5.0, seed=0)
    orders = [1, 2, 3, 4, 0, 2]
    rec, start = lt.tree_batch(params, 500, orders)
    assert list(np.diff(start)) == [sum(3 ** k for k in range(o + 1)) for o in orders]
    for i, o in enumerate(orders):
        b = O.build_tree(O.seeded3_tree_params(o, 500 + i), 1.0, [0.0, 0.0, 0.0])
        L, D, alpha, zmid = A.branch_geometry(b)
        r = rec[start[i]:start[i + 1]].astype(np.float64)
        assert np.allclose(r[:, 0], np.log10(D), atol=1e-6)
        assert np.allclose(r[:, 1], np.degrees(alpha), atol=2e-4)
        assert np.array_equal(r[:, 2], b[:, 7])
        assert np.allclose(r[:, 3], zmid - b[0, 2], atol=1e-6)
        assert np.allclose(r[:, 4], L * D, rtol=1e-6)
        assert np.allclose(r[:, 5:9], b[:, [1, 2, 4, 5]], atol=1e-6)
        assert np.allclose(r[:, 9], 0.5 * D, rtol=1e-6)
