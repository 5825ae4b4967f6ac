"""Throughput of the D3Q27 cumulant LBM hot path on one MI355X.

Workload (uniform grid): 512 x 256 x 256 cells (33,554,432), order-3 seeded
L-system tree with three children per node (pitch 35 +- 5 deg, 90 deg
phyllotaxis, ratios 0.7, seed 2) scaled to H = 128 cells with its centre of
mass at (128, 128, 128); Re_H = 2500, uniform inflow u = 0.05 along +x,
zero-gradient outlet, periodic lateral faces.  Synthetic: the tree and the
flow are generated here.

A step is one collide-and-stream pass over every fluid cell plus the
interpolated bounce-back and the FP64 force reduction of the tree.  The timed
region runs K steps with populations stored as FP32 deviations (the reported
value) and K steps with FP16 deviations; arithmetic is FP32 in both.

Prints one JSON line.  With the CPU leg on (default) it also times the FP64
oracle on a bounded sample of the same workload and compares C_D after that
many steps (GPU FP32 / FP16 against the oracle).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STREAM = None
TUNE = True
TUNE_CACHE = None  # file of tuned launch shapes shared by runs (None: tune afresh)
SURROGATE_DUMP = None  # .npz path for the surrogate's training samples and held-out runs (None: not kept)
SURROGATE_TRAIN = {}  # overrides of the scale's training settings (epochs, batch, lr)
NX, NY, NZ, H = 512, 256, 256, 128.0
RE_H, U_IN = 2500.0, 0.05


KERNEL_SOURCES = ("paper_2603_27954_amd/csrc/lbm_kernels.hip", "paper_2603_27954_amd/csrc/lbm_bodies.h",
                  "paper_2603_27954_amd/csrc/lbm_access.h", "paper_2603_27954_amd/csrc/lbm_device.h")


TRAFFIC_FILES = {"fp32": "profiles/k_collide_dense_uniform512x256x256_hbm_counters.txt",
                 "fp16": "profiles/k_collide_dense_fp16_uniform512x256x256_hbm_counters.txt"}


def measured_traffic(storage="fp32"):
    """HBM bytes per collide launch from the committed rocprofv3 counter
    summary of that storage format, or None when the kernel sources changed
    since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, TRAFFIC_FILES[storage])
    if not os.path.exists(prof):
        return None
    vals = {}
    for line in open(prof):
        if line and not line.startswith("#") and not line.startswith(" "):
            k, _, v = line.strip().partition(" ")
            vals[k] = v.strip()
    m = hashlib.sha256()
    for f in KERNEL_SOURCES:
        m.update(open(os.path.join(ROOT, f), "rb").read())
    if vals.get("kernel_sources_sha256_16") != m.hexdigest()[:16]:
        return None
    return float(vals["traffic_bytes_per_launch_mean"])


def build_tree(lt):
    p = lt.tree_params(3, 3, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                       jitter=5.0, seed=2)
    arr = lt.tree_generate(p)
    lt.tree_place(arr, H, [128.0, 128.0, 128.0])
    return arr


def run_storage(lt, torch, arr, storage, steps, warmup, drag_every):
    stream = STREAM
    g = lt.Grid(NX, NY, NZ, u_in=U_IN, re_h=RE_H, storage=storage, drag_every=drag_every,
                stream=stream.cuda_stream)
    g.set_geometry(arr)
    if TUNE:
        g.autotune(TUNE_CACHE)  # launch shapes picked by timing candidates on this grid (state restored)
    info = g.info()
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.timing(True)
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kt = g.timing_read()
    g.timing(False)
    d = g.drag()
    cells = info["updated_cells"][0]
    g.close()
    return {"ms": ms, "cells": cells, "mlups": cells * steps / (ms * 1e-3) / 1e6, "kernel": kt,
            "links": info["links"], "cd_mean": d["cd"], "device_bytes": info["device_bytes"],
            "tune": {"occ_even": info["occ_even"], "occ_odd": info["occ_odd"], "xcd_group": info["xcd_group"]}}


def cd_after(lt, torch, arr, storage, nsteps):
    stream = STREAM
    g = lt.Grid(NX, NY, NZ, u_in=U_IN, re_h=RE_H, storage=storage, drag_every=1, stream=stream.cuda_stream)
    g.set_geometry(arr)
    g.step(nsteps)
    s = g.drag_series(1)[0]
    ax = g.info()["area_x"]
    g.close()
    return s[0] / (0.5 * U_IN ** 2 * ax)


# Three-level workload: 16^3-cell blocks, finest box 1024 x 512 x 512 (4H x 2H
# x 2H, H = 256 finest cells), coarse level 256 x 128 x 128 (1024 coarse
# blocks); order-4 seeded three-child tree (seed 3, 121 branches); finest
# blocks within 16 finest cells of a branch surface, middle blocks within 32
# cells plus a wake box one H downstream; Re_H = 2e4.  The centre of mass sits
# at (272, 245, 282), which centres the tree's extent in y and z and leaves the
# refined region one coarse block clear of the box faces (wider bands do not
# fit a 2H cross-section).
AMR = dict(nx=1024, ny=512, nz=512, H=256.0, re_h=2.0e4, com=(272.0, 245.0, 282.0),
           band=[0, 32, 16], wake=[0, 256, 0])


def amr_tree(lt):
    p = lt.tree_params(3, 4, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                       jitter=5.0, seed=3)
    arr = lt.tree_generate(p)
    lt.tree_place(arr, AMR["H"], list(AMR["com"]))
    return arr


def amr_leg(lt, torch, steps, warmup):
    """Coarse steps of the three-level grid, eager launches and graph replay
    (FP32 storage, autotuned block tiles).  MLUPS counts leaf fluid cells of
    every level times its sub-steps per coarse step (2^l)."""
    import tempfile
    stream = STREAM
    arr = amr_tree(lt)
    res = {}
    # both modes use the tiles tuned once
    cache = TUNE_CACHE or os.path.join(tempfile.mkdtemp(), "tune.txt")
    for mode, flags, storage in (("eager", 0, "fp32"), ("graph", lt.LBM_F_GRAPH, "fp32"),
                                 ("graph_fp16", lt.LBM_F_GRAPH, "fp16")):
        g = lt.Grid(AMR["nx"], AMR["ny"], AMR["nz"], u_in=U_IN, re_h=AMR["re_h"], block_edge=16, levels=3,
                    storage=storage, drag_every=1, flags=flags, stream=stream.cuda_stream)
        t0 = time.time()
        g.set_geometry(arr, refine={"band": AMR["band"], "wake": AMR["wake"]})
        setup = time.time() - t0
        if TUNE:
            g.autotune(cache)
        info = g.info()
        leaf = info["updated_cells"][:3]  # leaf fluid cells per level
        upd = sum(leaf[l] << l for l in range(3))
        work = sum(info["collided_cells"][l] << l for l in range(3))
        g.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        d = g.drag()
        bpc = 216.0 if storage == "fp32" else 108.0
        r = {"mlups": upd * steps / (ms * 1e-3) / 1e6, "ms_per_coarse_step": ms / steps,
             "step_hbm_frac": bpc * work * steps / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), "cd": d["cd"]}
        if mode == "eager":
            g.timing(True)
            g.step(steps)
            torch.cuda.synchronize()
            kt = g.timing_read()
            g.timing(False)
            r["collide_gbs"] = 216.0 * work * steps / (kt["collide_ms"] * 1e-3) / 1e9
            res["grid"] = {"blocks": info["blocks"][:3], "leaf_fluid_cells": leaf,
                           "collided_cells": info["collided_cells"][:3],
                           "updates_per_coarse_step": upd, "links": info["links"], "branches": info["branches"],
                           "device_gb": round(info["device_bytes"] / 1e9, 2), "setup_s": round(setup, 1),
                           "tile_cells": info["tile_cells"], "threads": info["threads"],
                           "tuned": {"occ_even": info["occ_even"], "occ_odd": info["occ_odd"],
                                     "xcd_group": info["xcd_group"]},
                           "effective_finest_cells": AMR["nx"] * AMR["ny"] * AMR["nz"]}
        res[mode] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
        g.close()
    res["fp16_vs_fp32_mlups"] = round(res["graph_fp16"]["mlups"] / res["graph"]["mlups"], 3)
    # the stated aim for the FP32 octree steps is 70 % of HBM peak over the step
    res["step_hbm_frac_target"] = 0.70
    res["step_hbm_frac_gap"] = round(0.70 - res["graph"]["step_hbm_frac"], 4)
    return res


# Four-level workload: 16^3-cell blocks, finest box 2048 x 1024 x 1024,
# coarse level 256 x 128 x 128; order-5 seeded three-child tree (seed 5, 364
# branches) with H = 384 finest cells; finest blocks within 12 finest cells of
# a branch surface, the next levels within 24 / 48 cells and wake boxes of 2H
# and 1H on levels 1 and 2; Re_H = 1.2e5; FP16 deviation storage; turbulent
# inflow I_u = 8 % with integral length H/2 from 200 random Fourier modes.
AMR4 = dict(nx=2048, ny=1024, nz=1024, H=384.0, re_h=1.2e5, com=(544.0, 495.5, 540.5),
            band=[0, 48, 24, 12], wake=[0, 768, 384, 0], intensity=0.08, modes=200, seed=41)


def amr4_leg(lt, torch, steps, warmup):
    """Coarse steps of the four-level FP16 grid with turbulent inflow, replayed
    from graphs with tuned tiles: MLUPS, the mean and rms fluctuation of C_D
    over the timed coarse steps, and the per-branch mean forces."""
    import tempfile
    stream = STREAM
    p = lt.tree_params(3, 5, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                       jitter=5.0, seed=5)
    arr = lt.tree_generate(p)
    lt.tree_place(arr, AMR4["H"], list(AMR4["com"]))
    g = lt.Grid(AMR4["nx"], AMR4["ny"], AMR4["nz"], u_in=U_IN, re_h=AMR4["re_h"], block_edge=16, levels=4,
                storage="fp16", drag_every=1, flags=lt.LBM_F_GRAPH, stream=stream.cuda_stream,
                turb_intensity=AMR4["intensity"], turb_length=AMR4["H"] / 2, turb_seed=AMR4["seed"],
                turb_modes=AMR4["modes"])
    t0 = time.time()
    g.set_geometry(arr, refine={"band": AMR4["band"], "wake": AMR4["wake"]})
    setup = time.time() - t0
    if TUNE:
        g.autotune(TUNE_CACHE or os.path.join(tempfile.mkdtemp(), "tune.txt"))
    info = g.info()
    leaf = info["updated_cells"][:4]
    upd = sum(leaf[l] << l for l in range(4))
    work = sum(info["collided_cells"][l] << l for l in range(4))
    g.step(warmup)
    g.drag()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = g.drag(per_branch=True)
    # C_D of every coarse step of the timed run: the mean of its 8 finest samples
    series = g.drag_series(8 * steps)[:, 0]
    cd = series.reshape(steps, 8).mean(1) / (0.5 * U_IN ** 2 * info["area_x"])
    pb = d["per_branch"][:, 0]
    gen = lt.branches_to_numpy(arr)[:, 7].astype(int)
    g.close()
    return {"workload": "4-level octree, 16^3 blocks, finest 2048x1024x1024 (coarse 256x128x128), order-5 "
                        "seeded tree H=384, Re_H=1.2e5, FP16 deviations, turbulent inflow I_u=8% (L=H/2, "
                        "200 modes), bands 12/24/48 + wakes 2H/1H",
            "coarse_steps": steps, "mlups": round(upd * steps / (ms * 1e-3) / 1e6, 1),
            "ms_per_coarse_step": round(ms / steps, 4),
            "step_hbm_frac": round(108.0 * work * steps / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "cd_mean": round(float(cd.mean()), 5), "cd_rms_fluctuation": round(float(cd.std()), 5),
            "per_branch_mean_fx": {"sum": float(pb.sum()), "by_generation": [float(pb[gen == k].sum())
                                                                            for k in range(6)],
                                   "max_branch": int(np.argmax(np.abs(pb))), "max_fx": float(pb[np.argmax(np.abs(pb))])},
            "grid": {"blocks": info["blocks"][:4], "leaf_fluid_cells": leaf,
                     "updates_per_coarse_step": upd, "links": info["links"], "branches": info["branches"],
                     "device_gb": round(info["device_bytes"] / 1e9, 2), "setup_s": round(setup, 1),
                     "tuned": {"tile_cells": info["tile_cells"], "occ_even": info["occ_even"],
                               "occ_odd": info["occ_odd"], "xcd_group": info["xcd_group"]},
                     "effective_finest_cells": AMR4["nx"] * AMR4["ny"] * AMR4["nz"]}}


# The paper's own tree in the paper's setup (Table 2, Sec. 2.3): the binary
# family with n = 4 rewrites (trunk and three child levels, 15 branches), in a
# 32H x 16H x 16H box with the tree's centre of mass at (8H, 8H, 8H), on 8^3-cell
# leaf blocks.  Four levels at H = 128 finest cells: coarse H/16 (512 x 256 x
# 256), finest H/128 (box 4096 x 2048 x 2048); finest blocks within 8 finest
# cells of the surface, the middle levels within 16 / 32 cells, and a wake box
# 4H long on level 1 (H/32), two levels coarser than the surface as in the
# paper (H/256 wake against H/1024 surface).  Re_H = 2500, the lowest of the
# paper's runs.
# The n = 4 tree of Table 2 in the paper's 32H x 16H x 16H domain on 8^3
# blocks with a dense coarse level at H/16: at H = 128 finest cells (four
# levels, wake H/32), and at the paper's surface resolution H/1024 (seven
# levels, wake at the paper's H/256 for 2H downstream).  Bands in finest cells.
PAPER = dict(n=4, H=128.0, re_h=2500.0, levels=4, band=[0, 32, 16, 8], wake=[0, 512, 0, 0], storage="fp32",
             wake_level=1)
PAPER1024 = dict(n=4, H=1024.0, re_h=2500.0, levels=7, band=[0, 512, 256, 128, 64, 32, 16],
                 wake=[0, 0, 0, 0, 2048, 0, 0], storage="fp16", wake_level=4, shapes_from="paper H/128")
# the paper's other two trees at their surface resolutions: n = 6 at H/1024,
# n = 8 at H/2048 (eight levels, coarse H/16)
PAPER1024_N6 = dict(PAPER1024, n=6)
PAPER2048_N8 = dict(n=8, H=2048.0, re_h=2500.0, levels=8, band=[0, 1024, 512, 256, 128, 64, 32, 16],
                    wake=[0, 0, 0, 0, 4096, 0, 0, 0], storage="fp16", wake_level=4, shapes_from="paper H/128")


# the n = 6 tree at H/512 (six levels, wake at H/256) for the drag split of
# the LBM against the analytic model's
PAPER512_N6 = dict(n=6, H=512.0, re_h=2500.0, levels=6, band=[0, 256, 128, 64, 32, 16],
                   wake=[0, 0, 0, 0, 1024, 0], storage="fp32", wake_level=4, shapes_from="paper H/128")


def _paper_tree(lt, cfg):
    H = cfg["H"]
    wq = 0.5 ** 0.5
    p = lt.tree_params(2, cfg["n"] - 1, 100.0, 30.0, [0.8, 0.8], [wq, wq], [0.0, 0.0], [30.0, -30.0],
                       [137.0, 137.0])
    arr = lt.tree_generate(p)
    lt.tree_place(arr, H, [8 * H, 8 * H, 8 * H])
    return arr


def _shapes_of_paper128(lt, storage):
    """Launch shapes the autotuner picks on the paper tree at H = 128 (four
    levels of 8^3 blocks, the same kernels), for grids too large to search:
    one candidate there costs milliseconds, at H/1024 seconds."""
    import tempfile
    H = PAPER["H"]
    g = lt.Grid(int(32 * H), int(16 * H), int(16 * H), u_in=U_IN, re_h=PAPER["re_h"], block_edge=8,
                levels=PAPER["levels"], storage=storage, drag_every=1, stream=STREAM.cuda_stream)
    g.set_geometry(_paper_tree(lt, PAPER), refine={"band": PAPER["band"], "wake": PAPER["wake"]})
    g.autotune(os.path.join(tempfile.mkdtemp(), "tune.txt"))
    i = g.info()
    g.close()
    return i["threads"], i["tile_cells"], i["occ_even"], i["occ_odd"], i["xcd_group"]


def paper_tree_leg(lt, torch, steps, warmup, cfg=PAPER):
    """The n = 4 tree of Table 2 in the paper's domain (cfg: PAPER at H = 128,
    PAPER1024 at the paper's H/1024): device memory, cell counts per level,
    set-up time, MLUPS and C_D (graph replay, tuned tiles)."""
    import tempfile
    stream = STREAM
    H, L = cfg["H"], cfg["levels"]
    nx, ny, nz = int(32 * H), int(16 * H), int(16 * H)
    arr = _paper_tree(lt, cfg)
    shapes = None
    if TUNE and cfg.get("shapes_from"):
        t1 = time.time()
        shapes = _shapes_of_paper128(lt, cfg["storage"])
        print(f"paper tree H/{int(H)}: launch shapes {shapes} tuned on the tree at H/128 in {time.time() - t1:.1f} s",
              file=sys.stderr, flush=True)
    g = lt.Grid(nx, ny, nz, u_in=U_IN, re_h=cfg["re_h"], block_edge=8, levels=L, storage=cfg["storage"],
                drag_every=1, flags=lt.LBM_F_GRAPH, stream=stream.cuda_stream)
    t0 = time.time()
    g.set_geometry(arr, refine={"band": cfg["band"], "wake": cfg["wake"]})
    setup = time.time() - t0
    print(f"paper tree H/{int(H)}: geometry and {L}-level grid set up in {setup:.1f} s", file=sys.stderr, flush=True)
    if shapes is not None:
        # applied through a one-entry tune cache keyed as the library keys it
        path = os.path.join(tempfile.mkdtemp(), "tune.txt")
        key = f"nx{nx}_ny{ny}_nz{nz}_B8_L{L}_S{lt.STORAGE[cfg['storage']]}_links{g.info()['links']}"
        with open(path, "w") as f:
            f.write(key + " " + " ".join(str(int(v)) for v in shapes) + "\n")
        g.autotune(path)
    elif TUNE:
        t1 = time.time()
        g.autotune(TUNE_CACHE or os.path.join(tempfile.mkdtemp(), "tune.txt"))
        print(f"paper tree H/{int(H)}: launch shapes tuned in {time.time() - t1:.1f} s", file=sys.stderr, flush=True)
    info = g.info()
    if shapes is not None:
        assert (info["threads"], info["tile_cells"]) == tuple(shapes[:2])
    leaf = info["updated_cells"][:L]
    upd = sum(leaf[l] << l for l in range(L))
    work = sum(info["collided_cells"][l] << l for l in range(L))
    g.step(warmup)
    g.drag()
    torch.cuda.synchronize()
    print(f"paper tree H/{int(H)}: {warmup} warm-up coarse steps done", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(f"paper tree H/{int(H)}: {steps} timed coarse steps in {ms:.1f} ms", file=sys.stderr, flush=True)
    d = g.drag()
    g.close()
    b = lt.branches_to_numpy(arr)
    bpc = 216.0 if cfg["storage"] == "fp32" else 108.0
    wake_dx = int(H) >> (L - 1 - cfg["wake_level"])
    return {"workload": f"paper binary tree n={cfg['n']} (Table 2), domain 32Hx16Hx16H = {nx}x{ny}x{nz} finest cells, "
                        f"COM (8H,8H,8H), 8^3 blocks, {L} levels H/16..H/{int(H)}, wake H/{wake_dx}, "
                        f"Re_H={cfg['re_h']:g}, {cfg['storage'].upper()}",
            "coarse_steps": steps, "finest_steps_per_coarse_step": 1 << (L - 1),
            "mlups": round(upd * steps / (ms * 1e-3) / 1e6, 1), "ms_per_coarse_step": round(ms / steps, 4),
            "step_hbm_frac": round(bpc * work * steps / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "cd": round(d["cd"], 5), "d0_over_h": round(b[0, 6] / info["height"], 4),
            "launch_shapes": {"threads": info["threads"], "tile": info["tile_cells"], "occ_even": info["occ_even"],
                              "occ_odd": info["occ_odd"], "xcd_group": info["xcd_group"],
                              "tuned_on": cfg.get("shapes_from") or "this grid"},
            "grid": {"blocks": info["blocks"][:L], "leaf_fluid_cells": leaf, "updates_per_coarse_step": upd,
                     "total_leaf_cells": int(sum(info["active_cells"][:L])), "links": info["links"],
                     "device_gb": round(info["device_bytes"] / 1e9, 2), "setup_s": round(setup, 1),
                     "finest_dx_over_h": round(1.0 / H, 5)}}


def paper_split_leg(lt, torch, cfg=PAPER512_N6, warm_flow_times=3.0, mean_flow_times=3.0):
    """Drag split of one of the paper's trees (cfg: n = 6 at H/512, or at the
    paper's H/1024 with paper_split1024), LBM against the analytic model
    (Sec. 2.4 Eqs. (2)-(6), Sec. 3 Eqs. (7)-(9)): C_D, C_F and C_P = C_D - C_F
    of the LBM, averaged over mean_flow_times flow times H/U after
    warm_flow_times, and C_D-est, C_F-est, C_P-est of the same tree at the same
    Re_H (synthetic cylinder C_d curve, the C_f table from LBM runs of single
    cylinders), both normalised by the LBM's voxel frontal area."""
    import tempfile
    from paper_2603_27954_amd.cylinder import load_cf_table
    stream = STREAM
    H, L = cfg["H"], cfg["levels"]
    nx, ny, nz = int(32 * H), int(16 * H), int(16 * H)
    arr = _paper_tree(lt, cfg)
    t0 = time.time()
    shapes = _shapes_of_paper128(lt, cfg["storage"]) if TUNE else None
    print(f"paper split n={cfg['n']} H/{int(H)}: launch shapes {shapes} tuned on the tree at H/128 in "
          f"{time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    coarse = 1 << (L - 1)
    g = lt.Grid(nx, ny, nz, u_in=U_IN, re_h=cfg["re_h"], block_edge=8, levels=L, storage=cfg["storage"],
                drag_every=coarse, flags=lt.LBM_F_GRAPH | lt.LBM_F_FRICTION, stream=stream.cuda_stream)
    t0 = time.time()
    g.set_geometry(arr, refine={"band": cfg["band"], "wake": cfg["wake"]})
    print(f"paper split n={cfg['n']} H/{int(H)}: {L}-level grid set up in {time.time() - t0:.1f} s", file=sys.stderr,
          flush=True)
    if shapes is not None:
        path = os.path.join(tempfile.mkdtemp(), "tune.txt")
        key = f"nx{nx}_ny{ny}_nz{nz}_B8_L{L}_S{lt.STORAGE[cfg['storage']]}_links{g.info()['links']}"
        with open(path, "w") as f:
            f.write(key + " " + " ".join(str(int(v)) for v in shapes) + "\n")
        g.autotune(path)
    info = g.info()
    per_flow_time = max(1, int(round(H / U_IN / coarse)))  # coarse steps per H/U
    t0 = time.time()
    for k in range(int(warm_flow_times)):
        g.step(per_flow_time)
        d = g.drag()
        print(f"  warm-up flow time {k + 1}: C_D {d['cd']:.4f} C_F {d['cf']:.4f} ({time.time() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    acc = {"cd": 0.0, "cf": 0.0}
    n_mean = int(mean_flow_times)
    for k in range(n_mean):
        g.step(per_flow_time)
        d = g.drag()
        acc["cd"] += d["cd"] / n_mean
        acc["cf"] += d["cf"] / n_mean
        print(f"  averaged flow time {k + 1}: C_D {d['cd']:.4f} C_F {d['cf']:.4f} ({time.time() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    area_lbm = d["area_x"]
    height = d["height"]
    g.close()
    # the analytic model on the same tree at unit height
    wq = 0.5 ** 0.5
    p = lt.tree_params(2, cfg["n"] - 1, 100.0, 30.0, [0.8, 0.8], [wq, wq], [0.0, 0.0], [30.0, -30.0],
                       [137.0, 137.0])
    rec, start = lt.tree_batch(p, 0, [cfg["n"] - 1])
    rd, sd = torch.from_numpy(rec).cuda(), torch.from_numpy(start).cuda()
    area_raster = torch.empty(1, dtype=torch.float32, device="cuda")
    lt.frontal_area(rd, sd, 1.0 / 256, area_raster, stream.cuda_stream)
    area = torch.full((1,), area_lbm / height ** 2, dtype=torch.float32, device="cuda")
    cd, cf, cp = (torch.empty((1, 1), dtype=torch.float32, device="cuda") for _ in range(3))
    lt.analytic_split(rd, sd, area, cd, cf, [cfg["re_h"]], load_cf_table(), 0.0, cp, stream.cuda_stream)
    est = {"cd": float(cd.cpu()[0, 0]), "cf": float(cf.cpu()[0, 0]), "cp": float(cp.cpu()[0, 0])}
    lbm = {"cd": acc["cd"], "cf": acc["cf"], "cp": acc["cd"] - acc["cf"]}
    return {"workload": f"paper binary tree n={cfg['n']} (Table 2), domain 32Hx16Hx16H = {nx}x{ny}x{nz} finest "
                        f"cells, {L} levels H/16..H/{int(H)}, wake H/256, Re_H={cfg['re_h']:g}, "
                        f"{cfg['storage'].upper()}; means over {n_mean} flow times H/U after {int(warm_flow_times)}",
            "lbm": {k: round(v, 4) for k, v in lbm.items()},
            "analytic": {k: round(v, 4) for k, v in est.items()},
            "analytic_over_lbm": {k: round(est[k] / lbm[k], 3) for k in lbm},
            "area_x_over_h2": {"voxels": round(area_lbm / height ** 2, 5),
                               "raster_h_over_256": round(float(area_raster.cpu()[0]), 5)},
            "links": info["links"], "device_gb": round(info["device_bytes"] / 1e9, 2),
            "coarse_steps": per_flow_time * (int(warm_flow_times) + n_mean)}


MFMA_BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP = 8960  # 2 x (5 x 64 + 64 x 64 + 64) per inference


# Training sweeps of the surrogate.  "small": orders 1-3 at Re_H 100-800 (224
# runs, about a minute: the default bench leg).  "large": orders 1-4 at Re_H
# 100 to 2e4 (the seeded workloads' Reynolds numbers, 2500 and 2e4 included),
# about 1e5 per-branch samples from 3220 runs.  Both: I_u 0 and 8 %, trees of
# height 32 in a 128 x 64 x 64 box, held-out seeds disjoint from training.
SURROGATE_SWEEPS = {
    "small": dict(re_h=(100.0, 200.0, 400.0, 800.0),
                  train={1: range(1000, 1016), 2: range(1100, 1108), 3: range(1200, 1204)},
                  held={1: range(1057, 1060), 2: range(1127, 1130), 3: range(1212, 1215)},
                  fit=dict(epochs=40, batch=256, lr=2e-3)),
    "large": dict(re_h=(100.0, 300.0, 1000.0, 2500.0, 5000.0, 1.0e4, 2.0e4),
                  train={1: range(2000, 2100), 2: range(3000, 3060), 3: range(4000, 4040), 4: range(5000, 5030)},
                  held={1: range(9000, 9003), 2: range(9100, 9103), 3: range(9200, 9203), 4: range(9300, 9303)},
                  fit=dict(epochs=320, batch=256, lr=2e-3)),
}


def surrogate_leg(lt, torch, n_trees, chunk=1 << 17, scale="small"):
    """Learned per-branch drag surrogate: trained on per-branch forces from LBM
    runs of seeded trees (SURROGATE_SWEEPS[scale]: orders, Re_H, I_u 0 and
    8 %), checked on held-out seeds (mean and maximum tree-C_D error), then
    swept over n_trees seeded trees (orders 1-6 in turn) at 25 Re_H from 1e3 to
    1e9 on the matrix cores, with the analytic model (Eqs. (2), (4)) on the
    same trees."""
    from paper_2603_27954_amd import surrogate as S
    stream = STREAM
    t0 = time.time()
    sw = SURROGATE_SWEEPS[scale]
    fit = dict(sw["fit"], **SURROGATE_TRAIN)

    unstable = []

    def runs(seeds_by_order):
        out = []
        for order, seeds in seeds_by_order.items():
            for re_h in sw["re_h"]:
                for iu in (0.0, 0.08):
                    for seed in seeds:
                        try:
                            r = S.lbm_samples(order, seed, re_h, iu, stream=stream.cuda_stream)
                        except lt.LbmError as e:  # a run that went unstable gives no samples
                            if e.status != lt.LBM_E_UNSTABLE:
                                raise
                            unstable.append((order, seed, re_h, iu))
                            continue
                        r.update(order=order, re_h=re_h, iu=iu, seed=seed)
                        out.append(r)
                        if len(out) % 200 == 0:
                            print(f"surrogate: {len(out)} LBM runs ({time.time() - t0:.0f} s)", file=sys.stderr,
                                  flush=True)
        return out

    train = runs(sw["train"])
    held = runs(sw["held"])
    if SURROGATE_DUMP:
        # the training samples and the held-out runs, for studies of the
        # training settings without repeating the LBM runs
        hs = np.cumsum([0] + [len(r["feat"]) for r in held])
        np.savez(SURROGATE_DUMP, X=np.concatenate([r["feat"] for r in train]),
                 Y=np.concatenate([r["y"] for r in train]),
                 h_feat=np.concatenate([r["feat"] for r in held]), h_ld=np.concatenate([r["ld"] for r in held]),
                 h_start=hs, h_area=np.array([r["area_x"] for r in held]), h_cd=np.array([r["cd"] for r in held]),
                 h_re=np.array([r["re_h"] for r in held]), h_iu=np.array([r["iu"] for r in held]),
                 h_order=np.array([r["order"] for r in held]))
    lbm_s = time.time() - t0
    X = np.concatenate([r["feat"] for r in train])
    Y = np.concatenate([r["y"] for r in train])
    m = lt.Mlp(seed=3, stream=stream.cuda_stream)
    m.set_scaling(X.mean(0), np.maximum(X.std(0), 1e-3), Y.mean(), Y.std())
    t1 = time.time()
    losses = m.train(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), epochs=fit["epochs"],
                     batch=fit["batch"], lr=fit["lr"], seed=17)
    train_s = time.time() - t1
    err = np.array([abs(S.tree_cd(m, r["feat"], r["ld"], r["area_x"]) - r["cd"]) / r["cd"] for r in held])
    # the analytic model of Eqs. (2), (4) on the same held-out runs (the
    # method without the learned part), on the GPU: the run's tree as a unit-
    # height branch batch, its voxel frontal area over H^2
    params = lt.tree_params(3, 1, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                            jitter=5.0, seed=0)
    err_a = []
    for r in held:
        rec, start = lt.tree_batch(params, r["seed"], [r["order"]])
        rd, sd = torch.from_numpy(rec).cuda(), torch.from_numpy(start).cuda()
        area = torch.tensor([r["area_x"] / 32.0 ** 2], dtype=torch.float32, device="cuda")
        cda = torch.empty((1, 1), dtype=torch.float32, device="cuda")
        lt.analytic_sweep(rd, sd, area, cda, [r["re_h"]], r["iu"], stream.cuda_stream)
        torch.cuda.synchronize()
        err_a.append(abs(float(cda.cpu()[0, 0]) - r["cd"]) / r["cd"])
    err_a = np.array(err_a)
    by_re = {f"{re:g}": round(float(np.mean([e for e, r in zip(err, held) if r["re_h"] == re])), 4)
             for re in sw["re_h"]}
    re_d = 10.0 ** X[:, 0]
    env = (float(re_d.min()), float(re_d.max()))
    sweep = sweep_trees(lt, torch, m, env, n_trees, chunk)
    m.close()
    return {
        "training": {"lbm_runs": len(train), "samples": int(len(X)), "lbm_seconds": round(lbm_s, 1),
                     "epochs": fit["epochs"], "batch": fit["batch"],
                     "lr": fit["lr"], "train_seconds": round(train_s, 2), "final_loss": float(losses[-1]),
                     "re_d_envelope": [round(env[0], 2), round(env[1], 1)]},
        "held_out": {"runs": len(held), "cd_rel_err_mean": round(float(np.mean(err)), 4),
                     "cd_rel_err_max": round(float(np.max(err)), 4),
                     "cd_rel_err_p90": round(float(np.quantile(err, 0.9)), 4),
                     "analytic_cd_rel_err_mean": round(float(np.mean(err_a)), 4),
                     "mean_err_by_re_h": by_re},
        "scale": scale, "unstable_runs": len(unstable),
        "sweep": sweep,
    }


def sweep_trees(lt, torch, m, env, n_trees, chunk=1 << 17):
    """n_trees seeded trees (orders 1-6 in turn) at 25 Re_H from 1e3 to 1e9:
    frontal areas, the network m on the matrix cores (training envelope env
    of Re_D) and the analytic model, timed per kernel on the bench stream."""
    stream = STREAM
    params = lt.tree_params(3, 1, 1.0, 0.3, [0.7] * 3, [0.7] * 3, [0.0, 120.0, 240.0], [35.0] * 3, [90.0] * 3,
                            jitter=5.0, seed=0)
    re_h = 10.0 ** np.linspace(3.0, 9.0, 25)
    orders = 1 + (np.arange(n_trees) % 6)
    from paper_2603_27954_amd.cylinder import load_cf_table
    cf_table = load_cf_table()
    sweep_ms = analytic_ms = split_ms = area_ms = gen_s = 0.0
    n_branch = 0
    sum_s = np.zeros(len(re_h))
    sum_a = np.zeros(len(re_h))
    sum_f = np.zeros(len(re_h))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for c0 in range(0, n_trees, chunk):
        o = orders[c0:c0 + chunk]
        tg = time.time()
        rec, start = lt.tree_batch(params, 1 + c0, o)
        gen_s += time.time() - tg
        rd, sd = torch.from_numpy(rec).cuda(), torch.from_numpy(start).cuda()
        area = torch.empty(len(o), dtype=torch.float32, device="cuda")
        cd = torch.empty((len(o), len(re_h)), dtype=torch.float32, device="cuda")
        cda = torch.empty_like(cd)
        torch.cuda.synchronize()
        e0.record(stream)
        lt.frontal_area(rd, sd, 1.0 / 256, area, stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        area_ms += e0.elapsed_time(e1)
        e0.record(stream)
        m.sweep(rd, sd, area, cd, re_h, 0.0, env)
        e1.record(stream)
        e1.synchronize()
        sweep_ms += e0.elapsed_time(e1)
        e0.record(stream)
        lt.analytic_sweep(rd, sd, area, cda, re_h, 0.0, stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        analytic_ms += e0.elapsed_time(e1)
        # the friction split of Eqs. (3), (5), (6) with the LBM C_f table
        cdf, cff, cpf = torch.empty_like(cd), torch.empty_like(cd), torch.empty_like(cd)
        e0.record(stream)
        lt.analytic_split(rd, sd, area, cdf, cff, re_h, cf_table, 0.0, cpf, stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        split_ms += e0.elapsed_time(e1)
        n_branch += len(rec)
        sum_s += cd.double().sum(0).cpu().numpy()
        sum_a += cda.double().sum(0).cpu().numpy()
        sum_f += cff.double().sum(0).cpu().numpy()
        del rd, sd, area, cd, cda, cdf, cff, cpf
    inferences = n_branch * len(re_h)
    tflops = MLP_FLOP * inferences / (sweep_ms * 1e-3) / 1e12
    return {"trees": n_trees, "branches": n_branch, "re_h": [1e3, 1e9, len(re_h)], "inferences": inferences,
            "surrogate_ms": round(sweep_ms, 2), "inferences_per_s": round(inferences / (sweep_ms * 1e-3), 1),
            "analytic_ms": round(analytic_ms, 2), "analytic_split_ms": round(split_ms, 2),
            "frontal_area_ms": round(area_ms, 2),
            "host_tree_generation_s": round(gen_s, 2),
            "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": MFMA_BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4),
                         "flop_per_inference": MLP_FLOP, "dtype": "bf16 operands, fp32 accumulate"},
            "mean_cd_surrogate": [round(v / n_trees, 4) for v in sum_s],
            "mean_cd_analytic": [round(v / n_trees, 4) for v in sum_a],
            "mean_cf_analytic": [round(v / n_trees, 5) for v in sum_f]}


def sweep_only_leg(lt, torch, n_trees):
    """The many-tree sweep alone, with an untrained network (seeded weights,
    fixed feature scaling): the same kernels and work as in the surrogate leg,
    without the LBM training runs (for profiling)."""
    m = lt.Mlp(seed=3, stream=STREAM.cuda_stream)
    m.set_scaling(np.array([2.0, 45.0, 2.0, 0.04, 0.5]), np.array([0.5, 30.0, 1.5, 0.04, 0.3]), 1.1, 0.7)
    out = sweep_trees(lt, torch, m, (4.32, 152.3), n_trees)
    m.close()
    return out


GOLDEN_SERIES = os.path.join(ROOT, "tests", "golden", "cd_series_uniform512x256x256.txt")


def cd_series_error(lt, torch, arr):
    """C_D of every step of the first 1000 against the FP64 oracle's series of
    the same workload (stored by tests/golden/make_cd_series.py): the largest
    difference over the mean |C_D| and the relative error of the mean C_D over
    steps 501-1000, FP32 and FP16 storage.  None when the series is absent."""
    if not os.path.exists(GOLDEN_SERIES):
        return None
    ref = np.loadtxt(GOLDEN_SERIES, comments="#")[:, 1]
    out = {"oracle_mean_cd_501_1000": round(float(ref[500:].mean()), 6)}
    for storage in ("fp32", "fp16"):
        g = lt.Grid(NX, NY, NZ, u_in=U_IN, re_h=RE_H, storage=storage, drag_every=1, stream=STREAM.cuda_stream)
        g.set_geometry(arr)
        g.step(len(ref))
        f = g.drag_series(len(ref))
        ax = g.info()["area_x"]
        g.close()
        cd = f[:, 0] / (0.5 * U_IN ** 2 * ax)
        out[storage] = {"max_dev_over_mean_abs_cd": float(np.abs(cd - ref).max() / np.abs(ref).mean()),
                        "mean_cd_501_1000_rel": float(abs(cd[500:].mean() - ref[500:].mean()) / abs(ref[500:].mean()))}
    return out


def cpu_leg(lt, arr, nsteps):
    import oracle as O
    b = lt.branches_to_numpy(arr)
    t0 = time.time()
    solid = O.voxelize(b, NX, NY, NZ)
    lk = O.links(b, solid, NX, NY, NZ)
    ax = O.area_x(solid, NX, NY, NZ)
    setup = time.time() - t0
    nu = U_IN * O.tree_height(b) / RE_H
    sim = O.UniformSim(NX, NY, NZ, O.omega_from_nu(nu), u_in=U_IN, solid=solid, link=lk, n_branch=len(b))
    t0 = time.time()
    sim.step(nsteps)
    dt = time.time() - t0
    fluid = int((solid == 0).sum())
    cd = sim.last_force[0] / (0.5 * U_IN ** 2 * ax)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    del sim
    # the small 64 x 32 x 32 workload (order-1 tree, Re_H = 100), 100 steps, on
    # one thread and on all of them
    b1 = O.build_tree(O.cfg1_tree_params(), 0.0, [16.0, 16.0, 16.0])
    s1 = O.voxelize(b1, 64, 32, 32)
    l1 = O.links(b1, s1, 64, 32, 32)
    nu1 = U_IN * O.tree_height(b1) / 100.0
    small = {}
    for threads in (1, cores):
        O.set_threads(threads)
        sim1 = O.UniformSim(64, 32, 32, O.omega_from_nu(nu1), u_in=U_IN, solid=s1, link=l1, n_branch=len(b1))
        t1 = time.time()
        sim1.step(100)
        small[threads] = int((s1 == 0).sum()) * 100 / (time.time() - t1) / 1e6
    O.set_threads(cores)
    return {"mlups": fluid * nsteps / dt / 1e6, "seconds": dt, "setup_s": setup, "cores": cores, "cd": cd,
            "small_mlups_1_thread": small[1], "small_mlups_all": small[cores]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--drag-every", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--storage", choices=["both", "fp32", "fp16"], default="both")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="file that keeps the tuned launch shapes; a later run with the same file reuses them")
    ap.add_argument("--no-amr", action="store_true", help="skip the three-level AMR leg")
    ap.add_argument("--amr-steps", type=int, default=40)
    ap.add_argument("--amr-only", action="store_true", help="run only the three-level AMR leg (profiling)")
    ap.add_argument("--amr4-steps", type=int, default=16, help="timed coarse steps of the four-level leg")
    ap.add_argument("--paper-steps", type=int, default=16, help="timed coarse steps of the paper-tree leg")
    ap.add_argument("--paper1024-steps", type=int, default=4,
                    help="timed coarse steps (64 finest steps each) of the paper-tree leg at H/1024 (--legs paper1024)")
    ap.add_argument("--legs", default=None,
                    help="comma list of legs to run alone and print (amr3, amr4, paper, paper1024, paper1024n6, "
                         "paper2048n8, paper_split, paper_split_re, paper_split1024, paper_split1024n4, "
                         "paper_split1024n8)")
    ap.add_argument("--split-mean-flow-times", type=float, default=3.0,
                    help="flow times H/U averaged by the paper_split1024n8 leg (after two of warm-up)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the drag-surrogate leg")
    ap.add_argument("--surrogate-trees", type=int, default=1_000_000)
    ap.add_argument("--surrogate-scale", choices=list(SURROGATE_SWEEPS), default="small",
                    help="training sweep of the surrogate (large: about 1e5 samples, several minutes)")
    ap.add_argument("--surrogate-dump", default=None, help=".npz file for the surrogate's samples and held-out runs")
    ap.add_argument("--surrogate-epochs", type=int, default=None, help="training epochs (default: the scale's)")
    ap.add_argument("--surrogate-batch", type=int, default=None, help="training batch (default: the scale's)")
    ap.add_argument("--surrogate-lr", type=float, default=None, help="Adam rate (default: the scale's)")
    ap.add_argument("--surrogate-only", action="store_true", help="run only the drag-surrogate leg (profiling)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the many-tree sweep with an untrained network (profiling its kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 512 MiB device copy (torch) as the reference dispatch "
                         "for the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the sharding design is documented, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_27954_amd as lt

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    global STREAM
    # a stream of our own (default priority): the library enqueues on it and
    # the timing events are recorded on it
    STREAM = torch.cuda.Stream()
    if args.copy_calibration:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    global TUNE, TUNE_CACHE, SURROGATE_DUMP
    TUNE = not args.no_tune
    TUNE_CACHE = args.tune_cache
    SURROGATE_DUMP = args.surrogate_dump
    SURROGATE_TRAIN.update({k: v for k, v in (("epochs", args.surrogate_epochs), ("batch", args.surrogate_batch),
                                              ("lr", args.surrogate_lr)) if v is not None})
    if args.amr_only:
        print(json.dumps({"amr_3level": amr_leg(lt, torch, args.amr_steps, 4)}), flush=True)
        return
    if args.legs:
        legs = {"amr3": lambda: amr_leg(lt, torch, args.amr_steps, 4),
                "amr4": lambda: amr4_leg(lt, torch, args.amr4_steps, 2),
                "paper": lambda: paper_tree_leg(lt, torch, args.paper_steps, 2),
                "paper1024": lambda: paper_tree_leg(lt, torch, args.paper1024_steps, 1, PAPER1024),
                "paper1024n6": lambda: paper_tree_leg(lt, torch, args.paper1024_steps, 1, PAPER1024_N6),
                "paper2048n8": lambda: paper_tree_leg(lt, torch, max(1, args.paper1024_steps // 2), 1, PAPER2048_N8),
                "paper_split": lambda: paper_split_leg(lt, torch),
                "paper_split1024": lambda: paper_split_leg(lt, torch, dict(PAPER1024_N6, storage="fp32"), 2.0, 3.0),
                "paper_split_re": lambda: {f"re_h_{r:g}": paper_split_leg(lt, torch, dict(PAPER512_N6, re_h=r))
                                           for r in (2.0e4, 6.0e4, 1.2e5)},
                "paper_split1024n4": lambda: paper_split_leg(lt, torch, dict(PAPER1024, storage="fp32"), 2.0, 3.0),
                "paper_split1024n8": lambda: paper_split_leg(lt, torch, dict(PAPER1024, n=8, storage="fp32"), 2.0,
                                                             args.split_mean_flow_times)}
        print(json.dumps({k: legs[k]() for k in args.legs.split(",")}), flush=True)
        return
    if args.sweep_only:
        print(json.dumps({"sweep": sweep_only_leg(lt, torch, args.surrogate_trees)}), flush=True)
        return
    if args.surrogate_only:
        print(json.dumps({"surrogate": surrogate_leg(lt, torch, args.surrogate_trees, scale=args.surrogate_scale)}),
              flush=True)
        return
    arr = build_tree(lt)
    r32 = r16 = None
    if args.storage in ("both", "fp32"):
        r32 = run_storage(lt, torch, arr, "fp32", args.steps, args.warmup, args.drag_every)
    if args.storage in ("both", "fp16"):
        r16 = run_storage(lt, torch, arr, "fp16", args.steps, args.warmup, args.drag_every)
    if r32 is None:
        r32 = r16

    def roof(r, bytes_per_cell):
        kt = r["kernel"]
        avg_ms = kt["collide_ms"] / max(kt["collide_launches"], 1)
        achieved = bytes_per_cell * r["cells"] / (avg_ms * 1e-3) / 1e9
        # HBM bytes per launch from the committed counter summary of this
        # storage (null when the kernel sources changed since it was taken)
        st = "fp32" if bytes_per_cell == 216 else "fp16"
        tr = measured_traffic(st)
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
               "kernel": "k_collide_dense (even + odd launches)", "avg_launch_ms": round(avg_ms, 5),
               "bytes_per_cell": bytes_per_cell, "tuned": r["tune"]}
        if tr is not None:
            out["traffic_vs_algorithmic"] = round(tr / (bytes_per_cell * r["cells"]), 4)
            out["traffic_source"] = TRAFFIC_FILES[st]
        return out

    out = {
        "metric": "MLUPS & % HBM peak, D3Q27 cumulant FP32 vs FP16-store; C_d err vs FP64 oracle",
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uniform 512x256x256, order-3 seeded 3-child tree H=128, Re_H=2500, u=0.05",
                   "cells": NX * NY * NZ, "fluid_cells": r32["cells"], "links": r32["links"],
                   "storage": "fp32 deviations", "drag_every": args.drag_every},
        "roofline": roof(r32, 216 if args.storage != "fp16" else 108),
    }
    if args.storage == "both":
        out["fp16_storage"] = {"value": round(r16["mlups"], 1), "unit": "MLUPS",
                               "ratio_vs_fp32": round(r16["mlups"] / r32["mlups"], 3),
                               "ms_per_step": round(r16["ms"] / args.steps, 4), "roofline": roof(r16, 108)}
    if not args.no_cpu and args.storage == "both":
        c = cpu_leg(lt, arr, args.cpu_steps)
        cd32 = cd_after(lt, torch, arr, "fp32", args.cpu_steps)
        cd16 = cd_after(lt, torch, arr, "fp16", args.cpu_steps)
        out["cpu_baseline"] = {"value": round(c["mlups"], 2), "unit": "MLUPS", "cores": c["cores"],
                               "kind": "oracle",
                               "sample": f"full 512x256x256 workload, {args.cpu_steps} FP64 steps "
                                         f"({c['seconds']:.1f} s; geometry setup {c['setup_s']:.1f} s untimed)",
                               "small_64x32x32_100_steps": {"mlups_1_thread": round(c["small_mlups_1_thread"], 2),
                                                            f"mlups_{c['cores']}_threads":
                                                                round(c["small_mlups_all"], 2)}}
        out["cd_error"] = {"steps": args.cpu_steps, "cd_oracle": c["cd"],
                           "fp32_rel": abs(cd32 - c["cd"]) / abs(c["cd"]),
                           "fp16_rel": abs(cd16 - c["cd"]) / abs(c["cd"])}
        series = cd_series_error(lt, torch, arr)
        if series is not None:
            out["cd_error"]["series_1000_steps"] = series
    if not args.no_amr:
        a = amr_leg(lt, torch, args.amr_steps, 4)
        a["workload"] = ("3-level octree, 16^3 blocks, finest 1024x512x512 (coarse 256x128x128), order-4 "
                         "seeded tree H=256, Re_H=2e4, FP32, bands 16/32 + 1H wake")
        a["coarse_steps"] = args.amr_steps
        out["amr_3level"] = a
    if not args.no_amr:
        out["amr_4level_fp16_turbulent"] = amr4_leg(lt, torch, args.amr4_steps, 2)
        out["paper_tree_n4"] = paper_tree_leg(lt, torch, args.paper_steps, 2)
        out["paper_tree_n4_h1024"] = paper_tree_leg(lt, torch, args.paper1024_steps, 1, PAPER1024)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(lt, torch, args.surrogate_trees, scale=args.surrogate_scale)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
