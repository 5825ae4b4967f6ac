"""GPU runs of octree grids deeper than the oracle can hold in memory (five
and seven levels of 8^3 blocks in the paper's 32H x 16H x 16H domain, Sec.
2.2-2.3).  The body is one branch thinner than a cell: the refinement rule
builds the full level hierarchy around it, but no cell centre lies inside it,
so the grid has no solid cell and no link.  A uniform inflow is then an exact
steady state of every level and of every coarse/fine transfer: it stays
uniform to FP32 rounding at every level; eager and graph-replayed coarse steps
agree bit for bit; the mass stays put.  The block maps of such grids are
compared with the oracle's bit for bit on the host (test_capi_host.py)."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
U = 0.05

DEEP = {
    "five_level_H64": dict(L=5, H=64.0, band=[0, 64, 32, 16, 8], wake=[0, 0, 128, 0, 0]),
    "seven_level_H256": dict(L=7, H=256.0, band=[0, 256, 128, 64, 32, 16, 8], wake=[0, 0, 0, 0, 512, 0, 0]),
}


def _grid(gpu, c, storage="fp32", flags=0):
    H, L = c["H"], c["L"]
    # a vertical branch on a cell corner line: 0.7 cells from the nearest
    # cell centre, diameter 0.1
    b = np.array([[8 * H, 8 * H, 7.5 * H, 8 * H, 8 * H, 8.5 * H, 0.1, 0, -1, 0]])
    g = gpu.Grid(int(32 * H), int(16 * H), int(16 * H), u_in=U, re_h=2500.0, block_edge=8, levels=L,
                 storage=storage, drag_every=1, flags=flags)
    g.set_geometry(b, refine={"band": c["band"], "wake": c["wake"]})
    return g


def _sample(g, L, per_level=4096, seed=5):
    """Cells (indices over each level's box) of leaf blocks, sampled per level."""
    rng = np.random.default_rng(seed)
    B = 8
    out = []
    for l in range(L):
        nx, ny, nz = g.level_shape(l)
        m = g.block_map(l)
        leaf = np.flatnonzero(m == 1)
        assert len(leaf) > 0, f"level {l} has leaf blocks"
        bx, by, bz = leaf % (nx // B), (leaf // (nx // B)) % (ny // B), leaf // ((nx // B) * (ny // B))
        pick = rng.integers(0, len(leaf), per_level)
        c = rng.integers(0, B, (per_level, 3))
        x, y, z = bx[pick] * B + c[:, 0], by[pick] * B + c[:, 1], bz[pick] * B + c[:, 2]
        out.append(np.unique(x + nx * (y + ny * z.astype(np.int64))))
    return out


@pytest.mark.parametrize("name", list(DEEP))
def test_uniform_inflow_stays_uniform_through_every_level(gpu, name):
    c = DEEP[name]
    L = c["L"]
    print(f"[deep uniform] {name}", flush=True)
    g = _grid(gpu, c)
    info = g.info()
    assert info["links"] == 0
    print(f"  leaf cells per level {info['updated_cells'][:L]}", flush=True)
    cells = _sample(g, L)
    feq = O.equilibrium(1.0, [U, 0.0, 0.0])
    m0 = g.mass()
    g.step(2)
    for l in range(L):
        f = g.get_cells(cells[l], l)
        err = np.abs(f - feq[:, None]).max()
        print(f"  level {l}: {len(cells[l])} cells, max |f - f_eq(1, U)| = {err:.2e}", flush=True)
        assert np.isfinite(err) and err < 2e-6
    m1 = g.mass()
    assert abs(m1 - m0) < 1e-6 * m0


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_graph_replay_is_bitwise_eager_at_five_levels(gpu, storage):
    c = DEEP["five_level_H64"]
    L = c["L"]
    print(f"[deep graph] five_level_H64 {storage}", flush=True)
    ge = _grid(gpu, c, storage)
    gg = _grid(gpu, c, storage, gpu.LBM_F_GRAPH)
    cells = _sample(ge, L, per_level=2048, seed=9)
    for n in (1, 2):
        ge.step(n)
        gg.step(n)
        for l in range(L):
            a, b = ge.get_cells(cells[l], l), gg.get_cells(cells[l], l)
            assert np.array_equal(a, b), f"level {l} after a block of {n} coarse steps"
