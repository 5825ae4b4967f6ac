"""Checkpoints and instability reporting through the C-ABI: a run saved and
reloaded into a fresh grid continues bit for bit like the run that was never
interrupted (populations, force series, mean force), and a state holding a NaN
or a density outside [0.5, 1.5] is reported as LBM_E_UNSTABLE."""
import os
import tempfile

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
U = 0.05

CASES = {
    "uniform_fp32": dict(box=(64, 32, 32), com=(16.0, 16.0, 16.0), L=1, B=16, storage="fp32", refine=None),
    "uniform_fp16": dict(box=(64, 32, 32), com=(16.0, 16.0, 16.0), L=1, B=16, storage="fp16", refine=None),
    "two_level_fp32": dict(box=(96, 96, 96), com=(40.0, 48.0, 48.0), L=2, B=8, storage="fp32",
                           refine={"band": [0, 8], "wake": [0, 0]}),
}


def _grid(gpu, c, tree):
    g = gpu.Grid(*c["box"], u_in=U, re_h=100.0, block_edge=c["B"], levels=c["L"], storage=c["storage"],
                 drag_every=1)
    g.set_geometry(tree, refine=c["refine"])
    return g


@pytest.mark.parametrize("name", list(CASES))
def test_checkpoint_resumes_bit_for_bit(gpu, name):
    print(f"[checkpoint] {name}", flush=True)
    c = CASES[name]
    tree = O.build_tree(O.cfg1_tree_params(), 0.0, list(c["com"]))
    n = 6  # coarse steps before and after the checkpoint (even: every level at an even step)
    ref = _grid(gpu, c, tree)
    ref.step(2 * n)
    want_f = [ref.get_populations(l) for l in range(c["L"])]
    want_series = ref.drag_series()
    want_drag = ref.drag(per_branch=True)

    a = _grid(gpu, c, tree)
    a.step(n)
    path = os.path.join(tempfile.mkdtemp(), "ckpt.bin")
    a.save(path)
    a.close()
    b = _grid(gpu, c, tree)
    b.load(path)
    b.step(n)
    for l in range(c["L"]):
        got = b.get_populations(l)
        assert np.array_equal(np.isnan(got), np.isnan(want_f[l]))
        assert np.array_equal(got[~np.isnan(got)], want_f[l][~np.isnan(want_f[l])]), f"level {l}"
    got_series = b.drag_series()
    assert got_series.shape == want_series.shape == (2 * n << (c["L"] - 1), 3)
    assert np.array_equal(got_series, want_series)
    d = b.drag(per_branch=True)
    assert d["samples"] == want_drag["samples"]
    assert np.array_equal(d["force"], want_drag["force"])
    assert np.array_equal(d["per_branch"], want_drag["per_branch"])
    ref.close()
    b.close()


def test_checkpoint_of_another_grid_is_rejected(gpu):
    c = CASES["uniform_fp32"]
    tree = O.build_tree(O.cfg1_tree_params(), 0.0, list(c["com"]))
    a = _grid(gpu, c, tree)
    a.step(2)
    path = os.path.join(tempfile.mkdtemp(), "ckpt.bin")
    a.save(path)
    a.step(1)
    with pytest.raises(gpu.LbmError) as e:
        a.save(path)  # odd step count
    assert e.value.status == gpu.LBM_E_STATE
    b = _grid(gpu, CASES["uniform_fp16"], tree)
    with pytest.raises(gpu.LbmError) as e:
        b.load(path)
    assert e.value.status == gpu.LBM_E_INVALID
    a.close()
    b.close()


@pytest.mark.parametrize("poison", ["nan", "dense"])
def test_unstable_state_is_reported(gpu, poison):
    print(f"[unstable] {poison}", flush=True)
    c = CASES["uniform_fp32"]
    tree = O.build_tree(O.cfg1_tree_params(), 0.0, list(c["com"]))
    g = _grid(gpu, c, tree)
    g.step(2)
    d = g.drag()
    assert np.isfinite(d["cd"])
    f = g.get_populations(0)
    cell = 40 + 64 * (8 + 32 * 20)  # a fluid cell downstream of the tree
    assert g.solid()[cell] == 0
    if poison == "nan":
        f[:, cell] = np.nan
    else:
        f[:, cell] *= 2.0  # density 2
    g.set_populations(f, 0)
    with pytest.raises(gpu.LbmError) as e:
        g.drag()
    assert e.value.status == gpu.LBM_E_UNSTABLE
    g.close()


@pytest.mark.parametrize("name", ["uniform_fp32", "two_level_fp32", "uniform_fp16"])
def test_bound_memory_holds_the_populations(gpu, name):
    """Populations in a caller-owned torch tensor (lbm_bind_memory): the run is
    bit for bit the run in library memory, the tensor is where the state lives,
    and a tensor shorter than lbm_plan_levels' pop_bytes is refused."""
    import torch
    print(f"[bind memory] {name}", flush=True)
    c = CASES[name]
    tree = O.build_tree(O.cfg1_tree_params(), 0.0, list(c["com"]))
    nx, ny, nz = c["box"]
    plan = gpu.plan_levels(tree, refine=c["refine"], nx=nx, ny=ny, nz=nz, u_in=U, re_h=100.0, block_edge=c["B"],
                           levels=c["L"], storage=c["storage"])
    buf = torch.zeros(plan["pop_bytes"], dtype=torch.uint8, device="cuda")
    a = gpu.Grid(*c["box"], u_in=U, re_h=100.0, block_edge=c["B"], levels=c["L"], storage=c["storage"],
                 drag_every=1)
    a.bind_memory(buf)
    a.set_geometry(tree, refine=c["refine"])
    ref = _grid(gpu, c, tree)
    assert a.info()["device_bytes"] < ref.info()["device_bytes"]
    a.step(4)
    ref.step(4)
    torch.cuda.synchronize()
    before = buf.clone()
    a.step(1)
    ref.step(1)
    torch.cuda.synchronize()
    assert not torch.equal(before, buf)  # the step wrote the tensor
    for l in range(c["L"]):
        fa, fr = a.get_populations(l), ref.get_populations(l)
        assert np.array_equal(fa, fr, equal_nan=True), f"level {l}"
    assert np.array_equal(a.drag()["force"], ref.drag()["force"])
    a.close()
    ref.close()
    short = torch.zeros(plan["pop_bytes"] - 256, dtype=torch.uint8, device="cuda")
    b = gpu.Grid(*c["box"], u_in=U, re_h=100.0, block_edge=c["B"], levels=c["L"], storage=c["storage"])
    b.bind_memory(short)
    with pytest.raises(gpu.LbmError) as e:
        b.set_geometry(tree, refine=c["refine"])
    assert e.value.status == gpu.LBM_E_INVALID
    b.close()
