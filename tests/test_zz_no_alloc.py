"""The no-allocation gradient entry point (lbm_mlp_grad_noalloc) against the
allocating one (lbm_mlp_grad) through the C-ABI: the same kernels on a static
device workspace give the same bits, over two calls in a row (the second
smaller, so the workspace holds the first call's partial sums), and sizes
beyond the workspace are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(torch, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 5)).astype(np.float32) * [0.5, 20.0, 1.0, 0.05, 0.3] + [2.0, 45.0, 2.0, 0.04, 0.5]
    t = rng.standard_normal(n).astype(np.float32)
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev),
            torch.from_numpy(t).to(dev))


def test_noalloc_gradient_equals_the_allocating_entry_point(gpu):
    import torch
    print("[no-alloc] lbm_mlp_grad_noalloc vs lbm_mlp_grad", flush=True)
    m = gpu.Mlp(seed=7)
    m.set_scaling([2.0, 45.0, 2.0, 0.04, 0.5], [0.5, 20.0, 1.0, 0.05, 0.3], 0.3, 1.7)
    g_dev = torch.empty(4609, dtype=torch.float32, device="cuda:0")
    l_dev = torch.empty(1, dtype=torch.float32, device="cuda:0")
    for call, n in enumerate((20000, 333)):
        x, t = _inputs(torch, n, 100 + call)
        torch.cuda.synchronize()
        want, want_loss = m.grad(x, t)
        g_dev.fill_(float("nan"))
        l_dev.fill_(float("nan"))
        torch.cuda.synchronize()
        m.grad_noalloc(x, t, g_dev, l_dev)
        torch.cuda.synchronize()
        got = g_dev.cpu().numpy()
        print(f"  call {call + 1}: n = {n}, max |grad| = {np.abs(want).max():.3e}, loss = {want_loss:.6f}",
              flush=True)
        assert np.array_equal(got, want)
        assert float(l_dev.cpu()[0]) == want_loss
    x, t = _inputs(torch, 32769, 5)
    with pytest.raises(gpu.LbmError) as e:
        m.grad_noalloc(x, t, g_dev, l_dev)
    assert e.value.status == gpu.LBM_E_INVALID
    m.close()
