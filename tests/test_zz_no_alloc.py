"""The allocation-free gradient entry point (tr_mlp_grad_noalloc) against the
workspace one (tr_mlp_grad), through the C ABI: two calls in a row, the second
with fewer samples, and the size limit."""
import numpy as np
import pytest

from paper_2011_05427_amd import binding

from gpu_util import note

pytestmark = pytest.mark.gpu


def _data(torch, n, seed):
    rng = np.random.default_rng(seed)
    X = torch.as_tensor(rng.normal(0, 1, (n, 8)).astype(np.float32)).to("cuda")
    Y = torch.as_tensor(np.stack([rng.uniform(0.2, 0.8, n), rng.normal(0, 0.3, n)], 1).astype(np.float32)).to("cuda")
    return X, Y


def test_noalloc_gradient_equals_workspace_gradient():
    import torch

    lib = binding.load()
    nparam = lib.tr_mlp_nparam()
    rng = np.random.default_rng(21)
    net = binding.Mlp(rng.normal(0, 0.08, nparam).astype(np.float32))
    for n, seed in ((4096, 1), (1000, 2)):
        note(f"tr_mlp_grad_noalloc n={n}")
        X, Y = _data(torch, n, seed)
        g_ref, l_ref = net.grad(X, Y)
        g = torch.full((nparam,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        net.grad_noalloc(X, Y, g, loss)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), float((g - g_ref).abs().max())
        assert torch.equal(loss, l_ref)
        assert torch.isfinite(g).all() and float(g.abs().max()) > 0


def test_noalloc_gradient_rejects_sizes_beyond_its_scratch():
    import torch

    lib = binding.load()
    net = binding.Mlp(np.zeros(lib.tr_mlp_nparam(), dtype=np.float32))
    n = binding.TR_MLP_NOALLOC_MAX_N + 1
    X = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    Y = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    g = torch.zeros(lib.tr_mlp_nparam(), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(binding.TrError) as e:
        net.grad_noalloc(X, Y, g, loss)
    assert e.value.code == binding.TR_EINVAL
