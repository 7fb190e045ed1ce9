"""The allocation-free backward pass (static device work area) against the ordinary entry point that
takes a caller-owned work buffer: equal bit for bit, on two calls in a row (the second with fewer
samples, so the static area still holds the first call's larger contents), in both product modes; an
oversized request is refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


def _inputs(H, n, seed, npar):
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=1.0 / np.sqrt(32), size=npar).astype(np.float32)
    x = rng.normal(size=(n, 32)).astype(np.float32)
    t = rng.normal(size=(n, 8)).astype(np.float32)
    return p, torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()


@pytest.mark.parametrize("mode", ["bf16", "fp32"])
@pytest.mark.parametrize("H,sizes", [(128, (3001, 517)), (64, (20000, 33)), (32, (4097, 1))])
def test_noalloc_backward_equals_workspace_backward(bd, H, sizes, mode):
    npar = int(bd.lib().bmhd_mlp_n_params(H))
    for call, n in enumerate(sizes):
        print(f"noalloc backward H={H} n={n} mode={mode} call={call}", flush=True)
        p, x, t = _inputs(H, n, 100 + call, npar)
        net = bd.Mlp(H, torch.from_numpy(p))
        loss_ref, g_ref = net.loss_grad(x, t, mode=mode)
        loss, g = net.loss_grad(x, t, mode=mode, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), (H, n, mode, call)
        assert torch.equal(loss, loss_ref)
        assert torch.isfinite(g).all()


def test_noalloc_backward_refuses_oversized_n(bd):
    H = 128
    max_n = (8 << 20) // (16 + 2 * H)
    npar = int(bd.lib().bmhd_mlp_n_params(H))
    net = bd.Mlp(H, torch.zeros(npar))
    n = max_n + 1
    x = torch.zeros((n, 32), dtype=torch.float32, device="cuda")
    t = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(bd.BmhdError, match="exceeds the static scratch"):
        net.loss_grad(x, t, noalloc=True)
    # the largest accepted size runs and equals the work-buffer path
    p, x, t = _inputs(H, max_n, 7, npar)
    net = bd.Mlp(H, torch.from_numpy(p))
    _, g_ref = net.loss_grad(x, t)
    _, g = net.loss_grad(x, t, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(g, g_ref)
