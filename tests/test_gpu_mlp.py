"""GPU MLP (learned flux correction) against the FP64 oracle: forward and gradients in the FP32
reference mode to 1e-5; the BF16 matrix-core mode within a stated bound; Adam."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BF16_BOUND = 3e-2   # 8-bit mantissa operands over four layers, FP32 accumulation


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


def _setup(oracle_mod, H, n, seed):
    rng = np.random.default_rng(seed)
    npar = oracle_mod.mlp_n_params(H)
    p = rng.normal(scale=1.0 / np.sqrt(32), size=npar)
    x = rng.normal(size=(n, 32))
    t = rng.normal(size=(n, 8))
    return p, x, t


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("H,n", [(32, 37), (128, 200), (64, 16)])
@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_forward_matches_oracle(bd, oracle_mod, H, n, mode):
    p, x, _ = _setup(oracle_mod, H, n, 1)
    net = bd.Mlp(H, torch.from_numpy(p.astype(np.float32)))
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda(), mode=mode).cpu().numpy()
    ref = oracle_mod.mlp_forward(p.astype(np.float32).astype(np.float64), H, x.astype(np.float32).astype(np.float64))
    err = _rel(y, ref)
    print("forward", H, n, mode, err, flush=True)
    assert err <= (1e-5 if mode == "fp32" else BF16_BOUND)


@pytest.mark.parametrize("H,n", [(128, 70001), (64, 33), (32, 4097)])
def test_inference_kernel_equals_training_forward(bd, oracle_mod, H, n):
    """The persistent LDS-resident inference kernel (no saved activations) evaluates the same BF16
    products in the same order as the training forward: equal bitwise, also over many tiles per wave."""
    p, x, _ = _setup(oracle_mod, H, n, 3)
    net = bd.Mlp(H, torch.from_numpy(p.astype(np.float32)))
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    y_inf = net.forward(xd).cpu().numpy()
    y_tr, _ = net.forward(xd, save=True)
    assert np.array_equal(y_inf, y_tr.cpu().numpy())
    sel = np.arange(0, n, max(1, n // 50))
    ref = oracle_mod.mlp_forward(p.astype(np.float32).astype(np.float64), H, x[sel].astype(np.float32).astype(np.float64))
    assert _rel(y_inf[sel], ref) <= BF16_BOUND


@pytest.mark.parametrize("H,n", [(32, 50), (128, 96), (64, 1000)])
@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_gradients_match_oracle(bd, oracle_mod, H, n, mode):
    p, x, t = _setup(oracle_mod, H, n, 2)
    p32, x32, t32 = p.astype(np.float32), x.astype(np.float32), t.astype(np.float32)
    net = bd.Mlp(H, torch.from_numpy(p32))
    loss, g = net.loss_grad(torch.from_numpy(x32).cuda(), torch.from_numpy(t32).cuda(), mode=mode)
    g = g.cpu().numpy()
    rl, rg = oracle_mod.mlp_loss_grad(p32.astype(np.float64), H, x32.astype(np.float64), t32.astype(np.float64))
    assert abs(float(loss) - rl) <= (1e-5 if mode == "fp32" else BF16_BOUND) * abs(rl)
    # per parameter block (each layer's weights and biases), normwise
    import oracle as om
    offs = [0]
    for (o, i) in [(H, 32), (H, H), (H, H), (8, H)]:
        offs += [offs[-1] + o * i, offs[-1] + o * i + o]
    for a, b in zip(offs[:-1], offs[1:]):
        err = float(np.abs(g[a:b] - rg[a:b]).max() / np.abs(rg[a:b]).max())
        print("grad", H, mode, a, b, err, flush=True)
        assert err <= (1e-5 if mode == "fp32" else 2 * BF16_BOUND), (a, b, err)


def test_adam_matches_oracle(bd, oracle_mod):
    H = 32
    p, x, t = _setup(oracle_mod, H, 40, 3)
    p32 = p.astype(np.float32)
    net = bd.Mlp(H, torch.from_numpy(p32))
    rng = np.random.default_rng(4)
    pr, mr, vr = p32.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for step in range(1, 4):
        g = rng.normal(size=p.size).astype(np.float32)
        net.adam(torch.from_numpy(g).cuda(), lr=1e-2)
        oracle_mod.mlp_adam(pr, mr, vr, g.astype(np.float64), 1e-2, step)
    got = net.p.cpu().numpy()
    assert np.abs(got - pr).max() <= 1e-5 * np.abs(pr).max()
    # the BF16 copy is the round-to-nearest of the FP32 master
    pb = net.pb.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    assert np.abs(pb.view(np.float32) - got).max() <= np.abs(got).max() * 2 ** -8
