"""GPU parity of the closure network's kernels (through the C ABI) against
the CPU reference oracle/cnn.py.

Two references.  The independent one is the plain FP64 network: the bf16
mode of the network (bf16 weights and activations, FP32 accumulation) must
stay within 2e-2 relative of it, forward and per gradient tensor.  The
second is the FP64 network with bf16 rounding at the points where the
kernels store bf16 MFMA operands (bf16=True: operands rounded, FP64
products); it is shaped to the kernels, so it only localises a failure and
must agree to FP32-accumulation level (2e-3; a rare one-ulp bf16 flip
aside).  Tolerances are max-norm relative per tensor.
"""
import numpy as np
import pytest

from oracle import cnn as C
from paper_2608_25203_amd.inputs import cnn_init_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rel(a, b):
    r = float(np.max(np.abs(np.asarray(a, float) - np.asarray(b, float))) / max(np.max(np.abs(b)), 1e-300))
    print(f"  rel err {r:.3e}", flush=True)
    return r


def make_case(B, H, W, seed):
    params = cnn_init_params(seed)
    # larger than the initial scale so every GELU is exercised off its linear part
    params = [p * 2.0 if p.ndim == 4 else 0.1 * np.random.default_rng(seed + 1).standard_normal(p.shape)
              for p in params]
    rng = np.random.default_rng(seed + 2)
    samples = rng.standard_normal((B, 4, H, W))
    return params, samples


def flat32(params):
    return C.flatten(params).astype(np.float32)


@pytest.mark.parametrize("B,H,W", [(1, 8, 32), (2, 16, 64), (1, 21, 128)])
def test_forward_parity(torch, B, H, W):
    from paper_2608_25203_amd.zk import Net

    params, samples = make_case(B, H, W, 3)
    p32 = flat32(params)
    net = Net(B * H * W)
    net.set_params(p32)
    s = torch.tensor(samples, dtype=torch.float32, device="cuda")
    y = net.forward(s).cpu().numpy()
    # the reference sees exactly what the GPU sees: FP32 parameters, FP32 samples
    pref = C.unflatten(p32.astype(np.float64))
    x = samples.astype(np.float32).astype(np.float64)[:, :3]
    yq, _ = C.CNN(pref, bf16=True).forward(x)
    y64, _ = C.CNN(pref).forward(x)
    assert rel(y, yq[:, 0]) < 2e-3
    assert rel(y, y64[:, 0]) < 2e-2


@pytest.mark.parametrize("B,H,W,halo", [(2, 12, 64, 4), (1, 16, 128, 4)])
def test_gradient_parity(torch, B, H, W, halo):
    from paper_2608_25203_amd.zk import Net

    params, samples = make_case(B, H, W, 5)
    p32 = flat32(params)
    net = Net(B * H * W)
    net.set_params(p32)
    s = torch.tensor(samples, dtype=torch.float32, device="cuda")
    loss, g = net.gradient(s, halo)
    pref = C.unflatten(p32.astype(np.float64))
    sx = samples.astype(np.float32).astype(np.float64)
    ref = {}
    for bf in (True, False):
        cn = C.CNN(pref, bf16=bf)
        y, cache = cn.forward(sx[:, :3])
        l, dy = C.masked_mse(y, sx[:, 3:4], halo)
        gr, _ = cn.backward(cache, dy)
        ref[bf] = (l, gr)
    assert abs(loss / ref[True][0] - 1) < 2e-3
    gg = C.unflatten(g.astype(np.float64))
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    for i, name in enumerate(names):
        print(f" {name}", flush=True)
        assert rel(gg[i], ref[True][1][i]) < 2e-3, name
        assert rel(gg[i], ref[False][1][i]) < 2e-2, name


def test_adam_step_and_training(torch):
    """One step moves each parameter by lr g / (|g| + eps) (Adam from zero
    moments, with the GPU's own gradient); 60 further steps on a fixed batch
    reduce the loss at least 3x."""
    from paper_2608_25203_amd.zk import Net

    B, H, W, halo = 2, 16, 64, 4
    params, samples = make_case(B, H, W, 7)
    # a learnable target: a fixed 3 x 3 filter of the input planes
    k = np.zeros((1, 3, 3, 3))
    k[0, 0, 1, 1], k[0, 1, 0, 1], k[0, 2, 1, 2] = 0.5, -0.3, 0.2
    samples[:, 3:4] = C.conv3x3(samples[:, :3], k, np.zeros(1))
    p32 = flat32(params)
    net = Net(B * H * W)
    net.set_params(p32)
    s = torch.tensor(samples, dtype=torch.float32, device="cuda")
    l0, g = net.gradient(s, halo)
    lr = 1e-3
    net.train_step(s, halo, lr)
    p1 = net.get_params().astype(np.float64)
    expect = p32.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p1 - expect)) < 2e-3 * lr
    for _ in range(60):
        l = net.train_step(s, halo, 3e-3, want_loss=True)
    print(f"  loss {l0:.4e} -> {l:.4e}", flush=True)
    assert l < l0 / 3
