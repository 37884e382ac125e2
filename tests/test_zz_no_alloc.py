"""The allocation-free entry point zk_step_static (workspace in the library's
fixed device scratch) against zk_step on a bound workspace, through the C ABI:
two calls in a row on different contexts, the second on a smaller grid, each
held to the FP64 bar (1e-10 relative; the same kernels in the same order, so
the results are expected bit-identical), and a grid too large for the scratch
rejected with ZK_ENOWS."""
import math

import numpy as np
import pytest

from paper_2608_25203_amd.inputs import random_band_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_static_scratch_step_matches_bound_workspace(torch):
    from paper_2608_25203_amd import zk

    cases = [(256, 128, 4, 0.9, 0.004, 5), (64, 64, 3, 1.0, 0.01, 3)]  # second call: a smaller grid
    stream = torch.cuda.current_stream().cuda_stream
    for nx, ny, M, depth, dt, nsteps in cases:
        Lx, Ly = 2.0, 2.0 * ny / nx
        kmax = math.hypot(math.pi * nx / Lx, math.pi * ny / Ly)
        eta, psi = random_band_fields(nx, ny, 90 + M, min(nx, ny) // 2 - 1, amplitude=0.1 / kmax)
        ref = zk.Solver(nx, ny, Lx, Ly, depth, 9.81, M)
        e0 = torch.tensor(eta, dtype=torch.float64, device="cuda")
        p0 = torch.tensor(psi, dtype=torch.float64, device="cuda")
        ref.step(e0, p0, dt, nsteps)
        ctx = zk.zk_create(nx, ny, Lx, Ly, depth, 9.81, M)
        assert zk.zk_workspace_bytes(ctx) <= zk.ZK_STATIC_WS_BYTES
        e1 = torch.tensor(eta, dtype=torch.float64, device="cuda")
        p1 = torch.tensor(psi, dtype=torch.float64, device="cuda")
        zk.zk_step_static(ctx, e1.data_ptr(), p1.data_ptr(), dt, nsteps, stream)
        torch.cuda.synchronize()
        for a, b in ((e1, e0), (p1, p0)):
            r = float((a - b).abs().max() / b.abs().max())
            print(f"  {nx}x{ny} M={M}: rel diff {r:.3e}, identical {bool(torch.equal(a, b))}", flush=True)
            assert r < 1e-10
        zk.lib().zk_destroy(ctx)
        ref.close()
    big = zk.zk_create(1024, 1024, 1.0, 1.0, 1.0, 9.81, 4)
    assert zk.zk_workspace_bytes(big) > zk.ZK_STATIC_WS_BYTES
    x = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    with pytest.raises(zk.ZKError) as ei:
        zk.zk_step_static(big, x.data_ptr(), x.data_ptr(), 0.01, 1, stream)
    assert ei.value.code == zk.ZK_ENOWS
    zk.lib().zk_destroy(big)
