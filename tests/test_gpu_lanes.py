"""GPU parity of the padded row passes in their permuted-layout form
(ZK_OPT_ROW_FFT = ZK_ROW_FFT_LANES: lane-exchange butterflies inside a
wavefront, LDS stages only across wavefronts) against the CPU oracle, for
every team size it covers (64 to 1024 threads, one to sixteen wavefronts)
and first-pass radices 3, 6, 9 and 12, in FP64 (1e-10) and FP32 (2e-5 per
RHS); and against the default Stockham form of the same context (the two
differ only in rounding order)."""
import math

import numpy as np
import pytest

from oracle.hos import Grid, HOSModel
from paper_2608_25203_amd.inputs import random_band_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rel(a, b):
    r = float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))
    print(f"  rel err {r:.3e}", flush=True)
    return r


# (nx, ny, M, precision, padded-row team size T): E = 3 nx / 2 / T
CASES = [(128, 64, 4, 64, 64), (256, 128, 3, 64, 128), (512, 64, 4, 64, 256), (1024, 64, 3, 64, 512),
         (512, 64, 3, 64, 128), (512, 64, 3, 32, 64), (384, 64, 3, 64, 64), (768, 64, 2, 64, 128),
         (1536, 64, 2, 32, 256), (256, 1, 4, 64, 128), (2048, 64, 2, 32, 1024), (2048, 64, 2, 64, 1024),
         (1536, 64, 2, 64, 256), (512, 64, 3, 64, 64)]


def lanes_built(T, E, real_bytes):
    """the shapes the permuted-layout row kernels are built for (row_lanes_ok)"""
    N, tpb = T * E, max(T, 256) // T
    return T % 64 == 0 and T <= 1024 and 2 * tpb * N * 2 * real_bytes <= 100 * 1024


@pytest.mark.parametrize("nx,ny,M,prec,T", CASES)
def test_lanes_row_form_parity(torch, nx, ny, M, prec, T):
    from paper_2608_25203_amd.zk import ZK_OPT_ROW_FFT, ZK_ROW_FFT_LANES, ZK_ROW_FFT_STOCKHAM, Solver

    assert lanes_built(T, 3 * nx // 2 // T, prec // 8)
    Lx, Ly, h = 2.0, max(2.0 * ny / nx, 0.05), 0.6
    kmax = math.hypot(math.pi * nx / Lx, math.pi * ny / Ly)
    eta, psi = random_band_fields(nx, ny, 300 + T + M, max(min(nx, ny) // 2 - 1, nx // 2 - 1 if ny == 1 else 0),
                                  amplitude=0.1 / kmax)
    s = Solver(nx, ny, Lx, Ly, h, 9.81, M, precision=prec)
    s.set_team_shape(1, 1, T)
    print(f"  {nx}x{ny} M={M} FP{prec}: padded row team {s.team_shapes()['row_pad']}", flush=True)
    e = torch.tensor(eta, dtype=torch.float64, device="cuda")
    p = torch.tensor(psi, dtype=torch.float64, device="cuda")
    s.set_option(ZK_OPT_ROW_FFT, ZK_ROW_FFT_STOCKHAM)
    g_st = s.dtn(e, p).cpu().numpy()
    s.set_option(ZK_OPT_ROW_FFT, ZK_ROW_FFT_LANES)
    assert s.get_option(ZK_OPT_ROW_FFT) == ZK_ROW_FFT_LANES
    g = s.dtn(e, p).cpu().numpy()
    a, b = (x.cpu().numpy() for x in s.rhs(e, p))
    m = HOSModel(Grid(nx, ny, Lx, Ly, h), M)
    a0, b0 = m.rhs(eta, psi)
    tol = 1e-10 if prec == 64 else 2e-5
    assert rel(g, g_st) < (1e-12 if prec == 64 else 1e-5)
    assert rel(g, m.dtn(eta, psi)) < tol
    assert rel(a, a0) < tol and rel(b, b0) < tol
    if prec == 64:
        s.step(e, p, 0.002, 2)
        e0, p0 = m.step(eta, psi, 0.002, 2)
        assert rel(e.cpu().numpy(), e0) < 1e-10 and rel(p.cpu().numpy(), p0) < 1e-10
    s.close()
