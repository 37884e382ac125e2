"""GPU parity of the batched tile stepper (zk_batch_*).

Every tile of a batch must equal its own context's zk_step to 1e-12 (same
team shapes by default, but a single grid runs the last level's G task with
fold teams, which sum its folds and terms in another order, and autotuned
shapes round differently too), and the oracle at
the FP64 bar (1e-10).  The graph path is checked against the launch-by-
launch path on repeated calls with host synchronisation and eager work in
between (every replay compared).  FP32 batches: 2e-6 per step against the
FP64 oracle, as the single-grid FP32 form.
"""
import math

import numpy as np
import pytest

from oracle.hos import Grid, HOSModel
from paper_2608_25203_amd.inputs import jonswap_state, random_band_fields

pytestmark = pytest.mark.gpu

TILES = [
    dict(nx=64, ny=64, Lx=2 * math.pi, Ly=2 * math.pi, depth=math.inf, M=3),
    dict(nx=128, ny=64, Lx=4.0, Ly=2.0, depth=1.0, M=2),
    dict(nx=64, ny=128, Lx=2.0, Ly=4.0, depth=0.5, M=4),
    dict(nx=128, ny=128, Lx=2 * math.pi, Ly=2 * math.pi, depth=math.inf, M=6),
    dict(nx=256, ny=256, Lx=50.0, Ly=50.0, depth=8.0, M=5),
    dict(nx=64, ny=64, Lx=1.0, Ly=1.0, depth=0.3, M=1),
    dict(nx=128, ny=128, Lx=2 * math.pi, Ly=2 * math.pi, depth=math.inf, M=3),
    dict(nx=1024, ny=512, Lx=8.0, Ly=4.0, depth=2.0, M=3),  # 512- and 1024-thread team candidates
]
DT = 0.004


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    r = float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
    print(f"  rel err {r:.3e}", flush=True)
    return r


def states():
    out = []
    for k, t in enumerate(TILES):
        kmax = math.hypot(math.pi * t["nx"] / t["Lx"], math.pi * t["ny"] / t["Ly"])
        e, p = random_band_fields(t["nx"], t["ny"], 100 + k, min(t["nx"], t["ny"]) // 4, amplitude=0.05 / kmax)
        out.append((e, p))
    return out


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def run_batch(torch, precision, nsteps, graph=True, autotune=False):
    from paper_2608_25203_amd.zk import Batch

    st = states()
    b = Batch(TILES, precision=precision, graph=graph)
    es = [dev(torch, e) for e, _ in st]
    ps = [dev(torch, p) for _, p in st]
    b.set_fields(es, ps)
    if autotune:
        print(" ", b.autotune(DT, reps=2), flush=True)
    b.step(DT, nsteps)
    torch.cuda.synchronize()
    print(" ", b.stats(), flush=True)
    return st, [e.cpu().numpy() for e in es], [p.cpu().numpy() for p in ps]


def test_batch_equals_single_contexts_fp64(torch):
    from paper_2608_25203_amd.zk import Solver

    st, E, P = run_batch(torch, 64, 3)
    for k, t in enumerate(TILES):
        s = Solver(t["nx"], t["ny"], t["Lx"], t["Ly"], t["depth"], 9.81, t["M"])
        e, p = dev(torch, st[k][0]), dev(torch, st[k][1])
        s.step(e, p, DT, 3)
        assert rel(E[k], e.cpu().numpy()) < 1e-12 and rel(P[k], p.cpu().numpy()) < 1e-12
    for k in (0, 2, 3):
        t = TILES[k]
        dep = None if math.isinf(t["depth"]) else t["depth"]
        m = HOSModel(Grid(t["nx"], t["ny"], t["Lx"], t["Ly"], dep), t["M"])
        e0, p0 = m.step(st[k][0], st[k][1], DT, 3)
        assert rel(E[k], e0) < 1e-10 and rel(P[k], p0) < 1e-10


def test_batch_autotuned_fp64(torch):
    _, E0, P0 = run_batch(torch, 64, 2)
    _, E1, P1 = run_batch(torch, 64, 2, autotune=True)
    for k in range(len(TILES)):
        assert rel(E1[k], E0[k]) < 1e-12 and rel(P1[k], P0[k]) < 1e-12


def test_batch_fp32_against_oracle(torch):
    st, E, P = run_batch(torch, 32, 1, autotune=True)
    for k in (1, 3, 4):
        t = TILES[k]
        dep = None if math.isinf(t["depth"]) else t["depth"]
        m = HOSModel(Grid(t["nx"], t["ny"], t["Lx"], t["Ly"], dep), t["M"])
        e0, p0 = m.step(st[k][0], st[k][1], DT, 1)
        assert rel(E[k], e0) < 2e-6 and rel(P[k], p0) < 2e-6


def test_graph_replays_match_eager_launches(torch):
    """Five calls of one step each (entry, step and exit graphs replayed five
    times, with synchronisation and host work between calls) equal the same
    calls launched phase by phase, after every call."""
    from paper_2608_25203_amd.zk import Batch

    st = states()
    bg = Batch(TILES, precision=64, graph=True)
    be = Batch(TILES, precision=64, graph=False)
    eg = [dev(torch, e) for e, _ in st]
    pg = [dev(torch, p) for _, p in st]
    ee = [dev(torch, e) for e, _ in st]
    pe = [dev(torch, p) for _, p in st]
    bg.set_fields(eg, pg)
    be.set_fields(ee, pe)
    for call in range(5):
        bg.step(DT, 2)
        be.step(DT, 2)
        torch.cuda.synchronize()
        _ = [float(x.sum()) for x in eg]  # eager work between replays
        for k in range(len(TILES)):
            assert torch.equal(eg[k], ee[k]) and torch.equal(pg[k], pe[k]), (call, k)


# Tiles of 128 to 1024 points per axis: the sizes the persistent form hosts.
PTILES = [
    dict(nx=128, ny=128, Lx=2 * math.pi, Ly=2 * math.pi, depth=math.inf, M=3),
    dict(nx=256, ny=128, Lx=4.0, Ly=2.0, depth=1.0, M=2),
    dict(nx=128, ny=256, Lx=2.0, Ly=4.0, depth=0.5, M=4),
    dict(nx=256, ny=256, Lx=2 * math.pi, Ly=2 * math.pi, depth=math.inf, M=6),
    dict(nx=512, ny=256, Lx=50.0, Ly=25.0, depth=8.0, M=5),
    dict(nx=128, ny=128, Lx=1.0, Ly=1.0, depth=0.3, M=1),
    dict(nx=1024, ny=512, Lx=8.0, Ly=4.0, depth=2.0, M=3),
    dict(nx=512, ny=512, Lx=2 * math.pi, Ly=2 * math.pi, depth=math.inf, M=4),
]


def pstates():
    out = []
    for k, t in enumerate(PTILES):
        kmax = math.hypot(math.pi * t["nx"] / t["Lx"], math.pi * t["ny"] / t["Ly"])
        e, p = random_band_fields(t["nx"], t["ny"], 300 + k, min(t["nx"], t["ny"]) // 4, amplitude=0.05 / kmax)
        out.append((e, p))
    return out


@pytest.mark.parametrize("precision", [64, 32])
def test_persistent_batch_equals_graph_batch(torch, precision):
    """One persistent launch per step (workers taking units from a device
    queue, per-tile completion counters) gives every tile the same result as
    the graph of batched launches: the same bodies and team shapes, so the
    same arithmetic (held to 1e-12, expected bit-identical), over two calls
    (3 steps, then 2) so the counters are reset between launches; FP64 tiles
    also against the oracle at 1e-10."""
    from paper_2608_25203_amd.zk import Batch

    st = pstates()
    bp = Batch(PTILES, precision=precision, persistent=True)
    bg = Batch(PTILES, precision=precision)
    ep = [dev(torch, e) for e, _ in st]
    pp = [dev(torch, p) for _, p in st]
    eg = [dev(torch, e) for e, _ in st]
    pg = [dev(torch, p) for _, p in st]
    bp.set_fields(ep, pp)
    bg.set_fields(eg, pg)
    for n in (3, 2):
        bp.step(DT, n)
        bg.step(DT, n)
        torch.cuda.synchronize()
        same = sum(int(torch.equal(ep[k], eg[k]) and torch.equal(pp[k], pg[k])) for k in range(len(PTILES)))
        print(f"  {n} steps: {same} of {len(PTILES)} tiles bit-identical", flush=True)
        for k in range(len(PTILES)):
            assert rel(ep[k].cpu().numpy(), eg[k].cpu().numpy()) < 1e-12
            assert rel(pp[k].cpu().numpy(), pg[k].cpu().numpy()) < 1e-12
    assert bp.stats()["launches_per_step"] == 1
    if precision == 64:
        for k in (0, 3, 4):
            t = PTILES[k]
            dep = None if math.isinf(t["depth"]) else t["depth"]
            m = HOSModel(Grid(t["nx"], t["ny"], t["Lx"], t["Ly"], dep), t["M"])
            e0, p0 = m.step(st[k][0], st[k][1], DT, 5)
            assert rel(ep[k].cpu().numpy(), e0) < 1e-10 and rel(pp[k].cpu().numpy(), p0) < 1e-10
    bp.close()
    bg.close()


@pytest.mark.timeout(900)
def test_persistent_batch_c4_largest_tile_against_oracle(torch):
    """The largest tile of the batch workload's draw (1024 x 1024 at 1 m
    spacing, M = 6) in one persistent batch with smaller tiles, FP64, one RK4
    step (dt = 0.05 s) of a JONSWAP state (k_p = 2 pi / 16 m, steepness
    0.12): against the oracle at 1e-10."""
    from oracle.hos import PocketDFT
    from paper_2608_25203_amd.zk import Batch

    kp = 2 * math.pi / 16.0
    tiles = [dict(nx=1024, ny=1024, Lx=1024.0, Ly=1024.0, depth=120.0, M=6),
             dict(nx=256, ny=256, Lx=256.0, Ly=256.0, depth=30.0, M=3),
             dict(nx=128, ny=128, Lx=128.0, Ly=128.0, depth=12.0, M=5)]
    st = [jonswap_state(t["nx"], t["ny"], t["Lx"], t["Ly"], t["depth"], 9.81, kp, s, 1000 + k)
          for k, (t, s) in enumerate(zip(tiles, (0.12, 0.08, 0.05)))]
    b = Batch(tiles, precision=64, persistent=True)
    es = [dev(torch, e) for e, _ in st]
    ps = [dev(torch, p) for _, p in st]
    b.set_fields(es, ps)
    b.step(0.05, 1)
    torch.cuda.synchronize()
    t = tiles[0]
    m = HOSModel(Grid(t["nx"], t["ny"], t["Lx"], t["Ly"], t["depth"], dft=PocketDFT(workers=16)), t["M"])
    e0, p0 = m.step(st[0][0], st[0][1], 0.05, 1)
    assert rel(es[0].cpu().numpy(), e0) < 1e-10 and rel(ps[0].cpu().numpy(), p0) < 1e-10
    b.close()
