"""Host-side checks that need no GPU: the planner's schedules (validated and
executed by a numpy interpreter against the oracle) and the C ABI library
(loads, exports every symbol of include/zk.h, host-only argument checks)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle.hos import Grid, HOSModel
from paper_2608_25203_amd.inputs import jonswap_state, random_band_fields

from plan_interp import Interp, load_plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TWO_PI = 2 * np.pi


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("nx,ny", [(64, 64), (128, 64), (512, 512), (2048, 2048), (96, 96), (384, 64), (1536, 192),
                                   (32, 32), (32, 128), (16, 16), (48, 16), (16, 48), (16, 4), (16, 12), (48, 4),
                                   (80, 20), (160, 80), (1280, 640), (80, 1)])
@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6, 7, 8])
def test_plan_builds_and_validates(nx, ny, M):
    p = load_plan(nx, ny, M)
    assert p["nmix"] > 0 and p["nbase"] > 0
    # every launch of every sequence is non-empty
    for k in ("dtn", "rhs", "ham", "step_entry", "step_body0", "step_body1", "step_exit0", "step_exit1"):
        assert len(p[k]) > 0


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6, 7])
def test_schedule_algebra_matches_oracle_jonswap(M):
    """The planner's row programs and column tasks, executed literally, give
    the oracle's G psi, RHS, Hamiltonian and RK4 steps (64 x 64 deep-water
    JONSWAP state, steepness 0.05)."""
    n, L = 64, TWO_PI
    eta, psi = jonswap_state(n, n, L, L, None, 9.81, 4.0, 0.05, 0)
    I = Interp(n, n, L, L, None, 9.81, M)
    m = HOSModel(Grid(n, n, L, L, None), M)
    assert rel(I.dtn(eta, psi), m.dtn(eta, psi)) < 1e-13
    a, b = I.rhs(eta, psi)
    a0, b0 = m.rhs(eta, psi)
    assert rel(a, a0) < 1e-13 and rel(b, b0) < 1e-13
    assert abs(I.hamiltonian(eta, psi) / m.hamiltonian(eta, psi) - 1) < 1e-13
    s, t = I.step(eta, psi, 0.01, 3)
    s0, t0 = m.step(eta, psi, 0.01, 3)
    assert rel(s, s0) < 1e-13 and rel(t, t0) < 1e-13


@pytest.mark.parametrize("M", [3, 5])
def test_schedule_algebra_non_power_of_two_grid(M):
    """Axes of 3 2^k points (96 x 192: padded lengths 144 and 288): the
    schedule executed literally equals the oracle's G psi, RHS and steps."""
    nx, ny = 96, 192
    eta, psi = random_band_fields(nx, ny, 11, nx // 2 - 1, amplitude=0.02)
    I = Interp(nx, ny, 3.0, 6.0, 1.2, 9.81, M)
    m = HOSModel(Grid(nx, ny, 3.0, 6.0, 1.2), M)
    assert rel(I.dtn(eta, psi), m.dtn(eta, psi)) < 1e-13
    a, b = I.rhs(eta, psi)
    a0, b0 = m.rhs(eta, psi)
    assert rel(a, a0) < 1e-13 and rel(b, b0) < 1e-13
    s, t = I.step(eta, psi, 0.002, 2)
    s0, t0 = m.step(eta, psi, 0.002, 2)
    assert rel(s, s0) < 1e-13 and rel(t, t0) < 1e-13


@pytest.mark.parametrize("M", [2, 4, 6])
@pytest.mark.parametrize("eps,taper,filt", [(0.6, True, True), (1.0, False, False)])
def test_schedule_algebra_matches_oracle_broadband(M, eps, taper, filt):
    """Band-edge content, finite depth, non-square grid, options varied."""
    nx, ny = 32, 16
    eta, psi = random_band_fields(nx, ny, 3, 7, amplitude=0.02)
    I = Interp(nx, ny, 3.0, 2.0, 1.5, 9.81, M, eps=eps, taper=taper, filt=filt)
    m = HOSModel(Grid(nx, ny, 3.0, 2.0, 1.5), M, eps=eps, taper=taper, filt=filt)
    a, b = I.rhs(eta, psi)
    a0, b0 = m.rhs(eta, psi)
    assert rel(a, a0) < 1e-13 and rel(b, b0) < 1e-13
    s, t = I.step(eta, psi, 0.02, 2)
    s0, t0 = m.step(eta, psi, 0.02, 2)
    assert rel(s, s0) < 1e-13 and rel(t, t0) < 1e-13


@pytest.mark.parametrize("M", [2, 4])
def test_closure_pieces_match_oracle(M):
    """rhs_g (the RHS with G supplied on the grid, projected onto the band)
    and the stand-alone state filter, executed literally, against the
    oracle's Bernoulli term and filter."""
    nx, ny = 32, 16
    eta, psi = random_band_fields(nx, ny, 5, 7, amplitude=0.02)
    G = np.random.default_rng(6).standard_normal((ny, nx))  # any field, Nyquist content included
    I = Interp(nx, ny, 3.0, 2.0, 1.5, 9.81, M)
    m = HOSModel(Grid(nx, ny, 3.0, 2.0, 1.5), M)
    g = m.gr
    a, b = I.rhs_g(eta, psi, G)
    Gh = g.spec(G)
    eh, ph = g.spec(eta), g.spec(psi)
    assert rel(a, g.phys(Gh)) < 1e-13
    assert rel(b, g.phys(-9.81 * eh + m.bernoulli_spec(eh, ph, Gh))) < 1e-13
    fa, fb = I.filter(eta, psi)
    assert rel(fa, g.phys(eh * g.filt)) < 1e-13 and rel(fb, g.phys(ph * g.filt)) < 1e-13


@pytest.mark.parametrize("M,filt", [(1, True), (3, True), (4, False)])
def test_ab2_schedule_matches_oracle(M, filt):
    """The IF-AB2 schedules (bootstrap step, AB2 steps, ping-pong forcing),
    executed literally, give the oracle's step_ifab2 (Sec. 3.4)."""
    nx, ny = 32, 16
    eta, psi = random_band_fields(nx, ny, 9, 7, amplitude=0.02)
    I = Interp(nx, ny, 3.0, 2.0, 1.5, 9.81, M, filt=filt)
    m = HOSModel(Grid(nx, ny, 3.0, 2.0, 1.5), M, filt=filt)
    for n in (1, 2, 5):
        s, t = I.step_ab2(eta, psi, 0.02, n)
        s0, t0 = m.step_ifab2(eta, psi, 0.02, n)
        assert rel(s, s0) < 1e-13 and rel(t, t0) < 1e-13


@pytest.mark.parametrize("M", [1, 3, 4])
def test_inverse_dtn_schedule_matches_oracle(M):
    """The inverse-DNO schedules (seed, iterations, exit) executed literally
    equal the oracle's fixed-point iteration for 0, 1 and 8 iterations."""
    nx, ny = 32, 16
    eta, psi = random_band_fields(nx, ny, 13, 7, amplitude=0.02)
    I = Interp(nx, ny, 3.0, 2.0, 1.5, 9.81, M)
    m = HOSModel(Grid(nx, ny, 3.0, 2.0, 1.5), M)
    v = m.dtn(eta, psi)
    for it in (0, 1, 8):
        assert rel(I.inverse_dtn(eta, v, it), m.inverse_dtn(eta, v, it)) < 1e-13


@pytest.mark.parametrize("depth", [None, 1.5, 0.4])
def test_depth_velocity_schedule_matches_oracle(depth):
    """The depth-lift schedules (potential on the flat plane, then per layer
    the u, w and v lifts) executed literally equal the oracle's bulk
    velocity at seven depths from the surface plane to the bottom (or 1.5
    deep), for every chunking of the layers."""
    nx, ny, Lx, Ly = 32, 16, 3.0, 2.0
    eta, psi = random_band_fields(nx, ny, 17, 7, amplitude=0.02)
    I = Interp(nx, ny, Lx, Ly, depth, 9.81, 3)
    m = HOSModel(Grid(nx, ny, Lx, Ly, depth), 3)
    d = depth if depth else 1.5
    ys = [0.0, 0.2, d, 0.5 * d, 0.1, 0.7 * d, 0.3]
    ref = m.depth_velocity(eta, psi, ys)
    for chunk in (None, 1, 2, 3):  # full chunks, single layers, pairs, an odd chunk with a remainder
        got = I.depth_velocity(eta, psi, ys, chunk)
        for i in range(len(ys)):  # relative to the layer's largest component (v = 0 at a flat bottom)
            assert np.max(np.abs(got[i] - ref[i])) < 1e-13 * np.max(np.abs(ref[i])), (chunk, i)


# ---------------------------------------------------------------- the library
LIB = os.path.join(ROOT, "paper_2608_25203_amd", "libzk.so")


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "zk.h")).read()
    return sorted(set(re.findall(r"\b(zk_[a-z_]+)\s*\(", txt)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libzk.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    syms = _header_symbols()
    assert "zk_dtn" in syms and "zk_step" in syms and "zk_hamiltonian" in syms
    for s in syms:
        assert hasattr(lib, s), s
    from paper_2608_25203_amd import zk
    assert set(zk.EXPORTS) == set(syms)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libzk.so not built")
def test_library_host_side_argument_checks():
    from paper_2608_25203_amd import zk
    L = zk.lib()
    assert not L.zk_create(63, 64, 1.0, 1.0, 1.0, 9.81, 3)       # not 2^k, 3 2^k or 5 2^k
    assert not L.zk_create(100, 64, 1.0, 1.0, 1.0, 9.81, 3)      # 25 2^2: not 2^k, 3 2^k or 5 2^k
    assert not L.zk_create(64, 10, 1.0, 1.0, 1.0, 9.81, 3)       # 5 2^k below 20
    assert not L.zk_create(2560, 64, 1.0, 1.0, 1.0, 9.81, 3)     # 5 2^k above 1280
    assert not L.zk_create(160, 720, 1.0, 1.0, 1.0, 9.81, 3)     # 45 2^4: factors 3 and 5 together
    assert not L.zk_create(64, 6, 1.0, 1.0, 1.0, 9.81, 3)        # 3 2^k below 12
    assert not L.zk_create(64, 2, 1.0, 1.0, 1.0, 9.81, 3)        # 2^k below 4
    for nx in (4, 8, 12, 24):                                      # nx / 2 below a 64-byte column group
        assert not L.zk_create(nx, 64, 1.0, 1.0, 1.0, 9.81, 3)
    for nx, ny, T0 in ((16, 4, 2), (16, 8, 4), (16, 16, 8), (32, 32, 16), (48, 12, 2), (48, 24, 4),
                       (48, 48, 8)):  # the smallest axes: teams of 2 to 16 threads on the columns
        cs = L.zk_create(nx, ny, 1.0, 1.0, 1.0, 9.81, 3)
        assert cs
        T, E = ctypes.c_int(0), ctypes.c_int(0)
        assert L.zk_team_shape(cs, 0, 1, ctypes.byref(T), ctypes.byref(E)) == 0 and T.value == T0
        assert T.value * E.value == 3 * ny // 2
        assert L.zk_team_shape(cs, 0, 0, ctypes.byref(T), ctypes.byref(E)) == 0 and T.value * E.value == ny
        L.zk_destroy(cs)
    assert not L.zk_create(3072, 64, 1.0, 1.0, 1.0, 9.81, 3)     # 3 2^k above 1536
    for n in (96, 192, 384, 768, 1536):                            # 3 2^k axes from 96: teams of n / 6
        c3 = L.zk_create(n, 64, 1.0, 1.0, 1.0, 9.81, 3)
        assert c3
        T, E = ctypes.c_int(0), ctypes.c_int(0)
        assert L.zk_team_shape(c3, 1, 1, ctypes.byref(T), ctypes.byref(E)) == 0 and (T.value, E.value) == (n // 6, 9)
        assert L.zk_team_shape(c3, 1, 0, ctypes.byref(T), ctypes.byref(E)) == 0 and (T.value, E.value) == (n // 6, 6)
        L.zk_destroy(c3)
    for n in (80, 160, 320, 640, 1280):                            # 5 2^k axes: teams of n / 10, radix 15 and 10
        c5 = L.zk_create(n, 20, 1.0, 1.0, 1.0, 9.81, 3)
        assert c5
        T, E = ctypes.c_int(0), ctypes.c_int(0)
        assert L.zk_team_shape(c5, 1, 1, ctypes.byref(T), ctypes.byref(E)) == 0 and (T.value, E.value) == (n // 10, 15)
        assert L.zk_team_shape(c5, 1, 0, ctypes.byref(T), ctypes.byref(E)) == 0 and (T.value, E.value) == (n // 10, 10)
        assert L.zk_team_shape(c5, 0, 1, ctypes.byref(T), ctypes.byref(E)) == 0 and (T.value, E.value) == (2, 15)
        L.zk_destroy(c5)
    assert not L.zk_create(64, 4096, 1.0, 1.0, 1.0, 9.81, 3)     # too large
    assert not L.zk_create(64, 64, -1.0, 1.0, 1.0, 9.81, 3)      # bad length
    assert not L.zk_create(64, 64, 1.0, 1.0, 1.0, 9.81, 9)       # M out of range
    ctx = L.zk_create(512, 512, 200.0, 200.0, 20.0, 9.81, 4)
    assert ctx
    n64 = L.zk_workspace_bytes(ctx)
    assert L.zk_set_option(ctx, zk.ZK_OPT_PRECISION, 32.0) == 0
    n32 = L.zk_workspace_bytes(ctx)
    assert 0 < n32 < n64
    assert L.zk_set_option(ctx, zk.ZK_OPT_EPS, 1.5) == zk.ZK_EINVAL
    assert L.zk_set_option(ctx, 99, 0.0) == zk.ZK_EINVAL
    assert b"eps" in L.zk_last_error(ctx) or b"option" in L.zk_last_error(ctx)
    # calls before zk_bind report a missing workspace without touching a device
    assert L.zk_dtn(ctx, None, None, None) == zk.ZK_ENOWS
    assert L.zk_inverse_dtn(ctx, None, None, None, 8) == zk.ZK_ENOWS
    assert L.zk_depth_velocity(ctx, None, None, 1, None, None) == zk.ZK_ENOWS
    # team shapes by hand: T must split the transform (768 padded, 512 base) into a built shape
    for row, pad, T, ok in ((1, 1, 256, True), (1, 1, 128, True), (1, 1, 64, True), (1, 1, 512, False),
                            (1, 1, 32, False), (0, 0, 256, True), (0, 0, 64, True), (0, 0, 512, False),
                            (0, 0, 100, False), (1, 0, 0, True)):
        assert (L.zk_set_team_shape(ctx, row, pad, T) == 0) == ok, (row, pad, T)
    T, E = ctypes.c_int(0), ctypes.c_int(0)
    assert L.zk_set_team_shape(ctx, 1, 1, 128) == 0
    assert L.zk_team_shape(ctx, 1, 1, ctypes.byref(T), ctypes.byref(E)) == 0 and (T.value, E.value) == (128, 6)
    L.zk_destroy(ctx)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libzk.so not built")
def test_batch_create_host_checks():
    """zk_batch_create is host-only: it accepts valid tiles (workspace = the
    tiles' workspaces plus the argument and item tables) and rejects an
    invalid tile size, order or precision."""
    from paper_2608_25203_amd import zk

    L = zk.lib()
    good = (zk.ZkTile * 2)(zk.ZkTile(64, 64, 1.0, 1.0, 0.5, 3), zk.ZkTile(128, 64, 2.0, 1.0, math.inf, 5))
    b = L.zk_batch_create(2, good, 9.81, 32)
    assert b
    ws = L.zk_batch_workspace_bytes(b)
    c0 = L.zk_create(64, 64, 1.0, 1.0, 0.5, 9.81, 3)
    c1 = L.zk_create(128, 64, 2.0, 1.0, math.inf, 9.81, 5)
    for c in (c0, c1):
        assert L.zk_set_option(c, zk.ZK_OPT_PRECISION, 32) == 0
    assert ws > L.zk_workspace_bytes(c0) + L.zk_workspace_bytes(c1)
    L.zk_destroy(c0)
    L.zk_destroy(c1)
    L.zk_batch_destroy(b)
    for bad, prec in (((100, 64, 1.0, 1.0, 0.5, 3), 32), ((64, 64, 1.0, 1.0, 0.5, 9), 32),
                      ((64, 64, 1.0, 1.0, 0.5, 3), 16)):
        arr = (zk.ZkTile * 1)(zk.ZkTile(*bad))
        assert not L.zk_batch_create(1, arr, 9.81, prec)
    # stepping an unbound batch is an error, not a crash
    b = L.zk_batch_create(2, good, 9.81, 64)
    assert L.zk_batch_step(b, 0.01, 1) == zk.ZK_ENOWS
    L.zk_batch_destroy(b)


def test_generated_kernel_units_are_current(tmp_path):
    """The committed kernel-instance units equal what gen_batch_units.py
    writes now (a generator change must come with its units)."""
    import shutil
    import subprocess
    import sys

    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2608_25203_amd", "csrc")
    shutil.copy(os.path.join(csrc, "gen_batch_units.py"), tmp_path)
    subprocess.run([sys.executable, str(tmp_path / "gen_batch_units.py")], check=True)
    for kind in ("row", "col"):
        for tag in ("f64", "f32"):
            name = f"zk_batch_{kind}_{tag}.hip"
            with open(os.path.join(csrc, name)) as a, open(tmp_path / name) as b:
                assert a.read() == b.read(), name


@pytest.mark.parametrize("M", [2, 3, 5])
def test_schedule_algebra_1d_grid(M):
    """A 1D grid (ny = 1, the paper's Stokes-wave setting): no padding or
    transform along y, so the planner's fold factor is N / (3nx/2) and the
    taper's kNyq is the x axis's; the schedule executed literally equals the
    oracle's G psi, RHS and steps."""
    nx, L = 128, TWO_PI
    eta, psi = random_band_fields(nx, 1, 13, nx // 2 - 1, amplitude=0.02)
    I = Interp(nx, 1, L, 1.0, 0.8, 9.81, M)
    m = HOSModel(Grid(nx, 1, L, 1.0, 0.8), M)
    assert rel(I.dtn(eta, psi), m.dtn(eta, psi)) < 1e-13
    a, b = I.rhs(eta, psi)
    a0, b0 = m.rhs(eta, psi)
    assert rel(a, a0) < 1e-13 and rel(b, b0) < 1e-13
    s, t = I.step(eta, psi, 0.002, 2)
    s0, t0 = m.step(eta, psi, 0.002, 2)
    assert rel(s, s0) < 1e-13 and rel(t, t0) < 1e-13


def test_row_shape_table_is_current():
    """zk_row_shapes.hpp lists exactly the operation sequences (at most
    MAX_LEN ops) of the padded row programs the planner writes for HOS orders
    1 to 8, as gen_row_shapes.py collects them; and the C2 workload's
    programs (512^2, M = 4) and the 2048^2 M = 5 programs are all among them,
    so their padded row passes run compiled."""
    import re
    import sys

    from plan_interp import build_checker

    sys.path.insert(0, os.path.join(ROOT, "paper_2608_25203_amd", "csrc"))
    import gen_row_shapes as G

    txt = open(os.path.join(ROOT, "paper_2608_25203_amd", "csrc", "zk_row_shapes.hpp")).read()
    table = [tuple(int(x.rstrip("u"), 16) for x in row.split(", ")) for row in re.findall(r"\{(0x[^}]*)\}", txt)]
    lens = [int(x) for x in re.search(r"kRowShapeLen\[kRowShapes\] = \{([^}]*)\}", txt).group(1).split(", ")]
    assert [len(r) for r in table] == lens
    want = [tuple(G.word(o) for o in sh) for sh in G.collect(build_checker())]
    assert table == want
    for nx, M in ((512, 4), (2048, 5)):
        for sh in G.program_shapes(load_plan(nx, nx, M)):
            assert tuple(G.word(o) for o in sh) in table
