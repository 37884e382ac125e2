"""Host model of the team FFT schedules in csrc/zk_fft.hpp (no GPU).

The model follows the kernels' own index arithmetic: the pass plan (radix-E
step in registers, then radix-4/2 passes, radix 8 first for teams of 1024
threads and of 128 or more with E >= 6), the pass-ordered twiddle table as
the host builds it (pass p's factor W^(r k step_p) at Ns_p - E + (r-1) Ns_p +
k, conjugated for the inverse sign), and the three forms: team_fft (result in
LDS, natural order), team_fft_keep (the last pass's butterfly j keeps
elements j + NB r in registers) and team_fft_t (the passes transposed, input
in that last-pass layout, output element t + T r in registers).  Each is
checked against numpy's FFT for every team shape the kernels compile; so are
the permuted-layout forms of the padded row passes (perm_ifft, perm_fft)."""
import numpy as np
import pytest

SHAPES = ([(T, E) for T in (2, 4, 8, 16) for E in (2, 3, 4, 6)]
          + [(T, E) for T in (32, 64, 128, 256) for E in (2, 3, 4, 6, 8, 12)] + [(512, E) for E in (2, 3, 4, 6)]
          + [(1024, 2), (1024, 3)] + [(T, E) for T in (2, 4, 8, 16, 32, 64, 128, 256) for E in (6, 9)]
          + [(T, E) for T in (2, 4, 8, 16, 32, 64, 128) for E in (10, 15)])
SHAPES = sorted(set(SHAPES))


def pass_radix(T, E, rem):
    if (T >= 1024 or (T >= 128 and E >= 6)) and rem % 8 == 0 and rem != 16:
        return 8
    return 4 if rem % 4 == 0 else 2


def later_radix(T, E, p):
    rem = T
    for _ in range(1, p):
        rem //= pass_radix(T, E, rem)
    return pass_radix(T, E, rem)


def num_passes(T, E):
    n, rem = 1, T
    while rem > 1:
        rem //= pass_radix(T, E, rem)
        n += 1
    return n


def plan(T, E):
    """(p, Rp, nb, Ns, step) for the passes after the radix-E step"""
    N, out, ns = T * E, [], E
    for p in range(1, num_passes(T, E)):
        rp = later_radix(T, E, p)
        out.append((p, rp, N // rp, ns, N // (ns * rp)))
        ns *= rp
    return out


def table(T, E):
    """the host's pass-ordered twiddle table for (N, E), forward sign"""
    N = T * E
    tab = np.full(N - E, np.nan + 0j)
    for _, rp, _, ns, step in plan(T, E):
        for r in range(1, rp):
            for k in range(ns):
                tab[ns - E + (r - 1) * ns + k] = np.exp(-2j * np.pi * r * k * step / N)
    return tab


def small_dft(x, DIR):
    n = np.arange(len(x))
    return np.exp(DIR * 2j * np.pi * np.outer(n, n) / len(x)) @ x


def twid(tab, ns, E, r, k, DIR):
    w = tab[ns - E + (r - 1) * ns + k]
    return np.conj(w) if DIR > 0 else w


def team_fft(x, T, E, DIR, keep=False):
    N, tab = T * E, table(T, E)
    buf = np.zeros(N, complex)
    for t in range(T):
        v = small_dft(x[t + T * np.arange(E)], DIR)
        buf[t * E + np.arange(E)] = v
    kept = np.full(N, np.nan + 0j)
    passes = plan(T, E)
    for p, rp, nb, ns, step in passes:
        out = np.zeros(N, complex)
        for j in range(nb):
            k = j % ns
            w = buf[j + nb * np.arange(rp)].copy()
            for r in range(1, rp):
                w[r] *= twid(tab, ns, E, r, k, DIR)
            w = small_dft(w, DIR)
            base = (j // ns) * ns * rp + k
            if keep and p == passes[-1][0]:
                assert base == j
                kept[j + nb * np.arange(rp)] = w
            else:
                out[base + ns * np.arange(rp)] = w
        buf = out
    return kept if keep else buf


def team_fft_t(x, T, E, DIR):
    N, tab = T * E, table(T, E)
    buf = None
    for p, rp, nb, ns, step in reversed(plan(T, E)):
        out = np.zeros(N, complex)
        for j in range(nb):
            k = j % ns
            base = (j // ns) * ns * rp + k
            src = x if buf is None else buf  # the last pass's gather is the register layout (base = j)
            if buf is None:
                assert base == j
            w = small_dft(src[base + ns * np.arange(rp)], DIR)
            for r in range(1, rp):
                w[r] *= twid(tab, ns, E, r, k, DIR)
            out[j + nb * np.arange(rp)] = w
        buf = out
    res = np.zeros(N, complex)
    for t in range(T):
        res[t + T * np.arange(E)] = small_dft(buf[t * E + np.arange(E)], DIR)
    return res


@pytest.mark.parametrize("T,E", SHAPES)
def test_team_fft_forms_match_numpy(T, E):
    N = T * E
    x = np.random.default_rng(T * 100 + E).standard_normal((N, 2)) @ np.array([1, 1j])
    for DIR in (-1, 1):
        ref = np.fft.fft(x) if DIR < 0 else np.fft.ifft(x) * N
        scale = np.abs(ref).max()
        for got in (team_fft(x, T, E, DIR), team_fft(x, T, E, DIR, keep=True), team_fft_t(x, T, E, DIR)):
            assert np.abs(got - ref).max() / scale < 1e-13


def reg_dft(x, DIR):
    """the kernels' in-register DFT: closed butterflies for 2, 3, 4 and 5 points
    (5: sums and differences of the mirrored pairs), else RR = A B with A = 4,
    2 or 3 first, twiddle W_RR^(n2 k1), then B-point DFTs"""
    RR = len(x)
    if RR <= 4:
        return small_dft(x, DIR)
    if RR == 5:
        c1, s1, c2, s2 = np.cos(2 * np.pi / 5), np.sin(2 * np.pi / 5), np.cos(4 * np.pi / 5), np.sin(4 * np.pi / 5)
        t1, t2, t3, t4 = x[1] + x[4], x[2] + x[3], x[1] - x[4], x[2] - x[3]
        a1, a2 = x[0] + c1 * t1 + c2 * t2, x[0] + c2 * t1 + c1 * t2
        b1, b2 = DIR * 1j * (s1 * t3 + s2 * t4), DIR * 1j * (s2 * t3 - s1 * t4)
        return np.array([x[0] + t1 + t2, a1 + b1, a2 + b2, a2 - b2, a1 - b1])
    A = 4 if RR % 4 == 0 else (2 if RR % 2 == 0 else 3)
    B = RR // A
    y = np.zeros((B, A), complex)
    for n2 in range(B):
        t = reg_dft(x[B * np.arange(A) + n2], DIR)
        y[n2] = t * np.exp(DIR * 2j * np.pi * n2 * np.arange(A) / RR)
    out = np.zeros(RR, complex)
    for k1 in range(A):
        out[k1 + A * np.arange(B)] = reg_dft(y[:, k1], DIR)
    return out


@pytest.mark.parametrize("RR", (2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 18))
def test_register_dft_decomposition_matches_numpy(RR):
    x = np.random.default_rng(RR).standard_normal((RR, 2)) @ np.array([1, 1j])
    for DIR in (-1, 1):
        ref = np.fft.fft(x) if DIR < 0 else np.fft.ifft(x) * RR
        assert np.abs(reg_dft(x, DIR) - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("T,E", SHAPES)
def test_twiddle_table_slots_are_distinct_and_in_range(T, E):
    N, seen = T * E, set()
    for _, rp, _, ns, _ in plan(T, E):
        for r in range(1, rp):
            for k in range(ns):
                i = ns - E + (r - 1) * ns + k
                assert 0 <= i < N - E and i not in seen
                seen.add(i)


# ---- the permuted-layout forms (perm_ifft / perm_fft) --------------------------
# Team of T = 64 W threads, thread t = 64 w + l; twiddles from the natural table
# W_N^m (forward sign, conjugated for DIR > 0).  Index arithmetic as in the
# kernels: radix-E step and W_N^(64 w q); wavefront stages (radix 4 over spans
# (hw, hw/2) while two bits remain, else radix 2), decimation in frequency for
# the inverse; W_N^(l (q + E bitrev(w))); six radix-2 lane stages l ^ h.
LANE_SHAPES = [(T, E) for T, E in SHAPES if T % 64 == 0 and E % 3 == 0 and E % 5 != 0]


def natural(N, m, DIR):
    w = np.exp(-2j * np.pi * m / N)
    return np.conj(w) if DIR > 0 else w


def bitrev(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2) if bits else 0


def xw_spans(W):
    out, hw = [], W // 2
    while hw >= 1:
        out.append(hw)
        hw = hw // 4 if hw >= 2 else hw // 2
    return out


def lane_stages(V, N, DIR, dif):
    l = np.arange(64)
    for h in ([32, 16, 8, 4, 2, 1] if dif else [1, 2, 4, 8, 16, 32]):
        B = (l & h) != 0
        sg = np.where(B, -1.0, 1.0)[:, None]
        ws = np.array([natural(N, (li & (h - 1)) * (N // (2 * h)), DIR) if (li & h) and h > 1 else 1.0
                       for li in l])[:, None]
        if dif:
            V = (V[l ^ h] + sg * V) * ws
        else:
            c = V * ws
            V = c[l ^ h] + sg * c
    return V


def xw_stage(v, T, E, N, hw, DIR, dif):
    out = np.zeros_like(v)
    iD = 1j * DIR
    for t in range(T):
        w = t // 64
        if hw == 1:
            p = v[t ^ 64]
            out[t] = (p - v[t]) if w & 1 else v[t] + p
            continue
        h2 = hw // 2
        t0 = t & ~(96 * hw)
        w0 = w & ~(hw | h2)
        B1, B0 = w & hw, w & h2
        w1 = natural(N, (w0 % hw) * (N // (2 * hw)), DIR)
        w2 = natural(N, (w0 % h2) * (N // hw), DIR)
        i0, i1, i2, i3 = v[t0], v[t0 + 32 * hw], v[t0 + 64 * hw], v[t0 + 96 * hw]
        if dif:
            x0 = (i0 - i2) * w1 if B1 else i0 + i2
            x1 = (i1 - i3) * w1 * iD if B1 else i1 + i3
            out[t] = (x0 - x1) * w2 if B0 else x0 + x1
        else:
            c = i0 - w2 * i1 if B0 else i0 + w2 * i1
            d = i2 - w2 * i3 if B0 else i2 + w2 * i3
            fd = d * w1 * iD if B0 else d * w1
            out[t] = c - fd if B1 else c + fd
    return out


def perm_ifft(x, T, E, DIR):
    N, W = T * E, T // 64
    v = np.array([small_dft(x[t + T * np.arange(E)], DIR) for t in range(T)])
    for t in range(T):
        v[t] *= natural(N, 64 * (t // 64) * np.arange(E), DIR)
    for hw in xw_spans(W):
        v = xw_stage(v, T, E, N, hw, DIR, True)
    for t in range(T):
        kb = bitrev(t // 64, W.bit_length() - 1)
        v[t] *= natural(N, (t % 64) * (np.arange(E) + E * kb), DIR)
    for w in range(W):
        v[64 * w:64 * w + 64] = lane_stages(v[64 * w:64 * w + 64], N, DIR, True)
    return v


def perm_fft(y, T, E, DIR):
    N, W = T * E, T // 64
    v = y.copy()
    for w in range(W):
        v[64 * w:64 * w + 64] = lane_stages(v[64 * w:64 * w + 64], N, DIR, False)
    for t in range(T):
        kb = bitrev(t // 64, W.bit_length() - 1)
        v[t] *= natural(N, (t % 64) * (np.arange(E) + E * kb), DIR)
    for hw in reversed(xw_spans(W)):
        v = xw_stage(v, T, E, N, hw, DIR, False)
    for t in range(T):
        v[t] *= natural(N, 64 * (t // 64) * np.arange(E), DIR)
    return np.array([small_dft(v[t], DIR) for t in range(T)])


def lanes_perm(T, E):
    W = T // 64
    return np.array([[s + E * bitrev(t // 64, W.bit_length() - 1) + E * W * bitrev(t % 64, 6) for s in range(E)]
                     for t in range(T)])


@pytest.mark.parametrize("T,E", LANE_SHAPES)
def test_permuted_forms_match_numpy(T, E):
    """perm_ifft: natural order in, the transform at point s + E bitrev(w) +
    E W bitrev6(l) in thread t's register s; perm_fft: that order in, natural
    order out (element t + T r in register r); both against numpy's FFT."""
    N = T * E
    P = lanes_perm(T, E)
    assert sorted(P.ravel().tolist()) == list(range(N))
    rng = np.random.default_rng(T * 7 + E)
    x = rng.standard_normal((N, 2)) @ np.array([1, 1j])
    ref = np.fft.ifft(x) * N
    assert np.abs(perm_ifft(x, T, E, +1) - ref[P]).max() / np.abs(ref).max() < 1e-13
    F = np.fft.fft(x)
    got = perm_fft(x[P], T, E, -1)
    want = np.array([[F[t + T * r] for r in range(E)] for t in range(T)])
    assert np.abs(got - want).max() / np.abs(F).max() < 1e-13
