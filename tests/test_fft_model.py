"""Host model of the team FFT schedules in csrc/zk_fft.hpp (no GPU).

The model follows the kernels' own index arithmetic: the pass plan (radix-E
step in registers, then radix-4/2 passes), the pass-ordered twiddle table as
the host builds it (pass p's factor W^(r k step_p) at Ns_p - E + (r-1) Ns_p +
k, conjugated for the inverse sign), and the three forms: team_fft (result in
LDS, natural order), team_fft_keep (the last pass's butterfly j keeps
elements j + NB r in registers) and team_fft_t (the passes transposed, input
in that last-pass layout, output element t + T r in registers).  Each is
checked against numpy's FFT for every team shape the kernels compile."""
import numpy as np
import pytest

SHAPES = ([(T, E) for T in (32, 64, 128, 256) for E in (2, 3, 4, 6, 8, 12)] + [(512, E) for E in (2, 3, 4, 6)]
          + [(1024, 2), (1024, 3)] + [(T, E) for T in (16, 32, 64, 128, 256) for E in (6, 9)])
SHAPES = sorted(set(SHAPES))


def later_radix(T, p):
    rem = T
    for _ in range(1, p):
        rem //= 4 if rem % 4 == 0 else 2
    return 4 if rem % 4 == 0 else 2


def num_passes(T):
    n, rem = 1, T
    while rem > 1:
        rem //= 4 if rem % 4 == 0 else 2
        n += 1
    return n


def plan(T, E):
    """(p, Rp, nb, Ns, step) for the passes after the radix-E step"""
    N, out, ns = T * E, [], E
    for p in range(1, num_passes(T)):
        rp = later_radix(T, p)
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


@pytest.mark.parametrize("T,E", SHAPES)
def test_twiddle_table_slots_are_distinct_and_in_range(T, E):
    N, seen = T * E, set()
    for _, rp, _, ns, _ in plan(T, E):
        for r in range(1, rp):
            for k in range(ns):
                i = ns - E + (r - 1) * ns + k
                assert 0 <= i < N - E and i not in seen
                seen.add(i)
