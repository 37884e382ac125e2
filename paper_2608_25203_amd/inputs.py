"""Seeded synthetic input generators (no part of the method's arithmetic).

Both the CPU oracle tests and the GPU path take their inputs from here; the
module computes initial sea states and random test fields only.  Nothing in
it evaluates the DtN operator, products, filters or time steps.

* `jonswap_state`   random-phase sea state with a JONSWAP-shaped spectrum,
  cos^2 directional spreading about +x, psi from linear theory, rescaled to a
  target steepness k_p sqrt(2 <eta^2>).
* `random_band_fields`  smooth random real fields whose spectra live in
  |m_x|, |m_y| <= mmax (for parity and invariance tests).
* `WORKLOADS`       the five workload shapes used by tests and the bench.
"""
import math

import numpy as np


def _mode_ints(n):
    if n == 1:
        return np.zeros(1, dtype=np.int64)
    return np.rint(np.fft.fftfreq(n, 1.0 / n)).astype(np.int64)


def jonswap_state(nx, ny, Lx, Ly, depth, g, kp, steepness, seed, gamma=3.3, kmax=None):
    """Random-phase JONSWAP sea state (eta, psi), float64 arrays [ny][nx].

    omega(k) = sqrt(g |k| tanh(|k| h)) (deep: sqrt(g|k|));
    S_omega = g^2 omega^-5 exp(-1.25 (omega_p/omega)^4) gamma^r,
      r = exp(-(omega - omega_p)^2 / (2 sigma^2 omega_p^2)), sigma = 0.07 / 0.09;
    S_k = S_omega(omega(k)) d omega/dk; F(k) = S_k D(theta) / |k| with
    D = (2/pi) cos^2 theta for |theta| < pi/2 (2D) and D = 1 for kx > 0 (1D).
    Modes: every band mode with 0 < |k| <= min(4 k_p, kNyq/2) and D > 0,
    enumerated in array order (row-major over FFT-ordered (m_y, m_x));
    amplitude a = sqrt(2 F dkx dky), phase ~ U(0, 2 pi) from default_rng(seed)
    drawn in that order.  eta = sum a cos(k.x + phi),
    psi = sum (g a / omega) sin(k.x + phi); both rescaled by one factor so that
    k_p sqrt(2 <eta^2>) = steepness.
    """
    deep = depth is None or not np.isfinite(depth) or depth <= 0
    mx = _mode_ints(nx)[None, :]
    my = _mode_ints(ny)[:, None]
    kx = 2 * np.pi / Lx * mx * np.ones((ny, 1))
    ky = 2 * np.pi / Ly * my * np.ones((1, nx))
    kk = np.hypot(kx, ky)
    knyq = np.pi * nx / Lx if ny == 1 else min(np.pi * nx / Lx, np.pi * ny / Ly)
    klim = min(4.0 * kp, 0.5 * knyq) if kmax is None else kmax
    band = (np.abs(mx) <= nx // 2 - 1) & ((np.abs(my) <= ny // 2 - 1) if ny > 1 else True)

    with np.errstate(divide="ignore", invalid="ignore"):
        th = np.ones_like(kk) if deep else np.tanh(kk * depth)
        om = np.sqrt(g * kk * th)
        if deep:
            domdk = 0.5 * np.sqrt(g / np.maximum(kk, 1e-300))
        else:
            domdk = g * (th + kk * depth * (1.0 - th * th)) / (2.0 * np.maximum(om, 1e-300))
        omp = math.sqrt(g * kp * (1.0 if deep else math.tanh(kp * depth)))
        sig = np.where(om <= omp, 0.07, 0.09)
        r = np.exp(-((om - omp) ** 2) / (2.0 * sig * sig * omp * omp))
        s_om = g * g * om ** -5.0 * np.exp(-1.25 * (omp / om) ** 4) * gamma ** r
        s_k = s_om * domdk
        if ny > 1:
            theta = np.arctan2(ky, kx)
            spread = np.where(np.abs(theta) < np.pi / 2, (2.0 / np.pi) * np.cos(theta) ** 2, 0.0)
            F = s_k * spread / kk
        else:
            spread = np.where(kx > 0, 1.0, 0.0)
            F = s_k * spread
    sel = band & (kk > 0) & (kk <= klim) & (spread > 0)
    dkx = 2 * np.pi / Lx
    dky = 2 * np.pi / Ly if ny > 1 else 1.0
    amp = np.where(sel, np.sqrt(2.0 * np.where(sel, F, 0.0) * dkx * dky), 0.0)

    rng = np.random.default_rng(seed)
    iy, ix = np.nonzero(sel)  # row-major order
    phases = rng.uniform(0.0, 2.0 * np.pi, size=iy.size)

    # eta = Re sum a e^{i(k.x+phi)}; psi = Re sum (g a/omega)(-i) e^{i(k.x+phi)}.
    Z = np.zeros((ny, nx), dtype=complex)
    Zp = np.zeros((ny, nx), dtype=complex)
    a = amp[iy, ix] * np.exp(1j * phases)
    Z[iy, ix] = a
    Zp[iy, ix] = -1j * g * a / om[iy, ix]
    eta = np.real(np.fft.ifft2(Z)) * (nx * ny)
    psi = np.real(np.fft.ifft2(Zp)) * (nx * ny)
    rms = math.sqrt(float(np.mean(eta * eta)))
    scale = steepness / (kp * math.sqrt(2.0) * rms) if rms > 0 else 0.0
    return eta * scale, psi * scale


def random_band_fields(nx, ny, seed, mmax, nfields=2, amplitude=1.0, decay=0.0):
    """`nfields` smooth random real fields [ny][nx] whose Fourier modes lie in
    |m_x| <= mmax, |m_y| <= mmax (all modes inside, Nyquist never touched when
    mmax < n/2).  Coefficients are complex normal times exp(-decay |m|^2),
    then each field is scaled to max |f| = amplitude."""
    rng = np.random.default_rng(seed)
    mx = _mode_ints(nx)[None, :]
    my = _mode_ints(ny)[:, None]
    sel = (np.abs(mx) <= mmax) & (np.abs(my) <= (mmax if ny > 1 else 0))
    out = []
    for _ in range(nfields):
        C = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx)))
        C = C * sel * np.exp(-decay * (mx * mx + my * my))
        f = np.real(np.fft.ifft2(C))
        m = np.max(np.abs(f))
        out.append(f * (amplitude / m if m > 0 else 0.0))
    return out


# Workload shapes (sizes, physics, initial-state recipe).  C1 is the small
# case the oracle finishes in seconds; C2 is the FP64 throughput workload.
WORKLOADS = {
    "c1_64_m3": dict(nx=64, ny=64, Lx=2 * np.pi, Ly=2 * np.pi, depth=math.inf, g=9.81, M=3,
                     dt=0.01, steps=100, kp=4.0, steepness=0.05, seed=0),
    "c2_512_m4": dict(nx=512, ny=512, Lx=200.0, Ly=200.0, depth=20.0, g=9.81, M=4,
                      dt=0.05, steps=1000, kp=2 * np.pi / 12.5, steepness=0.1, seed=1),
    # peak at kNyq / 16 (32 grid points per peak wavelength), dt = T_p / 50
    "c3_2048_m5": dict(nx=2048, ny=2048, Lx=2 * np.pi, Ly=2 * np.pi, depth=math.inf, g=9.81, M=5,
                       dt=0.005, steps=500, kp=64.0, steepness=0.15, seed=2),
    "c5_1024_m6": dict(nx=1024, ny=1024, Lx=2 * np.pi, Ly=2 * np.pi, depth=math.inf, g=9.81, M=6,
                       dt=0.007, steps=1000, kp=32.0, steepness=0.1, seed=42),
}


def workload_state(name, **over):
    w = dict(WORKLOADS[name])
    w.update(over)
    eta, psi = jonswap_state(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"],
                             w["kp"], w["steepness"], w["seed"])
    return w, eta, psi


def tank_bump(nx, ny, Lx, Ly, A, sigma=1.0, R=6.0):
    """The wave-propagation tank's initial state: a Gaussian bump
    A exp(-r^2 / (2 sigma^2)) for r < R (zero outside), r measured from the
    tank centre, on cell-centred samples ((i + 1/2) Lx / nx, ...); the
    surface at rest, psi = 0.  float64 arrays [ny][nx]."""
    x = (np.arange(nx) + 0.5) * Lx / nx - 0.5 * Lx
    y = (np.arange(ny) + 0.5) * Ly / ny - 0.5 * Ly
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    eta = np.where(r2 < R * R, A * np.exp(-r2 / (2.0 * sigma * sigma)), 0.0)
    return eta, np.zeros_like(eta)


def cnn_init_params(seed, channels=(3, 32, 32, 32, 1)):
    """Seeded initial weights of the closure network: for each layer a
    (C_out, C_in, 3, 3) weight drawn N(0, 2 / (9 C_in)) (He) and a zero bias
    (C_out,); the last layer's weights are scaled by 0.1 so the initial
    prediction is small.  float64 arrays, in parameter order W1, b1, ... ."""
    rng = np.random.default_rng(seed)
    out = []
    nl = len(channels) - 1
    for l in range(nl):
        ci, co = channels[l], channels[l + 1]
        w = rng.standard_normal((co, ci, 3, 3)) * math.sqrt(2.0 / (9 * ci))
        if l == nl - 1:
            w *= 0.1
        out.append(w)
        out.append(np.zeros(co))
    return out
