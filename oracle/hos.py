"""Plain FP64 reference of the Zakharov/HOS wave step (test infrastructure only).

What it computes, and where each step comes from in the paper
(Hamiltonian Two-Way Coupling of Nonlinear Waves and 3D Flows, ACM TOG 2026):

* State: the canonical pair (eta, psi) on a periodic nx x ny grid
  (Sec. 3.1, canonical Zakharov formulation).
* Flat-state DNO symbol G0(k) = |k| tanh(|k| d) (Sec. 3.2, eq:G0) and the
  multiplier B0 with symbol |k|^2 (Sec. 3.2, below eq:G2).
* The Craig-Sulem / HOS expansion G = sum_j eps^j G_j (Sec. 3.2, eq:G1,
  eq:G2, eq:dno_truncated), generated to any order M by the surface-potential
  recursion Phi^(m) of Sec. 4.2 (eq:phi0, eq:phi1, eq:phi2).  Order M keeps
  G_0 .. G_{M-1}, so the paper's "Order 3 / HOS-3" is M = 3 (Sec. 3.2, last
  paragraph).  `dtn_explicit` evaluates eq:G1 and eq:G2 literally for M <= 3.
* The truncated Bernoulli equation with W (Sec. 3.2, eq:dyn_truncated, eq:W),
  which at eps = 1 is the exact dynamic condition eq:zakharov_dyn.
* 3/2-rule dealiasing of every product and the super-Gaussian taper
  exp(-(|k|/kc)^8), kc = 2/3 kNyq, on every nonlinear product (Sec. 6.1).
* The spectral state filter A(k) applied after each full step
  (Sec. 3.4, eq:state_filter).
* The Hamiltonian H = 1/2 int psi G psi + 1/2 g int eta^2 (Sec. 3.1,
  eq:hamiltonian).
* Time stepping: classical RK4 on the spectral state (the paper's own
  integrator, IF-AB2 of Sec. 3.4, is not used on this path).

Readings taken where the paper is silent:
  R1  order M keeps G_0..G_{M-1};  R2  G_j for j >= 3 from the Phi^(m)
  recursion;  R3  higher powers of eta are nested dealiased pairwise products
  eta^<l> = P(eta, eta^<l-1>);  R4  the taper sits inside every product P,
  including the Bernoulli fold;  R5  kNyq = min over axes;  R6  the Bernoulli
  term is evaluated pointwise on the padded grid from band-limited factors and
  folded once;  R7  A(k) once per full RK4 step;  R9  Nyquist rows/columns of
  every spectrum are zero;  R11 eps defaults to 1.

DFT convention: forward unnormalised, f_hat(k) = sum_x f(x) e^{-i k.x};
inverse carries 1/N.  Spectra are full complex (ny, nx) arrays in FFT order.
"""
import math

import numpy as np
import scipy.fft


# ----------------------------------------------------------------------------
# DFT backends
# ----------------------------------------------------------------------------
class NaiveDFT:
    """Dense DFT matrices applied along each axis (O(n^3)); correctness only."""

    name = "naive"

    def __init__(self):
        self._cache = {}

    def _mat(self, n, sign):
        key = (n, sign)
        w = self._cache.get(key)
        if w is None:
            j = np.arange(n)
            e = np.outer(j, j) % n  # exact integer phase index
            w = np.exp(sign * 2j * np.pi * e / n)
            self._cache[key] = w
        return w

    def fft2(self, f):
        ny, nx = f.shape
        return self._mat(ny, -1) @ np.asarray(f, dtype=complex) @ self._mat(nx, -1)

    def ifft2(self, F):
        ny, nx = F.shape
        return (self._mat(ny, +1) @ F @ self._mat(nx, +1)) / (nx * ny)


class PocketDFT:
    """pocketfft through scipy.fft; `workers` threads (None = 1)."""

    name = "pocketfft"

    def __init__(self, workers=None):
        self.workers = workers

    def fft2(self, f):
        return scipy.fft.fft2(np.asarray(f, dtype=complex), workers=self.workers)

    def ifft2(self, F):
        return scipy.fft.ifft2(F, workers=self.workers)


# ----------------------------------------------------------------------------
# Grid, wavenumbers, multipliers
# ----------------------------------------------------------------------------
class Grid:
    """Periodic grid x_i = i Lx/nx, y_j = j Ly/ny; arrays are [ny][nx].

    ny == 1 is the one-dimensional model ("one dimension lower", Sec. 3).
    depth <= 0, None or inf means deep water (tanh -> 1).
    pad: padded size per axis for the dealiased product, "3/2" (Sec. 6.1) or
    "2" (also alias-free for quadratic products; used by a pin).
    """

    def __init__(self, nx, ny, Lx, Ly, depth, g=9.81, pad="3/2", dft=None):
        if nx < 4 or nx % 2 or (ny != 1 and (ny < 4 or ny % 2)):
            raise ValueError("nx must be even >= 4; ny even >= 4 or 1")
        self.nx, self.ny, self.Lx, self.Ly, self.g = nx, ny, float(Lx), float(Ly), float(g)
        self.N = nx * ny
        self.deep = depth is None or not np.isfinite(depth) or depth <= 0
        self.h = math.inf if self.deep else float(depth)
        self.dft = dft if dft is not None else PocketDFT()

        mx = np.rint(np.fft.fftfreq(nx, 1.0 / nx)).astype(np.int64)
        my = np.rint(np.fft.fftfreq(ny, 1.0 / ny)).astype(np.int64) if ny > 1 else np.zeros(1, np.int64)
        self.mx, self.my = mx, my
        ones = np.ones((ny, nx))
        self.kx = (2 * np.pi / self.Lx) * mx[None, :] * ones
        self.ky = (2 * np.pi / self.Ly) * my[:, None] * ones
        self.kk = np.hypot(self.kx, self.ky)
        self.th = np.ones_like(self.kk) if self.deep else np.tanh(self.kk * self.h)

        # Band B: |m_x| <= nx/2 - 1, |m_y| <= ny/2 - 1; Nyquist excluded (R9).
        bx = np.abs(mx) <= nx // 2 - 1
        by = (np.abs(my) <= ny // 2 - 1) if ny > 1 else np.ones(1, bool)
        self.band = by[:, None] & bx[None, :]
        self.ix_b = np.nonzero(bx)[0]
        self.iy_b = np.nonzero(by)[0]

        # Padded grid for the dealiased product (Sec. 6.1).
        if pad == "3/2":
            self.px, self.py = 3 * nx // 2, (3 * ny // 2 if ny > 1 else 1)
        elif pad == "2":
            self.px, self.py = 2 * nx, (2 * ny if ny > 1 else 1)
        else:
            raise ValueError(pad)
        self.Np = self.px * self.py
        self.ix_p = mx[self.ix_b] % self.px
        self.iy_p = my[self.iy_b] % self.py

        # Taper exp(-(|k|/kc)^8), kc = 2/3 kNyq, kNyq = min over axes (R5).
        knyq = np.pi * nx / self.Lx
        if ny > 1:
            knyq = min(knyq, np.pi * ny / self.Ly)
        self.kc = 2.0 / 3.0 * knyq
        self.taper = np.exp(-((self.kk / self.kc) ** 8))

        # State filter A(k) (Sec. 3.4, eq:state_filter); pi|k_a|/kNyq_a = 2 pi |m_a| / n_a.
        def a1(m, n):
            th = 2.0 * np.pi * np.abs(m) / n
            return (5.0 + 4.0 * np.cos(th) - np.cos(2.0 * th)) / 8.0

        ay = a1(my, ny) if ny > 1 else np.ones(1)
        self.filt = ay[:, None] * a1(mx, nx)[None, :]

    # -- spectral helpers ----------------------------------------------------
    def L(self, l):
        """d_z^l of the flat-state harmonic extension cosh(|k|(z+d))/cosh(|k|d)
        at z = 0: |k|^l tanh(|k|d) for odd l, |k|^l for even l.  L(1) = G0
        (eq:G0), L(2) = B0, L(3) = G0 B0."""
        return self.kk ** l * (self.th if l % 2 else 1.0)

    @property
    def G0(self):
        return self.L(1)

    @property
    def B0(self):
        return self.kk ** 2

    def spec(self, f):
        """Forward DFT of a physical field, projected onto the band B."""
        return self.dft.fft2(np.asarray(f, dtype=float)) * self.band

    def phys(self, F):
        """Inverse DFT of a band spectrum back to the base grid (real part)."""
        return self.dft.ifft2(F).real

    def pad(self, F):
        out = np.zeros((self.py, self.px), dtype=complex)
        out[np.ix_(self.iy_p, self.ix_p)] = F[np.ix_(self.iy_b, self.ix_b)]
        return out

    def trunc(self, C):
        out = np.zeros((self.ny, self.nx), dtype=complex)
        out[np.ix_(self.iy_b, self.ix_b)] = C[np.ix_(self.iy_p, self.ix_p)]
        return out

    def lift(self, F):
        """Band spectrum -> values of its trigonometric interpolant on the
        padded grid: (1/N) sum_k F(k) e^{i k.x_p}."""
        return self.dft.ifft2(self.pad(F)).real * (self.Np / self.N)

    def fold(self, c, taper=True):
        """Padded physical values -> base-band spectrum, truncated to B and
        (taper=True) multiplied by the taper (Sec. 6.1)."""
        C = self.trunc(self.dft.fft2(c)) * (self.N / self.Np)
        return C * self.taper if taper else C


# ----------------------------------------------------------------------------
# The model
# ----------------------------------------------------------------------------
class HOSModel:
    """Zakharov/HOS model of order M on a Grid.

    eps    nonlinear-amplitude dial (Sec. 3.2, eq:dno_truncated); 1 = exact.
    taper  apply the super-Gaussian taper inside every product (Sec. 6.1).
    filt   apply A(k) after each RK4 step (Sec. 3.4, eq:state_filter).
    """

    def __init__(self, grid, M, eps=1.0, taper=True, filt=True):
        if M < 1:
            raise ValueError("M >= 1")
        self.gr, self.M, self.eps, self.taper, self.filt = grid, int(M), float(eps), bool(taper), bool(filt)

    # -- dealiased product (Sec. 6.1) -----------------------------------------
    def P(self, A, B):
        """T * Trunc_B[ (a b) ] for band spectra A, B: both factors are
        zero-padded, multiplied on the padded grid and truncated back."""
        g = self.gr
        return g.fold(g.lift(A) * g.lift(B), taper=self.taper)

    # -- DtN operator -------------------------------------------------------------
    def dtn_terms(self, eta_h, psi_h):
        """Homogeneous DNO terms [G_0 psi, ..., G_{M-1} psi] (spectra).

        Phi(x, eta) = sum_m sum_l eta^l/l! d_z^l Phi^(m)(x, 0) = psi order by
        order gives Phi^(0) = psi and
            Phi^(m) = - sum_{l=1..m} (1/l!) eta^l L_l Phi^(m-l)
        (Sec. 4.2, eq:phi0..eq:phi2 are m = 0, 1, 2).  The vertical velocity
        at the surface, W = d_z Phi |_{z=eta}, has homogeneous parts
            W_j = L_1 Phi^(j) + sum_{l=1..j} (1/l!) eta^l L_{l+1} Phi^(j-l),
        and G psi = (1 + |grad eta|^2) W - grad eta . grad psi, so
            G_0 = W_0,  G_1 = W_1 - grad eta . grad psi,
            G_j = W_j + |grad eta|^2 W_{j-2}   (j >= 2).
        For M <= 3 this equals eq:G1 / eq:G2 exactly (see dtn_explicit).
        Every product is the dealiased P; eta^l is the nested chain R3.
        """
        g, P, M = self.gr, self.P, self.M
        Dx, Dy = 1j * g.kx, 1j * g.ky
        etap = {1: eta_h}
        for l in range(2, M):
            etap[l] = P(eta_h, etap[l - 1])
        Phi = [psi_h]
        for m in range(1, M):
            acc = np.zeros_like(psi_h)
            for l in range(1, m + 1):
                acc = acc - P(etap[l], g.L(l) * Phi[m - l]) / math.factorial(l)
            Phi.append(acc)
        W = []
        for j in range(M):
            w = g.L(1) * Phi[j]
            for l in range(1, j + 1):
                w = w + P(etap[l], g.L(l + 1) * Phi[j - l]) / math.factorial(l)
            W.append(w)
        G = [W[0]]
        if M >= 2:
            G.append(W[1] - P(Dx * eta_h, Dx * psi_h) - P(Dy * eta_h, Dy * psi_h))
        if M >= 3:
            S = P(Dx * eta_h, Dx * eta_h) + P(Dy * eta_h, Dy * eta_h)
            for j in range(2, M):
                G.append(W[j] + P(S, W[j - 2]))
        return G

    def dtn_spec(self, eta_h, psi_h):
        """G^[M](eta) psi = sum_{j<M} eps^j G_j(eta) psi  (eq:dno_truncated)."""
        G = self.dtn_terms(eta_h, psi_h)
        out = np.zeros_like(psi_h)
        for j, gj in enumerate(G):
            out = out + self.eps ** j * gj
        return out

    def dtn_explicit(self, eta_h, psi_h):
        """eq:G0, eq:G1, eq:G2 written out literally (M <= 3), every product
        taken as the dealiased P, eta^2 = P(eta, eta), |grad eta|^2 =
        P(eta_x, eta_x) + P(eta_y, eta_y)."""
        if self.M > 3:
            raise ValueError("explicit formulas exist for M <= 3 only")
        g, P, e = self.gr, self.P, self.eps
        G0, B0 = g.G0, g.B0
        Dx, Dy = 1j * g.kx, 1j * g.ky
        g0psi = G0 * psi_h
        out = g0psi.copy()
        if self.M >= 2:
            div = Dx * P(eta_h, Dx * psi_h) + Dy * P(eta_h, Dy * psi_h)
            G1 = -G0 * P(eta_h, g0psi) - div
            out = out + e * G1
        if self.M >= 3:
            eta2 = P(eta_h, eta_h)
            grad2 = P(Dx * eta_h, Dx * eta_h) + P(Dy * eta_h, Dy * eta_h)
            G2 = (G0 * P(eta_h, G0 * P(eta_h, g0psi))
                  - 0.5 * G0 * P(eta2, B0 * psi_h)
                  - P(eta_h, B0 * P(eta_h, g0psi))
                  + 0.5 * P(eta2, G0 * (B0 * psi_h))
                  + P(grad2, g0psi))
            out = out + e * e * G2
        return out

    # -- Bernoulli and RHS ---------------------------------------------------------
    def bernoulli_spec(self, eta_h, psi_h, G_h):
        """Nonlinear part of d_t psi (eq:dyn_truncated with eq:W):
            S = 1 + eps^2 |grad eta|^2,  W = (G psi + eps grad eta . grad psi) / S,
            N = eps [ -1/2 |grad psi|^2 + 1/2 S W^2 ],
        evaluated pointwise on the padded grid and folded once (R6)."""
        g, e = self.gr, self.eps
        Dx, Dy = 1j * g.kx, 1j * g.ky
        ex, ey = g.lift(Dx * eta_h), g.lift(Dy * eta_h)
        qx, qy = g.lift(Dx * psi_h), g.lift(Dy * psi_h)
        G = g.lift(G_h)
        S = 1.0 + e * e * (ex * ex + ey * ey)
        W = (G + e * (ex * qx + ey * qy)) / S
        N = e * (-0.5 * (qx * qx + qy * qy) + 0.5 * S * W * W)
        return g.fold(N, taper=self.taper)

    def rhs_spec(self, eta_h, psi_h):
        """(d_t eta, d_t psi) = (G psi, -g eta + N)  (eq:zakharov_kin,
        eq:dyn_truncated)."""
        G = self.dtn_spec(eta_h, psi_h)
        Nh = self.bernoulli_spec(eta_h, psi_h, G)
        return G, -self.gr.g * eta_h + Nh

    # -- time stepping -------------------------------------------------------------
    def step_spec(self, eta_h, psi_h, dt, nsteps=1):
        """Classical RK4 with fixed dt, then A(k) after every full step."""
        for _ in range(int(nsteps)):
            k1 = self.rhs_spec(eta_h, psi_h)
            k2 = self.rhs_spec(eta_h + 0.5 * dt * k1[0], psi_h + 0.5 * dt * k1[1])
            k3 = self.rhs_spec(eta_h + 0.5 * dt * k2[0], psi_h + 0.5 * dt * k2[1])
            k4 = self.rhs_spec(eta_h + dt * k3[0], psi_h + dt * k3[1])
            eta_h = eta_h + dt / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
            psi_h = psi_h + dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
            if self.filt:
                eta_h = eta_h * self.gr.filt
                psi_h = psi_h * self.gr.filt
        return eta_h, psi_h

    # -- exact-linear Adams-Bashforth 2 (Sec. 3.4) -----------------------------------
    def if_coefficients(self, dt):
        """Per-mode coefficients of the exact linear flow (eq:lin_prop) and of
        its response to a forcing held constant over the step (the Duhamel
        integral behind eq:if_ab2_eta and eq:if_ab2_psi), omega = sqrt(g G0):
            c = cos(omega dt), a = G0 sin(omega dt) / omega, b = g sin(omega dt) / omega,
            s = sin(omega dt) / omega, u = (1 - c) / g, v = (1 - c) / G0,
        with the k = 0 limits a = 0, b = g dt, s = dt, u = 0, v = g dt^2 / 2."""
        g = self.gr
        G0 = g.G0
        om = np.sqrt(g.g * G0)
        zero = om == 0
        oms = np.where(zero, 1.0, om)
        c = np.cos(om * dt)
        sn = np.sin(om * dt)
        s = np.where(zero, dt, sn / oms)
        a = np.where(zero, 0.0, G0 * sn / oms)
        b = np.where(zero, g.g * dt, g.g * sn / oms)
        u = (1.0 - c) / g.g
        v = np.where(zero, 0.5 * g.g * dt * dt, (1.0 - c) / np.where(zero, 1.0, G0))
        return c, a, b, s, u, v

    def forcing_spec(self, eta_h, psi_h):
        """Nonlinear forcing of eq:split: (F_eta, F_psi) = (G^[M] psi - G0 psi, N),
        everything of the RHS beyond the linear part L = [[0, G0], [-g, 0]]."""
        G = self.dtn_spec(eta_h, psi_h)
        return G - self.gr.G0 * psi_h, self.bernoulli_spec(eta_h, psi_h, G)

    def if_propagate(self, eta_h, psi_h, Fe, Fp, dt):
        """One step of the exact linear flow plus the response to a forcing
        (Fe, Fp) held constant over the step (eq:if_ab2_eta, eq:if_ab2_psi)."""
        c, a, b, s, u, v = self.if_coefficients(dt)
        return (c * eta_h + a * psi_h + s * Fe + u * Fp,
                -b * eta_h + c * psi_h - v * Fe + s * Fp)

    def step_ifab2_spec(self, eta_h, psi_h, dt, nsteps=1):
        """IF-AB2 (Sec. 3.4): F* = 3/2 F_n - 1/2 F_{n-1}, the first step
        bootstrapped with F* = F_0 (integrating-factor Euler), then A(k)
        after every step."""
        prev = None
        for _ in range(int(nsteps)):
            Fe, Fp = self.forcing_spec(eta_h, psi_h)
            if prev is None:
                Se, Sp = Fe, Fp
            else:
                Se, Sp = 1.5 * Fe - 0.5 * prev[0], 1.5 * Fp - 0.5 * prev[1]
            prev = (Fe, Fp)
            eta_h, psi_h = self.if_propagate(eta_h, psi_h, Se, Sp, dt)
            if self.filt:
                eta_h = eta_h * self.gr.filt
                psi_h = psi_h * self.gr.filt
        return eta_h, psi_h

    def step_ifab2(self, eta, psi, dt, nsteps=1):
        g = self.gr
        a, b = self.step_ifab2_spec(g.spec(eta), g.spec(psi), dt, nsteps)
        return g.phys(a), g.phys(b)

    # -- inverse DNO map (Sec. 3.5, eq:psi_inverse) -----------------------------------
    def inverse_dtn_spec(self, eta_h, v_h, iters=8):
        """psi from (eta, v = G^[M](eta) psi) by the fixed-point iteration
        psi <- G0^{-1} (v - (G^[M] - G0) psi), seeded with G0^{-1} v.
        Reading: G0^{-1} is 1/G0 off k = 0 and 0 at k = 0 (the mean of psi
        enters no operator)."""
        G0 = self.gr.G0
        inv = np.where(G0 > 0, 1.0 / np.where(G0 > 0, G0, 1.0), 0.0)
        psi_h = inv * v_h
        for _ in range(int(iters)):
            psi_h = inv * (v_h - (self.dtn_spec(eta_h, psi_h) - G0 * psi_h))
        return psi_h

    def inverse_dtn(self, eta, v, iters=8):
        g = self.gr
        return g.phys(self.inverse_dtn_spec(g.spec(eta), g.spec(v), iters))

    # -- bulk velocity at depth layers (Alg. ComputeVolumeVelFrom2D) -------------------
    def depth_velocity(self, eta, psi, ys):
        """Velocities at depths y_i below the flat reference plane, [L][3][ny][nx]
        as (u, v, w) = (x velocity, upward velocity, y velocity):
          Phi|0 = psi - eps P(eta, G0 psi)                    (eq:phi1, first order)
          Phi|0 <- Phi|0 * prod_a exp(-(|k_a| / (kNyq_a / 2))^8)   (coupling taper)
          u_i = i kx C_i Phi|0, w_i = i ky C_i Phi|0, v_i = S_i Phi|0  (eq:ui, eq:wi, eq:vi)
        with C_i = cosh(|k|(d - y_i)) / cosh(|k| d), S_i = |k| sinh(|k|(d - y_i)) / cosh(|k| d)
        (eq:Ci, eq:Si; deep water: exp(-|k| y_i) and |k| exp(-|k| y_i)), C = 1, S = 0 at k = 0.
        The quotients are evaluated as exp(-|k| y) (1 +- exp(-2|k|(d - y))) / (1 + exp(-2|k|d)),
        the same functions without overflow."""
        g = self.gr
        eh, ph = g.spec(eta), g.spec(psi)
        phi0 = ph - self.eps * self.P(eh, g.G0 * ph)
        knx, kny = np.pi * g.nx / g.Lx, np.pi * g.ny / g.Ly
        phi0 = phi0 * np.exp(-(np.abs(g.kx) / (0.5 * knx)) ** 8 - (np.abs(g.ky) / (0.5 * kny)) ** 8)
        k = g.kk
        out = np.empty((len(ys), 3, g.ny, g.nx))
        for i, y in enumerate(ys):
            e1 = np.exp(-k * y)
            if g.deep:
                C, S = e1, k * e1
            else:
                e2 = np.exp(-2.0 * k * (g.h - y))
                den = 1.0 + np.exp(-2.0 * k * g.h)
                C, S = e1 * (1.0 + e2) / den, k * e1 * (1.0 - e2) / den
            C = np.where(k == 0, 1.0, C)
            S = np.where(k == 0, 0.0, S)
            out[i, 0] = g.phys(1j * g.kx * C * phi0)
            out[i, 1] = g.phys(S * phi0)
            out[i, 2] = g.phys(1j * g.ky * C * phi0)
        return out

    # -- Hamiltonian ----------------------------------------------------------------
    def hamiltonian_spec(self, eta_h, psi_h):
        """H = 1/2 dA sum_x psi G psi + 1/2 g dA sum_x eta^2 (eq:hamiltonian),
        the sums taken by Parseval: sum_x f g = (1/N) Re sum_k conj(f_hat) g_hat."""
        g = self.gr
        G = self.dtn_spec(eta_h, psi_h)
        dA = g.Lx * g.Ly / g.N
        kin = np.real(np.vdot(psi_h, G)) / g.N
        pot = np.real(np.vdot(eta_h, eta_h)) / g.N
        return 0.5 * dA * kin + 0.5 * g.g * dA * pot

    # -- physical-space entry points (mirror the C ABI) ------------------------------
    def dtn(self, eta, psi):
        g = self.gr
        return g.phys(self.dtn_spec(g.spec(eta), g.spec(psi)))

    def rhs(self, eta, psi):
        g = self.gr
        a, b = self.rhs_spec(g.spec(eta), g.spec(psi))
        return g.phys(a), g.phys(b)

    def step(self, eta, psi, dt, nsteps=1):
        g = self.gr
        a, b = self.step_spec(g.spec(eta), g.spec(psi), dt, nsteps)
        return g.phys(a), g.phys(b)

    def hamiltonian(self, eta, psi):
        g = self.gr
        return self.hamiltonian_spec(g.spec(eta), g.spec(psi))


# ---- reflecting walls by even extension (Sec. "Boundary conditions via even extension") ----
def even_extend(f):
    """Mirror an (ny, nx) field across each wall of the rectangle onto the
    doubled (2 ny, 2 nx) periodic grid (eq:even_ext).  Reading: samples are
    cell centred, so the reflection is half-sample symmetric,
    f~(2n - 1 - i) = f(i), which makes every odd derivative vanish on the
    walls (the Neumann condition)."""
    f = np.asarray(f, dtype=float)
    g = np.concatenate([f, f[::-1, :]], axis=0)
    return np.concatenate([g, g[:, ::-1]], axis=1)


def crop(f):
    """The physical quarter of a doubled field."""
    ny, nx = f.shape
    return np.array(f[: ny // 2, : nx // 2])


class ReflectingModel:
    """A tank of nx x ny cells of size Lx x Ly with reflecting walls: the
    periodic model on the doubled grid applied to the even extension, the
    result cropped back.  The Hamiltonian of the tank is a quarter of the
    doubled domain's."""

    def __init__(self, nx, ny, Lx, Ly, depth, M, g=9.81, **kw):
        self.m = HOSModel(Grid(2 * nx, 2 * ny, 2 * Lx, 2 * Ly, depth, g=g), M, **kw)

    def dtn(self, eta, psi):
        return crop(self.m.dtn(even_extend(eta), even_extend(psi)))

    def rhs(self, eta, psi):
        a, b = self.m.rhs(even_extend(eta), even_extend(psi))
        return crop(a), crop(b)

    def step(self, eta, psi, dt, nsteps=1):
        a, b = self.m.step(even_extend(eta), even_extend(psi), dt, nsteps)
        return crop(a), crop(b)

    def step_ifab2(self, eta, psi, dt, nsteps=1):
        a, b = self.m.step_ifab2(even_extend(eta), even_extend(psi), dt, nsteps)
        return crop(a), crop(b)

    def hamiltonian(self, eta, psi):
        return 0.25 * self.m.hamiltonian(even_extend(eta), even_extend(psi))


def truncated_convolution(grid, A, B, taper=True):
    """Brute-force definition of the dealiased product on tiny grids:
    T(k) * sum_{p, q in B, p + q = k} A(p) B(q) / N for k in B (an exact
    truncated linear convolution; no DFT of the product is involved)."""
    g = grid
    out = np.zeros((g.ny, g.nx), dtype=complex)
    modes = [(int(g.my[iy]), int(g.mx[ix]), iy, ix) for iy in g.iy_b for ix in g.ix_b]
    index = {(my, mx): (iy, ix) for my, mx, iy, ix in modes}
    for my1, mx1, iy1, ix1 in modes:
        a = A[iy1, ix1]
        if a == 0:
            continue
        for my2, mx2, iy2, ix2 in modes:
            tgt = index.get((my1 + my2, mx1 + mx2))
            if tgt is not None:
                out[tgt] += a * B[iy2, ix2]
    out /= g.N
    return out * g.taper if taper else out
