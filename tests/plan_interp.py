"""CPU interpreter of the HIP library's schedules (test infrastructure).

Executes the row programs and column tasks that the host planner
(paper_2608_25203_amd/csrc/zk_plan.cpp) emits, with the same meaning the
kernels give them, on numpy arrays: mixed fields are (rows, nx/2) complex
(y physical, kx spectral), base spectra (ny, nx/2) complex.  It lets the CPU
suite check the planner's algebra against the oracle before any GPU run.  It
shares no code with the oracle and is not part of the product path.
"""
import json
import os
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_25203_amd", "csrc")
EXE = os.path.join(ROOT, "_build", "zk_plan_check")

OP_LD2, OP_LDP, OP_MOV, OP_MAC, OP_ZERO, OP_BERN, OP_ST2, OP_STP = range(1, 9)
RS_NONE = 255
SYM_IKY, SYM_FILT, SYM_TAPER, SYM_IF = 0x10, 0x20, 0x40, 0x80
L_ROW_PAD, L_ROW_BASE, L_COL_PAD, L_COL_BASE, L_PARSEVAL = range(5)


def pow2_scale(a):
    """Per-row power-of-two scale bringing max(|re|, |im|) of each row to [1, 2),
    and its inverse, which is 0 for an all-zero row (whose result is exactly 0)."""
    a = np.asarray(a)
    m = np.max(np.maximum(np.abs(a.real), np.abs(a.imag)), axis=1, keepdims=True)
    with np.errstate(divide="ignore"):
        e = np.where(m > 0, np.floor(np.log2(np.where(m > 0, m, 1.0))), 0.0)
    return np.exp2(-e), np.where(m > 0, np.exp2(e), 0.0)


def build_checker():
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    src = [os.path.join(CSRC, "zk_plan.cpp"), os.path.join(CSRC, "zk_plan_check.cpp")]
    if not os.path.exists(EXE) or any(os.path.getmtime(s) > os.path.getmtime(EXE) for s in src + [
            os.path.join(CSRC, "zk_plan.hpp"), os.path.join(CSRC, "zk_program.hpp")]):
        tmp = f"{EXE}.{os.getpid()}"  # parallel test workers each build, then rename atomically
        subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC] + src + ["-o", tmp], check=True)
        os.replace(tmp, EXE)
    return EXE


def load_plan(nx, ny, M, eps=1.0, taper=True, filt=True, dt=1.0):
    exe = build_checker()
    out = subprocess.run([exe, str(nx), str(ny), str(M), repr(float(eps)), str(int(taper)), str(int(filt)),
                          repr(float(dt))], capture_output=True, text=True, check=True).stdout
    return json.loads(out)


class Interp:
    def __init__(self, nx, ny, Lx, Ly, depth, g, M, eps=1.0, taper=True, filt=True):
        self.nx, self.ny, self.Lx, self.Ly, self.g, self.M = nx, ny, Lx, Ly, g, M
        self.depth = depth if (depth is not None and np.isfinite(depth) and depth > 0) else 0.0
        self.eps, self.taper, self.filt = eps, taper, filt
        self.K = nx // 2
        self.mix = {}
        self.base = {}
        self.plan = None
        self.dt = None
        kx = 2 * np.pi / Lx * np.arange(self.K)
        b = np.arange(ny)
        my = np.where((b < ny // 2) | (ny == 1), b, b - ny)  # a 1D grid's one row is ky = 0
        self.kx, self.my = kx[None, :], my[:, None]
        self.ky = 2 * np.pi / Ly * self.my
        self.kk = np.sqrt(self.kx ** 2 + self.ky ** 2)
        self.th = np.tanh(self.kk * self.depth) if self.depth > 0 else np.ones_like(self.kk)
        kc = 2.0 / 3.0 * (min(np.pi * nx / Lx, np.pi * ny / Ly) if ny > 1 else np.pi * nx / Lx)
        self.taper_sym = np.exp(-((self.kk / kc) ** 8))

        def f1(m, n):
            t = 2 * np.pi * m / n
            return (5 + 4 * np.cos(t) - np.cos(2 * t)) / 8

        self.filt_sym = f1(np.arange(self.K)[None, :], nx) * f1(self.my, ny)

    def _plan(self, dt):
        if self.plan is None or dt != self.dt:
            self.plan = load_plan(self.nx, self.ny, self.M, self.eps, self.taper, self.filt, dt)
            self.dt = dt
        return self.plan

    # ---- symbols ---------------------------------------------------------------
    def sym(self, s):
        f = np.ones_like(self.kk)
        l = s & 0xF
        if l:
            f = self.kk ** l * (self.th if l % 2 else 1.0)
        if s & SYM_FILT:
            f = f * self.filt_sym
        if (s & SYM_TAPER) and self.taper:
            f = f * self.taper_sym
        if s & SYM_IF:
            f = f * self._ifcoef()[(s >> 8) & 7]
        if s & 0x800:  # 1 / G0, 0 at k = 0
            G0 = self.kk * self.th
            f = np.where(G0 > 0, f / np.where(G0 > 0, G0, 1.0), 0.0)
        if s & 0x1000:  # coupling taper of the depth lift
            rx = np.abs(self.kx) / (0.5 * np.pi * self.nx / self.Lx)
            ry = np.abs(self.ky) / (0.5 * np.pi * self.ny / self.Ly)
            f = f * np.exp(-rx ** 8 - ry ** 8)
        if s & 0x6000:  # C or S of layer (s >> 16) & 15 of the chunk
            y = self.layer_y[(s >> 16) & 15]
            k = self.kk
            e1 = np.exp(-k * y)
            if self.depth > 0:
                e2 = np.exp(-2 * k * (self.depth - y))
                den = 1 + np.exp(-2 * k * self.depth)
                C, S = e1 * (1 + e2) / den, k * e1 * (1 - e2) / den
            else:
                C, S = e1, k * e1
            f = f * (np.where(k == 0, 0.0, S) if s & 0x4000 else np.where(k == 0, 1.0, C))
        if s & SYM_IKY:
            return 1j * self.ky * f
        return f.astype(complex)

    def _ifcoef(self):
        """Exact linear flow and constant-forcing response over self.dt per
        mode, omega^2 = g G0 (k = 0: the limits)."""
        dt, g = self.dt, self.g
        G0 = self.kk * self.th
        om = np.sqrt(g * G0)
        z = om == 0
        o = np.where(z, 1.0, om)
        c, sn = np.cos(om * dt), np.sin(om * dt)
        return [c, np.where(z, 0.0, G0 * sn / o), np.where(z, g * dt, g * sn / o), np.where(z, dt, sn / o),
                (1 - c) / g, np.where(z, 0.5 * g * dt * dt, (1 - c) / np.where(z, 1.0, G0))]

    # ---- row pass ----------------------------------------------------------------
    def row(self, launch, phys):
        kind, first, count = launch[0], launch[1], launch[2]
        pad = kind == L_ROW_PAD
        N = 3 * self.nx // 2 if pad else self.nx
        rows = 3 * self.ny // 2 if pad else self.ny
        K = self.K
        kxs = 2 * np.pi / self.Lx * np.arange(K)
        P = self.plan
        for pi in range(first, first + count):
            op0, nop = P["progs"][pi]
            R = [np.zeros((rows, N)) for _ in range(6)]
            for o in P["ops"][op0:op0 + nop]:
                code, a, b, c, fa, fla, fb, flb, coef = o
                if code == OP_LD2:
                    def spec(f, fl):
                        S = np.array(self.mix[f][:rows, :K])
                        if fl & 1:
                            S = S * (1j * kxs[None, :])
                        return S
                    Sa = spec(fa, fla)
                    Sb = spec(fb, flb) if fb >= 0 else np.zeros_like(Sa)
                    (sa, ia), (sb, ib) = pow2_scale(Sa), pow2_scale(Sb)
                    Sa, Sb = Sa * sa, Sb * sb
                    Z = np.zeros((rows, N), complex)
                    Z[:, :K] = Sa + 1j * Sb
                    Z[:, N - K + 1:] = (np.conj(Sa) + 1j * np.conj(Sb))[:, 1:][:, ::-1]
                    z = np.fft.ifft(Z, axis=1) * N
                    R[0], R[1] = z.real * ia, z.imag * ib
                elif code == OP_LDP:
                    slot = lambda i: 4 if i == 2 else i  # phys: in0, in1, out0, out1, in2
                    R[0] = np.array(phys[slot(fa)], dtype=float)
                    R[1] = np.array(phys[slot(fb)], dtype=float) if fb >= 0 else np.zeros((rows, N))
                elif code == OP_MOV:
                    R[a] = R[b].copy()
                elif code == OP_MAC:
                    R[a] = R[a] + coef * R[b] * R[c]
                elif code == OP_ZERO:  # clears o0, o1, o2
                    for k in (3, 4, 5):
                        R[k] = np.zeros((rows, N))
                elif code == OP_BERN:
                    e = coef
                    S = 1 + e * e * R[3]
                    W = (R[0] + e * R[4]) / S
                    R[3] = e * (-0.5 * R[5] + 0.5 * S * W * W)
                elif code == OP_ST2:
                    x = R[a]
                    y = R[b] if b != RS_NONE else np.zeros_like(x)
                    (sx, ix), (sy, iy) = pow2_scale(x), pow2_scale(y)
                    Z = np.fft.fft(x * sx + 1j * (y * sy), axis=1)
                    k = np.arange(K)
                    Zk = Z[:, k]
                    Zm = Z[:, (N - k) % N]
                    self._mix_put(fa, rows, (Zk + np.conj(Zm)) / 2 * ix)
                    if fb >= 0:
                        self._mix_put(fb, rows, (Zk - np.conj(Zm)) / 2j * iy)
                elif code == OP_STP:
                    if fb >= 0:
                        phys[2 + fa][fb][...] = R[a]
                    else:
                        phys[2 + fa][...] = R[a]
                else:
                    raise ValueError(code)

    def _mix_put(self, f, rows, arr):
        m = self.mix.setdefault(f, np.zeros((3 * self.ny // 2, self.K), complex))
        m[:rows, :] = arr

    # ---- column pass ---------------------------------------------------------------
    def col(self, launch):
        kind, first, count = launch[0], launch[1], launch[2]
        pad = kind == L_COL_PAD
        ny = self.ny
        rows = 3 * ny // 2 if pad else ny
        b = np.arange(ny)
        idx = np.where(b < ny // 2, b, b + (rows - ny))
        P = self.plan
        for ti in range(first, first + count):
            fwds, fsyms, fcoefs, o0, no = P["tasks"][ti]
            X = None
            for fwd, fsym, fcoef in zip(fwds, fsyms, fcoefs):  # folds summed into X
                if fwd < 0:
                    continue
                V = np.fft.fft(self.mix[fwd][:rows, :], axis=0)
                Xf = V[idx, :] * fcoef * self.sym(fsym)
                X = Xf if X is None else X + Xf
            if X is not None and ny > 1:  # a 1D grid (ny = 1) has no ky Nyquist row
                X[ny // 2, :] = 0
            for oi in range(o0, o0 + no):
                dst_b, dst_m, t0, nt, lc, lsym = P["outs"][oi]
                acc = np.zeros((ny, self.K), complex)
                for src, s, coef in P["terms"][t0:t0 + nt]:
                    v = X if src < 0 else self.base[src]
                    acc = acc + coef * self.sym(s) * v
                if ny > 1:
                    acc[ny // 2, :] = 0
                if dst_b >= 0:
                    self.base[dst_b] = acc
                if dst_m >= 0:
                    Z = np.zeros((rows, self.K), complex)
                    Z[idx, :] = acc * lc * (self.sym(lsym).real if lsym else 1.0)
                    if pad and ny > 1:
                        Z[ny // 2 + (rows - ny), :] = 0  # the Nyquist slot mapped by idx is zero anyway
                    z = np.fft.ifft(Z, axis=0) * rows
                    self._mix_put(dst_m, rows, z)

    def parseval(self, launch):
        a, b, c, d = (self.base[i] for i in launch[1:5])
        w = np.where(np.arange(self.K) == 0, 1.0, 2.0)[None, :]
        return (float(np.sum(w * np.real(np.conj(a) * b))), float(np.sum(w * np.real(np.conj(c) * d))))

    def run(self, seq, phys):
        res = None
        for l in seq:
            if l[0] in (L_ROW_PAD, L_ROW_BASE):
                self.row(l, phys)
            elif l[0] in (L_COL_PAD, L_COL_BASE):
                self.col(l)
            else:
                res = self.parseval(l)
        return res

    # ---- entry points mirroring the C ABI ---------------------------------------------------
    def dtn(self, eta, psi):
        P = self._plan(self.dt if self.dt is not None else 1.0)
        phys = [eta, psi, np.zeros_like(eta), np.zeros_like(eta)]
        self.run(P["dtn"], phys)
        return phys[2]

    def rhs(self, eta, psi):
        P = self._plan(self.dt if self.dt is not None else 1.0)
        phys = [eta, psi, np.zeros_like(eta), np.zeros_like(eta)]
        self.run(P["rhs"], phys)
        return phys[2], phys[3]

    def hamiltonian(self, eta, psi):
        P = self._plan(self.dt if self.dt is not None else 1.0)
        phys = [eta, psi, None, None]
        s1, s2 = self.run(P["ham"], phys)
        N = self.nx * self.ny
        dA = self.Lx * self.Ly / N
        return 0.5 * dA * s1 / N + 0.5 * self.g * dA * s2 / N

    def rhs_g(self, eta, psi, G):
        P = self._plan(self.dt if self.dt is not None else 1.0)
        phys = [eta, psi, np.zeros_like(eta), np.zeros_like(eta), G]
        self.run(P["rhs_g"], phys)
        return phys[2], phys[3]

    def filter(self, eta, psi):
        P = self._plan(self.dt if self.dt is not None else 1.0)
        phys = [eta, psi, np.zeros_like(eta), np.zeros_like(eta)]
        self.run(P["filter"], phys)
        return phys[2], phys[3]

    def inverse_dtn(self, eta, v, iters):
        P = self._plan(self.dt if self.dt is not None else 1.0)
        phys = [eta, v, np.zeros_like(eta), np.zeros_like(eta)]
        self.run(P["inv_entry"], phys)
        for _ in range(iters):
            self.run(P["inv_iter"], phys)
        self.run(P["inv_exit"], phys)
        return phys[2]

    def depth_velocity(self, eta, psi, ys, chunk=None):
        """(u, v, w) at depths ys, [L][3][ny][nx]: the potential on the flat
        plane, then chunks of at most depth_chunk_max layers (or `chunk`)."""
        P = self._plan(self.dt if self.dt is not None else 1.0)
        lc = min(P["depth_chunk_max"], chunk or P["depth_chunk_max"])
        out = np.zeros((len(ys), 3, self.ny, self.nx))
        self.run(P["lift_phi"], [eta, psi, None, None])
        for i0 in range(0, len(ys), lc):
            r = min(lc, len(ys) - i0)
            self.layer_y = list(ys[i0:i0 + r])
            planes = out[i0:i0 + r].reshape(3 * r, self.ny, self.nx)
            self.run(P["depth_chunk%d" % r], [eta, psi, planes, None])
        return out

    def step_ab2(self, eta, psi, dt, nsteps):
        P = self._plan(dt)
        phys = [eta, psi, np.zeros_like(eta), np.zeros_like(eta)]
        self.run(P["step_entry"], phys)
        for i in range(nsteps):
            par = i & 1
            self.run(P[("ab2_first%d" if i == 0 else "ab2_body%d") % par], phys)
            if i + 1 < nsteps:
                self.run(P["step_lift%d" % (1 - par)], phys)
        self.run(P["step_exit%d" % (nsteps & 1)], phys)
        return phys[2], phys[3]

    def step(self, eta, psi, dt, nsteps):
        P = self._plan(dt)
        phys = [eta, psi, np.zeros_like(eta), np.zeros_like(eta)]
        self.run(P["step_entry"], phys)
        for i in range(nsteps):
            par = i & 1
            self.run(P["step_body%d" % par], phys)
            if i + 1 < nsteps:
                self.run(P["step_lift%d" % (1 - par)], phys)
        self.run(P["step_exit%d" % (nsteps & 1)], phys)
        return phys[2], phys[3]
