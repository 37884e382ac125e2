"""Dense direct solve of the Dirichlet-Neumann problem (test infrastructure only).

The DNO G(eta) psi is defined by a harmonic extension (Sec. 3.1, eq:dno_def):
Phi harmonic in -h <= z <= eta(x), Phi = psi on z = eta, d_z Phi = 0 on the
bed, G(eta) psi = sqrt(1 + |grad eta|^2) d_n Phi = Phi_z - grad eta . grad_h Phi
at the surface.  This module solves that Laplace problem directly -- no series,
no products, no dealiasing -- so it checks the HOS series independently.

Discretisation: the fluid column is mapped to s = (z + h) / D in [0, 1],
D = h + eta, Phi(x, z) = u(x, s).  With a_a = -s eta_a / D the Laplacian is
    sum_a [ u_aa + 2 a_a u_as + a_a^2 u_ss + (-s eta_aa / D + 2 s eta_a^2 / D^2) u_s ]
        + u_ss / D^2 = 0,
Fourier collocation in x, y (periodic) and Chebyshev-Gauss-Lobatto in s,
assembled as one dense matrix and solved by LU.  Rows at s = 1 impose u = psi,
rows at s = 0 impose u_s = 0.  Then, since grad psi = grad_h Phi + Phi_z grad eta,
    G psi = (1 + |grad eta|^2) u_s(x, 1) / D - grad eta . grad psi.
"""
import numpy as np
import scipy.linalg


def cheb(n):
    """Chebyshev-Gauss-Lobatto points x_j = cos(pi j / n), j = 0..n, and the
    collocation differentiation matrix on [-1, 1] (standard construction)."""
    x = np.cos(np.pi * np.arange(n + 1) / n)
    c = np.ones(n + 1)
    c[0] = c[-1] = 2.0
    c = c * (-1.0) ** np.arange(n + 1)
    X = np.tile(x, (n + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1.0 / c) / (dX + np.eye(n + 1))
    D = D - np.diag(D.sum(axis=1))
    return D, x


def fourier_diff(n, L):
    """First- and second-derivative collocation matrices on n periodic points
    of a period-L interval (spectral: multiply by i k, resp. -k^2, per mode;
    the first derivative drops the Nyquist mode)."""
    if n == 1:
        return np.zeros((1, 1)), np.zeros((1, 1))
    m = np.rint(np.fft.fftfreq(n, 1.0 / n))
    k = 2 * np.pi / L * m
    k1 = k.copy()
    k1[n // 2] = 0.0
    I = np.eye(n)
    F = np.fft.fft(I, axis=0)
    D1 = np.real(np.fft.ifft((1j * k1)[:, None] * F, axis=0))
    D2 = np.real(np.fft.ifft((-(k ** 2))[:, None] * F, axis=0))
    return D1, D2


def _solve(eta, psi, Lx, Ly, h, nz):
    """The harmonic extension u(x, s) on the collocation grid: returns u as
    [nz + 1][ny][nx] (s descending from 1 at the surface to 0 at the bed), the
    Chebyshev nodes s, the s-derivative of u at the surface, and the surface
    slopes and potential gradient."""
    ny, nx = eta.shape
    Dx1, Dx2 = fourier_diff(nx, Lx)
    Dy1, Dy2 = fourier_diff(ny, Ly)
    Dc, xc = cheb(nz)
    s = (xc + 1.0) / 2.0  # s[0] = 1 (surface), s[nz] = 0 (bed)
    Ds = 2.0 * Dc
    Dss = Ds @ Ds
    ns = nz + 1
    Ix, Iy, Is = np.eye(nx), np.eye(ny), np.eye(ns)

    # Surface slopes and curvatures (spectral derivatives of the given data).
    ex, exx = eta @ Dx1.T, eta @ Dx2.T
    ey, eyy = Dy1 @ eta, Dy2 @ eta
    px, py = psi @ Dx1.T, Dy1 @ psi
    D = h + eta

    def field3(f2):  # [ny][nx] -> flat over (s, y, x)
        return np.broadcast_to(f2[None, :, :], (ns, ny, nx)).reshape(-1)

    S3 = np.broadcast_to(s[:, None, None], (ns, ny, nx)).reshape(-1)
    D3, ex3, ey3 = field3(D), field3(ex), field3(ey)
    exx3, eyy3 = field3(exx), field3(eyy)
    ax, ay = -S3 * ex3 / D3, -S3 * ey3 / D3
    cs = (-S3 * exx3 / D3 + 2 * S3 * ex3 ** 2 / D3 ** 2) + (-S3 * eyy3 / D3 + 2 * S3 * ey3 ** 2 / D3 ** 2)
    css = ax ** 2 + ay ** 2 + 1.0 / D3 ** 2

    Kxx = np.kron(Is, np.kron(Iy, Dx2))
    Kyy = np.kron(Is, np.kron(Dy2, Ix))
    Kxs = np.kron(Ds, np.kron(Iy, Dx1))
    Kys = np.kron(Ds, np.kron(Dy1, Ix))
    Ks = np.kron(Ds, np.kron(Iy, Ix))
    Kss = np.kron(Dss, np.kron(Iy, Ix))

    A = Kxx + Kyy
    A += 2.0 * ax[:, None] * Kxs
    A += 2.0 * ay[:, None] * Kys
    A += cs[:, None] * Ks
    A += css[:, None] * Kss
    del Kxx, Kyy, Kxs, Kys, Kss
    rhs = np.zeros(A.shape[0])

    nxy = nx * ny
    top = slice(0, nxy)  # s = 1
    bot = slice((ns - 1) * nxy, ns * nxy)  # s = 0
    A[top, :] = 0.0
    A[top, top] = np.eye(nxy)
    rhs[top] = psi.reshape(-1)
    A[bot, :] = Ks[bot, :]
    rhs[bot] = 0.0

    u = scipy.linalg.solve(A, rhs, overwrite_a=True, check_finite=False)
    us_top = (Ks[top, :] @ u).reshape(ny, nx)
    return u.reshape(ns, ny, nx), s, us_top, (ex, ey, px, py, D)


def dno_direct(eta, psi, Lx, Ly, h, nz):
    """G(eta) psi by the dense direct solve; eta, psi are [ny][nx] (ny may be 1)."""
    _, _, us_top, (ex, ey, px, py, D) = _solve(eta, psi, Lx, Ly, h, nz)
    return (1.0 + ex ** 2 + ey ** 2) * us_top / D - ex * px - ey * py


def cheb_interp(s_nodes, f, s):
    """Value at s of the polynomial through (s_nodes[j], f[j]) on the
    Chebyshev-Gauss-Lobatto nodes of cheb() mapped to [0, 1] (barycentric
    form, weights (-1)^j halved at both ends)."""
    n = len(s_nodes) - 1
    w = (-1.0) ** np.arange(n + 1)
    w[0] *= 0.5
    w[-1] *= 0.5
    d = s - s_nodes
    hit = np.flatnonzero(d == 0.0)
    if hit.size:
        return float(f[hit[0]])
    q = w / d
    return float(np.dot(q, f) / np.sum(q))


def potential_at_depths(eta, psi, Lx, Ly, h, nz, depths):
    """The exact potential Phi(x, z = -y) on horizontal planes y in `depths`
    below the reference level z = 0 (each plane inside the fluid, -y < min eta),
    by the dense direct solve and interpolation along each mapped column:
    z = -y is s = (h - y) / (h + eta(x)).  Returns [len(depths)][ny][nx]."""
    u, s, _, _ = _solve(eta, psi, Lx, Ly, h, nz)
    ny, nx = eta.shape
    out = np.empty((len(depths), ny, nx))
    for i, y in enumerate(depths):
        sy = (h - y) / (h + eta)
        if np.any(sy <= 0.0) or np.any(sy >= 1.0):
            raise ValueError("plane z = -y must lie strictly inside the fluid")
        for iy in range(ny):
            for ix in range(nx):
                out[i, iy, ix] = cheb_interp(s, u[:, iy, ix], sy[iy, ix])
    return out
