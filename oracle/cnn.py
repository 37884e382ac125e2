"""Plain FP64 reference of the learned DtN closure network (test infrastructure only).

The closure predicts the high-order part of the Dirichlet-Neumann operator,
r = (G^[6] - G^[2]) psi, from low-order fields on the grid.  The network is a
stack of four 3 x 3 convolutions with periodic (circular) padding,
3 -> 32 -> 32 -> 32 -> 1 channels, with the exact-erf GELU after the first
three, trained on a masked mean-squared error with Adam (Kingma & Ba).  The
paper motivates the reduced-order DtN and its cost ranking (Sec. 3.2: every
additional order adds a comparable cost) and its FP32/low-order trade-off
(Sec. 8); the network itself is this project's addition and is defined here
in full.

Conventions (shared, by definition, with the GPU kernels):
  * activations (B, C, H, W); weights (C_out, C_in, 3, 3) and bias (C_out,);
  * convolution is cross-correlation with wrap-around:
      y[b, o, i, j] = bias[o] + sum_{c, u, v} W[o, c, u, v] x[b, c, (i+u-1) % H, (j+v-1) % W];
  * GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2;
  * loss = mean over the interior pixels (at least `halo` from every tile
    edge) of (y - t)^2; with halo >= 4 the wrap-around never reaches a pixel
    that influences the loss, so training on crops equals valid convolution;
  * parameter vector order: W1, b1, W2, b2, W3, b3, W4, b4 (flattened C order).

Optional bf16 emulation (`bf16=True`) rounds, at the points where the GPU
path stores bf16, the conv operands (weights, input activations and the
backpropagated pre-activation gradients) to bfloat16 (round to nearest even)
before an FP64 product, so that the GPU training kernels can be compared
element by element.  Biases and the loss stay unrounded.

Everything here is numpy (FP64) and written for clarity, not speed: im2col
with explicit index arithmetic, no blocking.
"""
import math

import numpy as np
from scipy.special import erf

CHANNELS = (3, 32, 32, 32, 1)
SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def param_shapes(channels=CHANNELS):
    shp = []
    for l in range(len(channels) - 1):
        shp.append((channels[l + 1], channels[l], 3, 3))
        shp.append((channels[l + 1],))
    return shp


def n_params(channels=CHANNELS):
    return int(sum(np.prod(s) for s in param_shapes(channels)))


def unflatten(vec, channels=CHANNELS):
    out, o = [], 0
    for s in param_shapes(channels):
        n = int(np.prod(s))
        out.append(np.asarray(vec[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def to_bf16(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def im2col(x):
    """(B, C, H, W) -> (B, H, W, C*9) with column index c*9 + u*3 + v holding
    x[b, c, (i+u-1) % H, (j+v-1) % W]."""
    B, C, H, W = x.shape
    cols = np.empty((B, H, W, C, 3, 3))
    ii = np.arange(H)
    jj = np.arange(W)
    for u in range(3):
        for v in range(3):
            rows = (ii + u - 1) % H
            cs = (jj + v - 1) % W
            cols[:, :, :, :, u, v] = x[:, :, rows][:, :, :, cs].transpose(0, 2, 3, 1)
    return cols.reshape(B, H, W, C * 9)


def col2im(dcols, C, H, W):
    """Adjoint of im2col: output pixel (i, j) read input pixel (i+u-1, j+v-1),
    so its column gradient is added back there (a circular shift by (u-1, v-1))."""
    B = dcols.shape[0]
    d = dcols.reshape(B, H, W, C, 3, 3)
    dx = np.zeros((B, C, H, W))
    for u in range(3):
        for v in range(3):
            contrib = d[:, :, :, :, u, v].transpose(0, 3, 1, 2)
            dx += np.roll(contrib, shift=(u - 1, v - 1), axis=(2, 3))
    return dx


def conv3x3(x, Wt, b):
    """Circular 3 x 3 cross-correlation (definition in the module header)."""
    B, C, H, W = x.shape
    O = Wt.shape[0]
    cols = im2col(x)
    y = cols @ Wt.reshape(O, C * 9).T + b
    return y.transpose(0, 3, 1, 2)


class CNN:
    """Forward, backward and loss of the closure network in FP64."""

    def __init__(self, params, channels=CHANNELS, bf16=False):
        self.channels = tuple(channels)
        self.params = [np.array(p, dtype=np.float64) for p in params]
        self.bf16 = bf16

    @property
    def nlayers(self):
        return len(self.channels) - 1

    def _q(self, a):
        return to_bf16(a) if self.bf16 else a

    def forward(self, x):
        """x: (B, C0, H, W).  Returns y (B, 1, H, W) and the cache for backward."""
        cache = []
        a = np.asarray(x, dtype=np.float64)
        for l in range(self.nlayers):
            Wt, b = self.params[2 * l], self.params[2 * l + 1]
            aq, Wq = self._q(a), self._q(Wt)
            z = conv3x3(aq, Wq, b)
            cache.append((aq, Wq, z))
            a = gelu(z) if l < self.nlayers - 1 else z
        return a, cache

    def backward(self, cache, dy):
        """Gradients of sum(dy * y) w.r.t. every parameter (list in parameter
        order) and w.r.t. the input."""
        grads = [None] * (2 * self.nlayers)
        d = np.asarray(dy, dtype=np.float64)
        for l in reversed(range(self.nlayers)):
            aq, Wq, z = cache[l]
            if l < self.nlayers - 1:
                d = d * gelu_grad(z)
            d = self._q(d)  # the GPU path stores pre-activation gradients in bf16
            B, C, H, W = aq.shape
            O = Wq.shape[0]
            dz = d.transpose(0, 2, 3, 1).reshape(-1, O)  # (B*H*W, O)
            cols = im2col(aq).reshape(-1, C * 9)
            grads[2 * l] = (dz.T @ cols).reshape(O, C, 3, 3)
            grads[2 * l + 1] = dz.sum(axis=0)
            dcols = (dz @ Wq.reshape(O, C * 9)).reshape(B, H, W, C * 9)
            d = col2im(dcols, C, H, W)
        return grads, d


def interior_mask(H, W, halo):
    m = np.zeros((H, W))
    m[halo:H - halo, halo:W - halo] = 1.0
    return m


def masked_mse(y, t, halo):
    """Mean of (y - t)^2 over the interior pixels of every tile, and its gradient."""
    B, _, H, W = y.shape
    m = interior_mask(H, W, halo)
    n = B * m.sum()
    r = (y - t) * m
    return float(np.sum(r * r) / n), 2.0 * r / n


class Adam:
    """Adam (Kingma & Ba 2015) with bias correction:
    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            out.append(p - lr * (self.m[i] / c1) / (np.sqrt(self.v[i] / c2) + self.eps))
        return out


# ---- the closure's inputs and output (normalisation) -------------------------------
def closure_features(eta, psi, g2psi, k0, eta_scale=0.1):
    """Network input channels for one field (H, W) triple:
    x0 = k0 eta / eta_scale (amplitude kept), x1 = k0 psi / s, x2 = G2psi / s
    with s = rms(G2psi) (the residual is linear in psi for fixed eta, so a
    per-sample psi scale is exact).  Returns (x of shape (3, H, W), s)."""
    s = float(np.sqrt(np.mean(np.asarray(g2psi) ** 2)))
    s = s if s > 0 else 1.0
    x = np.stack([k0 * np.asarray(eta) / eta_scale, k0 * np.asarray(psi) / s, np.asarray(g2psi) / s])
    return x, s


def closure_residual(cnn, eta, psi, g2psi, k0, out_scale, eta_scale=0.1):
    """r = out_scale * s * CNN(features): the predicted (G^[6] - G^[2]) psi."""
    x, s = closure_features(eta, psi, g2psi, k0, eta_scale)
    y, _ = cnn.forward(x[None])
    return out_scale * s * y[0, 0]


def closure_rhs_spec(model, net, eta_h, psi_h, k0, out_scale, eta_scale=0.1):
    """Zakharov RHS with the learned closure: the order-M DtN of `model` plus
    the network's residual, projected onto the band, in place of G^[M]:
        G = P_B(G^[M] psi + r),  d_t eta = G,  d_t psi = -g eta + N(eta, psi, G)
    (eq:zakharov_kin, eq:dyn_truncated with eq:W)."""
    g = model.gr
    eta, psi = g.phys(eta_h), g.phys(psi_h)
    g2 = g.phys(model.dtn_spec(eta_h, psi_h))
    r = closure_residual(net, eta, psi, g2, k0, out_scale, eta_scale)
    G_h = g.spec(g2 + r)
    return G_h, -g.g * eta_h + model.bernoulli_spec(eta_h, psi_h, G_h)


def closure_step(model, net, eta, psi, dt, nsteps, k0, out_scale, eta_scale=0.1):
    """Classical RK4 with the closure RHS, then the state filter A(k) after
    every full step (as HOSModel.step)."""
    g = model.gr
    eh, ph = g.spec(eta), g.spec(psi)
    f = lambda a, b: closure_rhs_spec(model, net, a, b, k0, out_scale, eta_scale)
    for _ in range(int(nsteps)):
        k1 = f(eh, ph)
        k2 = f(eh + 0.5 * dt * k1[0], ph + 0.5 * dt * k1[1])
        k3 = f(eh + 0.5 * dt * k2[0], ph + 0.5 * dt * k2[1])
        k4 = f(eh + dt * k3[0], ph + dt * k3[1])
        eh = eh + dt / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        ph = ph + dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        if model.filt:
            eh, ph = eh * g.filt, ph * g.filt
    return g.phys(eh), g.phys(ph)
