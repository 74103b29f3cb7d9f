"""Network operations of the learned warm start, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions (NCDHW arrays, cubic kernels of size K with zero padding K/2):
  y[n,o,d,h,w] = b[o] + sum_{c,i,j,k} w[o,c,i,j,k] x[n,c,d*sd+i-p,h*sh+j-p,w*sw+k-p]
  optional ReLU; gradients by the adjoint of the same sums.
  MSE L = 1/(2n) sum (y - t)^2.  Adam (Kingma and Ba, 2015) with bias
  correction.  Trace features and the coarse-grid interpolation follow the
  definitions stated at their functions.
"""
from __future__ import annotations

import numpy as np


def _out(n, K, s):
    return (n + 2 * (K // 2) - K) // s + 1


def conv3d_forward(x, w, b, strides, relu):
    N, C, D, H, W = x.shape
    O, _, K, _, _ = w.shape
    p = K // 2
    sd, sh, sw = strides
    Do, Ho, Wo = _out(D, K, sd), _out(H, K, sh), _out(W, K, sw)
    xp = np.zeros((N, C, D + 2 * p, H + 2 * p, W + 2 * p))
    xp[:, :, p:p + D, p:p + H, p:p + W] = x
    y = np.zeros((N, O, Do, Ho, Wo)) + (0.0 if b is None else b[None, :, None, None, None])
    for i in range(K):
        for j in range(K):
            for k in range(K):
                patch = xp[:, :, i:i + sd * (Do - 1) + 1:sd, j:j + sh * (Ho - 1) + 1:sh, k:k + sw * (Wo - 1) + 1:sw]
                y += np.einsum("oc,ncdhw->nodhw", w[:, :, i, j, k], patch)
    return np.maximum(y, 0.0) if relu else y


def conv3d_backward(x, w, y, dy, strides, relu):
    """(dx, dw, db) for L with dL/dy = dy; y is the activated output."""
    N, C, D, H, W = x.shape
    O, _, K, _, _ = w.shape
    p = K // 2
    sd, sh, sw = strides
    Do, Ho, Wo = dy.shape[2:]
    g = dy * (y > 0) if relu else dy
    xp = np.zeros((N, C, D + 2 * p, H + 2 * p, W + 2 * p))
    xp[:, :, p:p + D, p:p + H, p:p + W] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for i in range(K):
        for j in range(K):
            for k in range(K):
                sl = (slice(None), slice(None), slice(i, i + sd * (Do - 1) + 1, sd),
                      slice(j, j + sh * (Ho - 1) + 1, sh), slice(k, k + sw * (Wo - 1) + 1, sw))
                dw[:, :, i, j, k] = np.einsum("nodhw,ncdhw->oc", g, xp[sl])
                dxp[sl] += np.einsum("oc,nodhw->ncdhw", w[:, :, i, j, k], g)
    dx = dxp[:, :, p:p + D, p:p + H, p:p + W]
    db = g.sum(axis=(0, 2, 3, 4))
    return dx, dw, db


def mse(y, t):
    n = y.size
    r = y - t
    return 0.5 * float(np.sum(r * r)) / n, r / n


def adam_step(p, g, m, v, lr, b1, b2, eps, t):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def trace_features(traces, rec_idx, T, t0, tstride, comp, scale):
    """traces [nsrc][nsteps+1][nrec][3] -> [nsrc][T][len(rec_idx)]: component comp
    at the listed receivers and steps t0 + t*tstride (zero past the last step)."""
    nsrc, nt1 = traces.shape[:2]
    out = np.zeros((nsrc, T, len(rec_idx)))
    for t in range(T):
        step = t0 + t * tstride
        if step < nt1:
            out[:, t, :] = scale * traces[:, step, rec_idx, comp]
    return out


def grid_to_nodes(c, NIX, NIY, NIZ, base):
    """Coarse cell-centred relative perturbation c[gz][gy][gx] (z index 0 at the
    top) on a regular grid covering the closed interior -> base * (1 + c(x)),
    trilinear between cell centres and constant beyond the outer centres."""
    gz, gy, gx = c.shape

    def weights(n_nodes, G, reverse=False):
        W = np.zeros((n_nodes, G))
        for j in range(n_nodes):
            jj = n_nodes - 1 - j if reverse else j
            u = jj / (n_nodes - 1) * G - 0.5           # position in cell-centre units
            u = min(max(u, 0.0), G - 1)
            k0 = min(int(np.floor(u)), max(G - 2, 0))
            f = u - k0 if G > 1 else 0.0
            W[j, k0] += 1 - f
            if G > 1:
                W[j, k0 + 1] += f
        return W

    Wx, Wy, Wz = weights(NIX, gx), weights(NIY, gy), weights(NIZ, gz, reverse=True)
    field = np.einsum("zZ,yY,xX,ZYX->zyx", Wz, Wy, Wx, c)     # node grid [NIZ][NIY][NIX]
    return base * (1.0 + field.ravel())


def bf16_round(a):
    """Round to the nearest BF16 value, ties to even (the 16 high bits of the
    FP32 pattern after adding 0x7FFF plus the lowest kept bit); finite input."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(x, weights, biases, strides, relus):
    """The network's forward pass as BF16 inference defines it: input,
    weights and hidden activations rounded to BF16, sums in FP64 here (FP32 on
    the device), bias and ReLU before the rounding; the last output unrounded."""
    a = bf16_round(x)
    for li, (w, b, s, r) in enumerate(zip(weights, biases, strides, relus)):
        y = conv3d_forward(a, bf16_round(w), None if b is None else np.asarray(b, np.float64), s, r)
        a = y if li == len(weights) - 1 else bf16_round(y.astype(np.float32))
    return a
