"""CPU reference of the local-basis surrogate network (test infrastructure).

The surrogate maps a subdomain's permeability patch and its Robin
parameters to its local basis (the pressures of the basis problems of
Section 2.1, one field per boundary segment).  This module is the plain
FP64 definition of that network, used only to check the GPU kernels'
forward pass and gradients; it shares no code with them.

Network (patch side S, hidden width C, L >= 2 convolution layers, R
outputs):
    h_0 = x (2 input channels)
    h_{l+1} = relu(conv3x3(h_l, W_l) + b_l)        l = 0 .. L-2
    y = conv3x3(h_{L-1}, W_{L-1}) + b_{L-1} + Bmap
3x3 cross-correlation with zero padding 1; W_0: C x 2, W_l: C x C,
W_{L-1}: R x C; Bmap: R x S x S (a learned mean field per output).
The convolution weights enter in bfloat16 (round to nearest even of the
FP32 master weight); biases and Bmap stay FP32.  Gradients are taken with
respect to the rounded weights and applied to the master weights.
Loss: mean squared error over every output value.

Parameter vector order: for each layer W_l (row-major [co][ci][3][3]),
then b_l; finally Bmap ([R][S][S]).

Input features of a patch (`features`):
    channel 0: log K - mean(log K over the patch)
    channel 1: on boundary cells, the mean over the cell's boundary faces of
               log(beta_a) + mean(log K), beta_a the Robin parameter of the
               face's segment; 0 on interior cells.
Both channels are unchanged when K is scaled by c (beta scales by 1/c, the
Robin parameter equation of Section 5.1), as is the basis itself.
"""

from __future__ import annotations

import numpy as np


def layer_shapes(C: int, L: int, R: int):
    """(co, ci) of every convolution layer."""
    if L < 2:
        raise ValueError("at least two layers")
    sh = [(C, 2)] + [(C, C)] * (L - 2) + [(R, C)]
    return sh


def num_params(S: int, C: int, L: int, R: int) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(C, L, R)) + R * S * S


def unpack(theta, S, C, L, R):
    out, k = [], 0
    for co, ci in layer_shapes(C, L, R):
        W = theta[k:k + co * ci * 9].reshape(co, ci, 3, 3)
        k += co * ci * 9
        b = theta[k:k + co]
        k += co
        out.append((W, b))
    Bmap = theta[k:k + R * S * S].reshape(R, S, S)
    return out, Bmap


def bf16_round(a):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as
    float64 holding the rounded value."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, W, b):
    """y[n,co,i,j] = b[co] + sum_{ci,di,dj} W[co,ci,di,dj] x[n,ci,i+di-1,j+dj-1]
    (zero outside the patch); x: [N, ci, S, S] with [..., row j, column i]
    stored as [..., j, i] like the permeability arrays."""
    N, ci, S, _ = x.shape
    xp = np.zeros((N, ci, S + 2, S + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((N, W.shape[0], S, S))
    for a in range(3):
        for c in range(3):
            patch = xp[:, :, a:a + S, c:c + S]           # [N, ci, S, S]
            y += np.einsum("oc,ncij->noij", W[:, :, a, c], patch)
    return y + b[None, :, None, None]


def conv3x3_grads(x, W, dy):
    """Gradients of sum(dy * conv3x3(x, W, b)) with respect to x, W and b."""
    N, ci, S, _ = x.shape
    xp = np.zeros((N, ci, S + 2, S + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for a in range(3):
        for c in range(3):
            patch = xp[:, :, a:a + S, c:c + S]
            dW[:, :, a, c] = np.einsum("noij,ncij->oc", dy, patch)
            dxp[:, :, a:a + S, c:c + S] += np.einsum("oc,noij->ncij", W[:, :, a, c], dy)
    db = dy.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dW, db


def forward(theta, x, S, C, L, R, round_weights=True):
    layers, Bmap = unpack(np.asarray(theta, dtype=np.float64), S, C, L, R)
    hs = [np.asarray(x, dtype=np.float64)]
    for l, (W, b) in enumerate(layers):
        Wr = bf16_round(W) if round_weights else W
        z = conv3x3(hs[-1], Wr, b)
        if l < L - 1:
            z = np.maximum(z, 0.0)
        hs.append(z)
    y = hs[-1] + Bmap[None]
    return y, hs


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def loss_and_grad(theta, x, t, S, C, L, R, round_weights=True):
    """Loss and its gradient (with respect to the rounded weights, applied
    to the parameter vector)."""
    layers, Bmap = unpack(np.asarray(theta, dtype=np.float64), S, C, L, R)
    y, hs = forward(theta, x, S, C, L, R, round_weights)
    loss, dy = mse(y, t)
    grads = []
    g = dy
    dBmap = dy.sum(axis=0)
    for l in range(L - 1, -1, -1):
        W, b = layers[l]
        Wr = bf16_round(W) if round_weights else W
        if l < L - 1:
            g = g * (hs[l + 1] > 0.0)
        gx, gW, gb = conv3x3_grads(hs[l], Wr, g)
        grads.append((gW, gb))
        g = gx
    grads.reverse()
    flat = [np.concatenate([gW.ravel(), gb]) for gW, gb in grads] + [dBmap.ravel()]
    return loss, np.concatenate(flat)


def features(Kpatch, beta_sides, seg):
    """Input channels of one S x S patch.  beta_sides: (4, S // seg) Robin
    parameters of the W, E, S, N segments (bottom to top / left to right)."""
    S = Kpatch.shape[0]
    lk = np.log(Kpatch)
    m = lk.mean()
    x = np.zeros((2, S, S))
    x[0] = lk - m
    acc = np.zeros((S, S))
    cnt = np.zeros((S, S))
    lb = np.log(np.asarray(beta_sides, dtype=np.float64)) + m
    for t in range(S):
        s = t // seg
        acc[t, 0] += lb[0, s]
        cnt[t, 0] += 1      # W face of cell (0, t)
        acc[t, S - 1] += lb[1, s]
        cnt[t, S - 1] += 1  # E face of cell (S-1, t)
        acc[0, t] += lb[2, s]
        cnt[0, t] += 1      # S face of cell (t, 0)
        acc[S - 1, t] += lb[3, s]
        cnt[S - 1, t] += 1  # N face of cell (t, S-1)
    x[1] = np.where(cnt > 0, acc / np.maximum(cnt, 1), 0.0)
    return x
