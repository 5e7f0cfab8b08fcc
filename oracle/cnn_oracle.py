"""FP64 CPU reference of the orientation-proposal network (test infrastructure).

The proposal network maps one particle image to logits over the orientation
grid; its training targets are the per-orientation posteriors that the method
itself produces (Section 3, Extra features: the posterior restricted to each
orientation).  Architecture (fixed by the proposal design, sizes are
parameters):

    x      = (I - mean I) / sqrt(var I + 1e-12)                 per input
             (the input is normally network_input(image): the image's
             centred autocorrelation, which a shift does not change)
    y_l    = relu(conv3x3_stride2_pad1(y_{l-1}; W_l) + b_l),  l = 1..4
    f      = y_4 flattened, index c*P + p (P = (box/16)^2)     [c4*P]
    h      = relu(F1 f + g1)                                   [hidden]
    z      = F2 h + g2                                         [nq] logits
    loss   = mean over images of  logsumexp(z) - sum_t p_t z_{i_t}

with conv(y)[o][r][s] = b[o] + sum_{c,u,v} W[o][c][u][v] y[c][2r+u-1][2s+v-1]
(zero outside the image).  The targets (i_t, p_t) are a sparse distribution
over orientations (p sums to 1).

Parameters are one flat float vector in this order: W1 [c1][1][3][3], b1,
W2 [c2][c1][3][3], b2, W3, b3, W4, b4, F1 [hidden][c4*P], g1 [hidden],
F2 [nq][hidden], g2 [nq].

Everything here is plain numpy in float64, written for checking by eye, and
is used only by the tests.  Forward and backward are written out layer by
layer; the gradient is pinned by finite differences in the tests.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


@dataclass(frozen=True)
class Arch:
    box: int = 128
    c1: int = 32
    c2: int = 64
    c3: int = 128
    c4: int = 128
    hidden: int = 32
    nq: int = 36864

    def shapes(self) -> List[Tuple[str, Tuple[int, ...]]]:
        ch = [1, self.c1, self.c2, self.c3, self.c4]
        out = []
        for l in range(4):
            out.append((f"W{l + 1}", (ch[l + 1], ch[l], 3, 3)))
            out.append((f"b{l + 1}", (ch[l + 1],)))
        P = (self.box // 16) ** 2
        out += [("F1", (self.hidden, self.c4 * P)), ("g1", (self.hidden,)),
                ("F2", (self.nq, self.hidden)), ("g2", (self.nq,))]
        return out

    def num_params(self) -> int:
        return int(sum(np.prod(s) for _, s in self.shapes()))


def unflatten(arch: Arch, flat: np.ndarray) -> Dict[str, np.ndarray]:
    p, off = {}, 0
    for name, shape in arch.shapes():
        n = int(np.prod(shape))
        p[name] = np.asarray(flat[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    assert off == flat.size
    return p


def flatten(arch: Arch, p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([p[name].ravel() for name, _ in arch.shapes()])


def network_input(imgs: np.ndarray) -> np.ndarray:
    """Circular autocorrelation of each mean-free image, lag 0 moved to pixel
    (H/2, W/2) and set to 0: sum_x u(x) u(x + r) with u = I - mean(I)."""
    x = np.asarray(imgs, dtype=np.float64)
    u = x - x.mean(axis=(1, 2), keepdims=True)
    H, W = u.shape[1:]
    out = np.empty_like(u)
    for b in range(u.shape[0]):
        a = np.fft.irfft2(np.abs(np.fft.rfft2(u[b])) ** 2, s=(H, W))
        a[0, 0] = 0.0
        out[b] = np.roll(a, (H // 2, W // 2), axis=(0, 1))
    return out


def standardize(imgs: np.ndarray) -> np.ndarray:
    x = np.asarray(imgs, dtype=np.float64)
    m = x.mean(axis=(1, 2), keepdims=True)
    v = ((x - m) ** 2).mean(axis=(1, 2), keepdims=True)
    return (x - m) / np.sqrt(v + 1e-12)


def conv_s2(y: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3 convolution, stride 2, zero padding 1.  y [B][C][H][W]."""
    B, C, H, Wd = y.shape
    Ho, Wo = H // 2, Wd // 2
    yp = np.zeros((B, C, H + 2, Wd + 2))
    yp[:, :, 1:H + 1, 1:Wd + 1] = y
    out = np.zeros((B, W.shape[0], Ho, Wo))
    for u in range(3):
        for v in range(3):
            # input pixel (2r+u-1, 2s+v-1) sits at padded index (2r+u, 2s+v)
            patch = yp[:, :, u:u + 2 * Ho:2, v:v + 2 * Wo:2]          # [B][C][Ho][Wo]
            out += np.einsum("oc,bcrs->bors", W[:, :, u, v], patch)
    return out + b[None, :, None, None]


def conv_s2_backward(y: np.ndarray, W: np.ndarray, dout: np.ndarray):
    """Gradients of conv_s2 with respect to its input, weights and bias."""
    B, C, H, Wd = y.shape
    Ho, Wo = H // 2, Wd // 2
    yp = np.zeros((B, C, H + 2, Wd + 2))
    yp[:, :, 1:H + 1, 1:Wd + 1] = y
    dyp = np.zeros_like(yp)
    dW = np.zeros_like(W)
    for u in range(3):
        for v in range(3):
            patch = yp[:, :, u:u + 2 * Ho:2, v:v + 2 * Wo:2]
            dW[:, :, u, v] = np.einsum("bors,bcrs->oc", dout, patch)
            dyp[:, :, u:u + 2 * Ho:2, v:v + 2 * Wo:2] += np.einsum("oc,bors->bcrs", W[:, :, u, v], dout)
    db = dout.sum(axis=(0, 2, 3))
    return dyp[:, :, 1:H + 1, 1:Wd + 1], dW, db


def forward(arch: Arch, flat: np.ndarray, imgs: np.ndarray):
    """Logits [B][nq] and the activations the backward pass needs."""
    p = unflatten(arch, flat)
    x = standardize(imgs)[:, None]          # [B][1][box][box]
    acts = [x]
    y = x
    for l in range(1, 5):
        y = np.maximum(conv_s2(y, p[f"W{l}"], p[f"b{l}"]), 0.0)
        acts.append(y)
    f = y.reshape(y.shape[0], -1)           # [B][c4*P]
    h = np.maximum(f @ p["F1"].T + p["g1"], 0.0)
    z = h @ p["F2"].T + p["g2"]
    return z, (p, acts, f, h)


def softmax_xent(z: np.ndarray, tidx: np.ndarray, tp: np.ndarray):
    """Mean soft-label cross entropy and its gradient with respect to z."""
    B = z.shape[0]
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    s = e.sum(axis=1, keepdims=True)
    lse = (m + np.log(s))[:, 0]
    tgt = np.zeros_like(z)
    for b in range(B):
        np.add.at(tgt[b], tidx[b], tp[b])
    loss = float(np.mean(lse - (tgt * z).sum(axis=1)))
    dz = (e / s - tgt) / B
    return loss, dz


def loss_and_grad(arch: Arch, flat: np.ndarray, imgs: np.ndarray, tidx: np.ndarray, tp: np.ndarray):
    """Loss and its gradient with respect to every parameter (flat)."""
    z, (p, acts, f, h) = forward(arch, flat, imgs)
    loss, dz = softmax_xent(z, tidx, tp)
    g = {}
    g["F2"] = dz.T @ h
    g["g2"] = dz.sum(axis=0)
    dh = (dz @ p["F2"]) * (h > 0)
    g["F1"] = dh.T @ f
    g["g1"] = dh.sum(axis=0)
    df = dh @ p["F1"]                                   # [B][c4*P]
    dy = df.reshape(acts[4].shape)
    for l in range(4, 0, -1):
        dy = dy * (acts[l] > 0)                         # through the relu of layer l
        dx, g[f"W{l}"], g[f"b{l}"] = conv_s2_backward(acts[l - 1], p[f"W{l}"], dy)
        dy = dx
    return loss, flatten(arch, g)


def top_k(z: np.ndarray, K: int):
    """Per row: the K largest logits (ties to the lower index), returned in
    increasing index order, and the softmax mass they hold."""
    out = np.empty((z.shape[0], K), np.int64)
    mass = np.empty(z.shape[0])
    for b, row in enumerate(z):
        order = np.lexsort((np.arange(row.size), -row))[:K]
        out[b] = np.sort(order)
        e = np.exp(row - row.max())
        mass[b] = e[order].sum() / e.sum()
    return out, mass


def adam_step(w: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float, beta1: float,
              beta2: float, eps: float):
    """One Adam update with bias correction (Kingma and Ba, "Adam: a method
    for stochastic optimization", ICLR 2015, Algorithm 1), in FP64; t is the
    1-based step count.  The moments are exponential averages of g and g^2,
    divided by 1 - beta^t so that they are unbiased from a zero start; the
    parameter moves by lr times their ratio.  Returns (w, m, v) after the
    step; the inputs are not modified."""
    w = np.asarray(w, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
