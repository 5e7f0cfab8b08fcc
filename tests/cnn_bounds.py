"""Element-wise error bounds of the proposal network as the library computes
it, for the network parity tests.

The library's arithmetic: every matrix product (each convolution as
weights x im2col columns, the two dense layers, and every product of the
backward pass) rounds its FP32 operands to bf16 (round to nearest even, unit
roundoff u = 2^-8) and accumulates in FP32 (unit roundoff e = 2^-24);
standardisation, bias, ReLU, softmax, row sums and col2im are FP32.

A worst-case bound (every rounding error aligned) grows by the sum of
|weights| per layer and is useless after six layers, so the bound here is
statistical: each rounding is an independent error of variance at most
(u |x|)^2 / 3 (e for FP32), and a product C = A B whose operands carry
independent errors of standard deviations sA, sB has

    var(C_lib - C) = sA^2 B^2 + A^2 sB^2 + (2 u^2 / 3) (A B)^2
                     + (K e^2 / 3) (|A| |B|)^2        (element-wise squares)

(K the summation length).  Standard deviations are propagated layer by
layer in FP64 from the network reference (oracle/cnn_oracle.py); ReLU passes
an error through, softmax as d ln p_i = dz_i - sum_j p_j dz_j.  Where a
reference pre-activation lies within the bound of zero, the library's ReLU
mask may differ from the reference's: there the whole reference gradient
value is added as a deterministic term D, carried through the later products
by absolute values.  The bound of an element is K_SIGMA standard deviations
plus D.  ``emulate_loss_and_grad`` recomputes the network with the products'
operands rounded (FP64 elsewhere); the CPU tests check that its deviation
from the reference stays inside the bound and that coarser rounding does not.
"""
import numpy as np

from oracle import cnn_oracle as C

U = 2.0 ** -8     # bf16 unit roundoff
E = 2.0 ** -24    # FP32 unit roundoff
K_SIGMA = 8.0     # standard deviations allowed per element


def bf16_round(x, bits: int = 8):
    """Round to a binary significand of ``bits`` bits (8: bf16), nearest even,
    after rounding to FP32 (the library's operands are FP32 values)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    drop = 24 - bits
    half = (1 << (drop - 1)) - 1
    r = ((u + half + ((u >> drop) & 1)) >> drop) << drop
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _var_prod(mm, A, B, vA, vB, K):
    """Variance of a product's error: mm(x, y) is the product with squared
    (or absolute) operands substituted, e.g. x @ y."""
    return (mm(vA, B * B) + mm(A * A, vB) + (2 * U * U / 3) * mm(A * A, B * B)
            + (K * E * E / 3) * mm(np.abs(A), np.abs(B)) ** 2)


def _conv(a, w):
    return C.conv_s2(a, w, np.zeros(w.shape[0]))


def forward_bound(arch, flat, imgs):
    """(z, var_z, D_z, cache): reference logits, the variance of the library's
    error and the deterministic part (from ReLU masks near zero)."""
    z, (p, acts, f, h) = C.forward(arch, flat, imgs)
    B = z.shape[0]
    vacts = [(E * acts[0]) ** 2 / 3]              # FP64 standardisation stored as FP32
    Dacts = [np.zeros_like(acts[0])]
    pres, vpres, Dpres = [None], [None], [None]
    for l in range(1, 5):
        W, b = p[f"W{l}"], p[f"b{l}"]
        y = acts[l - 1]
        pre = C.conv_s2(y, W, b)
        K = W.shape[1] * 9
        vpre = _var_prod(lambda a, w: _conv(a, w), y, W, vacts[l - 1], 0.0 * W, K) + (E * pre) ** 2 / 3
        Dpre = _conv(Dacts[l - 1], np.abs(W)) * (1 + U)
        # ReLU: the error passes where the output is pre; where pre lies
        # below minus its bound both outputs are 0 and no error passes (in
        # between the deviation is at most that of pre)
        pres.append(pre)
        vpres.append(vpre)
        Dpres.append(Dpre)
        live = pre > -bound(vpre, Dpre)
        vacts.append(np.where(live, vpre, 0.0))
        Dacts.append(np.where(live, Dpre, 0.0))
    vf = vacts[4].reshape(B, -1)
    Df = Dacts[4].reshape(B, -1)
    F1, F2 = p["F1"], p["F2"]
    h_pre = f @ F1.T + p["g1"]
    vh_pre = _var_prod(lambda a, w: a @ w, f, F1.T, vf, 0.0 * F1.T, F1.shape[1]) + (E * h_pre) ** 2 / 3
    Dh_pre = (Df @ np.abs(F1).T) * (1 + U)
    live = h_pre > -bound(vh_pre, Dh_pre)
    vh, Dh = np.where(live, vh_pre, 0.0), np.where(live, Dh_pre, 0.0)
    vz = _var_prod(lambda a, w: a @ w, h, F2.T, vh, 0.0 * F2.T, F2.shape[1]) + (E * z) ** 2 / 3
    Dz = (Dh @ np.abs(F2).T) * (1 + U)
    cache = dict(p=p, acts=acts, vacts=vacts, Dacts=Dacts, pres=pres, vpres=vpres, Dpres=Dpres, f=f, vf=vf,
                 Df=Df, h=h, vh=vh, Dh=Dh, h_pre=h_pre, vh_pre=vh_pre, Dh_pre=Dh_pre)
    return z, vz, Dz, cache


def bound(v, D):
    return K_SIGMA * np.sqrt(v) + D


def _targets(z, tidx, tp):
    tgt = np.zeros_like(z)
    for b in range(z.shape[0]):
        np.add.at(tgt[b], tidx[b], tp[b])
    return tgt


def _masked(grad, vgrad, Dgrad, pre, vpre, Dpre):
    """Gradient through a ReLU: reference value, variance and deterministic
    part; where the pre-activation is within its bound of zero the mask may
    flip, and the whole reference value joins the deterministic part."""
    on = pre > 0
    uncertain = np.abs(pre) <= bound(vpre, Dpre)
    g = grad * on
    v = np.where(uncertain, vgrad, on * vgrad)
    D = np.where(uncertain, np.abs(grad) + Dgrad, on * Dgrad)
    return g, v, D


def grad_bound(arch, flat, imgs, tidx, tp):
    """(loss, g, z, loss_bound, g_bound, z_bound): reference loss, gradient
    (flat) and logits with element-wise bounds of the library's errors."""
    z, vz, Dz, c = forward_bound(arch, flat, imgs)
    p, acts = c["p"], c["acts"]
    B, nq = z.shape
    zm = z - z.max(axis=1, keepdims=True)
    pz = np.exp(zm) / np.exp(zm).sum(axis=1, keepdims=True)
    tgt = _targets(z, tidx, tp)
    # d ln p_i = dz_i - sum_j p_j dz_j (independent parts), plus FP32 softmax
    vp = pz ** 2 * (vz + (pz ** 2 * vz).sum(axis=1, keepdims=True)) + ((nq + 16) * E * pz) ** 2 / 3
    Dp = pz * np.expm1(np.minimum(Dz + Dz.max(axis=1, keepdims=True), 50.0))
    dz = (pz - tgt) / B
    vdz = (vp + (E * (pz - tgt)) ** 2 / 3) / B ** 2
    Ddz = Dp / B
    lse = z.max(axis=1) + np.log(np.exp(zm).sum(axis=1))
    loss = float(np.mean(lse - (tgt * z).sum(axis=1)))
    vloss = np.mean((pz ** 2 * vz).sum(axis=1) + (tgt ** 2 * vz).sum(axis=1)) / B \
        + ((nq + 16) * E * np.mean(np.abs(lse) + (tgt * np.abs(z)).sum(axis=1))) ** 2 / 3
    loss_bound = float(K_SIGMA * np.sqrt(vloss) + np.mean(Dz.max(axis=1) + (tgt * Dz).sum(axis=1)))
    g, v, D = {}, {}, {}
    h, vh, Dh, f, vf, Df = c["h"], c["vh"], c["Dh"], c["f"], c["vf"], c["Df"]
    F1, F2 = p["F1"], p["F2"]
    mm = lambda a, b: a @ b
    g["F2"] = dz.T @ h
    v["F2"] = _var_prod(mm, dz.T, h, vdz.T, vh, B)
    D["F2"] = (Ddz.T @ np.abs(h) + np.abs(dz).T @ Dh) * (1 + U)
    g["g2"] = dz.sum(axis=0)
    v["g2"] = vdz.sum(axis=0) + (B * E * np.abs(dz).sum(axis=0)) ** 2 / 3
    D["g2"] = Ddz.sum(axis=0)
    dh_pre = dz @ F2
    vdh = _var_prod(mm, dz, F2, vdz, 0.0 * F2, nq)
    Ddh = (Ddz @ np.abs(F2)) * (1 + U)
    dh, vdh, Ddh = _masked(dh_pre, vdh, Ddh, c["h_pre"], c["vh_pre"], c["Dh_pre"])
    g["F1"] = dh.T @ f
    v["F1"] = _var_prod(mm, dh.T, f, vdh.T, vf, B)
    D["F1"] = (Ddh.T @ np.abs(f) + np.abs(dh).T @ Df) * (1 + U)
    g["g1"] = dh.sum(axis=0)
    v["g1"] = vdh.sum(axis=0) + (B * E * np.abs(dh).sum(axis=0)) ** 2 / 3
    D["g1"] = Ddh.sum(axis=0)
    df = dh @ F1
    vdf = _var_prod(mm, dh, F1, vdh, 0.0 * F1, F1.shape[0])
    Ddf = (Ddh @ np.abs(F1)) * (1 + U)
    shape4 = acts[4].shape
    dy, vdy, Ddy = df.reshape(shape4), vdf.reshape(shape4), Ddf.reshape(shape4)
    for l in range(4, 0, -1):
        W = p[f"W{l}"]
        dym, vdym, Ddym = _masked(dy, vdy, Ddy, c["pres"][l], c["vpres"][l], c["Dpres"][l])
        n_pix = dym[:, 0].size
        g[f"b{l}"] = dym.sum(axis=(0, 2, 3))
        v[f"b{l}"] = vdym.sum(axis=(0, 2, 3)) + (n_pix * E * np.abs(dym).sum(axis=(0, 2, 3))) ** 2 / 3
        D[f"b{l}"] = Ddym.sum(axis=(0, 2, 3))
        y, vy, Dy = acts[l - 1], c["vacts"][l - 1], c["Dacts"][l - 1]
        dx, g[f"W{l}"], _ = C.conv_s2_backward(y, W, dym)
        dW = lambda a, b: C.conv_s2_backward(a, W, b)[1]            # bilinear in (y, dout)
        v[f"W{l}"] = _var_prod(dW, y, dym, vy, vdym, n_pix)
        D[f"W{l}"] = (dW(Dy, np.abs(dym)) + dW(np.abs(y), Ddym)) * (1 + U)
        if l > 1:
            dX = lambda a, b: C.conv_s2_backward(y, a, b)[0]          # bilinear in (W, dout)
            vdx = _var_prod(dX, W, dym, 0.0 * W, vdym, W.shape[0] + 4)
            Ddx = dX(np.abs(W), Ddym) * (1 + U)
            dy, vdy, Ddy = dx, vdx, Ddx
    flat_b = C.flatten(arch, {k: bound(v[k], D[k]) for k in g})
    return loss, C.flatten(arch, g), z, loss_bound, flat_b, bound(vz, Dz)


def emulate_loss_and_grad(arch, flat, imgs, tidx, tp, bits: int = 8):
    """The network with every product's operands rounded to ``bits``
    significand bits (FP64 elsewhere): (loss, flat gradient, logits)."""
    r = lambda x: bf16_round(x, bits)
    p = C.unflatten(arch, np.asarray(flat, np.float64))
    x = C.standardize(imgs)[:, None]
    acts, pres = [x], [None]
    y = x
    for l in range(1, 5):
        pre = C.conv_s2(r(y), r(p[f"W{l}"]), p[f"b{l}"])
        y = np.maximum(pre, 0.0)
        acts.append(y)
        pres.append(pre)
    f = y.reshape(y.shape[0], -1)
    h_pre = r(f) @ r(p["F1"]).T + p["g1"]
    h = np.maximum(h_pre, 0.0)
    z = r(h) @ r(p["F2"]).T + p["g2"]
    loss, dz = C.softmax_xent(z, tidx, tp)
    g = {}
    g["F2"] = r(dz).T @ r(h)
    g["g2"] = dz.sum(axis=0)
    dh = (r(dz) @ r(p["F2"])) * (h_pre > 0)
    g["F1"] = r(dh).T @ r(f)
    g["g1"] = dh.sum(axis=0)
    dy = (r(dh) @ r(p["F1"])).reshape(acts[4].shape)
    for l in range(4, 0, -1):
        dy = dy * (pres[l] > 0)
        dx, g[f"W{l}"], _ = C.conv_s2_backward(r(acts[l - 1]), r(p[f"W{l}"]), r(dy))
        g[f"b{l}"] = dy.sum(axis=(0, 2, 3))
        dy = dx
    return loss, C.flatten(arch, g), z
