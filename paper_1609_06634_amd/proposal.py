"""Learned orientation proposal: training data, training loop, pruned scoring.

The proposal network (bioem_cnn_* in include/bioem.h) maps a particle image
to logits over the orientation grid.  Its training targets are the
per-orientation posteriors that bioem_logpost computes on synthetic images
(the posterior restricted to each orientation, Section 3 Extra features):
for every training image the T most probable orientations and their
renormalised posterior probabilities.  At scoring time the network's top-K
orientations per image become bioem_logpost's candidate list (the log
posterior keeps the full-grid prior, so it is a lower bound of the exhaustive
value); images whose softmax mass in the top K is below tau are scored on the
full grid instead.

All arithmetic runs in the library (rendering, transforms, posteriors,
network forward/backward, top-K); this module sequences the calls and moves
small arrays (targets, masses, index lists).
"""
from __future__ import annotations

import time
from dataclasses import dataclass
import numpy as np

from . import bindings as B


def quaternion_features(quats: np.ndarray) -> np.ndarray:
    """The ten distinct products q_a q_b of each unit quaternion (invariant
    under q -> -q, so equal for both signs of one rotation)."""
    w, x, y, z = quats.T
    return np.stack([w * w, x * x, y * y, z * z, 2 * w * x, 2 * w * y, 2 * w * z, 2 * x * y, 2 * x * z,
                     2 * y * z], axis=1)


def _shapes(arch: B.CnnArch):
    ch = [1, arch.c1, arch.c2, arch.c3, arch.c4]
    out = []
    for l in range(4):
        out.append((f"W{l + 1}", (ch[l + 1], ch[l], 3, 3)))
        out.append((f"b{l + 1}", (ch[l + 1],)))
    P = (arch.box // 16) ** 2
    out += [("F1", (arch.hidden, arch.c4 * P)), ("g1", (arch.hidden,)),
            ("F2", (arch.nq, arch.hidden)), ("g2", (arch.nq,))]
    return out


def init_params(net: B.Net, quats: np.ndarray, seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Initial parameters: He-normal convolution and hidden weights, zero
    biases, and an output layer whose first 20 columns are +-scale times the
    quaternion products of each grid orientation, so that a hidden code can
    express logits of the form q^T M q (a Bingham density over rotations)
    from the start; the remaining columns are small random values."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in _shapes(net.arch):
        n = int(np.prod(shape))
        if name == "F2":
            F = rng.standard_normal(shape) * 0.01
            feat = quaternion_features(np.asarray(quats, np.float64))
            k = min(10, shape[1] // 2)
            F[:, :k] = scale * feat[:, :k]
            F[:, k:2 * k] = -scale * feat[:, :k]
            parts.append(F.ravel())
        elif name.startswith("W") or name == "F1":
            fan_in = int(np.prod(shape[1:]))
            parts.append(rng.standard_normal(n) * np.sqrt(2.0 / fan_in))
        else:
            parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


@dataclass
class TrainingSet:
    inputs: "object"          # torch CUDA tensor [n][box][box] float32: network inputs
    tidx: np.ndarray          # [n][T] int32
    tp: np.ndarray            # [n][T] float32
    mass: np.ndarray          # [n] posterior mass of the T targets
    seconds: float


def render_class_images(ctx: B.Context, model_dev, cls, i0: int, i1: int):
    """Images i0..i1 of a size class, rendered on the device with their own
    orientation, CTF, shift and noise (device tensor)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    pr = B.project(ctx, model_dev, torch.from_numpy(cls.img_quat[i0:i1]).to(dev), cls.nx, cls.ny, cls.pixel_A)
    out = B.render(ctx, pr, torch.from_numpy(cls.img_ctf[i0:i1]).to(dev),
                   torch.from_numpy(cls.img_shift[i0:i1]).to(dev),
                   noise=torch.from_numpy(cls.noise(i0, i1)).to(dev), snr=cls.snr, device_out=True)
    pr.free()
    return out


def smooth_targets(quats: np.ndarray, top: np.ndarray, T: int, sigma_deg: float):
    """Soft targets around each image's most probable orientation: the T grid
    orientations nearest to it (rotation angle 2 arccos|q.q'|) with weights
    exp(-angle^2 / (2 sigma^2)), normalised.  A training choice: the
    posteriors themselves are nearly one-hot at these signal levels, and a
    spread target gives neighbouring orientations a consistent gradient."""
    q = np.asarray(quats, np.float64)
    idx = np.empty((len(top), T), np.int32)
    p = np.empty((len(top), T), np.float32)
    s = np.deg2rad(sigma_deg)
    for i0 in range(0, len(top), 512):
        t = top[i0:i0 + 512]
        dots = np.abs(q[t] @ q.T).clip(0.0, 1.0)
        part = np.argpartition(-dots, T - 1, axis=1)[:, :T]
        ang = 2.0 * np.arccos(np.take_along_axis(dots, part, axis=1))
        w = np.exp(-ang ** 2 / (2 * s * s))
        idx[i0:i0 + 512] = part
        p[i0:i0 + 512] = w / w.sum(axis=1, keepdims=True)
    return idx, p


def make_training_set(ctx: B.Context, model: np.ndarray, cls, proj_grid: B.Projections, T: int = 32,
                      chunk: int = 1000, prec: str = "split_f16", smooth_deg: float = 0.0,
                      log=None) -> TrainingSet:
    """Render the class's images, keep their network inputs (``cnn_input``)
    and label each with its T most probable orientations under the
    exhaustive posterior (renormalised over the T), or, with smooth_deg > 0,
    with soft targets around its most probable orientation
    (``smooth_targets``)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    t0 = time.perf_counter()
    model_dev = torch.from_numpy(model).to(dev)
    ctf = torch.from_numpy(cls.ctf).to(dev)
    n = cls.n_images
    inputs = torch.empty((n, cls.ny, cls.nx), dtype=torch.float32, device=dev)
    tidx = np.empty((n, T), np.int32)
    tp = np.empty((n, T), np.float32)
    mass = np.empty(n, np.float32)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        imgs = render_class_images(ctx, model_dev, cls, i0, i1)
        inputs[i0:i1] = B.cnn_input(ctx, imgs, device_out=True)
        im = B.prepare_images(ctx, imgs)
        out = B.logpost(ctx, proj_grid, im, ctf, cls.max_shift, prec=prec, orient=True, device_out=True)
        im.free()
        lo = out["orient"].float()                  # log posterior per orientation
        idx, m = B.topk(ctx, lo, T, device_out=True)
        vals = torch.gather(out["orient"], 1, idx.long()).cpu().numpy()
        p = np.exp(vals - vals.max(axis=1, keepdims=True))
        tidx[i0:i1] = idx.cpu().numpy()
        tp[i0:i1] = (p / p.sum(axis=1, keepdims=True)).astype(np.float32)
        mass[i0:i1] = m.cpu().numpy()
        if log:
            log(f"labels {i1}/{n} ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    if smooth_deg > 0.0:
        best = tidx[np.arange(n), np.argmax(tp, axis=1)]
        tidx, tp = smooth_targets(cls.quats, best, T, smooth_deg)
    return TrainingSet(inputs=inputs, tidx=tidx, tp=tp, mass=mass, seconds=time.perf_counter() - t0)


def train(net: B.Net, data: TrainingSet, epochs: int = 4, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, log=None, plateau: float = 0.0, patience: int = 3) -> list:
    """Adam on shuffled mini-batches; returns the mean loss of every epoch.
    With plateau > 0 training stops early once the best epoch loss has not
    improved by that relative amount for ``patience`` epochs (at most
    ``epochs`` in all)."""
    import torch
    rng = np.random.default_rng(seed)
    n = data.inputs.shape[0]
    dev = data.inputs.device
    tidx = torch.from_numpy(data.tidx).to(dev)
    tp = torch.from_numpy(data.tp).to(dev)
    losses = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            sel = torch.from_numpy(order[b0:b0 + batch]).to(dev)
            loss, _ = net.backward(data.inputs[sel].contiguous(), tidx[sel].contiguous(), tp[sel].contiguous())
            net.adam(lr)
            tot += loss
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {losses[-1]:.4f}")
        if plateau > 0.0 and len(losses) > patience:
            before = min(losses[:-patience])
            if min(losses[-patience:]) > before * (1.0 - plateau):
                if log:
                    log(f"loss plateau after {ep + 1} epochs")
                break
    return losses


@dataclass
class ProposalResult:
    logp: np.ndarray          # [ni] log posterior (pruned, or exhaustive where fallen back)
    fallback: np.ndarray      # [ni] bool
    mass: np.ndarray          # [ni] network softmax mass in the top K
    seconds: float
    evals: float              # evaluations actually computed


def score_with_proposal(ctx: B.Context, net: B.Net, proj_grid: B.Projections, images, ctf, max_shift: int,
                        K: int = 256, tau: float = 0.5, prec: str = "split_f16") -> ProposalResult:
    """Posterior of every image with the network's top-K orientations, and
    the full grid for images whose top-K softmax mass is below tau."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nc = int(ctf.shape[0])
    cand, mass = net.propose(B.cnn_input(ctx, images, device_out=True), K, device_out=True)
    im = B.prepare_images(ctx, images)
    out = B.logpost(ctx, proj_grid, im, ctf, max_shift, prec=prec, cand_q=cand, device_out=True)
    logp = out["logp"]
    m = mass.cpu().numpy()
    fb = m < tau
    evals = float(images.shape[0]) * K * nc
    if fb.any():
        sel = torch.from_numpy(np.nonzero(fb)[0]).to(images.device)
        im2 = B.prepare_images(ctx, images[sel].contiguous())
        ex = B.logpost(ctx, proj_grid, im2, ctf, max_shift, prec=prec, device_out=True)
        logp[sel] = ex["logp"]
        im2.free()
        evals += float(fb.sum()) * proj_grid.n * nc
    im.free()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return ProposalResult(logp=logp.cpu().numpy(), fallback=fb, mass=m, seconds=dt, evals=evals)
