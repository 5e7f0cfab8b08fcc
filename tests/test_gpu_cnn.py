"""Proposal-network kernels vs the FP64 network reference (oracle/cnn_oracle.py).

The library's forward and backward passes (bf16 matrix-core products with
FP32 accumulation) are compared with the FP64 reference on the same seeded
parameters, images and targets; the top-K kernel is compared exactly (its
logits are taken from the library's own forward pass, so both sides rank
identical FP32 values).
"""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as C

pytestmark = pytest.mark.gpu

SMALL = C.Arch(box=32, c1=4, c2=8, c3=8, c4=8, hidden=8, nq=50)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1609_06634_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def _init(arch, seed):
    """He-style initial parameters, FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in arch.shapes():
        if name.startswith("W") or name.startswith("F"):
            fan_in = int(np.prod(shape[1:]))
            parts.append(rng.standard_normal(int(np.prod(shape))) * np.sqrt(2.0 / fan_in))
        else:
            parts.append(rng.standard_normal(int(np.prod(shape))) * 0.1)
    return np.concatenate(parts).astype(np.float32)


def _net(P, ctx, arch):
    return P.Net(ctx, arch.box, arch.c1, arch.c2, arch.c3, arch.c4, arch.hidden, arch.nq)


def _data(arch, B, T, seed):
    rng = np.random.default_rng(seed)
    imgs = rng.standard_normal((B, arch.box, arch.box)).astype(np.float32)
    imgs += np.linspace(0, 3, arch.box, dtype=np.float32)[None, None, :]   # some structure
    tidx = np.stack([rng.choice(arch.nq, T, replace=False) for _ in range(B)]).astype(np.int32)
    tp = rng.random((B, T)).astype(np.float32)
    tp /= tp.sum(axis=1, keepdims=True)
    return imgs, tidx, tp


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_forward_matches_reference(P, ctx):
    arch = SMALL
    net = _net(P, ctx, arch)
    w = _init(arch, 1)
    net.set_params(w)
    assert np.array_equal(net.get_params(), w)
    imgs, _, _ = _data(arch, 6, 3, 2)
    z = net.forward(imgs)
    zr, _ = C.forward(arch, w.astype(np.float64), imgs)
    _say(f"forward rel err {_rel(z, zr):.2e}")
    assert _rel(z, zr) < 2e-2
    net.close()


def test_gradient_matches_reference(P, ctx):
    arch = SMALL
    net = _net(P, ctx, arch)
    w = _init(arch, 3)
    net.set_params(w)
    imgs, tidx, tp = _data(arch, 5, 4, 4)
    loss, g = net.backward(imgs, tidx, tp, want_grad=True)
    lr, gr = C.loss_and_grad(arch, w.astype(np.float64), imgs, tidx, tp.astype(np.float64))
    _say(f"loss {loss:.6f} vs {lr:.6f}")
    assert abs(loss - lr) < 2e-2 * max(1.0, abs(lr))
    off = 0
    for name, shape in arch.shapes():
        n = int(np.prod(shape))
        e = _rel(g[off:off + n], gr[off:off + n])
        cos = float(np.dot(g[off:off + n], gr[off:off + n]) /
                    max(np.linalg.norm(g[off:off + n]) * np.linalg.norm(gr[off:off + n]), 1e-30))
        _say(f"  {name}: rel err {e:.2e} cos {cos:.6f}")
        assert e < 5e-2 and cos > 0.998, name
        off += n
    net.close()


def test_gradient_batch_split_and_large_k(P, ctx):
    """A box and batch large enough that the weight-gradient products use
    split-K partial sums: the gradient of two half batches averages to the
    gradient of the whole batch."""
    arch = C.Arch(box=128, c1=8, c2=8, c3=8, c4=8, hidden=8, nq=40)
    net = _net(P, ctx, arch)
    net.set_params(_init(arch, 5))
    imgs, tidx, tp = _data(arch, 8, 2, 6)
    _, g = net.backward(imgs, tidx, tp, want_grad=True)
    _, g1 = net.backward(imgs[:4], tidx[:4], tp[:4], want_grad=True)
    _, g2 = net.backward(imgs[4:], tidx[4:], tp[4:], want_grad=True)
    assert _rel(0.5 * (g1 + g2), g) < 1e-2
    w = _init(arch, 5).astype(np.float64)
    _, gr = C.loss_and_grad(arch, w, imgs, tidx, tp.astype(np.float64))
    assert _rel(g, gr) < 5e-2
    net.close()


def test_adam_reduces_loss(P, ctx):
    arch = SMALL
    net = _net(P, ctx, arch)
    net.set_params(_init(arch, 7))
    imgs, tidx, tp = _data(arch, 16, 2, 8)
    first = None
    for it in range(150):
        loss, _ = net.backward(imgs, tidx, tp)
        first = loss if first is None else first
        net.adam(3e-3)
    _say(f"loss {first:.4f} -> {loss:.4f}")
    assert loss < 0.5 * first
    net.close()


def test_topk_matches_reference(P, ctx):
    arch = C.Arch(box=32, c1=4, c2=8, c3=8, c4=8, hidden=8, nq=3000)
    net = _net(P, ctx, arch)
    net.set_params(_init(arch, 9))
    imgs, _, _ = _data(arch, 7, 1, 10)
    z = net.forward(imgs).astype(np.float64)
    for K in (1, 17, 256, 3000):
        cand, mass = net.propose(imgs, K)
        ref, mref = C.top_k(z, K)
        assert np.array_equal(cand, ref), K
        np.testing.assert_allclose(mass, mref, rtol=1e-5)
    net.close()


def test_topk_reads_torch_output_in_stream_order(P, ctx):
    """The library enqueues on torch's current stream, so a tensor that a
    torch kernel has only just been asked to write is complete when the
    library's kernels read it (top-K makes several passes over its input)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(5)
    big = torch.randn((512, 36864), device="cuda", dtype=torch.float64, generator=g)
    z = big.float()                                   # enqueued, not waited for
    idx, mass = P.topk(ctx, z, 32, device_out=True)
    vals = torch.gather(z, 1, idx.long())             # valid indices only
    ref, _ = C.top_k(z.cpu().numpy().astype(np.float64), 32)
    assert np.array_equal(idx.cpu().numpy(), ref)
    assert vals.shape == (512, 32)


def test_network_input_matches_reference(P, ctx):
    rng = np.random.default_rng(12)
    imgs = rng.standard_normal((5, 48, 40)).astype(np.float32) + 2.0
    got = P.cnn_input(ctx, imgs)
    ref = C.network_input(imgs)
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()


def test_cnn_invalid_arguments(P, ctx):
    with pytest.raises(P.BioemError):
        P.Net(ctx, 40, 4, 4, 4, 4, 4, 10)          # box not a multiple of 16
    net = _net(P, ctx, SMALL)
    net.set_params(_init(SMALL, 1))
    imgs, tidx, tp = _data(SMALL, 2, 2, 1)
    with pytest.raises(P.BioemError):
        net.propose(imgs, SMALL.nq + 1)
    with pytest.raises(P.BioemError):
        net.backward(imgs, tidx + SMALL.nq, tp)   # target outside the grid
    with pytest.raises(P.BioemError):
        net.adam(-1.0)
    net.close()
