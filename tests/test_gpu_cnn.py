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

import cnn_bounds as CB

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
    """Logits element by element within the bf16-product bound (cnn_bounds)."""
    arch = SMALL
    net = _net(P, ctx, arch)
    w = _init(arch, 1)
    net.set_params(w)
    assert np.array_equal(net.get_params(), w)
    imgs, _, _ = _data(arch, 6, 3, 2)
    z = net.forward(imgs)
    zr, vz, Dz, _ = CB.forward_bound(arch, w.astype(np.float64), imgs)
    Ez = CB.bound(vz, Dz)
    r = np.abs(z - zr) / Ez
    _say(f"forward: max |dz|/bound {r.max():.3f}, rel err {_rel(z, zr):.2e}")
    assert np.all(np.abs(z - zr) <= Ez)
    net.close()


def test_gradient_matches_reference(P, ctx):
    """Loss and every gradient element within the bf16-product bounds."""
    arch = SMALL
    net = _net(P, ctx, arch)
    w = _init(arch, 3)
    net.set_params(w)
    imgs, tidx, tp = _data(arch, 5, 4, 4)
    loss, g = net.backward(imgs, tidx, tp, want_grad=True)
    lr, gr, _, Eloss, Eg, _ = CB.grad_bound(arch, w.astype(np.float64), imgs, tidx, tp.astype(np.float64))
    _say(f"loss {loss:.6f} vs {lr:.6f} (bound {Eloss:.2e})")
    assert abs(loss - lr) <= Eloss
    off = 0
    for name, shape in arch.shapes():
        n = int(np.prod(shape))
        d, e = np.abs(g[off:off + n] - gr[off:off + n]), Eg[off:off + n]
        _say(f"  {name}: max |dg|/bound {np.max(d / np.maximum(e, 1e-300)):.3f}, rel err {_rel(g[off:off + n], gr[off:off + n]):.2e}")
        assert np.all(d <= e), name
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


def test_adam_matches_reference(P, ctx):
    """bioem_cnn_adam against the FP64 Adam step (cnn_oracle.adam_step).

    Phase 1: three steps with one gradient (backward once, adam three times):
    the corrected moments stay g and g^2, so both sides move each weight by
    3 lr g/(|g| + eps), checked where the reference gradient's sign is
    certain (|g| above its bf16 bound).  Phase 2: one more step with the
    gradient of another batch at the new parameters; where both gradients
    have the same sign and relative bounds rho <= 10%, the step changes by at
    most 2 rho / (1 - rho) of itself, so the library's step must match the
    reference within that; the same check against a reference with beta1 and
    beta2 swapped must fail somewhere (the test can tell)."""
    arch = SMALL
    lr, b1, b2, eps = 1e-3, 0.3, 0.99, 1e-10
    net = _net(P, ctx, arch)
    w0 = _init(arch, 9)
    net.set_params(w0)
    imgs_a, tidx_a, tp_a = _data(arch, 6, 3, 10)
    imgs_b, tidx_b, tp_b = _data(arch, 6, 3, 11)
    net.backward(imgs_a, tidx_a, tp_a)
    for _ in range(3):
        net.adam(lr, b1, b2, eps)
    w3 = net.get_params().astype(np.float64)
    W0 = w0.astype(np.float64)
    _, ga, _, _, Ega, _ = CB.grad_bound(arch, W0, imgs_a, tidx_a, tp_a.astype(np.float64))
    wr, m, v = W0, np.zeros_like(W0), np.zeros_like(W0)
    for t in range(1, 4):
        wr, m, v = C.adam_step(wr, ga, m, v, t, lr, b1, b2, eps)
    sure = np.abs(ga) > Ega + 1e-4
    fp32 = 4 * 2.0 ** -24 * (np.abs(W0) + 3 * lr)
    _say(f"adam phase 1: {sure.sum()} of {sure.size} weights with a certain gradient sign")
    assert sure.sum() > 0.3 * sure.size
    np.testing.assert_array_less(np.abs(w3 - wr)[sure], (3 * lr * 1e-5 + fp32)[sure])
    assert np.all(np.abs(w3 - W0) <= 3 * lr * (1 + 1e-5) + fp32)
    # phase 2: a different gradient, at the new parameters
    net.backward(imgs_b, tidx_b, tp_b)
    net.adam(lr, b1, b2, eps)
    w4 = net.get_params().astype(np.float64)
    _, gb, _, _, Egb, _ = CB.grad_bound(arch, wr, imgs_b, tidx_b, tp_b.astype(np.float64))
    w4r, _, _ = C.adam_step(wr, gb, m, v, 4, lr, b1, b2, eps)
    rho = np.maximum(Ega / np.abs(ga), Egb / np.maximum(np.abs(gb), 1e-300))
    sel = (np.sign(ga) == np.sign(gb)) & (rho <= 0.1) & (np.abs(gb) > 1e-6)
    step_r = w4r - wr
    tol = 2.5 * rho * np.abs(step_r) + lr * 1e-5 + 4 * 2.0 ** -24 * (np.abs(wr) + lr)
    _say(f"adam phase 2: {sel.sum()} weights checked")
    assert sel.sum() >= 50
    np.testing.assert_array_less(np.abs((w4 - w3) - step_r)[sel], tol[sel])
    # the check discriminates: swapped betas give other steps on these weights
    ws, ms, vs = W0, np.zeros_like(W0), np.zeros_like(W0)
    for t in range(1, 4):
        ws, ms, vs = C.adam_step(ws, ga, ms, vs, t, lr, b2, b1, eps)
    w4s, _, _ = C.adam_step(ws, gb, ms, vs, 4, lr, b2, b1, eps)
    assert np.any(np.abs((w4s - ws) - step_r)[sel] > tol[sel])
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
