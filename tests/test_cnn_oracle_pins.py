"""Pins of the proposal network's FP64 reference (oracle/cnn_oracle.py)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn_oracle as C

TINY = C.Arch(box=32, c1=2, c2=3, c3=4, c4=4, hidden=5, nq=7)


def _params(arch, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(arch.num_params()) * 0.5


def _targets(B, nq, T, seed):
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.choice(nq, T, replace=False) for _ in range(B)])
    p = rng.random((B, T))
    return idx, p / p.sum(axis=1, keepdims=True)


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(1)
    y = rng.standard_normal((1, 1, 12, 10))
    W = rng.standard_normal((1, 1, 3, 3))
    got = C.conv_s2(y, W, np.zeros(1))[0, 0]
    padded = np.pad(y[0, 0], 1)
    ref = correlate2d(padded, W[0, 0], mode="valid")[::2, ::2]
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_gradient_matches_finite_differences():
    arch = TINY
    flat = _params(arch, 2)
    imgs = np.random.default_rng(3).standard_normal((2, arch.box, arch.box))
    tidx, tp = _targets(2, arch.nq, 3, 4)
    loss, g = C.loss_and_grad(arch, flat, imgs, tidx, tp)
    eps = 1e-6
    num = np.empty_like(flat)
    for k in range(flat.size):
        d = np.zeros_like(flat)
        d[k] = eps
        lp, _ = C.softmax_xent(C.forward(arch, flat + d, imgs)[0], tidx, tp)
        lm, _ = C.softmax_xent(C.forward(arch, flat - d, imgs)[0], tidx, tp)
        num[k] = (lp - lm) / (2 * eps)
    np.testing.assert_allclose(g, num, rtol=1e-5, atol=1e-8)


def test_cross_entropy_properties():
    rng = np.random.default_rng(5)
    nq = 9
    tidx, tp = _targets(3, nq, 4, 6)
    z = rng.standard_normal((3, nq))
    loss, dz = C.softmax_xent(z, tidx, tp)
    np.testing.assert_allclose(dz.sum(axis=1), 0.0, atol=1e-15)
    # with logits equal to the log target (zero elsewhere), the loss is the
    # target's entropy, its minimum (Gibbs)
    zt = np.full((3, nq), -60.0)
    for b in range(3):
        zt[b, tidx[b]] = np.log(tp[b])
    lt, _ = C.softmax_xent(zt, tidx, tp)
    ent = float(np.mean([-(p * np.log(p)).sum() for p in tp]))
    assert abs(lt - ent) < 1e-12
    assert loss > ent


def test_top_k_and_mass():
    rng = np.random.default_rng(7)
    z = rng.standard_normal((4, 50))
    z[0, 10] = z[0, 3]                      # a tie: the lower index wins
    idx, mass = C.top_k(z, 5)
    for b in range(4):
        order = np.argsort(-z[b], kind="stable")[:5]
        assert list(idx[b]) == sorted(order)
    full, m1 = C.top_k(z, 50)
    np.testing.assert_allclose(m1, 1.0, rtol=1e-15)
    assert np.all((mass > 0) & (mass < 1))


def test_network_input_is_the_autocorrelation():
    rng = np.random.default_rng(11)
    img = rng.standard_normal((2, 8, 6))
    got = C.network_input(img)
    for b in range(2):
        u = img[b] - img[b].mean()
        for ry in range(8):
            for rx in range(6):
                ref = sum(u[y, x] * u[(y + ry) % 8, (x + rx) % 6] for y in range(8) for x in range(6))
                if ry == 0 and rx == 0:
                    ref = 0.0
                assert abs(got[b, (ry + 4) % 8, (rx + 3) % 6] - ref) < 1e-12
    # a circular shift of the particle leaves the input unchanged
    shifted = np.roll(img, (3, -2), axis=(1, 2))
    np.testing.assert_allclose(C.network_input(shifted), got, atol=1e-12)
