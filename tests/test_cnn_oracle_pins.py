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


# ---- Adam (the optimiser of the proposal network) ------------------------

def test_adam_first_step_moves_each_weight_by_lr():
    """From zero moments the bias-corrected moments of step 1 are g and g^2
    exactly, so every weight moves by lr * g / (|g| + eps): lr against the
    gradient's sign wherever |g| >> eps, whatever beta1 and beta2 are."""
    rng = np.random.default_rng(11)
    w = rng.standard_normal(1000)
    g = rng.standard_normal(1000) * 10.0 ** rng.uniform(-4, 2, 1000)
    for b1, b2 in [(0.9, 0.999), (0.5, 0.9), (0.0, 0.0)]:
        w1, m1, v1 = C.adam_step(w, g, np.zeros_like(w), np.zeros_like(w), 1, 0.01, b1, b2, 1e-12)
        np.testing.assert_allclose(w - w1, 0.01 * g / (np.abs(g) + 1e-12), rtol=1e-12)
        assert np.all(np.abs(np.abs(w - w1) - 0.01) <= 0.01 * 1e-12 / np.abs(g) + 1e-15 * (1 + np.abs(w)))
        np.testing.assert_allclose(m1, (1 - b1) * g, rtol=1e-15)
        np.testing.assert_allclose(v1, (1 - b2) * g * g, rtol=1e-15)


def test_adam_constant_gradient_takes_equal_steps():
    """With the same gradient every step the corrected moments stay g and
    g^2 (the corrections 1 - beta^t cancel the zero start exactly), so t
    steps move a weight by t * lr against the sign; a wrong power of beta in
    the correction breaks this from step 2 on."""
    rng = np.random.default_rng(12)
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w, m, v = w0, np.zeros(50), np.zeros(50)
    for t in range(1, 11):
        w, m, v = C.adam_step(w, g, m, v, t, 1e-3, 0.8, 0.95, 1e-12)
        np.testing.assert_allclose(w0 - w, t * 1e-3 * np.sign(g), rtol=1e-9)


def test_adam_moment_decay_and_zero_gradient():
    """After one step with gradient g, zero gradients leave the raw moments
    decaying as beta1^k and beta2^k (which catches swapped betas), and the
    update as the ratio of their corrected values; a zero gradient from zero
    moments moves nothing."""
    g = np.array([2.0, -0.5])
    w, m, v = C.adam_step(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, 0.1, 0.9, 0.99, 0.0)
    for k in range(1, 4):
        w_new, m, v = C.adam_step(w, np.zeros(2), m, v, 1 + k, 0.1, 0.9, 0.99, 0.0)
        np.testing.assert_allclose(m, 0.9 ** k * 0.1 * g, rtol=1e-14)
        np.testing.assert_allclose(v, 0.99 ** k * 0.01 * g * g, rtol=1e-14)
        mh = m / (1 - 0.9 ** (1 + k))
        vh = v / (1 - 0.99 ** (1 + k))
        ratio = (0.9 ** k * 0.1 / (1 - 0.9 ** (1 + k))) / np.sqrt(0.99 ** k * 0.01 / (1 - 0.99 ** (1 + k)))
        np.testing.assert_allclose(w - w_new, 0.1 * np.sign(g) * ratio, rtol=1e-12)
        np.testing.assert_allclose(mh / np.sqrt(vh), np.sign(g) * ratio, rtol=1e-12)
        w = w_new
    w0 = np.array([0.3, -1.2])
    w1, _, _ = C.adam_step(w0, np.zeros(2), np.zeros(2), np.zeros(2), 1, 0.1, 0.9, 0.999, 1e-8)
    assert np.array_equal(w1, w0)
