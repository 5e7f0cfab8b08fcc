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


# ---- the element-wise error bounds of the network parity tests -----------

def _bound_case():
    import cnn_bounds as CB
    arch = C.Arch(box=32, c1=4, c2=8, c3=8, c4=8, hidden=8, nq=50)
    rng = np.random.default_rng(21)
    parts = []
    for name, shape in arch.shapes():   # He-style scale, as the network is trained from
        scale = np.sqrt(2.0 / np.prod(shape[1:])) if name[0] in "WF" else 0.1
        parts.append(rng.standard_normal(int(np.prod(shape))) * scale)
    flat = np.concatenate(parts).astype(np.float32).astype(np.float64)
    imgs = (rng.standard_normal((5, 32, 32)) + np.linspace(0, 3, 32)[None, None, :]).astype(np.float32)
    tidx, tp = _targets(5, arch.nq, 4, 22)
    return CB, arch, flat, imgs, tidx, tp


def test_bf16_rounding_emulation():
    import cnn_bounds as CB
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 1e-20, 3.0e38])
    r = CB.bf16_round(x)
    # ties to even: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6 (= 1 + 4 2^-8)
    np.testing.assert_array_equal(r[:4], [1.0, 1.0, 1.0 + 2.0 ** -6, -2.5])
    rng = np.random.default_rng(3)
    v = rng.standard_normal(10000) * 10.0 ** rng.uniform(-10, 10, 10000)
    rv = CB.bf16_round(v)
    assert np.all(np.abs(rv - v.astype(np.float32)) <= 2.0 ** -8 * np.abs(v) * (1 + 1e-6))
    assert np.all((rv.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_network_bounds_hold_for_emulated_bf16_products():
    """The element-wise bounds of logits and gradients contain the deviation
    of a recomputation whose products take bf16-rounded operands; with
    operands rounded to 5 bits instead, some elements leave them."""
    CB, arch, flat, imgs, tidx, tp = _bound_case()
    loss, g, z, Eloss, Eg, Ez = CB.grad_bound(arch, flat, imgs, tidx, tp)
    lr, gr = C.loss_and_grad(arch, flat, imgs, tidx, tp)
    np.testing.assert_allclose(g, gr, rtol=1e-12, atol=1e-15)   # same reference
    le, ge, ze = CB.emulate_loss_and_grad(arch, flat, imgs, tidx, tp, bits=8)
    assert np.all(np.abs(ze - z) <= Ez)
    assert np.all(np.abs(ge - g) <= Eg)
    assert abs(le - loss) <= Eloss
    # the bounds have teeth: operands rounded to 6 bits (errors 4x those of
    # bf16) already leave them somewhere, and 5 bits in many places
    _, g6, z6 = CB.emulate_loss_and_grad(arch, flat, imgs, tidx, tp, bits=6)
    assert np.any(np.abs(z6 - z) > Ez) or np.any(np.abs(g6 - g) > Eg)
    _, g5, z5 = CB.emulate_loss_and_grad(arch, flat, imgs, tidx, tp, bits=5)
    assert np.sum(np.abs(z5 - z) > Ez) + np.sum(np.abs(g5 - g) > Eg) > 20
    assert np.median(Ez / np.maximum(np.abs(z), 1e-30)) < 0.2
