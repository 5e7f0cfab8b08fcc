"""Pins of the oracle's ensemble posterior, Eq. (pb2) of Section 2.

Each test takes a route other than the oracle's own: 50-digit arithmetic,
the product over images evaluated as printed (no logarithms), special weights
whose answer is known in closed form, bounds of a convex combination, and the
model discrimination the paper uses the posterior for (the generating model
wins).
"""
import math

import mpmath
import numpy as np
import pytest

import oracle as O


def test_ensemble_against_50_digit_arithmetic():
    # magnitudes of a 224^2 posterior (about -2.3e5) underflow a naive sum of
    # exponentials; spreads of a few hundred nat between models
    rng = np.random.default_rng(31)
    w = np.array([0.2, 0.5, 0.3])
    for offset, spread in [(0.0, 1.0), (-2.3e5, 300.0), (4e4, 1e-3)]:
        L = offset + spread * rng.standard_normal((3, 40))
        per, total = O.ensemble_logpost(L, w)
        mpmath.mp.dps = 50
        ref = [mpmath.log(mpmath.fsum(mpmath.mpf(float(w[m])) * mpmath.exp(mpmath.mpf(float(L[m, i])))
                                      for m in range(3))) for i in range(L.shape[1])]
        for i in range(L.shape[1]):
            assert abs(per[i] - float(ref[i])) <= 1e-12 * max(1.0, abs(float(ref[i])))
        tref = float(mpmath.fsum(ref))
        assert abs(total - tref) <= 1e-12 * max(1.0, abs(tref))


def test_ensemble_total_is_the_printed_product():
    # Eq. (pb2) as printed: the product over images of the weighted sums of
    # posteriors, in plain floating point on values where nothing underflows
    rng = np.random.default_rng(32)
    L = rng.uniform(-2.0, 2.0, (2, 12))
    w = np.array([0.7, 0.3])
    prod = 1.0
    for i in range(12):
        prod *= w[0] * math.exp(L[0, i]) + w[1] * math.exp(L[1, i])
    per, total = O.ensemble_logpost(L, w)
    assert abs(total - math.log(prod)) <= 1e-13 * 12
    for i in range(12):
        assert abs(per[i] - math.log(w[0] * math.exp(L[0, i]) + w[1] * math.exp(L[1, i]))) <= 1e-14


def test_ensemble_special_weights_and_bounds():
    rng = np.random.default_rng(33)
    L = -1e5 + 50.0 * rng.standard_normal((4, 30))
    # one model with all the weight: its own posterior, and its log evidence
    for m in range(4):
        w = np.zeros(4)
        w[m] = 1.0
        per, total = O.ensemble_logpost(L, w)
        np.testing.assert_array_equal(per, L[m])
        assert total == math.fsum(L[m])
    # identical models: the weights sum to one, so nothing changes
    same = np.repeat(L[:1], 4, axis=0)
    per, _ = O.ensemble_logpost(same, [0.1, 0.2, 0.3, 0.4])
    np.testing.assert_allclose(per, L[0], rtol=0, atol=1e-9)
    # a convex combination lies between the weighted extremes
    w = np.array([0.1, 0.2, 0.3, 0.4])
    per, _ = O.ensemble_logpost(L, w)
    lo = np.max(np.log(w)[:, None] + L, axis=0)
    hi = np.max(L, axis=0)
    assert np.all(per >= lo - 1e-9) and np.all(per <= hi + 1e-9)


def test_ensemble_degenerate_entries():
    nan, inf = math.nan, math.inf
    L = np.array([[nan, -3.0, -inf, 1.0],
                  [-2.0, nan, -inf, inf]])
    # model 0 carries no weight: its NaN takes no part
    per, total = O.ensemble_logpost(L, [0.0, 1.0])
    assert per[0] == -2.0 and math.isnan(per[1]) and per[2] == -inf and per[3] == inf
    assert math.isnan(total)
    per, total = O.ensemble_logpost(L[:, 2:3], [0.5, 0.5])
    assert per[0] == -inf and total == -inf
    per, total = O.ensemble_logpost(np.zeros((2, 0)), [0.5, 0.5])
    assert per.shape == (0,) and total == 0.0


@pytest.mark.parametrize("seed", [0])
def test_ensemble_discriminates_the_generating_model(seed):
    # Two random sphere models; images drawn from model 0 at SNR 1.  Under
    # one-hot weights the total is each model's log evidence: model 0 must win
    # overall and on most images, and the 50/50 ensemble lies in between.
    rng = np.random.default_rng([160906634, 99, seed])
    nx = ny = 32
    pix = 3.0

    def ball(ns, radius):
        pts = []
        while len(pts) < ns:
            p = rng.uniform(-radius, radius, 3)
            if p @ p <= radius * radius:
                pts.append(p)
        return np.column_stack([np.array(pts), np.full(ns, 2.0), np.ones(ns)])

    models = [ball(60, 30.0), ball(60, 30.0)]
    q = rng.standard_normal((12, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    ctfs = np.array([[0.0, 0.1, 10.0], [400.0, 0.1, 10.0]])
    S = 2
    imgs = np.array([O.render_image(models[0], q[i], ctfs[i % 2], (i % 3 - 1, 1 - i % 3), nx, ny, pix,
                                    1.0, 0.0, rng.standard_normal((ny, nx)), 1.0) for i in range(8)])
    L = np.array([O.logpost_oracle(imgs, m, q, ctfs, pix, S, method="fft").logp for m in models])
    _, t0 = O.ensemble_logpost(L, [1.0, 0.0])
    _, t1 = O.ensemble_logpost(L, [0.0, 1.0])
    _, th = O.ensemble_logpost(L, [0.5, 0.5])
    assert t0 > t1
    assert np.mean(L[0] > L[1]) >= 0.75
    assert t1 < th < t0
