"""Pins of the oracle's real-space variant with cropping (Section 3, Center
displacement): the calculated image moved by d loses the pixels that leave
the box and nothing wraps in.

Independent routes: circular correlation of zero-padded arrays by a library
FFT (padding by S leaves no wrap inside the window), the wrapped variant at
d = 0 and wherever the calculated image vanishes near the borders, and the
posterior of a shift-free window.
"""
import math

import numpy as np

import oracle as O
from workloads import make_workload


def _padded_route(img, i1, S):
    """X(d) and B(d) from FFT correlations of arrays zero-padded by S."""
    ny, nx = img.shape
    n = nx * ny
    Ic = img - img.mean()
    P = np.zeros((ny + S, nx + S))
    P[:ny, :nx] = i1
    P2 = np.zeros_like(P)
    P2[:ny, :nx] = i1 * i1
    M = np.zeros_like(P)
    M[:ny, :nx] = 1.0
    Ip = np.zeros_like(P)
    Ip[:ny, :nx] = Ic

    def corr(a, b):   # sum_r a(r) b(r + d), circular on the padded box
        return np.fft.irfft2(np.conj(np.fft.rfft2(a)) * np.fft.rfft2(b), s=a.shape)

    full_x, full_c, full_cc = corr(Ip, P), corr(M, P), corr(M, P2)
    d = np.arange(-S, S + 1)
    iy, ix = (d % (ny + S))[:, None], (d % (nx + S))[None, :]
    X = full_x[iy, ix]
    Cc, Ccc = full_c[iy, ix], full_cc[iy, ix]
    return X, Ccc - Cc * Cc / n


def test_cropped_correlation_equals_zero_padded_fft():
    rng = np.random.default_rng(41)
    for ny, nx, S in [(12, 10, 3), (16, 16, 2), (9, 14, 4)]:
        img = rng.standard_normal((ny, nx)) + 3.0
        i1 = rng.standard_normal((ny, nx)) - 0.5
        X, B = O.correlation_cropped(img, i1, S)
        Xr, Br = _padded_route(img, i1, S)
        np.testing.assert_allclose(X, Xr, rtol=0, atol=1e-10)
        np.testing.assert_allclose(B, Br, rtol=0, atol=1e-10)


def test_cropped_equals_wrapped_at_zero_shift_and_for_vanishing_borders():
    rng = np.random.default_rng(42)
    ny, nx, S = 14, 12, 3
    img = rng.standard_normal((3, ny, nx))
    i1 = rng.standard_normal((ny, nx))
    X, B = O.correlation_cropped(img, i1, S)
    Xw = O.correlation_direct(img, i1, S)
    np.testing.assert_allclose(X[:, S, S], Xw[:, S, S], rtol=0, atol=1e-12)
    assert abs(B[S, S] - O.projection_norm(i1)) <= 1e-12
    # a calculated image that is zero within S of every border: nothing is
    # lost and nothing would wrap, so the two variants agree at every d
    inner = np.zeros((ny, nx))
    inner[S:ny - S, S:nx - S] = rng.standard_normal((ny - 2 * S, nx - 2 * S))
    X, B = O.correlation_cropped(img, inner, S)
    np.testing.assert_allclose(X, O.correlation_direct(img, inner, S), rtol=0, atol=1e-12)
    np.testing.assert_allclose(B, O.projection_norm(inner), rtol=0, atol=1e-12)
    # otherwise the variants differ away from d = 0
    X, _ = O.correlation_cropped(img, i1, S)
    assert np.abs(X - Xw).max() > 1e-3


def test_cropped_posterior_reduces_to_wrapped_without_shifts():
    wl = make_workload(1, n_images=3)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    q = cls.quats[:5]
    a = O.logpost_oracle(imgs, wl.models[0], q, cls.ctf[:2], cls.pixel_A, 0, method="fft")
    b = O.logpost_oracle(imgs, wl.models[0], q, cls.ctf[:2], cls.pixel_A, 0, borders="crop")
    np.testing.assert_allclose(a.logp, b.logp, rtol=0, atol=1e-9)
    # with shifts the variants differ, by little for a particle inside the box
    a = O.logpost_oracle(imgs, wl.models[0], q, cls.ctf[:2], cls.pixel_A, 2, method="fft")
    b = O.logpost_oracle(imgs, wl.models[0], q, cls.ctf[:2], cls.pixel_A, 2, borders="crop")
    d = np.abs(a.logp - b.logp)
    assert d.max() > 0 and np.all(np.isfinite(b.logp))
    assert math.isfinite(float(b.best_logl.max()))


def test_loglik_at_crop_reproduces_the_grid_maximum():
    """The single-point cropped log-likelihood equals the cropped grid
    evaluation at its maximum (the loop form of the crop against the
    slicing form of ``correlation_cropped``)."""
    wl = make_workload(1, n_images=2)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    qs = cls.quats[:4]
    r = O.logpost_oracle(imgs, wl.models[0], qs, cls.ctf[:2], cls.pixel_A, 3, borders="crop")
    for i in range(2):
        l = O.loglik_at(imgs[i], wl.models[0], qs[r.best_q[i]], cls.ctf[r.best_c[i]], cls.pixel_A,
                        r.best_dx[i], r.best_dy[i], borders="crop")
        assert abs(l - r.best_logl[i]) <= 1e-10 * abs(l)
