"""Pins of the real-space PSF convolution (Eq. 5) of the oracle."""
import math

import numpy as np
import pytest

import oracle as O
from workloads import make_workload


def test_convolution_equals_fft_on_zero_padded_arrays():
    """The direct sum of Eq. (5) without wrap equals a circular FFT
    convolution of the arrays zero-padded by R on every side, for a kernel
    without symmetry (so a flipped or transposed offset shows)."""
    rng = np.random.default_rng(5)
    i0 = rng.standard_normal((13, 17))
    for R in (0, 1, 3, 5):
        K = rng.standard_normal((2 * R + 1, 2 * R + 1))
        got = O.psf_convolution(i0, K)
        ny, nx = i0.shape[0] + 2 * R, i0.shape[1] + 2 * R
        a = np.zeros((ny, nx))
        a[R:R + 13, R:R + 17] = i0
        k = np.zeros((ny, nx))
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                k[dy % ny, dx % nx] = K[dy + R, dx + R]
        ref = np.fft.irfft2(np.fft.rfft2(a) * np.fft.rfft2(k), s=(ny, nx))[R:R + 13, R:R + 17]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_flat_filter_gives_minus_delta():
    """a = 0, A = 1, b = 0: CTF Env = -1 at every frequency, so the PSF is
    minus a unit impulse and Eq. (5) returns -I0 exactly."""
    K = O.psf_kernel(0.0, 1.0, 0.0, 24, 20, 1.5, 4)
    ref = np.zeros((9, 9))
    ref[4, 4] = -1.0
    np.testing.assert_allclose(K, ref, atol=1e-15)
    i0 = np.random.default_rng(1).standard_normal((20, 24))
    np.testing.assert_allclose(O.psf_convolution(i0, K), -i0, atol=1e-14)


def test_envelope_alone_is_a_gaussian_blur():
    """a = 0, A = 1: the PSF is minus the inverse transform of exp(-b s^2/2),
    a Gaussian of variance b / pixel^2 in pixels, normalised to total -1
    (closed form, valid while the Gaussian is far narrower than the box)."""
    pixel = 1.3
    sigma = 2.0                                  # pixels
    b = (sigma * pixel) ** 2
    R = 12
    K = O.psf_kernel(0.0, 1.0, b, 64, 64, pixel, R)
    d = np.arange(-R, R + 1)
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    ref = -np.exp(-r2 / (2 * sigma ** 2)) / (2 * math.pi * sigma ** 2)
    ref[r2 > R * R] = 0.0
    np.testing.assert_allclose(K, ref, atol=1e-10)
    assert abs(K.sum() - ref.sum()) < 1e-10 and abs(ref.sum() + 1.0) < 1e-7


def test_real_space_equals_fourier_away_from_borders():
    """For a projection that vanishes within R of the borders and a PSF
    negligible beyond R, Eq. (5) and the Fourier filter of Eq. (4) give the
    same image; near the borders (a model shifted to the edge) they differ,
    because Eq. (4) wraps."""
    pixel = 2.0
    sph = np.array([[0.0, 0.0, 0.0, 2.0, 1.0], [4.0, -3.0, 1.0, 1.5, 0.5]])
    q = np.array([1.0, 0.0, 0.0, 0.0])
    # Gaussian PSF of sigma 2.5 px: its transform is below e^-30 at the
    # Nyquist frequency (no ringing on the grid) and it is below e^-28 of its
    # peak beyond 19 px
    ctf = (0.0, 1.0, (2.5 * pixel) ** 2)
    i1r = O.calculated_image(sph, q, ctf, 48, 40, pixel, psf_radius=19)
    i1f = O.calculated_image(sph, q, ctf, 48, 40, pixel)
    np.testing.assert_allclose(i1r, i1f, atol=1e-9 * np.abs(i1f).max())
    edge = sph.copy()
    edge[:, 0] += 46.0                          # centred on the right border
    e_r = O.calculated_image(edge, q, ctf, 48, 40, pixel, psf_radius=19)
    e_f = O.calculated_image(edge, q, ctf, 48, 40, pixel)
    assert np.abs(e_r - e_f).max() > 1e-3 * np.abs(e_f).max()


def test_posterior_with_real_space_psf_reduces_to_fourier_for_a_centred_model():
    """The whole posterior with the Eq. (5) images equals the Eq. (4) one
    when the calculated images stay clear of the borders (cropped
    displacements, small model in a large box)."""
    wl = make_workload(1, n_images=3)
    cls = wl.classes[0]
    rng = np.random.default_rng(7)
    sph = np.array([[0.0, 0.0, 0.0, 2.0, 1.0], [5.0, -4.0, 2.0, 2.0, 1.0], [-3.0, 6.0, -1.0, 2.0, 1.0]])
    quats = cls.quats[:4]
    ctf = np.array([[0.0, 1.0, (2.5 * cls.pixel_A) ** 2], [0.0, 1.0, (2.7 * cls.pixel_A) ** 2]])
    imgs = np.array([O.calculated_image(sph, cls.quats[i], ctf[i % 2], 64, 64, cls.pixel_A)
                     + 0.05 * rng.standard_normal((64, 64)) for i in range(3)])
    rr = O.logpost_oracle(imgs, sph, quats, ctf, cls.pixel_A, 2, borders="crop", psf_radius=21)
    rf = O.logpost_oracle(imgs, sph, quats, ctf, cls.pixel_A, 2, borders="crop")
    np.testing.assert_allclose(rr.logp, rf.logp, rtol=0, atol=1e-6)
    l_at = O.loglik_at(imgs[0], sph, quats[rr.best_q[0]], ctf[rr.best_c[0]], cls.pixel_A, rr.best_dx[0],
                       rr.best_dy[0], borders="crop", psf_radius=21)
    assert abs(l_at - rr.best_logl[0]) < 1e-9 * abs(rr.best_logl[0])
