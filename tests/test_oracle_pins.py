"""Pins of the CPU oracle against facts the paper and mathematics fix.

None of these retypes the oracle's formulas: each compares it with an
independent route (numerical integration of Eq. likeli, an exact symmetry,
a library FFT, a textbook value, high-precision arithmetic, brute force).
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

import oracle as O
from workloads import make_workload, ctf_abA_from_physical, electron_wavelength_A


# ---------------------------------------------------------------------------
# P1: closed-form marginal likelihood == brute-force triple integral
# ---------------------------------------------------------------------------

def _brute_force_log_evidence(img, i1_shifted):
    """ln int dmu int dN int dlambda/lambda of Eq. (likeli), numerically.

    (mu, N) are integrated on a whitened grid around the least-squares point
    found by a library solver (only to place the grid), lambda on a log grid.
    """
    y = np.asarray(img, np.float64).ravel()
    x = np.asarray(i1_shifted, np.float64).ravel()
    n = y.size
    M = np.stack([x, -np.ones(n)], axis=1)          # residual = y - (N x - mu)
    sol, res, *_ = np.linalg.lstsq(M, y, rcond=None)
    cov = np.linalg.inv(M.T @ M)
    L = np.linalg.cholesky(cov)
    t = np.linspace(-11.0, 11.0, 67)
    T1, T2 = np.meshgrid(t, t, indexing="ij")
    wt = np.full(t.size, t[1] - t[0])
    wt[0] *= 0.5
    wt[-1] *= 0.5
    W2 = np.log(np.outer(wt, wt))
    q_min = float(np.sum((y - M @ sol) ** 2))
    u0 = 0.5 * math.log(q_min / n)
    us = np.linspace(u0 - 7.0, u0 + 7.0, 421)
    logs = np.empty(us.size)
    for k, u in enumerate(us):
        lam = math.exp(u)
        N = sol[0] + lam * (L[0, 0] * T1)
        mu = sol[1] + lam * (L[1, 0] * T1 + L[1, 1] * T2)
        r = y[None, None, :] - (N[..., None] * x[None, None, :] - mu[..., None])
        ss = np.sum(r * r, axis=-1)
        logf = -ss / (2 * lam * lam) - 0.5 * n * math.log(2 * math.pi * lam * lam)
        logf = logf + W2 + 2 * u + math.log(abs(np.linalg.det(L)))
        m = logf.max()
        logs[k] = m + math.log(np.exp(logf - m).sum())
    du = us[1] - us[0]
    m = logs.max()
    wu = np.full(us.size, du)
    wu[0] *= 0.5
    wu[-1] *= 0.5
    return m + math.log(np.sum(wu * np.exp(logs - m)))


@pytest.mark.parametrize("shape,seed", [((3, 4), 0), ((4, 4), 1), ((2, 5), 2)])
def test_p1_closed_form_matches_triple_integral(shape, seed):
    rng = np.random.default_rng(seed)
    i1 = rng.standard_normal(shape) * 2.0 + 0.3
    img = 0.7 * np.roll(i1, (-1, 2), axis=(0, 1)) + 0.5 * rng.standard_normal(shape) - 0.2
    S = 1
    X = O.correlation_direct(img, i1, S)
    A = O.image_moments(img)[2]
    B = O.projection_norm(i1)
    n = img.size
    ell = O.log_likelihood(X, A, B, n)
    shifts = [(dy, dx) for dy in range(-S, S + 1) for dx in range(-S, S + 1)]
    for dy, dx in (shifts if seed == 0 else shifts[::4]):
        shifted = np.array([[i1[(k + dy) % shape[0], (j + dx) % shape[1]]
                             for j in range(shape[1])] for k in range(shape[0])])
        bf = _brute_force_log_evidence(img, shifted)
        assert abs(ell[dy + S, dx + S] - bf) < 2e-6, (dy, dx, ell[dy + S, dx + S], bf)


# ---------------------------------------------------------------------------
# P2: exact affine invariances of the marginal likelihood
# ---------------------------------------------------------------------------

def _ell_map(img, i1, S):
    A = O.image_moments(img)[2]
    B = O.projection_norm(i1)
    return O.log_likelihood(O.correlation_direct(img, i1, S), A, B, img.size)


def test_p2_affine_invariances():
    rng = np.random.default_rng(7)
    i1 = rng.standard_normal((8, 6))
    img = np.roll(i1, (1, -2), axis=(0, 1)) + rng.standard_normal((8, 6))
    n = img.size
    base = _ell_map(img, i1, 2)
    for alpha, beta in [(2.5, 1.0), (-0.3, -4.0)]:
        got = _ell_map(alpha * img + beta, i1, 2)
        np.testing.assert_allclose(got, base + (2 - n) * math.log(abs(alpha)), atol=1e-9)
    for k, beta in [(3.0, 0.5), (-0.25, 2.0)]:
        got = _ell_map(img, k * i1 + beta, 2)
        np.testing.assert_allclose(got, base - math.log(abs(k)), atol=1e-9)


# ---------------------------------------------------------------------------
# P3: Plancherel on the half spectrum; P4 direct == FFT correlation
# ---------------------------------------------------------------------------

def test_p3_plancherel_half_spectrum():
    rng = np.random.default_rng(3)
    for ny, nx in [(8, 6), (64, 64), (10, 14)]:
        img = rng.standard_normal((ny, nx)) + 1.5
        F = np.fft.rfft2(img)
        w = np.full(nx // 2 + 1, 2.0)
        w[0] = 1.0
        w[-1] = 1.0 if nx % 2 == 0 else 2.0
        power = (np.abs(F) ** 2) * w[None, :]
        c_o, c_oo, A = O.image_moments(img)
        assert abs(power.sum() / img.size - c_oo) < 1e-9 * c_oo
        assert abs((power.sum() - power[0, 0]) / img.size - A) < 1e-9 * A
        assert abs(F[0, 0].real - c_o) < 1e-9 * abs(c_o)


def test_p4_direct_equals_fft_correlation():
    rng = np.random.default_rng(4)
    imgs = rng.standard_normal((3, 16, 20))
    i1 = rng.standard_normal((16, 20))
    a = O.correlation_direct(imgs, i1, 5)
    b = O.correlation_fft(imgs, i1, 5)
    np.testing.assert_allclose(a, b, atol=1e-11)
    # a brute-force element with explicit modular indexing
    dy, dx = 3, -4
    ic = imgs[1] - imgs[1].mean()
    ref = sum(ic[k, j] * i1[(k + dy) % 16, (j + dx) % 20] for k in range(16) for j in range(20))
    assert abs(a[1, dy + 5, dx + 5] - ref) < 1e-11


# ---------------------------------------------------------------------------
# P5: shift equivariance
# ---------------------------------------------------------------------------

def test_p5_shift_equivariance():
    rng = np.random.default_rng(5)
    i1 = rng.standard_normal((12, 12))
    img = rng.standard_normal((12, 12))
    S = 5
    base = O.correlation_direct(img, i1, S)
    # I_o rolled by delta -> X_delta(d) = X(d + delta)
    delta = (2, -1)   # (dy, dx)
    rolled = np.roll(img, delta, axis=(0, 1))
    got = O.correlation_direct(rolled, i1, S)
    for dy in range(-S, S + 1):
        for dx in range(-S, S + 1):
            ty, tx = dy + delta[0], dx + delta[1]
            if abs(ty) <= S and abs(tx) <= S:
                assert abs(got[dy + S, dx + S] - base[ty + S, tx + S]) < 1e-10
    # with the window covering the whole circle the posterior is unchanged
    full = 6  # 2*6+1 = 13 > 12: every residue class covered (some twice)
    A = O.image_moments(img)[2]
    B = O.projection_norm(i1)
    n = img.size
    d = np.arange(-5, 7)   # exactly one representative per residue mod 12
    m1 = O.correlation_fft(img, i1, full)[(d + full)[:, None], (d + full)[None, :]]
    m2 = O.correlation_fft(rolled, i1, full)[(d + full)[:, None], (d + full)[None, :]]
    l1 = O.logsumexp_exact(O.log_likelihood(m1, A, B, n))
    l2 = O.logsumexp_exact(O.log_likelihood(m2, A, B, n))
    assert abs(l1 - l2) < 1e-9


# ---------------------------------------------------------------------------
# P6: recovery of orientation, CTF and shift for near-noise-free images
# ---------------------------------------------------------------------------

def test_p6_recovery_of_grid_parameters():
    wl = make_workload(1, n_images=1)
    cls = wl.classes[0]
    model = wl.models[0]
    rng = np.random.default_rng(11)
    cases = [(17, 2, (3, -2)), (63, 0, (-4, 1)), (5, 3, (0, 5))]
    imgs = []
    for q, c, d in cases:
        noise = rng.standard_normal((cls.ny, cls.nx))
        imgs.append(O.render_image(model, cls.quats[q], cls.ctf[c], d, cls.nx, cls.ny,
                                   cls.pixel_A, 1.3, 0.4, noise, snr=10.0))
    imgs = np.array(imgs)
    qsub = sorted(set([q for q, _, _ in cases] + list(range(0, 100, 9))))
    r = O.logpost_oracle(imgs, model, cls.quats, cls.ctf, cls.pixel_A, cls.max_shift,
                         method="fft", q_subset=qsub)
    for i, (q, c, d) in enumerate(cases):
        assert (r.best_q[i], r.best_c[i], r.best_dx[i], r.best_dy[i]) == (q, c, d[0], d[1])


# ---------------------------------------------------------------------------
# P7: log-sum-exp against 50-digit arithmetic; P10: LSE bounds
# ---------------------------------------------------------------------------

def test_p7_logsumexp_high_precision():
    rng = np.random.default_rng(8)
    for scale, offset in [(1.0, 0.0), (300.0, -2.3e5), (1e-3, 5e4)]:
        v = rng.standard_normal(500) * scale + offset
        mpmath.mp.dps = 50
        ref = mpmath.log(mpmath.fsum(mpmath.exp(mpmath.mpf(float(x))) for x in v))
        assert abs(O.logsumexp_exact(v) - float(ref)) <= 1e-12 * max(1.0, abs(float(ref)))


def test_p10_posterior_bounds():
    wl = make_workload(1, n_images=3)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    qsub = list(range(0, 100, 10))
    r = O.logpost_oracle(imgs, wl.models[0], cls.quats, cls.ctf, cls.pixel_A, cls.max_shift,
                         method="fft", q_subset=qsub)
    npts = len(qsub) * len(cls.ctf) * (2 * cls.max_shift + 1) ** 2
    for i in range(3):
        lo = r.best_logl[i] + r.log_prior
        assert lo <= r.logp[i] <= lo + math.log(npts)
        # per-orientation posteriors combine to the total
        assert abs(O.logsumexp_exact(r.logp_orient[i, qsub]) - r.logp[i]) < 1e-9


def _checkerboard_case(S, nq=5, nc=3):
    """One narrow sphere at the origin (every orientation projects alike),
    nc identical CTF rows, and a checkerboard image (plus an offset): the
    centred checkerboard correlates with any calculated image as
    X(d) = (-1)^(dx+dy) X(0), so l is one value over the whole grid."""
    nx = ny = 16
    pixel = 2.0
    sph = np.array([[0.0, 0.0, 0.0, 0.6, 1.0]])
    rng = np.random.default_rng(14)
    quats = rng.standard_normal((nq, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    ctf = np.array([[40.0, 0.1, 0.0]] * nc)
    j, k = np.meshgrid(np.arange(nx), np.arange(ny))
    cb = np.where((j + k) % 2 == 0, 1.0, -1.0)
    img = 2.5 + 0.7 * cb
    i1 = O.filtered_projection(O.project_model(sph, quats[0], nx, ny, pixel),
                               O.ctf_envelope_table(*ctf[0], nx, ny, pixel))
    n = nx * ny
    A = 0.49 * n                                   # sum of (0.7 cb)^2, exactly
    B = O.projection_norm(i1)
    X0 = math.fsum((0.7 * cb * i1).ravel())
    return img, sph, quats, ctf, pixel, O.log_likelihood(X0, A, B, n), X0 * X0 / (A * B)


@pytest.mark.parametrize("S", [0, 2, 5])
def test_p14_prior_normaliser_on_a_constant_likelihood(S):
    """With l constant over the grid, ln sum exp(l) - ln(Nq Nc Nd) = l exactly
    whatever the grid sizes: a wrong normaliser (2S+1 shifts instead of
    (2S+1)^2, or a missing -ln Nq or -ln Nc) is off by its logarithm."""
    img, sph, quats, ctf, pixel, l0, rho2 = _checkerboard_case(S)
    assert rho2 > 1e-3                      # a non-trivial correlation term
    r = O.logpost_oracle(img[None], sph, quats, ctf, pixel, S, method="direct")
    assert abs(r.logp[0] - l0) <= 1e-10 * abs(l0)
    assert abs(r.best_logl[0] - l0) <= 1e-10 * abs(l0)
    nd = (2 * S + 1) ** 2
    assert abs(r.log_prior + math.log(len(quats) * len(ctf) * nd)) < 1e-12
    for q in range(len(quats)):             # each orientation holds 1/Nq of the mass
        assert abs(r.logp_orient[0, q] - (l0 - math.log(len(quats)))) <= 1e-10 * abs(l0)


def test_loglik_at_reproduces_the_grid_maximum():
    """The single-point log-likelihood (used to check reported best points)
    equals the grid evaluation at its maximum and lies below it elsewhere."""
    wl = make_workload(1, n_images=2)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    qs = cls.quats[:6]
    r = O.logpost_oracle(imgs, wl.models[0], qs, cls.ctf, cls.pixel_A, cls.max_shift, method="direct")
    for i in range(2):
        l = O.loglik_at(imgs[i], wl.models[0], qs[r.best_q[i]], cls.ctf[r.best_c[i]], cls.pixel_A,
                        r.best_dx[i], r.best_dy[i])
        assert abs(l - r.best_logl[i]) <= 1e-10 * abs(l)
        other = O.loglik_at(imgs[i], wl.models[0], qs[(r.best_q[i] + 1) % 6], cls.ctf[0], cls.pixel_A, 1, -1)
        assert other <= r.best_logl[i]


# ---------------------------------------------------------------------------
# P8: projection (Eq. ideal)
# ---------------------------------------------------------------------------

def test_p8_quaternion_convention():
    th = 0.7
    q = (math.cos(th / 2), 0.0, 0.0, math.sin(th / 2))
    np.testing.assert_allclose(O.quat_to_matrix(q) @ [1, 0, 0],
                               [math.cos(th), math.sin(th), 0], atol=1e-15)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(4), rng.standard_normal(4)
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    ab = [w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
          w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2]
    np.testing.assert_allclose(O.quat_to_matrix(ab), O.quat_to_matrix(a) @ O.quat_to_matrix(b),
                               atol=1e-12)
    np.testing.assert_allclose(O.quat_to_matrix(-a), O.quat_to_matrix(a), atol=1e-15)


def test_p8_projection_mass_symmetry_and_rotation():
    wl = make_workload(1, n_images=1)
    model = wl.models[0]
    cls = wl.classes[0]
    q = cls.quats[3]
    i0 = O.project_model(model, q, 64, 64, 2.2)
    assert abs(i0.sum() - model[:, 4].sum()) < 1e-9 * model[:, 4].sum()
    np.testing.assert_allclose(O.project_model(model, -q, 64, 64, 2.2), i0, atol=1e-12)
    # 90 degrees about z maps (x, y) -> (-y, x): I0'[k][j] = I0[N - j][k]
    ident = O.project_model(model, (1, 0, 0, 0), 64, 64, 2.2)
    rz = O.project_model(model, (math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)), 64, 64, 2.2)
    j = np.arange(1, 64)
    np.testing.assert_allclose(rz[:, 1:], ident[(64 - j)[None, :], np.arange(64)[:, None]],
                               atol=1e-12)
    # identity orientation: z coordinate does not matter, x is the column axis
    one = np.array([[4.4, -2.2, 9.0, 1.0, 1.0]])
    img = O.project_model(one, (1, 0, 0, 0), 16, 16, 2.2)
    k, jj = np.unravel_index(np.argmax(img), img.shape)
    assert (jj - 8, k - 8) == (2, -1)


def test_p8_single_sphere_pixel_integral():
    sph = np.array([[0.7, -1.1, 3.0, 1.3, 2.0]])
    img = O.project_model(sph, (1, 0, 0, 0), 10, 8, 1.0)
    g = lambda y, x: 2.0 * math.exp(-((x - 0.7) ** 2 + (y + 1.1) ** 2) / (2 * 1.3 ** 2)) / (
        2 * math.pi * 1.3 ** 2)
    for (k, j) in [(4, 5), (3, 5), (5, 2), (0, 0)]:
        xc, yc = j - 5, k - 4
        ref, _ = integrate.dblquad(g, xc - 0.5, xc + 0.5, yc - 0.5, yc + 0.5, epsabs=1e-13)
        assert abs(img[k, j] - ref) < 1e-10


# ---------------------------------------------------------------------------
# P9: CTF and envelope
# ---------------------------------------------------------------------------

def test_p9_ctf_special_values():
    a, A, b = ctf_abA_from_physical(2.0e4, 0.1, 0.0)
    T = O.ctf_envelope_table(a, A, b, 64, 64, 2.0)
    assert abs(T[0, 0] + 0.1) < 1e-15
    assert np.all(np.abs(T) <= 1.0 + 1e-15)
    # electron wavelength at 300 kV (textbook 0.01969 A)
    assert abs(electron_wavelength_A(300.0) - 0.019687) < 2e-6


def test_p9_first_zero_textbook():
    # with no amplitude contrast CTF = -sin(pi lambda df k^2): first zero at
    # k = 1/sqrt(lambda df)
    df = 1.0e4
    a, A, b = ctf_abA_from_physical(df, 0.0, 0.0)
    nx = 512
    pix = 1.0
    T = O.ctf_envelope_table(a, A, b, nx, 2, pix)[0]
    k = np.arange(nx // 2 + 1) / (nx * pix)
    sign_change = np.nonzero(np.diff(np.sign(T[1:])))[0][0] + 1
    k0 = 1.0 / math.sqrt(electron_wavelength_A(300.0) * df)
    assert k[sign_change] <= k0 <= k[sign_change + 1]
    assert T[1] < 0   # phase contrast: negative at low frequency


def test_p9_envelope_is_gaussian_blur():
    # a = 0, A = 1: the filter is -exp(-b s^2/2), i.e. minus a Gaussian blur of
    # variance b (A^2) in real space, Eq. (5) with that PSF
    b = 6.0   # A^2
    pix = 0.8
    n = 64
    T = O.ctf_envelope_table(0.0, 1.0, b, n, n, pix)
    delta = np.zeros((n, n))
    delta[0, 0] = 1.0
    psf = O.filtered_projection(delta, T)
    sig2 = b / pix ** 2
    r = O.signed_freq(n)
    g = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2 * sig2)) / (2 * math.pi * sig2)
    np.testing.assert_allclose(psf, -g, atol=1e-9)


# ---------------------------------------------------------------------------
# Euler angles (the second orientation representation): convention pinned to
# a library rotation and to its special cases
# ---------------------------------------------------------------------------

def test_euler_zyz_matches_library_and_special_cases():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(51)
    for phi, theta, psi in rng.uniform(-math.pi, math.pi, (20, 3)):
        R = O.euler_to_matrix(phi, theta, psi)
        np.testing.assert_allclose(R, Rotation.from_euler("ZYZ", [phi, theta, psi]).as_matrix(), atol=1e-14)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) < 1e-14
        # no tilt: one rotation about z by phi + psi
        np.testing.assert_allclose(O.euler_to_matrix(phi, 0.0, psi), O.euler_to_matrix(phi + psi, 0.0, 0.0),
                                   atol=1e-14)
    # a quarter turn about y maps z to x
    np.testing.assert_allclose(O.euler_to_matrix(0.0, math.pi / 2, 0.0) @ [0, 0, 1], [1, 0, 0], atol=1e-15)
