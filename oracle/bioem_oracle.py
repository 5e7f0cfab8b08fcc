"""FP64 reference of the BioEM posterior (test infrastructure, see package doc).

Conventions (each one a reading of the paper, listed with its reason in the
design notes of the repository):

* Images are arrays ``I[k][j]`` with row index k along y and column index j
  along x; pixel (j, k) has centre ``x_j = (j - Nx/2) * pixel``,
  ``y_k = (k - Ny/2) * pixel``.
* Fourier transforms follow numpy: forward ``exp(-2 pi i (l k/Ny + m j/Nx))``
  without normalisation, inverse with ``1/Npix``; half spectra are laid out
  ``[Ny][Nx/2+1]`` and the signed row frequency is ``l`` for ``l <= Ny/2`` and
  ``l - Ny`` above.  The paper's Eqs. (1)-(2) print 1-based sums without the
  ``1/N`` inside the exponent; this is the standard 0-based DFT they denote.
* The displacement d enters as ``I_cal(r) = N I1(r + d) - mu`` (Section 2,
  calculated image), so the correlation at d is ``sum_r I_o(r) I1(r + d)``
  with indices taken modulo the box: the Fourier variant of Section 3
  (Center displacement) wraps around the borders, and the oracle computes the
  same circular function directly.
* Shifts cover the square window ``|dx|, |dy| <= S`` in 1-pixel steps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
from scipy.special import erf


# ---------------------------------------------------------------------------
# Model rotation and projection (Section 2, Eq. ideal; Section 3, Model rotation)
# ---------------------------------------------------------------------------

def quat_to_matrix(q: Sequence[float]) -> np.ndarray:
    """Rotation matrix of the unit quaternion q = (w, x, y, z) (Hamilton, active).

    The paper parametrises orientations by quaternions (Section 3, Model
    rotation); r' = R(q) r rotates the model about its origin.  q and -q give
    the same matrix.
    """
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def euler_to_matrix(phi: float, theta: float, psi: float) -> np.ndarray:
    """Rotation matrix of Euler angles (radians), the other orientation
    representation of Section 3 (Model rotation): rotate about z by phi,
    then about the new y by theta, then about the new z by psi (intrinsic
    z-y-z), i.e. R = Rz(phi) Ry(theta) Rz(psi) acting on column vectors.
    The paper does not fix the convention; z-y-z is the usual one in EM.
    """
    def rz(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])

    def ry(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])

    return rz(phi) @ ry(theta) @ rz(psi)


def matrix_to_quat(Rm: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z), w >= 0, of a rotation matrix (the inverse
    of ``quat_to_matrix``): from the matrix's largest diagonal combination,
    which keeps the square root away from zero."""
    m = np.asarray(Rm, dtype=np.float64)
    t = np.trace(m)
    cand = [t, m[0, 0], m[1, 1], m[2, 2]]
    k = int(np.argmax(cand))
    if k == 0:
        r = math.sqrt(1.0 + t) * 2.0
        q = [0.25 * r, (m[2, 1] - m[1, 2]) / r, (m[0, 2] - m[2, 0]) / r, (m[1, 0] - m[0, 1]) / r]
    elif k == 1:
        r = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2.0
        q = [(m[2, 1] - m[1, 2]) / r, 0.25 * r, (m[0, 1] + m[1, 0]) / r, (m[0, 2] + m[2, 0]) / r]
    elif k == 2:
        r = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2.0
        q = [(m[0, 2] - m[2, 0]) / r, (m[0, 1] + m[1, 0]) / r, 0.25 * r, (m[1, 2] + m[2, 1]) / r]
    else:
        r = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2.0
        q = [(m[1, 0] - m[0, 1]) / r, (m[0, 2] + m[2, 0]) / r, (m[1, 2] + m[2, 1]) / r, 0.25 * r]
    q = np.array(q)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def euler_to_quat(phi: float, theta: float, psi: float) -> np.ndarray:
    """Unit quaternion of z-y-z Euler angles (``euler_to_matrix``)."""
    return matrix_to_quat(euler_to_matrix(phi, theta, psi))


def _pixel_integrals(centres: np.ndarray, pos: np.ndarray, sigma: np.ndarray,
                     pixel: float) -> np.ndarray:
    """[n_spheres][n_pixels] integral of a unit 1-D Gaussian over each pixel."""
    s = np.sqrt(2.0) * sigma[:, None]
    u = centres[None, :] - pos[:, None]
    return 0.5 * (erf((u + 0.5 * pixel) / s) - erf((u - 0.5 * pixel) / s))


def project_model(spheres: np.ndarray, q: Sequence[float], nx: int, ny: int,
                  pixel: float) -> np.ndarray:
    """Ideal projection I0[k][j] of a Gaussian-sphere model, Eq. (ideal).

    The density is a sum of normalised 3-D Gaussians of weight w_a, centre
    r_a and width sigma_a.  Rotating by q and integrating along z over the
    whole line and over the pixel box in x and y leaves, for each sphere, the
    product of two 1-D pixel integrals, so
    I0[k][j] = sum_a w_a Ey[a][k] Ex[a][j].
    """
    sp = np.asarray(spheres, dtype=np.float64)
    r = sp[:, :3] @ quat_to_matrix(q).T
    xc = (np.arange(nx) - nx // 2) * pixel
    yc = (np.arange(ny) - ny // 2) * pixel
    ex = _pixel_integrals(xc, r[:, 0], sp[:, 3], pixel)
    ey = _pixel_integrals(yc, r[:, 1], sp[:, 3], pixel)
    return (ey * sp[:, 4][:, None]).T @ ex


# ---------------------------------------------------------------------------
# CTF and envelope, Fourier filtering (Section 2, Eqs. 3-4)
# ---------------------------------------------------------------------------

def signed_freq(n: int) -> np.ndarray:
    """Signed integer frequency of each index of an n-point DFT axis."""
    k = np.arange(n)
    return np.where(k <= n // 2, k, k - n)


def ctf_envelope_table(a: float, amp: float, b: float, nx: int, ny: int,
                       pixel: float) -> np.ndarray:
    """CTF(s|a,A) Env(s|b) on the half spectrum [Ny][Nx/2+1] (Section 2).

    CTF(s) = -A cos(a s^2/2) - sqrt(1 - A^2) sin(a s^2/2) and
    Env(s) = exp(-b s^2/2), where s = |s| and s = 2 pi (m/(Nx dx), l/(Ny dy))
    for signed integer frequencies (m, l).
    """
    m = np.arange(nx // 2 + 1)
    l = signed_freq(ny)
    s2 = (2.0 * np.pi) ** 2 * ((m[None, :] / (nx * pixel)) ** 2
                               + (l[:, None] / (ny * pixel)) ** 2)
    ph = 0.5 * a * s2
    ctf = -amp * np.cos(ph) - math.sqrt(1.0 - amp * amp) * np.sin(ph)
    return ctf * np.exp(-0.5 * b * s2)


def filtered_projection(i0: np.ndarray, table: np.ndarray) -> np.ndarray:
    """I1 = F^-1[F(I0) CTF Env], Eq. (4); real because the filter is radial."""
    ny, nx = i0.shape
    return np.fft.irfft2(np.fft.rfft2(i0) * table, s=(ny, nx))


def psf_kernel(a: float, amp: float, b: float, nx: int, ny: int, pixel: float, R: int) -> np.ndarray:
    """The real-space PSF of Eq. (3), truncated to radius R pixels:
    K[dy + R][dx + R] = PSF(dx, dy) where dx^2 + dy^2 <= R^2, else 0.

    PSF = F^-1[CTF Env] on the box grid (the inverse of Eq. 2, with its
    1/N_pix), the radially symmetric image that Section 3 (Imaging effects)
    precalculates; the real-space form is meant for a PSF that is negligible
    away from the origin, hence the truncation.  Needs R < min(nx, ny) / 2."""
    if not 0 <= R < min(nx, ny) // 2:
        raise ValueError(f"PSF radius {R} outside [0, min(nx, ny)/2)")
    psf = np.fft.irfft2(ctf_envelope_table(a, amp, b, nx, ny, pixel), s=(ny, nx))
    d = np.arange(-R, R + 1)
    K = psf[(d % ny)[:, None], (d % nx)[None, :]]
    K[(d[:, None] ** 2 + d[None, :] ** 2) > R * R] = 0.0
    return K


def psf_convolution(i0: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Eq. (5) on the box without wrap: I1(r) = sum over r' in the box of
    I0(r') PSF(r - r'), with PSF(delta) = K[delta + R] (zero outside the
    kernel); pixels of I0 outside the box count as zero.  Written as the sum
    over the kernel's offsets delta of K(delta) I0(r - delta)."""
    i0 = np.asarray(i0, dtype=np.float64)
    ny, nx = i0.shape
    R = K.shape[0] // 2
    out = np.zeros((ny, nx))
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            w = K[dy + R, dx + R]
            if w == 0.0:
                continue
            # out[y, x] += w i0[y - dy, x - dx] for 0 <= y - dy < ny, 0 <= x - dx < nx
            y0, y1 = max(0, dy), min(ny, ny + dy)
            x0, x1 = max(0, dx), min(nx, nx + dx)
            if y0 < y1 and x0 < x1:
                out[y0:y1, x0:x1] += w * i0[y0 - dy:y1 - dy, x0 - dx:x1 - dx]
    return out


def calculated_image(spheres: np.ndarray, q, ctf, nx: int, ny: int, pixel: float,
                     psf_radius: Optional[int] = None) -> np.ndarray:
    """I1 of Eq. (4) (Fourier filter, the default) or of Eq. (5) (real-space
    convolution with the PSF truncated to ``psf_radius`` pixels)."""
    a, amp, b = ctf
    i0 = project_model(spheres, q, nx, ny, pixel)
    if psf_radius is None:
        return filtered_projection(i0, ctf_envelope_table(a, amp, b, nx, ny, pixel))
    return psf_convolution(i0, psf_kernel(a, amp, b, nx, ny, pixel, psf_radius))


# ---------------------------------------------------------------------------
# Precomputed sums and the cross-correlation (Section 3; Center displacement)
# ---------------------------------------------------------------------------

def image_moments(img: np.ndarray):
    """(C_o, C_oo, A) of an observed image, in FP64 from pixels.

    C_o = sum I, C_oo = sum I^2 (the per-image constants the paper
    precomputes) and A = sum (I - C_o/n)^2 = C_oo - C_o^2/n, taken in two
    passes so that no cancellation occurs.
    """
    x = np.asarray(img, dtype=np.float64)
    c_o = math.fsum(x.ravel())
    c_oo = math.fsum((x * x).ravel())
    mean = c_o / x.size
    d = x - mean
    return c_o, c_oo, math.fsum((d * d).ravel())


def projection_norm(i1: np.ndarray) -> float:
    """B = sum (I1 - mean)^2 of a calculated image (shift-invariant, circular)."""
    x = np.asarray(i1, dtype=np.float64)
    d = x - math.fsum(x.ravel()) / x.size
    return math.fsum((d * d).ravel())


def correlation_direct(img: np.ndarray, i1: np.ndarray, S: int) -> np.ndarray:
    """X[dy+S][dx+S] = sum_r (I_o(r) - mean) I1((r + d) mod box), directly.

    This is the real-space cross-correlation of Section 3 with the wrap of
    the Fourier variant; centring the image removes the offset so X is the
    covariance-type sum the marginal likelihood needs.  Batched over a
    leading image axis when ``img`` is 3-D.
    """
    imgs = np.asarray(img, dtype=np.float64)
    single = imgs.ndim == 2
    if single:
        imgs = imgs[None]
    ni, ny, nx = imgs.shape
    ic = (imgs - imgs.reshape(ni, -1).mean(axis=1)[:, None, None]).reshape(ni, -1)
    p = np.asarray(i1, dtype=np.float64)
    w = 2 * S + 1
    out = np.empty((ni, w, w))
    for dy in range(-S, S + 1):
        stack = np.stack([np.roll(p, (-dy, -dx), axis=(0, 1)).ravel()
                          for dx in range(-S, S + 1)], axis=1)
        out[:, dy + S, :] = ic @ stack
    return out[0] if single else out


def correlation_fft(img: np.ndarray, i1: np.ndarray, S: int) -> np.ndarray:
    """The same window via Eq. (fourier): F^-1[conj(F(I_o)) F(I1)] at d.

    Faster reference for large boxes; equal to ``correlation_direct`` up to
    FP64 rounding (pinned by a test).  Batched like ``correlation_direct``.
    """
    imgs = np.asarray(img, dtype=np.float64)
    single = imgs.ndim == 2
    if single:
        imgs = imgs[None]
    ni, ny, nx = imgs.shape
    ic = imgs - imgs.reshape(ni, -1).mean(axis=1)[:, None, None]
    full = np.fft.irfft2(np.conj(np.fft.rfft2(ic)) * np.fft.rfft2(np.asarray(i1, np.float64)),
                         s=(ny, nx))
    d = np.arange(-S, S + 1)
    out = full[:, (d % ny)[:, None], (d % nx)[None, :]]
    return out[0] if single else out


def correlation_cropped(img: np.ndarray, i1: np.ndarray, S: int):
    """Real-space variant of Section 3 (Center displacement) with cropping.

    The calculated image moved by d is I1(r + d) where r + d lies in the box
    and 0 elsewhere: pixels moved out of the box are lost and none wrap in
    (the paper contrasts this cropping with the wrap of the Fourier variant).
    Returns (X, B): X[i][dy+S][dx+S] = sum_r (I_o(r) - mean) I1_d(r), the
    centred cross-correlation, and B[dy+S][dx+S] = sum_r (I1_d(r) - mean)^2
    over the whole box, which now depends on d (two-pass sums).
    """
    imgs = np.asarray(img, dtype=np.float64)
    single = imgs.ndim == 2
    if single:
        imgs = imgs[None]
    ni, ny, nx = imgs.shape
    ic = (imgs - imgs.reshape(ni, -1).mean(axis=1)[:, None, None]).reshape(ni, -1)
    p = np.asarray(i1, dtype=np.float64)
    w = 2 * S + 1
    X = np.empty((ni, w, w))
    B = np.empty((w, w))
    for dy in range(-S, S + 1):
        for dx in range(-S, S + 1):
            moved = np.zeros_like(p)
            moved[max(0, -dy):ny - max(0, dy), max(0, -dx):nx - max(0, dx)] = \
                p[max(0, dy):ny + min(0, dy), max(0, dx):nx + min(0, dx)]
            X[:, dy + S, dx + S] = ic @ moved.ravel()
            B[dy + S, dx + S] = projection_norm(moved)
    return (X[0] if single else X), B


# ---------------------------------------------------------------------------
# Marginal likelihood (Section 2, Eq. likeli; Section 3, analytic integration)
# ---------------------------------------------------------------------------

_RHO2_MAX = 1.0 - 2.0 ** -52


def log_likelihood(X, A: float, B: float, n: int):
    """ln of Eq. (likeli) integrated over offset mu, scale N and noise lambda.

    With I_cal = N I1' - mu, flat priors on mu and N over the real line and
    the scale-invariant prior 1/lambda, the three integrals are Gaussian,
    Gaussian and Gamma in turn:
      int dmu   -> sqrt(2 pi lambda^2 / n)
      int dN    -> sqrt(2 pi lambda^2 / B)
      int dl/l  -> (1/2) Gamma(n/2 - 1) (Q/2)^(1 - n/2),  Q = A - X^2/B,
    so L = (1/2) Gamma(n/2-1) (pi Q)^(1-n/2) / sqrt(n B).  Here A is the
    centred sum of squares of the image, B that of the calculated image and X
    their centred cross-correlation.  Writing Q = A (1 - X^2/(A B)) keeps the
    large terms separate from the small correlation term.  1 - rho^2 is
    clamped at 2^-52 (an exact noise-free fit would diverge).
    """
    X = np.asarray(X, dtype=np.float64)
    rho2 = np.minimum(X * X / (A * B), _RHO2_MAX)
    h = 0.5 * n
    const = (math.lgamma(h - 1.0) - math.log(2.0) - 0.5 * math.log(n)
             + (1.0 - h) * math.log(math.pi * A) - 0.5 * math.log(B))
    return const + (1.0 - h) * np.log1p(-rho2)


def loglik_at(image: np.ndarray, spheres: np.ndarray, q, ctf, pixel: float, dx: int, dy: int,
              borders: str = "wrap", psf_radius: Optional[int] = None) -> float:
    """l(q, c, d) of one image at one grid point (Eq. likeli integrated, as
    ``log_likelihood``), with the correlation at d summed directly:
    X = sum_r (I_o(r) - mean) I1_d(r), where I1_d(r) = I1((r + d) mod box)
    for the Fourier variant and I1(r + d) inside the box, 0 outside, with
    ``borders="crop"`` (then B is taken of I1_d).  -inf where nothing moved
    in (B = 0).  ``psf_radius`` takes I1 from Eq. (5) (``calculated_image``)."""
    img = np.asarray(image, dtype=np.float64)
    ny, nx = img.shape
    i1 = calculated_image(spheres, q, ctf, nx, ny, pixel, psf_radius)
    A = image_moments(img)[2]
    dx, dy = int(dx), int(dy)
    if borders == "wrap":
        moved = np.roll(i1, (-dy, -dx), axis=(0, 1))
    elif borders == "crop":
        moved = np.zeros_like(i1)
        for k in range(ny):
            for j in range(nx):
                if 0 <= k + dy < ny and 0 <= j + dx < nx:
                    moved[k, j] = i1[k + dy, j + dx]
    else:
        raise ValueError(f"borders must be 'wrap' or 'crop', not {borders!r}")
    B = projection_norm(moved)
    if not B > 0.0:
        return -math.inf
    X = math.fsum(((img - img.mean()) * moved).ravel())
    return float(log_likelihood(X, A, B, nx * ny))


def logsumexp_exact(values) -> float:
    """ln sum exp(v) as M + ln fsum(exp(v - M)) in FP64."""
    v = np.asarray(values, dtype=np.float64).ravel()
    m = float(np.max(v))
    return m + math.log(math.fsum(np.exp(v - m)))


def ensemble_logpost(logp: np.ndarray, w: Sequence[float]):
    """Log posterior of a model ensemble, Eq. (pb2) of Section 2.

    ``logp[m][i]`` is the log posterior of image i under model m (as returned
    by ``logpost_oracle``), ``w[m]`` the ensemble's relative weights (w >= 0,
    summing to 1).  Per image the ensemble's posterior is the weighted sum
    over models, ln sum_m w_m exp(logp[m][i]); the images are independent, so
    the ensemble's log posterior over the whole set is the sum of those over
    images (the log of the product in Eq. pb2, up to the same constant).
    Models with w_m = 0 take no part; a NaN among the others gives NaN; an
    infinite maximum is returned as it is.  Returns (per_image [ni], total).
    """
    L = np.asarray(logp, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    nm, ni = L.shape
    per = np.empty(ni)
    for i in range(ni):
        terms = [(float(w[m]), float(L[m, i])) for m in range(nm) if w[m] > 0.0]
        vals = [v for _, v in terms]
        if any(math.isnan(v) for v in vals):
            per[i] = math.nan
            continue
        M = max(vals)
        if math.isinf(M):
            per[i] = M
            continue
        per[i] = M + math.log(math.fsum(wm * math.exp(v - M) for wm, v in terms))
    if ni == 0:
        return per, 0.0
    if np.all(np.isfinite(per)):
        return per, math.fsum(per)
    # IEEE rules for the infinities: both signs (or a NaN) give NaN
    if np.any(np.isnan(per)) or (np.any(per == math.inf) and np.any(per == -math.inf)):
        return per, math.nan
    return per, math.inf if np.any(per == math.inf) else -math.inf


# ---------------------------------------------------------------------------
# Posterior over the grid (Eq. Pmom; Listing 1's loop nest)
# ---------------------------------------------------------------------------

@dataclass
class OracleResult:
    logp: np.ndarray          # [ni] log posterior per image (relative, see log_prior)
    best_logl: np.ndarray     # [ni] maximal log-likelihood
    best_q: np.ndarray        # [ni]
    best_c: np.ndarray        # [ni]
    best_dx: np.ndarray       # [ni]
    best_dy: np.ndarray       # [ni]
    logp_orient: np.ndarray   # [ni][nq] log posterior restricted to orientation q
    log_prior: float          # -ln(Nq Nc Nd): uniform normalised grid prior


def logpost_oracle(images: np.ndarray, spheres: np.ndarray, quats: np.ndarray,
                   ctfs: np.ndarray, pixel: float, S: int, method: str = "direct",
                   q_subset: Optional[Sequence[int]] = None, borders: str = "wrap",
                   psf_radius: Optional[int] = None) -> OracleResult:
    """log P_{m,omega} for every image over the orientation x CTF x shift grid.

    P is the integral of Eq. (Pmom) with mu, N and lambda integrated
    analytically (``log_likelihood``) and the remaining parameters summed over
    their grids with uniform normalised priors:
      log P = ln sum_{q,c,d} exp(l(q,c,d)) - ln(Nq Nc Nd).
    The loop nest follows Listing 1: rotation and projection outermost, then
    the CTF filter, then all images at every displacement.  Also returns the
    maximising grid point (ties go to the lowest (q, c, dy, dx)) and the
    posterior restricted to each orientation (LSE over c and d).
    ``q_subset`` evaluates only those orientations (the prior keeps Nq).
    ``borders="crop"`` takes the real-space variant with cropping
    (``correlation_cropped``: B depends on d) instead of the wrap.
    ``psf_radius`` builds each calculated image by the real-space PSF
    convolution of Eq. (5) (``psf_kernel``, ``psf_convolution``) instead of
    the Fourier filter of Eq. (4).
    """
    imgs = np.asarray(images, dtype=np.float64)
    ni, ny, nx = imgs.shape
    n = nx * ny
    nq, nc = len(quats), len(ctfs)
    nd = (2 * S + 1) ** 2
    corr = {"direct": correlation_direct, "fft": correlation_fft}[method]
    if borders not in ("wrap", "crop"):
        raise ValueError(f"borders must be 'wrap' or 'crop', not {borders!r}")
    A = np.array([image_moments(im)[2] for im in imgs])
    tables = [ctf_envelope_table(a, amp, b, nx, ny, pixel) for a, amp, b in ctfs]
    qs = range(nq) if q_subset is None else q_subset
    orient = np.full((ni, nq), -np.inf)
    best = np.full(ni, -np.inf)
    bq = np.zeros(ni, np.int64)
    bc = np.zeros(ni, np.int64)
    bdx = np.zeros(ni, np.int64)
    bdy = np.zeros(ni, np.int64)
    log_prior = -math.log(nq) - math.log(nc) - math.log(nd)
    for q in qs:
        i0 = project_model(spheres, quats[q], nx, ny, pixel)
        per_c = np.empty((ni, nc, 2 * S + 1, 2 * S + 1))
        for c in range(nc):
            if psf_radius is None:
                i1 = filtered_projection(i0, tables[c])
            else:
                i1 = psf_convolution(i0, psf_kernel(*ctfs[c], nx, ny, pixel, psf_radius))
            if borders == "crop":
                X, Bd = correlation_cropped(imgs, i1, S)
                for i in range(ni):
                    for dy in range(2 * S + 1):
                        for dx in range(2 * S + 1):
                            # nothing moved in (B = 0): that displacement is left out
                            per_c[i, c, dy, dx] = (log_likelihood(X[i, dy, dx], A[i], Bd[dy, dx], n)
                                                   if Bd[dy, dx] > 0.0 else -np.inf)
                continue
            B = projection_norm(i1)
            X = corr(imgs, i1, S)
            for i in range(ni):
                per_c[i, c] = log_likelihood(X[i], A[i], B, n)
        for i in range(ni):
            orient[i, q] = logsumexp_exact(per_c[i]) + log_prior
            flat = per_c[i].ravel()
            k = int(np.argmax(flat))      # first maximum = lowest (c, dy, dx)
            if flat[k] > best[i]:         # strict: an earlier q keeps a tie
                best[i] = flat[k]
                c, rem = divmod(k, (2 * S + 1) ** 2)
                dyi, dxi = divmod(rem, 2 * S + 1)
                bq[i], bc[i], bdy[i], bdx[i] = q, c, dyi - S, dxi - S
    sel = np.array(list(qs))
    logp = np.array([logsumexp_exact(orient[i, sel]) for i in range(ni)])
    return OracleResult(logp=logp, best_logl=best, best_q=bq, best_c=bc, best_dx=bdx,
                        best_dy=bdy, logp_orient=orient, log_prior=log_prior)


# ---------------------------------------------------------------------------
# Synthetic map (Section 3, Extra features): a calculated image for given theta
# ---------------------------------------------------------------------------

def render_image(spheres: np.ndarray, q, ctf, shift, nx: int, ny: int, pixel: float,
                 norm: float = 1.0, offset: float = 0.0, noise: Optional[np.ndarray] = None,
                 snr: Optional[float] = None) -> np.ndarray:
    """I_cal(r) = N I1(r + d) - mu, plus optional Gaussian noise at a given SNR.

    SNR is var(clean)/sigma_n^2 over the whole box with i.i.d. pixel noise,
    the noise model of Eq. (likeli).  Returns FP64; callers store FP32.
    """
    a, amp, b = ctf
    i1 = filtered_projection(project_model(spheres, q, nx, ny, pixel),
                             ctf_envelope_table(a, amp, b, nx, ny, pixel))
    dx, dy = int(shift[0]), int(shift[1])
    clean = np.roll(i1, (-dy, -dx), axis=(0, 1))
    out = norm * clean - offset
    if noise is not None:
        sigma = math.sqrt(float(np.var(clean)) / snr)
        out = out + sigma * np.asarray(noise, dtype=np.float64)
    return out


def render_images(cls, models, i0: int = 0, i1: Optional[int] = None) -> np.ndarray:
    """FP32 images [i1-i0][ny][nx] of a workload size class, rendered in FP64."""
    i1 = cls.n_images if i1 is None else i1
    noise = cls.noise(i0, i1)
    out = np.empty((i1 - i0, cls.ny, cls.nx), np.float32)
    for j, i in enumerate(range(i0, i1)):
        out[j] = render_image(models[cls.img_model[i]], cls.img_quat[i], cls.img_ctf[i],
                              cls.img_shift[i], cls.nx, cls.ny, cls.pixel_A,
                              cls.img_norm[i, 0], cls.img_norm[i, 1], noise[j], cls.snr)
    return out
