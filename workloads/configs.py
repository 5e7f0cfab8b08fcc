"""Workload recipes: shapes, sizes and value distributions of the paper's runs.

The paper's data sets (Frh hydrogenase micrographs at 224x224 px, 1.32 A/px,
and a ~82k-atom model; Section 4, Performance) are not available, so each
workload is synthetic with the same image size, pixel size and
orientation x PSF x shift grid structure.  Model: Gaussian spheres with unit
integrated density placed uniformly in a ball.  Orientation grids: uniform
random unit quaternions (Shoemake's method) made canonical with w >= 0.  CTF
grids: defocus evenly spaced over [0.5, 3.5] um, amplitude contrast 0.1,
B-factors as listed per workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BASE_SEED = 160906634

# Physical constants (CODATA 2018) for the relativistic electron wavelength.
_H = 6.62607015e-34        # Planck constant, J s
_M0 = 9.1093837015e-31     # electron rest mass, kg
_E = 1.602176634e-19       # elementary charge, C
_C = 299792458.0           # speed of light, m/s


def electron_wavelength_A(voltage_kV: float) -> float:
    """Relativistic de Broglie wavelength of an electron accelerated by V (in A)."""
    v = voltage_kV * 1e3
    p = math.sqrt(2.0 * _M0 * _E * v * (1.0 + _E * v / (2.0 * _M0 * _C * _C)))
    return _H / p * 1e10


def ctf_abA_from_physical(defocus_A: float, amp_contrast: float, bfactor_A2: float,
                          voltage_kV: float = 300.0):
    """Map (defocus, amplitude contrast, B-factor) to the paper's (a, A, b).

    The paper writes CTF(s|a,A) = -A cos(a s^2/2) - sqrt(1-A^2) sin(a s^2/2)
    and Env(s|b) = exp(-b s^2/2) with s = 2 pi k (Section 2, CTF and Env).
    Matching the phase to pi*lambda*defocus*k^2 gives a = lambda*defocus/(2 pi);
    matching exp(-b s^2/2) to the amplitude envelope exp(-B k^2/4) gives
    b = B/(8 pi^2).
    """
    lam = electron_wavelength_A(voltage_kV)
    a = lam * defocus_A / (2.0 * math.pi)
    b = bfactor_A2 / (8.0 * math.pi ** 2)
    return a, amp_contrast, b


def shoemake_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform random unit quaternions (w, x, y, z), canonical w >= 0."""
    u = rng.random((n, 3))
    r1 = np.sqrt(1.0 - u[:, 0])
    r2 = np.sqrt(u[:, 0])
    t1 = 2.0 * np.pi * u[:, 1]
    t2 = 2.0 * np.pi * u[:, 2]
    q = np.stack([r2 * np.cos(t2), r1 * np.sin(t1), r1 * np.cos(t1), r2 * np.sin(t2)], axis=1)
    q[q[:, 0] < 0] *= -1.0
    return q


def symmetric_model(rng: np.random.Generator, n_per_copy: int, n_fold: int, radius: float,
                    sigma: float) -> np.ndarray:
    """A C_n-symmetric sphere model [n_fold * n_per_copy][5]: spheres drawn
    uniformly in a ball, then copied by the rotations about the z axis by
    2 pi k / n_fold (the model's symmetry axis), unit weights."""
    base = _ball_spheres(rng, n_per_copy, radius, sigma)
    out = []
    for k in range(n_fold):
        a = 2.0 * np.pi * k / n_fold
        c, s_ = np.cos(a), np.sin(a)
        cp = base.copy()
        cp[:, 0] = c * base[:, 0] - s_ * base[:, 1]
        cp[:, 1] = s_ * base[:, 0] + c * base[:, 1]
        out.append(cp)
    return np.concatenate(out)


def symmetry_restricted_euler(rng: np.random.Generator, n: int, n_fold: int) -> np.ndarray:
    """n orientations as z-y-z Euler angles (phi, theta, psi) restricted for a
    C_n model: psi, the first turn about the model's own z axis, in
    [0, 2 pi / n_fold); phi uniform in [0, 2 pi), cos(theta) uniform."""
    u = rng.random((n, 3))
    return np.stack([2.0 * np.pi * u[:, 0], np.arccos(1.0 - 2.0 * u[:, 1]), 2.0 * np.pi * u[:, 2] / n_fold], axis=1)


def expand_symmetry(euler: np.ndarray, n_fold: int) -> np.ndarray:
    """The full set of a restricted one: each orientation with psi + 2 pi k /
    n_fold for k = 0..n_fold-1, copies of the restricted set in k order."""
    e = np.asarray(euler, np.float64)
    return np.concatenate([e + np.array([0.0, 0.0, 2.0 * np.pi * k / n_fold]) for k in range(n_fold)])


def _ball_spheres(rng: np.random.Generator, n: int, radius: float, sigma: float) -> np.ndarray:
    """[n][5] spheres (x, y, z, sigma, weight) uniform in a ball, unit weight."""
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    out = np.empty((n, 5))
    out[:, :3] = d * r[:, None]
    out[:, 3] = sigma
    out[:, 4] = 1.0
    return out


def _ctf_grid(defoci_um, bfactors, amp=0.1, voltage_kV=300.0) -> np.ndarray:
    rows = []
    for bf in bfactors:
        for df in defoci_um:
            rows.append(ctf_abA_from_physical(df * 1e4, amp, bf, voltage_kV))
    return np.array(rows, dtype=np.float64)


@dataclass
class SizeClass:
    """One image size with its own grids and images (one model's view)."""
    nx: int
    ny: int
    pixel_A: float
    max_shift: int
    quats: np.ndarray            # [nq][4] orientation grid
    ctf: np.ndarray              # [nc][3] (a, A, b) grid
    # per-image true parameters (the images themselves are rendered elsewhere)
    img_model: np.ndarray        # [ni] index of the generating model
    img_quat: np.ndarray         # [ni][4]
    img_shift: np.ndarray        # [ni][2] int (dx, dy)
    img_ctf: np.ndarray          # [ni][3]
    img_norm: np.ndarray         # [ni][2] (N, mu)
    snr: float
    noise_seed: tuple            # per-image noise streams: seed + (i,)

    @property
    def n_images(self) -> int:
        return int(self.img_quat.shape[0])

    def noise(self, i0: int = 0, i1: Optional[int] = None) -> np.ndarray:
        """Standard-normal float32 noise fields [i1-i0][ny][nx], one stream per image."""
        i1 = self.n_images if i1 is None else i1
        out = np.empty((i1 - i0, self.ny, self.nx), np.float32)
        for j, i in enumerate(range(i0, i1)):
            g = np.random.default_rng(list(self.noise_seed) + [i])
            out[j] = g.standard_normal((self.ny, self.nx), dtype=np.float32)
        return out

    def subset(self, n: int) -> "SizeClass":
        """The first n images of this class (same grids, same per-image draws)."""
        return SizeClass(nx=self.nx, ny=self.ny, pixel_A=self.pixel_A, max_shift=self.max_shift,
                         quats=self.quats, ctf=self.ctf, img_model=self.img_model[:n],
                         img_quat=self.img_quat[:n], img_shift=self.img_shift[:n],
                         img_ctf=self.img_ctf[:n], img_norm=self.img_norm[:n], snr=self.snr,
                         noise_seed=self.noise_seed)


@dataclass
class Workload:
    name: str
    models: List[np.ndarray]                 # each [ns][5]
    classes: List[SizeClass] = field(default_factory=list)
    # N and mu draws for invariance tests (never used by the configs themselves)
    test_norm: Optional[np.ndarray] = None


def _class(rng, seed, nx, pixel, S, nq, ctf_grid, ni, model_of_img, snr, img_ctf_fn):
    quats = shoemake_quaternions(rng, nq)
    img_quat = shoemake_quaternions(rng, ni)
    img_shift = rng.integers(-S, S + 1, size=(ni, 2)).astype(np.int32)
    img_ctf = img_ctf_fn(rng, ni)
    return SizeClass(nx=nx, ny=nx, pixel_A=pixel, max_shift=S, quats=quats, ctf=ctf_grid,
                     img_model=model_of_img, img_quat=img_quat, img_shift=img_shift,
                     img_ctf=img_ctf, img_norm=np.tile([1.0, 0.0], (ni, 1)), snr=snr,
                     noise_seed=tuple(seed))


def _img_ctf_uniform(b_lo, b_hi, amp=0.1):
    def f(rng, ni):
        df = rng.uniform(0.5, 3.5, ni) * 1e4
        bf = rng.uniform(b_lo, b_hi, ni) if b_hi > b_lo else np.full(ni, b_lo)
        return np.array([ctf_abA_from_physical(d, amp, b) for d, b in zip(df, bf)])
    return f


BOX_A = 224 * 1.32   # 295.68 A box shared by the multi-size workload


def make_workload(k: int, n_images: Optional[int] = None) -> Workload:
    """Build workload k (1..5).  ``n_images`` keeps the first images of each class
    (the draws do not depend on it, so a subset is a prefix of the full set).

    1: 200 spheres (sigma 2 A, ball radius 40 A), 64^2 at 2.2 A/px, 50 images,
       100 orientations x 4 CTFs (B=0), shifts +-5, SNR 0.1.
    2: 1500 spheres (sigma 1.5 A, radius 80 A), 224^2 at 1.32 A/px, 1000
       images, 4608 orientations x 8 CTFs (4 defoci x B in {25,75}),
       shifts +-20, image B ~ U[0,100], SNR 0.05.
    3: same inputs as 1 (precision form).
    4: 10,000 images in four size classes 96/128/180/224 px (box 295.7 A),
       two models (1000 spheres radius 70 A; 2500 spheres radius 85 A),
       (nq, nc) = (1152,4), (2304,8), (3456,12), (4608,16), shifts 8/11/16/20.
    5: 128^2 at 2.31 A/px, model of 1000 spheres (radius 70 A), 36,864
       orientations x 4 CTFs (B=50), shifts +-11, SNR 0.1.
    """
    sk = 1 if k == 3 else k
    rng = np.random.default_rng([BASE_SEED, sk])
    if k in (1, 3):
        model = _ball_spheres(rng, 200, 40.0, 2.0)
        ni = 50
        cls = _class(rng, [BASE_SEED, sk, 0, 1], 64, 2.2, 5, 100,
                     _ctf_grid(np.linspace(0.5, 3.5, 4), [0.0]), ni,
                     np.zeros(ni, np.int32), 0.1, _img_ctf_uniform(0.0, 0.0))
        wl = Workload(name=f"config{k}", models=[model], classes=[cls])
    elif k == 2:
        model = _ball_spheres(rng, 1500, 80.0, 1.5)
        ni = 1000
        cls = _class(rng, [BASE_SEED, sk, 0, 1], 224, 1.32, 20, 4608,
                     _ctf_grid(np.linspace(0.5, 3.5, 4), [25.0, 75.0]), ni,
                     np.zeros(ni, np.int32), 0.05, _img_ctf_uniform(0.0, 100.0))
        wl = Workload(name="config2", models=[model], classes=[cls])
    elif k == 4:
        models = [_ball_spheres(rng, 1000, 70.0, 1.5), _ball_spheres(rng, 2500, 85.0, 1.5)]
        specs = [(96, 8, 1152, _ctf_grid(np.linspace(0.5, 3.5, 4), [50.0])),
                 (128, 11, 2304, _ctf_grid(np.linspace(0.5, 3.5, 4), [25.0, 75.0])),
                 (180, 16, 3456, _ctf_grid(np.linspace(0.5, 3.5, 6), [25.0, 75.0])),
                 (224, 20, 4608, _ctf_grid(np.linspace(0.5, 3.5, 8), [25.0, 75.0]))]
        per = 2500
        classes = []
        for ci, (nx, S, nq, grid) in enumerate(specs):
            owner = (np.arange(per) % 2).astype(np.int32)
            classes.append(_class(rng, [BASE_SEED, sk, ci, 1], nx, BOX_A / nx, S, nq, grid, per,
                                  owner, 0.05, _img_ctf_uniform(0.0, 100.0)))
        wl = Workload(name="config4", models=models, classes=classes)
    elif k == 5:
        model = _ball_spheres(rng, 1000, 70.0, 1.5)
        ni = 1000
        cls = _class(rng, [BASE_SEED, sk, 0, 1], 128, BOX_A / 128, 11, 36864,
                     _ctf_grid(np.linspace(0.5, 3.5, 4), [50.0]), ni,
                     np.zeros(ni, np.int32), 0.1, _img_ctf_uniform(50.0, 50.0))
        wl = Workload(name="config5", models=[model], classes=[cls])
    else:
        raise ValueError(f"unknown workload {k}")
    wl.test_norm = np.stack([rng.uniform(0.5, 2.0, 64), rng.uniform(-1.0, 1.0, 64)], axis=1)
    if n_images is not None:
        wl.classes = [c.subset(n_images) for c in wl.classes]
    return wl


def proposal_training_images(n: int, stream: int = 2, nq_grid: Optional[int] = None) -> SizeClass:
    """Per-image parameters of n training images for the learned proposal
    (the 128^2 workload's model, grids and image distribution, drawn from the
    separate stream [160906634, 5, stream]; the held-out images are the
    workload's own).  ``nq_grid`` keeps the first orientations of the grid."""
    base = make_workload(5, n_images=1).classes[0]
    rng = np.random.default_rng([BASE_SEED, 5, stream])
    img_quat = shoemake_quaternions(rng, n)
    S = base.max_shift
    img_shift = rng.integers(-S, S + 1, size=(n, 2)).astype(np.int32)
    img_ctf = _img_ctf_uniform(50.0, 50.0)(rng, n)
    quats = base.quats if nq_grid is None else base.quats[:nq_grid]
    return SizeClass(nx=base.nx, ny=base.ny, pixel_A=base.pixel_A, max_shift=S, quats=quats,
                     ctf=base.ctf, img_model=np.zeros(n, np.int32), img_quat=img_quat,
                     img_shift=img_shift, img_ctf=img_ctf, img_norm=np.tile([1.0, 0.0], (n, 1)),
                     snr=base.snr, noise_seed=(BASE_SEED, 5, stream, 1))


CONFIGS = {1: "64^2 small", 2: "224^2 paper-shaped", 3: "64^2 split-bf16",
           4: "mixed sizes, two models", 5: "128^2 learned proposal"}
