"""Pins of symmetry-restricted orientation sets (Section 4: a particle's
symmetry can reduce the orientational search) on the oracle."""
import math

import numpy as np

import oracle as O
from workloads import expand_symmetry, symmetric_model, symmetry_restricted_euler


def test_matrix_to_quat_inverts_quat_to_matrix():
    rng = np.random.default_rng(31)
    for e in rng.uniform(-7, 7, (200, 3)):
        q = O.euler_to_quat(*e)
        np.testing.assert_allclose(O.quat_to_matrix(q), O.euler_to_matrix(*e), atol=1e-13)
        assert q[0] >= 0 and abs(np.linalg.norm(q) - 1) < 1e-14
    # half turns (trace -1) take the other branches
    for axis in np.eye(3):
        q = np.concatenate([[0.0], axis])
        np.testing.assert_allclose(O.matrix_to_quat(O.quat_to_matrix(q)) * np.sign(q @ q), q, atol=1e-14)
    np.testing.assert_allclose(O.matrix_to_quat(np.eye(3)), [1, 0, 0, 0], atol=1e-15)


def _case(n_fold, symmetric=True):
    rng = np.random.default_rng([160906634, 97])
    if symmetric:
        sph = symmetric_model(rng, 12, n_fold, 26.0, 2.0)
    else:
        sph = symmetric_model(rng, 12 * n_fold, 1, 26.0, 2.0)
    er = symmetry_restricted_euler(rng, 5, n_fold)
    ef = expand_symmetry(er, n_fold)
    qr = np.array([O.euler_to_quat(*e) for e in er])
    qf = np.array([O.euler_to_quat(*e) for e in ef])
    ctf = np.array([[40.0, 0.1, 2.0], [70.0, 0.1, 4.0]])
    nx = ny = 36
    pixel = 2.0
    imgs = np.array([O.render_image(sph, O.euler_to_quat(*rng.uniform(0, 6, 3)), ctf[i % 2], (i - 1, 2 - i), nx, ny,
                                    pixel, 1.0, 0.0, rng.standard_normal((ny, nx)), 0.5) for i in range(3)])
    return sph, qr, qf, ctf, pixel, imgs


def test_cn_model_restricted_set_gives_the_full_posterior():
    """For a C_n-symmetric model the full set is n copies of the restricted
    one (psi + 2 pi k/n leaves the rotated model unchanged), so every
    likelihood appears n times: log P over the restricted set with its own
    prior equals log P over the full set, the restricted orientations scored
    under the full set's prior give exactly ln n less, and the full set's
    per-orientation posteriors repeat with period N_restricted."""
    n = 4
    sph, qr, qf, ctf, pixel, imgs = _case(n)
    rr = O.logpost_oracle(imgs, sph, qr, ctf, pixel, 2, method="fft")
    rf = O.logpost_oracle(imgs, sph, qf, ctf, pixel, 2, method="fft")
    np.testing.assert_allclose(rr.logp, rf.logp, rtol=0, atol=1e-8)
    rs = O.logpost_oracle(imgs, sph, qf, ctf, pixel, 2, method="fft", q_subset=range(len(qr)))
    np.testing.assert_allclose(rs.logp, rf.logp - math.log(n), rtol=0, atol=1e-8)
    nr = len(qr)
    for k in range(1, n):
        np.testing.assert_allclose(rf.logp_orient[:, k * nr:(k + 1) * nr], rf.logp_orient[:, :nr], rtol=0, atol=1e-8)


def test_asymmetric_model_needs_the_full_set():
    """Without the symmetry the copies are different orientations: the
    restricted set's log P is not the full set's."""
    sph, qr, qf, ctf, pixel, imgs = _case(4, symmetric=False)
    rr = O.logpost_oracle(imgs, sph, qr, ctf, pixel, 2, method="fft")
    rf = O.logpost_oracle(imgs, sph, qf, ctf, pixel, 2, method="fft")
    assert np.abs(rr.logp - rf.logp).max() > 1e-3
