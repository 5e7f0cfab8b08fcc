"""Orientations as Euler angles (z-y-z): bioem_project_euler against the
oracle's posterior for the same rotations, and against bioem_project with
the equivalent quaternions.

The oracle's convention (Rz(phi) Ry(theta) Rz(psi)) is pinned to a library
rotation on the CPU; here the library's quaternions for the same angles come
from that library, so the GPU's angle-to-quaternion step is checked end to
end through the posterior.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1609_06634_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def test_euler_projection_matches_oracle_and_quaternions(P, ctx):
    from scipy.spatial.transform import Rotation
    wl = make_workload(1, n_images=6)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    rng = np.random.default_rng(61)
    euler = rng.uniform(-np.pi, np.pi, (37, 3))
    euler[:, 1] = np.abs(euler[:, 1])
    euler[0] = (0.0, 0.0, 0.0)
    xyzw = Rotation.from_euler("ZYZ", euler).as_quat()
    quats = np.column_stack([xyzw[:, 3], xyzw[:, :3]])
    _say("euler: 6 images x 37 orientations x 4 CTF sets, S=5")
    r = O.logpost_oracle(imgs, wl.models[0], quats, cls.ctf, cls.pixel_A, cls.max_shift, method="fft")
    pe = P.project_euler(ctx, wl.models[0], euler, cls.nx, cls.ny, cls.pixel_A)
    pq = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    im = P.prepare_images(ctx, imgs)
    oe = P.logpost(ctx, pe, im, cls.ctf, cls.max_shift, prec="f32", orient=True)
    oq = P.logpost(ctx, pq, im, cls.ctf, cls.max_shift, prec="f32", orient=True)
    d = np.abs(oe["logp"] - r.logp)
    _say(f"  max |dlogP| vs oracle {d.max():.3e}, vs quaternion input {np.abs(oe['logp'] - oq['logp']).max():.3e}")
    assert d.max() <= 0.01
    assert np.abs(oe["orient"] - r.logp_orient).max() <= 0.01
    assert np.abs(oe["logp"] - oq["logp"]).max() <= 1e-6
    for h in (pe, pq, im):
        h.free()


def test_euler_arguments(P, ctx):
    wl = make_workload(1, n_images=1)
    cls = wl.classes[0]
    with pytest.raises(P.BioemError):
        P.project_euler(ctx, wl.models[0], np.array([[0.0, np.nan, 0.0]]), cls.nx, cls.ny, cls.pixel_A)
    with pytest.raises(ValueError):
        P.project_euler(ctx, wl.models[0], np.zeros((3, 4)), cls.nx, cls.ny, cls.pixel_A)


@pytest.mark.parametrize("prec", ["f32", "split_f16"])
def test_symmetry_restricted_set(P, ctx, prec):
    """A C_4-symmetric model scored over a symmetry-restricted Euler set
    (psi in [0, pi/2)) and over its four-fold expansion: log P agrees with
    the oracle on the restricted set, equals the full set's, and the
    restricted orientations scored as candidates under the full set's prior
    give exactly ln 4 less."""
    from workloads import expand_symmetry, symmetric_model, symmetry_restricted_euler
    n = 4
    rng = np.random.default_rng([160906634, 98])
    sph = symmetric_model(rng, 40, n, 40.0, 2.0)
    er = symmetry_restricted_euler(rng, 24, n)
    ef = expand_symmetry(er, n)
    wl = make_workload(1, n_images=5)
    cls = wl.classes[0]
    imgs = np.array([O.render_image(sph, O.euler_to_quat(*rng.uniform(0, 6, 3)), cls.img_ctf[i], cls.img_shift[i],
                                    cls.nx, cls.ny, cls.pixel_A, 1.0, 0.0, rng.standard_normal((cls.ny, cls.nx)),
                                    0.5) for i in range(5)], dtype=np.float32)
    _say(f"symmetry {prec}: C_{n} model, 5 images x {len(er)} restricted / {len(ef)} full orientations")
    qr = np.array([O.euler_to_quat(*e) for e in er])
    r = O.logpost_oracle(imgs.astype(np.float64), sph, qr, cls.ctf, cls.pixel_A, cls.max_shift, method="fft")
    pr = P.project_euler(ctx, sph, er, cls.nx, cls.ny, cls.pixel_A)
    pf = P.project_euler(ctx, sph, ef, cls.nx, cls.ny, cls.pixel_A)
    im = P.prepare_images(ctx, imgs)
    o_r = P.logpost(ctx, pr, im, cls.ctf, cls.max_shift, prec=prec)
    o_f = P.logpost(ctx, pf, im, cls.ctf, cls.max_shift, prec=prec)
    cand = np.tile(np.arange(len(er), dtype=np.int32), (5, 1))
    o_s = P.logpost(ctx, pf, im, cls.ctf, cls.max_shift, prec=prec, cand_q=cand)
    d_or = np.abs(o_r["logp"] - r.logp).max()
    d_rf = np.abs(o_r["logp"] - o_f["logp"]).max()
    d_sf = np.abs(o_s["logp"] - (o_f["logp"] - np.log(n))).max()
    _say(f"  |restricted - oracle| {d_or:.2e}, |restricted - full| {d_rf:.2e}, |subset - (full - ln 4)| {d_sf:.2e}")
    assert d_or <= 0.01 and d_rf <= 0.01 and d_sf <= 0.01
    assert o_r["best"]["q"].max() < len(er)
