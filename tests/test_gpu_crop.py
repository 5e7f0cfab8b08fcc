"""Real-space variant with border cropping (Section 3, Center displacement):
bioem_logpost_crop against the FP64 oracle (``borders="crop"``).

Cases span several 16 x 16 workgroup tiles with ragged tails in images and
calculated images, every compiled window (S = 0..3), a non-square box, the
224^2 box of the paper's benchmark on a sample of its grid, and the argument
checks.  Bar: 0.01 nat per image, as for the FP32 Fourier form.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu

TOL = 0.01


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


def _check(out, r, tol=TOL, rescore=None):
    """log P and best points against the oracle; rescore = (imgs, model,
    quats, ctf, pixel): every reported point must attain the maximum by the
    oracle's own likelihood there."""
    d = np.abs(out["logp"] - r.logp)
    _say(f"  max |dlogP| = {d.max():.3e}")
    assert d.max() <= tol, d
    b = out["best"]
    assert np.all(b["status"] == 0)
    assert np.abs(b["logl"] - r.best_logl).max() <= tol
    same = (b["q"] == r.best_q) & (b["c"] == r.best_c) & (b["dx"] == r.best_dx) & (b["dy"] == r.best_dy)
    assert same.mean() >= 0.8, same
    if rescore is not None:
        imgs, model, quats, ctf, pixel = rescore[:5]
        psf = rescore[5] if len(rescore) > 5 else None
        for i in range(len(imgs)):
            l_at = O.loglik_at(imgs[i], model, quats[b["q"][i]], ctf[b["c"][i]], pixel, b["dx"][i], b["dy"][i],
                               borders="crop", psf_radius=psf)
            assert abs(l_at - r.best_logl[i]) <= tol, (i, l_at, r.best_logl[i])


@pytest.mark.parametrize("S", [0, 1, 2, 3])
def test_crop_matches_oracle_64px(P, ctx, S):
    wl = make_workload(1, n_images=20)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    quats = cls.quats[:11]
    ctf = cls.ctf[:3]          # 33 calculated images: three tiles, ragged
    _say(f"crop 64x64: 20 images x 11 q x 3 c, S={S}")
    r = O.logpost_oracle(imgs, wl.models[0], quats, ctf, cls.pixel_A, S, borders="crop")
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost_crop(ctx, proj, imgs, ctf, S)
    _check(out, r, rescore=(imgs, wl.models[0], quats, ctf, cls.pixel_A))
    if S == 0:
        # no displacement: the same function as the wrapped Fourier form
        im = P.prepare_images(ctx, imgs)
        f = P.logpost(ctx, proj, im, ctf, 0, prec="f32")
        assert np.abs(f["logp"] - out["logp"]).max() <= TOL
        im.free()
    proj.free()


def test_crop_ragged_box_device_memory(P, ctx):
    import torch
    wl = make_workload(1, n_images=4)
    cls = wl.classes[0]
    nx, ny, pix, S = 40, 26, 3.1, 3
    rng = np.random.default_rng(9)
    imgs = np.array([O.render_image(wl.models[0], cls.img_quat[i % 4], cls.img_ctf[i % 4], (2, -1), nx, ny, pix,
                                    1.5, -0.3, rng.standard_normal((ny, nx)), 0.5) for i in range(17)],
                    dtype=np.float32)
    quats = cls.quats[:7]
    ctf = cls.ctf[:2]
    _say("crop 40x26: 17 images x 7 q x 2 c, S=3, device memory")
    r = O.logpost_oracle(imgs.astype(np.float64), wl.models[0], quats, ctf, pix, S, borders="crop")
    proj = P.project(ctx, wl.models[0], quats, nx, ny, pix)
    out = P.logpost_crop(ctx, proj, torch.from_numpy(imgs).cuda(), torch.from_numpy(ctf).cuda(), S,
                         device_out=True)
    torch.cuda.synchronize()
    host = {"logp": out["logp"].cpu().numpy(), "best": P.best_from_bytes(out["best"])}
    _check(host, r, rescore=(imgs.astype(np.float64), wl.models[0], quats, ctf, pix))
    proj.free()


def test_crop_full_box_sample(P, ctx):
    # the 224^2, 1.32 A/px box of the benchmark, 16 orientations x 2 CTF sets
    wl = make_workload(2, n_images=3)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    quats = np.concatenate([cls.img_quat[:3], cls.quats[:13]])
    ctf = cls.ctf[:2]
    S = 2
    _say("crop 224x224: 3 images x 16 q x 2 c, S=2")
    r = O.logpost_oracle(imgs, wl.models[0], quats, ctf, cls.pixel_A, S, borders="crop")
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost_crop(ctx, proj, imgs, ctf, S)
    _check(out, r, rescore=(imgs, wl.models[0], quats, ctf, cls.pixel_A))
    proj.free()


def test_crop_arguments(P, ctx):
    wl = make_workload(1, n_images=2)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    proj = P.project(ctx, wl.models[0], cls.quats[:2], cls.nx, cls.ny, cls.pixel_A)
    with pytest.raises(P.BioemError) as e:
        P.logpost_crop(ctx, proj, imgs, cls.ctf[:1], 4)
    assert e.value.status == P.bindings.BIOEM_EUNSUPPORTED
    for bad in (-1, 32):
        with pytest.raises(P.BioemError) as e:
            P.logpost_crop(ctx, proj, imgs, cls.ctf[:1], bad)
        assert e.value.status == P.bindings.BIOEM_EINVAL
    with pytest.raises(ValueError):
        P.logpost_crop(ctx, proj, imgs[:, :32], cls.ctf[:1], 1)
    proj.free()


# ---- calculated images by the real-space PSF convolution, Eq. (5) --------

@pytest.mark.parametrize("S,R", [(0, 3), (2, 9), (3, 20)])
def test_crop_psf_matches_oracle_64px(P, ctx, S, R):
    wl = make_workload(1, n_images=12)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    quats = cls.quats[:7]
    ctf = cls.ctf[:3]
    _say(f"crop + real-space PSF 64x64: 12 images x 7 q x 3 c, S={S}, R={R}")
    r = O.logpost_oracle(imgs, wl.models[0], quats, ctf, cls.pixel_A, S, borders="crop", psf_radius=R)
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost_crop(ctx, proj, imgs, ctf, S, psf_radius=R)
    _check(out, r, rescore=(imgs, wl.models[0], quats, ctf, cls.pixel_A, R))
    # a different function from the Fourier-filtered form (the borders)
    f = P.logpost_crop(ctx, proj, imgs, ctf, S)
    assert np.abs(f["logp"] - out["logp"]).max() > 10 * TOL
    proj.free()


def test_crop_psf_ragged_box_device_memory(P, ctx):
    import torch
    wl = make_workload(1, n_images=4)
    cls = wl.classes[0]
    nx, ny, pix, S, R = 40, 26, 3.1, 2, 7
    rng = np.random.default_rng(19)
    imgs = np.array([O.render_image(wl.models[0], cls.img_quat[i % 4], cls.img_ctf[i % 4], (1, -2), nx, ny, pix,
                                    1.2, 0.4, rng.standard_normal((ny, nx)), 0.5) for i in range(9)],
                    dtype=np.float32)
    quats = cls.quats[:5]
    ctf = cls.ctf[:2]
    _say(f"crop + real-space PSF 40x26: 9 images x 5 q x 2 c, S={S}, R={R}, device memory")
    r = O.logpost_oracle(imgs.astype(np.float64), wl.models[0], quats, ctf, pix, S, borders="crop",
                         psf_radius=R)
    proj = P.project(ctx, wl.models[0], quats, nx, ny, pix)
    out = P.logpost_crop(ctx, proj, torch.from_numpy(imgs).cuda(), torch.from_numpy(ctf).cuda(), S,
                         device_out=True, psf_radius=R)
    torch.cuda.synchronize()
    host = {"logp": out["logp"].cpu().numpy(), "best": P.best_from_bytes(out["best"])}
    _check(host, r, rescore=(imgs.astype(np.float64), wl.models[0], quats, ctf, pix, R))
    proj.free()


def test_crop_psf_arguments(P, ctx):
    wl = make_workload(1, n_images=2)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    proj = P.project(ctx, wl.models[0], cls.quats[:2], cls.nx, cls.ny, cls.pixel_A)
    for R, status in [(-1, P.bindings.BIOEM_EINVAL), (32, P.bindings.BIOEM_EINVAL)]:
        with pytest.raises(P.BioemError) as e:
            P.logpost_crop(ctx, proj, imgs, cls.ctf[:1], 1, psf_radius=R)
        assert e.value.status == status
    big = P.project(ctx, wl.models[0], cls.quats[:1], 96, 96, cls.pixel_A)
    with pytest.raises(P.BioemError) as e:
        P.logpost_crop(ctx, big, np.zeros((1, 96, 96), np.float32) + 1.0, cls.ctf[:1], 1, psf_radius=33)
    assert e.value.status == P.bindings.BIOEM_EUNSUPPORTED
    proj.free()
    big.free()
