"""GPU path vs the FP64 oracle, through the C ABI (needs a gfx950 GPU)."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu

TOL_NAT = 0.01   # per-image |delta log P| bar for the plain path
# bar per transform mode: FP32 and the fp16 hi/lo split (about 22 significant
# bits) meet the plain-path bar; the bf16 hi/lo split (about 16 bits) is the
# precision form with the 0.1 nat bar.
TOL = {"f32": 0.01, "f32_valu": 0.01, "split_f16": 0.01, "split_bf16": 0.1}
PRECS = ["f32", "f32_valu", "split_f16", "split_bf16"]
# f32: the default plain form (FP32 matrix cores, factored transform);
# f32_valu: the direct pruned transform on the vector ALUs (bioem_opts.kernel 2)
KW = {"f32": dict(prec="f32"), "f32_valu": dict(prec="f32", kernel=2),
      "split_f16": dict(prec="split_f16"), "split_bf16": dict(prec="split_bf16")}


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


@pytest.fixture(scope="module")
def cfg1():
    wl = make_workload(1)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    return wl, cls, imgs


@pytest.fixture(scope="module")
def cfg1_oracle(cfg1):
    wl, cls, imgs = cfg1
    return O.logpost_oracle(imgs, wl.models[0], cls.quats, cls.ctf, cls.pixel_A, cls.max_shift,
                            method="direct")


def test_render_matches_oracle(P, ctx, cfg1):
    wl, cls, _ = cfg1
    _say("render: config1 5 images")
    sel = slice(0, 5)
    proj = P.project(ctx, wl.models[0], cls.img_quat[sel], cls.nx, cls.ny, cls.pixel_A)
    norm = np.array([[1.3, 0.4], [0.8, -0.2], [1.0, 0.0], [2.0, 1.0], [0.5, 0.5]])
    got = P.render(ctx, proj, cls.img_ctf[sel], cls.img_shift[sel], norm_offset=norm)
    for j, i in enumerate(range(5)):
        ref = O.render_image(wl.models[0], cls.img_quat[i], cls.img_ctf[i], cls.img_shift[i],
                             cls.nx, cls.ny, cls.pixel_A, norm[j, 0], norm[j, 1])
        scale = np.abs(ref).max()
        assert np.abs(got[j] - ref).max() < 2e-6 * scale, (i, np.abs(got[j] - ref).max(), scale)


def test_render_noise_snr(P, ctx, cfg1):
    wl, cls, _ = cfg1
    proj = P.project(ctx, wl.models[0], cls.img_quat[:3], cls.nx, cls.ny, cls.pixel_A)
    noise = cls.noise(0, 3)
    got = P.render(ctx, proj, cls.img_ctf[:3], cls.img_shift[:3], noise=noise, snr=cls.snr)
    ref = O.render_images(cls.subset(3), wl.models)
    assert np.abs(got - ref).max() < 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("prec", PRECS)
def test_config1_logpost_parity(P, ctx, cfg1, cfg1_oracle, prec):
    wl, cls, imgs = cfg1
    r = cfg1_oracle
    _say(f"config1 parity prec={prec}: 50 images x 100 q x 4 c, S=5")
    proj = P.project(ctx, wl.models[0], cls.quats, cls.nx, cls.ny, cls.pixel_A)
    im = P.prepare_images(ctx, imgs)
    out = P.logpost(ctx, proj, im, cls.ctf, cls.max_shift, orient=True, **KW[prec])
    tol = TOL[prec]
    d = np.abs(out["logp"] - r.logp)
    _say(f"  max |dlogP| = {d.max():.3e}")
    assert d.max() <= tol
    b = out["best"]
    assert np.all(b["status"] == 0)
    assert np.abs(b["logl"] - r.best_logl).max() <= tol
    # several grid points can attain the maximum within the tolerance: every
    # reported point must attain it by the oracle's own likelihood there
    for i in range(len(imgs)):
        l_at = O.loglik_at(imgs[i], wl.models[0], cls.quats[b["q"][i]], cls.ctf[b["c"][i]], cls.pixel_A,
                           b["dx"][i], b["dy"][i])
        assert abs(l_at - r.best_logl[i]) <= tol, (i, l_at, r.best_logl[i])
        assert abs(b["logl"][i] - l_at) <= tol, (i, b["logl"][i], l_at)
    do = np.abs(out["orient"] - r.logp_orient)
    _say(f"  max |dlogP(q)| = {do.max():.3e}")
    assert do.max() <= tol


@pytest.mark.parametrize("prec", PRECS)
def test_recovery_on_grid(P, ctx, prec):
    wl = make_workload(1, n_images=1)
    cls = wl.classes[0]
    rng = np.random.default_rng(21)
    cases = [(17, 2, (3, -2)), (63, 0, (-4, 1)), (5, 3, (0, 5)), (88, 1, (-5, -5))]
    imgs = np.array([O.render_image(wl.models[0], cls.quats[q], cls.ctf[c], d, cls.nx, cls.ny,
                                    cls.pixel_A, 1.0, 0.0, rng.standard_normal((cls.ny, cls.nx)), 10.0)
                     for q, c, d in cases], dtype=np.float32)
    proj = P.project(ctx, wl.models[0], cls.quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost(ctx, proj, P.prepare_images(ctx, imgs), cls.ctf, cls.max_shift, **KW[prec])
    b = out["best"]
    for i, (q, c, d) in enumerate(cases):
        assert (b["q"][i], b["c"][i], b["dx"][i], b["dy"][i]) == (q, c, d[0], d[1])


@pytest.mark.parametrize("prec", PRECS)
def test_ragged_box_and_edges(P, ctx, prec):
    """Non-square box, S = 0 and S at its maximum, a single CTF, a constant image."""
    wl = make_workload(1, n_images=4)
    cls = wl.classes[0]
    nx, ny, pix = 40, 26, 3.1
    rng = np.random.default_rng(5)
    quats = cls.quats[:7]
    imgs = np.array([O.render_image(wl.models[0], cls.img_quat[i], cls.img_ctf[i], (1, -2), nx, ny,
                                    pix, 1.0, 0.0, rng.standard_normal((ny, nx)), 0.5)
                     for i in range(3)] + [np.full((ny, nx), 3.0)], dtype=np.float32)
    proj = P.project(ctx, wl.models[0], quats, nx, ny, pix)
    im = P.prepare_images(ctx, imgs)
    for S, ctf in [(0, cls.ctf[:1]), (3, cls.ctf), (12, cls.ctf[1:3])]:
        _say(f"ragged box {nx}x{ny} S={S} nc={len(ctf)} prec={prec}")
        out = P.logpost(ctx, proj, im, ctf, S, orient=True, **KW[prec])
        r = O.logpost_oracle(imgs[:3].astype(np.float64), wl.models[0], quats, ctf, pix, S, method="fft")
        assert np.abs(out["logp"][:3] - r.logp).max() <= TOL[prec]
        assert np.abs(out["orient"][:3] - r.logp_orient).max() <= TOL[prec]
        assert out["best"]["status"][3] == 1 and math.isnan(out["logp"][3])
        assert np.all(out["best"]["status"][:3] == 0)


@pytest.mark.parametrize("prec", PRECS)
def test_candidate_subset_matches_oracle(P, ctx, cfg1, prec):
    wl, cls, imgs = cfg1
    sub = imgs[:6]
    rng = np.random.default_rng(3)
    cand = np.stack([np.sort(rng.choice(100, 12, replace=False)) for _ in range(6)]).astype(np.int32)
    proj = P.project(ctx, wl.models[0], cls.quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost(ctx, proj, P.prepare_images(ctx, sub), cls.ctf, cls.max_shift, cand_q=cand,
                    orient=True, **KW[prec])
    for i in range(6):
        r = O.logpost_oracle(sub[i:i + 1].astype(np.float64), wl.models[0], cls.quats, cls.ctf,
                             cls.pixel_A, cls.max_shift, method="fft", q_subset=list(cand[i]))
        assert abs(out["logp"][i] - r.logp[0]) <= TOL[prec]
        assert out["best"]["q"][i] in set(cand[i].tolist())
        mask = np.zeros(100, bool)
        mask[cand[i]] = True
        assert np.all(np.isneginf(out["orient"][i][~mask]))
        assert np.abs(out["orient"][i][mask] - r.logp_orient[0][mask]).max() <= TOL[prec]


def test_invalid_arguments(P, ctx, cfg1):
    wl, cls, imgs = cfg1
    proj = P.project(ctx, wl.models[0], cls.quats[:3], cls.nx, cls.ny, cls.pixel_A)
    im = P.prepare_images(ctx, imgs[:2])
    with pytest.raises(P.BioemError) as e:
        P.logpost(ctx, proj, im, cls.ctf, 32)            # S >= nx/2
    assert e.value.status == -1
    bad = cls.ctf.copy()
    bad[0, 1] = 1.5
    with pytest.raises(P.BioemError):
        P.logpost(ctx, proj, im, bad, 2)                  # amplitude contrast > 1
    with pytest.raises(P.BioemError):
        P.project(ctx, wl.models[0], cls.quats[:3], 63, 64, cls.pixel_A)   # odd box
    with pytest.raises(P.BioemError):
        P.logpost(ctx, proj, im, cls.ctf, 2, cand_q=np.full((2, 1), 7, np.int32))  # q out of range
    im2 = P.prepare_images(ctx, np.zeros((1, 32, 32), np.float32))
    with pytest.raises(P.BioemError):
        P.logpost(ctx, proj, im2, cls.ctf, 2)             # box mismatch


def test_empty_inputs_rejected(P, ctx, cfg1):
    """No spheres, no orientations, no images or no CTF sets is an invalid
    argument (EINVAL), found before any work; the handles made before stay
    usable."""
    wl, cls, imgs = cfg1
    proj = P.project(ctx, wl.models[0], cls.quats[:3], cls.nx, cls.ny, cls.pixel_A)
    im = P.prepare_images(ctx, imgs[:2])
    cases = [lambda: P.project(ctx, wl.models[0][:0], cls.quats[:3], cls.nx, cls.ny, cls.pixel_A),
             lambda: P.project(ctx, wl.models[0], cls.quats[:0], cls.nx, cls.ny, cls.pixel_A),
             lambda: P.prepare_images(ctx, imgs[:0]),
             lambda: P.logpost(ctx, proj, im, cls.ctf[:0], 2)]
    for f in cases:
        with pytest.raises(P.BioemError) as e:
            f()
        assert e.value.status == -1
    assert np.all(np.isfinite(P.logpost(ctx, proj, im, cls.ctf, 2)["logp"]))


def test_nonfinite_pixels_rejected(P, ctx, cfg1):
    """A NaN or infinite pixel is an invalid argument, found before any work
    (host and device images)."""
    import torch
    _, _, imgs = cfg1
    for bad in (np.nan, np.inf):
        x = imgs[:3].copy()
        x[1, 7, 9] = bad
        with pytest.raises(P.BioemError) as e:
            P.prepare_images(ctx, x)
        assert e.value.status == -1
        with pytest.raises(P.BioemError) as e:
            P.prepare_images(ctx, torch.from_numpy(x).cuda())
        assert e.value.status == -1
    P.prepare_images(ctx, torch.from_numpy(imgs[:3].copy()).cuda()).free()


def test_duplicate_candidates_rejected(P, ctx, cfg1):
    wl, cls, imgs = cfg1
    proj = P.project(ctx, wl.models[0], cls.quats[:10], cls.nx, cls.ny, cls.pixel_A)
    im = P.prepare_images(ctx, imgs[:2])
    cand = np.array([[1, 4, 7], [2, 5, 2]], np.int32)
    with pytest.raises(P.BioemError) as e:
        P.logpost(ctx, proj, im, cls.ctf, 2, cand_q=cand)
    assert e.value.status == -1


@pytest.mark.parametrize("prec", PRECS)
def test_zero_projections_degenerate(P, ctx, cfg1, prec):
    """A model of zero weight projects to zero everywhere (every B = 0): each
    image is degenerate, status 1 and log P = NaN, and the call succeeds."""
    wl, cls, imgs = cfg1
    model = wl.models[0].copy()
    model[:, 4] = 0.0
    proj = P.project(ctx, model, cls.quats[:5], cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost(ctx, proj, P.prepare_images(ctx, imgs[:3]), cls.ctf, 2, **KW[prec])
    assert np.all(out["best"]["status"] == 1)
    assert np.all(np.isnan(out["logp"]))


# Relative accuracy of the window correlation X for each transform form, in
# units of its operand rounding (FP32: 2^-24; the fp16 hi/lo split keeps about
# 22 bits, the bf16 split about 16).  Measured at 224^2, SNR 100 (rho^2 =
# 0.99): about 1.5 units for F32 on the matrix cores, 8 on the vector ALUs,
# 13 for the fp16 split and 1 for the bf16 split; the bars allow 16, 16, 32
# and 4 units.
XREL = {"f32": 16 * 2.0 ** -24, "f32_valu": 16 * 2.0 ** -24, "split_f16": 32 * 2.0 ** -22,
        "split_bf16": 4 * 2.0 ** -16}


def _snr_tol(prec, img, model, quat, ctf, pixel, best_logl, nx, ny):
    """The per-image bar at high SNR: max(bar, (n-2) rho^2/(1-rho^2) XREL)
    with rho^2 at the maximum taken from the oracle's maximal log-likelihood
    (written out from Eq. (likeli) integrated: l = K_n + (1-n/2) ln(pi A)
    - ln(B)/2 + (1-n/2) log1p(-rho^2))."""
    n = nx * ny
    A = O.image_moments(img.astype(np.float64))[2]
    h = 0.5 * n
    const = (math.lgamma(h - 1.0) - math.log(2.0) - 0.5 * math.log(n) + (1.0 - h) * math.log(math.pi * A))
    i1 = O.filtered_projection(O.project_model(model, quat, nx, ny, pixel), O.ctf_envelope_table(*ctf, nx, ny, pixel))
    B = O.projection_norm(i1)
    rho2 = -math.expm1((best_logl - const + 0.5 * math.log(B)) / (1.0 - h))
    return max(TOL[prec], (n - 2) * rho2 / (1.0 - rho2) * XREL[prec]), rho2


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("snr", [10.0, 100.0])
def test_high_snr_logp(P, ctx, prec, snr):
    """log P where rho^2 approaches 1.  An error dX/X in the correlation moves
    l by about (n-2) rho^2/(1-rho^2) dX/X, so the bar widens as the fit
    tightens: each image is held to max(bar, that bound at its own maximal
    rho^2, from the oracle).  The grid holds the images' own orientations
    and CTF sets, so the maximal rho^2 approaches snr / (1 + snr)."""
    wl = make_workload(1, n_images=4)
    cls = wl.classes[0]
    rng = np.random.default_rng(int(snr))
    imgs = np.array([O.render_image(wl.models[0], cls.img_quat[i], cls.img_ctf[i], cls.img_shift[i], cls.nx, cls.ny,
                                    cls.pixel_A, 1.0, 0.0, rng.standard_normal((cls.ny, cls.nx)), snr)
                     for i in range(4)], dtype=np.float32)
    quats = np.concatenate([cls.img_quat[:4], cls.quats[:16]])
    ctf = cls.img_ctf[:4]
    r = O.logpost_oracle(imgs.astype(np.float64), wl.models[0], quats, ctf, cls.pixel_A, cls.max_shift,
                         method="fft")
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost(ctx, proj, P.prepare_images(ctx, imgs), ctf, cls.max_shift, **KW[prec])
    for i in range(4):
        q, c = int(r.best_q[i]), int(r.best_c[i])
        assert (q, c) == (i, i)
        tol, rho2 = _snr_tol(prec, imgs[i], wl.models[0], quats[q], ctf[c], cls.pixel_A, r.best_logl[i],
                             cls.nx, cls.ny)
        assert rho2 > 0.8 * snr / (1 + snr)
        d = abs(out["logp"][i] - r.logp[i])
        _say(f"snr {snr} {prec} image {i}: rho2 {rho2:.4f} |dlogP| {d:.3e} (bar {tol:.3e})")
        assert d <= tol, (i, d, tol)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("snr", [10.0, 100.0])
def test_high_snr_logp_224px_sample(P, ctx, prec, snr):
    """The same at the benchmark's 224^2 box and S = 20: two images, their
    own orientations and six others, their own two CTF sets."""
    wl = make_workload(2, n_images=2)
    cls = wl.classes[0]
    rng = np.random.default_rng(224 + int(snr))
    imgs = np.array([O.render_image(wl.models[0], cls.img_quat[i], cls.img_ctf[i], cls.img_shift[i], cls.nx, cls.ny,
                                    cls.pixel_A, 1.0, 0.0, rng.standard_normal((cls.ny, cls.nx)), snr)
                     for i in range(2)], dtype=np.float32)
    quats = np.concatenate([cls.img_quat[:2], cls.quats[:6]])
    ctf = cls.img_ctf[:2]
    _say(f"224^2 high SNR {snr} {prec}: 2 images x 8 q x 2 c, S={cls.max_shift}")
    r = O.logpost_oracle(imgs.astype(np.float64), wl.models[0], quats, ctf, cls.pixel_A, cls.max_shift,
                         method="fft")
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost(ctx, proj, P.prepare_images(ctx, imgs), ctf, cls.max_shift, **KW[prec])
    for i in range(2):
        q, c = int(r.best_q[i]), int(r.best_c[i])
        assert (q, c) == (i, i)
        tol, rho2 = _snr_tol(prec, imgs[i], wl.models[0], quats[q], ctf[c], cls.pixel_A, r.best_logl[i],
                             cls.nx, cls.ny)
        assert rho2 > 0.8 * snr / (1 + snr)
        d = abs(out["logp"][i] - r.logp[i])
        _say(f"  image {i}: rho2 {rho2:.4f} |dlogP| {d:.3e} (bar {tol:.3e})")
        assert d <= tol, (i, d, tol)
