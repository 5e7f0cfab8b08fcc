"""bioem_logpost_noalloc (fixed per-device scratch, no allocation) against
bioem_logpost on the same inputs, through the C ABI (needs a gfx950 GPU).

Two calls in a row share the device's scratch: the first (150 images x 4608
orientations x 8 CTF sets at 64^2) needs two image chunks of it, the second
is smaller (20 x 100 x 4), so stale records of the first would show."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload
from workloads.configs import shoemake_quaternions

pytestmark = pytest.mark.gpu

TOL_NAT = 0.01   # per-image |delta log P| bar of the plain path


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
def data():
    wl = make_workload(1)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    # 150 images: the 50 rendered ones and two circularly shifted copies
    imgs = np.concatenate([imgs, np.roll(imgs, 3, axis=2), np.roll(imgs, -2, axis=1)])
    return wl, cls, np.ascontiguousarray(imgs)


def _pair(P, ctx, proj, ih, ctf, S):
    """(reference dict, no-alloc logp, no-alloc best) on the same inputs."""
    import torch
    ref = P.logpost(ctx, proj, ih, ctf, S, prec="f32", device_out=True)
    dev = torch.device("cuda", ctx.device)
    logp = torch.full((ih.n,), float("nan"), dtype=torch.float64, device=dev)
    best = torch.zeros(ih.n * P.BEST_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    P.logpost_noalloc(ctx, proj, ih, ctf, S, logp, best)
    torch.cuda.synchronize()
    return (ref["logp"].cpu().numpy(), P.best_from_bytes(ref["best"]), logp.cpu().numpy(),
            P.best_from_bytes(best))


def _check(ref_lp, ref_b, lp, b, label):
    d = np.abs(lp - ref_lp)
    _say(f"{label}: max |dlogP| = {d.max():.3e} over {lp.size} images")
    assert np.isfinite(lp).all()
    assert d.max() <= TOL_NAT, (label, d.max())
    for f in ("q", "c", "dx", "dy", "status"):
        assert np.array_equal(b[f], ref_b[f]), (label, f)
    assert np.abs(b["logl"] - ref_b["logl"]).max() <= TOL_NAT


def test_noalloc_matches_logpost_two_calls(P, ctx, data):
    wl, cls, imgs = data
    S = cls.max_shift
    quats = shoemake_quaternions(np.random.default_rng(20161), 4608)
    ctf8 = np.vstack([cls.ctf, cls.ctf * np.array([1.15, 1.0, 1.0])])
    _say(f"noalloc call 1: 150 images x 4608 orientations x 8 CTF sets, {cls.nx}^2, S={S}")
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    ih = P.prepare_images(ctx, imgs)
    _check(*_pair(P, ctx, proj, ih, ctf8, S), "call 1")
    _say("noalloc call 2: 20 images x 100 orientations x 4 CTF sets")
    proj2 = P.project(ctx, wl.models[0], cls.quats, cls.nx, cls.ny, cls.pixel_A)
    ih2 = P.prepare_images(ctx, imgs[:20])
    _check(*_pair(P, ctx, proj2, ih2, cls.ctf, S), "call 2")


def test_noalloc_rejects_oversize_and_bad_input(P, ctx, data):
    import torch
    wl, cls, imgs = data
    S = cls.max_shift
    dev = torch.device("cuda", ctx.device)
    proj = P.project(ctx, wl.models[0], shoemake_quaternions(np.random.default_rng(3), 4608), cls.nx, cls.ny,
                     cls.pixel_A)
    ih = P.prepare_images(ctx, imgs[:4])
    logp = torch.empty(4, dtype=torch.float64, device=dev)
    best = torch.empty(4 * P.BEST_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    # 4608 x 1024 records of one image (72 MiB) exceed the 64 MiB scratch
    big = np.tile(cls.ctf, (256, 1))
    with pytest.raises(P.BioemError) as e:
        P.logpost_noalloc(ctx, proj, ih, big, S, logp, best)
    assert e.value.status == P.bindings.BIOEM_EUNSUPPORTED and "scratch" in str(e.value)
    bad = cls.ctf.copy()
    bad[1, 0] = np.nan
    with pytest.raises(P.BioemError) as e:
        P.logpost_noalloc(ctx, proj, ih, bad, S, logp, best)
    assert e.value.status == P.bindings.BIOEM_EINVAL
    # a valid call after the rejected ones still matches bioem_logpost
    ref = P.logpost(ctx, proj, ih, cls.ctf, S, prec="f32")
    P.logpost_noalloc(ctx, proj, ih, cls.ctf, S, logp, best)
    torch.cuda.synchronize()
    assert np.abs(logp.cpu().numpy() - ref["logp"]).max() <= TOL_NAT
