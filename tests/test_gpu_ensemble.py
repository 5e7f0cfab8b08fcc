"""Ensemble posterior, Eq. (pb2): bioem_ensemble against the FP64 oracle.

Per-image values and the total are compared element by element with the
oracle on seeded inputs: magnitudes of real posteriors (-2.3e5 nat), ragged
image counts around the kernels' 256-thread blocks and 1024-thread sum,
weights with zeros, degenerate entries (NaN, -inf), host and device memory.
Then end to end: per-model log posteriors from bioem_logpost for two models
on images drawn from one of them, combined on the GPU and by the oracle.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu

RTOL = 1e-12   # FP64 exp/log and a different summation order


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


def _close(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    assert a.shape == b.shape
    same_nonfinite = (np.isnan(a) & np.isnan(b)) | (np.isinf(a) & (a == b))
    fin = np.isfinite(b)
    assert np.all(same_nonfinite | fin), "non-finite values differ"
    assert np.all(np.isfinite(a[fin]))
    err = np.abs(a[fin] - b[fin]) / np.maximum(1.0, np.abs(b[fin]))
    assert err.size == 0 or float(err.max()) <= RTOL, float(err.max())


@pytest.mark.parametrize("nm,ni", [(1, 1), (2, 255), (3, 257), (4, 1000), (2, 5000), (7, 3)])
def test_ensemble_matches_oracle(P, ctx, nm, ni):
    import torch
    rng = np.random.default_rng([nm, ni])
    L = -2.3e5 + 300.0 * rng.standard_normal((nm, ni))
    w = rng.uniform(0.0, 1.0, nm)
    if nm > 2:
        w[1] = 0.0
    w /= math.fsum(w)
    _say(f"ensemble nm={nm} ni={ni}")
    ref_per, ref_tot = O.ensemble_logpost(L, w)
    per, tot = P.ensemble(ctx, L, w)
    _close(per, ref_per)
    _close([tot], [ref_tot])
    # device in, device out
    dper, dtot = P.ensemble(ctx, torch.from_numpy(L).cuda(), w, device_out=True)
    torch.cuda.synchronize()
    _close(dper.cpu().numpy(), ref_per)
    _close(dtot.cpu().numpy(), [ref_tot])


def test_ensemble_degenerate_and_empty(P, ctx):
    nan, inf = math.nan, math.inf
    L = np.array([[nan, -3.0, -inf, 1.0, -inf, 2.0],
                  [-2.0, nan, -inf, inf, 5.0, -inf]])
    for w in ([0.0, 1.0], [1.0, 0.0], [0.5, 0.5]):
        ref_per, ref_tot = O.ensemble_logpost(L, w)
        per, tot = P.ensemble(ctx, L, w)
        _close(per, ref_per)
        _close([tot], [ref_tot])
    # finite part only
    ref_per, ref_tot = O.ensemble_logpost(L[:, 4:], [0.25, 0.75])
    per, tot = P.ensemble(ctx, L[:, 4:], [0.25, 0.75])
    _close(per, ref_per)
    _close([tot], [ref_tot])
    per, tot = P.ensemble(ctx, np.zeros((3, 0)), [0.2, 0.3, 0.5])
    assert per.shape == (0,) and tot == 0.0


def test_ensemble_rejects_bad_weights(P, ctx):
    L = np.zeros((2, 4))
    for w in ([0.6, 0.6], [1.5, -0.5], [math.nan, 1.0], [0.0, 0.0]):
        with pytest.raises(P.BioemError):
            P.ensemble(ctx, L, w)
    with pytest.raises(ValueError):
        P.ensemble(ctx, L, [1.0])


def test_ensemble_of_two_models_end_to_end(P, ctx):
    # images from model 0 of a two-model workload, scored under both models on
    # the GPU; the GPU ensemble of those posteriors equals the oracle's, and the
    # generating model has the larger log evidence
    wl = make_workload(4, n_images=8)
    cls = wl.classes[0]
    quats = np.concatenate([cls.img_quat[:8], cls.quats[:88]])
    ctf = cls.ctf
    imgs = []
    for i in range(8):
        imgs.append(O.render_image(wl.models[0], cls.img_quat[i], cls.img_ctf[i], cls.img_shift[i], cls.nx, cls.ny,
                                   cls.pixel_A, 1.0, 0.0, cls.noise(i, i + 1)[0], 1.0))
    imgs = np.array(imgs, dtype=np.float32)
    im = P.prepare_images(ctx, imgs)
    L = []
    for m in range(2):
        pr = P.project(ctx, wl.models[m], quats, cls.nx, cls.ny, cls.pixel_A)
        L.append(P.logpost(ctx, pr, im, ctf, cls.max_shift, prec="split_f16")["logp"])
        pr.free()
    im.free()
    L = np.array(L)
    _say(f"two-model posteriors: {L[:, :3]}")
    for w in ([1.0, 0.0], [0.0, 1.0], [0.5, 0.5], [0.9, 0.1]):
        ref_per, ref_tot = O.ensemble_logpost(L, w)
        per, tot = P.ensemble(ctx, L, w)
        _close(per, ref_per)
        _close([tot], [ref_tot])
    _, t0 = P.ensemble(ctx, L, [1.0, 0.0])
    _, t1 = P.ensemble(ctx, L, [0.0, 1.0])
    assert t0 > t1
