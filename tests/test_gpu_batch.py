"""Batched scoring of uneven jobs in one persistent launch, and the autotuner.

Jobs of the mixed-size workload (96, 128, 180, 224 px boxes with shift
windows 8, 11, 16, 20, CTF grids of 4 to 16 sets, two models) on reduced
orientation grids and a few images each, through bioem_logpost_batch:
* persistent mode vs the FP64 oracle per job;
* persistent mode vs one launch per job (the same per-evaluation arithmetic,
  so the results are identical);
* a job with a per-image candidate list inside the batch;
* the autotuner: entries keyed by (box, S, log2 Nq, precision) and results
  identical to the untuned shape.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu

NQ = 24


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
def mixed(P):
    wl = make_workload(4, n_images=4)
    ctx = P.Context(0)
    jobs, refs = [], []
    for ci, cls in enumerate(wl.classes):
        imgs = O.render_images(cls, wl.models)
        if ci == 0:
            imgs = imgs[:3]          # uneven image counts across jobs
        im = P.prepare_images(ctx, imgs)
        quats = cls.quats[:NQ]
        for m in range(2):
            _say(f"mixed job: {cls.nx}^2 S={cls.max_shift} nc={len(cls.ctf)} model {m}")
            proj = P.project(ctx, wl.models[m], quats, cls.nx, cls.ny, cls.pixel_A)
            jobs.append(dict(proj=proj, imgs=im, ctf=cls.ctf, max_shift=cls.max_shift))
            refs.append(O.logpost_oracle(imgs, wl.models[m], quats, cls.ctf, cls.pixel_A,
                                         cls.max_shift, method="fft"))
            refs[-1].rescore = (imgs, wl.models[m], quats, cls.ctf, cls.pixel_A)
    return ctx, wl, jobs, refs


@pytest.mark.parametrize("prec,tol", [("split_f16", 0.01), ("split_bf16", 0.1)])
def test_persistent_batch_matches_oracle(P, mixed, prec, tol):
    ctx, wl, jobs, refs = mixed
    _say(f"persistent batch of {len(jobs)} jobs, prec={prec}")
    outs = P.logpost_batch(ctx, jobs, prec=prec, mode="persistent", orient=True)
    for j, (o, r) in enumerate(zip(outs, refs)):
        d = np.abs(o["logp"] - r.logp).max()
        _say(f"  job {j}: max |dlogP| = {d:.2e}")
        assert d <= tol, j
        assert np.abs(o["best"]["logl"] - r.best_logl).max() <= tol, j
        assert np.all(o["best"]["status"] == 0)
        # every reported grid point attains the maximum by the oracle's own
        # likelihood there
        imgs, model, quats, ctf, pixel = r.rescore
        b = o["best"]
        for i in range(len(imgs)):
            l_at = O.loglik_at(imgs[i], model, quats[b["q"][i]], ctf[b["c"][i]], pixel, b["dx"][i], b["dy"][i])
            assert abs(l_at - r.best_logl[i]) <= tol, (j, i, l_at, r.best_logl[i])
        assert np.abs(o["orient"][:, :NQ] - r.logp_orient[:, :NQ]).max() <= tol, j


def test_persistent_equals_per_job(P, mixed):
    ctx, wl, jobs, refs = mixed
    a = P.logpost_batch(ctx, jobs, prec="split_f16", mode="persistent", orient=True)
    b = P.logpost_batch(ctx, jobs, prec="split_f16", mode="per_job", orient=True)
    for x, y in zip(a, b):
        assert np.array_equal(x["logp"], y["logp"])
        assert np.array_equal(x["orient"], y["orient"])
        assert np.array_equal(x["best"], y["best"])


def test_batch_with_candidates(P, mixed):
    ctx, wl, jobs, refs = mixed
    cls = wl.classes[1]
    sub = [1, 4, 5, 9, 17, 23]
    ni = jobs[2]["imgs"].n
    cand = np.tile(np.array(sub, np.int32), (ni, 1))
    jb = dict(jobs[2], cand_q=cand)
    outs = P.logpost_batch(ctx, [jobs[0], jb, jobs[5]], prec="split_f16", mode="persistent")
    imgs = O.render_images(cls, wl.models)
    r = O.logpost_oracle(imgs, wl.models[0], cls.quats[:NQ], cls.ctf, cls.pixel_A, cls.max_shift,
                         method="fft", q_subset=sub)
    assert np.abs(outs[1]["logp"] - r.logp).max() <= 0.01
    assert np.abs(outs[0]["logp"] - refs[0].logp).max() <= 0.01
    assert np.abs(outs[2]["logp"] - refs[5].logp).max() <= 0.01


def test_two_models_generating_model_wins(P, mixed):
    ctx, wl, jobs, refs = mixed
    outs = P.logpost_batch(ctx, jobs, prec="split_f16", mode="persistent")
    wins = total = 0
    for ci, cls in enumerate(wl.classes):
        a, b = outs[2 * ci]["logp"], outs[2 * ci + 1]["logp"]
        owner = cls.img_model[:len(a)]
        wins += int(np.sum(np.where(owner == 0, a > b, b > a)))
        total += len(a)
    _say(f"generating model preferred on {wins}/{total} images")
    assert wins >= 0.75 * total


def test_autotune_entries_and_identical_results(P, mixed):
    ctx0, wl, jobs, refs = mixed
    ctx = P.Context(0)
    ctx.set_autotune(True)
    jb = jobs[6]          # 224^2, S = 20
    ref = P.logpost(ctx0, jb["proj"], jb["imgs"], jb["ctf"], jb["max_shift"], prec="split_f16",
                    orient=True)
    got = P.logpost(ctx, jb["proj"], jb["imgs"], jb["ctf"], jb["max_shift"], prec="split_f16",
                    orient=True)
    t = ctx.tunings()
    _say(f"tuned: {t}")
    assert len(t) == 1
    e = t[0]
    assert (e["nx"], e["ny"], e["max_shift"], e["prec"]) == (224, 224, 20, 2)
    assert e["ew"] in (2, 4) and e["tile_images"] > 0 and e["tile_slots"] > 0
    assert e["ns_per_eval"] <= e["ns_per_eval_default"]
    assert np.array_equal(got["logp"], ref["logp"])
    assert np.array_equal(got["orient"], ref["orient"])
    P.logpost(ctx, jb["proj"], jb["imgs"], jb["ctf"], jb["max_shift"], prec="split_f16")
    assert len(ctx.tunings()) == 1       # the key is tuned once
    outs = P.logpost_batch(ctx, jobs[:2], prec="split_f16")
    assert len(ctx.tunings()) == 2       # the 96^2 key (both models share it)
    for o, r in zip(outs, refs[:2]):
        assert np.abs(o["logp"] - r.logp).max() <= 0.01
    ctx.close()


def test_batch_invalid_arguments(P, mixed):
    ctx, wl, jobs, refs = mixed
    bad = dict(jobs[0], imgs=jobs[2]["imgs"])     # 96^2 projections with 128^2 images
    with pytest.raises(P.BioemError):
        P.logpost_batch(ctx, [jobs[1], bad])
    with pytest.raises(P.BioemError):
        P.logpost_batch(ctx, [dict(jobs[0], max_shift=48)])
