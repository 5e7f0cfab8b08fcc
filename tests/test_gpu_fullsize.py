"""Full-size 224^2 parity: the HIP path at the bench's shapes vs the FP64 oracle.

The bench runs 1000 images over 4608 orientations x 8 CTF sets with shifts
+-20.  Here the first 16 images of that seeded workload go through the same
launch configuration (full orientation grid, all CTF sets, same shift window)
and are compared with

* stored oracle values (tests/golden/config2_full_grid.json, written by
  tests/golden/make_config2_golden.py, which calls only the oracle): log P per
  image, the maximal log-likelihood and its grid point, and the orientation
  posteriors of each image's 8 most probable orientations;
* live oracle evaluations of a few orientations sampled at random, computed
  one by one here.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_full_grid.json")
TOL = {"f32": 0.01, "split_f16": 0.01, "split_bf16": 0.1}


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
def setup(P):
    with open(GOLDEN) as f:
        gold = json.load(f)
    ni = len(gold["images"])
    wl = make_workload(2, n_images=ni)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    ctx = P.Context(0)
    _say(f"full-size setup: project {len(cls.quats)} orientations at {cls.nx}^2, {ni} images")
    proj = P.project(ctx, wl.models[0], cls.quats, cls.nx, cls.ny, cls.pixel_A)
    im = P.prepare_images(ctx, imgs)
    return ctx, wl, cls, imgs, proj, im, gold


@pytest.mark.parametrize("prec", ["split_f16", "f32", "split_bf16"])
def test_fullsize_matches_stored_oracle(P, setup, prec):
    ctx, wl, cls, imgs, proj, im, gold = setup
    _say(f"full-size parity prec={prec}: {len(imgs)} images x 4608 q x 8 c, S=20")
    out = P.logpost(ctx, proj, im, cls.ctf, cls.max_shift, prec=prec, orient=True)
    tol = TOL[prec]
    rows = gold["images"]
    ref = np.array([r["logp"] for r in rows])
    d = np.abs(out["logp"] - ref)
    _say(f"  max |dlogP| = {d.max():.3e}")
    assert d.max() <= tol, d
    b = out["best"]
    assert np.all(b["status"] == 0)
    for i, r in enumerate(rows):
        assert abs(b["logl"][i] - r["best_logl"]) <= tol, (i, b["logl"][i], r["best_logl"])
        if b["q"][i] == r["best_q"] and b["c"][i] == r["best_c"]:
            assert (b["dx"][i], b["dy"][i]) == (r["best_dx"], r["best_dy"])
        # the reported grid point attains the maximum by the oracle's own
        # likelihood there (several points can be within the tolerance)
        l_at = O.loglik_at(imgs[i], wl.models[0], cls.quats[b["q"][i]], cls.ctf[b["c"][i]], cls.pixel_A,
                           b["dx"][i], b["dy"][i])
        assert abs(l_at - r["best_logl"]) <= tol, (i, l_at, r["best_logl"])
        for q, v in r["orient"].items():
            assert abs(out["orient"][i, int(q)] - v) <= tol, (i, q, out["orient"][i, int(q)], v)
    # the per-orientation values and log P agree with each other at any size
    lse = np.logaddexp.reduce(out["orient"], axis=1)
    assert np.abs(lse - out["logp"]).max() < 1e-9 * np.abs(out["logp"]).max()


def test_fullsize_sampled_orientations_live(P, setup):
    ctx, wl, cls, imgs, proj, im, gold = setup
    rng = np.random.default_rng(4608)
    qs = sorted(int(q) for q in rng.choice(len(cls.quats), 3, replace=False))
    sel = [0, 1]
    _say(f"live oracle: images {sel}, orientations {qs}")
    out = P.logpost(ctx, proj, im, cls.ctf, cls.max_shift, prec="split_f16", orient=True)
    r = O.logpost_oracle(imgs[sel], wl.models[0], cls.quats, cls.ctf, cls.pixel_A, cls.max_shift,
                         method="fft", q_subset=qs)
    for j, i in enumerate(sel):
        for q in qs:
            assert abs(out["orient"][i, q] - r.logp_orient[j, q]) <= 0.01, (i, q)


@pytest.mark.parametrize("nc,S", [(3, 20), (5, 20), (4, 0), (8, 3), (4, 31)])
def test_224px_partial_ctf_passes(P, nc, S):
    """The 224^2 box's unrolled step sequence with CTF set counts that leave
    waves without a CTF set of their own (3: one idle wave; 5: a second pass
    with one set), with small shift windows (S = 0, 3) and with the largest
    window the matrix-core path takes (S = 31), on 12 orientations, against
    the oracle element by element (log P and the per-orientation values)."""
    wl = make_workload(2, n_images=2)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    rng = np.random.default_rng(224 + nc)
    quats = np.concatenate([cls.img_quat[:2], cls.quats[rng.choice(len(cls.quats), 10, replace=False)]])
    ctf = cls.ctf[:nc]
    _say(f"224^2 step sequence: 2 images x 12 q x {nc} c, S={S}")
    ctx = P.Context(0)
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost(ctx, proj, P.prepare_images(ctx, imgs), ctf, S, prec="f32", orient=True)
    r = O.logpost_oracle(imgs.astype(np.float64), wl.models[0], quats, ctf, cls.pixel_A, S, method="fft")
    d = np.abs(out["logp"] - r.logp)
    _say(f"  max |dlogP| = {d.max():.3e}")
    assert d.max() <= TOL["f32"], d
    assert np.abs(out["orient"] - r.logp_orient).max() <= TOL["f32"]
    assert np.all(out["best"]["status"] == 0)
    assert np.abs(out["best"]["logl"] - r.best_logl).max() <= TOL["f32"]


def test_224px_candidate_lists(P):
    """The 224^2 step sequence on per-image candidate lists (a proposal's
    pruned grid): log P over the candidates with the full grid's prior, the
    reported grid point among them, and the per-orientation values, against
    the oracle restricted to the same candidates."""
    wl = make_workload(2, n_images=3)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    rng = np.random.default_rng(2245)
    nq = 12
    quats = np.concatenate([cls.img_quat[:3], cls.quats[rng.choice(len(cls.quats), nq - 3, replace=False)]])
    cand = np.stack([np.sort(rng.choice(nq, 5, replace=False)) for _ in range(3)]).astype(np.int32)
    ctf = cls.ctf[:4]
    _say(f"224^2 candidate lists: 3 images x 5 of {nq} q x 4 c, S={cls.max_shift}")
    ctx = P.Context(0)
    proj = P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A)
    out = P.logpost(ctx, proj, P.prepare_images(ctx, imgs), ctf, cls.max_shift, prec="f32", cand_q=cand,
                    orient=True)
    for i in range(3):
        r = O.logpost_oracle(imgs[i:i + 1].astype(np.float64), wl.models[0], quats, ctf, cls.pixel_A,
                             cls.max_shift, method="fft", q_subset=list(cand[i]))
        d = abs(out["logp"][i] - r.logp[0])
        _say(f"  image {i}: |dlogP| = {d:.3e}")
        assert d <= TOL["f32"]
        assert out["best"]["q"][i] in set(cand[i].tolist())
        mask = np.zeros(nq, bool)
        mask[cand[i]] = True
        assert np.all(np.isneginf(out["orient"][i][~mask]))
        assert np.abs(out["orient"][i][mask] - r.logp_orient[0][mask]).max() <= TOL["f32"]
