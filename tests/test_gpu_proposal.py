"""The learned orientation proposal end to end on a reduced grid: what the
trained network gains over the method without it.

128^2 images of the proposal workload's model on the first 2304 orientations
of its grid at SNR 1, 20,000 training images labelled by the exhaustive
posterior, 20 epochs.  On 200 held-out images the network's top 64
orientations (2.8% of the grid) are scored and compared with the exhaustive
posterior of the same images:
* pruned log P never exceeds the exhaustive value (it is a sum over a subset
  with the full-grid prior);
* the trained network captures the posterior (|d log P| <= 0.1 nat) for far
  more images than the untrained network or a random 64-orientation subset;
* with the softmax-mass fallback every image falls back or is scored by
  the candidate list, and the evaluations computed drop accordingly.
"""
import sys

import numpy as np
import pytest

from workloads import make_workload, proposal_training_images

pytestmark = pytest.mark.gpu

NQ, NTRAIN, EPOCHS, K, SNR = 2304, 20000, 20, 64, 1.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1609_06634_amd as P
    from paper_1609_06634_amd import proposal as PR
    P.load()
    ctx = P.Context(0)
    dev = torch.device("cuda", 0)
    tr = proposal_training_images(NTRAIN, nq_grid=NQ)
    tr.snr = SNR
    wl = make_workload(5, n_images=200)
    model = wl.models[0]
    held = wl.classes[0]
    held.snr = SNR
    proj = P.project(ctx, torch.from_numpy(model).to(dev), torch.from_numpy(tr.quats).to(dev), tr.nx, tr.ny,
                     tr.pixel_A)
    _say(f"labelling {NTRAIN} training images over {NQ} orientations")
    data = PR.make_training_set(ctx, model, tr, proj, T=32)
    imgs = PR.render_class_images(ctx, torch.from_numpy(model).to(dev), held, 0, 200)
    ctf = torch.from_numpy(held.ctf).to(dev)
    im = P.prepare_images(ctx, imgs)
    ex = P.logpost(ctx, proj, im, ctf, held.max_shift, prec="split_f16")["logp"]
    return P, PR, ctx, tr, held, proj, data, imgs, ctf, ex


def test_trained_network_gains_over_untrained(setup):
    P, PR, ctx, tr, held, proj, data, imgs, ctf, ex = setup
    net = P.Net(ctx, 128, 32, 64, 64, 64, 32, NQ)
    net.set_params(PR.init_params(net, tr.quats))
    before = PR.score_with_proposal(ctx, net, proj, imgs, ctf, held.max_shift, K=K, tau=0.0)
    losses = PR.train(net, data, epochs=EPOCHS, batch=256, lr=2e-3)
    after = PR.score_with_proposal(ctx, net, proj, imgs, ctf, held.max_shift, K=K, tau=0.0)
    d0, d1 = ex - before.logp, ex - after.logp
    f0, f1 = float(np.mean(d0 <= 0.1)), float(np.mean(d1 <= 0.1))
    _say(f"loss {losses[0]:.3f} -> {losses[-1]:.3f}; captured (|d| <= 0.1): untrained {f0:.3f}, "
         f"trained {f1:.3f}, random subset {K / NQ:.3f}")
    assert np.all(d0 >= -1e-6) and np.all(d1 >= -1e-6)     # a subset never exceeds the full sum
    assert losses[-1] < losses[0]
    # the captured fraction moves by a few images when the labels move at the
    # 1e-3 nat level (0.285 and 0.240 measured on two library builds whose
    # labels agree in 99.85% of the top-32 lists): the claim is the gain
    assert f1 >= 0.2 and f1 >= 4 * max(f0, K / NQ)
    # fallback below the mass threshold: those images are exact, the rest pruned
    fb = PR.score_with_proposal(ctx, net, proj, imgs, ctf, held.max_shift, K=K, tau=0.5)
    exact = fb.fallback
    assert np.abs(fb.logp[exact] - ex[exact]).max(initial=0.0) <= 1e-9 * np.abs(ex).max()
    assert np.allclose(fb.logp[~exact], after.logp[~exact])
    frac = fb.evals / (200 * NQ * len(held.ctf))
    _say(f"fallback {exact.mean():.2f}, evaluations computed {frac:.3f} of exhaustive")
    assert frac < 1.0
    net.close()


def test_config5_grid_and_snr_capture_report():
    """At the proposal workload's own size and signal (36,864 orientations,
    SNR 0.1, top 256), with a short training run (5,000 labelled images, 3
    epochs): reports the fraction of held-out images the pruned posterior
    captures (|d log P| <= 0.1 against the exhaustive posterior) and the
    evaluations the mass fallback saves, and checks what must hold whatever
    the network learned: the pruned value never exceeds the exhaustive one,
    and fallen-back images are exact."""
    import torch
    import paper_1609_06634_amd as P
    from paper_1609_06634_amd import proposal as PR
    P.load()
    ctx = P.Context(0)
    dev = torch.device("cuda", 0)
    wl = make_workload(5, n_images=100)
    held = wl.classes[0]
    model = wl.models[0]
    nq = len(held.quats)
    proj = P.project(ctx, torch.from_numpy(model).to(dev), torch.from_numpy(held.quats).to(dev), held.nx, held.ny,
                     held.pixel_A)
    tr = proposal_training_images(5000)
    _say(f"config-5 size: labelling 5000 images over {nq} orientations at SNR {held.snr}")
    data = PR.make_training_set(ctx, model, tr, proj, T=32)
    net = P.Net(ctx, 128, 32, 64, 128, 128, 32, nq)
    net.set_params(PR.init_params(net, held.quats))
    PR.train(net, data, epochs=3, batch=256, lr=1e-3)
    imgs = PR.render_class_images(ctx, torch.from_numpy(model).to(dev), held, 0, 100)
    ctf = torch.from_numpy(held.ctf).to(dev)
    im = P.prepare_images(ctx, imgs)
    ex = P.logpost(ctx, proj, im, ctf, held.max_shift, prec="split_f16")["logp"]
    pr = PR.score_with_proposal(ctx, net, proj, imgs, ctf, held.max_shift, K=256, tau=0.0)
    fb = PR.score_with_proposal(ctx, net, proj, imgs, ctf, held.max_shift, K=256, tau=0.5)
    d = ex - pr.logp
    saved = 1.0 - fb.evals / (100 * nq * len(held.ctf))
    _say(f"captured (|d| <= 0.1): {np.mean(d <= 0.1):.3f} (random 256-subset {256 / nq:.4f}); fallback "
         f"{fb.fallback.mean():.2f}; evaluations saved {saved:.3f}")
    assert np.all(d >= -1e-6)
    exact = fb.fallback
    assert np.abs(fb.logp[exact] - ex[exact]).max(initial=0.0) <= 1e-9 * np.abs(ex).max()
    net.close()
