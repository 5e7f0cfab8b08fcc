"""The largest box the library takes (512 x 512, with the largest shift window
each form takes there: S = 25, which the LDS of the best-displacement pass
bounds, and S = 15 for the split forms, whose LDS tiles bound it) and a large
ragged box (512 x 386: the y axis
has n % 4 == 2, so its orbit pairing has no quarter point), through the plain
F32 form on the FP32 matrix cores and the two split forms, against the FP64
oracle element by element: log P, the per-orientation values and the best
log-likelihood.  Images are rendered by the oracle with a shift and noise at
SNR 0.5; the model is the 1500-sphere one of the 224^2 workload at 1.32 A/px.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu

# The error of log P from a relative error e of X grows as n rho^2/(1 - rho^2) e
# (n pixels), so at n = 262,144 (five times the 224^2 box) the FP32 form runs at
# about half of its 0.01 nat bound (5e-3 measured), the fp16 split form, whose
# hi/lo pairs are exact only to about 2^-24 of the largest operand (fp16's
# subnormal range) even with its operands scaled up, at a few 1e-2 (held to the
# split forms' 0.1 nat bound), and the bf16 split form (about 16 significant
# bits, e ~ 2^-17) at about 1.4 nat: beyond its 0.1 nat bound, which it meets
# up to the 224^2 box.  Its check here is its error model at this size,
# n rho^2/(1 - rho^2) 2^-16 with rho^2 up to 0.5, about 4 nat.
TOL = {"f32": 0.01, "split_f16": 0.1, "split_bf16": 4.0}
CASES = [(512, 512, 25), (512, 512, 15), (512, 386, 12)]
FORMS = {"f32": [(512, 512, 25), (512, 386, 12)], "split_f16": [(512, 512, 15), (512, 386, 12)],
         "split_bf16": [(512, 512, 15), (512, 386, 12)]}


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
def boxes(P):
    wl = make_workload(2, n_images=2)
    cls = wl.classes[0]
    model = wl.models[0]
    ctx = P.Context(0)
    rng = np.random.default_rng(512)
    out = []
    for nx, ny, S in CASES:
        imgs = np.array([O.render_image(model, cls.img_quat[i], cls.img_ctf[i], (3, -2), nx, ny, cls.pixel_A,
                                        1.0, 0.0, rng.standard_normal((ny, nx)), 0.5) for i in range(2)],
                        dtype=np.float32)
        quats = np.concatenate([cls.img_quat[:2], cls.quats[rng.choice(len(cls.quats), 4, replace=False)]])
        ctf = cls.ctf[:3]
        _say(f"box {nx}x{ny}, S={S}: 2 images x {len(quats)} q x {len(ctf)} c (oracle)")
        ref = O.logpost_oracle(imgs.astype(np.float64), model, quats, ctf, cls.pixel_A, S, method="fft")
        proj = P.project(ctx, model, quats, nx, ny, cls.pixel_A)
        out.append(dict(key=(nx, ny, S), name=f"{nx}x{ny} S={S}", proj=proj, im=P.prepare_images(ctx, imgs),
                        ctf=ctf, S=S, ref=ref))
    return ctx, out


@pytest.mark.parametrize("prec", ["f32", "split_f16", "split_bf16"])
def test_largest_boxes_match_oracle(P, boxes, prec):
    ctx, cases = boxes
    for c in [c for c in cases if c["key"] in FORMS[prec]]:
        _say(f"{c['name']} {prec}")
        out = P.logpost(ctx, c["proj"], c["im"], c["ctf"], c["S"], prec=prec, orient=True)
        r = c["ref"]
        d = np.abs(out["logp"] - r.logp)
        _say(f"  max |dlogP| = {d.max():.3e}")
        assert d.max() <= TOL[prec], (c["name"], d)
        assert np.abs(out["orient"] - r.logp_orient).max() <= TOL[prec], c["name"]
        assert np.all(out["best"]["status"] == 0), c["name"]
        assert np.abs(out["best"]["logl"] - r.best_logl).max() <= TOL[prec], c["name"]


def test_one_past_the_largest_window_is_refused(P, boxes):
    """One step past each form's largest window at 512 x 512 is refused with
    EUNSUPPORTED before anything is enqueued."""
    ctx, cases = boxes
    c = [c for c in cases if c["key"] == (512, 512, 25)][0]
    for prec, S in (("f32", 26), ("split_f16", 16), ("split_bf16", 16)):
        with pytest.raises(P.bindings.BioemError, match="EUNSUPPORTED"):
            P.logpost(ctx, c["proj"], c["im"], c["ctf"], S, prec=prec)
