"""Every compiled launch shape of the split-precision kernel vs the FP64 oracle.

The default shape is what the other tests exercise; the other variants (CTF
sets per wave item, waves per workgroup, load schedule, XCD-dealt tiles,
matrix-phase priority) are selectable and some are picked by the autotuner,
so each is checked here on a one-column-tile box (64^2, S = 5) and on a ragged
box whose last column tile has slots past nx/2 and whose rows are padded
(40 x 26, S = 12, two column tiles).  Every shape performs the same
arithmetic per evaluation; the compiler may contract the conjugate products
into FMAs differently per variant, so shapes are compared with each other to
a few 1e-4 nat rather than bitwise.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import make_workload

pytestmark = pytest.mark.gpu

N_SHAPES = 12          # compiled variants (an index past the last selects the default)
TOL = {"split_f16": 0.01, "split_bf16": 0.1}
SPREAD = {"split_f16": 2e-3, "split_bf16": 2e-2}   # between shapes


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
def cases(P, ctx):
    wl = make_workload(1, n_images=6)
    cls = wl.classes[0]
    out = []
    imgs = O.render_images(cls, wl.models)
    quats = cls.quats[:40]
    out.append(dict(name="64x64 S=5", proj=P.project(ctx, wl.models[0], quats, cls.nx, cls.ny, cls.pixel_A),
                    imgs=P.prepare_images(ctx, imgs), ctf=cls.ctf, S=cls.max_shift,
                    ref=O.logpost_oracle(imgs, wl.models[0], quats, cls.ctf, cls.pixel_A, cls.max_shift,
                                         method="fft").logp))
    nx, ny, pix = 40, 26, 3.1
    rng = np.random.default_rng(8)
    rimgs = np.array([O.render_image(wl.models[0], cls.img_quat[i], cls.img_ctf[i], (2, -1), nx, ny, pix,
                                     1.0, 0.0, rng.standard_normal((ny, nx)), 0.5) for i in range(4)],
                     dtype=np.float32)
    out.append(dict(name="40x26 S=12", proj=P.project(ctx, wl.models[0], quats[:11], nx, ny, pix),
                    imgs=P.prepare_images(ctx, rimgs), ctf=cls.ctf[:3], S=12,
                    ref=O.logpost_oracle(rimgs.astype(np.float64), wl.models[0], quats[:11], cls.ctf[:3], pix,
                                         12, method="fft").logp))
    return out


@pytest.mark.parametrize("prec", ["split_f16", "split_bf16"])
def test_every_launch_shape_matches_oracle(P, ctx, cases, prec):
    for c in cases:
        first = None
        for shape in range(N_SHAPES):
            lp = P.logpost(ctx, c["proj"], c["imgs"], c["ctf"], c["S"], prec=prec, kernel=shape + 1)["logp"]
            d = float(np.abs(lp - c["ref"]).max())
            _say(f"{c['name']} {prec} shape {shape}: max |dlogP| vs oracle {d:.2e}")
            assert d <= TOL[prec], (c["name"], shape, d)
            first = lp if first is None else first
            assert float(np.abs(lp - first).max()) <= SPREAD[prec], (c["name"], shape)


@pytest.mark.parametrize("tile", [None, (1, 1), (3, 5), (64, 64)])
def test_f32_matrix_core_tiles_match_oracle(P, ctx, cases, tile):
    """The FP32 matrix-core form under several item tiles (the tile only
    reorders the work: results are bitwise the same)."""
    for c in cases:
        lp = P.logpost(ctx, c["proj"], c["imgs"], c["ctf"], c["S"], prec="f32", kernel=1, tile=tile)["logp"]
        d = float(np.abs(lp - c["ref"]).max())
        _say(f"{c['name']} f32 matrix cores tile {tile}: max |dlogP| vs oracle {d:.2e}")
        assert d <= 0.01, (c["name"], tile, d)
        ref = P.logpost(ctx, c["proj"], c["imgs"], c["ctf"], c["S"], prec="f32", kernel=1)["logp"]
        assert np.array_equal(lp, ref)
