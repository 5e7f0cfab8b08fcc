#!/usr/bin/env python3
"""Throughput of the BioEM posterior hot path on one MI355X.

A step is one pass of the whole path over the paper-shaped workload
(224x224 px at 1.32 A/px, 1000 images, 4608 orientations x 8 CTF sets,
shifts +-20 px): Fourier projections of the 1500-sphere model over the
orientation grid, image spectra and sums, and the posterior over every
(image, orientation, CTF set, shift).  Inputs (model, grids, rendered
images) are resident in HBM before the timed region starts.

Prints one JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "posterior evals/s (image×orient×CTF, all shifts) @224² px; |Δlog P| vs FP64"



def alg_flops(n: int, S: int):
    """Algorithmic work of one evaluation (image x orientation x CTF set, all
    (2S+1)^2 shifts) on an n x n box: FP32 flops of the pointwise product
    (6 per half-spectrum coefficient) and of the pruned inverse transform
    counted as FFTs (stage 1: n/2+1 complex columns of 5 n log2 n; stage 2:
    2S+1 real rows of 2.5 n log2 n), and FP64 flops of the likelihood and
    log-sum-exp (45 per shift)."""
    h = n * (n // 2 + 1)
    lg = math.log2(n)
    fp32 = 6 * h + (n // 2 + 1) * 5 * n * lg + (2 * S + 1) * 2.5 * n * lg
    fp64 = (2 * S + 1) ** 2 * 45
    return fp32, fp64


ALG_FP32_PER_EVAL, ALG_FP64_PER_EVAL = alg_flops(224, 20)
# MI355X dense peaks (TFLOP/s): FP32 matrix cores (the FP32 vector ALUs reach
# the same figure only with packed instructions, which this build does not
# use), FP64, and fp16/bf16 matrix cores.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_F16_MFMA_TFLOPS = 2500.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "config2_full_grid.json")


def issued_mfma_flops(prec: str, n: int, S: int) -> float:
    """Matrix-core flops the kernel issues per evaluation (box n x n, window S).

    f32: per half group of 16 column pairs, one 16x16x4 FP32 product per
    stage-1 K-step and block (4 blocks, re and im) and 32 stage-2 products.
    split: per 16-column tile, 2 x 3 16x16x32 products per 32-row K-step and
    window tile plus 3 per pair of window tiles in stage 2."""
    if prec == "f32":
        H = n // 2
        j1 = n // 4 - 1 if n % 4 == 0 else (n - 2) // 4
        ks1 = (j1 + 1 + 3) // 4
        nreg = H // 2 - 1 if n % 4 == 0 else (H - 1) // 2
        nhg = (1 + nreg + 7) // 8
        return float((8 * ks1 + 32) * nhg * 2 * 16 * 16 * 4)
    nt = (S + 8) // 8
    ks = (n + 31) // 32
    mt = (n // 2 + 15) // 16
    return float(mt * (ks * nt * 2 * 3 + nt * nt * 3) * 2 * 16 * 16 * 32)


def roofline_of(prec: str, evals: float, t_launch: float, f32: float, f64: float, kernel: str, n: int, S: int,
                traffic=None) -> dict:
    """Roofline record of one posterior launch: the algorithmic work (the
    pruned transform and pointwise product at the peak of the unit that does
    the contraction, the likelihood epilogue at the FP64 peak) against the
    launch's measured duration.  frac = time at the roof / measured time;
    achieved = frac x peak."""
    peak = PEAK_FP32_TFLOPS if prec == "f32" else PEAK_F16_MFMA_TFLOPS
    roof_t = f32 / (peak * 1e12) + f64 / (PEAK_FP64_TFLOPS * 1e12)
    frac = evals * roof_t / t_launch
    issued = issued_mfma_flops(prec, n, S)
    return {"bound": "mfma", "achieved": round(frac * peak, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(frac, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
            "kernel": kernel, "kernel_ms_per_launch": round(t_launch * 1e3, 3), "evals_per_launch": evals,
            "roof_evals_per_s": round(1.0 / roof_t, 1),
            "alg_mflop_per_eval": {"transform_fp32": round(f32 / 1e6, 4), "epilogue_fp64": round(f64 / 1e6, 4)},
            "issued_mfma_mflop_per_eval": round(issued / 1e6, 4),
            "issued_over_algorithmic": round(issued / f32, 3),
            "peak_note": ("FP32 matrix cores (157.3 TF) for the transform, FP64 (78.6 TF) for the epilogue"
                          if prec == "f32" else
                          "fp16/bf16 matrix cores (2.5 PF dense) for the transform, FP64 (78.6 TF) for the epilogue")}


def source_hash() -> str:
    """SHA-256 over the library's HIP sources, in name order."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1609_06634_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel: str, prec: str, evals_per_launch: float):
    """HBM bytes per launch from the committed counter summaries, or None.

    The summaries under profiles/ carry one 'bench-traffic:' record per
    measured configuration; a record counts only if it was taken on the
    current sources, the same kernel, precision and launch size (default
    launch shape)."""
    import glob
    want = source_hash()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(f) as fh:
            for line in fh:
                if not line.startswith("bench-traffic:"):
                    continue
                rec = json.loads(line.split(":", 1)[1])
                if (rec.get("source_sha256") == want and rec.get("kernel") == kernel
                        and rec.get("prec") == prec
                        and float(rec.get("evals_per_launch", -1)) == float(evals_per_launch)):
                    return float(rec["traffic_bytes"])
    return None


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(sample: str, method: str = "fft"):
    """Time the FP64 oracle on a bounded sample of the same workload.

    method "fft": the correlation window by FP64 FFTs (numpy), the paper's
    own CPU formulation; "direct": the direct circular correlation."""
    import numpy as np
    import oracle as O
    from workloads import make_workload
    ni, nq, nc = (int(x) for x in sample.split("x"))
    wl = make_workload(2, n_images=ni)
    cls = wl.classes[0]
    imgs = O.render_images(cls, wl.models)
    t0, c0 = time.perf_counter(), time.process_time()
    O.logpost_oracle(imgs, wl.models[0], cls.quats[:nq], cls.ctf[:nc], cls.pixel_A, cls.max_shift,
                     method=method)
    dt, cpu_s = time.perf_counter() - t0, time.process_time() - c0
    # cores actually used: the process's CPU time over the wall time (numpy's
    # FFT is single-threaded; its matrix products may use several threads)
    threads = max(1.0, round(cpu_s / dt, 1))
    evals = ni * nq * nc
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{ni} images x {nq} orientations x {nc} CTF sets of the 224^2 workload, "
                      f"all 1681 shifts, FP64 {'FFT' if method == 'fft' else 'direct'} correlation; "
                      f"{dt:.1f} s on {cpu} "
                      f"(os.cpu_count()={os.cpu_count()})"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f32", choices=["f32", "split_f16", "split_bf16"])
    ap.add_argument("--images", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="16x128x8",
                    help="images x orientations x CTF sets for the oracle's FFT form")
    ap.add_argument("--cpu-sample-direct", default="2x16x2",
                    help="the same for the oracle's direct correlation")
    ap.add_argument("--workload", default="paper224", choices=["paper224", "mixed", "smalljobs", "proposal",
                                                                   "crossover"],
                    help="paper224: 224^2, 1000 images x 4608 orientations x 8 CTF sets (default); "
                         "mixed: 96/128/180/224 px classes x two models in one persistent launch; "
                         "proposal: 128^2 x 36,864 orientations with the learned top-K proposal; "
                         "crossover: real-space (cropping) against Fourier forms for S = 0..3 at 224^2")
    ap.add_argument("--train-images", type=int, default=100000)
    ap.add_argument("--epochs", type=int, default=60, help="proposal: at most this many epochs")
    ap.add_argument("--plateau", type=float, default=0.003,
                    help="proposal: stop when the loss has not improved by this fraction in 3 epochs")
    ap.add_argument("--topk", type=int, default=256)
    ap.add_argument("--tau", type=float, default=0.5)
    ap.add_argument("--channels", default="32,64,128,128", help="proposal: convolution channels")
    ap.add_argument("--snr", type=float, default=None, help="proposal: SNR of training and held-out images")
    ap.add_argument("--job-images", type=int, default=16, help="smalljobs: images per job")
    ap.add_argument("--job-orientations", type=int, default=288, help="smalljobs: orientations per job")
    ap.add_argument("--plain-images", type=int, default=8,
                    help="proposal workload: images scored by the plain FP32 form for comparison")
    ap.add_argument("--no-autotune", action="store_true",
                    help="mixed workload: default launch shape and item tiles for every job")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the reference "
                         "kernel for scaling HBM traffic counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding over orientations or images is described in the design notes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_1609_06634_amd as P
    from workloads import make_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    if args.copy_probe:
        x = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4, "launches": 3}), flush=True)
        return 0
    P.load()
    ctx = P.Context(0)
    if args.workload == "mixed":
        return run_mixed(args, P, ctx, torch, dev)
    if args.workload == "smalljobs":
        return run_smalljobs(args, P, ctx, torch, dev)
    if args.workload == "proposal":
        return run_proposal(args, P, ctx, torch, dev)
    if args.workload == "crossover":
        return run_crossover(args, P, ctx, torch, dev)

    # ---- inputs, resident in HBM ------------------------------------------------
    log("generating the 224^2 workload")
    wl = make_workload(2, n_images=args.images)
    cls = wl.classes[0]
    model = torch.from_numpy(wl.models[0]).to(dev)
    quats = torch.from_numpy(cls.quats).to(dev)
    ctf = torch.from_numpy(cls.ctf).to(dev)
    img_proj = P.project(ctx, torch.from_numpy(wl.models[0]).to(dev),
                         torch.from_numpy(cls.img_quat).to(dev), cls.nx, cls.ny, cls.pixel_A)
    images = P.render(ctx, img_proj, torch.from_numpy(cls.img_ctf).to(dev),
                      torch.from_numpy(cls.img_shift).to(dev),
                      noise=torch.from_numpy(cls.noise()).to(dev), snr=cls.snr, device_out=True)
    img_proj.free()
    torch.cuda.synchronize()
    ni, nq, nc, S = args.images, len(cls.quats), len(cls.ctf), cls.max_shift
    evals = ni * nq * nc
    log(f"inputs ready: {ni} images, {nq} orientations x {nc} CTF sets, S={S}")

    calls = {"project": 0.0, "prepare_images": 0.0, "logpost": 0.0}

    def step():
        t0 = time.perf_counter()
        proj = P.project(ctx, model, quats, cls.nx, cls.ny, cls.pixel_A)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        im = P.prepare_images(ctx, images)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = P.logpost(ctx, proj, im, ctf, S, prec=args.prec, device_out=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        calls["project"] += t1 - t0
        calls["prepare_images"] += t2 - t1
        calls["logpost"] += t3 - t2
        proj.free()
        im.free()
        return out

    for w in range(args.warmup):
        out = step()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    ctx.set_timing(True)
    for key in calls:
        calls[key] = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        torch.cuda.synchronize()
        log(f"step {k + 1}/{args.steps} done")
    dt = time.perf_counter() - t0
    kms, launches, kevals = ctx.kernel_time()
    ctx.set_timing(False)
    logp = out["logp"].cpu().numpy()
    assert np.all(np.isfinite(logp)), "non-finite log posterior"
    ms_step = dt / args.steps * 1e3
    value = evals / (dt / args.steps)

    # ---- roofline of the main kernel ------------------------------------------
    per_launch_evals = kevals / max(launches, 1)
    t_launch = kms / max(launches, 1) * 1e-3
    kname = "k_logpost_mf32" if args.prec == "f32" else "k_logpost_split"
    roofline = roofline_of(args.prec, per_launch_evals, t_launch, ALG_FP32_PER_EVAL, ALG_FP64_PER_EVAL, kname,
                           cls.nx, S, recorded_traffic(kname, args.prec, per_launch_evals))
    roofline["launches"] = launches

    # ---- accuracy of the timed run: its first images against the stored
    # FP64 oracle values of the same images (tests/golden) ----------------------
    dlogp = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            gold = json.load(f)
        ng = min(len(gold["images"]), ni)
        ref = np.array([r["logp"] for r in gold["images"][:ng]])
        d = np.abs(logp[:ng] - ref)
        dlogp = {"images": ng, "max": float(d.max()), "median": float(np.median(d)),
                 "against": "tests/golden/config2_full_grid.json (FP64 oracle, full grid)"}

    line = {"metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": {"f32": "f32 (FP32 matrix cores, FP32 accumulation), f64 likelihood terms",
                      "split_f16": "f16x2 split on MFMA (f32 acc), f64 likelihood terms",
                      "split_bf16": "bf16x2 split on MFMA (f32 acc), f64 likelihood terms"}[args.prec],
            "data": "synthetic",
            "config": {"workload": "224x224 px at 1.32 A/px, 1500-sphere model, "
                                   f"{ni} images x {nq} orientations x {nc} CTF sets, shifts +-{S}",
                       "images": ni, "orientations": nq, "ctf_sets": nc, "box": cls.nx,
                       "max_shift": S, "evals_per_step": evals, "prec": args.prec,
                       "step": "bioem_project + bioem_prepare_images + bioem_logpost"},
            "roofline": roofline,
            "dlogp_vs_fp64": dlogp,
            "ms_per_call": {k: round(v / args.steps * 1e3, 3) for k, v in calls.items()}}
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle (FFT form) on a {args.cpu_sample} sample")
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample, "fft")
        log(f"timing the CPU oracle (direct form) on a {args.cpu_sample_direct} sample")
        line["cpu_baseline_direct"] = cpu_baseline(args.cpu_sample_direct, "direct")
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def run_crossover(args, P, ctx, torch, dev) -> int:
    """Real-space (direct, border-cropping) against Fourier (wrapping) forms of
    the displacement sum as the window grows (S = 0..3): whole-call time per
    form on the 224^2 workload's full orientation x CTF grid, for a subset of
    its images.  Fourier calls include bioem_prepare_images; the real-space
    call includes making its nq x nc calculated images."""
    import numpy as np
    from workloads import make_workload
    ni = args.images if args.images != 1000 else 100
    log(f"generating the 224^2 workload ({ni} images)")
    wl = make_workload(2, n_images=ni)
    cls = wl.classes[0]
    model = torch.from_numpy(wl.models[0]).to(dev)
    pr = P.project(ctx, model, torch.from_numpy(cls.img_quat).to(dev), cls.nx, cls.ny, cls.pixel_A)
    imgs = P.render(ctx, pr, torch.from_numpy(cls.img_ctf).to(dev), torch.from_numpy(cls.img_shift).to(dev),
                    noise=torch.from_numpy(cls.noise(0, ni)).to(dev), snr=cls.snr, device_out=True)
    pr.free()
    ctf = torch.from_numpy(cls.ctf).to(dev)
    proj = P.project(ctx, model, torch.from_numpy(cls.quats).to(dev), cls.nx, cls.ny, cls.pixel_A)
    nq, nc = len(cls.quats), len(cls.ctf)
    evals = ni * nq * nc

    def fourier(S, prec):
        im = P.prepare_images(ctx, imgs)
        o = P.logpost(ctx, proj, im, ctf, S, prec=prec, device_out=True)
        im.free()
        return o["logp"]

    def crop(S):
        return P.logpost_crop(ctx, proj, imgs, ctf, S, device_out=True)["logp"]

    def timed(fn):
        fn()   # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, out

    points = []
    for S in range(4):
        tc, lc = timed(lambda: crop(S))
        tf, lf = timed(lambda: fourier(S, "f32"))
        ts, _ = timed(lambda: fourier(S, "split_f16"))
        d = float((lc - lf).abs().max())
        points.append({"S": S, "displacements": (2 * S + 1) ** 2, "crop_ms": tc * 1e3, "fourier_f32_ms": tf * 1e3,
                       "fourier_split_f16_ms": ts * 1e3, "crop_evals_per_s": evals / tc,
                       "fourier_f32_evals_per_s": evals / tf, "fourier_split_f16_evals_per_s": evals / ts,
                       "max_dlogp_crop_vs_wrap": d})
        log(f"S={S}: crop {tc * 1e3:.1f} ms, Fourier f32 {tf * 1e3:.1f} ms, split f16 {ts * 1e3:.1f} ms, "
            f"max |log P crop - wrap| {d:.3g}")
    proj.free()
    line = {"metric": "posterior evals/s per form vs shift window (real-space crop vs Fourier wrap)",
            "value": None, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "higher_is_better": True,
            "data": "synthetic",
            "config": {"workload": f"224x224 px at 1.32 A/px, {ni} images x {nq} orientations x {nc} CTF sets, "
                                   "S = 0..3", "evals_per_call": evals},
            "points": points}
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def run_mixed(args, P, ctx, torch, dev) -> int:
    """Four box sizes x two models scored in one persistent launch, against
    one launch per job.  A step is bioem_project of every (class, model) grid,
    bioem_prepare_images of every class and the posterior of every image
    under both models."""
    import numpy as np
    from workloads import make_workload
    per = args.images if args.images != 1000 else 2500
    log(f"generating the mixed-size workload ({per} images per class)")
    wl = make_workload(4, n_images=per)
    models = [torch.from_numpy(m).to(dev) for m in wl.models]
    classes = []
    evals = 0
    for cls in wl.classes:
        imgs = torch.empty((per, cls.ny, cls.nx), dtype=torch.float32, device=dev)
        for m in range(2):
            idx = np.nonzero(cls.img_model == m)[0]
            if len(idx) == 0:
                continue
            pr = P.project(ctx, models[m], torch.from_numpy(cls.img_quat[idx]).to(dev), cls.nx, cls.ny,
                           cls.pixel_A)
            noise = np.concatenate([cls.noise(int(i), int(i) + 1) for i in idx])
            imgs[torch.from_numpy(idx).to(dev)] = P.render(
                ctx, pr, torch.from_numpy(cls.img_ctf[idx]).to(dev),
                torch.from_numpy(cls.img_shift[idx]).to(dev), noise=torch.from_numpy(noise).to(dev),
                snr=cls.snr, device_out=True)
            pr.free()
        classes.append(dict(cls=cls, imgs=imgs, quats=torch.from_numpy(cls.quats).to(dev),
                            ctf=torch.from_numpy(cls.ctf).to(dev)))
        e = 2 * per * len(cls.quats) * len(cls.ctf)
        evals += e
    torch.cuda.synchronize()
    log(f"inputs ready: {evals} evaluations per step")

    def step(mode):
        handles, jobs = [], []
        for c in classes:
            cls = c["cls"]
            im = P.prepare_images(ctx, c["imgs"])
            handles.append(im)
            for m in range(2):
                pr = P.project(ctx, models[m], c["quats"], cls.nx, cls.ny, cls.pixel_A)
                handles.append(pr)
                jobs.append(dict(proj=pr, imgs=im, ctf=c["ctf"], max_shift=cls.max_shift))
        outs = P.logpost_batch(ctx, jobs, prec=args.prec, mode=mode, device_out=True)
        for h in handles:
            h.free()
        return outs

    ctx.set_autotune(not args.no_autotune)
    res = {}
    for mode in ("persistent", "per_job"):
        for w in range(args.warmup):
            step(mode)
            torch.cuda.synchronize()
            log(f"{mode}: warmup {w + 1}/{args.warmup} done")
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            outs = step(mode)
            torch.cuda.synchronize()
            log(f"{mode}: step {k + 1}/{args.steps} done")
        dt = (time.perf_counter() - t0) / args.steps
        kms, launches, kevals = ctx.kernel_time()
        ctx.set_timing(False)
        for o in outs:
            assert bool(torch.isfinite(o["logp"]).all()), "non-finite log posterior"
        res[mode] = dict(dt=dt, kms=kms / args.steps, launches=launches // args.steps)
        log(f"{mode}: {evals / dt:.4g} evals/s, kernel {kms / args.steps:.1f} ms per step")
    p, q = res["persistent"], res["per_job"]
    # the work of every class at its own box and window, against the launch
    # (or launches) of one step
    peak = PEAK_FP32_TFLOPS if args.prec == "f32" else PEAK_F16_MFMA_TFLOPS
    roof_t = 0.0
    for c in classes:
        f32c, f64c = alg_flops(c["cls"].nx, c["cls"].max_shift)
        roof_t += 2 * per * len(c["cls"].quats) * len(c["cls"].ctf) * (
            f32c / (peak * 1e12) + f64c / (PEAK_FP64_TFLOPS * 1e12))
    frac = roof_t / (p["kms"] * 1e-3)
    mixed_roof = {"bound": "mfma", "achieved": round(frac * peak, 3), "peak": peak, "unit": "TFLOP/s",
                  "frac": round(frac, 4), "traffic": None,
                  "kernel": ("k_logpost_batch" if args.prec != "f32" else
                             "k_logpost_mf32 (one launch per job: the F32 form has no persistent launch)"),
                  "kernel_ms_per_launch": round(p["kms"] / max(p["launches"], 1), 3), "launches": p["launches"]}
    # ensemble posterior, Eq. (pb2), of the two models over every image (each
    # class holds images of both): its log posterior on a grid of weights,
    # whose maximum estimates the mixing fraction, and how often the
    # generating model has the larger per-image posterior
    L = torch.stack([torch.cat([outs[2 * c + m]["logp"] for c in range(len(classes))])
                     for m in range(2)]).contiguous()
    truth = np.concatenate([c["cls"].img_model for c in classes])
    grid = np.linspace(0.0, 1.0, 21)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    totals = [P.ensemble(ctx, L, [w0, 1.0 - w0], device_out=True)[1] for w0 in grid]
    torch.cuda.synchronize()
    t_ens = (time.perf_counter() - t0) / len(grid)
    totals = np.array([float(t.item()) for t in totals])
    Lh = L.cpu().numpy()
    wins = float(np.mean(Lh[truth, np.arange(len(truth))] > Lh[1 - truth, np.arange(len(truth))]))
    ens = {"images": int(len(truth)), "weight_grid": len(grid),
           "best_weight_model0": float(grid[int(np.argmax(totals))]),
           "true_fraction_model0": float(np.mean(truth == 0)),
           "log_posterior_at_best": float(totals.max()),
           "log_bayes_factor_model0_over_model1": float(totals[-1] - totals[0]),
           "generating_model_wins": wins, "ms_per_call": t_ens * 1e3}
    log(f"ensemble: best w0 {ens['best_weight_model0']:.2f} (true {ens['true_fraction_model0']:.2f}), "
        f"generating model wins {wins:.3f}, {t_ens * 1e3:.3f} ms per call")
    line = {"metric": METRIC, "value": evals / p["dt"], "unit": "evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": p["dt"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"f32": "f32 transform, f64 likelihood",
                      "split_f16": "f16x2 split on MFMA (f32 acc), f64 likelihood",
                      "split_bf16": "bf16x2 split on MFMA (f32 acc), f64 likelihood"}[args.prec],
            "data": "synthetic",
            "config": {"workload": f"mixed sizes: 96/128/180/224 px x {per} images each, two models "
                                   "(1000 and 2500 spheres), grids (1152,4) (2304,8) (3456,12) "
                                   "(4608,16), shifts 8/11/16/20, "
                                   + ("one persistent launch" if args.prec != "f32" else
                                      "bioem_logpost_batch (one launch per job for F32)"),
                       "evals_per_step": evals, "prec": args.prec, "autotune": not args.no_autotune,
                       "step": "bioem_project + bioem_prepare_images + bioem_logpost_batch"},
            "roofline": mixed_roof,
            "per_job": {"value": evals / q["dt"], "ms_per_step": q["dt"] * 1e3,
                        "kernel_ms_per_step": q["kms"], "launches_per_step": q["launches"]},
            "persistent_over_per_job": q["dt"] / p["dt"],
            "ensemble": ens,
            "tuning": ctx.tunings()}
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def run_smalljobs(args, P, ctx, torch, dev) -> int:
    """Many small, uneven jobs in one call: for each of the mixed workload's
    four box sizes and two models, 6 jobs of 16 images over 288 orientations
    by default (--job-images, --job-orientations; the class's own CTF grid
    and window): 48 jobs, none of which fills the GPU alone.  Timed: bioem_logpost_batch in one persistent launch against
    one launch per job (inputs and projections prepared beforehand)."""
    import numpy as np
    from workloads import make_workload
    per, nq_job, reps = args.job_images, args.job_orientations, 6
    log(f"generating {len(range(reps)) * 8} small jobs ({per} images x {nq_job} orientations each)")
    wl = make_workload(4, n_images=per * reps)
    models = [torch.from_numpy(m).to(dev) for m in wl.models]
    jobs, handles = [], []
    evals = 0
    for cls in wl.classes:
        pr_img = P.project(ctx, models[0], torch.from_numpy(cls.img_quat).to(dev), cls.nx, cls.ny, cls.pixel_A)
        imgs = P.render(ctx, pr_img, torch.from_numpy(cls.img_ctf).to(dev), torch.from_numpy(cls.img_shift).to(dev),
                        noise=torch.from_numpy(cls.noise(0, per * reps)).to(dev), snr=cls.snr, device_out=True)
        pr_img.free()
        ctf = torch.from_numpy(cls.ctf).to(dev)
        for r in range(reps):
            im = P.prepare_images(ctx, imgs[r * per:(r + 1) * per].contiguous())
            handles.append(im)
            for m in range(2):
                q = torch.from_numpy(cls.quats[(r * nq_job) % len(cls.quats):][:nq_job].copy()).to(dev)
                pr = P.project(ctx, models[m], q, cls.nx, cls.ny, cls.pixel_A)
                handles.append(pr)
                jobs.append(dict(proj=pr, imgs=im, ctf=ctf, max_shift=cls.max_shift))
                evals += per * pr.n * len(cls.ctf)
    torch.cuda.synchronize()
    log(f"{len(jobs)} jobs, {evals} evaluations per call")
    res, outs = {}, {}
    for mode in ("persistent", "per_job"):
        for w in range(max(1, args.warmup)):
            P.logpost_batch(ctx, jobs, prec=args.prec, mode=mode, device_out=True)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for k in range(args.steps):
            outs[mode] = P.logpost_batch(ctx, jobs, prec=args.prec, mode=mode, device_out=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        kms, launches, _ = ctx.kernel_time()
        ctx.set_timing(False)
        res[mode] = dict(dt=dt, kms=kms / args.steps, launches=launches // args.steps)
        log(f"{mode}: {dt * 1e3:.2f} ms per call, main kernels {kms / args.steps:.2f} ms in "
            f"{launches // args.steps} launches")
    same = all(bool(torch.equal(a["logp"], b["logp"])) for a, b in zip(outs["persistent"], outs["per_job"]))
    p, q = res["persistent"], res["per_job"]
    line = {"metric": METRIC + " (many small jobs)", "value": evals / p["dt"], "unit": "evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": p["dt"] * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
            "config": {"workload": f"{len(jobs)} jobs: 96/128/180/224 px x 2 models x {reps}, {per} images x "
                                   f"{nq_job} orientations each, the class CTF grids (4-16 sets) and windows",
                       "evals_per_step": evals, "prec": args.prec, "step": "bioem_logpost_batch"},
            "persistent": {"ms_per_call": p["dt"] * 1e3, "kernel_ms": p["kms"], "launches": p["launches"]},
            "per_job": {"value": evals / q["dt"], "ms_per_call": q["dt"] * 1e3, "kernel_ms": q["kms"],
                        "launches": q["launches"]},
            "persistent_over_per_job": q["dt"] / p["dt"],
            "kernel_persistent_over_per_job": q["kms"] / max(p["kms"], 1e-9),
            "identical_results": same}
    print(json.dumps(line), flush=True)
    for h in handles:
        h.free()
    ctx.close()
    return 0


def run_proposal(args, P, ctx, torch, dev) -> int:
    """128^2 images over 36,864 orientations x 4 CTF sets: the exhaustive
    posterior against the learned proposal (network top-K orientations per
    image, exhaustive fallback below the softmax-mass threshold).  The
    network is trained here first, on images labelled by the exhaustive
    posterior (not timed).  value = effective evals/s of the proposal path
    (all images x full grid / its wall time, network included)."""
    import numpy as np
    from paper_1609_06634_amd import proposal as PR
    from workloads import make_workload, proposal_training_images
    held_n = args.images
    wl = make_workload(5, n_images=held_n)
    held = wl.classes[0]
    if args.snr is not None:
        held.snr = args.snr
    model = wl.models[0]
    model_dev = torch.from_numpy(model).to(dev)
    nq, nc, S = len(held.quats), len(held.ctf), held.max_shift
    proj = P.project(ctx, model_dev, torch.from_numpy(held.quats).to(dev), held.nx, held.ny, held.pixel_A)
    ctf = torch.from_numpy(held.ctf).to(dev)
    log(f"training set: {args.train_images} images labelled over {nq} orientations x {nc} CTF sets")
    tr = proposal_training_images(args.train_images)
    tr.snr = held.snr
    data = PR.make_training_set(ctx, model, tr, proj, T=32, chunk=2000, log=log)
    ch = [int(c) for c in args.channels.split(",")]
    net = P.Net(ctx, held.nx, ch[0], ch[1], ch[2], ch[3], 32, nq)
    net.set_params(PR.init_params(net, held.quats))
    t0 = time.perf_counter()
    losses = PR.train(net, data, epochs=args.epochs, batch=256, lr=1e-3, log=log, plateau=args.plateau)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    label_s, label_mass = data.seconds, float(np.median(data.mass))
    del data
    imgs = PR.render_class_images(ctx, model_dev, held, 0, held_n)
    torch.cuda.synchronize()
    evals = held_n * nq * nc

    def exhaustive():
        im = P.prepare_images(ctx, imgs)
        out = P.logpost(ctx, proj, im, ctf, S, prec=args.prec, device_out=True)
        im.free()
        return out["logp"]

    exhaustive()
    PR.score_with_proposal(ctx, net, proj, imgs, ctf, S, K=args.topk, tau=args.tau, prec=args.prec)
    t_ex, t_pr = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref = exhaustive()
        torch.cuda.synchronize()
        t_ex.append(time.perf_counter() - t0)
        r = PR.score_with_proposal(ctx, net, proj, imgs, ctf, S, K=args.topk, tau=args.tau, prec=args.prec)
        t_pr.append(r.seconds)
        log(f"step {k + 1}/{args.steps}: exhaustive {t_ex[-1] * 1e3:.1f} ms, proposal {r.seconds * 1e3:.1f} ms")
    ref = ref.cpu().numpy()
    d = ref - r.logp
    tex, tpr = float(np.mean(t_ex)), float(np.mean(t_pr))
    # the proposal alone (no fallback): what the network's top-K captures
    r0 = PR.score_with_proposal(ctx, net, proj, imgs, ctf, S, K=args.topk, tau=0.0, prec=args.prec)
    d0 = ref - r0.logp
    # the plain form (FP32 transforms, exhaustive grid) on the first images:
    # the posterior rate the proposal form is compared with, and its log P
    npl = min(args.plain_images, held_n)
    im_pl = P.prepare_images(ctx, imgs[:npl].contiguous())
    P.logpost(ctx, proj, im_pl, ctf, S, prec="f32", device_out=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = P.logpost(ctx, proj, im_pl, ctf, S, prec="f32", device_out=True)["logp"]
    torch.cuda.synchronize()
    t_pl = time.perf_counter() - t0
    im_pl.free()
    plain_rate = npl * nq * nc / t_pl
    d_pl = np.abs(r.logp[:npl] - plain.cpu().numpy())
    log(f"plain FP32 form: {plain_rate:.3g} evals/s on {npl} images; proposal form vs plain max |dlogP| "
        f"{d_pl.max():.3g}")
    line = {"metric": METRIC + " (effective, learned top-K proposal)", "value": evals / tpr,
            "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": tpr * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16 network; " + {"f32": "f32 posterior transforms",
                                          "split_f16": "f16x2 split posterior on MFMA (f32 acc)",
                                          "split_bf16": "bf16x2 split posterior on MFMA (f32 acc)"}[args.prec]
                     + ", f64 likelihood",
            "data": "synthetic",
            "config": {"workload": f"128x128 px at 2.31 A/px, 1000-sphere model, {held_n} held-out images x "
                                   f"{nq} orientations x {nc} CTF sets, shifts +-{S}, SNR {held.snr}; "
                                   f"top-{args.topk} proposal, exhaustive fallback below mass {args.tau}",
                       "network": {"channels": ch, "hidden": 32},
                       "evals_per_step": evals, "prec": args.prec},
            "exhaustive": {"value": evals / tex, "ms_per_step": tex * 1e3},
            "speedup_vs_exhaustive": tex / tpr,
            "dlogp": {"max": float(d.max()), "median": float(np.median(d)),
                      "frac_le_0.1": float(np.mean(d <= 0.1)), "min": float(d.min())},
            "fallback_fraction": float(r.fallback.mean()),
            "accepted": {"fraction": float(1.0 - r.fallback.mean()),
                         "dlogp_max": float(d[~r.fallback].max()) if (~r.fallback).any() else None,
                         "frac_le_0.1": float(np.mean(d[~r.fallback] <= 0.1)) if (~r.fallback).any() else None},
            "pruned_only": {"dlogp_median": float(np.median(d0)), "frac_le_0.1": float(np.mean(d0 <= 0.1)),
                            "random_topk_fraction_of_grid": args.topk / nq,
                            "network_mass_median": float(np.median(r0.mass)),
                            "ms_per_step": r0.seconds * 1e3},
            "evals_computed_fraction": r.evals / evals,
            "plain_f32": {"value": plain_rate, "images": npl, "speedup_of_proposal_form": (evals / tpr) / plain_rate,
                          "dlogp_max_vs_proposal_form": float(d_pl.max())},
            "training": {"images": args.train_images, "epochs": len(losses), "seconds": t_train,
                         "label_seconds": label_s, "loss_per_epoch": losses,
                         "label_mass_top32_median": label_mass}}
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
