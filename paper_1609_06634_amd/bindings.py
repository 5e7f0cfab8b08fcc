"""Thin ctypes binding of libbioem.so (argument marshalling only).

Every computation runs inside the HIP library; this module converts numpy
arrays (host memory) or torch CUDA tensors (device memory) into pointers and
calls the C ABI declared in include/bioem.h.  If the shared library has not
been built, importing works but the first call raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbioem.so")

BIOEM_OK, BIOEM_EINVAL, BIOEM_ENOMEM, BIOEM_EDEVICE, BIOEM_EUNSUPPORTED = 0, -1, -2, -3, -4
MEM_HOST, MEM_DEVICE = 0, 1
PREC = {"f32": 0, "split_bf16": 1, "split_f16": 2}

_STATUS = {BIOEM_EINVAL: "EINVAL", BIOEM_ENOMEM: "ENOMEM", BIOEM_EDEVICE: "EDEVICE",
           BIOEM_EUNSUPPORTED: "EUNSUPPORTED"}


class BioemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Best(ctypes.Structure):
    _fields_ = [("logl", ctypes.c_double), ("q", ctypes.c_int32), ("c", ctypes.c_int32),
                ("dx", ctypes.c_int32), ("dy", ctypes.c_int32), ("status", ctypes.c_int32)]


BEST_DTYPE = np.dtype({"names": ["logl", "q", "c", "dx", "dy", "status"],
                       "formats": ["<f8", "<i4", "<i4", "<i4", "<i4", "<i4"],
                       "offsets": [0, 8, 12, 16, 20, 24], "itemsize": ctypes.sizeof(Best)})


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("out_mem", ctypes.c_int32),
                ("cand_q", ctypes.c_void_p), ("k", ctypes.c_int32), ("cand_mem", ctypes.c_int32),
                ("logp_orient", ctypes.c_void_p), ("kernel", ctypes.c_int32),
                ("tile_images", ctypes.c_int32), ("tile_slots", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("proj", ctypes.c_void_p), ("imgs", ctypes.c_void_p), ("ctf", ctypes.c_void_p),
                ("nc", ctypes.c_int32), ("ctf_mem", ctypes.c_int32), ("max_shift", ctypes.c_int32),
                ("k", ctypes.c_int32), ("cand_q", ctypes.c_void_p), ("cand_mem", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("logp", ctypes.c_void_p), ("best", ctypes.c_void_p),
                ("logp_orient", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("max_shift", ctypes.c_int32),
                ("nq_log2", ctypes.c_int32), ("prec", ctypes.c_int32), ("ew", ctypes.c_int32),
                ("tile_images", ctypes.c_int32), ("tile_slots", ctypes.c_int32),
                ("ns_per_eval", ctypes.c_double), ("ns_per_eval_default", ctypes.c_double)]


class CnnArch(ctypes.Structure):
    _fields_ = [("box", ctypes.c_int32), ("c1", ctypes.c_int32), ("c2", ctypes.c_int32),
                ("c3", ctypes.c_int32), ("c4", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("nq", ctypes.c_int32), ("reserved", ctypes.c_int32)]


BATCH_PERSISTENT, BATCH_PER_JOB = 0, 1

_lib = None

# (name, restype, argtypes) of every exported entry point.
_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double
SIGNATURES = [
    ("bioem_create", _I, [ctypes.c_int, _P, ctypes.POINTER(_P)]),
    ("bioem_destroy", None, [_P]),
    ("bioem_last_error", ctypes.c_char_p, [_P]),
    ("bioem_version", ctypes.c_char_p, []),
    ("bioem_project", _I, [_P, _P, _I, _P, _I, _I, _I, _D, _I, ctypes.POINTER(_P)]),
    ("bioem_project_euler", _I, [_P, _P, _I, _P, _I, _I, _I, _D, _I, ctypes.POINTER(_P)]),
    ("bioem_prepare_images", _I, [_P, _P, _I, _I, _I, _I, ctypes.POINTER(_P)]),
    ("bioem_logpost", _I, [_P, _P, _P, _P, _I, _I, _I, ctypes.POINTER(Opts), _P, _P]),
    ("bioem_render", _I, [_P, _P, _P, _P, _P, _P, _D, _I, _P, _I]),
    ("bioem_free_proj", None, [_P]),
    ("bioem_free_imgs", None, [_P]),
    ("bioem_proj_info", _I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    ("bioem_imgs_info", _I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    ("bioem_ctf_from_physical", _I, [_D, _D, _D, _D, ctypes.POINTER(_D)]),
    ("bioem_set_timing", _I, [_P, _I]),
    ("bioem_get_kernel_time", _I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    ("bioem_logpost_batch", _I, [_P, ctypes.POINTER(Job), _I, _I, _I, _I]),
    ("bioem_logpost_noalloc", _I, [_P, _P, _P, _P, _I, _I, _P, _P]),
    ("bioem_set_autotune", _I, [_P, _I]),
    ("bioem_tuning_count", _I, [_P]),
    ("bioem_tuning_entry", _I, [_P, _I, ctypes.POINTER(Tuning)]),
    ("bioem_cnn_create", _I, [_P, ctypes.POINTER(CnnArch), ctypes.POINTER(_P)]),
    ("bioem_cnn_destroy", None, [_P]),
    ("bioem_cnn_num_params", ctypes.c_int64, [_P]),
    ("bioem_cnn_set_params", _I, [_P, _P, _P, _I]),
    ("bioem_cnn_get_params", _I, [_P, _P, _P, _I]),
    ("bioem_cnn_forward", _I, [_P, _P, _P, _I, _I, _P, _I]),
    ("bioem_cnn_backward", _I, [_P, _P, _P, _I, _P, _P, _I, _I, ctypes.POINTER(ctypes.c_float), _P, _I]),
    ("bioem_cnn_adam", _I, [_P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    ("bioem_cnn_propose", _I, [_P, _P, _P, _I, _I, _I, _P, _P, _I]),
    ("bioem_topk", _I, [_P, _P, _I, _I, _I, _I, _P, _P, _I]),
    ("bioem_ensemble", _I, [_P, _P, _I, _I, _I, _P, _P, _P, _I]),
    ("bioem_logpost_crop", _I, [_P, _P, _P, _I, _I, _P, _I, _I, _P, _P, _I]),
    ("bioem_logpost_crop_psf", _I, [_P, _P, _P, _I, _I, _P, _I, _I, _I, _P, _P, _I]),
    ("bioem_cnn_input", _I, [_P, _P, _I, _I, _I, _I, _P, _I]),
]


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libbioem.so once; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} not built: run paper_1609_06634_amd.build.build()")
        # torch ships its own HIP runtime; loading it first makes the library
        # bind to that same runtime (one runtime per process, shared streams)
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - torch is a dependency
            pass
        lib = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def version() -> str:
    return load().bioem_version().decode()


def _torch():
    import torch  # noqa: WPS433 (only needed for device memory)
    return torch


def _arg(x, dtype, shape=None):
    """(pointer, mem kind, keep-alive) of a numpy array or a CUDA tensor."""
    if x is None:
        return None, MEM_HOST, None
    if isinstance(x, np.ndarray) or np.isscalar(x) or isinstance(x, (list, tuple)):
        a = np.ascontiguousarray(x, dtype=dtype)
        if shape is not None and a.shape != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
        return a.ctypes.data, MEM_HOST, a
    torch = _torch()
    if isinstance(x, torch.Tensor):
        tdt = {np.float64: torch.float64, np.float32: torch.float32, np.int32: torch.int32}[dtype]
        if x.dtype != tdt:
            raise TypeError(f"expected {tdt}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if shape is not None and tuple(x.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(x.shape)}")
        return x.data_ptr(), (MEM_DEVICE if x.is_cuda else MEM_HOST), x
    raise TypeError(f"unsupported argument type {type(x)}")


class Context:
    """A library context on one device, enqueuing on torch's current stream
    (or on a new torch stream when ``own_stream`` is set)."""

    def __init__(self, device: int = 0, own_stream: bool = False):
        self._lib = load()
        torch = _torch()
        # the library enqueues on torch's current stream (or a new torch
        # stream), so torch ops on the tensors it reads or writes are ordered
        # with its kernels; handle 0 is the null stream
        self._stream = torch.cuda.Stream(device) if own_stream else torch.cuda.current_stream(device)
        stream = self._stream.cuda_stream or None
        h = ctypes.c_void_p()
        st = self._lib.bioem_create(device, stream, ctypes.byref(h))
        if st != BIOEM_OK:
            raise BioemError(st, f"bioem_create(device={device}) failed")
        self.h = h
        self.device = device

    def check(self, st: int):
        if st != BIOEM_OK:
            raise BioemError(st, self._lib.bioem_last_error(self.h).decode())

    def set_timing(self, enable: bool = True):
        self.check(self._lib.bioem_set_timing(self.h, 1 if enable else 0))

    def kernel_time(self):
        """(ms, launches, evals) of the main kernel in the last logpost call."""
        ms, n, ev = ctypes.c_double(), ctypes.c_int32(), ctypes.c_double()
        self.check(self._lib.bioem_get_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n),
                                                   ctypes.byref(ev)))
        return ms.value, n.value, ev.value

    def set_autotune(self, enable: bool = True):
        self.check(self._lib.bioem_set_autotune(self.h, 1 if enable else 0))

    def tunings(self):
        """Tuned entries of this context as a list of dicts."""
        out = []
        for i in range(self._lib.bioem_tuning_count(self.h)):
            t = Tuning()
            self.check(self._lib.bioem_tuning_entry(self.h, i, ctypes.byref(t)))
            out.append({f: getattr(t, f) for f, _ in Tuning._fields_})
        return out

    def close(self):
        if getattr(self, "h", None):
            self._lib.bioem_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class _Handle:
    _free = None

    def __init__(self, lib, h):
        self._lib = lib
        self.h = h
        n, nx, ny = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        getattr(lib, self._info)(h, ctypes.byref(n), ctypes.byref(nx), ctypes.byref(ny))
        self.n, self.nx, self.ny = n.value, nx.value, ny.value

    def free(self):
        if self.h:
            getattr(self._lib, self._free)(self.h)
            self.h = None

    def __del__(self):
        self.free()


class Projections(_Handle):
    _free, _info = "bioem_free_proj", "bioem_proj_info"


class Images(_Handle):
    _free, _info = "bioem_free_imgs", "bioem_imgs_info"


def project(ctx: Context, spheres, quats, nx: int, ny: int, pixel_A: float) -> Projections:
    sp, m1, k1 = _arg(spheres, np.float64)
    qp, m2, k2 = _arg(quats, np.float64)
    if m1 != m2:
        raise ValueError("spheres and quats must both be host or both device")
    ns = (k1.shape[0] if hasattr(k1, "shape") else len(k1))
    nq = (k2.shape[0] if hasattr(k2, "shape") else len(k2))
    h = ctypes.c_void_p()
    ctx.check(ctx._lib.bioem_project(ctx.h, sp, ns, qp, nq, nx, ny, pixel_A, m1, ctypes.byref(h)))
    return Projections(ctx._lib, h)


def project_euler(ctx: Context, spheres, euler, nx: int, ny: int, pixel_A: float) -> Projections:
    """Projections for z-y-z Euler angles [nq][3] (radians) instead of quaternions."""
    sp, m1, k1 = _arg(spheres, np.float64)
    ep, m2, k2 = _arg(euler, np.float64)
    if m1 != m2:
        raise ValueError("spheres and euler must both be host or both device")
    if len(k2.shape) != 2 or k2.shape[1] != 3:
        raise ValueError("euler must be [nq][3]")
    h = ctypes.c_void_p()
    ctx.check(ctx._lib.bioem_project_euler(ctx.h, sp, int(k1.shape[0]), ep, int(k2.shape[0]), nx, ny, pixel_A, m1,
                                           ctypes.byref(h)))
    return Projections(ctx._lib, h)


def prepare_images(ctx: Context, images) -> Images:
    ip, m, keep = _arg(images, np.float32)
    ni, ny, nx = (int(s) for s in keep.shape)
    h = ctypes.c_void_p()
    ctx.check(ctx._lib.bioem_prepare_images(ctx.h, ip, ni, nx, ny, m, ctypes.byref(h)))
    return Images(ctx._lib, h)


def logpost(ctx: Context, proj: Projections, imgs: Images, ctf, max_shift: int,
            prec: str = "f32", cand_q=None, orient: bool = False, device_out: bool = False,
            kernel: int = 0, tile=None):
    """Returns dict(logp [ni], best (structured) [ni], orient [ni][nq] or None).

    With ``device_out`` the outputs are torch CUDA tensors (best as a raw
    byte tensor of ni records) and nothing is synchronised.  ``kernel`` and
    ``tile`` (images, slots) are bioem_opts.kernel / tile_images, tile_slots."""
    cp, cm, ck = _arg(ctf, np.float64)
    nc = int(ck.shape[0])
    ni, nq = imgs.n, proj.n
    o = Opts()
    o.prec = PREC[prec]
    o.kernel = int(kernel)
    if tile is not None:
        o.tile_images, o.tile_slots = int(tile[0]), int(tile[1])
    keep = []
    if cand_q is not None:
        qp, qm, qk = _arg(cand_q, np.int32)
        o.cand_q, o.k, o.cand_mem = qp, int(qk.shape[1]), qm
        keep.append(qk)
    if device_out:
        torch = _torch()
        dev = torch.device("cuda", ctx.device)
        logp = torch.empty(ni, dtype=torch.float64, device=dev)
        best = torch.empty(ni * ctypes.sizeof(Best), dtype=torch.uint8, device=dev)
        orient_t = torch.empty((ni, nq), dtype=torch.float64, device=dev) if orient else None
        o.out_mem = MEM_DEVICE
        o.logp_orient = orient_t.data_ptr() if orient else None
        ctx.check(ctx._lib.bioem_logpost(ctx.h, proj.h, imgs.h, cp, nc, cm, max_shift, ctypes.byref(o),
                                         logp.data_ptr(), best.data_ptr()))
        return {"logp": logp, "best": best, "orient": orient_t}
    logp = np.empty(ni, np.float64)
    best = np.empty(ni, BEST_DTYPE)
    orient_a = np.empty((ni, nq), np.float64) if orient else None
    o.out_mem = MEM_HOST
    o.logp_orient = orient_a.ctypes.data if orient else None
    ctx.check(ctx._lib.bioem_logpost(ctx.h, proj.h, imgs.h, cp, nc, cm, max_shift, ctypes.byref(o),
                                     logp.ctypes.data, best.ctypes.data))
    return {"logp": logp, "best": best, "orient": orient_a}


def logpost_noalloc(ctx: Context, proj: Projections, imgs: Images, ctf, max_shift: int, logp, best):
    """bioem_logpost_noalloc: plain F32 log posterior written into the
    caller's device tensors ``logp`` (float64 [ni]) and ``best`` (uint8
    [ni * record size]); ``ctf`` is a host array.  Nothing is synchronised."""
    ck = np.ascontiguousarray(ctf, dtype=np.float64)
    if ck.ndim != 2 or ck.shape[1] != 3:
        raise ValueError("ctf must be [nc][3]")
    lp = logp.data_ptr() if logp is not None else None
    bp = best.data_ptr() if best is not None else None
    ctx.check(ctx._lib.bioem_logpost_noalloc(ctx.h, proj.h, imgs.h, ck.ctypes.data, int(ck.shape[0]),
                                             int(max_shift), lp, bp))


def logpost_batch(ctx: Context, jobs, prec: str = "split_f16", mode: str = "persistent",
                  orient: bool = False, device_out: bool = False):
    """Score several jobs in one call.  ``jobs`` is a list of dicts with keys
    proj, imgs, ctf, max_shift and optionally cand_q.  Returns one dict per
    job, as ``logpost`` does."""
    arr = (Job * len(jobs))()
    keep, outs = [], []
    torch = _torch() if device_out else None
    for j, jb in enumerate(jobs):
        proj, imgs = jb["proj"], jb["imgs"]
        cp, cm, ck = _arg(jb["ctf"], np.float64)
        keep.append(ck)
        J = arr[j]
        J.proj, J.imgs, J.ctf, J.nc, J.ctf_mem, J.max_shift = proj.h, imgs.h, cp, int(ck.shape[0]), cm, \
            int(jb["max_shift"])
        if jb.get("cand_q") is not None:
            qp, qm, qk = _arg(jb["cand_q"], np.int32)
            J.cand_q, J.k, J.cand_mem = qp, int(qk.shape[1]), qm
            keep.append(qk)
        ni, nq = imgs.n, proj.n
        if device_out:
            dev = torch.device("cuda", ctx.device)
            o = {"logp": torch.empty(ni, dtype=torch.float64, device=dev),
                 "best": torch.empty(ni * ctypes.sizeof(Best), dtype=torch.uint8, device=dev),
                 "orient": torch.empty((ni, nq), dtype=torch.float64, device=dev) if orient else None}
            J.logp, J.best = o["logp"].data_ptr(), o["best"].data_ptr()
            J.logp_orient = o["orient"].data_ptr() if orient else None
        else:
            o = {"logp": np.empty(ni, np.float64), "best": np.empty(ni, BEST_DTYPE),
                 "orient": np.empty((ni, nq), np.float64) if orient else None}
            J.logp, J.best = o["logp"].ctypes.data, o["best"].ctypes.data
            J.logp_orient = o["orient"].ctypes.data if orient else None
        outs.append(o)
    m = {"persistent": BATCH_PERSISTENT, "per_job": BATCH_PER_JOB}[mode]
    ctx.check(ctx._lib.bioem_logpost_batch(ctx.h, arr, len(jobs), PREC[prec],
                                           MEM_DEVICE if device_out else MEM_HOST, m))
    return outs


def cnn_input(ctx: Context, imgs, device_out: bool = False):
    """Centred autocorrelation of each mean-free image (the network input)."""
    ip, m, keep = _arg(imgs, np.float32)
    B, ny, nx = (int(v) for v in keep.shape)
    if device_out:
        torch = _torch()
        out = torch.empty((B, ny, nx), dtype=torch.float32, device=torch.device("cuda", ctx.device))
        ctx.check(ctx._lib.bioem_cnn_input(ctx.h, ip, B, nx, ny, m, out.data_ptr(), MEM_DEVICE))
        return out
    out = np.empty((B, ny, nx), np.float32)
    ctx.check(ctx._lib.bioem_cnn_input(ctx.h, ip, B, nx, ny, m, out.ctypes.data, MEM_HOST))
    return out


def topk(ctx: Context, z, K: int, device_out: bool = False):
    """(idx [B][K] int32, mass [B] float32) of the K largest entries per row."""
    zp, m, keep = _arg(z, np.float32)
    B, n = (int(v) for v in keep.shape)
    if device_out:
        torch = _torch()
        dev = torch.device("cuda", ctx.device)
        idx = torch.empty((B, K), dtype=torch.int32, device=dev)
        mass = torch.empty(B, dtype=torch.float32, device=dev)
        ctx.check(ctx._lib.bioem_topk(ctx.h, zp, B, n, K, m, idx.data_ptr(), mass.data_ptr(), MEM_DEVICE))
        return idx, mass
    idx = np.empty((B, K), np.int32)
    mass = np.empty(B, np.float32)
    ctx.check(ctx._lib.bioem_topk(ctx.h, zp, B, n, K, m, idx.ctypes.data, mass.ctypes.data, MEM_HOST))
    return idx, mass


def logpost_crop(ctx: Context, proj: Projections, images, ctf, max_shift: int, device_out: bool = False,
                 psf_radius=None):
    """Log posterior per image with the real-space, border-cropping form of
    the displacement sum (direct correlation, max_shift <= 3); images are the
    raw pixels [ni][ny][nx] (numpy or CUDA tensor).  With ``psf_radius`` the
    calculated images come from the real-space PSF convolution of Eq. (5)
    (bioem_logpost_crop_psf)."""
    ip, im, keep = _arg(images, np.float32)
    if keep.ndim != 3 or tuple(keep.shape[1:]) != (proj.ny, proj.nx):
        raise ValueError(f"images must be [ni][{proj.ny}][{proj.nx}]")
    ni = int(keep.shape[0])
    cp, cm, ck = _arg(ctf, np.float64)
    if cm != im:
        raise ValueError("images and ctf must both be host arrays or both device tensors")
    nc = int(ck.shape[0])

    def call(lp, bp, mem):
        if psf_radius is None:
            return ctx._lib.bioem_logpost_crop(ctx.h, proj.h, ip, ni, im, cp, nc, int(max_shift), lp, bp, mem)
        return ctx._lib.bioem_logpost_crop_psf(ctx.h, proj.h, ip, ni, im, cp, nc, int(max_shift), int(psf_radius),
                                               lp, bp, mem)

    if device_out:
        torch = _torch()
        dev = torch.device("cuda", ctx.device)
        logp = torch.empty(ni, dtype=torch.float64, device=dev)
        best = torch.empty(ni * BEST_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        ctx.check(call(logp.data_ptr(), best.data_ptr(), MEM_DEVICE))
        return {"logp": logp, "best": best}
    logp = np.empty(ni, np.float64)
    best = np.empty(ni, BEST_DTYPE)
    ctx.check(call(logp.ctypes.data, best.ctypes.data, MEM_HOST))
    return {"logp": logp, "best": best}


def ensemble(ctx: Context, logp, w, device_out: bool = False):
    """(per_image [ni], total) of the ensemble posterior, Eq. (pb2): logp
    [nm][ni] per-model log posteriors (numpy or CUDA tensor), w [nm] weights."""
    lp, m, keep = _arg(logp, np.float64)
    if keep.ndim != 2:
        raise ValueError("logp must be [nm][ni]")
    nm, ni = (int(v) for v in keep.shape)
    wa = np.ascontiguousarray(w, dtype=np.float64)
    if wa.shape != (nm,):
        raise ValueError(f"expected {nm} weights, got shape {wa.shape}")
    if device_out:
        torch = _torch()
        dev = torch.device("cuda", ctx.device)
        per = torch.empty(ni, dtype=torch.float64, device=dev)
        tot = torch.empty(1, dtype=torch.float64, device=dev)
        ctx.check(ctx._lib.bioem_ensemble(ctx.h, lp, nm, ni, m, wa.ctypes.data, per.data_ptr(), tot.data_ptr(),
                                          MEM_DEVICE))
        return per, tot
    per = np.empty(ni, np.float64)
    tot = np.empty(1, np.float64)
    ctx.check(ctx._lib.bioem_ensemble(ctx.h, lp, nm, ni, m, wa.ctypes.data, per.ctypes.data, tot.ctypes.data,
                                      MEM_HOST))
    return per, float(tot[0])


class Net:
    """The orientation-proposal network of a context (see bioem_cnn_* in
    include/bioem.h).  Arrays are numpy (host) or torch CUDA tensors."""

    def __init__(self, ctx: Context, box: int, c1: int, c2: int, c3: int, c4: int, hidden: int, nq: int):
        self.ctx = ctx
        self.arch = CnnArch(box, c1, c2, c3, c4, hidden, nq, 0)
        h = ctypes.c_void_p()
        ctx.check(ctx._lib.bioem_cnn_create(ctx.h, ctypes.byref(self.arch), ctypes.byref(h)))
        self.h = h
        self.nparams = int(ctx._lib.bioem_cnn_num_params(h))
        self.box, self.nq = box, nq

    def set_params(self, params):
        p, m, keep = _arg(params, np.float32, (self.nparams,))
        self.ctx.check(self.ctx._lib.bioem_cnn_set_params(self.ctx.h, self.h, p, m))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparams, np.float32)
        self.ctx.check(self.ctx._lib.bioem_cnn_get_params(self.ctx.h, self.h, out.ctypes.data, MEM_HOST))
        return out

    def forward(self, imgs) -> np.ndarray:
        ip, m, keep = _arg(imgs, np.float32)
        B = int(keep.shape[0])
        out = np.empty((B, self.nq), np.float32)
        self.ctx.check(self.ctx._lib.bioem_cnn_forward(self.ctx.h, self.h, ip, B, m, out.ctypes.data, MEM_HOST))
        return out

    def backward(self, imgs, tidx, tp, want_grad: bool = False):
        """(loss, gradient or None) of one batch; the gradient stays in the
        network for ``adam``."""
        ip, m, keep = _arg(imgs, np.float32)
        B = int(keep.shape[0])
        qi, m2, k2 = _arg(tidx, np.int32)
        qp, m3, k3 = _arg(tp, np.float32)
        if len({m, m2, m3}) != 1:
            raise ValueError("images and targets must all be host or all device")
        T = int(k2.shape[1])
        loss = ctypes.c_float()
        g = np.empty(self.nparams, np.float32) if want_grad else None
        self.ctx.check(self.ctx._lib.bioem_cnn_backward(
            self.ctx.h, self.h, ip, B, qi, qp, T, m, ctypes.byref(loss),
            g.ctypes.data if want_grad else None, MEM_HOST))
        return loss.value, g

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.ctx.check(self.ctx._lib.bioem_cnn_adam(self.ctx.h, self.h, lr, beta1, beta2, eps))

    def propose(self, imgs, K: int, device_out: bool = False):
        """(cand [B][K] int32, mass [B] float32)."""
        ip, m, keep = _arg(imgs, np.float32)
        B = int(keep.shape[0])
        if device_out:
            torch = _torch()
            dev = torch.device("cuda", self.ctx.device)
            cand = torch.empty((B, K), dtype=torch.int32, device=dev)
            mass = torch.empty(B, dtype=torch.float32, device=dev)
            self.ctx.check(self.ctx._lib.bioem_cnn_propose(self.ctx.h, self.h, ip, B, m, K, cand.data_ptr(),
                                                           mass.data_ptr(), MEM_DEVICE))
            return cand, mass
        cand = np.empty((B, K), np.int32)
        mass = np.empty(B, np.float32)
        self.ctx.check(self.ctx._lib.bioem_cnn_propose(self.ctx.h, self.h, ip, B, m, K, cand.ctypes.data,
                                                       mass.ctypes.data, MEM_HOST))
        return cand, mass

    def close(self):
        if getattr(self, "h", None):
            self.ctx._lib.bioem_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def best_from_bytes(t) -> np.ndarray:
    """Structured view of a device best-record tensor copied to the host."""
    return np.frombuffer(t.cpu().numpy().tobytes(), dtype=BEST_DTYPE)


def render(ctx: Context, proj: Projections, ctf, shifts, norm_offset=None, noise=None,
           snr: float = 1.0, device_out: bool = False):
    """Synthetic maps, one per projection; host numpy or device tensor output."""
    n = proj.n
    cp, m, k1 = _arg(ctf, np.float64, (n, 3))
    sp, m2, k2 = _arg(shifts, np.int32, (n, 2))
    npp, m3, k3 = _arg(norm_offset, np.float64, (n, 2))
    zp, m4, k4 = _arg(noise, np.float32, (n, proj.ny, proj.nx))
    kinds = {m, m2} | ({m3} if norm_offset is not None else set()) | ({m4} if noise is not None else set())
    if len(kinds) != 1:
        raise ValueError("all render inputs must be host or all device")
    if device_out:
        torch = _torch()
        out = torch.empty((n, proj.ny, proj.nx), dtype=torch.float32,
                          device=torch.device("cuda", ctx.device))
        ctx.check(ctx._lib.bioem_render(ctx.h, proj.h, cp, sp, npp, zp, snr, m, out.data_ptr(), MEM_DEVICE))
        return out
    out = np.empty((n, proj.ny, proj.nx), np.float32)
    ctx.check(ctx._lib.bioem_render(ctx.h, proj.h, cp, sp, npp, zp, snr, m, out.ctypes.data, MEM_HOST))
    return out


def ctf_from_physical(defocus_A: float, amp_contrast: float, bfactor_A2: float,
                      voltage_kV: float = 300.0) -> np.ndarray:
    out = (ctypes.c_double * 3)()
    st = load().bioem_ctf_from_physical(defocus_A, amp_contrast, bfactor_A2, voltage_kV, out)
    if st != BIOEM_OK:
        raise BioemError(st, "invalid CTF parameters")
    return np.array(list(out))
