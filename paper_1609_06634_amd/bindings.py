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
                ("logp_orient", ctypes.c_void_p), ("reserved", ctypes.c_int32 * 4)]


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
]


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libbioem.so once; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} not built: run paper_1609_06634_amd.build.build()")
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
    (or on a stream of its own when ``own_stream`` is set)."""

    def __init__(self, device: int = 0, own_stream: bool = False):
        self._lib = load()
        stream = None
        if not own_stream:
            torch = _torch()
            stream = torch.cuda.current_stream(device).cuda_stream
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


def prepare_images(ctx: Context, images) -> Images:
    ip, m, keep = _arg(images, np.float32)
    ni, ny, nx = (int(s) for s in keep.shape)
    h = ctypes.c_void_p()
    ctx.check(ctx._lib.bioem_prepare_images(ctx.h, ip, ni, nx, ny, m, ctypes.byref(h)))
    return Images(ctx._lib, h)


def logpost(ctx: Context, proj: Projections, imgs: Images, ctf, max_shift: int,
            prec: str = "f32", cand_q=None, orient: bool = False, device_out: bool = False):
    """Returns dict(logp [ni], best (structured) [ni], orient [ni][nq] or None).

    With ``device_out`` the outputs are torch CUDA tensors (best as a raw
    byte tensor of ni records) and nothing is synchronised."""
    cp, cm, ck = _arg(ctf, np.float64)
    nc = int(ck.shape[0])
    ni, nq = imgs.n, proj.n
    o = Opts()
    o.prec = PREC[prec]
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
