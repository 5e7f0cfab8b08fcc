"""Host-only checks of the C ABI: the library loads and exports every symbol
include/bioem.h declares, and the entry points that need no device behave."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1609_06634_amd as P
from workloads import ctf_abA_from_physical

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "bioem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bioem_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        P.build_library()
    return P.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in P.bindings.SIGNATURES}
    assert set(names) == bound


def test_version(lib):
    assert "gfx950" in P.version()


def test_ctf_conversion_matches_input_recipe(lib):
    for df, amp, bf, kv in [(5000.0, 0.1, 25.0, 300.0), (3.5e4, 0.0, 100.0, 200.0)]:
        np.testing.assert_allclose(P.ctf_from_physical(df, amp, bf, kv),
                                   ctf_abA_from_physical(df, amp, bf, kv), rtol=1e-13)
    with pytest.raises(P.BioemError):
        P.ctf_from_physical(5000.0, 1.5, 0.0)


def test_struct_layouts(lib):
    assert ctypes.sizeof(P.bindings.Best) == 32
    assert P.BEST_DTYPE.itemsize == 32
    assert ctypes.sizeof(P.bindings.Opts) == 48
    assert ctypes.sizeof(P.bindings.Job) == 80
    assert ctypes.sizeof(P.bindings.Tuning) == 48
    assert ctypes.sizeof(P.bindings.CnnArch) == 32


def test_null_context_calls(lib):
    assert lib.bioem_set_autotune(None, 1) == P.bindings.BIOEM_EINVAL
    assert lib.bioem_tuning_count(None) == 0
    assert lib.bioem_logpost_batch(None, None, 0, 2, 0, 0) == P.bindings.BIOEM_EINVAL
    assert lib.bioem_cnn_create(None, None, None) == P.bindings.BIOEM_EINVAL
    assert lib.bioem_cnn_num_params(None) == 0
    assert lib.bioem_ensemble(None, None, 1, 0, 0, None, None, None, 0) == P.bindings.BIOEM_EINVAL
    assert lib.bioem_logpost_crop(None, None, None, 1, 0, None, 1, 0, None, None, 0) == P.bindings.BIOEM_EINVAL
    assert lib.bioem_project_euler(None, None, 1, None, 1, 64, 64, 1.0, 0, None) == P.bindings.BIOEM_EINVAL
    assert lib.bioem_logpost_noalloc(None, None, None, None, 1, 0, None, None) == P.bindings.BIOEM_EINVAL


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.bioem_create(0, None, ctypes.byref(h)) == P.bindings.BIOEM_EDEVICE
    assert not h.value
    assert lib.bioem_last_error(None) == b"null context"
