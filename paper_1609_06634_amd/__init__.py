"""MI355X-native BioEM posterior engine (gfx950 HIP kernels behind a C ABI).

The computation lives in libbioem.so (include/bioem.h); this package only
builds it and marshals arguments to it.
"""
from .bindings import (  # noqa: F401
    Context, Projections, Images, BioemError, project, project_euler, prepare_images, logpost, render,
    ctf_from_physical, version, load, best_from_bytes, BEST_DTYPE, LIB_PATH, logpost_batch, Net, topk, cnn_input, ensemble, logpost_crop,
    logpost_noalloc,
)


def build_library(verbose: bool = False) -> str:
    """Compile libbioem.so for gfx950 in place (hipcc)."""
    from .build import build
    return build(verbose=verbose)
