"""MI355X (gfx950) per-view Gaussian rendering step of streamlined street-scene
reconstruction (S3R-GS, arXiv 2503.08217).

The computation lives in `libs3r.so` (HIP kernels behind the C ABI declared in
`include/s3r.h`); this package loads it with ctypes and manages device memory
with PyTorch.  Build the library with `python -m paper_2503_08217_amd.build`.
"""

from . import _abi  # noqa: F401
from ._abi import (  # noqa: F401
    S3R_LOD,
    S3R_PLAIN,
    S3R_TEMPORAL,
    S3R_VIS_FOLD,
    S3R_VIS_RESET,
    S3R_VIS_UPDATE,
    S3RError,
    load,
)


def __getattr__(name):
    # the torch-side renderer is imported lazily so that `import
    # paper_2503_08217_amd` stays cheap for tools that only need the ABI
    if name in ("Renderer", "RenderFn", "tile_layout"):
        from . import renderer

        return getattr(renderer, name)
    raise AttributeError(name)
