"""MI355X-native parallel heat method for geodesic distance (arXiv 1812.06060).

The compute path is the HIP library ``libhgeo.so`` (C ABI in
``include/hgeo.h``); this package is its Python binding.  Build the library
with ``python -m paper_1812_06060_amd.build``.
"""
from ._hgeo import (  # noqa: F401
    EXPORTED,
    FORM_EDGE,
    FORM_FACE,
    HgeoError,
    Mesh,
    NotConverged,
    Opts,
    Server,
    default_opts,
    paper_opts,
    load_library,
    solve_batch,
)
