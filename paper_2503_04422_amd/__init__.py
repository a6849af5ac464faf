"""PDX K-nearest-neighbour scan for AMD Instinct MI355X (gfx950).

The search itself lives in ``libpdx.so`` (HIP kernels behind the C ABI of
``include/pdx.h``); this package is its Python binding.  Importing the
binding requires the built library; there is no CPU fallback.
"""
from .api import (  # noqa: F401
    MlpState,
    PdxIndex,
    ivf_test_points,
    pdx_build,
    pdx_distances,
    pdx_exact_tune,
    pdx_ivf_build,
    pdx_ivf_export,
    pdx_ivf_tune,
    pdx_layout_blocks,
    pdx_query_order,
    pdx_search_exact,
    pdx_search_exact_workspace,
    pdx_search_ivf,
    pdx_search_ivf_workspace,
    pdx_version,
)
from . import learn  # noqa: F401,E402
