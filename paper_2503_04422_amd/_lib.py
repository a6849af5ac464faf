"""ctypes view of libpdx.so (the C ABI declared in include/pdx.h).

The library is loaded after torch so that both share one HIP runtime (the
same ``libamdhip64.so.7`` soname), which lets torch tensors and streams be
handed to the library directly.  There is no fallback: if the library is
missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdx.so")

PDX_OK = 0
PDX_EINVAL = -1
PDX_EWORKSPACE = -2
PDX_EHIP = -3
PDX_EUNSUPPORTED = -4
PDX_MAX_K = 64
PDX_MAX_RERANK = 8192
PDX_MAX_DIM = 4096
PDX_NOALLOC_SCRATCH_BYTES = 64 << 20

PDX_MODE_LINEAR = 0
PDX_MODE_BOND = 1

PDX_METRIC_L2 = 0
PDX_METRIC_L1 = 1
PDX_METRIC_IP = 2

PDX_ORDER_NATURAL = 0
PDX_ORDER_BOND = 1
PDX_ORDER_ZONES = 2

PDX_LAYOUT_NARY = 0
PDX_LAYOUT_PDX = 1

PDX_ROTATION_RANDOM = 0
PDX_ROTATION_PCA = 1

PDX_DTYPE_F32 = 0
PDX_DTYPE_BF16 = 1
PDX_DTYPE_FP8 = 2

PDX_LOSS_BCE = 0
PDX_LOSS_PINBALL = 1

MLP_IN = 72
MLP_PARAMS = 8960

c_void_p = ctypes.c_void_p
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_size_t = ctypes.c_size_t


class pdx_build_params(ctypes.Structure):
    _fields_ = [("group", c_int32), ("start_rows", c_int32)]


class pdx_search_params(ctypes.Structure):
    _fields_ = [("mode", c_int32), ("chunk", c_int32), ("tile_groups", c_int32),
                ("queries_per_block", c_int32), ("phase_events", c_void_p), ("counters", c_void_p),
                ("metric", c_int32), ("start_rows", c_int32), ("chunk_survivors", c_void_p),
                ("rounds", c_int32), ("dense_min", c_int32)]


class pdx_ivf_params(ctypes.Structure):
    _fields_ = [("kmeans_iters", c_int32), ("lowp_mask", c_int32), ("gaussian", c_void_p),
                ("init_rows", c_void_p), ("rotation", c_void_p), ("centroids", c_void_p),
                ("assign", c_void_p), ("rotation_kind", c_int32), ("pca_iters", c_int32)]


class pdx_ivf_search_params(ctypes.Structure):
    _fields_ = [("eps0", ctypes.c_float), ("delta_d", c_int32), ("dtype", c_int32),
                ("rerank", c_int32), ("phase_events", c_void_p), ("counters", c_void_p),
                ("mlp", c_void_p), ("mlp_threshold", ctypes.c_float), ("trace_features", c_void_p),
                ("trace_need", c_void_p), ("queries_per_wave", c_int32), ("bucket_order", c_int32),
                ("engine", c_int32), ("bucket_split", c_int32), ("bound", c_int32),
                ("prune_mlp", c_void_p), ("prune_scale", ctypes.c_float), ("prune_table", c_void_p),
                ("trace_prune_features", c_void_p), ("trace_prune_target", c_void_p),
                ("zone_rows", c_int32), ("bsa_m", ctypes.c_float), ("rerank_capacity", c_int32)]


class pdx_ivf_schedule(ctypes.Structure):
    _fields_ = [("engine", c_int32), ("queries_per_wave", c_int32), ("bucket_order", c_int32),
                ("delta_d", c_int32), ("ms", ctypes.c_float)]


TUNE_CANDIDATES = 14


class pdx_exact_schedule(ctypes.Structure):
    _fields_ = [("start_rows", c_int32), ("rounds", c_int32), ("dense_min", c_int32), ("ms", ctypes.c_float)]


EXACT_TUNE_CANDIDATES = 27

# name -> (restype, argtypes)
SIGNATURES = {
    "pdx_build_bytes": (c_size_t, [c_int64, c_int32, ctypes.POINTER(pdx_build_params)]),
    "pdx_build": (c_int32, [c_void_p, c_int64, c_int32, ctypes.POINTER(pdx_build_params), c_void_p,
                            c_size_t, c_void_p, ctypes.POINTER(c_void_p)]),
    "pdx_search_exact_workspace": (c_size_t, [c_void_p, c_int64, c_int32,
                                              ctypes.POINTER(pdx_search_params)]),
    "pdx_search_exact": (c_int32, [c_void_p, c_void_p, c_int64, c_int32,
                                   ctypes.POINTER(pdx_search_params), c_void_p, c_size_t,
                                   c_void_p, c_void_p, c_void_p]),
    "pdx_search_exact_noalloc": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, ctypes.POINTER(pdx_search_params),
                                           c_void_p, c_void_p, c_void_p]),
    "pdx_query_order_workspace": (c_size_t, [c_void_p, c_int64]),
    "pdx_query_order": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_size_t, c_void_p]),
    "pdx_ivf_build_bytes": (c_size_t, [c_int64, c_int32, c_int32, ctypes.POINTER(pdx_ivf_params)]),
    "pdx_ivf_build": (c_int32, [c_void_p, c_int64, c_int32, c_int32, ctypes.POINTER(pdx_ivf_params),
                                c_void_p, c_size_t, c_void_p, ctypes.POINTER(c_void_p)]),
    "pdx_ivf_export": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pdx_search_ivf_workspace": (c_size_t, [c_void_p, c_int64, c_int32, c_int32,
                                            ctypes.POINTER(pdx_ivf_search_params)]),
    "pdx_search_ivf": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32,
                                 ctypes.POINTER(pdx_ivf_search_params), c_void_p, c_size_t,
                                 c_void_p, c_void_p, c_void_p]),
    "pdx_exact_tune_workspace": (c_size_t, [c_void_p, c_int64, c_int32, ctypes.POINTER(pdx_search_params)]),
    "pdx_exact_tune": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, ctypes.POINTER(pdx_search_params), c_int32,
                                 ctypes.POINTER(pdx_exact_schedule), c_void_p, c_size_t, c_void_p]),
    "pdx_ivf_tune_workspace": (c_size_t, [c_void_p, c_int64, c_int32, c_int32,
                                          ctypes.POINTER(pdx_ivf_search_params)]),
    "pdx_ivf_tune": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32,
                               ctypes.POINTER(pdx_ivf_search_params), c_int32, c_int32,
                               ctypes.POINTER(pdx_ivf_schedule), c_void_p, c_size_t, c_void_p]),
    "pdx_mlp_bytes": (c_size_t, []),
    "pdx_mlp_workspace": (c_size_t, [c_int64]),
    "pdx_mlp_init": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "pdx_mlp_forward": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "pdx_mlp_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, ctypes.c_float, c_void_p,
                               c_size_t, c_void_p, c_void_p, c_void_p]),
    "pdx_mlp_export": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "pdx_mlp_train_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, ctypes.c_float,
                                     ctypes.c_float, c_int64, c_void_p, c_size_t, c_void_p, c_void_p]),
    "pdx_free": (None, [c_void_p]),
    "pdx_layout_blocks_bytes": (c_size_t, [c_int64, c_int32, c_int32]),
    "pdx_layout_blocks": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p]),
    "pdx_distances": (c_int32, [c_void_p, c_int32, c_int32, c_int64, c_int32, c_void_p, c_int64, c_int32,
                                c_void_p, c_void_p]),
    "pdx_last_error": (ctypes.c_char_p, []),
    "pdx_version": (ctypes.c_char_p, []),
}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libpdx.so is not built ({LIB_PATH}); run `python -m paper_2503_04422_amd.build` "
            "or __graft_entry__.build() -- there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class PdxError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.pdx_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != PDX_OK:
        raise PdxError(status, where)
