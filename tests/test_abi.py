"""The C-ABI library loads and exports every entry point of include/pdx.h,
and its host-side argument checks answer without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdx.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"PDX_API\s+[\w\s\*]+?\b(pdx_\w+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for want in ("pdx_build", "pdx_search_exact", "pdx_ivf_build", "pdx_search_ivf"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2503_04422_amd import _lib
    for name in _declared():
        assert hasattr(_lib.lib, name), name
        assert name in _lib.SIGNATURES, name


def test_host_side_argument_errors():
    from paper_2503_04422_amd import _lib
    lib = _lib.lib
    h = ctypes.c_void_p()
    assert lib.pdx_build_bytes(0, 8, None) == 0
    assert lib.pdx_build_bytes(10, 0, None) == 0
    assert lib.pdx_build_bytes(10, _lib.PDX_MAX_DIM + 1, None) == 0
    assert lib.pdx_build_bytes(100, 16, None) >= 2 * 64 * 16 * 4
    assert lib.pdx_build(None, 10, 8, None, None, 0, None, ctypes.byref(h)) == _lib.PDX_EINVAL
    assert b"null" in lib.pdx_last_error()
    assert lib.pdx_build(ctypes.c_void_p(256), 0, 8, None, ctypes.c_void_p(256), 1 << 20, None,
                         ctypes.byref(h)) == _lib.PDX_EINVAL
    assert lib.pdx_search_exact(None, None, 1, 10, None, None, 0, None, None, None) == _lib.PDX_EINVAL
    assert lib.pdx_search_exact_workspace(None, 1, 10, None) == 0
    assert lib.pdx_exact_tune_workspace(None, 1, 10, None) == 0
    assert lib.pdx_exact_tune(None, None, 1, 10, None, 1, None, None, 0, None) == _lib.PDX_EINVAL
    assert lib.pdx_search_ivf(None, None, 1, 10, 1, None, None, 0, None, None, None) == _lib.PDX_EINVAL
    assert lib.pdx_query_order(None, None, 1, 1, None, None, None, None, 0, None) == _lib.PDX_EINVAL
    assert lib.pdx_query_order_workspace(None, 1) == 0
    bad_rot = _lib.pdx_ivf_params(0, 0, None, None, None, None, None, 7, 0)
    assert lib.pdx_ivf_build_bytes(64, 8, 2, ctypes.byref(bad_rot)) == 0
    pca = _lib.pdx_ivf_params(0, 0, None, None, None, None, None, _lib.PDX_ROTATION_PCA, 0)
    assert lib.pdx_ivf_build_bytes(64, 8, 2, ctypes.byref(pca)) > lib.pdx_ivf_build_bytes(64, 8, 2, None)
    assert lib.pdx_version().startswith(b"pdx ")


def test_network_loss_arguments_checked_on_the_host():
    from paper_2503_04422_amd import _lib
    lib = _lib.lib
    fake = ctypes.c_void_p(4096)  # never dereferenced: the arguments are rejected first
    for kind, w in ((7, 0.5), (_lib.PDX_LOSS_PINBALL, 0.0), (_lib.PDX_LOSS_PINBALL, 1.0),
                    (_lib.PDX_LOSS_BCE, -1.0), (_lib.PDX_LOSS_BCE, float("inf"))):
        assert lib.pdx_mlp_grad(fake, fake, fake, 4, kind, w, fake, 1 << 30, fake, None, None) == _lib.PDX_EINVAL
        assert lib.pdx_mlp_train_step(fake, fake, fake, 4, kind, w, 1e-3, 1, fake, 1 << 30, None,
                                      None) == _lib.PDX_EINVAL
    assert b"loss" in lib.pdx_last_error()


def test_distance_kernel_arguments_checked_on_the_host():
    """pdx_layout_blocks / pdx_distances: sizes, block, layout, metric and
    null pointers are rejected before any GPU call; nq = 0 is a no-op."""
    from paper_2503_04422_amd import _lib
    lib = _lib.lib
    assert lib.pdx_layout_blocks_bytes(100, 8, 64) == 2 * 64 * 8 * 4
    assert lib.pdx_layout_blocks_bytes(64, 3, 16) == 64 * 3 * 4
    assert lib.pdx_layout_blocks_bytes(1, 1, 512) == 512 * 4
    for n, d, b in ((0, 8, 64), (10, 0, 64), (10, 8, 48), (10, 8, 1024), (10, 8, 0)):
        assert lib.pdx_layout_blocks_bytes(n, d, b) == 0
    assert lib.pdx_layout_blocks(None, 10, 8, 48, None, None) == _lib.PDX_EINVAL
    assert b"block" in lib.pdx_last_error()
    assert lib.pdx_layout_blocks(None, 10, 8, 64, None, None) == _lib.PDX_EINVAL
    assert b"null" in lib.pdx_last_error()
    D = lib.pdx_distances
    P, N = _lib.PDX_LAYOUT_PDX, _lib.PDX_LAYOUT_NARY
    assert D(None, P, 64, 10, 8, None, 0, _lib.PDX_METRIC_L2, None, None) == _lib.PDX_OK
    assert D(None, P, 64, 10, 8, None, 1, _lib.PDX_METRIC_L2, None, None) == _lib.PDX_EINVAL
    assert b"null" in lib.pdx_last_error()
    assert D(None, 7, 64, 10, 8, None, 1, _lib.PDX_METRIC_L2, None, None) == _lib.PDX_EINVAL
    assert b"layout" in lib.pdx_last_error()
    assert D(None, P, 100, 10, 8, None, 1, _lib.PDX_METRIC_L2, None, None) == _lib.PDX_EINVAL
    assert b"block" in lib.pdx_last_error()
    assert D(None, N, 0, 10, 8, None, 1, 9, None, None) == _lib.PDX_EINVAL
    assert b"metric" in lib.pdx_last_error()
    for n, d, nq in ((0, 8, 1), (10, 0, 1), (10, 8, -1), (10, 8, 65536)):
        assert D(None, N, 0, n, d, None, nq, _lib.PDX_METRIC_L2, None, None) == _lib.PDX_EINVAL
    # misaligned row-major data (checked before any launch)
    assert D(ctypes.c_void_p(0x1004), N, 0, 10, 8, ctypes.c_void_p(0x2000), 1, _lib.PDX_METRIC_L2,
             ctypes.c_void_p(0x3000), None) == _lib.PDX_EINVAL
    assert b"aligned" in lib.pdx_last_error()
