"""The PCA rotation of the IVF build (BSA's projection, Section 2.3) on the
GPU, checked against the FP64 oracle (oracle.rotation.pca_rotation, pinned
by a hand-worked case and numpy's SVD), through the C ABI.

What is unique is checked: the rotation is orthogonal; it diagonalises the
covariance (R C R^T off its diagonal is at the float32 rounding level);
every leading block of m rows captures the variance of the m largest
eigenvalues (the Ky Fan maximum, which only the top-m eigenspace reaches);
the rows come by non-increasing variance; where eigenvalues are well
separated the leading rows are the eigenvectors themselves.  Any orthogonal rotation preserves
distances, so the searches on a PCA index stay exact where they were:
ADSampling with eps0 = inf and PDX-BOND over all buckets return the exact
k-NN of the original rows.  Two builds give the same rotation bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import exact, rotation
from tests.parity import check_knn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_04422_amd as pdx  # fails loudly if libpdx.so is missing
    return pdx


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pca_index(pdx, x, nlist, seed=1, iters=0):
    rng = np.random.default_rng(seed)
    init = rng.choice(x.shape[0], nlist, replace=False).astype(np.int64)
    return pdx.pdx_ivf_build(_dev(x), nlist, None, _dev(init), kmeans_iters=4, rotation_kind="pca", pca_iters=iters)


def _spread_rows(n, d, seed):
    """Gaussian rows with eigenvalues 2^(-i/4) in a random basis, offset by
    a non-zero mean (the covariance must be centred)."""
    rng = np.random.default_rng(seed)
    basis = rotation.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    s = 2.0 ** (-np.arange(d) / 8.0)
    return (rng.standard_normal((n, d)) * s[None, :] @ basis.T + 5.0).astype(np.float32)


def _check_rotation(r, x, lead_aligned, tol=1e-5):
    """tol (of lambda_0): the float32 rounding of the covariance and of a
    d-term row product, about d 2^-24 (8e-6 at d = 130)."""
    ro, lam = rotation.pca_rotation(x)
    d = x.shape[1]
    r = r.astype(np.float64)
    assert np.max(np.abs(r @ r.T - np.eye(d))) <= 2e-6
    cov = rotation.covariance(x)
    rcr = r @ cov @ r.T
    off = np.max(np.abs(rcr - np.diag(np.diag(rcr))))
    assert off <= tol * lam[0], off / lam[0]
    rho = np.diag(rcr)  # variance along each row
    assert np.all(np.diff(rho) <= tol * lam[0]), "rows not by non-increasing variance"
    short = np.cumsum(lam) - np.cumsum(rho)
    assert np.all(short <= tol * lam[0]), np.max(short) / lam[0]
    if lead_aligned:
        align = np.abs(np.sum(r[:lead_aligned] * ro[:lead_aligned], axis=1))
        assert np.all(align >= 1.0 - 1e-4), align


def test_pca_rotation_separated_spectrum(pdx):
    import torch
    x = _spread_rows(8192, 64, seed=3)
    print("pca separated spectrum 8192 x 64", flush=True)
    ix = _pca_index(pdx, x, 8)
    r = pdx.pdx_ivf_export(ix)[0].cpu().numpy()
    torch.cuda.synchronize()
    _check_rotation(r, x, lead_aligned=16)
    # a second build gives the same bits
    r2 = pdx.pdx_ivf_export(_pca_index(pdx, x, 8))[0].cpu().numpy()
    assert np.array_equal(r.view(np.int32), r2.view(np.int32))


@pytest.mark.parametrize("d", [96, 130])
def test_pca_rotation_skewed_mixture(pdx, d):
    """The exact search's workload shape (skewed Gaussian mixture) at small
    D, ragged against the 64-wide covariance tiles at D = 130."""
    mix = synth.skewed_mixture(d, 16, 32.0, 4.0, 5)
    x = mix.data(20_000)
    print(f"pca skewed mixture 20000 x {d}", flush=True)
    r = pdx.pdx_ivf_export(_pca_index(pdx, x, 16))[0].cpu().numpy()
    _check_rotation(r, x, lead_aligned=0)


@pytest.mark.parametrize("bound", ["ads", "bond"])
def test_pca_index_search_stays_exact(pdx, bound):
    """eps0 = inf (ADSampling) or PDX-BOND over every bucket of a PCA index:
    the exact k-NN of the original rows (distances are preserved by any
    orthogonal rotation), under the tie rule."""
    import torch
    mix = synth.skewed_mixture(96, 16, 32.0, 4.0, 6)
    x = mix.data(12_000)
    q = mix.queries(24, 77)
    nlist = 12
    ix = _pca_index(pdx, x, nlist)
    print(f"pca index search bound={bound}", flush=True)
    ids, dist = pdx.pdx_search_ivf(ix, _dev(q), 10, nlist, eps0=float("inf"), bound=bound)
    torch.cuda.synchronize()
    wi, wd = exact.knn_exact(x, q, 10)
    check_knn(x, q, ids.cpu().numpy(), dist.cpu().numpy(), wi, wd)


def test_pca_argument_errors(pdx):
    with pytest.raises(ValueError):
        pdx.pdx_ivf_build(_dev(np.zeros((64, 8), np.float32)), 2, None, _dev(np.arange(2, dtype=np.int64)),
                          rotation_kind="svd")
