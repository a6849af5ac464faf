"""Random orthogonal rotation and PCA rotation -- oracle (test
infrastructure).

Section 2.3 (ADSampling) and Section 7: the collection and the queries are
transformed by one random orthogonal matrix, which preserves Euclidean
distances.  The paper does not say how the matrix is drawn; the reading
used here is the standard Haar construction: QR-factorise a matrix of iid
standard normal entries (drawn by the caller and passed in) and flip the
sign of every column of Q whose diagonal entry of R is negative.  A
vector v is rotated as R v (rows: X R^T).

Section 2.3 (BSA): a PCA projection of the collection in place of the
random one.  Its rows are the eigenvectors of the rows' covariance
(1/n) sum (x - mean)(x - mean)^T, largest eigenvalue first; each row's sign
is fixed so that its largest-magnitude entry (the first of equal ones) is
positive.  Parity unpinned for the GPU's rows themselves where eigenvalues
are (nearly) equal: any orthonormal basis of such an eigenspace is a
correct answer, so the GPU is checked by what is unique (orthogonality,
the variance each leading block of rows captures, the order by variance).
"""
from __future__ import annotations

import numpy as np


def orthogonal_from_gaussian(g: np.ndarray) -> np.ndarray:
    """Q diag(sign(diag(R))) from the QR factorisation of ``g`` (float64)."""
    g = np.asarray(g, dtype=np.float64)
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def rotate_rows(x: np.ndarray, rot: np.ndarray) -> np.ndarray:
    """Rows of x rotated: X R^T, in float64."""
    return np.asarray(x, dtype=np.float64) @ np.asarray(rot, dtype=np.float64).T


def householder_qr(g: np.ndarray):
    """A plain Householder QR (textbook form), float64: returns (Q, R) with
    Q orthogonal and R upper triangular, g = Q R.  Used to pin the library
    QR above by an independent construction."""
    a = np.array(g, dtype=np.float64)
    m = a.shape[0]
    qacc = np.eye(m)
    for j in range(m - 1):
        col = a[j:, j]
        alpha = -np.copysign(np.linalg.norm(col), col[0] if col[0] != 0 else 1.0)
        v = col.copy()
        v[0] -= alpha
        vn = np.linalg.norm(v)
        if vn == 0:
            continue
        v /= vn
        a[j:, :] -= 2.0 * np.outer(v, v @ a[j:, :])
        qacc[:, j:] -= 2.0 * np.outer(qacc[:, j:] @ v, v)
    return qacc, np.triu(a)


def pca_rotation(x: np.ndarray):
    """(R, eigenvalues): the rows' principal directions as the rows of R,
    by non-increasing eigenvalue of the float64 covariance (population
    form, 1/n), each row signed so its largest-magnitude entry is positive."""
    x = np.asarray(x, dtype=np.float64)
    xc = x - x.mean(axis=0)
    cov = xc.T @ xc / x.shape[0]
    lam, vec = np.linalg.eigh(cov)          # ascending
    order = np.argsort(-lam, kind="stable")
    lam, r = lam[order], vec[:, order].T    # rows = eigenvectors
    lead = np.argmax(np.abs(r), axis=1)
    sign = np.sign(r[np.arange(r.shape[0]), lead])
    sign[sign == 0] = 1.0
    return r * sign[:, None], lam


def covariance(x: np.ndarray) -> np.ndarray:
    """Population covariance (1/n) of the rows, float64."""
    x = np.asarray(x, dtype=np.float64)
    xc = x - x.mean(axis=0)
    return xc.T @ xc / x.shape[0]
