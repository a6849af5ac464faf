"""Pins for the layout, rotation and k-means oracles.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import kmeans, layout, rotation
from tests.conftest import golden


def test_pdx_layout_hand_example():
    g = golden("hand_layout.json")
    x = np.array(g["vectors"], dtype=np.float32)
    p = layout.to_pdx(x, g["group"])
    assert p.reshape(-1).tolist() == g["pdx_flat"]
    assert layout.column_means(x).tolist() == g["means"]


@pytest.mark.parametrize("n,d,grp", [(1, 1, 64), (63, 5, 64), (64, 3, 64), (130, 7, 32), (257, 2, 128)])
def test_pdx_round_trip(n, d, grp):
    x = np.random.default_rng(n).standard_normal((n, d)).astype(np.float32)
    p = layout.to_pdx(x, grp)
    assert p.shape == ((n + grp - 1) // grp, d, grp)
    assert np.array_equal(layout.from_pdx(p, n), x)
    tail = n % grp
    if tail:
        assert not p[-1, :, tail:].any()


@pytest.mark.parametrize("d", [2, 16, 96])
def test_rotation_orthogonal_and_distance_preserving(d):
    g = np.random.default_rng(d).standard_normal((d, d))
    r = rotation.orthogonal_from_gaussian(g)
    assert np.abs(r.T @ r - np.eye(d)).max() < 1e-12
    assert np.abs(r.astype(np.float32).astype(np.float64).T @ r.astype(np.float32) - np.eye(d)).max() < 1e-6
    x = np.random.default_rng(d + 1).standard_normal((20, d))
    xr = rotation.rotate_rows(x, r)
    d0 = ((x[:, None] - x[None]) ** 2).sum(-1)
    d1 = ((xr[:, None] - xr[None]) ** 2).sum(-1)
    np.testing.assert_allclose(d1, d0, rtol=1e-10, atol=1e-10)


def test_library_qr_matches_textbook_householder():
    g = np.random.default_rng(5).standard_normal((24, 24))
    qh, rh = rotation.householder_qr(g)
    s = np.sign(np.diag(rh))
    want = qh * s[None, :]
    np.testing.assert_allclose(rotation.orthogonal_from_gaussian(g), want, atol=1e-10)
    np.testing.assert_allclose(qh @ rh, g, atol=1e-10)


def test_kmeans_hand_example():
    g = golden("hand_kmeans.json")
    x = np.array(g["points"], dtype=np.float64)
    c, lab, obj = kmeans.lloyd(x, np.array(g["init_rows"]), g["iters"])
    np.testing.assert_allclose(c, g["centroids"], rtol=0, atol=1e-12)
    assert lab.tolist() == g["labels"]
    np.testing.assert_allclose(obj[:2], g["objective_first_two"], rtol=1e-12)


def test_kmeans_invariants():
    mix = synth.anisotropic_unit_mixture(32, 8, 3)
    x = mix.data(2000)
    init = np.random.default_rng(0).choice(2000, 20, replace=False)
    c, lab, obj = kmeans.lloyd(x, init, 60)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(obj, obj[1:]))
    assert obj[-1] == obj[-2]  # converged: the last update used these labels
    assert kmeans.check_nearest(x, c, lab) == 0
    lists = kmeans.lists_from_labels(lab, 20)
    allm = np.sort(np.concatenate(lists))
    assert np.array_equal(allm, np.arange(2000))
    for i, m in enumerate(lists):
        if m.size:
            np.testing.assert_allclose(x[m].astype(np.float64).mean(0), c[i], atol=1e-12)
    # a planted mistake (labels shifted by one bucket) is caught
    assert kmeans.check_nearest(x, c, (lab + 1) % 20) > 0


def test_pca_rotation_hand_worked():
    """Section 2.3 (BSA's PCA projection): hand-worked 2-D case."""
    from tests.conftest import golden
    g = golden("hand_pca.json")
    r, lam = rotation.pca_rotation(np.array(g["x"]))
    np.testing.assert_allclose(lam, g["eigenvalues"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(r, g["rotation"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(rotation.rotate_rows(np.array(g["x"]), r), g["rotated"], rtol=0, atol=1e-12)


def test_pca_rotation_against_svd_and_invariants():
    """The principal directions equal the right singular vectors of the
    centred rows (a library routine, up to sign) with eigenvalues s^2 / n;
    the rotation is orthogonal; the rotated covariance is diagonal with
    non-increasing variances; a planted ascending order is caught."""
    rng = np.random.default_rng(9)
    n, d = 3000, 24
    scale = np.linspace(3.0, 0.2, d)
    x = rng.standard_normal((n, d)) * scale[None, :] @ rotation.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    r, lam = rotation.pca_rotation(x)
    np.testing.assert_allclose(r @ r.T, np.eye(d), atol=1e-12)
    xc = x - x.mean(axis=0)
    _, s, vt = np.linalg.svd(xc, full_matrices=False)
    np.testing.assert_allclose(lam, s ** 2 / n, rtol=1e-10)
    np.testing.assert_allclose(np.abs(np.sum(r * vt, axis=1)), 1.0, atol=1e-9)  # same directions
    cr = rotation.covariance(rotation.rotate_rows(x, r))
    np.testing.assert_allclose(cr, np.diag(lam), atol=1e-9 * lam[0])
    assert np.all(np.diff(np.diag(cr)) <= 1e-9 * lam[0])
    planted = r[::-1]
    assert not np.all(np.diff(np.diag(rotation.covariance(rotation.rotate_rows(x, planted)))) <= 1e-9 * lam[0])


def test_mixture_labels_are_the_components_the_rows_came_from():
    """synth.Mixture.labels: with far-apart means and tiny spreads every row
    lies nearest the mean of its own component, across block boundaries."""
    import synth
    from synth.gen import Mixture
    rng = np.random.default_rng(3)
    means = (rng.standard_normal((12, 16)) * 100).astype(np.float32)
    mix = Mixture(means, np.full((12, 16), 0.01, np.float32), np.full(12, 1 / 12), 7)
    start, n = 60_000, 10_000  # spans a block boundary
    x = mix.data(n, start)
    lab = mix.labels(n, start)
    near = np.argmin(((x[:, None, :] - means[None]) ** 2).sum(-1), axis=1)
    assert np.array_equal(near, lab)
    assert np.array_equal(mix.labels(n // 2, start + n // 2), lab[n // 2:])
