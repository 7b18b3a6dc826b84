"""Pins of the mini-batch k-means oracle (the QUANTIZE step of Alg. 1,
Sec. 3.6; Sculley's mini-batch algorithm) against facts fixed outside it:
a hand-worked example, the running-mean identity, a library nearest-point
search, the k = 1 closed form and recovery of well-separated clusters."""

import numpy as np
import pytest
from scipy.spatial.distance import cdist


def test_hand_worked_example(oracle):
    # points 0, 2, 10, 12, 11; centres seeded at pixels 0 and 2 (0 and 10);
    # one batch [2, 0, 12, 11] in that order: centre 0 takes 2 (v = 1: 2),
    # then 0 (v = 2: 0.5*2 + 0.5*0 = 1); centre 1 takes 12 (12), then 11
    # (0.5*12 + 0.5*11 = 11.5)
    img = np.array([[0, 2, 10, 12, 11]], np.float32)
    c = oracle.kmeans_minibatch(img, 2, init_idx=[0, 2], batches=[[1, 0, 3, 4]])
    assert c.ravel().tolist() == [1.0, 11.5]
    assert oracle.kmeans_labels(img, c).ravel().tolist() == [0, 0, 1, 1, 1]
    # out-of-range indices are skipped
    c2 = oracle.kmeans_minibatch(img, 2, init_idx=[0, 2],
                                 batches=[[1, -1, 0, 3, 99, 4]])
    assert np.array_equal(c, c2)


def test_one_pass_is_the_mean_of_the_assigned_points(oracle):
    rng = np.random.default_rng(5)
    img = rng.normal(size=(40, 30, 3)).astype(np.float32)
    x = img.reshape(-1, 3).astype(np.float64)
    k = 6
    init = rng.choice(x.shape[0], size=k, replace=False)
    batch = rng.permutation(x.shape[0])
    c = oracle.kmeans_minibatch(img, k, init_idx=init, batches=[batch])
    c0 = x[init]
    lab = np.argmin(cdist(x, c0, "sqeuclidean"), axis=1)
    for j in range(k):
        pts = x[lab == j]
        want = pts.mean(axis=0) if len(pts) else c0[j]
        np.testing.assert_allclose(c[j], want, rtol=1e-12, atol=1e-12)


def test_labels_are_the_library_nearest_centres(oracle):
    rng = np.random.default_rng(6)
    img = rng.normal(size=(50, 20, 2)).astype(np.float32)
    centers = rng.normal(size=(9, 2))
    got = oracle.kmeans_labels(img, centers).ravel()
    want = np.argmin(cdist(img.reshape(-1, 2).astype(np.float64), centers,
                           "sqeuclidean"), axis=1)
    assert np.array_equal(got, want)
    mask = (rng.random((50, 20)) < 0.5).astype(np.uint8)
    gm = oracle.kmeans_labels(img, centers, mask).ravel()
    assert np.all(gm[mask.ravel() == 0] == 0)
    assert np.array_equal(gm[mask.ravel() == 1], want[mask.ravel() == 1])


def test_single_centre_is_the_mean_of_all_samples(oracle):
    rng = np.random.default_rng(7)
    img = rng.uniform(0, 255, size=(32, 32)).astype(np.float32)
    batches = rng.integers(0, img.size, size=(5, 100))
    c = oracle.kmeans_minibatch(img, 1, init_idx=[3], batches=batches)
    want = img.reshape(-1)[batches.ravel()].astype(np.float64).mean()
    assert c[0, 0] == pytest.approx(want, rel=1e-12)
    assert np.all(oracle.kmeans_labels(img, c) == 0)


def test_separated_clusters_are_recovered(oracle):
    rng = np.random.default_rng(8)
    means = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 10.0]])
    comp = rng.integers(0, 3, size=600)
    pts = (means[comp] + rng.normal(scale=0.5, size=(600, 2))).astype(np.float32)
    img = pts.reshape(20, 30, 2)
    init = [int(np.flatnonzero(comp == j)[0]) for j in range(3)]
    batches = rng.integers(0, 600, size=(25, 100))
    c = oracle.kmeans_minibatch(img, 3, init_idx=init, batches=batches)
    np.testing.assert_allclose(c, means, atol=0.3)
    assert np.array_equal(oracle.kmeans_labels(img, c).ravel(), comp)
