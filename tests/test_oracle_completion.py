"""Pins of the oracle's quaternion matrix completion (Sec. 7): the Gaussian smoothing against
scipy's filter, and the alternating updates recovering a planted low-rank matrix."""
import numpy as np
import pytest
from scipy import ndimage

import workloads as W


@pytest.mark.parametrize("sigma", [0.6, 1.0, 1.7])
def test_smoothing_is_scipys_gaussian_filter(oracle, sigma):
    X = np.random.default_rng(4).standard_normal((4, 23, 31))
    ref = np.stack([ndimage.gaussian_filter(X[p], sigma, mode="nearest", truncate=np.ceil(3 * sigma) / sigma)
                    for p in range(4)])
    assert np.abs(oracle.smooth(X, sigma) - ref).max() < 1e-13


def test_smoothing_keeps_constants(oracle):
    X = np.full((4, 9, 7), 2.5)
    assert np.abs(oracle.smooth(X, 0.6) - 2.5).max() < 1e-14
    assert np.array_equal(oracle.smooth(X, 0.0), X)


def test_completion_recovers_a_planted_low_rank_matrix(oracle):
    """Rank 5, 60 % of the entries observed, rank-5 approximations with 4 passes: the misfit on
    the observed entries falls and the whole matrix is recovered."""
    M = W.planted(5, 80, 70, 5)
    mask = (np.random.default_rng(1).random((80, 70)) < 0.6).astype(np.uint8)
    X, fit = oracle.complete(M, mask, 5, 5, 4, 0, 1, 30, 0.0)
    assert fit[-1] < 1e-3 * fit[0]
    assert np.sqrt(np.sum((X - M) ** 2) / np.sum(M ** 2)) < 1e-3


def test_completion_with_everything_observed_is_one_approximation(oracle):
    """mask = 1: C stays M, so every iteration returns the rank-R approximation of M."""
    M = W.random_quat(3, 40, 30)
    mask = np.ones((40, 30), dtype=np.uint8)
    X, fit = oracle.complete(M, mask, 6, 4, 3, 1, 2, 3, 0.0)
    U, S, V, _ = oracle.qlra(M, 6, 4, 3, 1, 2)
    assert np.abs(X - oracle.reconstruct(U, S, V)).max() < 1e-12
    assert np.allclose(fit, fit[0])


def test_completion_on_the_adjoint_completes_the_adjoint(oracle):
    """Running each rank-R step on C^H (and exchanging the factors) is the completion of M^H with
    the mask transposed, transposed back."""
    M = W.planted(6, 30, 44, 3)
    mask = (np.random.default_rng(2).random((30, 44)) < 0.5).astype(np.uint8)
    X, fit = oracle.complete(M, mask, 3, 3, 3, 0, 4, 4, 0.6, adjoint=True)
    Mh = M.transpose(0, 2, 1).copy()
    Mh[1:] *= -1
    Xh, fith = oracle.complete(Mh, mask.T, 3, 3, 3, 0, 4, 4, 0.6)
    Xb = Xh.transpose(0, 2, 1).copy()
    Xb[1:] *= -1
    assert np.abs(X - Xb).max() < 1e-12
    assert np.allclose(fit, fith, rtol=1e-12)
