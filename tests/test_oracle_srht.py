"""Pins of the oracle's structured (subsampled randomized Hadamard) sketch: the sampling is a
permutation, the columns are orthogonal when n is a power of two, the signs are balanced, and
A Omega equals the columns s_j of (A D) H computed with scipy's Hadamard matrix."""
import numpy as np
import pytest
from scipy.linalg import hadamard

import workloads as W


@pytest.mark.parametrize("n_pad", [1, 2, 8, 32, 512, 2048])
def test_sampling_is_a_permutation(oracle, n_pad):
    img = [oracle.srht_perm(9, x, n_pad) for x in range(n_pad)]
    assert sorted(img) == list(range(n_pad))


@pytest.mark.parametrize("n_pad", [16, 128])
def test_odd_bit_counts_walk_back_into_range(oracle, n_pad):
    # 16 = 2^4 (even), 128 = 2^7 (odd: the Feistel works on 8 bits and walks)
    img = [oracle.srht_perm(3, x, n_pad) for x in range(n_pad)]
    assert sorted(img) == list(range(n_pad))


def test_columns_orthogonal_for_power_of_two(oracle):
    n, l = 256, 40
    Om = oracle.omega_srht(5, n, l).astype(np.float64)
    G = Om[0].T @ Om[0]
    assert np.abs(G - (n / l) * np.eye(l)).max() < 1e-5 * n / l
    assert np.all(Om[1:] == 0)
    assert np.allclose(np.abs(Om[0]), np.float32(1 / np.sqrt(l)))


def test_signs_balanced(oracle):
    d = oracle.srht_signs(11, 4000)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 4 / np.sqrt(4000)


@pytest.mark.parametrize("m,n,l", [(20, 64, 10), (17, 50, 12)])
def test_product_is_the_subsampled_transform(oracle, m, n, l):
    """A Omega = ((A D) padded to n_pad columns) H, columns s_j, over sqrt(l)."""
    A = W.random_quat(m + n, m, n)
    n_pad = oracle.srht_pad(n)
    d = oracle.srht_signs(7, n)
    cols = [oracle.srht_perm(7, j, n_pad) for j in range(l)]
    AD = np.zeros((4, m, n_pad))
    AD[:, :, :n] = A * d[None, None, :]
    ref = (AD @ hadamard(n_pad).astype(np.float64))[:, :, cols] / np.sqrt(l)
    Om = oracle.omega_srht(7, n, l).astype(np.float64)
    got = oracle.qgemm(A, Om)
    # Omega holds the FP32 rounding of 1 / sqrt(l)
    assert np.abs(got - ref).max() < 1e-6 * np.abs(ref).max()
