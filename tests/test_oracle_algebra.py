"""Oracle pins: quaternion algebra (Sec. 2, eq. (1)) and the view products.

The oracle's Hamilton-product loops are checked against facts fixed outside
it: the unit rules i^2 = j^2 = k^2 = ijk = -1 (Sec. 2) and the complex-adjoint
homomorphism chi(AB) = chi(A) chi(B), chi(A^H) = chi(A)^H computed with numpy
complex matmul.  A dropped term or a wrong sign in any of the 16 products
fails the homomorphism check.
"""
import numpy as np
import pytest

import workloads as W
from tests import qref


def unit(p):
    q = np.zeros((4, 1, 1))
    q[p, 0, 0] = 1.0
    return q


@pytest.mark.parametrize("a,b,expect,sign", [
    (1, 1, 0, -1), (2, 2, 0, -1), (3, 3, 0, -1),          # i^2 = j^2 = k^2 = -1
    (1, 2, 3, +1), (2, 1, 3, -1),                          # ij = k, ji = -k
    (2, 3, 1, +1), (3, 2, 1, -1),                          # jk = i, kj = -i
    (3, 1, 2, +1), (1, 3, 2, -1),                          # ki = j, ik = -j
])
def test_unit_rules(oracle, a, b, expect, sign):
    c = oracle.qgemm(unit(a), unit(b))
    ref = sign * unit(expect)
    np.testing.assert_array_equal(c, ref)


def test_ijk_is_minus_one(oracle):
    ij = oracle.qgemm(unit(1), unit(2))
    np.testing.assert_array_equal(oracle.qgemm(ij, unit(3)), -unit(0))


@pytest.mark.parametrize("m,n,w", [(7, 5, 3), (33, 17, 9), (1, 1, 1)])
def test_product_homomorphism(oracle, m, n, w):
    A = W.random_quat(10 + m, m, n)
    B = W.random_quat(20 + n, n, w)
    C = oracle.qgemm(A, B)
    ref = qref.chi(A) @ qref.chi(B)
    assert np.abs(qref.chi(C) - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("m,n,w", [(7, 5, 3), (33, 17, 9)])
def test_adjoint_product_homomorphism(oracle, m, n, w):
    A = W.random_quat(30 + m, m, n)
    B = W.random_quat(40 + n, m, w)
    C = oracle.qgemm_adj(A, B)
    ref = qref.chi(A).conj().T @ qref.chi(B)
    assert np.abs(qref.chi(C) - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_adjoint_is_product_with_conjugate_transpose(oracle):
    A = W.random_quat(3, 12, 8)
    B = W.random_quat(4, 12, 5)
    np.testing.assert_allclose(oracle.qgemm_adj(A, B), oracle.qgemm(qref.adj(A), B), atol=1e-13)


def test_product_is_associative_and_noncommutative(oracle):
    A = W.random_quat(5, 6, 6)
    B = W.random_quat(6, 6, 6)
    C = W.random_quat(7, 6, 6)
    np.testing.assert_allclose(oracle.qgemm(oracle.qgemm(A, B), C), oracle.qgemm(A, oracle.qgemm(B, C)), atol=1e-12)
    assert np.abs(oracle.qgemm(A, B) - oracle.qgemm(B, A)).max() > 1e-3


def test_empty_inner_dimension(oracle):
    A = np.zeros((4, 3, 0))
    B = np.zeros((4, 0, 2))
    np.testing.assert_array_equal(oracle.qgemm(A, B), np.zeros((4, 3, 2)))
