"""Oracle pins: quaternion QR (eq. (QQR)) and QSVD (eq. (qsvd)).

QR: Q^H Q = I, Q R = Y, R upper triangular with a real nonnegative diagonal,
and uniqueness (same factors from a second, different route: the complex QR
of the interleaved chi(Y), which is unique for a positive real diagonal).
QSVD: singular values against numpy's LAPACK SVD of chi(R) (each quaternion
singular value appears twice there), reconstruction and unitarity, also for
rank-deficient and repeated-singular-value inputs.
"""
import numpy as np
import pytest

import workloads as W
from tests import qref


@pytest.mark.parametrize("m,w", [(40, 12), (12, 12), (200, 35), (5, 1)])
def test_qr_invariants(oracle, m, w):
    Y = W.random_quat(m * 7 + w, m, w)
    Q, R = oracle.qr(Y)
    np.testing.assert_allclose(qref.mul(qref.adj(Q), Q), np.eye(w)[None] * np.array([1, 0, 0, 0])[:, None, None], atol=1e-13)
    np.testing.assert_allclose(qref.mul(Q, R), Y, atol=1e-12)
    for p in range(4):
        assert np.abs(np.tril(R[p], -1)).max() == 0.0
    assert np.all(R[0].diagonal() >= 0)
    assert np.abs(R[1:].diagonal(axis1=1, axis2=2)).max() == 0.0


def test_qr_unique_against_complex_qr(oracle):
    """Thin QR with a real positive diagonal is unique: compare with the QR of
    the interleaved complex adjoint (2x2 blocks), computed by LAPACK."""
    m, w = 30, 9
    Y = W.random_quat(77, m, w)
    Q, R = oracle.qr(Y)
    a, b = Y[0] + 1j * Y[1], Y[2] + 1j * Y[3]
    C = np.empty((2 * m, 2 * w), dtype=complex)
    C[0::2, 0::2], C[0::2, 1::2], C[1::2, 0::2], C[1::2, 1::2] = a, b, -np.conj(b), np.conj(a)
    Qc, Rc = np.linalg.qr(C)
    d = np.diag(Rc)
    Qc = Qc * (d / np.abs(d))[None, :]
    Qref = np.stack([Qc[0::2, 0::2].real, Qc[0::2, 0::2].imag, Qc[0::2, 1::2].real, Qc[0::2, 1::2].imag])
    np.testing.assert_allclose(Q, Qref, atol=1e-12)


def test_qr_rank_deficient_still_orthonormal(oracle):
    B = W.random_quat(1, 25, 3)
    C = W.random_quat(2, 3, 8)
    Y = qref.mul(B, C)                        # rank 3, width 8
    Q, R = oracle.qr(Y)
    np.testing.assert_allclose(qref.mul(qref.adj(Q), Q)[0], np.eye(8), atol=1e-12)
    np.testing.assert_allclose(qref.mul(Q, R), Y, atol=1e-12)


@pytest.mark.parametrize("w", [1, 2, 7, 20])
def test_qsvd_against_lapack(oracle, w):
    R = W.random_quat(100 + w, w, w)
    U, S, V = oracle.qsvd(R)
    ref = np.linalg.svd(qref.chi(R), compute_uv=False)
    np.testing.assert_allclose(S, ref[0::2], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ref[0::2], ref[1::2], rtol=1e-12)
    np.testing.assert_allclose(qref.reconstruct(U, S, V), R, atol=1e-12)
    eye = np.zeros((4, w, w)); eye[0] = np.eye(w)
    np.testing.assert_allclose(qref.mul(qref.adj(U), U), eye, atol=1e-12)
    np.testing.assert_allclose(qref.mul(qref.adj(V), V), eye, atol=1e-12)
    assert np.all(np.diff(S) <= 0)


def test_qsvd_repeated_singular_values(oracle):
    """sigma = (3, 2, 2, 2, 1): the chi pairs and the repeated quaternion values
    form a 6-fold complex cluster; vectors must still be quaternion-orthonormal."""
    rng = np.random.default_rng(5)
    Ua, Ub = W.haar_unitary(rng, 5)
    Va, Vb = W.haar_unitary(rng, 5)
    sig = np.array([3.0, 2.0, 2.0, 2.0, 1.0])
    a, b = W.from_svd(Ua, Ub, sig, Va, Vb)
    R = W.from_pair(a, b)
    U, S, V = oracle.qsvd(R)
    np.testing.assert_allclose(S, sig, rtol=1e-12)
    np.testing.assert_allclose(qref.reconstruct(U, S, V), R, atol=1e-12)
    eye = np.zeros((4, 5, 5)); eye[0] = np.eye(5)
    np.testing.assert_allclose(qref.mul(qref.adj(U), U), eye, atol=1e-10)
    np.testing.assert_allclose(qref.mul(qref.adj(V), V), eye, atol=1e-10)


def test_qsvd_rank_deficient(oracle):
    B = W.random_quat(8, 9, 2)
    C = W.random_quat(9, 2, 9)
    R = qref.mul(B, C)
    U, S, V = oracle.qsvd(R)
    np.testing.assert_allclose(S[:2], qref.qsv(R)[:2], rtol=1e-12)
    assert np.abs(S[2:]).max() < 1e-12 * S[0]
    np.testing.assert_allclose(qref.reconstruct(U, S, V), R, atol=1e-12)
    eye = np.zeros((4, 9, 9)); eye[0] = np.eye(9)
    np.testing.assert_allclose(qref.mul(qref.adj(U), U), eye, atol=1e-10)
    np.testing.assert_allclose(qref.mul(qref.adj(V), V), eye, atol=1e-10)


def test_qsvd_zero_matrix(oracle):
    U, S, V = oracle.qsvd(np.zeros((4, 4, 4)))
    assert np.all(S == 0)
    eye = np.zeros((4, 4, 4)); eye[0] = np.eye(4)
    np.testing.assert_allclose(qref.mul(qref.adj(U), U), eye, atol=1e-14)
    np.testing.assert_allclose(qref.mul(qref.adj(V), V), eye, atol=1e-14)
