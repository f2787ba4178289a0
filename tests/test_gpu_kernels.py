"""GPU parity of the individual steps against the FP64 oracle, through the C ABI.

- sketch (Sec. 2, Gaussian quaternion matrix): bit-exact with the oracle's independent
  Philox + Box-Muller implementation;
- view products A B and A^H B (eq. (1), conjugate transpose): FP32 MFMA against the FP64
  oracle, error bounded by a multiple of u32 sqrt(K) times the sum of term magnitudes;
- thin QR (eq. (QQR)): unique for a positive real diagonal, so the CholeskyQR2 factors are
  compared with the oracle's Householder factors directly;
- small QSVD (eq. (qsvd)): singular values to 1e-12 against the oracle's complex-adjoint
  Jacobi, vectors through the reconstruction and unitarity.
"""
import numpy as np
import pytest

import workloads as W
from tests import qref

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def gq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_13731_amd import qlra as Q
    return Q


def dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("seed,n,l", [(0, 256, 15), (1, 2048, 60), (0xDEADBEEFCAFEF00D, 1537, 80), (7, 1, 1),
                                      (2 ** 32 + 5, 333, 17)])
def test_omega_bit_exact(gq, oracle, seed, n, l):
    print(f"omega seed={seed} n={n} l={l}", flush=True)
    got = host(gq.qlra_omega(seed, n, l))
    ref = oracle.omega(seed, n, l)
    assert got.dtype == np.float32
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def qgemm_bound(A, B, op):
    """Sum over the 16 plane products of |A_q| |B_r|: a bound on every output entry's sum of
    term magnitudes."""
    a = np.abs(A).sum(axis=0)
    b = np.abs(B).sum(axis=0)
    return (a @ b) if op == 0 else (a.T @ b)


@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("m,n,w", [(300, 257, 15), (1000, 700, 60), (130, 2050, 80), (64, 64, 1), (1, 37, 3),
                                   (513, 129, 160), (200, 300, 240)])
def test_qgemm_against_oracle(gq, oracle, op, m, n, w):
    print(f"qgemm op={op} m={m} n={n} w={w}", flush=True)
    rng = np.random.default_rng(m * 31 + n * 7 + w + op)
    A = rng.standard_normal((4, m, n)).astype(np.float32)
    B = rng.standard_normal((4, m if op else n, w)).astype(np.float32)
    got = host(gq.qlra_qgemm(op, dev(A), dev(B)))
    ref = oracle.qgemm(A.astype(np.float64), B.astype(np.float64)) if op == 0 else \
        oracle.qgemm_adj(A.astype(np.float64), B.astype(np.float64))
    K = n if op == 0 else m
    tol = 8 * U32 * np.sqrt(4 * K) * qgemm_bound(A.astype(np.float64), B.astype(np.float64), op) + 1e-30
    err = np.abs(got - ref)
    assert np.all(err <= tol[None]), float((err / tol[None]).max())


def test_qgemm_config1_view_sampled(gq, oracle):
    """Full 2048 x 2048, w = 60 (the benchmark's view shape, same launch configuration):
    every output entry of both views checked against the oracle on sampled rows."""
    A, _ = W.config1(noise_std=0.01)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((4, 2048, 60)).astype(np.float32)
    dA, dB = dev(A), dev(B)
    for op in (0, 1):
        got = host(gq.qlra_qgemm(op, dA, dB))
        rows = rng.choice(2048, 64, replace=False)
        A64, B64 = A.astype(np.float64), B.astype(np.float64)
        if op == 0:
            ref = oracle.qgemm(A64[:, rows, :], B64)
            bound = np.abs(A64[:, rows, :]).sum(0) @ np.abs(B64).sum(0)
        else:
            ref = oracle.qgemm_adj(A64[:, :, rows], B64)
            bound = np.abs(A64[:, :, rows]).sum(0).T @ np.abs(B64).sum(0)
        tol = 8 * U32 * np.sqrt(4 * 2048) * bound
        assert np.all(np.abs(got[:, rows, :] - ref) <= tol[None])


@pytest.mark.parametrize("m,w", [(37, 1), (500, 15), (333, 33), (2048, 60), (1001, 64), (64, 64), (1024, 80), (80, 80),
                                 (777, 96), (500, 97), (3000, 160), (2500, 200), (1500, 289)])
def test_cholqr_matches_householder(gq, oracle, m, w):
    print(f"cholqr m={m} w={w}", flush=True)
    rng = np.random.default_rng(m + w)
    Y = rng.standard_normal((4, m, w)).astype(np.float32)
    Qg, Rg = gq.qlra_cholqr(dev(Y))
    Qg, Rg = host(Qg), host(Rg)
    Qo, Ro = oracle.qr(Y.astype(np.float64))
    # orthonormal in FP32, and equal to the unique QR with positive real diagonal
    gram = qref.mul(qref.adj(Qg.astype(np.float64)), Qg.astype(np.float64))
    eye = np.zeros_like(gram); eye[0] = np.eye(w)
    assert np.abs(gram - eye).max() < 50 * U32 * np.sqrt(m)
    cond = np.linalg.cond(qref.chi(Y.astype(np.float64)))
    assert np.abs(Qg - Qo).max() < 50 * U32 * cond
    assert np.abs(Rg - Ro).max() < 50 * U32 * cond * np.abs(Ro).max()
    np.testing.assert_allclose(qref.mul(Qg.astype(np.float64), Rg), Y, atol=1e-4 * np.abs(Y).max())


def test_cholqr_many_tiles(gq):
    """A Gram of 544 columns (153 upper tiles of 32: K split eight ways, one split per XCD) and its
    blocked factorization (six diagonal blocks of 91: the inverse's last workgroup holds three
    columns).  The QR with positive real diagonal is unique, so an orthonormal Q (FP32 level), an
    upper triangular R with positive real diagonal and Q R = Y pin it (the oracle's QR of this
    size takes a minute on the host)."""
    m, w = 2048, 544
    print(f"cholqr m={m} w={w}", flush=True)
    rng = np.random.default_rng(m + w)
    Y = rng.standard_normal((4, m, w)).astype(np.float32)
    Qg, Rg = gq.qlra_cholqr(dev(Y))
    Qg, Rg = host(Qg).astype(np.float64), host(Rg)
    gram = qref.mul(qref.adj(Qg), Qg)
    eye = np.zeros_like(gram); eye[0] = np.eye(w)
    assert np.abs(gram - eye).max() < 50 * U32 * np.sqrt(m)
    low = np.tril(np.ones((w, w), dtype=bool), -1)
    assert np.all(Rg[:, low] == 0)
    assert np.all(np.diag(Rg[0]) > 0) and np.all(np.diagonal(Rg[1:], axis1=1, axis2=2) == 0)
    np.testing.assert_allclose(qref.mul(Qg, Rg), Y, atol=1e-4 * np.abs(Y).max())


@pytest.mark.parametrize("m,w", [(600, 20), (900, 130)])
def test_cholqr_rank_deficient_uses_shift(gq, oracle, m, w):
    """Exactly rank-deficient input: plain CholeskyQR breaks down; the shifted round and the
    rounds after it (gated on the shift flag) make Q orthonormal, and Q R = Y (w = 130: the
    blocked factorization's gated rerun)."""
    print(f"cholqr rank 5, m={m} w={w}", flush=True)
    B = W.random_quat(3, m, 5)
    C = W.random_quat(4, 5, w)
    Y = qref.mul(B, C).astype(np.float32)
    Qg, Rg, ws = gq.qlra_cholqr(dev(Y), return_workspace=True)
    Qg, Rg = host(Qg).astype(np.float64), host(Rg)
    gram = qref.mul(qref.adj(Qg), Qg)
    eye = np.zeros_like(gram); eye[0] = np.eye(w)
    assert np.abs(gram - eye).max() < 1e-6
    np.testing.assert_allclose(qref.mul(Qg, Rg), Y, atol=1e-4 * np.abs(Y).max())
    flags = host(ws[:64].view(dtype=__import__("torch").int32))
    assert flags[1] == 1          # the first round was shifted
    assert (flags[0] & 2) == 0    # and the factorization did not fail


@pytest.mark.parametrize("w", [1, 2, 15, 60, 64, 65, 81, 96, 97])
def test_qsvd_against_oracle(gq, oracle, w):
    print(f"qsvd w={w}", flush=True)
    R = W.random_quat(w + 1000, w, w)
    Uh, S, Vh = gq.qlra_qsvd(dev(R))
    Uh, S, Vh = host(Uh), host(S), host(Vh)
    _, So, _ = oracle.qsvd(R)
    np.testing.assert_allclose(S, So, rtol=1e-12, atol=1e-13 * So[0])
    np.testing.assert_allclose(qref.reconstruct(Uh, S, Vh), R, atol=1e-11 * So[0])
    eye = np.zeros((4, w, w)); eye[0] = np.eye(w)
    np.testing.assert_allclose(qref.mul(qref.adj(Uh), Uh), eye, atol=1e-11)
    np.testing.assert_allclose(qref.mul(qref.adj(Vh), Vh), eye, atol=1e-11)


def test_qsvd_block_diagonal(gq, oracle):
    """A block-diagonal R of order 130 (blocks of 70 and 60) through the large-order eigensolver:
    the Householder tridiagonalisation of its block-diagonal Gram keeps the blocks apart exactly,
    so the tridiagonal has an exact zero at the block boundary (a reflector of tau = 0, the
    phase chain restarting at 1, Sturm counts and twisted factorisations with b_j = 0)."""
    w, w1 = 130, 70
    print(f"qsvd block-diagonal w={w}", flush=True)
    R = np.zeros((4, w, w))
    R[:, :w1, :w1] = W.random_quat(7201, w1, w1)
    R[:, w1:, w1:] = W.random_quat(7202, w - w1, w - w1)
    Uh, S, Vh = gq.qlra_qsvd(dev(R))
    Uh, S, Vh = host(Uh), host(S), host(Vh)
    _, So, _ = oracle.qsvd(R)
    np.testing.assert_allclose(S, So, rtol=1e-12, atol=1e-13 * So[0])
    np.testing.assert_allclose(qref.reconstruct(Uh, S, Vh), R, atol=1e-11 * So[0])
    # eigenvectors of the Gram are orthogonal to about u64 lambda_max / (smallest gap of its
    # eigenvalues); here that is 4e-12
    lam = So ** 2
    tol = max(1e-11, 50 * 2.0 ** -52 * lam[0] / np.min(np.abs(np.diff(lam))))
    eye = np.zeros((4, w, w)); eye[0] = np.eye(w)
    np.testing.assert_allclose(qref.mul(qref.adj(Uh), Uh), eye, atol=tol)
    np.testing.assert_allclose(qref.mul(qref.adj(Vh), Vh), eye, atol=tol)


def test_qsvd_upper_triangular_graded(gq, oracle):
    """The solve feeds the QSVD upper triangular R factors with graded diagonals.  For
    w <= 96 the GPU takes the QSVD from the eigendecomposition of R^H R, whose eigenvalues
    carry an absolute error ~ eps sigma_1^2: sigma_j is then accurate to
    ~ eps sigma_1^2 / sigma_j, and to ~ sqrt(eps) sigma_1 for the tiniest ones."""
    w = 40
    R = W.random_quat(9, w, w)
    for p in range(4):
        R[p] = np.triu(R[p])
    R[1:, np.arange(w), np.arange(w)] = 0.0
    R[0, np.arange(w), np.arange(w)] = np.abs(R[0].diagonal()) * (0.7 ** np.arange(w))
    _, S, _ = gq.qlra_qsvd(dev(R), vectors=False)
    _, So, _ = oracle.qsvd(R)
    S = host(S)
    eps = 2.0 ** -52
    tol = 50 * eps * So[0] ** 2 / np.maximum(So, np.sqrt(eps) * So[0]) + 1e-12 * So
    assert np.all(np.abs(S - So) <= tol), float(np.max(np.abs(S - So) / tol))
    # the well-conditioned part is accurate to FP64 level
    big = So > 1e-3 * So[0]
    np.testing.assert_allclose(S[big], So[big], rtol=1e-10)
