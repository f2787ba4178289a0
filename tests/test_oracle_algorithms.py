"""Oracle pins: Alg. 1-4 end to end (Sec. 3, Sec. 4, Sec. 5).

- planted rank (Sec. 8, Example "random quaternion matrices": A = B C) is
  recovered to 1e-12 for every pass budget and both schemes;
- Eckart-Young: the rank-k error is never below the optimum, which a full QSVD
  (LAPACK on chi) gives on tiny inputs, and large budgets reach it;
- the equivalences stated in the paper: Alg. 2 at v = 2q+2 is Alg. 1 (Sec. 3),
  Alg. 4 at v < 4 is Alg. 2 (Sec. 6), Alg. 4 at v = 2(q+1) is Alg. 3 (Sec. 5);
- the block-Krylov range inclusion (Sec. 5, Lemma "corrected block-Krylov
  bound"), deterministically for a shared sketch;
- the mean spectral error over seeds obeys Thm. (flex-Krylov) and
  eqs. (mn11)/(mn12), and falls as the budget grows;
- the per-pass error estimate equals the directly computed residual.
"""
import numpy as np
import pytest

import workloads as W
from tests import qref


def relerr(A, U, S, V):
    return qref.fro(qref.reconstruct(U, S, V) - A) / qref.fro(A)


def decaying(seed, m, n, sigma):
    rng = np.random.default_rng(seed)
    Ua, Ub = W.haar_unitary(rng, m)
    Va, Vb = W.haar_unitary(rng, n)
    r = min(m, n)
    a, b = W.from_svd(Ua[:, :r], Ub[:, :r], sigma[:r], Va[:, :r], Vb[:, :r])
    return W.from_pair(a, b)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("v", [2, 3, 4, 5, 6])
def test_planted_rank_exact(oracle, scheme, v):
    A = W.planted(11, 70, 50, 6)
    U, S, V, e = oracle.qlra(A, 6, 3, v, scheme, 5)
    assert relerr(A, U, S, V) <= 1e-12
    assert np.isnan(e[0]) and np.all(e[1:] <= 1e-6)


@pytest.mark.parametrize("scheme", [0, 1])
def test_eckart_young_and_optimum(oracle, scheme):
    m, n, k, p = 40, 32, 5, 3
    sigma = 0.8 ** np.arange(n)
    A = decaying(3, m, n, sigma)
    sv = qref.qsv(A)
    np.testing.assert_allclose(sv, sigma, rtol=1e-10)
    opt_f = np.sqrt(np.sum(sv[k:] ** 2)) / qref.fro(A)
    for v in (2, 3, 4, 8):
        U, S, V, _ = oracle.qlra(A, k, p, v, scheme, 1)
        resid = A - qref.reconstruct(U, S, V)
        assert qref.spec(resid) >= sv[k] * (1 - 1e-12)
        assert relerr(A, U, S, V) >= opt_f * (1 - 1e-12)
        # the returned singular values never exceed the true ones
        assert np.all(S <= sv[:k] * (1 + 1e-12))
    U, S, V, _ = oracle.qlra(A, k, p, 12, scheme, 1)
    assert relerr(A, U, S, V) <= opt_f * (1 + 1e-9)
    np.testing.assert_allclose(S, sv[:k], rtol=1e-9)


def test_alg2_even_is_alg1(oracle):
    A, _ = W.config0()
    for v in (2, 4, 6):
        r1 = oracle.qlra(A, 10, 5, v, 2, 0)
        r2 = oracle.qlra(A, 10, 5, v, 0, 0)
        for x, y in zip(r1, r2):
            np.testing.assert_allclose(x, y, atol=1e-12, equal_nan=True)


@pytest.mark.parametrize("v", [2, 3])
def test_alg4_short_budget_is_alg2(oracle, v):
    A, _ = W.config0()
    r4 = oracle.qlra(A, 10, 5, v, 1, 0)
    r2 = oracle.qlra(A, 10, 5, v, 0, 0)
    for x, y in zip(r4, r2):
        np.testing.assert_allclose(x, y, atol=1e-12, equal_nan=True)


def test_alg4_even_is_alg3(oracle):
    """Same range, different construction: unnormalised Krylov blocks (Alg. 3)
    vs orthonormalised ones (Alg. 4).  A moderately decaying spectrum keeps the
    unnormalised stack well conditioned enough to compare at 1e-9."""
    m, n, k, p = 60, 48, 6, 4
    A = decaying(4, m, n, 0.9 ** np.arange(n))
    r3 = oracle.qlra(A, k, p, 4, 3, 2)
    r4 = oracle.qlra(A, k, p, 4, 1, 2)
    np.testing.assert_allclose(qref.reconstruct(*r3[:3]), qref.reconstruct(*r4[:3]), atol=1e-9)
    np.testing.assert_allclose(r3[1], r4[1], rtol=1e-9)
    np.testing.assert_allclose(r3[0], r4[0], atol=1e-7)   # canonical phases make the factors comparable
    np.testing.assert_allclose(r3[2], r4[2], atol=1e-7)


@pytest.mark.parametrize("v", [4, 6])
def test_krylov_range_inclusion(oracle, v):
    """||X - Q Q^H X||_2 <= ||X - Q_pow Q_pow^H X||_2 for the same sketch, Q from
    Alg. 4 (even v) and Q_pow from the power scheme with the same v (Alg. 2)."""
    m, n, k, p = 50, 40, 4, 2
    A = decaying(6, m, n, 1.0 / np.arange(1, n + 1))
    rng = np.random.default_rng(0)
    Om = rng.standard_normal((4, n, k + p))
    *_, Q1k, _ = oracle.qlra_sketch(A, k, p, v, 1, Om, bases=True)
    *_, Q1p, _ = oracle.qlra_sketch(A, k, p, v, 0, Om, bases=True)
    ek = qref.spec(A - qref.mul(Q1k, qref.mul(qref.adj(Q1k), A)))
    ep = qref.spec(A - qref.mul(Q1p, qref.mul(qref.adj(Q1p), A)))
    assert ek <= ep * (1 + 1e-12)


def _projector_errors(oracle, A, k, p, v, scheme, seed):
    n = A.shape[2]
    Om = oracle.omega(seed, n, k + p).astype(np.float64)
    *_, Q1, Q2 = oracle.qlra_sketch(A, k, p, v, scheme, Om, bases=True)
    e1 = qref.spec(A - qref.mul(Q1, qref.mul(qref.adj(Q1), A)))          # ||X - Q1 Q1^H X||
    e2 = qref.spec(A - qref.mul(qref.mul(A, Q2), qref.adj(Q2)))          # ||X - X Q2 Q2^H||
    return e1, e2


@pytest.mark.parametrize("scheme", [0, 1])
def test_mean_error_bounds(oracle, scheme):
    """Averages over 12 seeds against Thm. (flex-Krylov) (alpha_v = v - 1 for
    the returned projector) and, for Alg. 2, against eqs. (mn11)/(mn12)
    (exponent v for the other side)."""
    m, n, k, p = 48, 36, 4, 3
    sigma = 1.0 / np.arange(1, n + 1)
    A = decaying(7, m, n, sigma)
    means = {}
    for v in (2, 3, 4, 5):
        errs = np.array([_projector_errors(oracle, A, k, p, v, scheme, s) for s in range(12)])
        m1, m2 = errs.mean(axis=0)
        ret, other = (m1, m2) if v % 2 == 0 else (m2, m1)
        assert ret <= qref.flex_bound(sigma, k, p, v - 1)
        if scheme == 0:
            assert other <= qref.flex_bound(sigma, k, p, v)
        means[v] = ret
    assert means[3] <= means[2] * 1.01 and means[5] <= means[4] * 1.01


def test_truncated_error_falls_with_budget(oracle):
    A, _ = W.config0()
    for scheme in (0, 1):
        errs = [np.mean([relerr(A, *oracle.qlra(A, 10, 5, v, scheme, s)[:3]) for s in range(3)]) for v in (2, 3, 4, 6)]
        assert all(b <= a * 1.01 for a, b in zip(errs, errs[1:])), errs


def test_pass_estimates_equal_residuals(oracle):
    """Alg. 2 runs the same first i views for every budget v >= i, so the
    estimate of view i in a v = 6 run must equal the direct residual of the
    i-view result."""
    A, _ = W.config0()
    *_, e6 = oracle.qlra(A, 10, 5, 6, 0, 0)
    assert np.isnan(e6[0])
    for i in range(2, 7):
        U, S, V, _ = oracle.qlra(A, 10, 5, i, 0, 0)
        assert abs(e6[i - 1] - relerr(A, U, S, V)) <= 1e-10 * relerr(A, U, S, V) + 1e-14


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("v", [2, 5, 6])
def test_last_estimate_is_final_residual(oracle, scheme, v):
    A, _ = W.config0()
    U, S, V, e = oracle.qlra(A, 10, 5, v, scheme, 0)
    assert abs(e[-1] - relerr(A, U, S, V)) <= 1e-9 * e[-1]


def test_config0_reference_numbers(oracle):
    """sigma_11 = 1/121 and the optimum rank-10 Frobenius error for sigma_i = i^-2."""
    A, sigma = W.config0()
    sv = qref.qsv(A)
    np.testing.assert_allclose(sv[:12], sigma[:12], rtol=1e-10)
    opt = np.sqrt(np.sum(sigma[10:] ** 2) / np.sum(sigma ** 2))
    U, S, V, e = oracle.qlra(A, 10, 5, 3, 0, 0)
    r = relerr(A, U, S, V)
    assert opt <= r <= qref.flex_bound(sigma, 10, 5, 2) * np.sqrt(10)


def test_argument_errors(oracle):
    A = np.zeros((4, 10, 8))
    for args in [(0, 2, 2, 0), (3, -1, 2, 0), (3, 2, 1, 0), (7, 2, 2, 0), (3, 2, 3, 2), (3, 2, 2, 9)]:
        with pytest.raises(ValueError):
            oracle.qlra(A, *args, 0)


@pytest.mark.parametrize("scheme,v", [(0, 2), (0, 3), (1, 4), (1, 5)])
def test_canonical_phase_convention(oracle, scheme, v):
    """The phase convention of the returned factors (a reading: the paper leaves the unit
    quaternion phase of each singular pair free): in every column of V the entry of largest
    modulus (lowest row on ties) is real and positive, and the same right factor is applied to
    the column of U, so that A v_j = u_j s_j still holds (a phase taken from U, a negative real
    entry, a left instead of a right multiplication or a phase applied to one side only all fail
    one of these checks)."""
    m, n, k = 60, 45, 6
    sigma = np.concatenate([2.0 ** -np.arange(k), np.zeros(n - k)])
    A = decaying(31, m, n, sigma)
    U, S, V, _ = oracle.qlra(A, k, 4, v, scheme, 3)
    mod = (V ** 2).sum(axis=0)
    for j in range(k):
        i = int(np.argmax(mod[:, j]))
        q = V[:, i, j]
        assert q[0] > 0.0 and np.abs(q[1:]).max() <= 1e-13 * q[0], (j, q)
    # A V = U diag(S) column by column (exact rank k: the factors are exact up to rounding)
    AV = qref.mul(A, V)
    np.testing.assert_allclose(AV, U * S[None, None, :], atol=1e-12)
    np.testing.assert_allclose(qref.mul(qref.adj(A), U), V * S[None, None, :], atol=1e-12)
