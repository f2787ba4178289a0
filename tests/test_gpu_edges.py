"""Edge cases of the method on the GPU against the FP64 oracle (same seeded inputs, same sketch):

- k above the numerical rank of A (planted rank r < k): the returned U and V still have
  orthonormal columns (the factor Y E S^{-1} of the final QSVD is completed where S_j is at the
  rounding level, as the oracle's QSVD completes its basis), and U diag(S) V^H matches the
  oracle's to the FP32 tolerance;
- a full-rank, fast-decaying spectrum sigma_i = 10^(-i/3): the views are ill-conditioned (for
  l = 28 near the FP32 floor of A); approximations, estimates and orthonormality match;
- a first view whose Gram is numerically singular (condition near 1e9); a view of exact rank
  below l reports the breakdown;
- non-finite input (one NaN or one Inf entry): the status word reports QLRA_E_NUMERIC;
- ragged shapes on a spectrum with gaps (sigma_i = 1 / i), compared element by element: the
  singular values, the factors themselves (canonical phases), U diag(S) V^H and the estimates;
- per-pass estimates of views wider than the single-workgroup eigensolver (l = 97, 160) beside
  l = 96, on a slowly decaying spectrum;
- the orthogonality gate of the second CholeskyQR round, in both branches.
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


def run_gpu(gq, A32, k, p, v, scheme, seed, **kw):
    import torch
    U, S, V, e, ws = gq.qlra(torch.from_numpy(np.ascontiguousarray(A32)).cuda(), k, p, v, scheme, seed, **kw)
    st = gq.qlra_status(ws)
    torch.cuda.synchronize()
    return U.cpu().numpy().astype(np.float64), S.cpu().numpy(), V.cpu().numpy().astype(np.float64), \
        e.cpu().numpy(), st


def orth_err(X):
    g = qref.mul(qref.adj(X), X)
    g[0] -= np.eye(X.shape[2])
    return float(np.abs(g).max())


def ahat_rel(A, r1, r2):
    from oracle import oracle as O
    return qref.fro(O.reconstruct(*r1) - O.reconstruct(*r2)) / qref.fro(A)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("v", [2, 3, 4])
@pytest.mark.parametrize("m,n,r,k,p", [(300, 200, 6, 10, 4), (150, 260, 3, 40, 8), (2048, 128, 20, 64, 16)])
def test_k_above_rank(gq, oracle, scheme, v, m, n, r, k, p):
    print(f"k above rank: {m} x {n} rank {r}, k={k} p={p} v={v} scheme={scheme}", flush=True)
    A = W.planted(m + n + r, m, n, r).astype(np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A, k, p, v, scheme, 5)
    assert st == gq.QLRA_OK
    A64 = A.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A64, k, p, v, scheme, 5)
    assert orth_err(Ug) <= 1e-5 and orth_err(Vg) <= 1e-5
    assert ahat_rel(A64, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    np.testing.assert_allclose(Sg[:r], So[:r], rtol=1e-5)
    assert np.all(Sg[r:] <= 1e-5 * Sg[0])
    assert np.all(np.abs(eg[1:] ** 2 - eo[1:] ** 2) <= 16 * U32)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("k,p,v", [(10, 5, 3), (10, 5, 4), (20, 8, 3), (20, 8, 6)])
def test_fast_decay(gq, oracle, scheme, k, p, v):
    m, n = 400, 300
    print(f"fast decay {m} x {n} k={k} p={p} v={v} scheme={scheme}", flush=True)
    sigma = 10.0 ** (-np.arange(1, n + 1) / 3.0)
    A = np.ascontiguousarray(W.spectrum_matrix(61, m, n, sigma, nrefl=4), dtype=np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A, k, p, v, scheme, 7)
    assert st == gq.QLRA_OK
    A64 = A.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A64, k, p, v, scheme, 7)
    assert orth_err(Ug) <= 1e-5 and orth_err(Vg) <= 1e-5
    d = ahat_rel(A64, (Ug, Sg, Vg), (Uo, So, Vo))
    print(f"  ahat diff {d:.3e}", flush=True)
    assert d <= 1e-5
    # singular values: FP32 views give each an absolute error of a few u32 sigma_1
    assert np.all(np.abs(Sg - So) <= 1e-5 * So + 64 * U32 * So[0])
    # e^2 = 1 - sum S_j^2 / ||A||^2 resolves to a few units of FP32 roundoff
    assert np.isnan(eg[0]) and np.all(np.abs(eg[1:] ** 2 - eo[1:] ** 2) <= 16 * U32)


def test_ill_conditioned_first_view(gq, oracle):
    """Five rows of ordinary size and twenty rows scaled by 1e-9 (zero elsewhere): A Omega has a
    condition number near 1e9 and its FP64 Gram is numerically singular (whether the first
    CholeskyQR round breaks down and takes the shifted path, int 1 of the workspace, depends on
    the rounding; the shifted path itself is pinned by the CholeskyQR kernel test on an exactly
    rank-deficient block).  The solve ends without a breakdown, with orthonormal factors (k = 10
    above the numerical rank: completed) and the oracle's approximation."""
    import torch
    A = np.zeros((4, 400, 300), dtype=np.float32)
    A[:, :5, :] = W.random_quat(71, 5, 300)
    A[:, 5:25, :] = 1e-9 * W.random_quat(72, 20, 300)
    A64 = A.astype(np.float64)
    for scheme in (0, 1):
        print(f"shifted first view scheme={scheme}", flush=True)
        U, S, V, e, ws = gq.qlra(torch.from_numpy(A).cuda(), 10, 6, 2, scheme, 7)
        assert gq.qlra_status(ws) == gq.QLRA_OK
        flags = ws[:64].view(torch.int32).cpu().numpy()
        print(f"  first view shifted: {flags[1]}", flush=True)
        Ug, Sg, Vg = (x.cpu().numpy().astype(np.float64) for x in (U, S, V))
        assert orth_err(Ug) <= 1e-5 and orth_err(Vg) <= 1e-5
        Uo, So, Vo, _ = oracle.qlra(A64, 10, 6, 2, scheme, 7)
        assert ahat_rel(A64, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
        np.testing.assert_allclose(Sg[:5], So[:5], rtol=1e-5)


def test_exactly_rank_deficient_view_reports_breakdown(gq):
    """A zero outside a 5 x 5 block: A Omega has 5 nonzero rows, so no CholeskyQR round (shifted
    or not) can give it l = 16 orthonormal columns; the solve reports QLRA_E_NUMERIC, as for the
    zero matrix (the oracle's Householder QR completes such a basis with arbitrary columns)."""
    import torch
    A = np.zeros((4, 400, 300), dtype=np.float32)
    A[:, 100:105, 40:45] = W.random_quat(71, 5, 5)
    U, S, V, e, ws = gq.qlra(torch.from_numpy(A).cuda(), 10, 6, 2, 0, 7)
    assert gq.qlra_status(ws) == gq.QLRA_E_NUMERIC


@pytest.mark.parametrize("scheme,v,prec", [(0, 3, 0), (1, 4, 0), (0, 4, 1), (1, 2, 0)])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_input(gq, scheme, v, prec, bad):
    import torch
    print(f"non-finite {bad} scheme={scheme} v={v} prec={prec}", flush=True)
    A = W.random_quat(5, 120, 90).astype(np.float32)
    A[2, 17, 33] = bad
    U, S, V, e, ws = gq.qlra(torch.from_numpy(A).cuda(), 8, 4, v, scheme, 1, precision=prec)
    assert gq.qlra_status(ws) == gq.QLRA_E_NUMERIC


@pytest.mark.parametrize("m,n,k,p,v,scheme", [
    (97, 61, 5, 0, 2, 0), (61, 97, 7, 3, 3, 1), (130, 40, 30, 10, 2, 0), (33, 40, 4, 4, 6, 1),
    (300, 17, 10, 7, 4, 1), (50, 40, 1, 0, 2, 0), (1, 7, 1, 0, 2, 0), (9, 1, 1, 0, 3, 1), (1, 1, 1, 0, 2, 0),
    (64, 64, 1, 0, 5, 1), (333, 211, 9, 6, 5, 0), (211, 333, 9, 6, 4, 1)])
def test_ragged_gapped_elementwise(gq, oracle, m, n, k, p, v, scheme):
    print(f"ragged gapped {m} x {n} k={k} p={p} v={v} scheme={scheme}", flush=True)
    sigma = 1.0 / np.arange(1, min(m, n) + 1)
    A = np.ascontiguousarray(W.spectrum_matrix(m * 7 + n, m, n, sigma, nrefl=4), dtype=np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A, k, p, v, scheme, 9)
    assert st == gq.QLRA_OK
    A64 = A.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A64, k, p, v, scheme, 9)
    np.testing.assert_allclose(Sg, So, rtol=1e-5)
    # gaps of at least S_k / (k + 1): an FP32 perturbation of the views moves the j-th pair by
    # about u32 S_0 / gap_j, well below 1e-4 for k <= 30
    assert np.abs(Ug - Uo).max() <= 1e-4
    assert np.abs(Vg - Vo).max() <= 1e-4
    assert ahat_rel(A64, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    assert np.isnan(eg[0]) and np.all(np.abs(eg[1:] ** 2 - eo[1:] ** 2) <= 16 * U32)


@pytest.mark.parametrize("k,p", [(80, 16), (81, 16), (128, 32)])
def test_wide_view_estimates(gq, oracle, k, p):
    """Per-pass estimates of views of width l = 96 (the single-workgroup eigensolver), 97 and 160
    (the large-order solver's batched values-only path), subspace scheme with a budget of 6, on a
    slowly decaying spectrum (sigma_i = i^-1/2, reflector-product unitaries, 1024 x 768); the
    budgets 3 .. 5 end with the final QSVD on the same views, whose last estimate is the error
    of the returned factors.  Estimate bound as at full size: 4 (i - 1) u32 sqrt(n) on e_i^2
    (measured here: below 1e-7)."""
    m, n = 1024, 768
    print(f"wide estimates {m} x {n} k={k} p={p}", flush=True)
    sigma = np.arange(1, n + 1) ** -0.5
    A = W.reflector_spectrum_matrix(4, m, n, sigma)
    Uo, So, Vo, eo = oracle.qlra(A.astype(np.float64), k, p, 6, 0, 11)
    tol = 4 * np.arange(1, 6) * U32 * np.sqrt(n)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A, k, p, 6, 0, 11)
    assert st == gq.QLRA_OK
    assert np.isnan(eg[0]) and np.all(np.abs(eg[1:] ** 2 - eo[1:] ** 2) <= tol)
    for v in (3, 4, 5):
        _, _, _, ev, st = run_gpu(gq, A, k, p, v, 0, 11)
        assert st == gq.QLRA_OK
        assert abs(ev[-1] ** 2 - eo[v - 1] ** 2) <= tol[v - 2]


@pytest.mark.parametrize("w", [60, 160])
def test_cholqr_orthogonality_gate(gq, w):
    """Without R the second CholeskyQR round runs only when the first left max |Q^H Q - I| above
    1e-7: skipped for a well-conditioned Y, taken for cond(Y) ~ 1e6 (one round in FP64 leaves an
    error up to about u64 cond^2), Q orthonormal and Q R = Y either way (w = 160: the blocked
    factorization, whose second round goes through a copy; Q aliases Y there, as in the Krylov
    stack)."""
    import torch
    m = 2048
    for sv, want in ((np.ones(w), 0), (np.logspace(0, -6, w), 1)):
        # singular values sv between reflector-product unitaries (column scaling alone would not
        # do: CholeskyQR is invariant to it)
        Ys = np.ascontiguousarray(W.spectrum_matrix(3, m, w, sv, nrefl=4), dtype=np.float32)
        Y = torch.from_numpy(Ys).cuda()
        Q, R, ws = gq.qlra_cholqr(Y, Q=Y if w > 96 else None, return_workspace=True, want_r=False)
        assert R is None
        torch.cuda.synchronize()
        flags = ws[:64].view(torch.int32).cpu().numpy()
        assert flags[3] == want, (flags[:5], want)
        if w > 96:
            assert flags[4] == 1 - want, flags[:5]
        Qh = Q.cpu().numpy().astype(np.float64)
        assert orth_err(Qh) <= 2e-6
        # the same range: Q Q^H Y = Y
        Y64 = Ys.astype(np.float64)
        P = qref.mul(Qh, qref.mul(qref.adj(Qh), Y64))
        assert np.abs(P - Y64).max() <= 1e-5 * np.abs(Y64).max()
