"""End-to-end GPU parity of qlra() (Alg. 2 and Alg. 4) against the FP64 oracle on the
same seeded inputs and the same sketch seed.

Tolerance (FP32 path): ||A_gpu - A_oracle||_F / ||A||_F <= 1e-5 for the rank-k
approximation where the spectrum separates sigma_k from sigma_{k+1}; singular values to
FP32 level; the per-pass estimates agree with the oracle's.  For the noise-dominated
2048 x 2048 workload (noise std 0.01, so sigma_50 / sigma_51 of A is 1 + O(1e-3)) the rank-k
truncation is ill-conditioned; the errors are compared as well, and the 1e-5 bound still holds.
"""
import numpy as np
import pytest

import workloads as W
from tests import qref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_13731_amd import qlra as Q
    return Q


_CACHE = {}


def config1(noise_std=0.01):
    if noise_std not in _CACHE:
        _CACHE[noise_std] = W.config1(noise_std=noise_std)
    return _CACHE[noise_std]


def run_gpu(gq, A32, k, p, v, scheme, seed):
    import torch
    U, S, V, e, ws = gq.qlra(torch.from_numpy(np.ascontiguousarray(A32)).cuda(), k, p, v, scheme, seed)
    st = gq.qlra_status(ws)
    torch.cuda.synchronize()
    return U.cpu().numpy().astype(np.float64), S.cpu().numpy(), V.cpu().numpy().astype(np.float64), \
        e.cpu().numpy(), st


def ahat_diff(A, r1, r2):
    return qref.fro(oracle_reconstruct(*r1[:3]) - oracle_reconstruct(*r2[:3])) / qref.fro(A)


def oracle_reconstruct(U, S, V):
    from oracle import oracle as O
    return O.reconstruct(U, S, V)


@pytest.mark.parametrize("scheme", ["subspace", "block_krylov"])
@pytest.mark.parametrize("v", [2, 3, 4, 5, 6])
def test_config0_parity(gq, oracle, scheme, v):
    """256 x 256, sigma_i = i^-2, k = 10, p = 5 (v = 3 subspace is the paper-shaped config)."""
    print(f"config0 scheme={scheme} v={v}", flush=True)
    A, sigma = W.config0()
    A32 = A.astype(np.float32)
    sch = 0 if scheme == "subspace" else 1
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 10, 5, v, sch, 0)
    assert st == gq.QLRA_OK
    Uo, So, Vo, eo = oracle.qlra(A32.astype(np.float64), 10, 5, v, sch, 0)
    assert ahat_diff(A, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    np.testing.assert_allclose(Sg, So, rtol=2e-5)
    assert np.isnan(eg[0]) and np.isnan(eo[0])
    np.testing.assert_allclose(eg[1:], eo[1:], rtol=2e-3)
    # canonical phases make the factors themselves comparable (distinct sigma)
    assert np.abs(Ug - Uo).max() < 1e-3
    assert np.abs(Vg - Vo).max() < 1e-3
    # orthonormality of the returned factors
    for X in (Ug, Vg):
        g = qref.mul(qref.adj(X), X)
        assert np.abs(g[0] - np.eye(10)).max() < 1e-5 and np.abs(g[1:]).max() < 1e-5


@pytest.mark.parametrize("scheme", [0, 1])
def test_planted_rank(gq, oracle, scheme):
    """A = B C with rank 12 <= k: the GPU recovers A to FP32 accuracy for every budget."""
    A = W.planted(21, 700, 500, 12).astype(np.float32)
    for v in (2, 3, 5):
        print(f"planted scheme={scheme} v={v}", flush=True)
        Ug, Sg, Vg, eg, st = run_gpu(gq, A, 12, 8, v, scheme, 3)
        assert st == gq.QLRA_OK
        rel = qref.fro(oracle_reconstruct(Ug, Sg, Vg) - A) / qref.fro(A)
        assert rel < 1e-5
        assert np.all(eg[1:] < 1e-2)


@pytest.mark.parametrize("v", [2, 3, 4, 6])
def test_config1_parity(gq, oracle, v):
    """2048 x 2048, sigma_i = exp(-i/20) + noise (std 0.01 per real component), k = 50,
    p = 10: the benchmark workload.  The noise makes the rank-50 truncation ill-conditioned
    (sigma_50 and sigma_51 of R differ by ~1e-3 relative), so the comparison is made on the
    untruncated projection error, the singular values, and the estimates; the truncated
    approximations are compared with a tolerance scaled by the truncation gap."""
    print(f"config1 v={v}", flush=True)
    A, _ = config1()
    Ug, Sg, Vg, eg, st = run_gpu(gq, A, 50, 10, v, 0, 1)
    assert st == gq.QLRA_OK
    Uo, So, Vo, eo = oracle.qlra(A.astype(np.float64), 50, 10, v, 0, 1)
    np.testing.assert_allclose(Sg, So, rtol=2e-5)
    np.testing.assert_allclose(eg[1:], eo[1:], rtol=1e-4)
    err_g = qref.fro(oracle_reconstruct(Ug, Sg, Vg) - A) / qref.fro(A)
    err_o = qref.fro(oracle_reconstruct(Uo, So, Vo) - A) / qref.fro(A)
    assert abs(err_g / err_o - 1) < 1e-4
    # the specification's bound on the approximation itself holds here as well (measured
    # about 3e-7 at every budget)
    d = ahat_diff(A, (Ug, Sg, Vg), (Uo, So, Vo))
    print(f"  ahat diff {d:.3e}", flush=True)
    assert d <= 1e-5
    # S_49 / S_0 = 0.086 is above the re-orthonormalisation trigger (1/64): the factors come
    # straight from the Gram form, orthonormal to about u32 S_0 / S_49
    for X in (Ug, Vg):
        g = qref.mul(qref.adj(X), X)
        assert np.abs(g[0] - np.eye(50)).max() < 1e-5 and np.abs(g[1:]).max() < 1e-5


def test_config1_low_noise_ahat(gq, oracle):
    """Same construction with noise std 1e-4: the rank-50 approximation is well separated and
    the 1e-5 bound on ||A_gpu - A_oracle||_F / ||A||_F applies."""
    A, _ = config1(noise_std=1e-4)
    for v in (3, 4):
        print(f"config1-lownoise v={v}", flush=True)
        Ug, Sg, Vg, eg, st = run_gpu(gq, A, 50, 10, v, 0, 1)
        Uo, So, Vo, eo = oracle.qlra(A.astype(np.float64), 50, 10, v, 0, 1)
        assert ahat_diff(A, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5


def test_config2_krylov(gq, oracle):
    """Pure quaternion 1024 x 1536 smooth random field, block Krylov, k = 64, p = 16, v = 6."""
    A = W.config2()
    print("config2 krylov v=6", flush=True)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A, 64, 16, 6, 1, 2)
    assert st == gq.QLRA_OK
    Uo, So, Vo, eo = oracle.qlra(A.astype(np.float64), 64, 16, 6, 1, 2)
    # FP32 view products carry an absolute error ~ u32 sqrt(K) sigma_1; with entries in [0, 1]
    # sigma_1 ~ 1100 is a mean-field component far above the rest, so small singular values are
    # compared absolutely against sigma_1.
    np.testing.assert_allclose(Sg, So, rtol=1e-4, atol=4e-6 * So[0])
    # That absolute error (~1e-3) exceeds the gaps between neighbouring sigma_j near j = 64, so
    # the rank-64 truncation itself is not FP32-stable here; singular vectors are compared where
    # the spectrum separates them (relative gap > 5 %).
    # Perturbation bound: angle(u_j, u_j') <~ delta / gap_j with delta the absolute error above.
    gap = np.minimum(np.r_[np.inf, So[:-1] - So[1:]], np.r_[So[:-1] - So[1:], np.inf])
    sep = np.where(gap[:-1] / So[:-1] > 0.05)[0]
    assert len(sep) >= 10
    delta = 4e-6 * So[0]
    for j in sep:
        for X, Y in ((Ug, Uo), (Vg, Vo)):
            ip = qref.mul(qref.adj(X[:, :, j:j + 1]), Y[:, :, j:j + 1])[:, 0, 0]
            assert 1 - np.sqrt(np.sum(ip ** 2)) <= 0.5 * (3 * delta / gap[j]) ** 2 + 1e-6, j
    err_g = qref.fro(oracle_reconstruct(Ug, Sg, Vg) - A) / qref.fro(A)
    err_o = qref.fro(oracle_reconstruct(Uo, So, Vo) - A) / qref.fro(A)
    assert abs(err_g / err_o - 1) < 1e-3
    np.testing.assert_allclose(eg[1:], eo[1:], rtol=1e-3)


def test_ragged_and_degenerate_shapes(gq, oracle):
    """Tall and wide, sizes off every tile boundary, p = 0, k + p = min(m, n), rank 1 (k = 1,
    l = 1) including a single row, a single column and 1 x 1."""
    for (m, n, k, p, v, sch) in [(97, 61, 5, 0, 2, 0), (61, 97, 7, 3, 3, 1), (130, 40, 30, 10, 2, 0),
                                 (33, 40, 4, 4, 6, 1), (300, 17, 10, 7, 4, 1), (50, 40, 1, 0, 2, 0),
                                 (1, 7, 1, 0, 2, 0), (9, 1, 1, 0, 3, 1), (1, 1, 1, 0, 2, 0), (64, 64, 1, 0, 5, 1)]:
        print(f"ragged m={m} n={n} k={k} p={p} v={v} scheme={sch}", flush=True)
        A = W.random_quat(m + n, m, n).astype(np.float32)
        Ug, Sg, Vg, eg, st = run_gpu(gq, A, k, p, v, sch, 9)
        assert st == gq.QLRA_OK
        Uo, So, Vo, eo = oracle.qlra(A.astype(np.float64), k, p, v, sch, 9)
        np.testing.assert_allclose(Sg, So, rtol=1e-4)
        err_g = qref.fro(oracle_reconstruct(Ug, Sg, Vg) - A) / qref.fro(A)
        err_o = qref.fro(oracle_reconstruct(Uo, So, Vo) - A) / qref.fro(A)
        assert abs(err_g - err_o) < 1e-4


@pytest.mark.parametrize("v,scheme", [(2, 0), (4, 1)])
def test_zero_matrix_reports_breakdown(gq, v, scheme):
    """A = 0: every view is zero, the CholeskyQR cannot produce a basis, and the status word says
    QLRA_E_NUMERIC (the singular values come out zero, the factors are not valid)."""
    import torch
    print(f"zero matrix v={v} scheme={scheme}", flush=True)
    A = torch.zeros((4, 64, 48), device="cuda")
    U, S, V, e, ws = gq.qlra(A, 5, 3, v, scheme, 3)
    assert gq.qlra_status(ws) == gq.QLRA_E_NUMERIC
    assert np.all(S.cpu().numpy() == 0.0)


def test_argument_errors(gq):
    import torch
    A = torch.zeros((4, 10, 8), device="cuda")
    for (k, p, v) in [(0, 2, 2), (3, -1, 2), (3, 2, 1), (7, 2, 2)]:
        with pytest.raises(gq.QlraError) as ei:
            gq.qlra(A, k, p, v, 0, 0)
        assert ei.value.code == gq.QLRA_E_ARG
    # an unknown view precision
    with pytest.raises(gq.QlraError) as ei:
        gq.qlra(A, 3, 2, 2, 0, 0, precision=7)
    assert ei.value.code == gq.QLRA_E_UNSUPPORTED


@pytest.mark.parametrize("v", [4, 6])
def test_wide_krylov_final(gq, oracle, v):
    """Block Krylov with k = 40, p = 8: the final view stacks up to 3 blocks (144 columns), past
    the single-workgroup eigensolver; the wide one must agree with the oracle as well."""
    print(f"wide krylov v={v}", flush=True)
    A, _ = W.config0()
    A32 = A.astype(np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 40, 8, v, 1, 5)
    assert st == gq.QLRA_OK
    Uo, So, Vo, eo = oracle.qlra(A32.astype(np.float64), 40, 8, v, 1, 5)
    assert ahat_diff(A, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    np.testing.assert_allclose(Sg, So, rtol=1e-4, atol=1e-6 * So[0])
    # e^2 = 1 - sum sigma_j^2 / ||A||^2: FP32 rounding of the view outputs moves the sum of
    # squares by a few units of FP32 roundoff relative to ||A||^2, whatever the size of e
    assert np.all(np.abs(eg[1:] ** 2 - eo[1:] ** 2) <= 4 * 2.0 ** -24)


def test_wide_subspace_final(gq, oracle):
    """Subspace scheme with k + p = 108 columns (past the single-workgroup eigensolver) on a
    spectrum with a clear gap after sigma_100."""
    print("wide subspace", flush=True)
    m, n = 400, 360
    sigma = np.concatenate([np.linspace(1.0, 0.5, 100), 1e-3 / np.arange(1, n - 99)])
    A = W.spectrum_matrix(17, m, n, sigma, dtype=np.float64)
    A32 = np.ascontiguousarray(A, dtype=np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 100, 8, 3, 0, 9)
    assert st == gq.QLRA_OK
    A64 = A32.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A64, 100, 8, 3, 0, 9)
    assert ahat_diff(A64, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    np.testing.assert_allclose(Sg, So, rtol=1e-5)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("v", [3, 4])
def test_transpose_runs_the_scheme_on_the_adjoint(gq, oracle, scheme, v):
    """transpose = 1 applies the scheme to A^H (sketch m x l, first view A^H Omega): the result is
    the oracle's on A^H with the two factors exchanged, since A = (A^H)^H = V S U^H."""
    print(f"transpose scheme={scheme} v={v}", flush=True)
    import torch
    m, n = 200, 320
    sigma = np.arange(1, m + 1, dtype=np.float64) ** -2.0
    A32 = np.ascontiguousarray(W.spectrum_matrix(31, m, n, sigma, nrefl=4), dtype=np.float32)
    U, S, V, e, ws = gq.qlra(torch.from_numpy(A32).cuda(), 10, 5, v, scheme, 3, transpose=True)
    assert gq.qlra_status(ws) == gq.QLRA_OK
    torch.cuda.synchronize()
    Ug, Sg, Vg, eg = (x.cpu().numpy().astype(np.float64) for x in (U, S, V, e))
    assert Ug.shape == (4, m, 10) and Vg.shape == (4, n, 10)
    A64 = A32.astype(np.float64)
    Ub, Sb, Vb, eb = oracle.qlra(np.ascontiguousarray(qref.adj(A64)), 10, 5, v, scheme, 3)
    Uo, So, Vo = Vb, Sb, Ub                       # the factors of A
    assert ahat_diff(A64, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    np.testing.assert_allclose(Sg, So, rtol=2e-5)
    assert np.abs(Ug - Uo).max() < 1e-3 and np.abs(Vg - Vo).max() < 1e-3
    assert np.isnan(eg[0]) and np.all(np.abs(eg[1:] ** 2 - eb[1:] ** 2) <= 4 * 2.0 ** -24)


def test_classical_forms_are_budgets(gq):
    """Alg. 1 with q power iterations is the subspace scheme at 2 q + 2 passes, and Alg. 3 with q
    iterations is the block Krylov scheme at 2 q + 2 passes (the oracle pins both equivalences):
    the aliases give bitwise the same results as the budget calls."""
    import torch
    A = torch.from_numpy(W.random_quat(9, 300, 260).astype(np.float32)).cuda()
    for alias, scheme in ((gq.qlra_power_iteration, 0), (gq.qlra_block_krylov_q, 1)):
        r1 = alias(A, 12, 4, 1, 5)
        r2 = gq.qlra(A, 12, 4, 4, scheme, 5)
        torch.cuda.synchronize()
        for a, b in zip(r1[:4], r2[:4]):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy(), equal_nan=True)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("v", [2, 3, 4])
def test_real_sketch(gq, oracle, scheme, v):
    """The real Gaussian sketch (the real plane of the quaternion sketch, the other planes zero):
    the first view uses only the q = p terms of eq. (1); the result equals the oracle's with the
    same sketch."""
    print(f"real sketch scheme={scheme} v={v}", flush=True)
    import torch
    A, _ = W.config0()
    A32 = A.astype(np.float32)
    U, S, V, e, ws = gq.qlra(torch.from_numpy(A32).cuda(), 10, 5, v, scheme, 4, sketch=gq.QLRA_SKETCH_REAL)
    assert gq.qlra_status(ws) == gq.QLRA_OK
    torch.cuda.synchronize()
    Ug, Sg, Vg, eg = (x.cpu().numpy().astype(np.float64) for x in (U, S, V, e))
    Om = oracle.omega(4, 256, 15).astype(np.float64)
    Om[1:] = 0.0
    Uo, So, Vo, eo = oracle.qlra_sketch(A32.astype(np.float64), 10, 5, v, scheme, Om)
    assert ahat_diff(A, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    np.testing.assert_allclose(Sg, So, rtol=2e-5)
    assert np.abs(Ug - Uo).max() < 1e-3 and np.abs(Vg - Vo).max() < 1e-3
    assert np.isnan(eg[0]) and np.all(np.abs(eg[1:] ** 2 - eo[1:] ** 2) <= 4 * 2.0 ** -24)


def test_real_sketch_on_the_adjoint(gq, oracle):
    """Real sketch with transpose = 1: the first view is A^H Omega with a real Omega (m x l)."""
    import torch
    m, n = 200, 320
    sigma = np.arange(1, m + 1, dtype=np.float64) ** -2.0
    A32 = np.ascontiguousarray(W.spectrum_matrix(33, m, n, sigma, nrefl=4), dtype=np.float32)
    U, S, V, e, ws = gq.qlra(torch.from_numpy(A32).cuda(), 10, 5, 3, 0, 6, transpose=True,
                             sketch=gq.QLRA_SKETCH_REAL)
    assert gq.qlra_status(ws) == gq.QLRA_OK
    torch.cuda.synchronize()
    Ug, Sg, Vg = (x.cpu().numpy().astype(np.float64) for x in (U, S, V))
    Om = oracle.omega(6, m, 15).astype(np.float64)
    Om[1:] = 0.0
    A64 = A32.astype(np.float64)
    Ub, Sb, Vb, _ = oracle.qlra_sketch(np.ascontiguousarray(qref.adj(A64)), 10, 5, 3, 0, Om)
    assert ahat_diff(A64, (Ug, Sg, Vg), (Vb, Sb, Ub)) <= 1e-5
    np.testing.assert_allclose(Sg, Sb, rtol=2e-5)


@pytest.mark.parametrize("n,l", [(256, 15), (100, 12), (2048, 60), (3000, 40), (1, 1)])
def test_srht_sketch_bit_exact(gq, oracle, n, l):
    """The structured sketch on the device equals the oracle's bit for bit (n = 100 and 3000 pad
    to 2^7 and 2^12: the first needs the permutation's cycle walking)."""
    print(f"srht sketch n={n} l={l}", flush=True)
    got = gq.qlra_omega_srht(13, n, l).cpu().numpy()
    want = oracle.omega_srht(13, n, l)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("scheme,v", [(0, 2), (0, 3), (1, 4)])
def test_srht_sketch_solve(gq, oracle, scheme, v):
    """opts.sketch = QLRA_SKETCH_SRHT: the result equals the oracle's solve with the same sketch."""
    print(f"srht solve scheme={scheme} v={v}", flush=True)
    import torch
    A, _ = W.config0()
    A32 = A.astype(np.float32)
    U, S, V, e, ws = gq.qlra(torch.from_numpy(A32).cuda(), 10, 5, v, scheme, 8, sketch=gq.QLRA_SKETCH_SRHT)
    assert gq.qlra_status(ws) == gq.QLRA_OK
    torch.cuda.synchronize()
    Ug, Sg, Vg, eg = (x.cpu().numpy().astype(np.float64) for x in (U, S, V, e))
    Om = oracle.omega_srht(8, 256, 15).astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra_sketch(A32.astype(np.float64), 10, 5, v, scheme, Om)
    assert ahat_diff(A, (Ug, Sg, Vg), (Uo, So, Vo)) <= 1e-5
    np.testing.assert_allclose(Sg, So, rtol=2e-5)
    assert np.isnan(eg[0]) and np.all(np.abs(eg[1:] ** 2 - eo[1:] ** 2) <= 4 * 2.0 ** -24)


@pytest.mark.parametrize("m,n,transpose,prec", [(300, 200, False, 0), (200, 300, True, 0), (260, 180, False, 1)])
def test_srht_sketch_solve_shapes(gq, oracle, m, n, transpose, prec):
    """The structured sketch with n padded to a power of two, on A^H (an m x l sketch) and with
    BF16 views: the result equals the oracle's solve with the same sketch."""
    print(f"srht solve {m}x{n} transpose={transpose} prec={prec}", flush=True)
    import torch
    sigma = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -1.5
    A32 = np.ascontiguousarray(W.spectrum_matrix(44, m, n, sigma, nrefl=4), dtype=np.float32)
    v = 4 if prec else 3
    U, S, V, e, ws = gq.qlra(torch.from_numpy(A32).cuda(), 12, 4, v, 0, 21, transpose=transpose,
                             sketch=gq.QLRA_SKETCH_SRHT, precision=prec)
    assert gq.qlra_status(ws) == gq.QLRA_OK
    torch.cuda.synchronize()
    Ug, Sg, Vg = (x.cpu().numpy().astype(np.float64) for x in (U, S, V))
    A64 = A32.astype(np.float64)
    if transpose:
        Om = oracle.omega_srht(21, m, 16).astype(np.float64)
        Ub, Sb, Vb, _ = oracle.qlra_sketch(np.ascontiguousarray(qref.adj(A64)), 12, 4, v, 0, Om)
        Uo, So, Vo = Vb, Sb, Ub
    else:
        Om = oracle.omega_srht(21, n, 16).astype(np.float64)
        Uo, So, Vo, _ = oracle.qlra_sketch(A64, 12, 4, v, 0, Om)
    d = ahat_diff(A64, (Ug, Sg, Vg), (Uo, So, Vo))
    print(f"  ahat diff {d:.3e}", flush=True)
    assert d <= (1e-5 if prec == 0 else 1e-2)


@pytest.mark.parametrize("scheme", [0, 1])
def test_phase_convention_tall(gq, oracle, scheme):
    """The phase normalisation of the returned factors: in every column of V the entry of largest
    modulus is real and positive.  n = 3000 rows give 94 partial arg-maxes per column, several
    batches of the apply pass's scan; the factors also match the oracle's (same rule)."""
    m, n, k = 400, 3000, 8
    print(f"phase convention {m} x {n} scheme={scheme}", flush=True)
    A32 = (W.planted(81, m, n, k) + 1e-3 * W.random_quat(82, m, n)).astype(np.float32)
    Ug, Sg, Vg, _, st = run_gpu(gq, A32, k, 4, 3, scheme, 2)
    assert st == gq.QLRA_OK
    mod = (Vg ** 2).sum(axis=0)
    for j in range(k):
        q = Vg[:, int(np.argmax(mod[:, j])), j]
        assert q[0] > 0.0 and np.abs(q[1:]).max() <= 1e-6 * q[0], (j, q)
    Uo, So, Vo, _ = oracle.qlra(A32.astype(np.float64), k, 4, 3, scheme, 2)
    assert np.abs(Vg - Vo).max() < 1e-4
    assert np.abs(Ug - Uo).max() < 1e-4
