"""qlra_noalloc(): the solve of qlra() with its workspace in the library's own device array (for
callers that cannot allocate).  Called through the C ABI on two solves in a row, the second
smaller, each checked against qlra() on the same inputs (the same kernels: bitwise equal
results are expected, the FP32 bound of the other parity tests is asserted); a solve whose
workspace exceeds the array is rejected before anything runs."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_13731_amd import qlra as Q
    L = ctypes.CDLL(Q.LIB_PATH)
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.qlra_noalloc.argtypes = [P, I64, I64, I64, I64, I, I, I, I, ctypes.c_uint64, ctypes.POINTER(Q.Opts),
                               P, I64, I64, P, P, I64, I64, P]
    L.qlra_noalloc.restype = I
    L.qlra_noalloc_status.argtypes = [P, ctypes.POINTER(I)]
    L.qlra_noalloc_status.restype = I
    L.qlra_noalloc_max_bytes.argtypes = []
    L.qlra_noalloc_max_bytes.restype = ctypes.c_size_t
    return Q, L


def noalloc_solve(Q, L, A, k, p, v, scheme, seed, precision=0):
    import torch
    m, n = A.shape[1], A.shape[2]
    U = torch.full((4, m, k), np.nan, device="cuda")
    V = torch.full((4, n, k), np.nan, device="cuda")
    S = torch.full((k,), np.nan, dtype=torch.float64, device="cuda")
    e = torch.full((v,), 7.0, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    o = Q.Opts(precision, 1, ctypes.c_void_p(st), None, 0, 1, 0, 0)
    rc = L.qlra_noalloc(ctypes.c_void_p(A.data_ptr()), m, n, n, m * n, k, p, v, scheme, ctypes.c_uint64(seed),
                        ctypes.byref(o), ctypes.c_void_p(U.data_ptr()), k, m * k, ctypes.c_void_p(S.data_ptr()),
                        ctypes.c_void_p(V.data_ptr()), k, n * k, ctypes.c_void_p(e.data_ptr()))
    status = ctypes.c_int(-1)
    if rc == 0:
        assert L.qlra_noalloc_status(ctypes.c_void_p(st), ctypes.byref(status)) == 0
    return rc, status.value, U, S, V, e


@pytest.mark.parametrize("scheme,prec", [(0, 0), (1, 0), (1, 1)])
def test_noalloc_matches_qlra(lib, scheme, prec):
    import torch
    Q, L = lib
    for (m, n, k, p, v) in ((700, 520, 24, 8, 5), (260, 190, 10, 5, 3)):
        print(f"noalloc {m}x{n} k={k} p={p} v={v} scheme={scheme} prec={prec}", flush=True)
        sigma = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -1.0
        A = torch.from_numpy(np.ascontiguousarray(W.spectrum_matrix(m + n, m, n, sigma, nrefl=4),
                                                  dtype=np.float32)).cuda()
        rc, status, U, S, V, e = noalloc_solve(Q, L, A, k, p, v, scheme, 4, prec)
        assert rc == Q.QLRA_OK and status == Q.QLRA_OK
        U2, S2, V2, e2, ws = Q.qlra(A, k, p, v, scheme, 4, precision=prec)
        assert Q.qlra_status(ws) == Q.QLRA_OK
        torch.cuda.synchronize()
        Sa, Sb = S.cpu().numpy(), S2.cpu().numpy()
        ea, eb = e.cpu().numpy(), e2.cpu().numpy()
        np.testing.assert_allclose(Sa, Sb, rtol=1e-6)
        assert np.isnan(ea[0]) and np.allclose(ea[1:], eb[1:], rtol=1e-6, atol=1e-7)
        for X, Y in ((U, U2), (V, V2)):
            assert np.abs(X.cpu().numpy() - Y.cpu().numpy()).max() <= 1e-5
        same = all(np.array_equal(a.cpu().numpy(), b.cpu().numpy(), equal_nan=True)
                   for a, b in ((U, U2), (V, V2), (S, S2), (e, e2)))
        print(f"  bitwise equal to qlra(): {same}", flush=True)


def test_noalloc_rejects_too_large(lib):
    import torch
    Q, L = lib
    cap = L.qlra_noalloc_max_bytes()
    m = n = 8192
    need = Q.qlra_workspace_size(m, n, 64, 16, 6, 1)
    assert need > cap
    A = torch.zeros((4, m, n), device="cuda")
    rc, _, _, _, _, _ = noalloc_solve(Q, L, A, 64, 16, 6, 1, 1)
    assert rc == Q.QLRA_E_TOO_LARGE
    assert Q.strerror(rc) == "request larger than supported"
