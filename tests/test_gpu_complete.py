"""Quaternion matrix completion (Sec. 7) on the GPU against the oracle's completion: the same
seeded sketch, mask and iteration count; X and the per-iteration misfits compared element by
element.  The GPU solves run in FP32 (views, bases) against the oracle's FP64, and the iteration
is a contraction towards the observed entries, so the per-solve rounding does not grow across
iterations (a 1e-7 relative perturbation of M moves X by 6e-8 after ten iterations of the image
workload): the tolerances are those of one solve."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL_X = 1e-5       # max |X_gpu - X_oracle| / max |X_oracle| (measured <= 7e-7)
TOL_FIT = 1e-5     # relative, per iteration (measured <= 5e-7)


@pytest.fixture(scope="module")
def gq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_13731_amd import qlra as Q
    return Q


def run_gpu(gq, M32, mask, rank, p, v, scheme, seed, iters, sigma, **kw):
    import torch
    Md = torch.from_numpy(M32).cuda()
    Kd = torch.from_numpy(mask).cuda()
    X, fit, ws = gq.qlra_complete(Md, Kd, rank, p, v, scheme, seed, iters, sigma, **kw)
    st = gq.qlra_status(ws)
    return X.cpu().numpy().astype(np.float64), fit.cpu().numpy(), st


def compare(Xg, fg, Xo, fo):
    dx = np.abs(Xg - Xo).max() / np.abs(Xo).max()
    df = np.abs(fg - fo) / np.abs(fo)
    print(f"  max rel X diff {dx:.3e}, fit rel diff {df.max():.3e}, fit {fo[0]:.4f} -> {fo[-1]:.4f}", flush=True)
    assert dx <= TOL_X
    assert np.all(df <= TOL_FIT)


CASES = {
    # name: (m, n, rank, p, v, scheme, observed, sigma, iters)
    "planted-subspace-v2-sigma0.6": (120, 100, 5, 5, 2, 0, 0.4, 0.6, 6),
    "planted-krylov-v4-unsmoothed": (97, 130, 6, 4, 4, 1, 0.5, 0.0, 5),
    "planted-subspace-v3-radius8": (70, 50, 4, 3, 3, 0, 0.6, 8.0 / 3.0, 4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_completion_matches_oracle(gq, oracle, name):
    m, n, rank, p, v, scheme, observed, sigma, iters = CASES[name]
    print(f"completion {name}: {m} x {n} rank {rank} p {p} v {v} scheme {scheme} sigma {sigma:.3f}", flush=True)
    M = W.planted(21, m, n, rank) + 0.01 * W.random_quat(22, m, n)
    M32 = M.astype(np.float32)
    mask = W.random_mask(23, m, n, observed)
    Xg, fg, st = run_gpu(gq, M32, mask, rank, p, v, scheme, 5, iters, sigma)
    assert st == gq.QLRA_OK
    Xo, fo = oracle.complete(M32.astype(np.float64), mask, rank, p, v, scheme, 5, iters, sigma)
    compare(Xg, fg, Xo, fo)


def test_image_workload_matches_oracle(gq, oracle):
    """The inpainting set-up: 256 x 256 pure quaternion image, 70 % of the pixels missing, rank 30,
    oversampling 10, two passes (Alg. 2), Gaussian smoothing 0.6 after each iteration."""
    print("completion image 256 x 256, 70% missing, rank 30, 2 passes, sigma 0.6", flush=True)
    M32 = W.image_like(31, 256, 256)
    mask = W.random_mask(32, 256, 256, 0.3)
    Xg, fg, st = run_gpu(gq, M32, mask, 30, 10, 2, 0, 9, 10, 0.6)
    assert st == gq.QLRA_OK
    Xo, fo = oracle.complete(M32.astype(np.float64), mask, 30, 10, 2, 0, 9, 10, 0.6)
    compare(Xg, fg, Xo, fo)
    assert fo[-1] < fo[0]


def test_real_sketch_on_the_adjoint(gq, oracle):
    """opts.sketch = real and opts.transpose: each step runs on C^H with the real plane of the
    quaternion sketch (m x l here)."""
    m, n, rank, p = 60, 90, 4, 4
    print(f"completion real sketch on the adjoint {m} x {n}", flush=True)
    M32 = (W.planted(41, m, n, rank) + 0.01 * W.random_quat(42, m, n)).astype(np.float32)
    mask = W.random_mask(43, m, n, 0.5)
    Xg, fg, st = run_gpu(gq, M32, mask, rank, p, 2, 0, 6, 4, 0.6, transpose=True, sketch=gq.QLRA_SKETCH_REAL)
    assert st == gq.QLRA_OK
    Om = gq.qlra_omega(6, m, rank + p).cpu().numpy().astype(np.float64)
    Om[1:] = 0.0
    Xo, fo = oracle.complete(M32.astype(np.float64), mask, rank, p, 2, 0, 6, 4, 0.6, Om=Om, adjoint=True)
    compare(Xg, fg, Xo, fo)


def test_graph_replays_equal_eager(gq):
    """graph = 1 captures one iteration and replays it; the results are bitwise those of the eager
    launches, on the first (capturing) call and on a second call that replays the cached graph
    after other work changed the output buffers."""
    import torch
    m, n = 88, 75
    print(f"completion graph vs eager {m} x {n}", flush=True)
    M = torch.from_numpy((W.planted(51, m, n, 4) + 0.01 * W.random_quat(52, m, n)).astype(np.float32)).cuda()
    K = torch.from_numpy(W.random_mask(53, m, n, 0.5)).cuda()
    Xe, fe, _ = gq.qlra_complete(M, K, 4, 4, 3, 1, 8, 5, 0.6)
    X = torch.empty_like(M)
    fit = torch.empty(5, dtype=torch.float64, device="cuda")
    ws = None
    for call in range(2):
        X.fill_(7.0)
        fit.fill_(-1.0)
        _, _, ws = gq.qlra_complete(M, K, 4, 4, 3, 1, 8, 5, 0.6, X=X, fit=fit, workspace=ws, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(X, Xe), call
        assert torch.equal(fit, fe), call


def test_everything_observed_is_one_smoothed_approximation(gq, oracle):
    """mask = 1: C stays M, so X is the smoothed rank-R approximation of M from one qlra() call,
    and every iteration has the same misfit."""
    import torch
    m, n = 64, 72
    print(f"completion with a full mask {m} x {n}", flush=True)
    M32 = W.random_quat(61, m, n).astype(np.float32)
    mask = np.ones((m, n), dtype=np.uint8)
    Xg, fg, st = run_gpu(gq, M32, mask, 6, 4, 3, 0, 12, 3, 0.6)
    assert st == gq.QLRA_OK
    U, S, V, _, _ = gq.qlra(torch.from_numpy(M32).cuda(), 6, 4, 3, 0, 12, estimate=False)
    ref = oracle.smooth(oracle.reconstruct(U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()), 0.6)
    assert np.abs(Xg - ref).max() <= 1e-5 * np.abs(ref).max()
    assert np.all(np.abs(fg - fg[0]) <= 1e-12 * fg[0])


def test_nothing_observed(gq):
    """An empty mask: C^(0) = 0, every misfit is 0 / 0 = NaN, and from the second iteration the
    solve breaks down on the non-finite C, which the status reports."""
    m, n = 40, 36
    print(f"completion with an empty mask {m} x {n}", flush=True)
    M32 = W.random_quat(71, m, n).astype(np.float32)
    mask = np.zeros((m, n), dtype=np.uint8)
    _, fg, st = run_gpu(gq, M32, mask, 3, 2, 2, 0, 1, 2, 0.0)
    assert np.all(np.isnan(fg))
    assert st == gq.QLRA_E_NUMERIC


def test_argument_errors(gq):
    import torch
    M = torch.zeros((4, 10, 8), device="cuda")
    K = torch.ones((10, 8), dtype=torch.uint8, device="cuda")
    for args, code in [((3, 2, 2, 0, 0, 0), gq.QLRA_E_ARG),           # iters = 0
                       ((9, 2, 2, 0, 0, 1), gq.QLRA_E_ARG),           # rank + p > min(m, n)
                       ((3, 2, 1, 0, 0, 1), gq.QLRA_E_ARG)]:          # one pass
        with pytest.raises(gq.QlraError) as ei:
            gq.qlra_complete(M, K, *args)
        assert ei.value.code == code
    with pytest.raises(gq.QlraError) as ei:
        gq.qlra_complete(M, K, 3, 2, 2, 0, 0, 1, sigma=3.0)            # radius 9
    assert ei.value.code == gq.QLRA_E_UNSUPPORTED
