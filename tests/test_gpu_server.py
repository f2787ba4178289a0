"""The continuous-batching server through the C ABI.

Every request served in a mix (several in flight, steps interleaved on different streams,
admission by HBM footprint) gives exactly the result of the same qlra() call made alone: all
kernels are deterministic (no atomics, fixed reduction orders), so the comparison is bitwise.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_13731_amd import qlra as Q
    return Q


def mix(count, seed=0):
    """Mixed sizes, ranks, budgets, schemes and precisions (sigma_i = i^-1, dense or pure)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        m = int(rng.choice([256, 384, 512, 640]))
        n = int(rng.choice([256, 320, 448, 704]))
        k = int(rng.integers(8, 33))
        p = k // 4
        v = int(rng.integers(2, 7))
        scheme = i % 2
        prec = [0, 1, 2, 3, 4][i % 5]          # FP32, BF16, FP16 and the two split forms
        sigma = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -1.0
        A = W.spectrum_matrix(100 + i, m, n, sigma, nrefl=4)
        if i % 4 == 3:
            A[0] = 0.0           # pure quaternion
        reqs.append(dict(A=np.ascontiguousarray(A, dtype=np.float32), k=k, p=p, v=v, scheme=scheme, seed=7 + i, prec=prec))
    return reqs


def alone(gq, r):
    import torch
    U, S, V, e, _ = gq.qlra(torch.from_numpy(r["A"]).cuda(), r["k"], r["p"], r["v"], r["scheme"], r["seed"],
                            precision=r["prec"])
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (U, S, V, e)]


def serve(gq, reqs, hbm, max_active, graphs, use_wait=False):
    import torch
    srv = gq.Server(hbm, max_active=max_active, graphs=graphs)
    tickets = []
    for r in reqs:
        tickets.append(srv.submit(torch.from_numpy(r["A"]).cuda(), r["k"], r["p"], r["v"], r["scheme"], r["seed"],
                                  precision=r["prec"]))
    if not use_wait:
        srv.drain()
    out = []
    for t in tickets:
        st, lat, (U, S, V, e) = srv.wait(t) if use_wait else srv.poll(t, wait=True)
        torch.cuda.synchronize()
        out.append((st, lat, [x.cpu().numpy() for x in (U, S, V, e)]))
    stats = srv.stats()
    srv.close()
    return out, stats


@pytest.mark.parametrize("graphs", [False, True])
def test_server_mix_equals_alone(gq, graphs):
    print(f"server mix graphs={graphs}", flush=True)
    reqs = mix(12)
    out, stats = serve(gq, reqs, 2 << 30, 4, graphs)
    assert stats["max_active_seen"] > 1            # requests really overlapped
    for r, (st, lat, got) in zip(reqs, out):
        assert st == gq.QLRA_OK
        assert lat > 0
        ref = alone(gq, r)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b, equal_nan=True)


def test_server_admission_by_footprint(gq):
    """An arena that holds one large request at a time: large requests never overlap each
    other, the arena is never overcommitted, and every result is still the alone result."""
    print("server admission", flush=True)
    reqs = mix(6, seed=3)
    for r in reqs:
        r["A"] = np.ascontiguousarray(np.tile(r["A"], (1, 2, 2)))
    sizes = [gq.qlra_workspace_size(r["A"].shape[1], r["A"].shape[2], r["k"], r["p"], r["v"], r["scheme"],
                                    precision=r["prec"]) for r in reqs]
    hbm = int(max(sizes) * 1.2)
    out, stats = serve(gq, reqs, hbm, 8, False, use_wait=True)
    assert stats["max_arena_used"] <= hbm
    assert stats["max_active_seen"] <= 8
    for r, (st, lat, got) in zip(reqs, out):
        assert st == gq.QLRA_OK
        ref = alone(gq, r)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b, equal_nan=True)


def test_server_rejects_requests_larger_than_the_arena(gq):
    import torch
    srv = gq.Server(1 << 20, max_active=2)
    A = torch.zeros((4, 512, 512), device="cuda")
    with pytest.raises(gq.QlraError) as ei:
        srv.submit(A, 16, 4, 3, 0, 1)
    assert ei.value.code == gq.QLRA_E_TOO_LARGE
    srv.close()
