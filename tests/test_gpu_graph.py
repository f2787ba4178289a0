"""Graph capture of a whole solve: replays of the captured graph, interleaved with other
eager GPU work and synchronisations, give bit-identical results to the eager solve."""
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


@pytest.mark.parametrize("scheme,v", [("subspace", 4), ("block_krylov", 5)])
def test_graph_replays_match_eager(gq, scheme, v):
    import torch
    A, _ = W.config0()
    dA = torch.from_numpy(A.astype(np.float32)).cuda()
    k, p = 10, 5
    U, S, V, e, ws = gq.qlra(dA, k, p, v, scheme, 0, graph=False)
    torch.cuda.synchronize()
    ref = [x.cpu().numpy().copy() for x in (U, S, V, e)]
    for rep in range(3):
        print(f"graph replay {scheme} v={v} rep={rep}", flush=True)
        # unrelated eager work between replays, including the same workspace being reused
        junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        for x in (U, S, V, e):
            x.zero_()
        gq.qlra(dA, k, p, v, scheme, 0, U=U, S=S, V=V, pass_err=e, workspace=ws, graph=True)
        torch.cuda.synchronize()
        assert gq.qlra_status(ws) == gq.QLRA_OK
        got = [x.cpu().numpy() for x in (U, S, V, e)]
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        del junk
