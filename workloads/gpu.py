"""Seeded synthetic inputs generated on the device with torch (for the serving stream, where
hundreds of matrices of mixed sizes are needed quickly).  Same construction as
workloads.spectrum_matrix: A = U diag(sigma) V^H with U, V products of random quaternion
Householder reflectors and a random unit-quaternion diagonal, quaternion matrices handled as
complex pairs (a, b) for a + b j.  None of the method's arithmetic lives here."""
import numpy as np
import torch


def _mul(Xa, Xb, Ya, Yb):
    return Xa @ Ya - Xb @ torch.conj(Yb), Xa @ Yb + Xb @ torch.conj(Ya)


def _adj(Xa, Xb):
    return torch.conj(Xa.T), -Xb.T


def _left_unitary(gen, Ma, Mb, nrefl):
    n = Ma.shape[0]
    dev = Ma.device
    q = torch.randn((4, n), generator=gen, device=dev, dtype=torch.float64)
    q = q / torch.linalg.norm(q, dim=0, keepdim=True)
    da, db = torch.complex(q[0], q[1]), torch.complex(q[2], q[3])
    Ma, Mb = da[:, None] * Ma - db[:, None] * torch.conj(Mb), da[:, None] * Mb + db[:, None] * torch.conj(Ma)
    for _ in range(nrefl):
        u = torch.randn((4, n), generator=gen, device=dev, dtype=torch.float64)
        ua, ub = torch.complex(u[0], u[1])[:, None], torch.complex(u[2], u[3])[:, None]
        nrm2 = torch.sum(torch.abs(ua) ** 2 + torch.abs(ub) ** 2)
        uha, uhb = _adj(ua, ub)
        ta, tb = _mul(uha, uhb, Ma, Mb)
        ta, tb = ta * (2.0 / nrm2), tb * (2.0 / nrm2)
        da_, db_ = _mul(ua, ub, ta, tb)
        Ma, Mb = Ma - da_, Mb - db_
    return Ma, Mb


def spectrum_matrix(seed, m, n, sigma, pure=False, nrefl=8, device="cuda"):
    """(4, m, n) float32 device tensor U diag(sigma) V^H; pure: real plane set to zero."""
    gen = torch.Generator(device=device).manual_seed(int(seed))
    r = min(m, n)
    Ma = torch.zeros((m, n), dtype=torch.complex128, device=device)
    idx = torch.arange(r, device=device)
    Ma[idx, idx] = torch.as_tensor(np.asarray(sigma[:r], dtype=np.float64), device=device).to(torch.complex128)
    Mb = torch.zeros_like(Ma)
    Ma, Mb = _left_unitary(gen, Ma, Mb, nrefl)
    Ma, Mb = _adj(Ma, Mb)
    Ma, Mb = _left_unitary(gen, Ma, Mb, nrefl)
    Ma, Mb = _adj(Ma, Mb)
    A = torch.stack([Ma.real, Ma.imag, Mb.real, Mb.imag]).to(torch.float32)
    if pure:
        A[0].zero_()
    return A.contiguous()


def serving_stream(seed, count, device="cuda"):
    """The serving workload: m, n uniform in {256, ..., 2048} (steps of 128), sigma_i = i^-1,
    dense or pure 50/50, k uniform in {8, ..., 64}, p = floor(k / 4), pass budget uniform in
    {2, ..., 6}, subspace or block Krylov 50/50.  Returns a list of request dicts (A on the
    device)."""
    rng = np.random.default_rng(seed)
    sizes = np.arange(256, 2049, 128)
    reqs = []
    for i in range(count):
        m, n = int(rng.choice(sizes)), int(rng.choice(sizes))
        k = int(rng.integers(8, 65))
        p = k // 4
        v = int(rng.integers(2, 7))
        scheme = int(rng.integers(0, 2))
        pure = bool(rng.integers(0, 2))
        sigma = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -1.0
        A = spectrum_matrix(1000 + i, m, n, sigma, pure=pure, device=device)
        reqs.append(dict(A=A, m=m, n=n, k=k, p=p, v=v, scheme=scheme, seed=i + 1, pure=pure))
    return reqs
