"""GPU parity of the reduced-precision form (BF16 / FP16 views with FP32 accumulation) through
the C ABI.

- the low-precision copies of A are bit-exact with round-to-nearest-even of s A (s = 1 for
  BF16, a power of two for FP16), rounded independently here with integer arithmetic
  (BF16) or numpy's float16 conversion;
- the view product from those copies equals the oracle's FP64 product of the *rounded*
  operands up to FP32 accumulation error (8 u32 sqrt(4K) times the sum of term magnitudes),
  so the only approximation left is the input rounding itself;
- end to end, views 1 .. v-2 in BF16 / FP16 and the last two in FP32 give an approximation
  error within 5 % of the FP64 oracle's (error ratio <= 1.05), and v = 2 (no reduced view)
  is bitwise the FP32 result.
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


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def round_bf16_bits(x32):
    """Round-to-nearest-even FP32 -> BF16 by integer arithmetic; returns the 16-bit patterns."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_bits_to_f64(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rounded(x32, prec, scale=1.0):
    """The value the kernel multiplies: s x rounded to the low-precision type, as FP64."""
    xs = (np.asarray(x32, dtype=np.float32) * np.float32(scale)).astype(np.float32)
    if prec == "bf16":
        return bf16_bits_to_f64(round_bf16_bits(xs))
    return xs.astype(np.float16).astype(np.float64)


PREC = {"bf16": 1, "fp16": 2}


def tiled(x):
    """(4, R, K) array -> the flat tiled order of include/qlra.h: tiles of 16 rows x 64
    reduction elements, the four planes of a tile adjacent, inside a tile [h][kq][r][8]."""
    _, R, K = x.shape
    RT, KT = -(-R // 16), -(-K // 64)
    pad = np.zeros((4, RT * 16, KT * 64), dtype=x.dtype)
    pad[:, :R, :K] = x
    t = pad.reshape(4, RT, 16, KT, 2, 4, 8)          # p, rt, r, kt, h, kq, e
    return np.ascontiguousarray(t.transpose(1, 3, 0, 4, 5, 2, 6)).reshape(-1)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("m,n", [(300, 200), (129, 67)])
def test_lowp_copy_bit_exact(gq, prec, m, n):
    import torch
    print(f"lowp copy {prec} {m}x{n}", flush=True)
    A = (W.random_quat(m + n, m, n) * 3.0).astype(np.float32)
    scale = 2.0 ** 5 if prec == "fp16" else 1.0
    s = torch.tensor([scale], dtype=torch.float32, device="cuda")
    Alo, Alo_t = gq.qlra_lowp_copy(dev(A), PREC[prec], scale=s)
    torch.cuda.synchronize()
    got = Alo.cpu().view(torch.int16).numpy().view(np.uint16)
    got_t = Alo_t.cpu().view(torch.int16).numpy().view(np.uint16)
    xs = (A * np.float32(scale)).astype(np.float32)
    if prec == "bf16":
        want = round_bf16_bits(xs)
    else:
        want = xs.astype(np.float16).view(np.uint16)
    assert np.array_equal(got, tiled(want))
    assert np.array_equal(got_t, tiled(np.ascontiguousarray(want.transpose(0, 2, 1))))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("m,n,w", [(300, 200, 15), (512, 1024, 60), (1000, 777, 80), (640, 900, 96), (64, 2048, 1),
                                   (900, 700, 112), (333, 1500, 160), (520, 260, 200),
                                   (700, 500, 100), (400, 1300, 160)])
def test_qgemm_lp_against_rounded_oracle(gq, oracle, prec, op, m, n, w):
    import torch
    print(f"qgemm_lp {prec} op={op} {m}x{n} w={w}", flush=True)
    A = W.random_quat(7 * m + n + w, m, n).astype(np.float32)
    kdim = n if op == 0 else m
    B = W.random_quat(w + 11, kdim, w).astype(np.float32)
    Alo, Alo_t = gq.qlra_lowp_copy(dev(A), PREC[prec])
    C = gq.qlra_qgemm_lp(op, PREC[prec], Alo if op == 0 else Alo_t, m, n, dev(B))
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    Ar, Br = rounded(A, prec), rounded(B, prec)
    ref = oracle.qgemm(Ar, Br) if op == 0 else oracle.qgemm_adj(Ar, Br)
    if op == 0:
        bound = np.abs(Ar).sum(0) @ np.abs(Br).sum(0)
    else:
        bound = np.abs(Ar).sum(0).T @ np.abs(Br).sum(0)
    tol = 8 * U32 * np.sqrt(4 * kdim) * bound + 1e-30
    assert np.all(np.abs(got - ref) <= tol[None])


def test_qgemm_lp_fp16_scale(gq, oracle):
    """FP16 with a power-of-two scale: entries of size 1e6 would overflow FP16 unscaled; with
    s = 2^-10 on the copy and 1/s on the result the product matches the rounded oracle."""
    import torch
    m, n, w = 256, 384, 20
    A = (W.random_quat(5, m, n) * 1e6).astype(np.float32)
    B = W.random_quat(6, n, w).astype(np.float32)
    s = 2.0 ** -10
    st = torch.tensor([s], dtype=torch.float32, device="cuda")
    inv = torch.tensor([1.0 / s], dtype=torch.float32, device="cuda")
    Alo, _ = gq.qlra_lowp_copy(dev(A), 2, scale=st)
    C = gq.qlra_qgemm_lp(0, 2, Alo, m, n, dev(B), inv_scale=inv)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    Ar, Br = rounded(A, "fp16", s), rounded(B, "fp16")
    ref = oracle.qgemm(Ar, Br) / s
    bound = (np.abs(Ar).sum(0) @ np.abs(Br).sum(0)) / s
    assert np.all(np.abs(got - ref) <= 8 * U32 * np.sqrt(4 * n) * bound[None])


def run_gpu(gq, A32, k, p, v, scheme, seed, precision):
    import torch
    U, S, V, e, ws = gq.qlra(dev(A32), k, p, v, scheme, seed, precision=precision)
    st = gq.qlra_status(ws)
    torch.cuda.synchronize()
    return U.cpu().numpy().astype(np.float64), S.cpu().numpy(), V.cpu().numpy().astype(np.float64), \
        e.cpu().numpy(), st


def rel_err(oracle, A, U, S, V):
    return qref.fro(oracle.reconstruct(U, S, V) - A) / qref.fro(A)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("v", [3, 4, 6])
def test_lowp_solve_config0_error_ratio(gq, oracle, prec, scheme, v):
    """256 x 256, sigma_i = i^-2, k = 10, p = 5: error ratio to the FP64 oracle <= 1.05."""
    print(f"lowp config0 {prec} scheme={scheme} v={v}", flush=True)
    A, _ = W.config0()
    A32 = A.astype(np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 10, 5, v, scheme, 0, PREC[prec])
    assert st == gq.QLRA_OK
    Uo, So, Vo, eo = oracle.qlra(A, 10, 5, v, scheme, 0)
    ratio = rel_err(oracle, A, Ug, Sg, Vg) / rel_err(oracle, A, Uo, So, Vo)
    print(f"  error ratio {ratio:.6f}", flush=True)
    assert ratio <= 1.05
    assert np.all(np.isfinite(eg[1:]))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_lowp_v2_is_fp32(gq, prec):
    """With v = 2 no view is reduced: the result is bitwise the FP32 one."""
    A = W.random_quat(3, 300, 240).astype(np.float32)
    r32 = run_gpu(gq, A, 12, 4, 2, 0, 5, 0)
    rlp = run_gpu(gq, A, 12, 4, 2, 0, 5, PREC[prec])
    for a, b in zip(r32[:4], rlp[:4]):
        assert np.array_equal(a, b, equal_nan=True)


_C1 = {}


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("v", [4, 6])
def test_lowp_solve_config1_error_ratio(gq, oracle, prec, v):
    """The 2048 x 2048 benchmark matrix: error ratio to the FP64 oracle <= 1.05."""
    print(f"lowp config1 {prec} v={v}", flush=True)
    if "A" not in _C1:
        _C1["A"] = W.config1()[0]
    A32 = _C1["A"]
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 50, 10, v, 0, 1, PREC[prec])
    assert st == gq.QLRA_OK
    A = A32.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A, 50, 10, v, 0, 1)
    ratio = rel_err(oracle, A, Ug, Sg, Vg) / rel_err(oracle, A, Uo, So, Vo)
    print(f"  error ratio {ratio:.8f}", flush=True)
    assert ratio <= 1.05


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_lowp_solve_wide_views(gq, oracle, prec):
    """k + p = 110 (views of two column tiles): error ratio to the FP64 oracle <= 1.05."""
    print(f"lowp wide views {prec}", flush=True)
    m, n = 500, 420
    sigma = np.concatenate([np.linspace(1.0, 0.3, 100), 1e-2 / np.arange(1, n - 99)])
    A32 = np.ascontiguousarray(W.spectrum_matrix(23, m, n, sigma, nrefl=6), dtype=np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 100, 10, 5, 0, 4, PREC[prec])
    assert st == gq.QLRA_OK
    A = A32.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A, 100, 10, 5, 0, 4)
    ratio = rel_err(oracle, A, Ug, Sg, Vg) / rel_err(oracle, A, Uo, So, Vo)
    print(f"  error ratio {ratio:.8f}", flush=True)
    assert ratio <= 1.05


def test_lowp_solve_config2_error_ratio(gq, oracle):
    """Pure quaternion 1024 x 1536 smooth field, block Krylov k = 64, p = 16, v = 6, BF16 views."""
    print("lowp config2 bf16", flush=True)
    A32 = W.config2()
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 64, 16, 6, 1, 2, 1)
    assert st == gq.QLRA_OK
    A = A32.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A, 64, 16, 6, 1, 2)
    ratio = rel_err(oracle, A, Ug, Sg, Vg) / rel_err(oracle, A, Uo, So, Vo)
    print(f"  error ratio {ratio:.8f}", flush=True)
    assert ratio <= 1.05


# ---- the split form: a_hi b_hi + a_hi b_lo + a_lo b_hi ----

def residual(x32, prec, scale=1.0):
    """The residual the kernel multiplies: s x minus its rounded value (exact in FP32), rounded."""
    xs = (np.asarray(x32, dtype=np.float32) * np.float32(scale)).astype(np.float32)
    r = (xs - rounded(xs, prec).astype(np.float32)).astype(np.float32)
    return rounded(r, prec)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_lowp_residual_copy_bit_exact(gq, prec):
    import torch
    m, n = 200, 131
    print(f"residual copy {prec} {m}x{n}", flush=True)
    A = (W.random_quat(m + 2 * n, m, n) * 3.0).astype(np.float32)
    Ar, Ar_t = gq.qlra_lowp_copy_residual(dev(A), PREC[prec])
    torch.cuda.synchronize()
    got = Ar.cpu().view(torch.int16).numpy().view(np.uint16)
    got_t = Ar_t.cpu().view(torch.int16).numpy().view(np.uint16)
    r = residual(A, prec).astype(np.float32)
    want = round_bf16_bits(r) if prec == "bf16" else r.astype(np.float16).view(np.uint16)
    assert np.array_equal(got, tiled(want))
    assert np.array_equal(got_t, tiled(np.ascontiguousarray(want.transpose(0, 2, 1))))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("m,n,w", [(300, 200, 15), (1000, 777, 80), (700, 500, 100), (64, 2048, 1), (450, 900, 160),
                                   (600, 300, 320)])
def test_qgemm_split_against_oracle(gq, oracle, prec, op, m, n, w):
    """The three products from the rounded pieces, each the oracle's FP64 product, summed: equal up
    to FP32 accumulation; and the sum is within the split's dropped terms (a_lo b_lo and the
    residual roundings, about 3 u_lp^2 per product) of the exact product."""
    import torch
    print(f"qgemm_split {prec} op={op} {m}x{n} w={w}", flush=True)
    A = W.random_quat(3 * m + n + w, m, n).astype(np.float32)
    kdim = n if op == 0 else m
    B = W.random_quat(w + 17, kdim, w).astype(np.float32)
    Alo, Alo_t = gq.qlra_lowp_copy(dev(A), PREC[prec])
    Ar, Ar_t = gq.qlra_lowp_copy_residual(dev(A), PREC[prec])
    C = gq.qlra_qgemm_split(op, PREC[prec], Alo if op == 0 else Alo_t, Ar if op == 0 else Ar_t, m, n, dev(B))
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    Ah, Al, Bh, Bl = rounded(A, prec), residual(A, prec), rounded(B, prec), residual(B, prec)
    prod = oracle.qgemm if op == 0 else oracle.qgemm_adj
    ref = prod(Ah, Bh) + prod(Ah, Bl) + prod(Al, Bh)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    mag = (np.abs(A64).sum(0) if op == 0 else np.abs(A64).sum(0).T) @ np.abs(B64).sum(0)
    assert np.all(np.abs(got - ref) <= 3 * 8 * U32 * np.sqrt(4 * kdim) * mag[None] + 1e-30)
    ulp = 2.0 ** -8 if prec == "bf16" else 2.0 ** -11
    exact = prod(A64, B64)
    assert np.all(np.abs(got - exact) <= (4 * ulp * ulp + 8 * U32 * np.sqrt(4 * kdim)) * mag[None] + 1e-30)


SPLIT = {"bf16": 3, "fp16": 4}


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("scheme,v", [(0, 2), (0, 3), (1, 4), (0, 6)])
def test_split_solve_config0(gq, oracle, prec, scheme, v):
    """The split precisions end to end (views v-1 and v in the split form; every view at v = 2):
    error ratio to the FP64 oracle <= 1.05, and the approximation close to the oracle's."""
    print(f"split config0 {prec} scheme={scheme} v={v}", flush=True)
    A, _ = W.config0()
    A32 = A.astype(np.float32)
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 10, 5, v, scheme, 0, SPLIT[prec])
    assert st == gq.QLRA_OK
    Uo, So, Vo, eo = oracle.qlra(A, 10, 5, v, scheme, 0)
    Ag, Ao = oracle.reconstruct(Ug, Sg, Vg), oracle.reconstruct(Uo, So, Vo)
    ratio = qref.fro(Ag - A) / qref.fro(Ao - A)
    diff = qref.fro(Ag - Ao) / qref.fro(A)
    print(f"  error ratio {ratio:.8f}, ahat diff {diff:.3e}", flush=True)
    assert ratio <= 1.05
    assert diff <= 1e-3


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_split_solve_config1(gq, oracle, prec):
    """The 2048 x 2048 benchmark matrix at v = 4 in the split precision: error ratio <= 1.05."""
    print(f"split config1 {prec}", flush=True)
    if "A" not in _C1:
        _C1["A"] = W.config1()[0]
    A32 = _C1["A"]
    Ug, Sg, Vg, eg, st = run_gpu(gq, A32, 50, 10, 4, 0, 1, SPLIT[prec])
    assert st == gq.QLRA_OK
    A = A32.astype(np.float64)
    Uo, So, Vo, eo = oracle.qlra(A, 50, 10, 4, 0, 1)
    ratio = rel_err(oracle, A, Ug, Sg, Vg) / rel_err(oracle, A, Uo, So, Vo)
    print(f"  error ratio {ratio:.8f}", flush=True)
    assert ratio <= 1.05
