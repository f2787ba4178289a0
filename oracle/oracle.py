"""ctypes binding of the FP64 CPU oracle (oracle/qlra_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  It never imports the GPU package and the GPU
package never imports it.

Quaternion matrices are numpy arrays of shape (4, rows, cols): planes
(real, i, j, k) of X = X0 + X1 i + X2 j + X3 k (Sec. 2).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qlra_oracle.c")
_LIB = os.path.join(_HERE, "libqlra_oracle.so")

SUBSPACE, BLOCK_KRYLOV, ALG1, ALG3 = 0, 1, 2, 3


def build(force=True):
    """Compile the oracle with gcc (FP contraction off: the Gaussian
    generator's operation sequence is part of its definition)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-Wall",
           "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.qo_philox4x32_10.argtypes = [P, P, P]
        L.qo_log_unit.argtypes = [ctypes.c_double]
        L.qo_log_unit.restype = ctypes.c_double
        L.qo_sqrt_pos.argtypes = [ctypes.c_double]
        L.qo_sqrt_pos.restype = ctypes.c_double
        L.qo_sincos_2pi.argtypes = [ctypes.c_double, P, P]
        L.qo_omega.argtypes = [ctypes.c_uint64, i64, i64, P]
        L.qo_qgemm.argtypes = [P, i64, i64, P, i64, P]
        L.qo_qgemm_adj.argtypes = [P, i64, i64, P, i64, P]
        L.qo_qr.argtypes = [P, i64, i64, P, P]
        L.qo_qsvd.argtypes = [P, i64, P, P, P]
        L.qo_qlra.argtypes = [P, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, ctypes.c_uint64, P, P, P, P]
        L.qo_qlra_sketch.argtypes = [P, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, P, P, P, P, P, P, P, P, P]
        for name in ("qo_qgemm", "qo_qgemm_adj", "qo_qr", "qo_qsvd", "qo_qlra", "qo_qlra_sketch"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _planes(x, dtype=np.float64):
    x = np.ascontiguousarray(x, dtype=dtype)
    assert x.ndim == 3 and x.shape[0] == 4, x.shape
    return x


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().qo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def log_unit(u):
    return lib().qo_log_unit(float(u))


def sqrt_pos(x):
    return lib().qo_sqrt_pos(float(x))


def sincos_2pi(u):
    s = ctypes.c_double()
    c = ctypes.c_double()
    lib().qo_sincos_2pi(float(u), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def omega(seed, n, l):
    """Gaussian quaternion sketch, FP32 planes (4, n, l)."""
    out = np.empty((4, n, l), dtype=np.float32)
    lib().qo_omega(ctypes.c_uint64(seed), n, l, _p(out))
    return out


# ------------------------------------------------------------------------------------------
# Structured sketch (the SRFT-like generator the paper's cost section mentions as a faster
# alternative, footnote of Sec. 6; its bounds are not those of Lemma 1): a subsampled
# randomized Hadamard transform Omega = D H S / sqrt(l), real, with
#   n_pad = the smallest power of two >= n, H the +-1 Hadamard matrix of order n_pad
#   (H[i, s] = (-1)^popcount(i & s)), rows i < n kept;
#   D = diag(d_i), d_i = -1 when bit 0 of word 0 of Philox4x32-10 at counter (i, 0, 2, 0)
#   (key (seed mod 2^32, seed div 2^32)) is set, else +1;
#   S = the columns s_j = pi(j), j < l, of a keyed permutation pi of [0, n_pad): a four-round
#   Feistel network on the bits of x (split into halves of h = ceil(log2 n_pad / 2) bits; round
#   r maps (L, R) to (R, L xor F), F = word 0 of Philox at counter (R, r, 3, 0) masked to h
#   bits), applied again while the result is >= n_pad (cycle walking).
# The scale is the FP32 rounding of 1 / sqrt(l).

def _key(seed):
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)


def srht_signs(seed, n):
    k = _key(seed)
    return np.array([-1.0 if philox4x32_10([i, 0, 2, 0], k)[0] & 1 else 1.0 for i in range(n)])


def srht_pad(n):
    p = 1
    while p < n:
        p *= 2
    return p


def srht_perm(seed, x, n_pad):
    bits = n_pad.bit_length() - 1
    h = (bits + 1) // 2
    mask = (1 << h) - 1
    k = _key(seed)

    def rounds(v):
        L, R = v >> h, v & mask
        for r in range(4):
            F = int(philox4x32_10([R, r, 3, 0], k)[0]) & mask
            L, R = R, L ^ F
        return (L << h) | R

    y = rounds(x)
    while y >= n_pad:
        y = rounds(y)
    return y


def omega_srht(seed, n, l):
    """The structured sketch as FP32 planes (4, n, l): real plane D H S / sqrt(l), others zero."""
    n_pad = srht_pad(n)
    d = srht_signs(seed, n)
    cols = np.array([srht_perm(seed, j, n_pad) for j in range(l)], dtype=np.int64)
    i = np.arange(n, dtype=np.int64)[:, None]
    par = np.vectorize(lambda v: bin(int(v)).count("1") & 1)(i & cols[None, :])
    out = np.zeros((4, n, l), dtype=np.float32)
    out[0] = (d[:, None] * np.where(par == 1, -1.0, 1.0)).astype(np.float32) * np.float32(1.0 / np.sqrt(l))
    return out


def qgemm(A, B):
    A = _planes(A)
    B = _planes(B)
    m, n = A.shape[1:]
    assert B.shape[1] == n
    C = np.empty((4, m, B.shape[2]))
    _check(lib().qo_qgemm(_p(A), m, n, _p(B), B.shape[2], _p(C)), "qgemm")
    return C


def qgemm_adj(A, B):
    A = _planes(A)
    B = _planes(B)
    m, n = A.shape[1:]
    assert B.shape[1] == m
    C = np.empty((4, n, B.shape[2]))
    _check(lib().qo_qgemm_adj(_p(A), m, n, _p(B), B.shape[2], _p(C)), "qgemm_adj")
    return C


def qr(Y):
    Y = _planes(Y)
    m, w = Y.shape[1:]
    Q = np.empty((4, m, w))
    R = np.empty((4, w, w))
    _check(lib().qo_qr(_p(Y), m, w, _p(Q), _p(R)), "qr")
    return Q, R


def qsvd(R):
    R = _planes(R)
    w = R.shape[1]
    assert R.shape[2] == w
    U = np.empty((4, w, w))
    V = np.empty((4, w, w))
    S = np.empty(w)
    _check(lib().qo_qsvd(_p(R), w, _p(U), _p(S), _p(V)), "qsvd")
    return U, S, V


def qlra(A, k, p, v, scheme, seed):
    """Full method on FP64 planes A (4, m, n) with the seeded sketch.
    Returns U (4, m, k), S (k,), V (4, n, k), pass_err (v,)."""
    A = _planes(A)
    m, n = A.shape[1:]
    U = np.empty((4, m, k))
    V = np.empty((4, n, k))
    S = np.empty(k)
    e = np.empty(v)
    _check(lib().qo_qlra(_p(A), m, n, k, p, v, scheme, ctypes.c_uint64(seed),
                         _p(U), _p(S), _p(V), _p(e)), "qlra")
    return U, S, V, e


def qlra_sketch(A, k, p, v, scheme, Om, bases=False):
    """Full method with an explicit sketch Om (4, n, k+p).  With bases=True
    also returns the final range/co-range bases Q1, Q2."""
    A = _planes(A)
    Om = _planes(Om)
    m, n = A.shape[1:]
    l = k + p
    assert Om.shape == (4, n, l), Om.shape
    U = np.empty((4, m, k))
    V = np.empty((4, n, k))
    S = np.empty(k)
    e = np.empty(v)
    wmax = min(min(m, n), (v // 2 + 1) * l)
    if bases:
        Q1 = np.empty(4 * m * wmax)
        Q2 = np.empty(4 * n * wmax)
        w1 = ctypes.c_int64()
        w2 = ctypes.c_int64()
        rc = lib().qo_qlra_sketch(_p(A), m, n, k, p, v, scheme, _p(Om), _p(U), _p(S), _p(V), _p(e),
                                  _p(Q1), ctypes.byref(w1), _p(Q2), ctypes.byref(w2))
        _check(rc, "qlra_sketch")
        Q1 = Q1[: 4 * m * w1.value].reshape(4, m, w1.value)
        Q2 = Q2[: 4 * n * w2.value].reshape(4, n, w2.value)
        return U, S, V, e, Q1, Q2
    rc = lib().qo_qlra_sketch(_p(A), m, n, k, p, v, scheme, _p(Om), _p(U), _p(S), _p(V), _p(e),
                              None, None, None, None)
    _check(rc, "qlra_sketch")
    return U, S, V, e


def reconstruct(U, S, V):
    """U diag(S) V^H with the oracle's own product (FP64 planes)."""
    US = np.asarray(U, dtype=np.float64) * np.asarray(S)[None, None, :]
    Vh = np.asarray(V, dtype=np.float64).transpose(0, 2, 1).copy()
    Vh[1:] *= -1.0                     # (V^H) planes: V0^T, -V1^T, -V2^T, -V3^T
    return qgemm(US, Vh)


# ------------------------------------------------------------------------------------------
# Quaternion matrix completion (Sec. 7, the alternating updates of the completion problem):
#   X^(t) <- L(C^(t)),   C^(t+1) <- mask . M + (1 - mask) . X^(t)
# with L the rank-R approximation by the randomized scheme (one sketch, drawn from `seed`, for
# every iteration), and, as in the image experiments of Sec. 8, a Gaussian smoothing of X^(t)
# before the update (sigma = 0: none).  Start: C^(0) = mask . M.

def gauss_weights(sigma):
    """Normalised Gaussian taps exp(-t^2 / (2 sigma^2)), t = -r .. r, r = ceil(3 sigma)."""
    r = int(np.ceil(3.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-t * t / (2.0 * sigma * sigma))
    return w / w.sum()


def smooth(X, sigma):
    """Separable Gaussian smoothing of every plane of X (4, m, n), edges replicated: along the
    rows, then along the columns; written as plain sums over the taps."""
    if sigma <= 0:
        return X.copy()
    w = gauss_weights(sigma)
    r = (len(w) - 1) // 2
    m, n = X.shape[1:]
    Y = np.zeros_like(X)
    for t in range(-r, r + 1):                       # along each row (column index moves)
        idx = np.clip(np.arange(n) + t, 0, n - 1)
        Y += w[t + r] * X[:, :, idx]
    Z = np.zeros_like(X)
    for t in range(-r, r + 1):                       # along each column (row index moves)
        idx = np.clip(np.arange(m) + t, 0, m - 1)
        Z += w[t + r] * Y[:, idx, :]
    return Z


def complete(M, mask, rank, p, v, scheme, seed, iters, sigma, Om=None, adjoint=False):
    """The completion iterations on FP64 planes M (4, m, n) with a 0/1 mask (m, n); returns the
    last X and, per iteration, the relative misfit on the observed entries
    ||mask . (X - M)||_F / ||mask . M||_F.  Om: an explicit sketch instead of the seeded one;
    adjoint: each rank-R step runs the scheme on C^H (C = V S U^H there)."""
    M = _planes(M)
    mk = np.asarray(mask, dtype=np.float64)[None]
    C = mk * M
    ref = np.sqrt(np.sum((mk * M) ** 2))
    fit = []
    X = C
    for t in range(iters):
        Cs = C
        if adjoint:
            Cs = C.transpose(0, 2, 1).copy()
            Cs[1:] *= -1.0
        if Om is None:
            U, S, V, _ = qlra(Cs, rank, p, v, scheme, seed)
        else:
            U, S, V, _ = qlra_sketch(Cs, rank, p, v, scheme, Om)
        if adjoint:
            U, V = V, U
        X = smooth(reconstruct(U, S, V), sigma)
        fit.append(np.sqrt(np.sum((mk * (X - M)) ** 2)) / ref)
        C = mk * M + (1.0 - mk) * X
    return X, np.array(fit)
