"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module only makes data.  It holds none of the method's arithmetic (no
sketch, no view products, no QR or QSVD of the method) and imports neither the
GPU package nor the oracle.  Quaternion matrices are numpy arrays of shape
(4, rows, cols) holding the planes (real, i, j, k).

Internally a quaternion matrix X = Xa + Xb j is handled in its Cayley-Dickson
complex form (Xa = X0 + X1 i, Xb = X2 + X3 i), where
    (Xa + Xb j)(Ya + Yb j) = (Xa Ya - Xb conj(Yb)) + (Xa Yb + Xb conj(Ya)) j,
    (Xa + Xb j)^H = Xa^H - Xb^T j.

Workloads (stand-ins for the paper's experiments; no dataset item is used):
  config0  dense 256 x 256, sigma_i = i^-2, Haar unitaries (QR of quaternion
           Gaussians), FP64.
  config1  dense 2048 x 2048, sigma_i = exp(-i/20) plus i.i.d. N(0, s^2) noise
           per real component (s = 0.01, i.e. variance 1e-4), FP32.
  config2  pure quaternion 1024 x 1536: three imaginary planes from a seeded
           smooth Gaussian random field (Gaussian kernel, std 16 px) mapped to
           [0, 1], plus U(-0.02, 0.02), clipped; real plane zero.  FP32.
  config4  dense 16384 x 16384, sigma_i = i^-1/2, unitaries that are products of
           8 random quaternion Householder reflectors and a random unit
           quaternion diagonal.  FP32, built on the host in a form whose bits do
           not depend on the machine (reflector_spectrum_matrix).
  planted  A = B C with quaternion Gaussian B (m x r), C (r x n) (exact rank r).
"""
import numpy as np


# --------------------------------------------------------------------------
# complex-pair helpers
# --------------------------------------------------------------------------

def to_pair(P):
    P = np.asarray(P, dtype=np.float64)
    return P[0] + 1j * P[1], P[2] + 1j * P[3]


def from_pair(a, b, dtype=np.float64):
    return np.stack([a.real, a.imag, b.real, b.imag]).astype(dtype)


def _mul(Xa, Xb, Ya, Yb):
    return Xa @ Ya - Xb @ np.conj(Yb), Xa @ Yb + Xb @ np.conj(Ya)


def _adj(Xa, Xb):
    return np.conj(Xa.T), -Xb.T


def qgauss(rng, r, c, dtype=np.float64):
    """Quaternion Gaussian matrix: four independent N(0, 1) planes."""
    return rng.standard_normal((4, r, c)).astype(dtype)


def haar_unitary(rng, n):
    """Haar-distributed quaternion unitary (n x n) as a complex pair.

    QR of a quaternion Gaussian with a real positive diagonal of R (Mezzadri's
    construction).  It is taken as the complex QR of the interleaved complex
    adjoint chi(G) (2x2 blocks [[a, b], [-conj b, conj a]]): chi(Q) chi(R) is a
    complex QR with positive diagonal, and that QR is unique, so the complex
    factor normalised to a positive diagonal of R is chi(Q).
    """
    G = rng.standard_normal((4, n, n))
    a, b = G[0] + 1j * G[1], G[2] + 1j * G[3]
    C = np.empty((2 * n, 2 * n), dtype=np.complex128)
    C[0::2, 0::2] = a
    C[0::2, 1::2] = b
    C[1::2, 0::2] = -np.conj(b)
    C[1::2, 1::2] = np.conj(a)
    Qc, Rc = np.linalg.qr(C)
    d = np.diag(Rc)
    Qc = Qc * (d / np.abs(d))[None, :]
    return Qc[0::2, 0::2].copy(), Qc[0::2, 1::2].copy()


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q[0] + 1j * q[1], q[2] + 1j * q[3]


def _apply_reflector_left(Ma, Mb, ua, ub):
    """M <- (I - 2 u u^H / (u^H u)) M for a quaternion vector u (complex pair)."""
    nrm2 = np.sum(np.abs(ua) ** 2 + np.abs(ub) ** 2)
    # t = u^H M  (row vector), then M -= u (2 t / nrm2)
    uha, uhb = _adj(ua[:, None], ub[:, None])
    ta, tb = _mul(uha, uhb, Ma, Mb)
    ta *= 2.0 / nrm2
    tb *= 2.0 / nrm2
    da, db = _mul(ua[:, None], ub[:, None], ta, tb)
    return Ma - da, Mb - db


def reflector_unitary_apply(rng, Ma, Mb, nrefl=8, side="left"):
    """Multiply M by a random unitary H_1 ... H_nrefl D (side='left': U M) or
    by its adjoint on the right (side='right': M U^H), where each H_i is a
    quaternion Householder reflector with a Gaussian vector and D is a
    diagonal of random unit quaternions."""
    if side == "right":
        Ma, Mb = _adj(Ma, Mb)
    n = Ma.shape[0]
    da, db = _unit_quats(rng, n)
    # D M: row i scaled on the left by the quaternion d_i
    Ma, Mb = (da[:, None] * Ma - db[:, None] * np.conj(Mb),
              da[:, None] * Mb + db[:, None] * np.conj(Ma))
    for _ in range(nrefl):
        u = rng.standard_normal((4, n))
        Ma, Mb = _apply_reflector_left(Ma, Mb, u[0] + 1j * u[1], u[2] + 1j * u[3])
    if side == "right":
        Ma, Mb = _adj(Ma, Mb)
    return Ma, Mb


def from_svd(Ua, Ub, sigma, Va, Vb):
    """U diag(sigma) V^H (complex pairs in, complex pair out)."""
    Sa = Ua * sigma[None, :]
    Sb = Ub * sigma[None, :]
    Vha, Vhb = _adj(Va, Vb)
    return _mul(Sa, Sb, Vha, Vhb)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def config0(seed=0):
    """Dense 256 x 256, sigma_i = i^-2, Haar U, V; FP64 planes."""
    rng = np.random.default_rng(seed)
    n = 256
    Ua, Ub = haar_unitary(rng, n)
    Va, Vb = haar_unitary(rng, n)
    sigma = np.arange(1, n + 1, dtype=np.float64) ** -2.0
    a, b = from_svd(Ua, Ub, sigma, Va, Vb)
    return from_pair(a, b), sigma


def config1(seed=1, n=2048, noise_std=0.01, haar=True):
    """Dense n x n, sigma_i = exp(-i/20) plus i.i.d. N(0, noise_std^2) per real
    component; FP32 planes.  Returns (A, sigma_of_signal)."""
    rng = np.random.default_rng(seed)
    sigma = np.exp(-np.arange(1, n + 1, dtype=np.float64) / 20.0)
    if haar:
        Ua, Ub = haar_unitary(rng, n)
        Va, Vb = haar_unitary(rng, n)
        a, b = from_svd(Ua, Ub, sigma, Va, Vb)
    else:
        Ma = np.diag(sigma).astype(np.complex128)
        Mb = np.zeros_like(Ma)
        Ma, Mb = reflector_unitary_apply(rng, Ma, Mb, side="left")
        a, b = reflector_unitary_apply(rng, Ma, Mb, side="right")
    A = from_pair(a, b)
    if noise_std > 0:
        A = A + noise_std * rng.standard_normal(A.shape)
    return A.astype(np.float32), sigma


def grf_plane(rng, m, n, corr=16.0):
    """Smooth Gaussian random field on an m x n periodic grid: white noise
    convolved (FFT) with an isotropic Gaussian of std `corr` pixels, min-max
    mapped to [0, 1]."""
    white = rng.standard_normal((m, n))
    fy = np.fft.fftfreq(m)[:, None]
    fx = np.fft.fftfreq(n)[None, :]
    kern = np.exp(-2.0 * (np.pi * corr) ** 2 * (fx ** 2 + fy ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(white) * kern))
    f -= f.min()
    f /= f.max()
    return f


def config2(seed=2, m=1024, n=1536):
    """Pure quaternion m x n: real plane 0, three GRF planes + U(-0.02, 0.02),
    clipped to [0, 1]; FP32 planes."""
    rng = np.random.default_rng(seed)
    A = np.zeros((4, m, n))
    for p in range(1, 4):
        A[p] = np.clip(grf_plane(rng, m, n) + rng.uniform(-0.02, 0.02, (m, n)), 0.0, 1.0)
    return A.astype(np.float32)


def spectrum_matrix(seed, m, n, sigma, nrefl=8, dtype=np.float32):
    """U diag(sigma) V^H with reflector-product unitaries (m x n)."""
    rng = np.random.default_rng(seed)
    r = min(m, n)
    Ma = np.zeros((m, n), dtype=np.complex128)
    Ma[np.arange(r), np.arange(r)] = sigma[:r]
    Mb = np.zeros_like(Ma)
    Ma, Mb = reflector_unitary_apply(rng, Ma, Mb, nrefl=nrefl, side="left")
    Ma, Mb = reflector_unitary_apply(rng, Ma, Mb, nrefl=nrefl, side="right")
    return from_pair(Ma, Mb, dtype=dtype)


# Hamilton product (eq. (1)) as a table: plane p of a b is the sum of sign * a_q * b_r
# over the entries (q, r, sign) of row p.
_HT = (
    ((0, 0, 1), (1, 1, -1), (2, 2, -1), (3, 3, -1)),
    ((0, 1, 1), (1, 0, 1), (2, 3, 1), (3, 2, -1)),
    ((0, 2, 1), (1, 3, -1), (2, 0, 1), (3, 1, 1)),
    ((0, 3, 1), (1, 2, 1), (2, 1, -1), (3, 0, 1)),
)


def _pq(a, b):
    """Elementwise quaternion product of broadcastable plane arrays (4, ...)."""
    return np.stack([sum(s * a[q] * b[r] for q, r, s in _HT[p]) for p in range(4)])


def _pconj(a):
    return np.stack([a[0], -a[1], -a[2], -a[3]])


def _pdot(a, b):
    """sum_r conj(a_r) b_r of two quaternion vectors (planes (4, n)); every plane summed with
    math.fsum (correctly rounded, so the same on any machine)."""
    import math
    pr = _pq(_pconj(a), b)
    return np.array([math.fsum(pr[p]) for p in range(4)])


def _compact_unitary(rng, n, nrefl):
    """The unitary H_nrefl ... H_1 D of reflector_unitary_apply (same draws, same order) in the
    form (I - W Z^H) D: returns d (4, n), W (4, n, nrefl) and Z^H (4, nrefl, n).  With
    H_i = I - tau_i u_i u_i^H, prepending H_i to I - W Z^H appends u_i to W and the row
    tau_i (u_i^H - (u_i^H W) Z^H) to Z^H."""
    import math
    q = rng.standard_normal((4, n))
    d = q / np.linalg.norm(q, axis=0, keepdims=True)
    Wm = np.zeros((4, n, nrefl))
    ZH = np.zeros((4, nrefl, n))
    for i in range(nrefl):
        u = rng.standard_normal((4, n))
        tau = 2.0 / math.fsum((u * u).ravel())
        z = _pconj(u)
        for c in range(i):
            z = z - _pq(_pdot(u, Wm[:, :, c])[:, None], ZH[:, c, :])
        ZH[:, i, :] = tau * z
        Wm[:, :, i] = u
    return d, Wm, ZH


def reflector_spectrum_matrix(seed, m, n, sigma, nrefl=8, threads=8, block=32):
    """U diag(sigma) V^H (m x n, FP32 planes) for the unitaries of spectrum_matrix (the same
    random draws: U = H_nrefl ... H_1 D_u, then V likewise), built without forming U or V.

    With U = (I - Wu Zu^H) D_u, V = (I - Wv Zv^H) D_v and the diagonal L = D_u diag(sigma) D_v^H,
        A = L - Wu F - G Wv^H,   F = Zu^H L - (Zu^H L Zv) Wv^H,   G = L Zv,
    a diagonal plus 2 nrefl quaternion outer products.  Every sum of more than a few terms is a
    math.fsum and the outer products are accumulated in FP64 elementwise in a fixed order (no
    BLAS), so the FP32 result is the same bits on any machine and for any thread count.  Rows
    are built in blocks on `threads` threads (numpy releases the GIL)."""
    import math
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(seed)
    r = min(m, n)
    du, Wu, ZHu = _compact_unitary(rng, m, nrefl)
    dv, Wv, ZHv = _compact_unitary(rng, n, nrefl)
    lam = _pq(du[:, :r] * np.asarray(sigma[:r], dtype=np.float64)[None], _pconj(dv[:, :r]))   # (4, r)
    ZHL = np.zeros((4, nrefl, n))
    ZHL[:, :, :r] = _pq(ZHu[:, :, :r], lam[:, None, :])            # Zu^H L
    Zv = np.transpose(_pconj(ZHv), (0, 2, 1))                         # (4, n, nrefl)
    Cm = np.zeros((4, nrefl, nrefl))                                  # Zu^H L Zv
    for a in range(nrefl):
        for b in range(nrefl):
            pr = _pq(ZHL[:, a, :], Zv[:, :, b])
            Cm[:, a, b] = [math.fsum(pr[p]) for p in range(4)]
    WvH = np.transpose(_pconj(Wv), (0, 2, 1))                         # (4, nrefl, n)
    F = ZHL.copy()
    for b in range(nrefl):
        F = F - _pq(Cm[:, :, b][:, :, None], WvH[:, b, :][:, None, :])
    G = np.zeros((4, m, nrefl))
    G[:, :r, :] = _pq(lam[:, :, None], Zv[:, :r, :])                 # L Zv
    Lf = np.ascontiguousarray(np.concatenate([Wu, G], axis=2))        # (4, m, 2 nrefl)
    Rf = np.ascontiguousarray(np.concatenate([F, WvH], axis=1))       # (4, 2 nrefl, n)
    out = np.empty((4, m, n), dtype=np.float32)

    def rows(r0):
        r1 = min(m, r0 + block)
        acc = np.zeros((4, r1 - r0, n))
        tmp = np.empty((r1 - r0, n))
        for t in range(2 * nrefl):
            for p in range(4):
                for q, s_, sg in _HT[p]:
                    np.multiply.outer(Lf[q, r0:r1, t], Rf[s_, t, :], out=tmp)
                    if sg > 0:
                        np.subtract(acc[p], tmp, out=acc[p])
                    else:
                        np.add(acc[p], tmp, out=acc[p])
        d = np.arange(r0, min(r1, r))
        for p in range(4):
            acc[p, d - r0, d] += lam[p, d]
            out[p, r0:r1] = acc[p]

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(rows, range(0, m, block)))
    return out


def config4(seed=4, n=16384, threads=8):
    """Dense n x n, sigma_i = i^-1/2, reflector-product unitaries; FP32.  Built on the host by
    reflector_spectrum_matrix (the same bits on any machine)."""
    sigma = np.arange(1, n + 1, dtype=np.float64) ** -0.5
    return reflector_spectrum_matrix(seed, n, n, sigma, threads=threads), sigma


def planted(seed, m, n, r, dtype=np.float64):
    """A = B C, B (m x r) and C (r x n) quaternion Gaussians: rank exactly r."""
    rng = np.random.default_rng(seed)
    B = qgauss(rng, m, r)
    C = qgauss(rng, r, n)
    a, b = _mul(B[0] + 1j * B[1], B[2] + 1j * B[3], C[0] + 1j * C[1], C[2] + 1j * C[3])
    return from_pair(a, b, dtype=dtype)


def random_quat(seed, r, c, dtype=np.float64):
    return qgauss(np.random.default_rng(seed), r, c, dtype)


def image_like(seed, m, n, corr=4.0):
    """Pure quaternion colour-image stand-in: real plane 0, three smooth Gaussian random fields
    (correlation `corr` pixels) with U(-0.02, 0.02) noise, clipped to [0, 1]; FP32 planes."""
    rng = np.random.default_rng(seed)
    A = np.zeros((4, m, n))
    for q in range(1, 4):
        A[q] = np.clip(grf_plane(rng, m, n, corr=corr) + rng.uniform(-0.02, 0.02, (m, n)), 0.0, 1.0)
    return A.astype(np.float32)


def random_mask(seed, m, n, observed):
    """0/1 uint8 mask, each entry observed independently with probability `observed`."""
    return (np.random.default_rng(seed).random((m, n)) < observed).astype(np.uint8)
