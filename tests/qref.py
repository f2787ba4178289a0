"""Independent numpy helpers for the tests: the complex adjoint chi and norms.

These are textbook constructions (Zhang 1997, cited in Sec. 2 of the paper),
written here separately from both the oracle and the GPU library so that each
can be checked against them.
"""
import numpy as np


def chi(P):
    """Complex adjoint of a quaternion matrix given as planes (4, r, c):
    chi(X) = [[Xa, Xb], [-conj(Xb), conj(Xa)]], Xa = X0 + i X1, Xb = X2 + i X3."""
    P = np.asarray(P, dtype=np.float64)
    a = P[0] + 1j * P[1]
    b = P[2] + 1j * P[3]
    return np.block([[a, b], [-np.conj(b), np.conj(a)]])


def unchi(C):
    """Inverse of chi for a matrix known to have chi structure."""
    r, c = C.shape[0] // 2, C.shape[1] // 2
    a = C[:r, :c]
    b = C[:r, c:]
    return np.stack([a.real, a.imag, b.real, b.imag])


def qsv(P):
    """Quaternion singular values (descending): every other singular value of chi."""
    s = np.linalg.svd(chi(P), compute_uv=False)
    return s[0::2]


def spec(P):
    return qsv(P)[0]


def fro(P):
    return float(np.sqrt(np.sum(np.asarray(P, dtype=np.float64) ** 2)))


def adj(P):
    """Conjugate transpose in planes: (X0^T, -X1^T, -X2^T, -X3^T) (Sec. 2)."""
    P = np.asarray(P)
    out = P.transpose(0, 2, 1).copy()
    out[1:] *= -1
    return out


def mul(X, Y):
    """Quaternion product through chi (independent of the oracle's Hamilton loops)."""
    return unchi(chi(X) @ chi(Y))


def reconstruct(U, S, V):
    return mul(np.asarray(U) * np.asarray(S)[None, None, :], adj(V))


def flex_bound(sigma, k, p, alpha):
    """Right-hand side of the bound of Thm. (flex-Krylov) and eqs. (mn11)/(mn12):
    ((1 + 3 sqrt(k/(4p+2))) s_{k+1}^a + 3e sqrt(4k+4p+2)/(2p+2) (sum_{j>k} s_j^{2a})^{1/2})^{1/a}."""
    s = np.asarray(sigma, dtype=np.float64)
    t1 = (1.0 + 3.0 * np.sqrt(k / (4.0 * p + 2.0))) * s[k] ** alpha
    t2 = 3.0 * np.e * np.sqrt(4.0 * k + 4.0 * p + 2.0) / (2.0 * p + 2.0) * np.sqrt(np.sum(s[k:] ** (2 * alpha)))
    return (t1 + t2) ** (1.0 / alpha)
