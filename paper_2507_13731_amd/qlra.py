"""Thin Python binding of libqlra.so (include/qlra.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and streams.  Quaternion matrices are tensors
of shape (4, rows, cols) whose last dimension is contiguous: plane stride = stride(0),
leading dimension = stride(1).

The library must have been built (``python -m paper_2507_13731_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqlra.so")

QLRA_OK, QLRA_E_ARG, QLRA_E_WORKSPACE, QLRA_E_HIP, QLRA_E_NUMERIC, QLRA_E_TOO_LARGE, QLRA_E_UNSUPPORTED = range(7)
QLRA_SUBSPACE, QLRA_BLOCK_KRYLOV = 0, 1
QLRA_SKETCH_QUATERNION, QLRA_SKETCH_REAL, QLRA_SKETCH_SRHT = 0, 1, 2
QLRA_FP32, QLRA_BF16, QLRA_FP16, QLRA_BF16_SPLIT, QLRA_FP16_SPLIT = 0, 1, 2, 3, 4
SCHEMES = {"subspace": QLRA_SUBSPACE, "block_krylov": QLRA_BLOCK_KRYLOV, "krylov": QLRA_BLOCK_KRYLOV}


class QlraError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} (status {code})")
        self.code = code


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int), ("graphs", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("a_plane_stride", ctypes.c_int64), ("k", ctypes.c_int), ("p", ctypes.c_int),
                ("pass_budget", ctypes.c_int), ("scheme", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("pass_precision", ctypes.c_int), ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("u_plane_stride", ctypes.c_int64), ("S", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("ldv", ctypes.c_int64), ("v_plane_stride", ctypes.c_int64), ("pass_err", ctypes.c_void_p),
                ("arrival_time", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int), ("active", ctypes.c_int), ("max_active_seen", ctypes.c_int),
                ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
                ("max_arena_used", ctypes.c_size_t), ("ticks", ctypes.c_int64)]


class Opts(ctypes.Structure):
    _fields_ = [("pass_precision", ctypes.c_int),
                ("estimate_passes", ctypes.c_int),
                ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t),
                ("graph", ctypes.c_int),
                ("transpose", ctypes.c_int),
                ("sketch", ctypes.c_int)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (paper_2507_13731_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_SZ = ctypes.POINTER(ctypes.c_size_t)

_lib.qlra_strerror.argtypes = [_I]
_lib.qlra_strerror.restype = ctypes.c_char_p
_lib.qlra_workspace_size.argtypes = [_I64, _I64, _I, _I, _I, _I, ctypes.POINTER(Opts), _SZ]
_lib.qlra.argtypes = [_P, _I64, _I64, _I64, _I64, _I, _I, _I, _I, ctypes.c_uint64, ctypes.POINTER(Opts),
                      _P, _I64, _I64, _P, _P, _I64, _I64, _P]
_lib.qlra_status.argtypes = [_P, _P, ctypes.POINTER(_I)]
_lib.qlra_complete_workspace_size.argtypes = [_I64, _I64, _I, _I, _I, _I, ctypes.c_double, ctypes.POINTER(Opts), _SZ]
_lib.qlra_complete.argtypes = [_P, _I64, _I64, _I64, _I64, _P, _I64, _I, _I, _I, _I, ctypes.c_uint64, _I,
                               ctypes.c_double, ctypes.POINTER(Opts), _P, _I64, _I64, _P]
_lib.qlra_omega.argtypes = [ctypes.c_uint64, _I64, _I64, _P, _I64, _I64, _P]
_lib.qlra_omega_srht.argtypes = [ctypes.c_uint64, _I64, _I64, _P, _I64, _I64, _P]
_lib.qlra_qgemm_workspace_size.argtypes = [_I, _I64, _I64, _I64, _SZ]
_lib.qlra_qgemm.argtypes = [_I, _P, _I64, _I64, _I64, _I64, _P, _I64, _I64, _I64, _P, _I64, _I64, _P,
                            ctypes.c_size_t, _P]
_lib.qlra_lowp_copy_bytes.argtypes = [_I64, _I64, _SZ, _SZ]
_lib.qlra_lowp_copy.argtypes = [_P, _I64, _I64, _I64, _I64, _I, _P, _P, _P, _P]
_lib.qlra_qgemm_lp_workspace_size.argtypes = [_I, _I, _I64, _I64, _I64, _SZ]
_lib.qlra_qgemm_lp.argtypes = [_I, _I, _P, _I64, _I64, _P, _I64, _I64, _I64, _P, _I64, _I64, _P, _P,
                               ctypes.c_size_t, _P]
_lib.qlra_lowp_copy_residual.argtypes = [_P, _I64, _I64, _I64, _I64, _I, _P, _P, _P, _P]
_lib.qlra_qgemm_split_workspace_size.argtypes = [_I, _I, _I64, _I64, _I64, _SZ]
_lib.qlra_qgemm_split.argtypes = [_I, _I, _P, _P, _I64, _I64, _P, _I64, _I64, _I64, _P, _I64, _I64, _P, _P,
                                  ctypes.c_size_t, _P]
_lib.qlra_cholqr_workspace_size.argtypes = [_I64, _I64, _SZ]
_lib.qlra_cholqr.argtypes = [_P, _I64, _I64, _I64, _I64, _P, _I64, _I64, _P, _P, ctypes.c_size_t, _P]
_lib.qlra_qsvd_workspace_size.argtypes = [_I64, _SZ]
_lib.qlra_qsvd.argtypes = [_P, _I64, _P, _P, _P, _P, ctypes.c_size_t, _P]
_lib.qlra_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]
_lib.qlra_server_submit.argtypes = [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
_lib.qlra_server_poll.argtypes = [_P, ctypes.c_uint64, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                  ctypes.POINTER(ctypes.c_double)]
_lib.qlra_server_wait.argtypes = [_P, ctypes.c_uint64, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double)]
_lib.qlra_server_drain.argtypes = [_P]
_lib.qlra_server_stats.argtypes = [_P, ctypes.POINTER(ServerStats)]
_lib.qlra_server_destroy.argtypes = [_P]
_lib.qlra_server_clock.argtypes = []
_lib.qlra_server_clock.restype = ctypes.c_double
for _name in ("qlra_server_create", "qlra_server_submit", "qlra_server_poll", "qlra_server_wait", "qlra_server_drain",
              "qlra_server_stats", "qlra_server_destroy"):
    getattr(_lib, _name).restype = _I
for _name in ("qlra_workspace_size", "qlra", "qlra_status", "qlra_complete_workspace_size", "qlra_complete",
              "qlra_omega", "qlra_omega_srht", "qlra_qgemm_workspace_size",
              "qlra_qgemm", "qlra_lowp_copy_bytes", "qlra_lowp_copy", "qlra_qgemm_lp_workspace_size", "qlra_qgemm_lp",
              "qlra_cholqr_workspace_size", "qlra_cholqr", "qlra_qsvd_workspace_size", "qlra_qsvd",
              "qlra_lowp_copy_residual", "qlra_qgemm_split_workspace_size", "qlra_qgemm_split"):
    getattr(_lib, _name).restype = _I

EXPORTS = ("qlra", "qlra_workspace_size", "qlra_status", "qlra_strerror", "qlra_complete", "qlra_omega_srht",
           "qlra_complete_workspace_size", "qlra_omega", "qlra_qgemm",
           "qlra_qgemm_workspace_size", "qlra_lowp_copy_bytes", "qlra_lowp_copy", "qlra_qgemm_lp", "qlra_qgemm_lp_workspace_size",
           "qlra_cholqr", "qlra_cholqr_workspace_size", "qlra_qsvd", "qlra_qsvd_workspace_size",
           "qlra_lowp_copy_residual", "qlra_qgemm_split", "qlra_qgemm_split_workspace_size",
           "qlra_server_create", "qlra_server_submit", "qlra_server_poll", "qlra_server_wait", "qlra_server_drain",
           "qlra_server_stats", "qlra_server_destroy", "qlra_server_clock")


def strerror(code):
    return _lib.qlra_strerror(int(code)).decode()


def _check(rc, what):
    if rc != QLRA_OK:
        raise QlraError(rc, what)


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _planes(t, rows, cols, what, dtype=torch.float32):
    if t.dtype != dtype or t.dim() != 3 or t.shape[0] != 4 or t.shape[1] != rows or t.shape[2] != cols:
        raise ValueError(f"{what}: expected a (4, {rows}, {cols}) {dtype} tensor, got {tuple(t.shape)} {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a device tensor")
    if cols > 1 and t.stride(2) != 1:
        raise ValueError(f"{what}: the last dimension must be contiguous")
    return ctypes.c_void_p(t.data_ptr()), t.stride(1) if rows > 1 else max(cols, 1), t.stride(0)


def _workspace(nbytes, device):
    # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def qlra_workspace_size(m, n, k, p, pass_budget, scheme, estimate=True, precision=QLRA_FP32, transpose=False,
                        sketch=QLRA_SKETCH_QUATERNION):
    o = Opts(precision, 1 if estimate else 0, None, None, 0, 0, 1 if transpose else 0, sketch)
    out = ctypes.c_size_t()
    _check(_lib.qlra_workspace_size(m, n, k, p, pass_budget, SCHEMES.get(scheme, scheme), ctypes.byref(o),
                                    ctypes.byref(out)), "qlra_workspace_size")
    return out.value


def qlra(A, k, p, pass_budget, scheme, seed, U=None, S=None, V=None, pass_err=None, workspace=None,
         estimate=True, stream=None, precision=QLRA_FP32, graph=False, transpose=False,
         sketch=QLRA_SKETCH_QUATERNION):
    """Truncated QSVD of A (4, m, n) FP32 on the GPU: returns (U, S, V, pass_err, workspace).
    Enqueued on `stream` (default: torch's current stream); no synchronisation.  transpose: run
    the scheme on A^H (U and V stay the factors of A)."""
    scheme = SCHEMES.get(scheme, scheme)
    m, n = A.shape[1], A.shape[2]
    dev = A.device
    pa, lda, aps = _planes(A, m, n, "A")
    if U is None:
        U = torch.empty((4, m, k), dtype=torch.float32, device=dev)
    if V is None:
        V = torch.empty((4, n, k), dtype=torch.float32, device=dev)
    if S is None:
        S = torch.empty(k, dtype=torch.float64, device=dev)
    if estimate and pass_err is None:
        pass_err = torch.empty(pass_budget, dtype=torch.float64, device=dev)
    pu, ldu, ups = _planes(U, m, k, "U")
    pv, ldv, vps = _planes(V, n, k, "V")
    need = qlra_workspace_size(m, n, k, p, pass_budget, scheme, estimate, precision, transpose, sketch)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    o = Opts(precision, 1 if estimate else 0, _stream_ptr(stream), ctypes.c_void_p(workspace.data_ptr()),
             workspace.numel(), 1 if graph else 0, 1 if transpose else 0, sketch)
    rc = _lib.qlra(pa, m, n, lda, aps, k, p, pass_budget, scheme, ctypes.c_uint64(seed), ctypes.byref(o),
                   pu, ldu, ups, ctypes.c_void_p(S.data_ptr()), pv, ldv, vps,
                   ctypes.c_void_p(pass_err.data_ptr()) if pass_err is not None else None)
    _check(rc, "qlra")
    return U, S, V, pass_err, workspace


def qlra_power_iteration(A, k, p, q, seed, **kw):
    """Randomized subspace iteration with q power iterations (Alg. 1): the subspace scheme with
    a budget of 2 q + 2 passes."""
    return qlra(A, k, p, 2 * q + 2, QLRA_SUBSPACE, seed, **kw)


def qlra_block_krylov_q(A, k, p, q, seed, **kw):
    """Block Krylov with q iterations (Alg. 3): the pass-efficient block Krylov scheme with a
    budget of 2 q + 2 passes, which spans the same subspace."""
    return qlra(A, k, p, 2 * q + 2, QLRA_BLOCK_KRYLOV, seed, **kw)


def qlra_complete_workspace_size(m, n, rank, p, pass_budget, scheme, sigma, precision=QLRA_FP32, transpose=False,
                                 sketch=QLRA_SKETCH_QUATERNION):
    o = Opts(precision, 0, None, None, 0, 0, 1 if transpose else 0, sketch)
    out = ctypes.c_size_t()
    _check(_lib.qlra_complete_workspace_size(m, n, rank, p, pass_budget, SCHEMES.get(scheme, scheme), float(sigma),
                                             ctypes.byref(o), ctypes.byref(out)), "qlra_complete_workspace_size")
    return out.value


def qlra_complete(M, mask, rank, p, pass_budget, scheme, seed, iters, sigma=0.0, X=None, fit=None, workspace=None,
                  stream=None, precision=QLRA_FP32, graph=False, transpose=False, sketch=QLRA_SKETCH_QUATERNION):
    """Quaternion matrix completion (Sec. 7) of M (4, m, n) FP32 observed where the (m, n) uint8
    `mask` is nonzero: `iters` alternating updates with the rank-`rank` approximation and, for
    sigma > 0, Gaussian smoothing after each.  Returns (X, fit, workspace); enqueued on `stream`
    without synchronisation.  fit=False skips the per-iteration misfits."""
    scheme = SCHEMES.get(scheme, scheme)
    m, n = M.shape[1], M.shape[2]
    dev = M.device
    pm, ldm, mps = _planes(M, m, n, "M")
    if mask.dtype != torch.uint8 or tuple(mask.shape) != (m, n) or not mask.is_cuda:
        raise ValueError(f"mask: expected a ({m}, {n}) uint8 device tensor")
    if n > 1 and mask.stride(1) != 1:
        raise ValueError("mask: the last dimension must be contiguous")
    ldk = mask.stride(0) if m > 1 else n
    if X is None:
        X = torch.empty((4, m, n), dtype=torch.float32, device=dev)
    px, ldx, xps = _planes(X, m, n, "X")
    if fit is None:
        fit = torch.empty(iters, dtype=torch.float64, device=dev)
    elif fit is False:
        fit = None
    need = qlra_complete_workspace_size(m, n, rank, p, pass_budget, scheme, sigma, precision, transpose, sketch)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    o = Opts(precision, 0, _stream_ptr(stream), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
             1 if graph else 0, 1 if transpose else 0, sketch)
    rc = _lib.qlra_complete(pm, m, n, ldm, mps, ctypes.c_void_p(mask.data_ptr()), ldk, rank, p, pass_budget, scheme,
                            ctypes.c_uint64(seed), iters, float(sigma), ctypes.byref(o), px, ldx, xps,
                            ctypes.c_void_p(fit.data_ptr()) if fit is not None else None)
    _check(rc, "qlra_complete")
    return X, fit, workspace


def qlra_status(workspace, stream=None):
    st = ctypes.c_int()
    _check(_lib.qlra_status(ctypes.c_void_p(workspace.data_ptr()), _stream_ptr(stream), ctypes.byref(st)),
           "qlra_status")
    return st.value


def qlra_omega(seed, n, l, out=None, stream=None, device="cuda"):
    if out is None:
        out = torch.empty((4, n, l), dtype=torch.float32, device=device)
    po, ld, ps = _planes(out, n, l, "Om")
    _check(_lib.qlra_omega(ctypes.c_uint64(seed), n, l, po, ld, ps, _stream_ptr(stream)), "qlra_omega")
    return out


def qlra_omega_srht(seed, n, l, out=None, stream=None, device="cuda"):
    """The structured sketch (subsampled randomized Hadamard transform), FP32 planes (4, n, l)."""
    if out is None:
        out = torch.empty((4, n, l), dtype=torch.float32, device=device)
    po, ld, ps = _planes(out, n, l, "Om")
    _check(_lib.qlra_omega_srht(ctypes.c_uint64(seed), n, l, po, ld, ps, _stream_ptr(stream)), "qlra_omega_srht")
    return out


def qlra_qgemm_workspace(op, m, n, w, device="cuda"):
    """A zero-filled workspace for qlra_qgemm with these sizes (reusable across calls)."""
    need = ctypes.c_size_t()
    _check(_lib.qlra_qgemm_workspace_size(op, m, n, w, ctypes.byref(need)), "qlra_qgemm_workspace_size")
    return torch.zeros(max(need.value, 1), dtype=torch.uint8, device=device)


def qlra_qgemm(op, A, B, C=None, stream=None, workspace=None):
    """op 0: C = A B (A m x n, B n x w); op 1: C = A^H B (B m x w)."""
    m, n = A.shape[1], A.shape[2]
    w = B.shape[2]
    rows = m if op == 0 else n
    kdim = n if op == 0 else m
    if C is None:
        C = torch.empty((4, rows, w), dtype=torch.float32, device=A.device)
    pa, lda, aps = _planes(A, m, n, "A")
    pb, ldb, bps = _planes(B, kdim, w, "B")
    pc, ldc, cps = _planes(C, rows, w, "C")
    ws = workspace if workspace is not None else qlra_qgemm_workspace(op, m, n, w, A.device)
    _check(_lib.qlra_qgemm(op, pa, m, n, lda, aps, pb, w, ldb, bps, pc, ldc, cps, ctypes.c_void_p(ws.data_ptr()),
                           ws.numel(), _stream_ptr(stream)), "qlra_qgemm")
    return C


_LP_DTYPES = {QLRA_BF16: torch.bfloat16, QLRA_FP16: torch.float16}


def qlra_lowp_copy_bytes(m, n):
    a, t = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.qlra_lowp_copy_bytes(m, n, ctypes.byref(a), ctypes.byref(t)), "qlra_lowp_copy_bytes")
    return a.value, t.value


def qlra_lowp_copy(A, precision, scale=None, stream=None):
    """BF16 / FP16 copies of A (4, m, n) in the tiled layout of include/qlra.h: returns flat tensors
    (Alo, Alo_t), each scaled by the device scalar `scale` (a one-element float32 tensor, or None
    for 1)."""
    m, n = A.shape[1], A.shape[2]
    pa, lda, aps = _planes(A, m, n, "A")
    dt = _LP_DTYPES[precision]
    na, nt = qlra_lowp_copy_bytes(m, n)
    Alo = torch.empty(na // 2, dtype=dt, device=A.device)
    Alo_t = torch.empty(nt // 2, dtype=dt, device=A.device)
    _check(_lib.qlra_lowp_copy(pa, m, n, lda, aps, precision,
                               ctypes.c_void_p(scale.data_ptr()) if scale is not None else None,
                               ctypes.c_void_p(Alo.data_ptr()), ctypes.c_void_p(Alo_t.data_ptr()), _stream_ptr(stream)),
           "qlra_lowp_copy")
    return Alo, Alo_t


def qlra_qgemm_lp_workspace(op, precision, m, n, w, device="cuda"):
    need = ctypes.c_size_t()
    _check(_lib.qlra_qgemm_lp_workspace_size(op, precision, m, n, w, ctypes.byref(need)),
           "qlra_qgemm_lp_workspace_size")
    return _workspace(need.value, device)


def qlra_qgemm_lp(op, precision, Alo, m, n, B, C=None, inv_scale=None, stream=None, workspace=None):
    """Reduced-precision view product: op 0: C = A B from the copy of A; op 1: C = A^H B from the
    copy of A^T (both from qlra_lowp_copy).  B and C are FP32."""
    rows, kdim = (m, n) if op == 0 else (n, m)
    need = qlra_lowp_copy_bytes(m, n)[op] // 2
    if Alo.dtype != _LP_DTYPES[precision] or Alo.numel() < need or not Alo.is_contiguous():
        raise ValueError("Alo: expected the copy made by qlra_lowp_copy for this op")
    w = B.shape[2]
    if C is None:
        C = torch.empty((4, rows, w), dtype=torch.float32, device=B.device)
    pb, ldb, bps = _planes(B, kdim, w, "B")
    pc, ldc, cps = _planes(C, rows, w, "C")
    ws = workspace if workspace is not None else qlra_qgemm_lp_workspace(op, precision, m, n, w, B.device)
    _check(_lib.qlra_qgemm_lp(op, precision, ctypes.c_void_p(Alo.data_ptr()), m, n, pb, w, ldb, bps, pc, ldc, cps,
                              ctypes.c_void_p(inv_scale.data_ptr()) if inv_scale is not None else None,
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)), "qlra_qgemm_lp")
    return C


def qlra_lowp_copy_residual(A, precision, scale=None, stream=None):
    """The residual copies (s a minus its rounded value, rounded) of A (4, m, n) in the layout of
    qlra_lowp_copy: returns flat tensors (Alo_res, Alo_t_res)."""
    m, n = A.shape[1], A.shape[2]
    pa, lda, aps = _planes(A, m, n, "A")
    dt = _LP_DTYPES[precision]
    na, nt = qlra_lowp_copy_bytes(m, n)
    Ar = torch.empty(na // 2, dtype=dt, device=A.device)
    Ar_t = torch.empty(nt // 2, dtype=dt, device=A.device)
    _check(_lib.qlra_lowp_copy_residual(pa, m, n, lda, aps, precision,
                                        ctypes.c_void_p(scale.data_ptr()) if scale is not None else None,
                                        ctypes.c_void_p(Ar.data_ptr()), ctypes.c_void_p(Ar_t.data_ptr()),
                                        _stream_ptr(stream)), "qlra_lowp_copy_residual")
    return Ar, Ar_t


def qlra_qgemm_split_workspace(op, precision, m, n, w, device="cuda"):
    size = ctypes.c_size_t()
    _check(_lib.qlra_qgemm_split_workspace_size(op, precision, m, n, w, ctypes.byref(size)),
           "qlra_qgemm_split_workspace_size")
    return torch.empty(max(size.value, 1), dtype=torch.uint8, device=device)


def qlra_qgemm_split(op, precision, Alo, Alo_res, m, n, B, C=None, inv_scale=None, stream=None, workspace=None):
    """Split-form view product (qlra_qgemm_lp's product as Ahi Bhi + Ahi Blo + Alo Bhi) from a
    copy and its residual copy."""
    rows, kdim = (m, n) if op == 0 else (n, m)
    need = qlra_lowp_copy_bytes(m, n)[op] // 2
    for t, what in ((Alo, "Alo"), (Alo_res, "Alo_res")):
        if t.dtype != _LP_DTYPES[precision] or t.numel() < need or not t.is_contiguous():
            raise ValueError(f"{what}: expected a copy made for this op")
    w = B.shape[2]
    if C is None:
        C = torch.empty((4, rows, w), dtype=torch.float32, device=B.device)
    pb, ldb, bps = _planes(B, kdim, w, "B")
    pc, ldc, cps = _planes(C, rows, w, "C")
    ws = workspace if workspace is not None else qlra_qgemm_split_workspace(op, precision, m, n, w, B.device)
    _check(_lib.qlra_qgemm_split(op, precision, ctypes.c_void_p(Alo.data_ptr()), ctypes.c_void_p(Alo_res.data_ptr()),
                                 m, n, pb, w, ldb, bps, pc, ldc, cps,
                                 ctypes.c_void_p(inv_scale.data_ptr()) if inv_scale is not None else None,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)), "qlra_qgemm_split")
    return C


def qlra_cholqr(Y, Q=None, stream=None, return_workspace=False, want_r=True):
    """Thin QR of Y (4, m, w) FP32: returns (Q, R) (R None when want_r is False), and the
    workspace (its status words) with return_workspace."""
    m, w = Y.shape[1], Y.shape[2]
    if Q is None:
        Q = torch.empty((4, m, w), dtype=torch.float32, device=Y.device)
    R = torch.empty((4, w, w), dtype=torch.float64, device=Y.device) if want_r else None
    py, ldy, yps = _planes(Y, m, w, "Y")
    pq, ldq, qps = _planes(Q, m, w, "Q")
    need = ctypes.c_size_t()
    _check(_lib.qlra_cholqr_workspace_size(m, w, ctypes.byref(need)), "qlra_cholqr_workspace_size")
    ws = _workspace(need.value, Y.device)
    _check(_lib.qlra_cholqr(py, m, w, ldy, yps, pq, ldq, qps, ctypes.c_void_p(R.data_ptr()) if want_r else None,
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)), "qlra_cholqr")
    if return_workspace:
        return Q, R, ws
    return Q, R


def qlra_qsvd(R, vectors=True, stream=None):
    w = R.shape[1]
    R = R.contiguous()
    if R.dtype != torch.float64 or tuple(R.shape) != (4, w, w):
        raise ValueError("R must be a (4, w, w) float64 tensor")
    S = torch.empty(w, dtype=torch.float64, device=R.device)
    Uh = torch.empty((4, w, w), dtype=torch.float64, device=R.device) if vectors else None
    Vh = torch.empty((4, w, w), dtype=torch.float64, device=R.device) if vectors else None
    need = ctypes.c_size_t()
    _check(_lib.qlra_qsvd_workspace_size(w, ctypes.byref(need)), "qlra_qsvd_workspace_size")
    ws = _workspace(need.value, R.device)
    _check(_lib.qlra_qsvd(ctypes.c_void_p(R.data_ptr()), w,
                          ctypes.c_void_p(Uh.data_ptr()) if vectors else None, ctypes.c_void_p(S.data_ptr()),
                          ctypes.c_void_p(Vh.data_ptr()) if vectors else None,
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)), "qlra_qsvd")
    return Uh, S, Vh


def server_clock():
    return _lib.qlra_server_clock()


class Server:
    """Continuous-batching server of the library (include/qlra.h).  submit() returns a ticket;
    the caller keeps A and the outputs alive until poll() reports the request done."""

    def __init__(self, hbm_bytes, max_active=8, graphs=False):
        o = ServerOpts(int(hbm_bytes), int(max_active), 1 if graphs else 0)
        h = ctypes.c_void_p()
        _check(_lib.qlra_server_create(ctypes.byref(o), ctypes.byref(h)), "qlra_server_create")
        self._h = h
        self._keep = {}

    def submit(self, A, k, p, pass_budget, scheme, seed, U=None, S=None, V=None, pass_err=None, estimate=True,
               precision=QLRA_FP32, arrival_time=0.0):
        scheme = SCHEMES.get(scheme, scheme)
        m, n = A.shape[1], A.shape[2]
        dev = A.device
        pa, lda, aps = _planes(A, m, n, "A")
        U = U if U is not None else torch.empty((4, m, k), dtype=torch.float32, device=dev)
        V = V if V is not None else torch.empty((4, n, k), dtype=torch.float32, device=dev)
        S = S if S is not None else torch.empty(k, dtype=torch.float64, device=dev)
        if estimate and pass_err is None:
            pass_err = torch.empty(pass_budget, dtype=torch.float64, device=dev)
        pu, ldu, ups = _planes(U, m, k, "U")
        pv, ldv, vps = _planes(V, n, k, "V")
        r = Request(pa, m, n, lda, aps, k, p, pass_budget, scheme, ctypes.c_uint64(seed), precision, pu, ldu, ups,
                    ctypes.c_void_p(S.data_ptr()), pv, ldv, vps,
                    ctypes.c_void_p(pass_err.data_ptr()) if pass_err is not None else None, float(arrival_time))
        t = ctypes.c_uint64()
        _check(_lib.qlra_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "qlra_server_submit")
        self._keep[t.value] = (A, U, S, V, pass_err)
        return t.value

    def poll(self, ticket, wait=False):
        """None while running; (status, latency_s, (U, S, V, pass_err)) once done."""
        done, st, lat = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(_lib.qlra_server_poll(self._h, ctypes.c_uint64(ticket), 1 if wait else 0, ctypes.byref(done),
                                     ctypes.byref(st), ctypes.byref(lat)), "qlra_server_poll")
        if not done.value:
            return None
        A, U, S, V, e = self._keep.pop(ticket)
        return st.value, lat.value, (U, S, V, e)

    def wait(self, ticket):
        """Block until the request is done: (status, latency_s, (U, S, V, pass_err))."""
        st, lat = ctypes.c_int(), ctypes.c_double()
        _check(_lib.qlra_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(st), ctypes.byref(lat)),
               "qlra_server_wait")
        A, U, S, V, e = self._keep.pop(ticket)
        return st.value, lat.value, (U, S, V, e)

    def drain(self):
        _check(_lib.qlra_server_drain(self._h), "qlra_server_drain")

    def stats(self):
        s = ServerStats()
        _check(_lib.qlra_server_stats(self._h, ctypes.byref(s)), "qlra_server_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            _check(_lib.qlra_server_destroy(self._h), "qlra_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
