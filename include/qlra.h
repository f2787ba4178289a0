/*
 * qlra.h -- C ABI of the MI355X (gfx950) library for pass-efficient randomized
 * low-rank approximation of quaternion matrices (arXiv 2507.13731).
 *
 * The problem (Sec. 3): given a quaternion matrix A (m x n), a target rank k,
 * an oversampling p and a budget of v passes (views) over A, return an
 * approximate truncated QSVD  A ~ U diag(S) V^H  (eq. (qsvd)) with U (m x k)
 * and V (n x k) having orthonormal columns and S real and descending.
 *
 * Storage of every quaternion matrix X = X0 + X1 i + X2 j + X3 k (Sec. 2):
 * four real planes; plane p starts at X + p * plane_stride (in elements), each
 * plane row-major with leading dimension ld (elements) >= cols.
 *
 * Memory: all matrix pointers are DEVICE pointers on the current HIP device,
 * allocated and owned by the caller (for example torch.empty((4, m, n),
 * device="cuda") on ROCm).  The library never allocates device memory in a
 * solve; scratch memory comes from the caller's workspace.
 *
 * Execution: every call enqueues its kernels on the caller's stream (NULL =
 * the null stream) and returns without waiting, unless stated otherwise.
 * Outputs are valid once that stream has completed the work.  Argument errors
 * are reported synchronously through the return value; numerical breakdown is
 * reported through a device-side status word in the workspace, read with
 * qlra_status() (which synchronises the stream).
 *
 * Thread safety: calls on different workspaces may run concurrently; two
 * calls that share a workspace must be ordered on one stream.
 */
#ifndef QLRA_H
#define QLRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    QLRA_OK = 0,
    QLRA_E_ARG = 1,          /* invalid argument (sizes, strides, null pointer)          */
    QLRA_E_WORKSPACE = 2,    /* workspace missing, too small or misaligned               */
    QLRA_E_HIP = 3,          /* a HIP runtime call failed                                */
    QLRA_E_NUMERIC = 4,      /* non-finite data or Cholesky breakdown after the fallback */
    QLRA_E_TOO_LARGE = 5,    /* request larger than the supported maximum                */
    QLRA_E_UNSUPPORTED = 6   /* option not supported by this build                       */
};

/* Schemes.  QLRA_SUBSPACE is Alg. 2 (randomized truncated SVD with an
 * arbitrary number of passes, Sec. 3); QLRA_BLOCK_KRYLOV is Alg. 4 (block
 * randomized truncated SVD with an arbitrary number of views, Sec. 5). */
enum { QLRA_SUBSPACE = 0, QLRA_BLOCK_KRYLOV = 1 };

/* Arithmetic of the pass products (the views).  QLRA_FP32: FP32 inputs,
 * FP32 MFMA.  QLRA_BF16 / QLRA_FP16: views 1 .. v-2 multiply BF16 / FP16
 * copies of A (made once per solve; FP16 with a power-of-two scale from
 * ||A||_F) by a rounded copy of the thin operand on MFMA with FP32
 * accumulation; views v-1 and v stay FP32 (v = 2 is plain FP32).
 * QLRA_BF16_SPLIT / QLRA_FP16_SPLIT: views 1 .. v-2 as for QLRA_BF16 /
 * QLRA_FP16, and views v-1 and v (every view when v = 2) as three products
 * of the same type on MFMA, a_hi b_hi + a_hi b_lo + a_lo b_hi with x_hi the
 * rounded x and x_lo the rounded residual x - x_hi, FP32 accumulation: about
 * 16 (BF16) or 22 (FP16) significant bits per product instead of FP32's 24,
 * at a fraction of the FP32 MFMA time.  The Gram, Cholesky and small QSVD
 * steps are always FP64. */
enum { QLRA_FP32 = 0, QLRA_BF16 = 1, QLRA_FP16 = 2, QLRA_BF16_SPLIT = 3, QLRA_FP16_SPLIT = 4 };

/* The sketch.  QLRA_SKETCH_QUATERNION: the Gaussian quaternion test matrix of
 * Sec. 2 (four independent N(0, 1) planes; see qlra_omega()).  QLRA_SKETCH_REAL:
 * a real Gaussian test matrix, as the experiments of Sec. 8 use; it is the real
 * plane of the quaternion sketch with the other three planes zero, and its
 * first view costs a quarter of the matrix products.  QLRA_SKETCH_SRHT: a
 * structured real sketch, the subsampled randomized Hadamard transform of
 * qlra_omega_srht(), one of the faster generators the cost section (Sec. 6)
 * mentions; the error bounds of Lemma 1 and Thm. 3 do not cover it. */
enum { QLRA_SKETCH_QUATERNION = 0, QLRA_SKETCH_REAL = 1, QLRA_SKETCH_SRHT = 2 };

typedef struct {
    int pass_precision;      /* QLRA_FP32, QLRA_BF16 or QLRA_FP16 (see above)         */
    int estimate_passes;     /* nonzero: compute the per-pass error estimates         */
    void* stream;            /* hipStream_t; NULL = null stream                      */
    void* workspace;         /* device memory, 256-byte aligned                       */
    size_t workspace_bytes;  /* size of workspace                                     */
    int graph;               /* nonzero: capture the solve as a HIP graph on first use and
                                replay it when a later call has identical arguments (same
                                pointers, sizes, seed); the library keeps up to 32 graphs  */
    int transpose;           /* nonzero: run the scheme on A^H (the sketch is m x l and the
                                first view is A^H Omega, cheaper when n > m); U and V are
                                still the left and right factors of A.  The results differ
                                from transpose = 0 (another sketch), not the guarantees     */
    int sketch;              /* QLRA_SKETCH_QUATERNION (0) or QLRA_SKETCH_REAL             */
} qlra_opts_t;

/* Bytes of device workspace a qlra() call with these sizes needs (written to
 * *bytes).  Depends only on m, n, k, p, pass_budget, scheme, opts->pass_precision
 * and opts->transpose (opts may be NULL: FP32 with estimates, A as given).
 *
 * The classical forms are budgets of these two schemes: randomized subspace
 * iteration with q power iterations (Alg. 1) is QLRA_SUBSPACE with
 * pass_budget = 2q + 2, and the block Krylov method with q iterations (Alg. 3)
 * spans the same subspace as QLRA_BLOCK_KRYLOV with pass_budget = 2q + 2. */
int qlra_workspace_size(int64_t m, int64_t n, int k, int p, int pass_budget, int scheme,
                        const qlra_opts_t* opts, size_t* bytes);

/*
 * The truncated QSVD of A by Alg. 2 (scheme QLRA_SUBSPACE) or Alg. 4
 * (QLRA_BLOCK_KRYLOV), using exactly pass_budget products with A or A^H.
 *
 *   A        m x n, FP32 planes (lda >= n, a_plane_stride >= m * lda), read only.
 *   k, p     target rank k >= 1 and oversampling p >= 0 with k + p <= min(m, n)
 *            (Lemma 1 and Lemma 2, Sec. 4); the sketch has l = k + p columns.
 *   pass_budget  v >= 2 (Alg. 2, Alg. 4).
 *   seed     key of the Gaussian sketch Omega (n x l, Sec. 2, Def. of a Gaussian
 *            quaternion matrix), generated by qlra_omega().
 *   U        m x k FP32 planes (ldu >= k), written.
 *   S        k doubles, descending, written.
 *   V        n x k FP32 planes (ldv >= k), written.
 *   pass_err v doubles or NULL.  Entry i (0-based) estimates
 *            ||A - A_i||_F / ||A||_F for the rank-k approximation A_i available
 *            after view i+1; entry 0 is NaN (the sketch is not orthonormal), the
 *            last entry is the error of the returned U diag(S) V^H.
 *
 * Singular vectors are normalised so that, in every column of V, the entry of
 * largest modulus (lowest row on ties) is real and positive.
 * Returns QLRA_OK or an error code; see the header comment for when outputs
 * are valid.
 */
int qlra(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_plane_stride,
         int k, int p, int pass_budget, int scheme, uint64_t seed, const qlra_opts_t* opts,
         float* U, int64_t ldu, int64_t u_plane_stride,
         double* S,
         float* V, int64_t ldv, int64_t v_plane_stride,
         double* pass_err);

/* ---- quaternion matrix completion (Sec. 7) ----
 *
 * Fills in the unobserved entries of M (m x n, FP32 planes, read only) by the
 * alternating updates of the completion problem:
 *   C^(0) = mask . M;  for t = 0 .. iters-1:
 *     X^(t)   = G_sigma * L(C^(t))
 *     C^(t+1) = mask . M + (1 - mask) . X^(t)
 * with L(C) = U diag(S) V^H the rank-`rank` approximation of C computed exactly
 * as qlra(C, rank, p, pass_budget, scheme, seed, opts) computes it (the same
 * sketch every iteration), and G_sigma the separable Gaussian smoothing the
 * image experiments of Sec. 8 apply after each iteration: along every row and
 * then every column of each plane, the normalised taps
 * exp(-t^2 / (2 sigma^2)), t = -r .. r, r = ceil(3 sigma), edge entries
 * replicated.  sigma <= 0: no smoothing; r must be <= 8 (sigma <= 8/3), else
 * QLRA_E_UNSUPPORTED.
 *
 *   mask     m x n bytes (row-major, ld_mask >= n, device): nonzero = observed.
 *   X        m x n FP32 planes, written: X^(iters-1).
 *   fit      iters doubles (device) or NULL: fit[t] = ||mask . (X^(t) - M)||_F
 *            / ||mask . M||_F (NaN when nothing is observed).
 *   opts     pass_precision, transpose, sketch, stream and workspace as for
 *            qlra(); estimate_passes is ignored; graph != 0 captures one
 *            iteration as a HIP graph (cached under the call's arguments) and
 *            replays it iters times.
 * The workspace (qlra_complete_workspace_size() bytes) holds C, the factors and
 * the solve's own pieces; qlra_status() on it reports QLRA_E_NUMERIC when any
 * iteration's solve broke down (e.g. an all-zero C).  Argument codes as for
 * qlra(); iters >= 1. */
int qlra_complete_workspace_size(int64_t m, int64_t n, int rank, int p, int pass_budget, int scheme, double sigma,
                                 const qlra_opts_t* opts, size_t* bytes);
int qlra_complete(const float* M, int64_t m, int64_t n, int64_t ldm, int64_t m_plane_stride,
                  const unsigned char* mask, int64_t ld_mask,
                  int rank, int p, int pass_budget, int scheme, uint64_t seed,
                  int iters, double sigma, const qlra_opts_t* opts,
                  float* X, int64_t ldx, int64_t x_plane_stride,
                  double* fit);

/* ---- continuous-batching server ----
 *
 * A scheduler thread (one per server, on the device current at creation) serves qlra()
 * requests as they arrive.  Admission is in arrival order, when one of max_active slots is free
 * and the request's workspace (qlra_workspace_size()) fits in the server's HBM arena of
 * hbm_bytes (allocated at creation; first fit).  Every admitted request advances by one
 * view-step per scheduler tick (step s = view s+1 with its QR; the first step also the set-up,
 * the last one the final QSVD); each slot has its own stream pair, so steps of different
 * requests overlap on the device.  graphs != 0: each step's launches are captured into a HIP
 * graph and launched as one.  The per-request state (bases, factors, Grams) stays on the device
 * from admission to completion.  Results are identical to a qlra() call with the same
 * arguments.  A, U, S, V and pass_err are device memory owned by the caller and must stay valid
 * until the request is reported done.  Errors: qlra_server_submit returns QLRA_E_TOO_LARGE when
 * the workspace exceeds the arena, the qlra() argument codes otherwise; a request's own status
 * (QLRA_OK, QLRA_E_NUMERIC, QLRA_E_HIP) comes from qlra_server_poll. */
typedef struct qlra_server qlra_server_t;

typedef struct {
    size_t hbm_bytes;        /* device arena for request workspaces                        */
    int max_active;          /* slots: requests in flight at once (1 .. 64); each slot's
                                stream runs on one of the process's hardware queues (4 by
                                default on ROCm), and slots beyond that share queues and
                                serialize: 4 slots gave the highest throughput here          */
    int graphs;              /* nonzero: launch each view-step as a captured HIP graph      */
} qlra_server_opts_t;

typedef struct {
    const float* A; int64_t m, n, lda, a_plane_stride;
    int k, p, pass_budget, scheme;
    uint64_t seed;
    int pass_precision;      /* QLRA_FP32, QLRA_BF16 or QLRA_FP16                          */
    float* U; int64_t ldu, u_plane_stride;
    double* S;
    float* V; int64_t ldv, v_plane_stride;
    double* pass_err;        /* v doubles or NULL (no estimates)                            */
    double arrival_time;     /* qlra_server_clock() time of arrival; <= 0: time of submit   */
} qlra_request_t;

typedef struct {
    int pending, active, max_active_seen;
    size_t arena_bytes, arena_used, max_arena_used;
    int64_t ticks;
} qlra_server_stats_t;

int qlra_server_create(const qlra_server_opts_t* opts, qlra_server_t** server);
/* Queue a request; *ticket identifies it.  Thread safe. */
int qlra_server_submit(qlra_server_t* server, const qlra_request_t* request, uint64_t* ticket);
/* *done = 1 once the request's results are complete in device memory (wait != 0: block until
 * then); its status and latency (completion minus arrival, seconds) are reported once, after
 * which the ticket is forgotten. */
int qlra_server_poll(qlra_server_t* server, uint64_t ticket, int wait, int* done, int* status,
                     double* latency_s);
/* Block until the request is done, then report it as qlra_server_poll(wait = 1) does. */
int qlra_server_wait(qlra_server_t* server, uint64_t ticket, int* status, double* latency_s);
/* Block until every submitted request has completed. */
int qlra_server_drain(qlra_server_t* server);
int qlra_server_stats(qlra_server_t* server, qlra_server_stats_t* stats);
/* Finish the queued work, stop the scheduler and free the arena and streams. */
int qlra_server_destroy(qlra_server_t* server);
/* Seconds on the server's monotonic clock (for arrival times). */
double qlra_server_clock(void);

/* Device status word of the last solve (or completion) that used this
 * workspace: QLRA_OK or QLRA_E_NUMERIC.  Synchronises `stream` (hipStream_t, may be NULL) first. */
int qlra_status(const void* workspace, void* stream, int* status);

/* Human-readable text of a status code (static storage). */
const char* qlra_strerror(int status);

/* ---- the steps of the method, exposed for testing and composition ---- */

/* Gaussian quaternion sketch (Sec. 2, Def. of a Gaussian quaternion matrix):
 * entry (i, j), i < n, j < l, of the four FP32 planes of Om is a function of
 * (seed, i, j) only: Philox4x32-10 (Salmon et al., SC'11) at counter
 * (i, j, 0, 0) with key (seed mod 2^32, seed div 2^32); the four words give
 * u_t = (2 (x_t >> 9) + 1) 2^-24; planes 0, 1 = sqrt(-2 ln u0) (cos, sin)(2 pi u1),
 * planes 2, 3 = sqrt(-2 ln u2) (cos, sin)(2 pi u3), evaluated in FP64 with
 * series-based log/sin/cos and Newton square roots, rounded to FP32. */
int qlra_omega(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t plane_stride,
               void* stream);

/* The structured sketch: Om (n x l, l <= n <= 2^30) = D H S / sqrt(l) in the
 * real plane, the other three planes zero.  n_pad = the smallest power of two
 * >= n; H the +-1 Hadamard matrix of order n_pad, entry (i, s) =
 * (-1)^popcount(i & s), rows i < n; D = diag(d_i) with d_i = -1 when bit 0 of
 * word 0 of Philox4x32-10 at counter (i, 0, 2, 0) (key as for qlra_omega) is
 * set, else +1; S picks the columns s_j = pi(j), j < l, where pi is a keyed
 * permutation of [0, n_pad): with h = ceil(log2(n_pad) / 2), x = (L, R) in
 * h-bit halves goes through four Feistel rounds (round r: (L, R) ->
 * (R, L xor F), F = word 0 of Philox at counter (R, r, 3, 0) masked to h
 * bits), repeated while the result is >= n_pad.  The scale is the FP32
 * rounding of 1 / sqrt(l). */
int qlra_omega_srht(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t plane_stride,
                    void* stream);

/* Quaternion product of one view (Sec. 2, eq. (1)):
 *   op = 0:  C (m x w) = A (m x n) * B (n x w)
 *   op = 1:  C (n x w) = A^H * B (m x w), A^H the conjugate transpose.
 * FP32 planes in and out, FP32 MFMA with FP32 accumulation.  Needs
 * qlra_qgemm_workspace_size() bytes of device workspace (split-K partial tiles,
 * summed in a fixed order by a second kernel; no initialisation needed). */
int qlra_qgemm_workspace_size(int op, int64_t m, int64_t n, int64_t w, size_t* bytes);
int qlra_qgemm(int op, const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_ps,
               const float* B, int64_t w, int64_t ldb, int64_t b_ps,
               float* C, int64_t ldc, int64_t c_ps,
               void* workspace, size_t workspace_bytes, void* stream);

/* Low-precision copies of A for the reduced-precision views: Alo holds s A
 * (rows m, reduction n) and Alo_t holds s A^T (rows n, reduction m), elements
 * BF16 (precision QLRA_BF16) or FP16 (QLRA_FP16) rounded to nearest even, in
 * the tiled order the view kernel reads: for a copy with R rows and K
 * reduction elements, tiles of 16 rows x 64 elements, tile (rt, kt) of plane p
 * at element ((rt * ceil(K/64) + kt) * 4 + p) * 1024, and inside a tile
 * element (r, kk) at (kk / 32) * 512 + ((kk / 8) % 4) * 128 + r * 8 + kk % 8;
 * padding rows and elements are zero.  Sizes from qlra_lowp_copy_bytes();
 * device memory owned by the caller.  scale: device float holding s (NULL:
 * s = 1). */
int qlra_lowp_copy_bytes(int64_t m, int64_t n, size_t* alo_bytes, size_t* alo_t_bytes);
int qlra_lowp_copy(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_ps, int precision,
                   const float* scale, void* Alo, void* Alo_t, void* stream);

/* Reduced-precision view product (Sec. 2, eq. (1)) from a copy made by
 * qlra_lowp_copy():
 *   op = 0:  C (m x w) = A * B (n x w)    with Alo = the copy of A
 *   op = 1:  C (n x w) = A^H * B (m x w)  with Alo = the copy of A^T
 * B is FP32 (rounded to the copy's type in the kernel), C is FP32, the
 * products accumulate in FP32 on MFMA and are multiplied by *inv_scale
 * (device float; NULL: 1).  Needs qlra_qgemm_lp_workspace_size()
 * bytes of device workspace (the rounded B and split-K partial tiles). */
int qlra_qgemm_lp_workspace_size(int op, int precision, int64_t m, int64_t n, int64_t w, size_t* bytes);
int qlra_qgemm_lp(int op, int precision, const void* Alo, int64_t m, int64_t n,
                  const float* B, int64_t w, int64_t ldb, int64_t b_ps,
                  float* C, int64_t ldc, int64_t c_ps, const float* inv_scale,
                  void* workspace, size_t workspace_bytes, void* stream);

/* The split form's pieces (precisions QLRA_BF16_SPLIT / QLRA_FP16_SPLIT).
 * qlra_lowp_copy_residual() writes, in the layout of qlra_lowp_copy() and
 * with the same scale, the residual copies: each element s a minus its
 * rounded value (FP32), rounded to BF16 (precision QLRA_BF16) or FP16
 * (QLRA_FP16); buffers of qlra_lowp_copy_bytes() bytes.
 * qlra_qgemm_split() is the view product of qlra_qgemm_lp() computed as
 * Ahi Bhi + Ahi Blo + Alo Bhi (Sec. 2, eq. (1) for each product), with Ahi
 * the copy (Alo argument), Alo the residual copy (Alo_res), Bhi the rounded
 * B and Blo the rounded B - Bhi, FP32 accumulation, times *inv_scale.  Needs
 * qlra_qgemm_split_workspace_size() bytes of workspace (the rounded B and its
 * residual, and three sets of split-K partial tiles, summed in a fixed
 * order). */
int qlra_lowp_copy_residual(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_ps, int precision,
                            const float* scale, void* Alo_res, void* Alo_t_res, void* stream);
int qlra_qgemm_split_workspace_size(int op, int precision, int64_t m, int64_t n, int64_t w, size_t* bytes);
int qlra_qgemm_split(int op, int precision, const void* Alo, const void* Alo_res, int64_t m, int64_t n,
                     const float* B, int64_t w, int64_t ldb, int64_t b_ps,
                     float* C, int64_t ldc, int64_t c_ps, const float* inv_scale,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Thin quaternion QR (eq. (QQR)) of a tall Y (m x w, m >= w) by CholeskyQR2:
 * FP64 Gram Y^H Y, FP64 quaternion Cholesky, FP64 triangular inverse, applied
 * twice; a shifted first round replaces a failed one (shifted CholeskyQR), and
 * one more round follows it.  Q (m x w, FP32) has orthonormal columns; R
 * (w x w, FP64 planes, ld = w, plane stride w*w) is upper triangular with a
 * real positive diagonal and Y = Q R.  Q may alias Y.  R may be NULL: then
 * the second round's Cholesky and triangular solve (w <= 96) or product with
 * R^{-1} (larger w) run only when the first round left max |Q^H Q - I| above
 * 1e-7 (decided on the device; the decision is int 3 of the workspace, 1 =
 * ran; for w > 96 int 4 holds its opposite).  Int 1 of the workspace is 1
 * when the first round was shifted, int 0 has bit 1 (value 2) set when the
 * factorization failed even with the shift. */
int qlra_cholqr_workspace_size(int64_t m, int64_t w, size_t* bytes);
int qlra_cholqr(const float* Y, int64_t m, int64_t w, int64_t ldy, int64_t y_ps,
                float* Q, int64_t ldq, int64_t q_ps, double* R,
                void* workspace, size_t workspace_bytes, void* stream);

/* Full QSVD (eq. (qsvd)) of a small square quaternion matrix R (w x w, FP64
 * planes, ld = w, plane stride w*w): R = Uh diag(S) Vh^H, S descending, Uh and
 * Vh w x w (same layout), FP64 throughout.  For w <= 96 it is taken from the
 * Hermitian eigendecomposition of R^H R (Householder tridiagonalisation with
 * quaternion reflectors): S_j = sqrt(lambda_j), Vh the eigenvectors, Uh =
 * R Vh diag(1/S); the eigenvalues carry an absolute error of about
 * u64 S_1^2, so S_j is accurate to about u64 S_1^2 / S_j (relative accuracy
 * for S_j >> sqrt(u64) S_1) and Uh's columns of negligible S_j are not
 * meaningful.  Above 96, by one-sided Jacobi on the complex adjoint kept in
 * structure-preserving (quaternion) form, accurate to u64 S_1 in every S_j. */
int qlra_qsvd_workspace_size(int64_t w, size_t* bytes);
int qlra_qsvd(const double* R, int64_t w, double* Uh, double* S, double* Vh,
              void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* QLRA_H */
