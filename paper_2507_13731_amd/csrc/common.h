// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "qlra.h"

namespace qlra_impl {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Plane-major quaternion matrix view: plane p at ptr + p * ps, row-major, leading dim ld.
template <class T>
struct QView {
    T* ptr;
    int64_t ld;
    int64_t ps;
};

// Which product a qgemm launch computes.
enum QOp { OP_NN = 0, OP_HN = 1 };   // C = A B  |  C = A^H B

// How the result is stored.
enum QStore { ST_SET = 0, ST_SUB = 1 };   // C = R  |  C = C - R

// Arithmetic of a qgemm launch.  MATH_BF16 / MATH_F16: A is a low-precision copy laid out as
// the rows of the output (for OP_HN the transposed copy A^T; op then only selects the
// conjugation signs) in the tiled layout of lowp_copy_launch (lda, aps unused), B is FP32 and
// converted per launch, C is FP32 and multiplied by *cscale.
// MATH_BF16X3 / MATH_F16X3: the split form, A_hi B_hi + A_hi B_lo + A_lo B_hi with A = the
// low-precision copy and A_lo its residual copy (same layout), B_hi / B_lo the rounded thin
// operand and its rounded residual.
enum QMath { MATH_F32 = 0, MATH_F64 = 1, MATH_BF16 = 2, MATH_F16 = 3, MATH_BF16X3 = 4, MATH_F16X3 = 5 };

struct QgemmDesc {
    QOp op;
    QMath math;
    QStore store;
    int a_f64, b_f64, c_f64;   // element types of A, B, C (0 = float, 1 = double)
    const void* A; int64_t lda, aps;
    const void* B; int64_t ldb, bps;
    void* C; int64_t ldc, cps;
    int64_t M, N, K;           // C is M x N, reduction length K
    const int* skip_flag;      // if non-null and *skip_flag == 0 the launch does nothing
    const float* cscale;       // low-precision math: device scalar the result is multiplied by
    double* fro2_part;         // FP32 A X only (optional): per-wave sums of squares of A, fro2_slots(d) entries
    int b_real;                // FP32 views: B has zero imaginary planes (only its real plane is read)
    const void* A_lo;          // split forms: the residual copy of A
    int b_upper;               // FP64 A B: B is upper triangular (rows below a column's diagonal are not read)
};

// Device workspace carved into aligned regions.
struct Arena {
    char* base;
    size_t size;
    size_t used;
    bool dry;   // sizing pass: count only; regions get placeholder addresses (never dereferenced)
    void* take(size_t bytes) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + ((bytes + 255) & ~size_t(255));
        if (dry) return reinterpret_cast<void*>(static_cast<uintptr_t>(kDryBase + off));
        return base + off;
    }
    static constexpr uintptr_t kDryBase = uintptr_t(1) << 44;
};

// Scratch a qgemm launch needs: split-K partials and per-tile counters.
struct QgemmScratch {
    void* partial;          // bytes given by qgemm_scratch_bytes
    unsigned* counters;     // qgemm_counter_count entries, zero at rest
};

size_t qgemm_partial_bytes(const QgemmDesc& d);    // split-K partials (+ the converted B, low precision)
size_t fro2_slots(const QgemmDesc& d);             // entries of fro2_part written by an FP32 A X launch
size_t qgemm_counter_count(const QgemmDesc& d);
hipError_t qgemm_launch(const QgemmDesc& d, const QgemmScratch& s, hipStream_t st);

// Low-precision copies of A (m x n, four FP32 planes): Alo (rows m, reduction n) and Alo_t =
// A^T (rows n, reduction m), both scaled by *scale (read on the device; null: 1), elements
// bf16 or fp16 by prec (QLRA_BF16 / QLRA_FP16), in the tiled MFMA-operand layout (16 x 64 tiles,
// four planes per tile; lowp_copy_elems(rows, k) elements each, padding zero).
size_t lowp_copy_elems(int64_t rows, int64_t k);
// Ar, Ar_t (both or neither): the residual copies (s a - (float)(rounded s a), rounded), written in
// the same pass; Alo = Alo_t = null with Ar given: the residual copies alone.  fro (optional):
// lowp_copy_fro_slots(m, n) partial sums of squares of A, summed by fro2_final_launch.
size_t lowp_copy_fro_slots(int64_t m, int64_t n);
hipError_t lowp_copy_launch(const float* A, int64_t m, int64_t n, int64_t lda, int64_t aps, int prec, void* Alo,
                            void* Alo_t, const float* scale, hipStream_t st, void* Ar = nullptr, void* Ar_t = nullptr,
                            double* fro = nullptr);
// FP16 scale from ||A||_F^2 (nA2): scale = 2^e with e = 14 - ceil(log2 ||A||_F) (so that every
// |a| * scale <= 2^14), inv = 1 / scale; BF16: scale = inv = 1.
hipError_t lowp_scale_launch(const double* nA2, int prec, float* scale, float* inv, hipStream_t st);

hipError_t omega_launch(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t ps,
                        hipStream_t st, int real_only = 0);
// The structured sketch (subsampled randomized Hadamard transform, real plane; l <= n).
hipError_t omega_srht_launch(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t ps, hipStream_t st);

// Cholesky of a Hermitian quaternion Gram G (w x w FP64 planes, ld = w): G (+ shift I) = R^H R,
// Rout = R * Rprev (Rprev null: Rout = R) and Rinv = R^{-1} (if non-null).  If the unshifted
// factorization breaks down and allow_shift is set, it is redone with
// shift = shift_scale * trace(G) and *shift_out (if non-null) is set to 1 (else 0).  A failure
// that remains ORs 2 into *status.  If gate is non-null and *gate == 0 nothing is done.  work:
// 8*w*w doubles (the new factor when Rprev is given, R^{-1} when Rinv is null).
hipError_t chol_launch(const double* G, int64_t w, double* Rout, double* Rinv, const double* Rprev,
                       double* work, int* status, int* shift_out, const int* gate, int allow_shift,
                       double shift_scale, hipStream_t st);
int chol_lds_max();   // chol_launch handles w <= chol_lds_max(); larger orders are factored by blocks
// The same factorization and inverse in place inside larger matrices: G, R and Rinv with their own
// row strides and plane strides; with band_w > 0 the w x w block sits at column band_off of a row
// band of width band_w whose other columns are set to zero in R and Rinv (w <= chol_lds_max()).
hipError_t chol_inv_launch(const double* G, int64_t ldg, int64_t gps, int64_t w, double* R, int64_t ldr, int64_t rps,
                           double* Rinv, int64_t ldi, int64_t ips, int64_t band_off, int64_t band_w, int* status,
                           int* shift_out, const int* gate, int allow_shift, double shift_scale, hipStream_t st);
// Pieces of the blocked factorization (each does nothing when gate && *gate == 0):
// W = G with a real diagonal (+ shift_scale * trace(G) on it when `shifted`);
hipError_t chol_prep_launch(const double* G, int64_t w, double* W, const int* gate, int shifted, double shift_scale,
                            hipStream_t st);
// dst (rows x cols FP64 planes) = src;
hipError_t copy_f64_planes_launch(const double* src, int64_t lds, int64_t sps, double* dst, int64_t ldd, int64_t dps,
                                  int64_t rows, int64_t cols, const int* gate, hipStream_t st);
// p[0..count) = 0;
hipError_t zero_f64_launch(double* p, int64_t count, const int* gate, hipStream_t st);
// *dst = (*src != 0).
hipError_t flag_nonzero_launch(int* dst, const int* src, hipStream_t st);
// *gate_out = 1 when max |G - I| (G a w x w Gram, FP64 planes) exceeds tol or is not finite, else
// 0; always 0 when gate_in is given and *gate_in == 0.  *gate_not (if given) = 1 - *gate_out.
hipError_t orth_gate_launch(const double* G, int64_t w, double tol, int* gate_out, const int* gate_in,
                            hipStream_t st, int* gate_not = nullptr);
// Cholesky alone for w <= chol_reg_max(), factor to R (no inverse) and to Rpk, R's upper
// triangle packed by rows with the four components of an entry side by side (4 w (w + 1) / 2
// doubles, the input of trsm_launch); same status, shift and gate behaviour as chol_launch.
// With gate_out, the kernel first sets *gate_out = 1 when max |G - I| exceeds gate_tol or is not
// finite, else 0, and factors only when it is 1.
int chol_reg_max();
hipError_t chol_reg_launch(const double* G, int64_t w, double* R, double* Rpk, int* status, int* shift_out,
                           const int* gate, int allow_shift, double shift_scale, hipStream_t st,
                           int* gate_out = nullptr, double gate_tol = 0.0);
// Q = Y R^{-1} (rows x w FP32 planes, Q may alias Y), R upper triangular FP64 given packed as
// chol_reg_launch writes it, w <= chol_reg_max().
hipError_t trsm_launch(const float* Y, int64_t ldy, int64_t yps, float* Q, int64_t ldq, int64_t qps,
                       const double* Rpk, int64_t w, int64_t rows, const int* gate, hipStream_t st);
// Rout = R2 * R1 (upper triangular w x w); nothing if gate && !*gate.
hipError_t rmul_launch(const double* R2, const double* R1, double* Rout, int64_t w,
                       const int* gate, hipStream_t st);
// dst = src (FP64 planes w x w) when gate is null or *gate != 0.
hipError_t rcopy_launch(const double* src, double* dst, int64_t w, const int* gate, hipStream_t st);

// dst (rows x cols FP32 planes) = src, when gate is null or *gate != 0.
hipError_t copy_planes_launch(const float* src, int64_t lds, int64_t sps, float* dst, int64_t ldd,
                              int64_t dps, int64_t rows, int64_t cols, const int* gate, hipStream_t st);
// dst[0..count) = src[0..count) (FP64).
hipError_t copy_f64_launch(const double* src, double* dst, int64_t count, hipStream_t st);
// p[0..count) = value.
hipError_t fill_int_launch(int* p, int64_t count, int value, hipStream_t st);
// status[0 .. nstatus) = 0, counters[0 .. ncnt) = 0 and *nan_at = NaN (if nan_at) in one launch.
hipError_t solve_prologue_launch(int* status, int nstatus, unsigned* counters, int64_t ncnt, double* nan_at,
                                 hipStream_t st);

// One-sided Jacobi QSVD of X (w x w FP64 planes): S descending, U = left vectors, V right
// vectors (if want_vectors).  work: 8*w*w + 2*w doubles.
hipError_t qsvd_launch(const double* X, int64_t w, double* U, double* S, double* V, double* work,
                       int want_vectors, hipStream_t st);
size_t qsvd_work_doubles(int64_t w);

// Hermitian quaternion eigendecomposition of G (w x w FP64 planes, full storage, w <= heig_max()):
// lam descending, E eigenvectors as columns (may be null).  work: heig_work_doubles(1).
int heig_max();
size_t heig_work_doubles(int64_t nprob);
hipError_t heig_launch(const double* G, int64_t w, double* lam, double* E, double* work, hipStream_t st);
// QSVD of a small square X (w <= heig_max()) through the eigendecomposition of X^H X.
hipError_t qsvd_gram_launch(const double* X, int64_t w, double* U, double* S, double* V, double* work,
                            hipStream_t st);
size_t qsvd_gram_work_doubles(int64_t w);
// S_j = sqrt(max(lam_j, 0)) (j < k) and, when E is given, Wk = E[:, :k] diag(1 / S) (w x k FP64
// planes, ld k), from lam (descending) and E (w x >= k, ld lde) of a Gram's eigendecomposition;
// with est also *est = sqrt(max(0, *nA2 - sum_{j<k} S_j^2) / *nA2) (as estimate_launch).
// Columns with S_j <= kDegenerate S_0 (rounding level of an FP32 view: no direction left in
// Y E_j / S_j) get zero columns in Wk.  *degen (if given) = 1 when there is any such column or
// S_{k-1} < S_0 / 64 (the factor Y Wk is then re-orthonormalised), else 0.
constexpr double kDegenerate = 1.0 / 1048576.0;   // 2^-20
hipError_t svals_launch(const double* lam, const double* E, int64_t lde, int64_t w, int k, double* S, double* Wk,
                        hipStream_t st, const double* nA2 = nullptr, double* est = nullptr, int* degen = nullptr);
// Column j < k of X (rows x k FP32 planes) with S_j <= kDegenerate S_0 is overwritten by a fixed
// pseudo-random vector (entries in [-1, 1) from a hash of (row, column, plane)), when *flag != 0.
hipError_t fill_degenerate_launch(float* X, int64_t rows, int k, int64_t ldx, int64_t xps, const double* S,
                                  const int* flag, hipStream_t st);
// Larger orders (up to heig_big_max()): lam (W, descending) and, if E, the nout eigenvectors of
// the largest eigenvalues (W x nout, ld nout).  work: heig_big_work_doubles(W, nvec) doubles with
// nvec >= nout vector slots (0 without vectors).
int heig_big_max();
size_t heig_big_work_doubles(int64_t W, int64_t nvec);
hipError_t heig_big_launch(const double* G, int64_t W, double* lam, double* E, int64_t nout, double* work,
                           int64_t nvec, hipStream_t st);
// The per-pass estimates of nprob Grams of one order W <= heig_big_max() (problem b at
// G + b * gstride) in one launch sequence: e[b] = sqrt(max(0, nA2 - sum of the k largest
// eigenvalues of G_b) / nA2).  work: nprob * heig_big_work_doubles(W, 0) doubles.
hipError_t heig_big_estimates_launch(const double* G, int64_t gstride, int64_t W, int nprob, int k,
                                     const double* nA2, double* e, double* work, hipStream_t st);
// Estimates of nprob problems from their Grams (problem b at G + b * gstride, w <= heig_max()):
// e[b] = sqrt(max(0, nA2 - sum of the k largest eigenvalues of G_b) / nA2).
// work: heig_work_doubles(nprob).
hipError_t estimate_batch_launch(const double* G, int64_t gstride, int64_t w, int nprob, int k, const double* nA2,
                                 double* e, double* work, hipStream_t st);

// The batched problems of estimate_batch_launch (nest of them) and one more, problem nest, whose
// eigenvalues (descending, lam) and eigenvectors (E, may be null) are wanted, in one launch
// sequence; work: heig_work_doubles(nest + 1).
hipError_t heig_with_estimates_launch(const double* G, int64_t gstride, int64_t w, int nest, int k, const double* nA2,
                                      double* e, double* lam, double* E, double* work, hipStream_t st);

// e = sqrt(max(0, nA2 - sum_{j<k} S_j^2) / nA2)
hipError_t estimate_launch(const double* S, int k, const double* nA2, double* e, hipStream_t st);

// ||A||_F^2 (FP64) into *out; partial: 1024 doubles.
// ||A||_F^2 = the sum, in order, of nb partial sums (deterministic)
hipError_t fro2_final_launch(const double* partial, int64_t nb, double* out, hipStream_t st);
hipError_t fro2_launch(const float* A, int64_t m, int64_t n, int64_t lda, int64_t aps,
                       double* partial, double* out, hipStream_t st);

// Canonical phase: for each column j < k of V (n x k), the entry of largest modulus (lowest row
// on ties) is made real positive by right-multiplying columns j of U and V by its conjugate phase.
size_t phase_work_bytes(int64_t n, int k);
hipError_t phase_launch(float* U, int64_t m, int64_t ldu, int64_t ups, float* V, int64_t n, int64_t ldv,
                        int64_t vps, int k, void* work, hipStream_t st);

// Quaternion matrix completion (Sec. 7), one iteration after the rank-R step: C = mask . M +
// (1 - mask) . X with X = G_sigma * (U diag(S) V^H) (separable Gaussian, radius ceil(3 sigma) <=
// kCompleteMaxRadius, edges replicated; sigma <= 0: no smoothing), X written to the output when
// *iter == iters - 1, fit[*iter] = ||mask . (X - M)||_F / ||mask . M||_F (fit may be null), then
// *iter += 1.  part: 2 * complete_blocks(m, n, radius) doubles.
constexpr int kCompleteMaxRadius = 8;
struct CompleteStep {
    const float* U; int64_t ldu, ups;
    const double* S;
    const float* V; int64_t ldv, vps;
    int R;
    const float* M; int64_t ldm, mps;
    const unsigned char* mask; int64_t ldk;
    float* C; int64_t ldc, cps;
    float* X; int64_t ldx, xps;
    int64_t m, n;
    double sigma;
    int* iter; int iters;
    double* part;
    double* fit;
};
int complete_radius(double sigma);
int complete_tile(int radius);
int64_t complete_blocks(int64_t m, int64_t n, int radius);
hipError_t complete_step_launch(const CompleteStep& s, hipStream_t st);
// C = mask . M, *iter = 0, status[0] = 0.
hipError_t complete_init_launch(const float* M, int64_t ldm, int64_t mps, const unsigned char* mask, int64_t ldk,
                                int64_t m, int64_t n, float* C, int64_t ldc, int64_t cps, int* iter, int* status,
                                hipStream_t st);
// dst[0] |= src[0].
hipError_t status_or_launch(int* dst, const int* src, hipStream_t st);

// The solve behind qlra() (same arguments).  no_alloc: create no streams, events or graphs (the
// per-pass estimates run on the solve's stream, opts->graph is ignored).
int solve_entry(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_plane_stride, int k, int p,
                int pass_budget, int scheme, uint64_t seed, const qlra_opts_t* opts, float* U, int64_t ldu,
                int64_t u_plane_stride, double* S, float* V, int64_t ldv, int64_t v_plane_stride, double* pass_err,
                bool no_alloc);

}  // namespace qlra_impl
