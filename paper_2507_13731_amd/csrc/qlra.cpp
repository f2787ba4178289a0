// Host side of the library: argument checks, workspace layout and the per-view launch sequence
// of Alg. 2 (Sec. 3) and Alg. 4 (Sec. 5), plus the C ABI declared in include/qlra.h.
//
// Everything between views stays on the device: a solve is a fixed sequence of kernel
// launches on the caller's stream with no host synchronisation.  The per-pass error
// estimates need the singular values of each view's R, i.e. the eigenvalues of the view's
// Gram, which the CholeskyQR forms anyway: each intermediate view leaves its Gram in a slot,
// and one batched eigenvalue launch on a side stream (fork/join with events) turns all of
// them into estimates while the final QSVD runs on the main stream.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena_alloc.h"
#include "common.h"

namespace qlra_impl {
namespace {

// ---------------------------------------------------------------------------------------
// launch context: a dry run only sizes the qgemm scratch

struct Ctx {
    bool dry = false;
    hipStream_t st = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    QgemmScratch scr{};
    size_t part_need = 0, cnt_need = 0;
    hipError_t err = hipSuccess;
    int* status = nullptr;          // status[0]: sticky solve status bits, status[1..]: gates
    double* chol_work = nullptr;
    double* G = nullptr;            // Gram, wmax x wmax
    double* R1 = nullptr;
    double* R2 = nullptr;
    double* blk = nullptr;          // blocked Cholesky: one (<= chol_lds_max())^2 quaternion FP64 block
    double* Rinv = nullptr;
    float* T2 = nullptr;            // CholQR intermediate, rows x wmax
    int64_t T2_rows = 0;
    double* Rjunk = nullptr;        // R of QRs whose factor is not needed
    // Step mode: a solve is v steps, step s holding view s + 1 (the first also the set-up, the
    // last also the final QSVD).  step_only >= 0 enqueues that step's launches only, so that a
    // scheduler can advance many solves one view at a time.
    int views = 0;                  // views begun so far
    int step_only = -1;
    bool forked = false;            // this step forked work to the side stream
    bool fro_next = false;          // the next FP32 A X view also forms ||A||_F^2
    int step_now() const { return views > 0 ? views - 1 : 0; }
    bool live() const { return !dry && (step_only < 0 || step_now() == step_only); }
};

void note(Ctx& c, hipError_t e) {
    if (c.err == hipSuccess && e != hipSuccess) c.err = e;
}

void qg(Ctx& c, const QgemmDesc& d) {
    if (c.dry) {
        c.part_need = std::max(c.part_need, qgemm_partial_bytes(d));
        c.cnt_need = std::max(c.cnt_need, qgemm_counter_count(d));
        return;
    }
    if (!c.live()) return;
    note(c, qgemm_launch(d, c.scr, c.st));
}

QgemmDesc desc(QOp op, QMath math, const void* A, int64_t lda, int64_t aps, int a64, const void* B, int64_t ldb,
               int64_t bps, int b64, void* C, int64_t ldc, int64_t cps, int c64, int64_t M, int64_t N, int64_t K,
               QStore store = ST_SET, const int* skip = nullptr) {
    QgemmDesc d{};
    d.op = op; d.math = math; d.store = store;
    d.a_f64 = a64; d.b_f64 = b64; d.c_f64 = c64;
    d.A = A; d.lda = lda; d.aps = aps;
    d.B = B; d.ldb = ldb; d.bps = bps;
    d.C = C; d.ldc = ldc; d.cps = cps;
    d.M = M; d.N = N; d.K = K;
    d.skip_flag = skip;
    return d;
}

// eigenvector slots of the large-order solver: the k wanted ones and as many again below them,
// so that a cluster reaching under the k-th eigenvalue is orthogonalised whole
int64_t big_nvec(int64_t w, int64_t k) { return std::min<int64_t>(w, 2 * k); }

double shift_scale(int64_t rows, int64_t w) {
    // Shifted CholeskyQR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020):
    // s = 11 (m w + w (w + 1)) u ||Y||_2^2, with ||Y||_F^2 = trace(Y^H Y) as the bound.
    return 11.0 * ((double)rows * w + (double)w * (w + 1)) * 1.1102230246251565e-16;
}

size_t chol_blk_doubles() { return (size_t)4 * chol_lds_max() * chol_lds_max(); }

// Cholesky G (+ shift I) = R^H R and R^{-1} for orders above chol_lds_max(): right-looking by
// diagonal blocks of at most chol_lds_max().  Block k: R_kk and R_kk^{-1} from the register
// kernel on the updated diagonal block, in place (it also clears the rest of its row band in R
// and R^{-1}), the block row R_k,rest = R_kk^{-H} W_k,rest and the trailing update
// W_rest -= R_k,rest^H R_k,rest as FP64 products; then the off-diagonal blocks of R^{-1}, column
// by column from the diagonal up: X_ij = -X_ii (R_i,(i+1..j) X_(i+1..j),j).  With allow_shift a
// breakdown of the unshifted pass (flag in status[2]) reruns everything, gated on that flag, on
// G + shift_scale tr(G) I; a breakdown that remains ORs 2 into status[0].  Rout = R Rprev when
// Rprev is given.  Scratch: chol_work (W), blk, and R2 when Rprev is given.  With `outer`,
// nothing is computed (and *shift_out is set to 0) when *outer == 0.
void chol_blocked(Ctx& c, const double* G, int64_t w, double* Rout, double* Rinv, const double* Rprev, int* shift_out,
                  int allow_shift, double sscale, const int* outer = nullptr) {
    const int64_t nb = (w + chol_lds_max() - 1) / chol_lds_max();
    const int64_t b = (w + nb - 1) / nb;
    const int64_t ps = w * w;
    double* W = c.chol_work;
    double* Rw = Rprev ? c.R2 : Rout;
    double* T = c.blk;
    int* fail = c.status ? c.status + 2 : nullptr;
    if (c.live() && allow_shift) note(c, fill_int_launch(fail, 1, 0, c.st));
    for (int attempt = 0; attempt < (allow_shift ? 2 : 1); attempt++) {
        // the retry runs only when the first attempt ran and broke down
        const int* gate = attempt ? fail : outer;
        int* st = (allow_shift && attempt == 0) ? fail : c.status;
        if (c.live()) note(c, chol_prep_launch(G, w, W, gate, attempt, sscale, c.st));
        for (int64_t k0 = 0; k0 < w; k0 += b) {
            const int64_t kb = std::min(b, w - k0), k1 = k0 + kb, rest = w - k1;
            double* Ik = Rinv + k0 * w + k0;
            if (c.live())
                note(c, chol_inv_launch(W + k0 * w + k0, w, ps, kb, Rw + k0 * w + k0, w, ps, Ik, w, ps, k0, w, st,
                                        nullptr, gate, 0, 0.0, c.st));
            if (rest > 0) {
                qg(c, desc(OP_HN, MATH_F64, Ik, w, ps, 1, W + k0 * w + k1, w, ps, 1, Rw + k0 * w + k1, w, ps, 1,
                           kb, rest, kb, ST_SET, gate));
                qg(c, desc(OP_HN, MATH_F64, Rw + k0 * w + k1, w, ps, 1, Rw + k0 * w + k1, w, ps, 1, W + k1 * w + k1, w,
                           ps, 1, rest, rest, kb, ST_SUB, gate));
            }
        }
        for (int64_t j0 = b; j0 < w; j0 += b) {
            const int64_t jb = std::min(b, w - j0);
            for (int64_t i0 = j0 - b; i0 >= 0; i0 -= b) {
                const int64_t t0 = i0 + b, tk = j0 + jb - t0;
                qg(c, desc(OP_NN, MATH_F64, Rw + i0 * w + t0, w, ps, 1, Rinv + t0 * w + j0, w, ps, 1, T, jb, b * jb, 1,
                           b, jb, tk, ST_SET, gate));
                qg(c, desc(OP_NN, MATH_F64, Rinv + i0 * w + i0, w, ps, 1, T, jb, b * jb, 1, Rinv + i0 * w + j0, w, ps, 1,
                           b, jb, b, ST_SUB, gate));
            }
        }
    }
    if (Rprev) qg(c, desc(OP_NN, MATH_F64, Rw, w, ps, 1, Rprev, w, ps, 1, Rout, w, ps, 1, w, w, w, ST_SET, outer));
    if (shift_out && allow_shift && c.live()) note(c, flag_nonzero_launch(shift_out, fail, c.st));
}

// One CholeskyQR round on X (rows x w, in place), every launch gated on *gate (0: nothing done):
// G = X^H X, G = Rx^H Rx, X = X Rx^{-1} and, when R is given, R = Rx R.  allow_shift: a breakdown
// of the factorization is retried with a shift (for orders above chol_reg_max() the retry is a
// second set of launches, each costing a few microseconds even when its gate is closed).
// Scratch: G, R1, R2, chol_work, Rinv, blk and T2.
void cholqr_round_gated(Ctx& c, float* X, int64_t rows, int64_t w, int64_t ldx, int64_t xps, double* R,
                        const int* gate, int allow_shift = 1) {
    const int64_t ps = w * w;
    qg(c, desc(OP_HN, MATH_F64, X, ldx, xps, 0, X, ldx, xps, 0, c.G, w, ps, 1, w, w, rows, ST_SET, gate));
    if (w <= chol_reg_max()) {
        if (c.live()) {
            note(c, chol_reg_launch(c.G, w, c.R1, c.chol_work, c.status, nullptr, gate, allow_shift, shift_scale(rows, w),
                                    c.st));
            note(c, trsm_launch(X, ldx, xps, X, ldx, xps, c.chol_work, w, rows, gate, c.st));
            if (R) {
                note(c, rmul_launch(c.R1, R, c.R2, w, gate, c.st));
                note(c, rcopy_launch(c.R2, R, w, gate, c.st));
            }
        }
        return;
    }
    chol_blocked(c, c.G, w, c.R1, c.Rinv, R, nullptr, allow_shift, shift_scale(rows, w), gate);
    QgemmDesc ap = desc(OP_NN, MATH_F64, X, ldx, xps, 0, c.Rinv, w, ps, 1, c.T2, w, rows * w, 0, rows, w, w, ST_SET, gate);
    ap.b_upper = 1;                            // R^{-1} is upper triangular
    qg(c, ap);
    if (c.live()) {
        note(c, copy_planes_launch(c.T2, w, rows * w, X, ldx, xps, rows, w, gate, c.st));
        if (R) note(c, rcopy_launch(c.R1, R, w, gate, c.st));
    }
}

// Thin QR of Y (rows x w): Q (ld ldq, plane stride qps) and R (w x w FP64, ld w; may be null
// when only Q is wanted), Q may alias Y.  Each round is CholeskyQR with an FP64 Gram (exact
// products of FP32 data), FP64 Cholesky and an FP64 application of R^{-1}.  With an FP64
// Cholesky the orthogonality error of one round is about u64 cond(Y)^2 + u32, so for the views
// (cond(Y) <= 1e4, the FP32 storage of Q dominating) one round suffices; rounds = 2 is
// CholeskyQR2 (R = R2 R1), used where the basis is returned or stacked.  A breakdown in the
// first round is retried with a shift (shifted CholeskyQR).  G0 (optional) receives the first
// round's Gram Y^H Y (w x w, FP64 planes) and keeps it.
// For w <= chol_reg_max() R^{-1} is applied by forward substitution along the rows of Y;
// larger factors are inverted explicitly and applied as a product.
void cholqr(Ctx& c, const float* Y, int64_t rows, int64_t w, int64_t ldy, int64_t yps, float* Q, int64_t ldq,
            int64_t qps, double* R, int rounds, double* G0 = nullptr) {
    const int64_t tps = rows * w;
    int* shifted = c.status ? c.status + 1 : nullptr;
    const float* src = Y;
    int64_t lds = ldy, sps = yps;
    const bool small = w <= chol_reg_max();
    // Without a wanted R, the second round of the small path runs only where the first left the
    // basis measurably non-orthonormal: its Gram Q^H Q is formed anyway, and when max |Q^H Q - I|
    // <= 1e-7 (a second round would move Q by less than its FP32 rounding) the Cholesky and the
    // triangular solve of that round are skipped on the device.  The first round then writes Q
    // directly and the second works in place.
    // The larger orders gate their second round the same way: the first round writes T2, whose
    // Gram goes through the orthogonality test (a separate launch, gate in status[3], its
    // opposite in status[4]); then either the factorization and the product T2 R^{-1} into Q run,
    // or T2 is copied to Q.  (The product cannot work in place: other column tiles still read
    // the rows it writes.)
    const bool gated = rounds == 2 && !R && c.status;
    int* gate = gated ? c.status + 3 : nullptr;
    int* gate_not = gated ? c.status + 4 : nullptr;
    const double* Rprev = nullptr;
    for (int round = 0; round < rounds; round++) {
        const bool last = round == rounds - 1;
        const bool to_q = last || (gated && small);
        float* dst = to_q ? Q : c.T2;
        const int64_t ldd = to_q ? ldq : w, dps = to_q ? qps : tps;
        double* G = (round == 0 && G0) ? G0 : c.G;
        qg(c, desc(OP_HN, MATH_F64, src, lds, sps, 0, src, lds, sps, 0, G, w, w * w, 1, w, w, rows));
        if (small) {
            // this round's own factor; the product R2 R1 is formed at the end when R is wanted
            double* Rr = (rounds == 1 && R) ? R : (round == 0 ? c.R1 : c.R2);
            int* g = (gated && round == 1) ? gate : nullptr;
            if (c.live()) {
                // the packed copy of the factor for the triangular solve goes to chol_work, which
                // only the larger orders use otherwise; a gated round's Cholesky forms the gate
                note(c, chol_reg_launch(G, w, Rr, c.chol_work, c.status, round == 0 ? shifted : nullptr, nullptr,
                                        round == 0 ? 1 : 0, shift_scale(rows, w), c.st, g, 1e-7));
                note(c, trsm_launch(src, lds, sps, dst, ldd, dps, c.chol_work, w, rows, g, c.st));
            }
        } else {
            double* Rout = last ? (R ? R : c.Rjunk) : c.R1;
            // the product R = R2 R1 only when R is wanted
            const double* rp = R ? Rprev : nullptr;
            const int* g = (gated && round == 1) ? gate : nullptr;
            if (g && c.live()) {
                note(c, orth_gate_launch(G, w, 1e-7, gate, nullptr, c.st, gate_not));
                note(c, copy_planes_launch(src, lds, sps, Q, ldq, qps, rows, w, gate_not, c.st));
            }
            if (w <= chol_lds_max()) {
                if (c.live())
                    note(c, chol_launch(G, w, Rout, c.Rinv, rp, c.chol_work, c.status,
                                        round == 0 ? shifted : nullptr, g, round == 0 ? 1 : 0,
                                        shift_scale(rows, w), c.st));
            } else {
                chol_blocked(c, G, w, Rout, c.Rinv, rp, round == 0 ? shifted : nullptr, round == 0 ? 1 : 0,
                             shift_scale(rows, w), g);
            }
            QgemmDesc ap = desc(OP_NN, MATH_F64, src, lds, sps, 0, c.Rinv, w, w * w, 1, dst, ldd, dps, 0, rows, w, w,
                                ST_SET, g);
            ap.b_upper = 1;                        // R^{-1} is upper triangular
            qg(c, ap);
            Rprev = Rout;
        }
        src = dst; lds = ldd; sps = dps;
    }
    if (small && rounds == 2 && R && c.live()) note(c, rmul_launch(c.R2, c.R1, R, w, nullptr, c.st));
    // A shifted first round leaves Q with a condition number up to about
    // (11 (rows w + w (w + 1)) u64)^{-1/2}, 1e4 to 1e5 at the sizes here: one more round, in place
    // and gated on the device by the shift flag (its launches do nothing when it is 0), brings
    // the loss of orthogonality to about u64 cond^2 (shifted CholeskyQR followed by CholeskyQR,
    // three rounds in all for the two-round calls as in Fukaya et al. 2020).
    // That round's Gram has a condition number of at most about 1e10, far from a breakdown in
    // FP64, so it takes no shifted retry (a failure still sets the status flag).
    if (shifted || c.dry) cholqr_round_gated(c, Q, rows, w, ldq, qps, R, shifted, 0);
}

// A returned factor of the final QSVD from the Gram (rows x k, in place): the Y side Y E_k S^{-1}
// or the X side X E_k.  Column j of the Y side carries the FP32 rounding of Y divided by S_j, an
// error of about u32 S_0 / S_j, and column j of E (either side) the FP64 eigensolver's error
// u64 S_0^2 / gap_j in the Gram's eigenvalues: both lose orthogonality when the spectrum falls
// steeply, and at the rounding level (S_j <= kDegenerate S_0, when k exceeds the numerical rank
// of A) the Y side carries no direction at all (the singular value kernel zeroed the column) and
// the eigenvectors of the degenerate cluster are arbitrary.  The singular value kernel sets
// status[5] when either can happen (S_{k-1} < S_0 / 64, where the first error reaches about
// 64 u32 = 4e-6, or a degenerate column); then the
// degenerate columns get fixed pseudo-random vectors and the factor goes through CholeskyQR2,
// all gated on that word.  The factor of a CholeskyQR is upper triangular, so a column is
// orthogonalised against the columns of larger singular values only: a kept column moves by
// its own orthogonality error, which changes U diag(S) V^H by about u32 S_0.  A degenerate
// column becomes a unit vector orthogonal to the others, as the oracle's completion of the
// basis.
void reorthonormalize(Ctx& c, float* X, int64_t rows, int64_t k, int64_t ldx, int64_t xps, const double* S) {
    int* gate = c.status ? c.status + 5 : nullptr;
    if (c.live()) note(c, fill_degenerate_launch(X, rows, (int)k, ldx, xps, S, gate, c.st));
    // no shifted retry: the factor's kept columns are orthonormal to about u32 S_0 / S_{k-1} and
    // the filled ones are independent of them, so neither round's Gram is near a breakdown
    for (int r = 0; r < 2; r++) cholqr_round_gated(c, X, rows, k, ldx, xps, nullptr, gate, 0);
}

// Orthonormalise the columns of a stack of blocks (rows x W, ld W) of width l: CholeskyQR2 of
// the first block, then for each further block block Gram-Schmidt with reorthogonalisation (two
// projections against all earlier blocks) and CholeskyQR2 of the block in place.
void orth_stack(Ctx& c, float* K, int64_t rows, int64_t W, int64_t l, double* Cbuf) {
    const int64_t kps = rows * W;
    cholqr(c, K, rows, std::min(l, W), W, kps, K, W, kps, nullptr, 2);
    for (int64_t b0 = l; b0 < W; b0 += l) {
        const int64_t lb = std::min(l, W - b0);
        float* Z = K + b0;
        for (int pass = 0; pass < 2; pass++) {
            // C = K_prev^H Z (b0 x lb, FP64), then Z -= K_prev C
            qg(c, desc(OP_HN, MATH_F64, K, W, kps, 0, Z, W, kps, 0, Cbuf, lb, b0 * lb, 1, b0, lb, rows));
            qg(c, desc(OP_NN, MATH_F64, K, W, kps, 0, Cbuf, lb, b0 * lb, 1, Z, W, kps, 0, rows, lb, b0, ST_SUB));
        }
        cholqr(c, Z, rows, lb, W, kps, Z, W, kps, nullptr, 2);
    }
}

// ---------------------------------------------------------------------------------------
// solve layout

bool prec_split(int prec) { return prec == QLRA_BF16_SPLIT || prec == QLRA_FP16_SPLIT; }
bool prec_bf(int prec) { return prec == QLRA_BF16 || prec == QLRA_BF16_SPLIT; }
enum { VIEW_F32 = 0, VIEW_LOWP = 1, VIEW_SPLIT = 2 };

struct Problem {
    // m, n, U, V: the matrix the scheme runs on (A, or A^H when transpose is set) and its factors;
    // A, mr, nr, lda, aps: A as stored
    const float* A; int64_t m, n, lda, aps;
    int transpose;
    int64_t mr, nr;
    int k, p, v, scheme;
    uint64_t seed;
    float* U; int64_t ldu, ups;
    double* S;
    float* V; int64_t ldv, vps;
    double* pass_err;
    int estimate;
    int prec;               // QLRA_FP32, QLRA_BF16 or QLRA_FP16 for views 1 .. v-2
    int sketch;             // QLRA_SKETCH_QUATERNION or QLRA_SKETCH_REAL
};

// Arithmetic of view i (1-based): the reduced-precision forms take views 1 .. v-2 from the
// low-precision copies and views v-1 and v in FP32, or in the split form.
int view_mode(const Problem& pr, int i) {
    if (pr.prec == QLRA_FP32) return VIEW_F32;
    if (pr.v > 2 && i <= pr.v - 2) return VIEW_LOWP;
    return prec_split(pr.prec) ? VIEW_SPLIT : VIEW_F32;
}

// Run the scheme on A^H: swap the logical sizes and the two factors (A^H = V S U^H).
void orient(Problem& pr, int transpose) {
    pr.mr = pr.m;
    pr.nr = pr.n;
    pr.transpose = transpose ? 1 : 0;
    if (!pr.transpose) return;
    std::swap(pr.m, pr.n);
    std::swap(pr.U, pr.V);
    std::swap(pr.ldu, pr.ldv);
    std::swap(pr.ups, pr.vps);
}

// The reduced-precision forms copy A once at the start; for BF16 (scale 1, not derived from the
// norm) that pass also forms ||A||_F^2.
bool fro_in_copy(const Problem& pr) {
    return (pr.prec == QLRA_BF16 && pr.v > 2) || pr.prec == QLRA_BF16_SPLIT;
}

struct Dims {
    int64_t l, Wk, wmax, rows_max, stack_rows;
    bool krylov, even;
    int s;
};

Dims dims_of(int64_t m, int64_t n, int k, int p, int v, int scheme) {
    Dims d{};
    d.l = (int64_t)k + p;
    d.krylov = scheme == QLRA_BLOCK_KRYLOV;
    d.even = (v % 2) == 0;
    d.s = (v - 1) / 2;
    const int64_t cap = std::min(m, n);
    if (d.krylov) {
        const int64_t nb = d.even ? v / 2 : d.s;
        d.Wk = std::min(nb * d.l, cap);
        d.stack_rows = d.even ? m : n;
    } else {
        d.Wk = d.l;
        d.stack_rows = 0;
    }
    d.wmax = std::max(d.l, d.Wk);
    d.rows_max = std::max(m, n);
    return d;
}

// Subspace scheme with l <= heig_max(): the estimates of views 2 .. v-1 ride along with the final
// eigendecomposition (one batched launch sequence on the solve's own stream, no side stream).
bool merged_estimates(const Problem& pr, const Dims& d) {
    return pr.estimate && !d.krylov && pr.v > 2 && d.l <= heig_max();
}

struct Bufs {
    int* status;            // 16 ints
    unsigned* counters;
    double* nA2;
    double* fro_part;       // 1024
    float* Om;              // n x l
    float* Q1;              // m x wmax
    float* Q2;              // n x wmax
    float* T;               // rows_max x wmax
    float* T2;              // rows_max x wmax
    float* stack;           // stack_rows x Wk
    double* G; double* R1; double* R2; double* blk; double* Rinv; double* chol_work;
    double* Rv;             // v x (l x l)
    double* Rfin;           // wmax x wmax
    double* Cbuf;           // Wk x l
    double* Lh; double* Rh; double* Sw; double* qsvd_work;
    double* side_S; double* side_work;
    double* Gs;             // Grams of views 2 .. v-1, (v - 2) x (l x l)
    double* est_work;
    double* big_work;       // the large-order eigensolver of the final view
    void* Alo; void* Alo_t;  // low-precision copies of A and A^T (views 1 .. v-2)
    void* Alo_lo; void* Alo_t_lo;  // split forms: their residual copies (views v-1 and v)
    float* lp_scale;        // [scale, 1 / scale]
    void* phase_work;       // partial arg-max of the phase normalisation
    void* partial;
};

void carve(const Problem& pr, const Dims& d, Arena& ar, Bufs& b, size_t part_bytes, size_t cnt) {
    const int64_t w2 = d.wmax * d.wmax, l2 = d.l * d.l;
    b.status = (int*)ar.take(16 * sizeof(int));
    b.counters = (unsigned*)ar.take(std::max<size_t>(cnt, 1) * sizeof(unsigned));
    b.nA2 = (double*)ar.take(sizeof(double));
    {
        // ||A||_F^2: partial sums of the separate pass (<= 1024) or of the first view's waves
        QgemmDesc v1{};
        v1.op = OP_NN; v1.math = MATH_F32; v1.M = pr.m; v1.N = d.l; v1.K = pr.n;
        size_t slots = std::max<size_t>(1024, fro2_slots(v1));
        if (fro_in_copy(pr)) slots = std::max(slots, lowp_copy_fro_slots(pr.mr, pr.nr));
        b.fro_part = (double*)ar.take(slots * sizeof(double));
    }
    b.Om = (float*)ar.take(4 * pr.n * d.l * sizeof(float));
    b.Q1 = (float*)ar.take(4 * pr.m * d.wmax * sizeof(float));
    b.Q2 = (float*)ar.take(4 * pr.n * d.wmax * sizeof(float));
    b.T = (float*)ar.take(4 * d.rows_max * d.wmax * sizeof(float));
    b.T2 = (float*)ar.take(4 * d.rows_max * d.wmax * sizeof(float));
    b.stack = d.krylov ? (float*)ar.take(4 * d.stack_rows * d.Wk * sizeof(float)) : nullptr;
    b.G = (double*)ar.take(4 * w2 * sizeof(double));
    b.R1 = (double*)ar.take(4 * w2 * sizeof(double));
    b.R2 = (double*)ar.take(4 * w2 * sizeof(double));
    b.blk = d.wmax > chol_lds_max() ? (double*)ar.take(chol_blk_doubles() * sizeof(double)) : nullptr;
    b.Rinv = (double*)ar.take(4 * w2 * sizeof(double));
    b.chol_work = (double*)ar.take(4 * w2 * sizeof(double));
    b.Rv = (double*)ar.take((size_t)pr.v * 4 * l2 * sizeof(double));
    b.Rfin = (double*)ar.take(4 * w2 * sizeof(double));
    b.Cbuf = (double*)ar.take(4 * d.Wk * d.l * sizeof(double));
    b.Lh = (double*)ar.take(4 * w2 * sizeof(double));
    b.Rh = (double*)ar.take(4 * w2 * sizeof(double));
    b.Sw = (double*)ar.take(d.wmax * sizeof(double));
    b.qsvd_work = (double*)ar.take(qsvd_work_doubles(d.wmax) * sizeof(double));
    // estimates from the Grams of views 2 .. v-1: batched for l <= heig_max(), one after another
    // with the large-order solver up to heig_big_max(), otherwise from R by the Jacobi QSVD
    const bool batched = d.l <= heig_big_max();
    const bool small_l = d.l <= heig_max();
    const int64_t nest = pr.v > 2 ? pr.v - 2 : 0;
    b.side_S = (double*)ar.take(d.l * sizeof(double));
    b.side_work = batched ? nullptr : (double*)ar.take(qsvd_work_doubles(d.l) * sizeof(double));
    const int64_t extra = merged_estimates(pr, d) ? 1 : 0;   // the final Gram joins the batch
    b.Gs = batched && nest ? (double*)ar.take((size_t)(nest + extra) * 4 * l2 * sizeof(double)) : nullptr;
    b.est_work = batched && nest ? (double*)ar.take((small_l ? heig_work_doubles(nest + extra)
                                                             : (size_t)nest * heig_big_work_doubles(d.l, 0)) *
                                                    sizeof(double))
                                 : nullptr;
    // the final QSVD of a view wider than heig_max()
    const int64_t wf = d.krylov ? d.Wk : d.l;
    b.big_work = (wf > heig_max() && wf <= heig_big_max())
                     ? (double*)ar.take(heig_big_work_doubles(wf, big_nvec(wf, pr.k)) * sizeof(double))
                     : nullptr;
    const bool split = prec_split(pr.prec);
    const bool lowp = pr.prec != QLRA_FP32 && (pr.v > 2 || split);
    b.Alo = lowp ? ar.take(lowp_copy_elems(pr.mr, pr.nr) * 2) : nullptr;
    b.Alo_t = lowp ? ar.take(lowp_copy_elems(pr.nr, pr.mr) * 2) : nullptr;
    b.Alo_lo = split ? ar.take(lowp_copy_elems(pr.mr, pr.nr) * 2) : nullptr;
    b.Alo_t_lo = split ? ar.take(lowp_copy_elems(pr.nr, pr.mr) * 2) : nullptr;
    b.lp_scale = (float*)ar.take(2 * sizeof(float));
    b.phase_work = ar.take(phase_work_bytes(pr.n, pr.k));
    b.partial = part_bytes ? ar.take(part_bytes) : nullptr;
}

// Side stream and events for the estimates, one set per (device, caller stream) pair (default
// priority): solves issued on different streams then share no side stream, so that one solve's
// join never waits behind another solve's estimates.
struct Side {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_side_mu;
std::map<std::pair<int, hipStream_t>, Side> g_sides;

hipError_t get_side(hipStream_t main, Side* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_side_mu);
    Side& sd = g_sides[std::make_pair(dev, main)];
    if (!sd.s) {
        if ((e = hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&sd.join, hipEventDisableTiming)) != hipSuccess) return e;
    }
    *out = sd;
    return hipSuccess;
}

// Captured solves, replayed when a call repeats with identical arguments (same buffers).
struct GraphKey {
    int dev;
    const void* A; int64_t m, n, lda, aps;
    int k, p, v, scheme, estimate, prec, transpose, sketch;
    uint64_t seed;
    const void* U; int64_t ldu, ups;
    const void* S;
    const void* V; int64_t ldv, vps;
    const void* pass_err;
    const void* ws;
    // completion iterations (zero for a solve): mask, output, misfit, smoothing, iteration count
    int completion;
    const void* mask; int64_t ldk;
    const void* X; int64_t ldx, xps;
    const void* fit;
    double sigma;
    int iters;
    bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    uint64_t last;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
hipStream_t g_capture[64] = {};
constexpr size_t kMaxGraphs = 32;

hipError_t get_capture_stream(int dev, hipStream_t* out) {
    if (!g_capture[dev]) {
        hipError_t e = hipStreamCreateWithFlags(&g_capture[dev], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    *out = g_capture[dev];
    return hipSuccess;
}

// The executable graph cached under `key`, or a new capture of enqueue(stream) (which returns the
// first launch error) cached under it, least recently used evicted.  Caller holds g_graph_mu.
template <class F>
hipError_t graph_for(const GraphKey& key, F enqueue, hipGraphExec_t* out) {
    for (auto& ge : g_graphs) {
        if (ge.key == key) {
            ge.last = ++g_graph_clock;
            *out = ge.exec;
            return hipSuccess;
        }
    }
    hipStream_t cap;
    hipError_t e = get_capture_stream(key.dev, &cap);
    if (e != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t le = enqueue(cap);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cap, &graph);
    if (le != hipSuccess || ee != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return le != hipSuccess ? le : (ee != hipSuccess ? ee : hipErrorUnknown);
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (g_graphs.size() >= kMaxGraphs) {
        size_t lru = 0;
        for (size_t i = 1; i < g_graphs.size(); i++)
            if (g_graphs[i].last < g_graphs[lru].last) lru = i;
        // the evicted graph may still be in flight on some stream
        if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
        (void)hipGraphExecDestroy(g_graphs[lru].exec);
        g_graphs.erase(g_graphs.begin() + (long)lru);
    }
    g_graphs.push_back(GraphEntry{key, exec, ++g_graph_clock});
    *out = exec;
    return hipSuccess;
}

// Gram slot of view `i` (1-based) for the batched estimates (views 2 .. v-1), or null.
double* gram_slot(const Bufs& b, const Problem& pr, int64_t l, int i) {
    if (!pr.estimate || !b.Gs || i < 2 || i >= pr.v) return nullptr;
    return b.Gs + (size_t)(i - 2) * 4 * l * l;
}

// Estimates of views 2 .. v-1 from their Grams on the side stream: one batched launch, or the
// large-order solver (values only) one Gram after another.
// The stream the estimates go to: the side stream, forked from the solve's stream, or without
// one (a call that may create no streams) the solve's stream itself.
// marked: the fork point was recorded earlier (fork_point).
hipStream_t est_stream(Ctx& c, bool marked = false) {
    if (!c.side) return c.st;
    c.forked = true;
    if (!marked) note(c, hipEventRecord(c.ev_fork, c.st));
    note(c, hipStreamWaitEvent(c.side, c.ev_fork, 0));
    return c.side;
}


void fork_estimates(Ctx& c, const Bufs& b, const Problem& pr, int64_t l, bool marked = false) {
    if (!c.live() || !pr.estimate || !b.Gs) return;
    const hipStream_t es = est_stream(c, marked);
    if (l <= heig_max()) {
        note(c, estimate_batch_launch(b.Gs, 4 * l * l, l, pr.v - 2, pr.k, b.nA2, pr.pass_err + 1, b.est_work, es));
        return;
    }
    note(c, heig_big_estimates_launch(b.Gs, 4 * l * l, l, pr.v - 2, pr.k, b.nA2, pr.pass_err + 1, b.est_work, es));
}

// The fork point of the batched estimates, where their Grams are complete.  When one call
// enqueues the whole solve, only the event is recorded there, and the side stream's launches are
// enqueued after the next long main-stream kernel (the last view: fork_deferred), so that the
// host's launches of the large-order estimate solver (one per reflector) never leave the main
// stream's queue empty (between the views the host only just keeps ahead of the GPU).  A solve
// enqueued one step at a time (the server) forks here, inside the step: a step is captured as a
// graph of its own, and the side stream must wait on an event recorded in the same step.
bool defer_fork(const Ctx& c) { return c.step_only < 0; }

void fork_point(Ctx& c, const Bufs& b, const Problem& pr, int64_t l) {
    if (!defer_fork(c)) {
        fork_estimates(c, b, pr, l);
        return;
    }
    if (c.live() && pr.estimate && b.Gs && c.side) note(c, hipEventRecord(c.ev_fork, c.st));
}

void fork_deferred(Ctx& c, const Bufs& b, const Problem& pr, int64_t l) {
    if (defer_fork(c)) fork_estimates(c, b, pr, l, true);
}

// Side-stream estimate of view `i` (1-based) from its R (l x l), for widths above the batched
// eigensolver's limit.
void fork_estimate(Ctx& c, const Bufs& b, const Problem& pr, const double* R, int64_t l, int i) {
    if (!c.live() || !pr.estimate || b.Gs || i >= pr.v) return;
    const hipStream_t es = est_stream(c);
    note(c, qsvd_launch(R, l, nullptr, b.side_S, nullptr, b.side_work, 0, es));
    note(c, estimate_launch(b.side_S, pr.k, b.nA2, pr.pass_err + (i - 1), es));
}

// The final TSVD of the last view's R (w x w) and the back-multiplication U = Q1 Uh,
// V = Q2 Vh (Alg. 2 and Alg. 4, last lines).  r_is_r2: even budget (A^H Q1 = Q2 R2, so
// R2 = Vh S Uh^H); otherwise A Q2 = Q1 R1 and R1 = Uh S Vh^H.
void finish(Ctx& c, const Bufs& b, const Problem& pr, const double* R, int64_t w, const float* Q1, int64_t ldq1,
            const float* Q2, int64_t ldq2, bool r_is_r2) {
    const int k = pr.k;
    if (c.live()) {
        note(c, qsvd_launch(R, w, b.Lh, b.Sw, b.Rh, b.qsvd_work, 1, c.st));
        if (pr.estimate) note(c, estimate_launch(b.Sw, k, b.nA2, pr.pass_err + (pr.v - 1), c.st));
    }
    const double* Uh = r_is_r2 ? b.Rh : b.Lh;
    const double* Vh = r_is_r2 ? b.Lh : b.Rh;
    qg(c, desc(OP_NN, MATH_F64, Q1, ldq1, pr.m * ldq1, 0, Uh, w, w * w, 1, pr.U, pr.ldu, pr.ups, 0, pr.m, k, w));
    qg(c, desc(OP_NN, MATH_F64, Q2, ldq2, pr.n * ldq2, 0, Vh, w, w * w, 1, pr.V, pr.ldv, pr.vps, 0, pr.n, k, w));
    if (c.live()) {
        note(c, phase_launch(pr.U, pr.m, pr.ldu, pr.ups, pr.V, pr.n, pr.ldv, pr.vps, k, b.phase_work, c.st));
        note(c, copy_f64_launch(b.Sw, pr.S, k, c.st));
    }
}

// The last view without its QR.  With Y = A X (or A^H X) = Q R, R^H R = Y^H Y, so the truncated
// QSVD of R (Alg. 2 and Alg. 4, last lines) follows from the eigendecomposition
// Y^H Y = E diag(lam) E^H: S = sqrt(lam_k), the Y-side factor Q Uh = Y E_k S^{-1} and the
// X-side factor X E_k.  y_is_u: odd budget (Y = A Q2 gives U, X = Q2 gives V); otherwise Y gives
// V and X = Q1 gives U.  For w <= heig_big_max() (the single-workgroup solver up to heig_max()).
void finish_gram(Ctx& c, const Bufs& b, const Problem& pr, const float* Y, int64_t rows_y, const float* X,
                 int64_t ldx, int64_t rows_x, int64_t w, bool y_is_u, bool merge_est = false) {
    const int k = pr.k;
    const bool big = w > heig_max();
    const int64_t lde = big ? k : w;     // eigenvectors in b.Rh: all w, or the k largest
    // merged: the Gram goes to the slot after the estimate Grams of views 2 .. v-1
    const int nest = pr.v - 2;
    double* Gf = merge_est ? b.Gs + (size_t)nest * 4 * w * w : c.G;
    qg(c, desc(OP_HN, MATH_F64, Y, w, rows_y * w, 0, Y, w, rows_y * w, 0, Gf, w, w * w, 1, w, w, rows_y));
    if (c.live()) {
        if (merge_est)
            note(c, heig_with_estimates_launch(b.Gs, 4 * w * w, w, nest, k, b.nA2, pr.pass_err + 1, b.Sw, b.Rh,
                                               b.est_work, c.st));
        else if (big) note(c, heig_big_launch(c.G, w, b.Sw, b.Rh, k, b.big_work, big_nvec(w, k), c.st));
        else note(c, heig_launch(c.G, w, b.Sw, b.Rh, b.qsvd_work, c.st));
        note(c, svals_launch(b.Sw, b.Rh, lde, w, k, pr.S, b.Lh, c.st, b.nA2,
                             pr.estimate ? pr.pass_err + (pr.v - 1) : nullptr, c.status ? c.status + 5 : nullptr));
    }
    float* Oy = y_is_u ? pr.U : pr.V;
    float* Ox = y_is_u ? pr.V : pr.U;
    const int64_t ldoy = y_is_u ? pr.ldu : pr.ldv, psoy = y_is_u ? pr.ups : pr.vps;
    const int64_t ldox = y_is_u ? pr.ldv : pr.ldu, psox = y_is_u ? pr.vps : pr.ups;
    qg(c, desc(OP_NN, MATH_F64, Y, w, rows_y * w, 0, b.Lh, k, w * k, 1, Oy, ldoy, psoy, 0, rows_y, k, w));
    qg(c, desc(OP_NN, MATH_F64, X, ldx, rows_x * ldx, 0, b.Rh, lde, w * lde, 1, Ox, ldox, psox, 0, rows_x, k, w));
    reorthonormalize(c, Oy, rows_y, k, ldoy, psoy, pr.S);
    reorthonormalize(c, Ox, rows_x, k, ldox, psox, pr.S);
    if (c.live()) note(c, phase_launch(pr.U, pr.m, pr.ldu, pr.ups, pr.V, pr.n, pr.ldv, pr.vps, k, b.phase_work, c.st));
}

// The product of a view alone: T = A X (forward, m x w) or T = A^H X (adjoint, n x w), ld w.
// mode VIEW_LOWP: from the BF16 / FP16 copies (A for the forward product, A^T for the adjoint
// one); VIEW_SPLIT: the split form from those copies and their residual copies.
void view_product(Ctx& c, const Problem& pr, const Bufs& b, bool adjoint, const float* X, int64_t ldx, int64_t w,
                  float* T, int mode = VIEW_F32) {
    c.views++;
    const int64_t rows_out = adjoint ? pr.n : pr.m;
    const int64_t kdim = adjoint ? pr.m : pr.n;
    // the product with A as stored: a view of A^H is the other orientation of A
    const bool adj = adjoint != (pr.transpose != 0);
    if (mode != VIEW_F32) {
        const bool bf = prec_bf(pr.prec), sp = mode == VIEW_SPLIT;
        QgemmDesc d = desc(adj ? OP_HN : OP_NN, sp ? (bf ? MATH_BF16X3 : MATH_F16X3) : (bf ? MATH_BF16 : MATH_F16),
                           adj ? b.Alo_t : b.Alo, kdim, pr.m * pr.n, 0, X, ldx, kdim * ldx, 0, T, w, rows_out * w, 0,
                           rows_out, w, kdim);
        if (sp) d.A_lo = adj ? b.Alo_t_lo : b.Alo_lo;
        d.cscale = b.lp_scale ? b.lp_scale + 1 : nullptr;
        qg(c, d);
        return;
    }
    QgemmDesc d = desc(adj ? OP_HN : OP_NN, MATH_F32, pr.A, pr.lda, pr.aps, 0, X, ldx, kdim * ldx, 0, T, w,
                       rows_out * w, 0, rows_out, w, kdim);
    d.b_real = (pr.sketch != QLRA_SKETCH_QUATERNION && X == b.Om) ? 1 : 0;    // the first view of a real sketch
    const bool fro = c.fro_next && !adj;
    if (fro) {
        d.fro2_part = b.fro_part;
        c.fro_next = false;
    }
    qg(c, d);
    if (fro && c.live()) note(c, fro2_final_launch(b.fro_part, (int64_t)fro2_slots(d), b.nA2, c.st));
}

// One view: C = A X (forward) or C = A^H X (adjoint), then its QR.
void view(Ctx& c, const Problem& pr, const Bufs& b, bool adjoint, const float* X, int64_t ldx, int64_t w, float* T,
          float* Q, int64_t ldq, double* R, int rounds = 1, double* G0 = nullptr, int mode = VIEW_F32) {
    const int64_t rows_out = adjoint ? pr.n : pr.m;
    view_product(c, pr, b, adjoint, X, ldx, w, T, mode);
    cholqr(c, T, rows_out, w, w, rows_out * w, Q, ldq, rows_out * ldq, R, rounds, G0);
}

void run_solve(Ctx& c, const Problem& pr, const Dims& d, const Bufs& b) {
    const int64_t l = d.l, l2 = l * l;
    // ||A||_F^2: fused into the first view when that is an FP32 A X, else (the reduced-precision
    // form, whose scale needs it first, or the scheme on A^H) one separate pass
    const bool fro_apart = b.Alo || pr.transpose;
    c.fro_next = !fro_apart;
    if (c.live()) {
        note(c, solve_prologue_launch(b.status, 16, b.counters, (int64_t)std::max<size_t>(c.cnt_need, 1),
                                      pr.estimate ? pr.pass_err : nullptr, c.st));
        const bool in_copy = b.Alo && fro_in_copy(pr);
        if (fro_apart && !in_copy) note(c, fro2_launch(pr.A, pr.mr, pr.nr, pr.lda, pr.aps, b.fro_part, b.nA2, c.st));
        if (pr.sketch == QLRA_SKETCH_SRHT) note(c, omega_srht_launch(pr.seed, pr.n, l, b.Om, l, pr.n * l, c.st));
        else note(c, omega_launch(pr.seed, pr.n, l, b.Om, l, pr.n * l, c.st, pr.sketch == QLRA_SKETCH_REAL ? 1 : 0));
        if (b.Alo) {
            note(c, lowp_scale_launch(b.nA2, pr.prec, b.lp_scale, b.lp_scale + 1, c.st));
            note(c, lowp_copy_launch(pr.A, pr.mr, pr.nr, pr.lda, pr.aps, pr.prec, b.Alo, b.Alo_t, b.lp_scale, c.st,
                                     b.Alo_lo, b.Alo_t_lo, in_copy ? b.fro_part : nullptr));
            if (in_copy)
                note(c, fro2_final_launch(b.fro_part, (int64_t)lowp_copy_fro_slots(pr.mr, pr.nr), b.nA2, c.st));
        }
    }
    // views 1 .. v-2 in reduced precision when asked; the last two keep FP32
    auto lowp_view = [&](int i) { return view_mode(pr, i); };
    const float* Q2cur = b.Om;
    if (!d.krylov) {
        // Alg. 2: odd views [Q1, R1] = QR(A Q2), even views [Q2, R2] = QR(A^H Q1)
        const bool gram_final = l <= heig_big_max();
        for (int i = 1; i <= pr.v; i++) {
            if (i == pr.v && gram_final) {
                const bool merge = merged_estimates(pr, d) && b.Gs;
                if (!merge) fork_point(c, b, pr, l);
                const bool odd = i % 2 == 1;
                view_product(c, pr, b, !odd, odd ? Q2cur : b.Q1, l, l, b.T, view_mode(pr, i));
                if (!merge) fork_deferred(c, b, pr, l);
                finish_gram(c, b, pr, b.T, odd ? pr.m : pr.n, odd ? Q2cur : b.Q1, l, odd ? pr.n : pr.m, l, odd, merge);
                return;
            }
            // R is kept for the last view (the final QSVD) and for side-stream estimates from R
            double* R = (i == pr.v || (pr.estimate && !b.Gs)) ? b.Rv + (size_t)(i - 1) * 4 * l2 : nullptr;
            // the last two views produce the returned bases: CholeskyQR2 there
            const int rounds = i >= pr.v - 1 ? 2 : 1;
            double* G0 = gram_slot(b, pr, l, i);
            if (i % 2 == 1) view(c, pr, b, false, Q2cur, l, l, b.T, b.Q1, l, R, rounds, G0, lowp_view(i));
            else { view(c, pr, b, true, b.Q1, l, l, b.T, b.Q2, l, R, rounds, G0, lowp_view(i)); Q2cur = b.Q2; }
            if (i >= 2) fork_estimate(c, b, pr, R, l, i);
        }
        fork_estimates(c, b, pr, l);
        finish(c, b, pr, b.Rv + (size_t)(pr.v - 1) * 4 * l2, l, b.Q1, l, Q2cur, l, d.even);
        return;
    }
    // Alg. 4: ping-pong views, Krylov blocks stacked (range blocks for even v, co-range for odd)
    const int64_t Wk = d.Wk, rs = d.stack_rows, sps = rs * Wk;
    int i = 0;
    auto stack_in = [&](const float* Qb, int slot) {
        const int64_t c0 = (int64_t)slot * l;
        if (!c.live() || c0 >= Wk) return;
        note(c, copy_planes_launch(Qb, l, rs * l, b.stack + c0, Wk, sps, rs, std::min(l, Wk - c0), nullptr, c.st));
    };
    const bool keepR = pr.estimate && !b.Gs;
    for (int j = 1; j <= d.s; j++) {
        double* R = keepR ? b.Rv + (size_t)i * 4 * l2 : nullptr;
        view(c, pr, b, false, Q2cur, l, l, b.T, b.Q1, l, R, 1, gram_slot(b, pr, l, i + 1), lowp_view(i + 1));
        i++;
        if (i >= 2) fork_estimate(c, b, pr, R, l, i);
        if (d.even) stack_in(b.Q1, j - 1);
        R = keepR ? b.Rv + (size_t)i * 4 * l2 : nullptr;
        view(c, pr, b, true, b.Q1, l, l, b.T, b.Q2, l, R, 1, gram_slot(b, pr, l, i + 1), lowp_view(i + 1));
        i++;
        fork_estimate(c, b, pr, R, l, i);
        Q2cur = b.Q2;
        if (!d.even) stack_in(b.Q2, j - 1);
    }
    if (d.even) {
        double* R = keepR ? b.Rv + (size_t)i * 4 * l2 : nullptr;
        view(c, pr, b, false, Q2cur, l, l, b.T, b.Q1, l, R, 1, gram_slot(b, pr, l, i + 1), lowp_view(i + 1));
        i++;
        if (i >= 2) fork_estimate(c, b, pr, R, l, i);
        stack_in(b.Q1, d.s);
        fork_point(c, b, pr, l);
        orth_stack(c, b.stack, pr.m, Wk, l, b.Cbuf);
        if (Wk <= heig_big_max()) {
            view_product(c, pr, b, true, b.stack, Wk, Wk, b.T, view_mode(pr, pr.v));
            fork_deferred(c, b, pr, l);
            finish_gram(c, b, pr, b.T, pr.n, b.stack, Wk, pr.m, Wk, false);
        } else {
            view(c, pr, b, true, b.stack, Wk, Wk, b.T, b.Q2, Wk, b.Rfin, 2, nullptr, view_mode(pr, pr.v));
            fork_deferred(c, b, pr, l);
            finish(c, b, pr, b.Rfin, Wk, b.stack, Wk, b.Q2, Wk, true);
        }
    } else {
        fork_point(c, b, pr, l);
        orth_stack(c, b.stack, pr.n, Wk, l, b.Cbuf);
        if (Wk <= heig_big_max()) {
            view_product(c, pr, b, false, b.stack, Wk, Wk, b.T, view_mode(pr, pr.v));
            fork_deferred(c, b, pr, l);
            finish_gram(c, b, pr, b.T, pr.m, b.stack, Wk, pr.n, Wk, true);
        } else {
            view(c, pr, b, false, b.stack, Wk, Wk, b.T, b.Q1, Wk, b.Rfin, 2, nullptr, view_mode(pr, pr.v));
            fork_deferred(c, b, pr, l);
            finish(c, b, pr, b.Rfin, Wk, b.Q1, Wk, b.stack, Wk, false);
        }
    }
}

void bind_ctx(Ctx& c, const Bufs& b, const Dims& d) {
    c.status = b.status;
    c.chol_work = b.chol_work;
    c.G = b.G; c.R1 = b.R1; c.R2 = b.R2; c.blk = b.blk; c.Rinv = b.Rinv;
    c.T2 = b.T2; c.T2_rows = d.rows_max;
    c.Rjunk = b.Rfin;
    c.scr.partial = b.partial;
    c.scr.counters = b.counters;
}

// Sizes of the workspace pieces: run the solve dry to find the largest split-K scratch.
void size_solve(const Problem& pr, const Dims& d, size_t* part, size_t* cnt, size_t* total) {
    Ctx c;
    c.dry = true;
    Arena ar{nullptr, 0, 0, true};
    Bufs b{};
    carve(pr, d, ar, b, 0, 0);
    bind_ctx(c, b, d);
    run_solve(c, pr, d, b);
    *part = c.part_need;
    *cnt = c.cnt_need;
    Arena ar2{nullptr, 0, 0, true};
    Bufs b2{};
    carve(pr, d, ar2, b2, c.part_need, c.cnt_need);
    *total = ar2.used;
}

int check_problem(const Problem& pr) {
    if (pr.m < 1 || pr.n < 1 || pr.k < 1 || pr.p < 0 || pr.v < 2) return QLRA_E_ARG;
    if (pr.scheme != QLRA_SUBSPACE && pr.scheme != QLRA_BLOCK_KRYLOV) return QLRA_E_ARG;
    const int64_t l = (int64_t)pr.k + pr.p;
    if (l > pr.m || l > pr.n) return QLRA_E_ARG;
    if (pr.v > 64) return QLRA_E_TOO_LARGE;
    if (pr.prec != QLRA_FP32 && pr.prec != QLRA_BF16 && pr.prec != QLRA_FP16 && !prec_split(pr.prec))
        return QLRA_E_UNSUPPORTED;
    if (pr.sketch != QLRA_SKETCH_QUATERNION && pr.sketch != QLRA_SKETCH_REAL && pr.sketch != QLRA_SKETCH_SRHT)
        return QLRA_E_UNSUPPORTED;
    return QLRA_OK;
}

int check_layout(const void* P, int64_t rows, int64_t cols, int64_t ld, int64_t ps) {
    if (!P) return QLRA_E_ARG;
    if (ld < cols || ps < rows * ld) return QLRA_E_ARG;
    return QLRA_OK;
}


// ---------------------------------------------------------------------------------------
// Continuous-batching server: a scheduler thread admits requests in arrival order while a slot
// and enough of the HBM arena are free, then advances every admitted request by one view-step
// per tick (the view's product, its QR and, on the last step, the final QSVD), each request on
// its own stream pair so that steps of different requests overlap on the device.  A request's
// workspace (its bases, factors and Grams) lives in the arena from admission to completion.

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct SrvRequest {
    qlra_request_t r{};
    uint64_t ticket = 0;
    Problem pr{};
    Dims d{};
    size_t part = 0, cnt = 0, bytes = 0, off = 0;
    int slot = -1;
    int next_step = 0;
    bool all_enqueued = false;
    int done = 0;              // 0 pending / running, 1 finished
    int status = QLRA_OK;
    double t_arrival = 0, t_admit = 0, t_done = 0;
    std::vector<hipGraphExec_t> graphs;
};

struct SrvSlot {
    hipStream_t st = nullptr, side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, done = nullptr;
    int* status_host = nullptr;   // pinned: the request's status word, copied after its last step
    SrvRequest* req = nullptr;
};

}  // namespace
}  // namespace qlra_impl

struct qlra_server {
    int dev = 0;
    int graphs = 0;
    char* arena = nullptr;
    size_t cap = 0;
    qlra_impl::ArenaAlloc alloc{0};
    std::vector<qlra_impl::SrvSlot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<qlra_impl::SrvRequest*> pending;
    std::unordered_map<uint64_t, std::unique_ptr<qlra_impl::SrvRequest>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    int active = 0, max_active_seen = 0;
    size_t max_used_seen = 0;
    int64_t ticks = 0;
    hipError_t err = hipSuccess;
    std::thread th;
};

namespace qlra_impl {
namespace {

// Enqueue step s of a request on its slot's streams (captured as a graph when asked).
void srv_enqueue_step(qlra_server* sv, SrvRequest* q, int s) {
    SrvSlot& sl = sv->slots[q->slot];
    Arena ar{sv->arena + q->off, q->bytes, 0, false};
    Bufs b{};
    carve(q->pr, q->d, ar, b, q->part, q->cnt);
    Ctx c;
    c.cnt_need = q->cnt;
    bind_ctx(c, b, q->d);
    c.side = sl.side; c.ev_fork = sl.fork; c.ev_join = sl.join;
    c.step_only = s;
    const bool last = s == q->pr.v - 1;
    hipGraph_t g = nullptr;
    // a step whose capture cannot begin is launched eagerly (the same launches, in order)
    const bool cap = sv->graphs != 0 && hipStreamBeginCapture(sl.st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    c.st = sl.st;
    run_solve(c, q->pr, q->d, b);
    // a step rejoins whatever it forked (a captured step must, and the slot's events are reused)
    if (c.forked) {
        note(c, hipEventRecord(c.ev_join, c.side));
        note(c, hipStreamWaitEvent(c.st, c.ev_join, 0));
    }
    if (cap) {
        const hipError_t ee = hipStreamEndCapture(sl.st, &g);
        hipGraphExec_t ex = nullptr;
        if (ee == hipSuccess && g && c.err == hipSuccess && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
            note(c, hipGraphLaunch(ex, sl.st));
            q->graphs.push_back(ex);
        } else {
            c.err = c.err == hipSuccess ? hipErrorUnknown : c.err;
        }
        if (g) (void)hipGraphDestroy(g);
    }
    if (last) {
        note(c, hipMemcpyAsync(sl.status_host, b.status, sizeof(int), hipMemcpyDeviceToHost, sl.st));
        note(c, hipEventRecord(sl.done, sl.st));
    }
    if (c.err != hipSuccess) q->status = QLRA_E_HIP;
}

void srv_loop(qlra_server* sv) {
    if (hipSetDevice(sv->dev) != hipSuccess) { sv->err = hipErrorInvalidDevice; return; }
    std::unique_lock<std::mutex> lk(sv->mu);
    while (true) {
        // admission: arrival order, a free slot and room in the arena
        while (!sv->pending.empty()) {
            SrvRequest* q = sv->pending.front();
            int slot = -1;
            for (size_t i = 0; i < sv->slots.size(); i++)
                if (!sv->slots[i].req) { slot = (int)i; break; }
            size_t off = 0;
            if (slot < 0 || !sv->alloc.alloc(q->bytes, &off)) break;
            sv->pending.pop_front();
            q->off = off;
            q->slot = slot;
            q->t_admit = now_s();
            sv->slots[slot].req = q;
            sv->active++;
            sv->max_active_seen = std::max(sv->max_active_seen, sv->active);
            sv->max_used_seen = std::max(sv->max_used_seen, sv->alloc.used());
        }
        bool work = false;
        // one view-step per admitted request
        for (auto& sl : sv->slots) {
            SrvRequest* q = sl.req;
            if (!q || q->all_enqueued) continue;
            lk.unlock();
            srv_enqueue_step(sv, q, q->next_step);
            lk.lock();
            q->next_step++;
            if (q->next_step >= q->pr.v) q->all_enqueued = true;
            work = true;
        }
        // completions
        for (auto& sl : sv->slots) {
            SrvRequest* q = sl.req;
            if (!q || !q->all_enqueued) continue;
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipErrorNotReady) continue;
            q->t_done = now_s();
            if (e != hipSuccess) q->status = QLRA_E_HIP;
            else if (q->status == QLRA_OK && (*sl.status_host & 2)) q->status = QLRA_E_NUMERIC;
            for (auto ex : q->graphs) (void)hipGraphExecDestroy(ex);
            q->graphs.clear();
            sv->alloc.release(q->off, q->bytes);
            sl.req = nullptr;
            sv->active--;
            q->done = 1;
            work = true;
            sv->cv.notify_all();
        }
        sv->ticks++;
        if (sv->stop && sv->pending.empty() && sv->active == 0) break;
        if (!work) sv->cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

}  // namespace
}  // namespace qlra_impl

namespace qlra_impl {
namespace {

// ---------------------------------------------------------------------------------------
// Quaternion matrix completion (Sec. 7): every iteration is a full solve of the rank-R problem on
// the current C (same sketch), followed by the fused reconstruct / smooth / update kernel.  The
// workspace holds the completion's status word first (so that qlra_status() reads it), its
// iteration counter, C, the factors and the misfit sums, then the solve's own pieces.

struct Completion {
    Problem pr;             // the solve on C (A = C), oriented
    Dims d;
    size_t part = 0, cnt = 0;
    int* status = nullptr;
    int* iter = nullptr;
    float* C = nullptr;
    float* U = nullptr;
    float* V = nullptr;
    double* S = nullptr;
    double* fit_part = nullptr;
    Bufs b{};
};

int completion_layout(int64_t m, int64_t n, int R, int p, int v, int scheme, double sigma, const qlra_opts_t* opts,
                      char* base, size_t size, bool dry, Completion& cp, size_t* total) {
    if (sigma != sigma || complete_radius(sigma) > kCompleteMaxRadius) return QLRA_E_UNSUPPORTED;
    Problem& pr = cp.pr;
    pr = Problem{};
    pr.m = m; pr.n = n; pr.lda = n; pr.aps = m * n;
    pr.k = R; pr.p = p; pr.v = v; pr.scheme = scheme;
    pr.ldu = R; pr.ups = m * R; pr.ldv = R; pr.vps = n * R;
    pr.estimate = 0;
    pr.prec = opts ? opts->pass_precision : QLRA_FP32;
    pr.sketch = opts ? opts->sketch : QLRA_SKETCH_QUATERNION;
    int rc = check_problem(pr);
    if (rc) return rc;
    const int transpose = opts ? opts->transpose : 0;
    {
        Problem po = pr;
        orient(po, transpose);
        cp.d = dims_of(po.m, po.n, R, p, v, scheme);
        size_t solve_total;
        size_solve(po, cp.d, &cp.part, &cp.cnt, &solve_total);
    }
    Arena ar{base, size, 0, dry};
    cp.status = (int*)ar.take(16 * sizeof(int));
    cp.iter = (int*)ar.take(sizeof(int));
    cp.C = (float*)ar.take(4 * m * n * sizeof(float));
    cp.U = (float*)ar.take(4 * m * R * sizeof(float));
    cp.V = (float*)ar.take(4 * n * R * sizeof(float));
    cp.S = (double*)ar.take(R * sizeof(double));
    cp.fit_part = (double*)ar.take(2 * complete_blocks(m, n, complete_radius(sigma)) * sizeof(double));
    pr.A = cp.C;
    pr.U = cp.U; pr.S = cp.S; pr.V = cp.V;
    orient(pr, transpose);
    carve(pr, cp.d, ar, cp.b, cp.part, cp.cnt);
    *total = ar.used;
    return QLRA_OK;
}

}  // namespace
}  // namespace qlra_impl

using namespace qlra_impl;

extern "C" {

const char* qlra_strerror(int status) {
    switch (status) {
        case QLRA_OK: return "success";
        case QLRA_E_ARG: return "invalid argument";
        case QLRA_E_WORKSPACE: return "workspace missing, too small or misaligned";
        case QLRA_E_HIP: return "HIP runtime error";
        case QLRA_E_NUMERIC: return "numerical breakdown (non-finite data or failed Cholesky)";
        case QLRA_E_TOO_LARGE: return "request larger than supported";
        case QLRA_E_UNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

int qlra_workspace_size(int64_t m, int64_t n, int k, int p, int pass_budget, int scheme, const qlra_opts_t* opts,
                        size_t* bytes) {
    if (!bytes) return QLRA_E_ARG;
    Problem pr{};
    pr.m = m; pr.n = n; pr.k = k; pr.p = p; pr.v = pass_budget; pr.scheme = scheme;
    pr.lda = n; pr.aps = m * n; pr.ldu = k; pr.ups = m * k; pr.ldv = k; pr.vps = n * k;
    pr.estimate = opts ? opts->estimate_passes : 1;
    pr.prec = opts ? opts->pass_precision : QLRA_FP32;
    pr.sketch = opts ? opts->sketch : QLRA_SKETCH_QUATERNION;
    orient(pr, opts ? opts->transpose : 0);
    int rc = check_problem(pr);
    if (rc) return rc;
    const Dims d = dims_of(pr.m, pr.n, k, p, pass_budget, scheme);
    size_t part, cnt, total;
    size_solve(pr, d, &part, &cnt, &total);
    *bytes = total;
    return QLRA_OK;
}

int qlra(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_plane_stride, int k, int p,
         int pass_budget, int scheme, uint64_t seed, const qlra_opts_t* opts, float* U, int64_t ldu,
         int64_t u_plane_stride, double* S, float* V, int64_t ldv, int64_t v_plane_stride, double* pass_err) {
    return qlra_impl::solve_entry(A, m, n, lda, a_plane_stride, k, p, pass_budget, scheme, seed, opts, U, ldu,
                                  u_plane_stride, S, V, ldv, v_plane_stride, pass_err, false);
}

}  // extern "C"

namespace qlra_impl {

int solve_entry(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_plane_stride, int k, int p,
                int pass_budget, int scheme, uint64_t seed, const qlra_opts_t* opts, float* U, int64_t ldu,
                int64_t u_plane_stride, double* S, float* V, int64_t ldv, int64_t v_plane_stride, double* pass_err,
                bool no_alloc) {
    if (!opts) return QLRA_E_ARG;
    Problem pr{};
    pr.A = A; pr.m = m; pr.n = n; pr.lda = lda; pr.aps = a_plane_stride;
    pr.k = k; pr.p = p; pr.v = pass_budget; pr.scheme = scheme; pr.seed = seed;
    pr.U = U; pr.ldu = ldu; pr.ups = u_plane_stride; pr.S = S;
    pr.V = V; pr.ldv = ldv; pr.vps = v_plane_stride;
    pr.pass_err = pass_err;
    pr.estimate = (opts->estimate_passes && pass_err) ? 1 : 0;
    pr.prec = opts->pass_precision;
    pr.sketch = opts->sketch;
    int rc = check_problem(pr);
    if (rc) return rc;
    if ((rc = check_layout(A, m, n, lda, a_plane_stride))) return rc;
    if ((rc = check_layout(U, m, k, ldu, u_plane_stride))) return rc;
    if ((rc = check_layout(V, n, k, ldv, v_plane_stride))) return rc;
    if (!S) return QLRA_E_ARG;
    orient(pr, opts->transpose);
    const Dims d = dims_of(pr.m, pr.n, k, p, pass_budget, scheme);
    size_t part, cnt, total;
    size_solve(pr, d, &part, &cnt, &total);
    if (!opts->workspace || opts->workspace_bytes < total || ((uintptr_t)opts->workspace & 255))
        return QLRA_E_WORKSPACE;
    Arena ar{(char*)opts->workspace, opts->workspace_bytes, 0, false};
    Bufs b{};
    carve(pr, d, ar, b, part, cnt);
    Ctx c;
    c.st = (hipStream_t)opts->stream;
    c.cnt_need = cnt;
    bind_ctx(c, b, d);
    Side sd;
    // without allocations the estimates run on the solve's own stream (no side stream is created)
    const bool forks = pr.estimate && !merged_estimates(pr, d) && !no_alloc;
    if (forks) {
        if (get_side((hipStream_t)opts->stream, &sd) != hipSuccess) return QLRA_E_HIP;
        c.side = sd.s; c.ev_fork = sd.fork; c.ev_join = sd.join;
    }
    auto enqueue = [&]() {
        run_solve(c, pr, d, b);
        if (c.forked) {
            note(c, hipEventRecord(c.ev_join, c.side));
            note(c, hipStreamWaitEvent(c.st, c.ev_join, 0));
        }
    };
    if (!opts->graph || no_alloc) {
        enqueue();
        return c.err == hipSuccess ? QLRA_OK : QLRA_E_HIP;
    }
    // graph path: replay a captured solve with the same arguments, or capture one
    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    if (hipGetDevice(&key.dev) != hipSuccess || key.dev < 0 || key.dev >= 64) return QLRA_E_HIP;
    key.A = A; key.m = m; key.n = n; key.lda = lda; key.aps = a_plane_stride;
    key.k = k; key.p = p; key.v = pass_budget; key.scheme = scheme; key.estimate = pr.estimate; key.seed = seed;
    key.prec = pr.prec;
    key.transpose = pr.transpose;
    key.sketch = pr.sketch;
    key.U = U; key.ldu = ldu; key.ups = u_plane_stride; key.S = S; key.V = V; key.ldv = ldv;
    key.vps = v_plane_stride; key.pass_err = pass_err; key.ws = opts->workspace;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    hipGraphExec_t exec = nullptr;
    const hipError_t ge = graph_for(key, [&](hipStream_t cap) { c.st = cap; enqueue(); return c.err; }, &exec);
    if (ge != hipSuccess) return QLRA_E_HIP;
    return hipGraphLaunch(exec, (hipStream_t)opts->stream) == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

}  // namespace qlra_impl

extern "C" {

int qlra_status(const void* workspace, void* stream, int* status) {
    if (!workspace || !status) return QLRA_E_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return QLRA_E_HIP;
    int word = 0;
    if (hipMemcpy(&word, workspace, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return QLRA_E_HIP;
    *status = (word & 2) ? QLRA_E_NUMERIC : QLRA_OK;
    return QLRA_OK;
}

int qlra_complete_workspace_size(int64_t m, int64_t n, int rank, int p, int pass_budget, int scheme, double sigma,
                                 const qlra_opts_t* opts, size_t* bytes) {
    if (!bytes) return QLRA_E_ARG;
    Completion cp;
    size_t total = 0;
    const int rc = completion_layout(m, n, rank, p, pass_budget, scheme, sigma, opts, nullptr, 0, true, cp, &total);
    if (rc) return rc;
    *bytes = total;
    return QLRA_OK;
}

int qlra_complete(const float* M, int64_t m, int64_t n, int64_t ldm, int64_t m_plane_stride, const unsigned char* mask,
                  int64_t ld_mask, int rank, int p, int pass_budget, int scheme, uint64_t seed, int iters, double sigma,
                  const qlra_opts_t* opts, float* X, int64_t ldx, int64_t x_plane_stride, double* fit) {
    if (!opts || iters < 1 || m < 1 || n < 1) return QLRA_E_ARG;
    int rc;
    if ((rc = check_layout(M, m, n, ldm, m_plane_stride))) return rc;
    if ((rc = check_layout(X, m, n, ldx, x_plane_stride))) return rc;
    if (!mask || ld_mask < n) return QLRA_E_ARG;
    Completion cp;
    size_t total = 0;
    if ((rc = completion_layout(m, n, rank, p, pass_budget, scheme, sigma, opts, nullptr, 0, true, cp, &total)))
        return rc;
    if (!opts->workspace || opts->workspace_bytes < total || ((uintptr_t)opts->workspace & 255))
        return QLRA_E_WORKSPACE;
    if ((rc = completion_layout(m, n, rank, p, pass_budget, scheme, sigma, opts, (char*)opts->workspace,
                                opts->workspace_bytes, false, cp, &total)))
        return rc;
    cp.pr.seed = seed;
    CompleteStep cs{};
    cs.U = cp.U; cs.ldu = rank; cs.ups = m * rank;
    cs.S = cp.S;
    cs.V = cp.V; cs.ldv = rank; cs.vps = n * rank;
    cs.R = rank;
    cs.M = M; cs.ldm = ldm; cs.mps = m_plane_stride;
    cs.mask = mask; cs.ldk = ld_mask;
    cs.C = cp.C; cs.ldc = n; cs.cps = m * n;
    cs.X = X; cs.ldx = ldx; cs.xps = x_plane_stride;
    cs.m = m; cs.n = n;
    cs.sigma = sigma;
    cs.iter = cp.iter; cs.iters = iters;
    cs.part = cp.fit_part;
    cs.fit = fit;
    // one iteration: the rank-R solve on C, its status bits into the completion's, the update
    auto iteration = [&](hipStream_t s) -> hipError_t {
        Ctx c;
        c.st = s;
        c.cnt_need = cp.cnt;
        bind_ctx(c, cp.b, cp.d);
        run_solve(c, cp.pr, cp.d, cp.b);
        note(c, status_or_launch(cp.status, cp.b.status, s));
        note(c, complete_step_launch(cs, s));
        return c.err;
    };
    const hipStream_t st = (hipStream_t)opts->stream;
    if (complete_init_launch(M, ldm, m_plane_stride, mask, ld_mask, m, n, cp.C, n, m * n, cp.iter, cp.status, st) !=
        hipSuccess)
        return QLRA_E_HIP;
    if (!opts->graph) {
        for (int t = 0; t < iters; t++)
            if (iteration(st) != hipSuccess) return QLRA_E_HIP;
        return QLRA_OK;
    }
    // graph path: one captured iteration, replayed `iters` times (the iteration counter lives on
    // the device), cached under the call's arguments like the solves
    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    if (hipGetDevice(&key.dev) != hipSuccess || key.dev < 0 || key.dev >= 64) return QLRA_E_HIP;
    key.completion = 1;
    key.A = M; key.m = m; key.n = n; key.lda = ldm; key.aps = m_plane_stride;
    key.k = rank; key.p = p; key.v = pass_budget; key.scheme = scheme; key.seed = seed;
    key.prec = cp.pr.prec; key.transpose = cp.pr.transpose; key.sketch = cp.pr.sketch;
    key.ws = opts->workspace;
    key.mask = mask; key.ldk = ld_mask;
    key.X = X; key.ldx = ldx; key.xps = x_plane_stride;
    key.fit = fit; key.sigma = sigma; key.iters = iters;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    hipGraphExec_t exec = nullptr;
    if (graph_for(key, iteration, &exec) != hipSuccess) return QLRA_E_HIP;
    for (int t = 0; t < iters; t++)
        if (hipGraphLaunch(exec, st) != hipSuccess) return QLRA_E_HIP;
    return QLRA_OK;
}

int qlra_omega_srht(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t plane_stride, void* stream) {
    if (n < 0 || l < 0 || l > n || n > ((int64_t)1 << 30)) return QLRA_E_ARG;
    if (n * l == 0) return QLRA_OK;
    int rc;
    if ((rc = check_layout(Om, n, l, ld, plane_stride))) return rc;
    return omega_srht_launch(seed, n, l, Om, ld, plane_stride, (hipStream_t)stream) == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

int qlra_omega(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t plane_stride, void* stream) {
    if (n < 0 || l < 0) return QLRA_E_ARG;
    if (n * l == 0) return QLRA_OK;
    int rc = check_layout(Om, n, l, ld, plane_stride);
    if (rc) return rc;
    return omega_launch(seed, n, l, Om, ld, plane_stride, (hipStream_t)stream) == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

static QgemmDesc view_desc(int op, const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_ps, const float* B,
                           int64_t w, int64_t ldb, int64_t b_ps, float* C, int64_t ldc, int64_t c_ps) {
    return op == 0 ? desc(OP_NN, MATH_F32, A, lda, a_ps, 0, B, ldb, b_ps, 0, C, ldc, c_ps, 0, m, w, n)
                   : desc(OP_HN, MATH_F32, A, lda, a_ps, 0, B, ldb, b_ps, 0, C, ldc, c_ps, 0, n, w, m);
}

int qlra_qgemm_workspace_size(int op, int64_t m, int64_t n, int64_t w, size_t* bytes) {
    if (!bytes || (op != 0 && op != 1) || m < 0 || n < 0 || w < 0) return QLRA_E_ARG;
    const QgemmDesc d = view_desc(op, nullptr, m, n, n, m * n, nullptr, w, w, 0, nullptr, w, 0);
    Arena ar{nullptr, 0, 0, true};
    ar.take(std::max<size_t>(qgemm_counter_count(d), 1) * sizeof(unsigned));
    ar.take(qgemm_partial_bytes(d));
    *bytes = ar.used;
    return QLRA_OK;
}

int qlra_qgemm(int op, const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_ps, const float* B, int64_t w,
               int64_t ldb, int64_t b_ps, float* C, int64_t ldc, int64_t c_ps, void* workspace,
               size_t workspace_bytes, void* stream) {
    if (op != 0 && op != 1) return QLRA_E_ARG;
    if (m < 0 || n < 0 || w < 0) return QLRA_E_ARG;
    const int64_t kdim = op == 0 ? n : m, rows = op == 0 ? m : n;
    if (rows == 0 || w == 0) return QLRA_OK;
    int rc;
    if ((rc = check_layout(A, m, n, lda, a_ps))) return rc;
    if ((rc = check_layout(B, kdim, w, ldb, b_ps))) return rc;
    if ((rc = check_layout(C, rows, w, ldc, c_ps))) return rc;
    size_t need = 0;
    qlra_qgemm_workspace_size(op, m, n, w, &need);
    if (workspace_bytes < need || (need > 0 && !workspace) || ((uintptr_t)workspace & 255)) return QLRA_E_WORKSPACE;
    const QgemmDesc d = view_desc(op, A, m, n, lda, a_ps, B, w, ldb, b_ps, C, ldc, c_ps);
    Arena ar{(char*)workspace, workspace_bytes, 0, false};
    const size_t cnt = qgemm_counter_count(d);
    QgemmScratch s{};
    s.counters = (unsigned*)ar.take(std::max<size_t>(cnt, 1) * sizeof(unsigned));
    s.partial = ar.take(qgemm_partial_bytes(d));
    return qgemm_launch(d, s, (hipStream_t)stream) == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

int qlra_lowp_copy_bytes(int64_t m, int64_t n, size_t* alo_bytes, size_t* alo_t_bytes) {
    if (m < 0 || n < 0 || !alo_bytes || !alo_t_bytes) return QLRA_E_ARG;
    *alo_bytes = lowp_copy_elems(m, n) * 2;
    *alo_t_bytes = lowp_copy_elems(n, m) * 2;
    return QLRA_OK;
}

int qlra_lowp_copy(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_ps, int precision,
                   const float* scale, void* Alo, void* Alo_t, void* stream) {
    if (m < 0 || n < 0 || (precision != QLRA_BF16 && precision != QLRA_FP16)) return QLRA_E_ARG;
    if (m * n == 0) return QLRA_OK;
    int rc;
    if ((rc = check_layout(A, m, n, lda, a_ps))) return rc;
    if (!Alo || !Alo_t) return QLRA_E_ARG;
    return lowp_copy_launch(A, m, n, lda, a_ps, precision, Alo, Alo_t, scale, (hipStream_t)stream) == hipSuccess
               ? QLRA_OK
               : QLRA_E_HIP;
}

int qlra_lowp_copy_residual(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_ps, int precision,
                            const float* scale, void* Alo_res, void* Alo_t_res, void* stream) {
    if (m < 0 || n < 0 || (precision != QLRA_BF16 && precision != QLRA_FP16)) return QLRA_E_ARG;
    if (m * n == 0) return QLRA_OK;
    int rc;
    if ((rc = check_layout(A, m, n, lda, a_ps))) return rc;
    if (!Alo_res || !Alo_t_res) return QLRA_E_ARG;
    return lowp_copy_launch(A, m, n, lda, a_ps, precision, nullptr, nullptr, scale, (hipStream_t)stream, Alo_res,
                            Alo_t_res) == hipSuccess
               ? QLRA_OK
               : QLRA_E_HIP;
}
static QgemmDesc lp_desc(int op, int precision, const void* Alo, int64_t m, int64_t n, const float* B, int64_t w,
                         int64_t ldb, int64_t b_ps, float* C, int64_t ldc, int64_t c_ps, const float* inv_scale) {
    const int64_t rows = op == 0 ? m : n, kdim = op == 0 ? n : m;
    QgemmDesc d = desc(op == 0 ? OP_NN : OP_HN, precision == QLRA_BF16 ? MATH_BF16 : MATH_F16, Alo, kdim, m * n, 0, B,
                       ldb, b_ps, 0, C, ldc, c_ps, 0, rows, w, kdim);
    d.cscale = inv_scale;
    return d;
}

int qlra_qgemm_lp_workspace_size(int op, int precision, int64_t m, int64_t n, int64_t w, size_t* bytes) {
    if (!bytes || (op != 0 && op != 1) || m < 0 || n < 0 || w < 0) return QLRA_E_ARG;
    if (precision != QLRA_BF16 && precision != QLRA_FP16) return QLRA_E_ARG;
    const QgemmDesc d = lp_desc(op, precision, nullptr, m, n, nullptr, w, w, 0, nullptr, w, 0, nullptr);
    *bytes = (m * n * w == 0) ? 0 : qgemm_partial_bytes(d);
    return QLRA_OK;
}

int qlra_qgemm_lp(int op, int precision, const void* Alo, int64_t m, int64_t n, const float* B, int64_t w, int64_t ldb,
                  int64_t b_ps, float* C, int64_t ldc, int64_t c_ps, const float* inv_scale, void* workspace,
                  size_t workspace_bytes, void* stream) {
    size_t need = 0;
    int rc = qlra_qgemm_lp_workspace_size(op, precision, m, n, w, &need);
    if (rc) return rc;
    const int64_t kdim = op == 0 ? n : m, rows = op == 0 ? m : n;
    if (rows == 0 || w == 0) return QLRA_OK;
    if (!Alo) return QLRA_E_ARG;
    if ((rc = check_layout(B, kdim, w, ldb, b_ps))) return rc;
    if ((rc = check_layout(C, rows, w, ldc, c_ps))) return rc;
    if (workspace_bytes < need || !workspace || ((uintptr_t)workspace & 255)) return QLRA_E_WORKSPACE;
    const QgemmDesc d = lp_desc(op, precision, Alo, m, n, B, w, ldb, b_ps, C, ldc, c_ps, inv_scale);
    QgemmScratch s{};
    s.partial = workspace;
    return qgemm_launch(d, s, (hipStream_t)stream) == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

static QgemmDesc split_desc(int op, int precision, const void* Alo, const void* Alo_res, int64_t m, int64_t n,
                            const float* B, int64_t w, int64_t ldb, int64_t b_ps, float* C, int64_t ldc, int64_t c_ps,
                            const float* inv_scale) {
    QgemmDesc d = lp_desc(op, precision, Alo, m, n, B, w, ldb, b_ps, C, ldc, c_ps, inv_scale);
    d.math = precision == QLRA_BF16 ? MATH_BF16X3 : MATH_F16X3;
    d.A_lo = Alo_res;
    return d;
}
int qlra_qgemm_split_workspace_size(int op, int precision, int64_t m, int64_t n, int64_t w, size_t* bytes) {
    if (!bytes || (op != 0 && op != 1) || m < 0 || n < 0 || w < 0) return QLRA_E_ARG;
    if (precision != QLRA_BF16 && precision != QLRA_FP16) return QLRA_E_ARG;
    const QgemmDesc d = split_desc(op, precision, nullptr, nullptr, m, n, nullptr, w, w, 0, nullptr, w, 0, nullptr);
    *bytes = (m * n * w == 0) ? 0 : qgemm_partial_bytes(d);
    return QLRA_OK;
}
int qlra_qgemm_split(int op, int precision, const void* Alo, const void* Alo_res, int64_t m, int64_t n, const float* B,
                     int64_t w, int64_t ldb, int64_t b_ps, float* C, int64_t ldc, int64_t c_ps, const float* inv_scale,
                     void* workspace, size_t workspace_bytes, void* stream) {
    size_t need = 0;
    int rc = qlra_qgemm_split_workspace_size(op, precision, m, n, w, &need);
    if (rc) return rc;
    const int64_t kdim = op == 0 ? n : m, rows = op == 0 ? m : n;
    if (rows == 0 || w == 0) return QLRA_OK;
    if (!Alo || !Alo_res) return QLRA_E_ARG;
    if ((rc = check_layout(B, kdim, w, ldb, b_ps))) return rc;
    if ((rc = check_layout(C, rows, w, ldc, c_ps))) return rc;
    if (workspace_bytes < need || !workspace || ((uintptr_t)workspace & 255)) return QLRA_E_WORKSPACE;
    const QgemmDesc d = split_desc(op, precision, Alo, Alo_res, m, n, B, w, ldb, b_ps, C, ldc, c_ps, inv_scale);
    QgemmScratch s{};
    s.partial = workspace;
    return qgemm_launch(d, s, (hipStream_t)stream) == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

// CholeskyQR workspace: status words, counters, Gram and factors, intermediate, qgemm scratch.
static void cholqr_carve(int64_t m, int64_t w, Arena& ar, Ctx& c, size_t part, size_t cnt) {
    const int64_t w2 = w * w;
    c.status = (int*)ar.take(16 * sizeof(int));
    c.scr.counters = (unsigned*)ar.take(std::max<size_t>(cnt, 1) * sizeof(unsigned));
    c.G = (double*)ar.take(4 * w2 * sizeof(double));
    c.R1 = (double*)ar.take(4 * w2 * sizeof(double));
    c.R2 = (double*)ar.take(4 * w2 * sizeof(double));
    c.Rjunk = (double*)ar.take(4 * w2 * sizeof(double));   // the last factor when R is not wanted
    c.blk = w > chol_lds_max() ? (double*)ar.take(chol_blk_doubles() * sizeof(double)) : nullptr;
    c.Rinv = (double*)ar.take(4 * w2 * sizeof(double));
    c.chol_work = (double*)ar.take(4 * w2 * sizeof(double));
    c.T2 = (float*)ar.take(4 * m * w * sizeof(float));
    c.T2_rows = m;
    c.scr.partial = part ? ar.take(part) : nullptr;
}

static void cholqr_sizes(int64_t m, int64_t w, size_t* part, size_t* cnt, size_t* total) {
    Ctx c;
    c.dry = true;
    Arena ar{nullptr, 0, 0, true};
    cholqr_carve(m, w, ar, c, 0, 0);
    cholqr(c, nullptr, m, w, w, m * w, nullptr, w, m * w, nullptr, 2);
    *part = c.part_need;
    *cnt = c.cnt_need;
    Arena ar2{nullptr, 0, 0, true};
    Ctx c2;
    c2.dry = true;
    cholqr_carve(m, w, ar2, c2, *part, *cnt);
    *total = ar2.used;
}

int qlra_cholqr_workspace_size(int64_t m, int64_t w, size_t* bytes) {
    if (!bytes || w < 1 || m < w) return QLRA_E_ARG;
    size_t part, cnt;
    cholqr_sizes(m, w, &part, &cnt, bytes);
    return QLRA_OK;
}

int qlra_cholqr(const float* Y, int64_t m, int64_t w, int64_t ldy, int64_t y_ps, float* Q, int64_t ldq,
                int64_t q_ps, double* R, void* workspace, size_t workspace_bytes, void* stream) {
    if (w < 1 || m < w) return QLRA_E_ARG;
    int rc;
    if ((rc = check_layout(Y, m, w, ldy, y_ps))) return rc;
    if ((rc = check_layout(Q, m, w, ldq, q_ps))) return rc;
    size_t part, cnt, total;
    cholqr_sizes(m, w, &part, &cnt, &total);
    if (!workspace || workspace_bytes < total || ((uintptr_t)workspace & 255)) return QLRA_E_WORKSPACE;
    Arena ar{(char*)workspace, workspace_bytes, 0, false};
    Ctx c;
    c.st = (hipStream_t)stream;
    cholqr_carve(m, w, ar, c, part, cnt);
    note(c, solve_prologue_launch(c.status, 16, c.scr.counters, (int64_t)std::max<size_t>(cnt, 1), nullptr, c.st));
    cholqr(c, Y, m, w, ldy, y_ps, Q, ldq, q_ps, R, 2);
    return c.err == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

int qlra_qsvd_workspace_size(int64_t w, size_t* bytes) {
    if (!bytes || w < 1) return QLRA_E_ARG;
    *bytes = qsvd_work_doubles(w) * sizeof(double);
    return QLRA_OK;
}

int qlra_qsvd(const double* R, int64_t w, double* Uh, double* S, double* Vh, void* workspace,
              size_t workspace_bytes, void* stream) {
    if (!R || !S || w < 1) return QLRA_E_ARG;
    if (!workspace || workspace_bytes < qsvd_work_doubles(w) * sizeof(double) || ((uintptr_t)workspace & 7))
        return QLRA_E_WORKSPACE;
    return qsvd_launch(R, w, Uh, S, Vh, (double*)workspace, (Uh || Vh) ? 1 : 0, (hipStream_t)stream) == hipSuccess
               ? QLRA_OK
               : QLRA_E_HIP;
}

int qlra_server_create(const qlra_server_opts_t* opts, qlra_server_t** out) {
    if (!opts || !out || opts->max_active < 1 || opts->max_active > 64 || opts->hbm_bytes < 256) return QLRA_E_ARG;
    auto sv = std::make_unique<qlra_server>();
    if (hipGetDevice(&sv->dev) != hipSuccess) return QLRA_E_HIP;
    sv->graphs = opts->graphs;
    sv->cap = opts->hbm_bytes;
    if (hipMalloc((void**)&sv->arena, sv->cap) != hipSuccess) return QLRA_E_HIP;
    sv->alloc = ArenaAlloc(sv->cap);
    sv->slots.resize(opts->max_active);
    for (auto& sl : sv->slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&sl.side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&sl.join, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&sl.status_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
            qlra_server_destroy(sv.release());
            return QLRA_E_HIP;
        }
        *sl.status_host = 0;
    }
    qlra_server* raw = sv.release();
    raw->th = std::thread(srv_loop, raw);
    *out = raw;
    return QLRA_OK;
}

int qlra_server_submit(qlra_server_t* sv, const qlra_request_t* r, uint64_t* ticket) {
    if (!sv || !r || !ticket) return QLRA_E_ARG;
    auto q = std::make_unique<SrvRequest>();
    q->r = *r;
    Problem& pr = q->pr;
    pr.A = r->A; pr.m = r->m; pr.n = r->n; pr.lda = r->lda; pr.aps = r->a_plane_stride;
    pr.k = r->k; pr.p = r->p; pr.v = r->pass_budget; pr.scheme = r->scheme; pr.seed = r->seed;
    pr.U = r->U; pr.ldu = r->ldu; pr.ups = r->u_plane_stride; pr.S = r->S;
    pr.V = r->V; pr.ldv = r->ldv; pr.vps = r->v_plane_stride;
    pr.pass_err = r->pass_err;
    pr.estimate = r->pass_err ? 1 : 0;
    pr.prec = r->pass_precision;
    orient(pr, 0);
    int rc = check_problem(pr);
    if (rc) return rc;
    if ((rc = check_layout(r->A, r->m, r->n, r->lda, r->a_plane_stride))) return rc;
    if ((rc = check_layout(r->U, r->m, r->k, r->ldu, r->u_plane_stride))) return rc;
    if ((rc = check_layout(r->V, r->n, r->k, r->ldv, r->v_plane_stride))) return rc;
    if (!r->S) return QLRA_E_ARG;
    q->d = dims_of(pr.m, pr.n, pr.k, pr.p, pr.v, pr.scheme);
    size_solve(pr, q->d, &q->part, &q->cnt, &q->bytes);
    if (q->bytes > sv->cap) return QLRA_E_TOO_LARGE;
    q->t_arrival = r->arrival_time > 0 ? r->arrival_time : now_s();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return QLRA_E_ARG;
    q->ticket = sv->next_ticket++;
    *ticket = q->ticket;
    sv->pending.push_back(q.get());
    sv->reqs.emplace(q->ticket, std::move(q));
    sv->cv.notify_all();
    return QLRA_OK;
}

int qlra_server_poll(qlra_server_t* sv, uint64_t ticket, int wait, int* done, int* status, double* latency_s) {
    if (!sv || !done) return QLRA_E_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return QLRA_E_ARG;
    SrvRequest* q = it->second.get();
    if (wait) sv->cv.wait(lk, [&] { return q->done != 0; });
    *done = q->done;
    if (q->done) {
        if (status) *status = q->status;
        if (latency_s) *latency_s = q->t_done - q->t_arrival;
        sv->reqs.erase(it);
    }
    return QLRA_OK;
}

int qlra_server_wait(qlra_server_t* sv, uint64_t ticket, int* status, double* latency_s) {
    int done = 0;
    return qlra_server_poll(sv, ticket, 1, &done, status, latency_s);
}

int qlra_server_drain(qlra_server_t* sv) {
    if (!sv) return QLRA_E_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [&] { return sv->pending.empty() && sv->active == 0; });
    return sv->err == hipSuccess ? QLRA_OK : QLRA_E_HIP;
}

int qlra_server_stats(qlra_server_t* sv, qlra_server_stats_t* st) {
    if (!sv || !st) return QLRA_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    st->pending = (int)sv->pending.size();
    st->active = sv->active;
    st->max_active_seen = sv->max_active_seen;
    st->arena_bytes = sv->cap;
    st->arena_used = sv->alloc.used();
    st->max_arena_used = sv->max_used_seen;
    st->ticks = sv->ticks;
    return QLRA_OK;
}

int qlra_server_destroy(qlra_server_t* sv) {
    if (!sv) return QLRA_E_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    for (auto& sl : sv->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.side) (void)hipStreamSynchronize(sl.side);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.side) (void)hipStreamDestroy(sl.side);
        if (sl.fork) (void)hipEventDestroy(sl.fork);
        if (sl.join) (void)hipEventDestroy(sl.join);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.status_host) (void)hipHostFree(sl.status_host);
    }
    if (sv->arena) (void)hipFree(sv->arena);
    delete sv;
    return QLRA_OK;
}

double qlra_server_clock(void) { return now_s(); }

}  // extern "C"
