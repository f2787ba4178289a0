// Tall-skinny quaternion products on MFMA (Sec. 2: eq. (1) and the conjugate transpose).
//
// A view multiplies the big matrix A (four FP32 planes) by a thin quaternion block B:
//   C = A B      C_p = sum_q s(p, q) A_q B_{p^q}
//   C = A^H B    C_p = sum_q s(p, q) e_q A_q^T B_{p^q},   e = (+1, -1, -1, -1)
// where e_q e_{p^q} = s(p, q) e_p is the Hamilton product of the units (eq. (1)).  All 16
// plane products are real GEMMs that share operands: each A_q fragment feeds four output
// planes and each B_r fragment feeds four, so one pass over A computes the whole quaternion
// product with A read once.
//
// Kernel families:
//  - k_qview (math = MATH_F32): the views.  FP32 operands loaded straight from global memory
//    in MFMA operand order (the thin block transposed first by k_thin_t), v_mfma_f32_16x16x4f32,
//    FP32 accumulation; see the section below.
//  - k_qgemm_hn / k_qgemm_nn (math = MATH_F64, FP32 operands, and FP64 for the small right
//    operand of A B): Gram matrices, Krylov projections, CholeskyQR applies and the
//    back-multiplication.  Four waves of 16 x 16 per 32 x 32 output tile of all four planes, the
//    operands loaded straight from global memory in v_mfma_f64_16x16x4f64 operand order and
//    converted to FP64 (exact for FP32 data), no LDS and no barrier in the K loop.
//  - k_qgemm (math = MATH_F64): the products of FP64 operands (the blocked Cholesky's off-diagonal
//    blocks) and the fallback for layouts the direct kernels do not take.  A workgroup of 4 waves
//    owns a BM x BN tile of all four output planes; per K step the four planes of an A tile and of
//    a B tile are staged through LDS in FP64; the MFMA A operand always comes from the A tile,
//    stored row-major for A B and k-major for A^H B, so one kernel serves both orientations.
//  - k_qgemm_lp (MATH_BF16 / MATH_F16): the reduced-precision views, and (with the residual
//    copies staged beside the values) the split forms (MATH_BF16X3 / MATH_F16X3).
// When the output tiles cannot fill the chip, K is split across workgroups; partial tiles go to
// scratch and an element-parallel kernel adds them in split order (deterministic, no
// floating-point atomics).
#include "common.h"

#include <algorithm>
#include <type_traits>

namespace qlra_impl {
namespace {

template <class T>
struct Mma;

template <>
struct Mma<float> {
    using acc_t = f32x4;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // D element (lane, i) sits at row 4 (lane / 16) + i, column lane % 16.
    static __device__ __forceinline__ int row_of(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <>
struct Mma<double> {
    using acc_t = f64x4;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // D element (lane, i) sits at row lane / 16 + 4 i, column lane % 16.
    static __device__ __forceinline__ int row_of(int lane, int i) { return (lane >> 4) + 4 * i; }
};

// e_q e_{p^q} = hsign(p, q) e_p (eq. (1)).
__host__ __device__ constexpr int hsign(int p, int q) {
    return (p == 0) ? (q == 0 ? 1 : -1)
         : (p == 1) ? (q == 3 ? -1 : 1)
         : (p == 2) ? (q == 1 ? -1 : 1)
                    : (q == 2 ? -1 : 1);
}
template <bool ADJ>
__host__ __device__ constexpr int term_sign(int p, int q) {
    return ADJ && q != 0 ? -hsign(p, q) : hsign(p, q);
}

struct KParams {
    const void* A; int64_t lda, aps;
    const void* B; int64_t ldb, bps;
    void* C; int64_t ldc, cps;
    int64_t M, N, K;
    int64_t kchunk;
    int splits;
    void* part;
    int64_t Mp, Np;
    int store;
    int avec, bvec;      // 4-element vector loads allowed for A / B
    const int* skip;
    int sym;             // Hermitian Gram A^H A (B = A, square tiles): only tiles on or above the
                         // diagonal are computed, the others are their conjugate transposes
    int b_upper;         // B upper triangular: a column tile's reduction stops at its last column
    int xcd;             // Hermitian Gram in k_qgemm_hn on a 1-D grid of xtiles upper tiles x (splits
    int xtiles;          // rounded up to a multiple of 8) workgroups: split s on XCD s mod 8
};

// Four consecutive elements (along the contiguous dimension) of a plane, zero outside
// [0, valid).  Vector load when all four are valid and the layout allows it.
template <class TG, class T>
__device__ __forceinline__ void load4(const TG* __restrict__ p, int valid, bool vec, T out[4]) {
    if (valid >= 4 && vec) {
        if constexpr (sizeof(TG) == 4) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(p);
            out[0] = (T)v[0]; out[1] = (T)v[1]; out[2] = (T)v[2]; out[3] = (T)v[3];
        } else {
            typedef double d2 __attribute__((ext_vector_type(2)));
            const d2 v0 = reinterpret_cast<const d2*>(p)[0], v1 = reinterpret_cast<const d2*>(p)[1];
            out[0] = (T)v0[0]; out[1] = (T)v0[1]; out[2] = (T)v1[0]; out[3] = (T)v1[1];
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; t++) out[t] = t < valid ? (T)p[t] : (T)0;
    }
}

template <class T, int WM, int WN, int RM, int CN, int BK, bool ADJ, class TA, class TB, class TC>
__global__ __launch_bounds__(256) void k_qgemm(KParams P) {
    static_assert(WM * WN == 4, "four waves");
    static_assert(BK % 4 == 0, "BK");
    constexpr int BM = WM * RM * 16, BN = WN * CN * 16;
    constexpr int AROWS = ADJ ? BK : BM;       // A tile rows in LDS
    constexpr int AST = ADJ ? BM + 4 : BK + 4; // A tile row stride (elements)
    constexpr int BST = BN + 4;
    // chunks of 4 contiguous elements per plane and their share per thread
    constexpr int ACH = BM * BK / 4, BCH = BK * BN / 4;
    constexpr int APT = (4 * ACH + 255) / 256, BPT = (4 * BCH + 255) / 256;
    __shared__ __attribute__((aligned(16))) T sA[4 * AROWS * AST];
    __shared__ __attribute__((aligned(16))) T sB[4 * BK * BST];

    if (P.skip && *P.skip == 0) return;
    if (P.sym && blockIdx.x > blockIdx.y) return;     // below the diagonal: the mirror of (y, x)
    using M_ = Mma<T>;
    using acc_t = typename M_::acc_t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t row0 = (int64_t)blockIdx.x * BM, col0 = (int64_t)blockIdx.y * BN;
    const int split = blockIdx.z;
    const int64_t kb = (int64_t)split * P.kchunk;
    int64_t ke = P.K < kb + P.kchunk ? P.K : kb + P.kchunk;
    if (P.b_upper && ke > col0 + BN) ke = col0 + BN;   // B(k, c) = 0 for k > c
    const TA* __restrict__ A = (const TA*)P.A;
    const TB* __restrict__ B = (const TB*)P.B;
    const bool avec = P.avec != 0, bvec = P.bvec != 0;

    acc_t acc[RM][CN][4];
#pragma unroll
    for (int rm = 0; rm < RM; rm++)
#pragma unroll
        for (int cn = 0; cn < CN; cn++)
#pragma unroll
            for (int p = 0; p < 4; p++) acc[rm][cn][p] = acc_t{0, 0, 0, 0};

    T ra[APT][4], rb[BPT][4];   // register stage of the next tiles

    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int it = 0; it < APT; it++) {
            const int ch = it * 256 + tid;
            if (ch >= 4 * ACH) break;
            const int q = ch / ACH, rem = ch % ACH;
            if (!ADJ) {
                const int r = rem / (BK / 4), kq = rem % (BK / 4);
                const int64_t gr = row0 + r, gk = k0 + 4 * kq;
                const int valid = gr < P.M ? (int)std::min<int64_t>(4, std::max<int64_t>(0, ke - gk)) : 0;
                load4<TA, T>(A + q * P.aps + gr * P.lda + gk, valid, avec, ra[it]);
            } else {
                const int kk = rem / (BM / 4), cq = rem % (BM / 4);
                const int64_t gk = k0 + kk, gr = row0 + 4 * cq;
                const int valid = gk < ke ? (int)std::min<int64_t>(4, std::max<int64_t>(0, P.M - gr)) : 0;
                load4<TA, T>(A + q * P.aps + gk * P.lda + gr, valid, avec, ra[it]);
            }
        }
#pragma unroll
        for (int it = 0; it < BPT; it++) {
            const int ch = it * 256 + tid;
            if (ch >= 4 * BCH) break;
            const int q = ch / BCH, rem = ch % BCH;
            const int kk = rem / (BN / 4), cq = rem % (BN / 4);
            const int64_t gk = k0 + kk, gc = col0 + 4 * cq;
            const int valid = gk < ke ? (int)std::min<int64_t>(4, std::max<int64_t>(0, P.N - gc)) : 0;
            load4<TB, T>(B + q * P.bps + gk * P.ldb + gc, valid, bvec, rb[it]);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int it = 0; it < APT; it++) {
            const int ch = it * 256 + tid;
            if (ch >= 4 * ACH) break;
            const int q = ch / ACH, rem = ch % ACH;
            T* dst;
            if (!ADJ) {
                const int r = rem / (BK / 4), kq = rem % (BK / 4);
                dst = &sA[(q * AROWS + r) * AST + 4 * kq];
            } else {
                const int kk = rem / (BM / 4), cq = rem % (BM / 4);
                dst = &sA[(q * AROWS + kk) * AST + 4 * cq];
            }
            dst[0] = ra[it][0]; dst[1] = ra[it][1]; dst[2] = ra[it][2]; dst[3] = ra[it][3];
        }
#pragma unroll
        for (int it = 0; it < BPT; it++) {
            const int ch = it * 256 + tid;
            if (ch >= 4 * BCH) break;
            const int q = ch / BCH, rem = ch % BCH;
            const int kk = rem / (BN / 4), cq = rem % (BN / 4);
            T* dst = &sB[(q * BK + kk) * BST + 4 * cq];
            dst[0] = rb[it][0]; dst[1] = rb[it][1]; dst[2] = rb[it][2]; dst[3] = rb[it][3];
        }
    };

    const int g = lane >> 4, r16 = lane & 15;
    if (kb < ke) fetch(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();          // previous tile fully consumed
        stash();
        __syncthreads();
        if (k0 + BK < ke) fetch(k0 + BK);   // in flight during the MFMAs below
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            T a[4][RM];
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int rm = 0; rm < RM; rm++) {
                    const int r = (wm * RM + rm) * 16 + r16, kk = ks + g;
                    a[q][rm] = ADJ ? sA[(q * AROWS + kk) * AST + r] : sA[(q * AROWS + r) * AST + kk];
                }
            T b[CN][4], nb[CN][4];
#pragma unroll
            for (int cn = 0; cn < CN; cn++) {
                const int c = (wn * CN + cn) * 16 + r16;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    b[cn][q] = sB[(q * BK + ks + g) * BST + c];
                    nb[cn][q] = -b[cn][q];
                }
            }
            // q outermost: consecutive MFMAs update different accumulators
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int rm = 0; rm < RM; rm++)
#pragma unroll
                    for (int cn = 0; cn < CN; cn++)
#pragma unroll
                        for (int p = 0; p < 4; p++)
                            acc[rm][cn][p] = M_::mma(a[q][rm],
                                                     term_sign<ADJ>(p, q) > 0 ? b[cn][p ^ q] : nb[cn][p ^ q],
                                                     acc[rm][cn][p]);
        }
    }

    if (P.splits == 1) {
        TC* __restrict__ C = (TC*)P.C;
#pragma unroll
        for (int rm = 0; rm < RM; rm++)
#pragma unroll
            for (int cn = 0; cn < CN; cn++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int64_t r = row0 + (wm * RM + rm) * 16 + M_::row_of(lane, i);
                    const int64_t c = col0 + (wn * CN + cn) * 16 + r16;
                    if (r < P.M && c < P.N) {
#pragma unroll
                        for (int p = 0; p < 4; p++) {
                            TC* dst = C + p * P.cps + r * P.ldc + c;
                            const T v = acc[rm][cn][p][i];
                            *dst = P.store == ST_SUB ? (TC)((T)*dst - v) : (TC)v;
                            // an off-diagonal tile of a Hermitian Gram also gives (c, r) = conj(r, c)
                            if (P.sym && blockIdx.x < blockIdx.y) C[p * P.cps + c * P.ldc + r] = (TC)(p ? -v : v);
                        }
                    }
                }
        return;
    }
    // split K: publish this split's partial tile
    T* __restrict__ part = (T*)P.part;
#pragma unroll
    for (int rm = 0; rm < RM; rm++)
#pragma unroll
        for (int cn = 0; cn < CN; cn++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t r = row0 + (wm * RM + rm) * 16 + M_::row_of(lane, i);
                const int64_t c = col0 + (wn * CN + cn) * 16 + r16;
#pragma unroll
                for (int p = 0; p < 4; p++)
                    part[(((int64_t)split * 4 + p) * P.Mp + r) * P.Np + c] = acc[rm][cn][p][i];
            }
}

// C (M x N, 4 planes) = sum over splits of the partial tiles: one thread per output entry, the
// splits added in order (deterministic), eight loads in flight; the threads of a wave read 64
// consecutive entries of one partial tile.  sym_bm > 0 (a Hermitian Gram with square tiles of
// sym_bm): only the tiles on and above the diagonal have partials; the thread of an entry in a
// tile above the diagonal also writes its mirror, the conjugate.
template <class T, class TC>
__global__ __launch_bounds__(256) void k_splitk_reduce(const T* __restrict__ part, int splits, int64_t Mp, int64_t Np,
                                                       TC* __restrict__ C, int64_t ldc, int64_t cps, int64_t M,
                                                       int64_t N, int store, const int* skip, int sym_bm) {
    if (skip && *skip == 0) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4 * M * N) return;
    const int64_t p = e / (M * N), rem = e - p * M * N, r = rem / N, c = rem - r * N;
    if (sym_bm > 0 && r / sym_bm > c / sym_bm) return;        // written by the thread of its mirror
    const int64_t stride = 4 * Mp * Np;
    const T* src = part + (p * Mp + r) * Np + c;
    T s = 0;
    int sp = 0;
    for (; sp + 8 <= splits; sp += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = src[(int64_t)(sp + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; u++) s += v[u];
    }
    for (; sp < splits; sp++) s += src[(int64_t)sp * stride];
    TC* dst = C + p * cps + r * ldc + c;
    *dst = store == ST_SUB ? (TC)((T)*dst - s) : (TC)s;
    if (sym_bm > 0 && r / sym_bm < c / sym_bm) C[p * cps + c * ldc + r] = (TC)(p ? -s : s);
}

// The same sum for FP32 partials and outputs whose rows are 16-byte aligned: one thread per
// four consecutive outputs, the splits added in order (deterministic).
__global__ __launch_bounds__(256) void k_splitk_reduce4(const float* __restrict__ part, int splits, int64_t Mp,
                                                        int64_t Np, float* __restrict__ C, int64_t ldc, int64_t cps,
                                                        int64_t M, int64_t N, int store, const int* skip) {
    if (skip && *skip == 0) return;
    const int64_t nq = N / 4;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4 * M * nq) return;
    const int64_t p = e / (M * nq), rem = e - p * M * nq, r = rem / nq, c = 4 * (rem - r * nq);
    const int64_t stride = 4 * Mp * Np;
    const float* src = part + (p * Mp + r) * Np + c;
    f32x4 s = *reinterpret_cast<const f32x4*>(src);
    for (int sp = 1; sp < splits; sp++) s += *reinterpret_cast<const f32x4*>(src + sp * stride);
    f32x4* dst = reinterpret_cast<f32x4*>(C + p * cps + r * ldc + c);
    *dst = store == ST_SUB ? *dst - s : s;
}

// C = sum of the partial tiles, with the vector form when the layout allows it
hipError_t reduce_f32(const float* part, int splits, int64_t Mp, int64_t Np, float* C, int64_t ldc, int64_t cps,
                      int64_t M, int64_t N, int store, const int* skip, hipStream_t st) {
    if (N % 4 == 0 && ldc % 4 == 0 && cps % 4 == 0 && ((uintptr_t)C % 16) == 0) {
        const int64_t total = 4 * M * (N / 4);
        hipLaunchKernelGGL(k_splitk_reduce4, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, splits,
                           Mp, Np, C, ldc, cps, M, N, store, skip);
    } else {
        const int64_t total = 4 * M * N;
        hipLaunchKernelGGL((k_splitk_reduce<float, float>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           part, splits, Mp, Np, C, ldc, cps, M, N, store, skip, 0);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// FP32 views: operands straight from global memory, no LDS in the K loop.
//
// Each wave owns one output tile of 16 rows x 16 CN columns in all four planes (4 CN
// accumulators of 16 x 16) over a contiguous stretch of K, and loads both operands in the
// order the MFMA consumes them.  Lane (r, g) = (l % 16, l / 16) supplies, for the j-th of the
// four MFMAs of a 16-wide K step, reduction index k0 + 4 g + j:
//  - A X:    A_q[row r][k0 + 4 g .. + 3], one 16-byte load per plane (element j feeds MFMA j);
//  - A^H X:  the same elements of A^T, A_q[k0 + 4 g + j][row r]: four loads per plane, the 16
//            lanes of a group reading 64 contiguous bytes of a row of A;
//  - B:      the thin block is first transposed to Bt[q][column][k] (k contiguous, zero padded
//            to Kp and Np), so that B_q[k0 + 4 g .. + 3][column r] is one 16-byte load.
// Every A element is loaded by exactly one wave, once; Bt is re-read from L2 by every row tile.
// There is no barrier in the K loop: each wave streams on its own, operands one step ahead in
// ping-pong registers (A^H X: A slice j refilled right after its use).  The signs of eq. (1)
// go on the A operand (one negated copy per plane), shared by all output planes and column
// tiles.  KW waves of a workgroup may share an output tile, each over 1/KW of the workgroup's
// K range; their sums are added in wave order through LDS (deterministic), and K splits across
// workgroups go through the ordered split-K reduction.

constexpr int VBK = 16;   // K per step: four MFMAs of k = 4

struct VParams {
    const float* A; int64_t lda, aps;
    const float* Bt; int64_t kp, bps;   // Bt[q][c][k]: column stride kp, plane stride bps
    float* C; int64_t ldc, cps;
    int64_t M, N, K;
    int64_t kchunk;      // K per workgroup, a multiple of VBK * kw
    int splits;
    int kw;              // waves per output tile: 1, 2 or 4
    int64_t tiles, gy;   // output tiles (row tiles x column tiles) and column tiles
    float* part; int64_t Mp, Np;
    int store;
    const int* skip;
    double* fro;         // FRO: per-wave sums of squares of the A elements (slot = wave of the grid)
};

// B (K x N, four planes, row-major) -> Bt[q][c][k] (Np x Kp per plane), zero outside K x N;
// tiles of 16 reduction rows x 64 columns through LDS (reads coalesced along the columns,
// writes 64-byte runs along k), enough workgroups to spread over the chip
__global__ __launch_bounds__(256) void k_thin_t(const float* __restrict__ B, int64_t ldb, int64_t bps, int64_t K,
                                                int64_t N, float* __restrict__ Bt, int64_t Np, int64_t Kp,
                                                const int* skip) {
    __shared__ float t[16][65];
    if (skip && *skip == 0) return;
    const int64_t k0 = (int64_t)blockIdx.x * 16, c0 = (int64_t)blockIdx.y * 64;
    const int q = blockIdx.z, tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int i = ty; i < 16; i += 4) {
        const int64_t k = k0 + i, c = c0 + tx;
        t[i][tx] = (k < K && c < N) ? B[q * bps + k * ldb + c] : 0.0f;
    }
    __syncthreads();
    const int kk = threadIdx.x & 15, cc = threadIdx.x >> 4;
#pragma unroll
    for (int i = cc; i < 64; i += 16) {
        const int64_t c = c0 + i, k = k0 + kk;
        if (c < Np && k < Kp) Bt[((int64_t)q * Np + c) * Kp + k] = t[kk][i];
    }
}

template <int CN, bool ADJ, bool AVEC, bool FRO, bool REALB>
__global__ __launch_bounds__(256, CN <= 3 ? 2 : 1) void k_qview(VParams P) {
    __shared__ f32x4 xch[4][CN * 4][64];
    if (P.skip && *P.skip == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kw = P.kw;
    // workgroups go round-robin to the 8 XCDs; give each XCD a contiguous run of row tiles so that
    // neighbouring tiles (which share 128-byte lines of A in A^H X) meet in the same L2
    const int64_t G = gridDim.x;
    const int64_t bx = (G % 8 == 0) ? (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : (int64_t)blockIdx.x;
    const int64_t tile_raw = bx * (4 / kw) + wave / kw;
    const bool tile_ok = tile_raw < P.tiles;
    const int64_t tile = tile_ok ? tile_raw : P.tiles - 1;
    const int kpart = wave % kw;
    const int64_t rt = tile / P.gy, ct = tile % P.gy;
    const int64_t row0 = rt * 16, col0 = ct * 16 * CN;
    const int64_t kc0 = (int64_t)blockIdx.z * P.kchunk;
    const int64_t kc1 = P.K < kc0 + P.kchunk ? P.K : kc0 + P.kchunk;
    const int64_t sub = P.kchunk / kw;
    const int64_t kb = kc0 + kpart * sub < kc1 ? kc0 + kpart * sub : kc1;
    const int64_t ke = kb + sub < kc1 ? kb + sub : kc1;
    const int r = lane & 15, g = lane >> 4;
    // rows past the edge are clamped (never stored); Bt is zero past K and N, so only A needs
    // masking in a ragged last step
    const int64_t arow = row0 + r < P.M ? row0 + r : P.M - 1;
    const float* __restrict__ A = P.A;
    const float* bcol[CN];
#pragma unroll
    for (int cn = 0; cn < CN; cn++) bcol[cn] = P.Bt + (col0 + 16 * cn + r) * P.kp + 4 * g;
    const int64_t klast = ke - 1;

    f32x4 acc[CN][4];
#pragma unroll
    for (int cn = 0; cn < CN; cn++)
#pragma unroll
        for (int p = 0; p < 4; p++) acc[cn][p] = f32x4{0, 0, 0, 0};
    // FRO (A X): ||A||_F^2 on the side, from the first column tile's waves, rows inside A only
    double fro = 0.0;
    const double fro_w = (FRO && ct == 0 && row0 + r < P.M) ? 1.0 : 0.0;

    constexpr bool A4 = AVEC && !ADJ;   // A as 16-byte loads
    auto a_elem = [&](int q, int64_t k) -> const float* {
        return ADJ ? A + q * P.aps + k * P.lda + arow : A + q * P.aps + arow * P.lda + k;
    };
    auto load_a = [&](int64_t k0, f32x4 (&a)[4]) {
        if constexpr (A4) {
#pragma unroll
            for (int q = 0; q < 4; q++) a[q] = *reinterpret_cast<const f32x4*>(a_elem(q, k0 + 4 * g));
        } else {
#pragma unroll
            for (int j = 0; j < 4; j++)
#pragma unroll
                for (int q = 0; q < 4; q++) a[q][j] = *a_elem(q, k0 + 4 * g + j);
        }
    };
    // REALB: the thin block is real (a real sketch); only its real plane is read and only the
    // q = p terms of eq. (1) remain, a quarter of the MFMAs
    auto load_b = [&](int64_t k0, f32x4 (&b)[CN][4]) {
#pragma unroll
        for (int cn = 0; cn < CN; cn++)
#pragma unroll
            for (int q = 0; q < (REALB ? 1 : 4); q++)
                b[cn][q] = *reinterpret_cast<const f32x4*>(bcol[cn] + q * P.bps + k0);
    };
    auto mma_slice = [&](const f32x4 (&a)[4], int j, const f32x4 (&b)[CN][4]) {
        float av[4], nav[4];
#pragma unroll
        for (int q = 0; q < 4; q++) { av[q] = a[q][j]; nav[q] = -av[q]; }
        if constexpr (FRO) {
#pragma unroll
            for (int q = 0; q < 4; q++) fro = fma((double)av[q], (double)av[q], fro);
        }
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int cn = 0; cn < CN; cn++)
#pragma unroll
                for (int pp = 0; pp < 4; pp++) {
                    if (REALB && pp != q) continue;
                    acc[cn][pp] = __builtin_amdgcn_mfma_f32_16x16x4f32(term_sign<ADJ>(pp, q) > 0 ? av[q] : nav[q],
                                                                       b[cn][pp ^ q][j], acc[cn][pp], 0, 0, 0);
                }
    };
    // one full step from registers; the loads of the step `kn` go out a quarter after each slice
    // of MFMAs, so that no burst of loads stalls the issue of the matrix instructions
    // (A^H X: A slice j refilled right after slice j is used)
    auto step = [&](f32x4 (&a)[4], const f32x4 (&b)[CN][4], f32x4 (&an)[4], f32x4 (&bn)[CN][4], int64_t kn) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            __builtin_amdgcn_sched_barrier(0);
            mma_slice(a, j, b);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int e = j * CN; e < (j + 1) * CN; e++) {
                const int cn = e / 4, q = e % 4;
                if (REALB && q != 0) continue;
                bn[cn][q] = *reinterpret_cast<const f32x4*>(bcol[cn] + q * P.bps + kn);
            }
            if constexpr (A4) {
                an[j] = *reinterpret_cast<const f32x4*>(a_elem(j, kn + 4 * g));
            } else {
#pragma unroll
                for (int q = 0; q < 4; q++) a[q][j] = *a_elem(q, kn + 4 * g + j);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    };

    const int64_t len = (tile_ok && ke > kb) ? ke - kb : 0;
    const int64_t nfull = len / VBK;
    if (nfull > 0) {
        f32x4 a0[4], a1[4], b0[CN][4], b1[CN][4];
        load_a(kb, a0);
        load_b(kb, b0);
        // steps in pairs with ping-pong registers (no copies); a step past the last full one
        // reloads the last (in bounds, unused)
        const int64_t kl = kb + (nfull - 1) * VBK;
#pragma unroll 1
        for (int64_t st = 0; st < nfull; st += 2) {
            const int64_t k0 = kb + st * VBK;
            const int64_t k1 = k0 + VBK <= kl ? k0 + VBK : kl;
            const int64_t k2 = k0 + 2 * VBK <= kl ? k0 + 2 * VBK : kl;
            if constexpr (A4) {
                step(a0, b0, a1, b1, k1);
                if (st + 1 < nfull) step(a1, b1, a0, b0, k2);
            } else {
                // the A ring refills a in place: both steps use the same registers
                step(a0, b0, a0, b1, k1);
                if (st + 1 < nfull) step(a0, b1, a0, b0, k2);
            }
        }
    }
    if (len % VBK) {
        // ragged last step: A clamped and zeroed past ke (Bt is zero there already)
        const int64_t k0 = kb + nfull * VBK;
        f32x4 a[4], b[CN][4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t k = k0 + 4 * g + j;
            const int64_t kk = k < ke ? k : klast;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float v = *a_elem(q, kk);
                a[q][j] = k < ke ? v : 0.0f;
            }
        }
        load_b(k0, b);
#pragma unroll
        for (int j = 0; j < 4; j++) mma_slice(a, j, b);
    }

    if constexpr (FRO) {
        fro *= fro_w;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) fro += __shfl_xor(fro, o, 64);
        if (lane == 0) P.fro[((int64_t)blockIdx.z * gridDim.x + bx) * 4 + wave] = fro;
    }

    if (kw > 1) {
        if (kpart > 0) {
#pragma unroll
            for (int cn = 0; cn < CN; cn++)
#pragma unroll
                for (int pp = 0; pp < 4; pp++) xch[wave][cn * 4 + pp][lane] = acc[cn][pp];
        }
        __syncthreads();
        if (kpart == 0) {
            for (int t = 1; t < kw; t++) {
#pragma unroll
                for (int cn = 0; cn < CN; cn++)
#pragma unroll
                    for (int pp = 0; pp < 4; pp++) acc[cn][pp] += xch[wave + t][cn * 4 + pp][lane];
            }
        }
    }
    if (kpart != 0 || !tile_ok) return;

    // D element (lane, i) of the 16 x 16 x 4 FP32 MFMA sits at row 4 (lane / 16) + i, column lane % 16
    if (P.splits == 1) {
#pragma unroll
        for (int cn = 0; cn < CN; cn++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t row = row0 + 4 * g + i, col = col0 + 16 * cn + r;
                if (row < P.M && col < P.N) {
#pragma unroll
                    for (int pp = 0; pp < 4; pp++) {
                        float* dst = P.C + pp * P.cps + row * P.ldc + col;
                        *dst = P.store == ST_SUB ? *dst - acc[cn][pp][i] : acc[cn][pp][i];
                    }
                }
            }
        return;
    }
#pragma unroll
    for (int cn = 0; cn < CN; cn++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t row = row0 + 4 * g + i, col = col0 + 16 * cn + r;
#pragma unroll
            for (int pp = 0; pp < 4; pp++)
                P.part[(((int64_t)blockIdx.z * 4 + pp) * P.Mp + row) * P.Np + col] = acc[cn][pp][i];
        }
}

// ------------------------------------------------------------------------------------------
// FP64 A^H B of FP32 operands (Grams, Krylov projections): operands straight from global memory.
//
// The same tiles, K splits and partial layout as k_qgemm (32 x 32 output tiles, four waves of
// 16 x 16, steps of 16 reduction rows), but no LDS and no barrier: each wave loads its own
// fragments in the order v_mfma_f64_16x16x4f64 consumes them.  Lane (r, g) = (l % 16, l / 16)
// supplies, for the j-th of the four MFMAs of a step, reduction row k0 + 4 g + j: A_q(k, i0 + r)
// for the A^H operand and B_q(k, j0 + r) for B, each a 4-byte load (the 16 lanes of a group
// read 64 contiguous bytes of a row), converted to FP64 (exact).  The loads of step s + 1 are in
// flight during the MFMAs of step s.  The signs of eq. (1) go on a negated copy of the A^H
// fragment.  Rows past the K range and columns past M or N load zeros.
template <bool SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_qgemm_hn(KParams P) {
    if (P.skip && *P.skip == 0) return;
    int bx = blockIdx.x, by = blockIdx.y, split = blockIdx.z;
    if (SYM && P.xcd) {
        // workgroup L is dispatched to XCD L mod 8: split 8 q + (L mod 8) takes upper tile
        // t = (L / 8) mod xtiles, so that all the tiles of a split (one range of K rows) share one
        // XCD's L2; the grid is rounded up to whole rounds of 8 splits, and the workgroups past
        // the last split do nothing
        const int L = blockIdx.x, u = L >> 3, t = u % P.xtiles;
        split = 8 * (u / P.xtiles) + (L & 7);
        if (split >= P.splits) return;
        // t = by (by + 1) / 2 + bx, 0 <= bx <= by
        by = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while (by * (by + 1) / 2 > t) by--;
        while ((by + 1) * (by + 2) / 2 <= t) by++;
        bx = t - by * (by + 1) / 2;
    }
    if (SYM && bx > by) return;     // below the diagonal: the mirror of (by, bx)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t row0 = (int64_t)bx * 32 + wm * 16, col0 = (int64_t)by * 32 + wn * 16;
    const int64_t kb = (int64_t)split * P.kchunk;
    int64_t ke = P.K < kb + P.kchunk ? P.K : kb + P.kchunk;
    if (P.b_upper && ke > (int64_t)by * 32 + 32) ke = (int64_t)by * 32 + 32;   // B(k, c) = 0 for k > c
    const float* __restrict__ A = (const float*)P.A;
    const float* __restrict__ B = (const float*)P.B;
    const int r = lane & 15, g = lane >> 4;
    const bool aok = row0 + r < P.M, bok = col0 + r < P.N;
    // per-lane byte offsets (32-bit: the launcher checks the range) from uniform row bases
    const unsigned aofs = (unsigned)((4 * g * P.lda + (aok ? row0 + r : 0)) * sizeof(float));
    const unsigned bofs = (unsigned)((4 * g * P.ldb + (bok ? col0 + r : 0)) * sizeof(float));

    f64x4 acc[4];
#pragma unroll
    for (int p = 0; p < 4; p++) acc[p] = f64x4{0, 0, 0, 0};

    // one step's operands: fa[q][j] = A_q(k0 + 4 g + j, i0 + r), fb[q][j] likewise for B
    // a full step (rows k0 .. k0 + 15 all below ke) loads unconditionally: a lane past M or N reads
    // column 0, which only reaches output rows or columns that are never stored
    auto fetch = [&](int64_t k0, float (&fa)[4][4], float (&fb)[4][4]) {
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const char* arow = (const char*)(A + q * P.aps + (k0 + j) * P.lda);   // uniform over the wave
                const char* brow = (const char*)(B + q * P.bps + (k0 + j) * P.ldb);
                fa[q][j] = *(const float*)(arow + aofs);
                fb[q][j] = *(const float*)(brow + bofs);
            }
    };
    // a ragged last step masks its rows (they may lie past K)
    auto fetch_tail = [&](int64_t k0, float (&fa)[4][4], float (&fb)[4][4]) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const bool kin = k0 + 4 * g + j < ke;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const char* arow = (const char*)(A + q * P.aps + (k0 + j) * P.lda);
                const char* brow = (const char*)(B + q * P.bps + (k0 + j) * P.ldb);
                fa[q][j] = kin ? *(const float*)(arow + aofs) : 0.0f;
                fb[q][j] = kin ? *(const float*)(brow + bofs) : 0.0f;
            }
        }
    };
    auto step = [&](const float (&fa)[4][4], const float (&fb)[4][4]) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            double a[4], na[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                a[q] = (double)fa[q][j];
                na[q] = -a[q];
                b[q] = (double)fb[q][j];
            }
            // q outermost: consecutive MFMAs update different accumulators
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int p = 0; p < 4; p++)
                    acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(term_sign<true>(p, q) > 0 ? a[q] : na[q], b[p ^ q],
                                                                  acc[p], 0, 0, 0);
        }
    };

    // nf full steps, then a ragged one if K's range does not end on a step; the operands of the
    // next step are in flight during the MFMAs of the current one (ping-pong x / y; a fetch
    // past the last full step reloads it, so that every fetch in the loop is unconditional)
    const int64_t nf = kb < ke ? (ke - kb) / 16 : 0;
    float xa[4][4], xb[4][4], ya[4][4], yb[4][4];
    if (nf > 0) fetch(kb, xa, xb);
    int64_t t = 0;
    for (; t + 1 < nf; t += 2) {
        // the order is pinned (sched_barrier): a step's conversions and MFMAs stay after the next
        // step's loads are issued and never wait for them
        fetch(kb + 16 * (t + 1), ya, yb);
        __builtin_amdgcn_sched_barrier(0);
        step(xa, xb);
        __builtin_amdgcn_sched_barrier(0);
        fetch(kb + 16 * (t + 2 < nf ? t + 2 : nf - 1), xa, xb);
        __builtin_amdgcn_sched_barrier(0);
        step(ya, yb);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (t < nf) step(xa, xb);
    if (kb + 16 * nf < ke) {
        fetch_tail(kb + 16 * nf, ya, yb);
        step(ya, yb);
    }

    // D element (lane, i) of v_mfma_f64_16x16x4f64 sits at row lane / 16 + 4 i, column lane % 16
    if (P.splits == 1) {
        double* __restrict__ C = (double*)P.C;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t rr = row0 + g + 4 * i, c = col0 + r;
            if (rr < P.M && c < P.N) {
#pragma unroll
                for (int p = 0; p < 4; p++) {
                    const double v = acc[p][i];
                    double* dst = C + p * P.cps + rr * P.ldc + c;
                    *dst = P.store == ST_SUB ? *dst - v : v;
                    // an off-diagonal tile of a Hermitian Gram also gives (c, rr) = conj(rr, c)
                    if (SYM && bx < by) C[p * P.cps + c * P.ldc + rr] = p ? -v : v;
                }
            }
        }
        return;
    }
    double* __restrict__ part = (double*)P.part;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int64_t rr = row0 + g + 4 * i, c = col0 + r;
#pragma unroll
        for (int p = 0; p < 4; p++) part[(((int64_t)split * 4 + p) * P.Mp + rr) * P.Np + c] = acc[p][i];
    }
}

// ------------------------------------------------------------------------------------------
// FP64 A B of an FP32 tall operand and an FP64 small one (CholeskyQR applies, Krylov
// projections, the back-multiplication): operands straight from global memory, the tiles, K
// splits and partial layout of the 2 x 2 plan.  Lane (r, g) supplies, for the j-th of the four
// MFMAs of a step, reduction index k0 + 4 g + j: A_q(i0 + r, k0 + 4 g .. + 3) is one 16-byte load
// per plane (element j feeds MFMA j) and B_q(k0 + 4 g + j, j0 + r) an 8-byte load.  The loads of
// step s + 1 are in flight during the MFMAs of step s.  Rows past M and columns past N read row
// or column 0 and are never stored; a ragged last step masks its elements.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_qgemm_nn(KParams P) {
    if (P.skip && *P.skip == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    // with a triangular right operand the column tiles further right reduce over more rows: they
    // are dispatched first, so that the short ones fill in behind them
    const int64_t ty = P.b_upper ? (int64_t)gridDim.y - 1 - blockIdx.y : (int64_t)blockIdx.y;
    const int64_t row0 = (int64_t)blockIdx.x * 32 + wm * 16, col0 = ty * 32 + wn * 16;
    const int split = blockIdx.z;
    const int64_t kb = (int64_t)split * P.kchunk;
    int64_t ke = P.K < kb + P.kchunk ? P.K : kb + P.kchunk;
    if (P.b_upper && ke > ty * 32 + 32) ke = ty * 32 + 32;   // B(k, c) = 0 for k > c
    const float* __restrict__ A = (const float*)P.A;
    const double* __restrict__ B = (const double*)P.B;
    const int r = lane & 15, g = lane >> 4;
    // per-lane byte offsets (32-bit: the launcher checks the range) from uniform bases
    const unsigned aofs = (unsigned)(((row0 + r < P.M ? row0 + r : 0) * P.lda + 4 * g) * sizeof(float));
    const unsigned bofs = (unsigned)(((col0 + r < P.N ? col0 + r : 0) + 4 * g * P.ldb) * sizeof(double));
    auto at_a = [&](int64_t e) -> const float* { return (const float*)((const char*)(A + e) + aofs); };
    auto at_b = [&](int64_t e) -> const double* { return (const double*)((const char*)(B + e) + bofs); };

    f64x4 acc[4];
#pragma unroll
    for (int p = 0; p < 4; p++) acc[p] = f64x4{0, 0, 0, 0};

    auto fetch = [&](int64_t k0, f32x4 (&fa)[4], double (&fb)[4][4]) {
#pragma unroll
        for (int q = 0; q < 4; q++) fa[q] = *reinterpret_cast<const f32x4*>(at_a(q * P.aps + k0));
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) fb[q][j] = *at_b(q * P.bps + (k0 + j) * P.ldb);
    };
    auto fetch_tail = [&](int64_t k0, f32x4 (&fa)[4], double (&fb)[4][4]) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const bool kin = k0 + 4 * g + j < ke;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                fa[q][j] = kin ? *at_a(q * P.aps + k0 + j) : 0.0f;
                fb[q][j] = kin ? *at_b(q * P.bps + (k0 + j) * P.ldb) : 0.0;
            }
        }
    };
    auto step = [&](const f32x4 (&fa)[4], const double (&fb)[4][4]) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            double a[4], na[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                a[q] = (double)fa[q][j];
                na[q] = -a[q];
            }
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int p = 0; p < 4; p++)
                    acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(term_sign<false>(p, q) > 0 ? a[q] : na[q],
                                                                  fb[p ^ q][j], acc[p], 0, 0, 0);
        }
    };

    const int64_t nf = kb < ke ? (ke - kb) / 16 : 0;
    f32x4 xa[4], ya[4];
    double xb[4][4], yb[4][4];
    if (nf > 0) fetch(kb, xa, xb);
    int64_t t = 0;
    for (; t + 1 < nf; t += 2) {
        // the order is pinned (sched_barrier): a step's conversions and MFMAs stay after the next
        // step's loads are issued and never wait for them
        fetch(kb + 16 * (t + 1), ya, yb);
        __builtin_amdgcn_sched_barrier(0);
        step(xa, xb);
        __builtin_amdgcn_sched_barrier(0);
        fetch(kb + 16 * (t + 2 < nf ? t + 2 : nf - 1), xa, xb);
        __builtin_amdgcn_sched_barrier(0);
        step(ya, yb);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (t < nf) step(xa, xb);
    if (kb + 16 * nf < ke) {
        fetch_tail(kb + 16 * nf, ya, yb);
        step(ya, yb);
    }

    // D element (lane, i) of v_mfma_f64_16x16x4f64 sits at row lane / 16 + 4 i, column lane % 16
    if (P.splits == 1) {
        float* __restrict__ C = (float*)P.C;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t rr = row0 + g + 4 * i, c = col0 + r;
            if (rr < P.M && c < P.N) {
#pragma unroll
                for (int p = 0; p < 4; p++) {
                    float* dst = C + p * P.cps + rr * P.ldc + c;
                    const double v = acc[p][i];
                    *dst = P.store == ST_SUB ? (float)((double)*dst - v) : (float)v;
                }
            }
        }
        return;
    }
    double* __restrict__ part = (double*)P.part;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int64_t rr = row0 + g + 4 * i, c = col0 + r;
#pragma unroll
        for (int p = 0; p < 4; p++) part[(((int64_t)split * 4 + p) * P.Mp + rr) * P.Np + c] = acc[p][i];
    }
}

// ------------------------------------------------------------------------------------------
// configuration choice

struct Plan {
    int WM, WN, RM, CN, BK;
    int64_t gx, gy, splits, kchunk, Mp, Np;
    bool xcd;   // Hermitian Gram of FP32 data in 8 splits, each on one XCD
};

constexpr int kCUs = 256;
constexpr int kGramWgPerCU = 4;   // split-K workgroups per CU for Gram-like (A^H B) products

// A Hermitian Gram X^H X: the same operand on both sides, a square output set outright.
bool is_sym_gram(const QgemmDesc& d) {
    return d.math == MATH_F64 && d.op == OP_HN && d.A == d.B && d.lda == d.ldb && d.aps == d.bps &&
           d.a_f64 == d.b_f64 && d.M == d.N && d.store == ST_SET;
}

// FP32 A times FP64 B into FP32, with 16-byte aligned rows of A: the direct kernel k_qgemm_nn
bool nn_direct(const QgemmDesc& d) {
    return d.math == MATH_F64 && d.op == OP_NN && !d.a_f64 && d.b_f64 && !d.c_f64 && ((uintptr_t)d.A % 16) == 0 &&
           d.lda % 4 == 0 && d.aps % 4 == 0;
}

Plan make_plan(const QgemmDesc& d) {
    Plan p{};
    if (d.op == OP_HN || d.b_upper || nn_direct(d)) {
        // Gram-like products: small M x N output, long K; 32 x 32 tiles so that K splits
        // spread the FP64 MFMA work over many CUs.  Products with an upper triangular right
        // operand (Y R^{-1}) take them too: a column tile's reduction then stops 32 columns
        // apart, and w = 160 needs no padded columns.
        // FP32 times FP64 products (applies, projections, back-multiplication) take them in the
        // direct kernel: 160 columns are five tiles, no padding.
        p.BK = 16; p.WM = 2; p.WN = 2; p.RM = 1; p.CN = 1;
    } else {
        // tall times small with FP64 operands
        p.BK = 16; p.WM = 1; p.WN = 4; p.RM = 1; p.CN = 1;
    }
    const int64_t BM = p.WM * p.RM * 16, BN = p.WN * p.CN * 16;
    p.gx = (d.M + BM - 1) / BM;
    p.gy = (d.N + BN - 1) / BN;
    p.Mp = p.gx * BM;
    p.Np = p.gy * BN;
    // a Hermitian Gram computes the tiles on and above the diagonal only
    const int64_t tiles = is_sym_gram(d) ? p.gx * (p.gx + 1) / 2 : p.gx * p.gy;
    // split K so that several workgroups per CU run (Gram-like products: four, which hide the
    // latency of one another's loads, and no more, so that all of them run in the one round that
    // the direct kernel's occupancy holds; the others about one), each over at least 2 K steps
    const int64_t min_steps = 2;
    const bool gram_like = d.op == OP_HN;
    const int64_t target = gram_like ? kGramWgPerCU * kCUs : kCUs;
    int64_t splits = 1;
    // a tiny product with a short reduction (the blocked Cholesky's off-diagonal blocks) runs
    // unsplit: its few K steps cost less than the extra launch that would sum the partial tiles
    const bool tiny = d.K <= 128 && (double)d.M * (double)d.N * (double)d.K <= 1048576.0;
    if (tiles < target && !tiny) {
        splits = std::min<int64_t>(gram_like ? target / tiles : (target + tiles - 1) / tiles,
                                   (d.K + min_steps * p.BK - 1) / (min_steps * p.BK));
        splits = std::max<int64_t>(splits, 1);
    }
    // a Hermitian Gram of many tiles and a long reduction (fewer than 8 splits by the rule above,
    // e.g. 640 columns) in the direct kernel: 8 splits, one per XCD, whose tiles then read the
    // same K rows through that XCD's L2 instead of every XCD streaming all of K
    const bool direct_gram = is_sym_gram(d) && !d.a_f64 && !d.b_f64 && d.c_f64;
    const int64_t max_splits = (d.K + min_steps * p.BK - 1) / (min_steps * p.BK);
    const bool xcd8 = direct_gram && !tiny && tiles < target && splits < 8 && max_splits >= 8;
    if (xcd8) splits = 8;
    int64_t kchunk = (d.K + splits - 1) / splits;
    kchunk = ((kchunk + p.BK - 1) / p.BK) * p.BK;
    if (kchunk < p.BK) kchunk = p.BK;
    splits = (d.K + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    p.splits = splits;
    p.kchunk = kchunk;
    p.xcd = xcd8 && splits == 8;
    return p;
}

// the ordered sum of the split-K partial tiles into C (sym_bm > 0: Hermitian Gram with square
// tiles of sym_bm, the tiles below the diagonal mirrored)
template <class T, class TC>
hipError_t reduce_parts(const Plan& pl, const KParams& kp, int sym_bm, hipStream_t st) {
    const int64_t total = 4 * kp.M * kp.N;
    hipLaunchKernelGGL((k_splitk_reduce<T, TC>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       (const T*)kp.part, (int)pl.splits, pl.Mp, pl.Np, (TC*)kp.C, kp.ldc, kp.cps, kp.M, kp.N,
                       kp.store, kp.skip, sym_bm);
    return hipGetLastError();
}

template <class T, int WM, int WN, int RM, int CN, int BK, bool ADJ, class TA, class TB, class TC>
hipError_t launch_t(const Plan& pl, const KParams& kp, hipStream_t st) {
    dim3 grid((unsigned)pl.gx, (unsigned)pl.gy, (unsigned)pl.splits);
    hipLaunchKernelGGL((k_qgemm<T, WM, WN, RM, CN, BK, ADJ, TA, TB, TC>), grid, dim3(256), 0, st, kp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || pl.splits == 1) return e;
    if constexpr (std::is_same<T, float>::value && std::is_same<TC, float>::value)
        return reduce_f32((const float*)kp.part, (int)pl.splits, pl.Mp, pl.Np, (float*)kp.C, kp.ldc, kp.cps, kp.M,
                          kp.N, kp.store, kp.skip, st);
    return reduce_parts<T, TC>(pl, kp, kp.sym ? WM * RM * 16 : 0, st);
}

// k_qgemm_nn for the FP32 x FP64 products (the 2 x 2 plan; partials in FP64)
hipError_t launch_nn(const Plan& pl, const KParams& kp, hipStream_t st) {
    // the kernel's per-lane offsets are 32-bit
    const int64_t lim = (int64_t)1 << 30;
    if (kp.M * kp.lda + 16 >= lim || 2 * (kp.N + 12 * kp.ldb) >= lim)
        return launch_t<double, 2, 2, 1, 1, 16, false, float, double, float>(pl, kp, st);
    dim3 grid((unsigned)pl.gx, (unsigned)pl.gy, (unsigned)pl.splits);
    hipLaunchKernelGGL(k_qgemm_nn, grid, dim3(256), 0, st, kp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || pl.splits == 1) return e;
    return reduce_parts<double, float>(pl, kp, 0, st);
}

// k_qgemm_hn for the FP32 A^H B products (the tiles and partial layout of the 2 x 2 plan)
hipError_t launch_hn(const Plan& pl, const KParams& kp, hipStream_t st) {
    // the kernel's per-lane offsets are 32-bit
    const int64_t lim = (int64_t)1 << 30;
    if (12 * kp.lda + kp.M >= lim || 12 * kp.ldb + kp.N >= lim)
        return launch_t<double, 2, 2, 1, 1, 16, true, float, float, double>(pl, kp, st);
    dim3 grid((unsigned)pl.gx, (unsigned)pl.gy, (unsigned)pl.splits);
    KParams kx = kp;
    if (pl.xcd && kp.sym) {
        kx.xcd = 1;
        kx.xtiles = (int)(pl.gx * (pl.gx + 1) / 2);
        grid = dim3((unsigned)(kx.xtiles * ((pl.splits + 7) / 8 * 8)), 1, 1);   // past the last split: none
    }
    if (kp.sym) hipLaunchKernelGGL(k_qgemm_hn<true>, grid, dim3(256), 0, st, kx);
    else hipLaunchKernelGGL(k_qgemm_hn<false>, grid, dim3(256), 0, st, kx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || pl.splits == 1) return e;
    return reduce_parts<double, double>(pl, kp, kp.sym ? 32 : 0, st);
}

struct VPlan {
    int CN, kw;
    int64_t gy, tiles, splits, kchunk, Mp, Np, Kp, gx;
};

VPlan make_vplan(const QgemmDesc& d) {
    VPlan p{};
    if (d.N <= 64) {
        p.CN = (int)std::max<int64_t>(1, (d.N + 15) / 16);
    } else {
        // column tiles of at most 80, as even as possible (96 = 2 x 48, 160 = 2 x 80)
        const int64_t gy0 = (d.N + 79) / 80;
        p.CN = (int)((d.N + 16 * gy0 - 1) / (16 * gy0));
    }
    p.gy = (d.N + 16 * p.CN - 1) / (16 * p.CN);
    const int64_t rt = (d.M + 15) / 16;
    p.tiles = rt * p.gy;
    p.Mp = rt * 16;
    p.Np = p.gy * 16 * p.CN;
    p.Kp = (d.K + VBK - 1) / VBK * VBK;
    // one round of waves over the chip: two per SIMD where the registers allow it (CN <= 3), one
    // otherwise, so that every wave streams a long K range; the K range of a tile is cut into
    // parts of at least 4 steps, up to 4 parts inside a workgroup (combined in LDS), the rest
    // across workgroups
    const int64_t waves = (p.CN <= 3 ? 8 : 4) * kCUs;
    const int64_t need = (waves + p.tiles - 1) / p.tiles;
    const int64_t maxparts = std::max<int64_t>(1, d.K / (4 * VBK));
    const int64_t parts = std::min(need, maxparts);
    p.kw = parts >= 4 ? 4 : (parts >= 2 ? 2 : 1);
    const int64_t splits = (parts + p.kw - 1) / p.kw;
    const int64_t unit = VBK * p.kw;
    int64_t kchunk = (d.K + splits - 1) / splits;
    kchunk = std::max<int64_t>(unit, (kchunk + unit - 1) / unit * unit);
    p.kchunk = kchunk;
    p.splits = std::max<int64_t>(1, (d.K + kchunk - 1) / kchunk);
    p.gx = (p.tiles + 4 / p.kw - 1) / (4 / p.kw);
    return p;
}

size_t vplan_slots(const VPlan& p) { return (size_t)p.gx * 4 * (size_t)p.splits; }
size_t vplan_thin_bytes(const VPlan& p) { return ((size_t)4 * p.Np * p.Kp * sizeof(float) + 255) & ~size_t(255); }
size_t vplan_part_bytes(const VPlan& p) { return p.splits > 1 ? (size_t)p.splits * 4 * p.Mp * p.Np * sizeof(float) : 0; }

template <int CN, bool ADJ, bool AVEC, bool FRO, bool REALB>
hipError_t launch_v(const VPlan& pl, const VParams& vp, hipStream_t st) {
    hipLaunchKernelGGL((k_qview<CN, ADJ, AVEC, FRO, REALB>), dim3((unsigned)pl.gx, 1, (unsigned)pl.splits), dim3(256), 0, st, vp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || pl.splits == 1) return e;
    return reduce_f32(vp.part, (int)pl.splits, pl.Mp, pl.Np, vp.C, vp.ldc, vp.cps, vp.M, vp.N, vp.store, vp.skip, st);
}

template <int CN, bool REALB>
hipError_t launch_v_cr(const VPlan& pl, const VParams& vp, bool adj, bool avec, hipStream_t st) {
    if (adj) return launch_v<CN, true, false, false, REALB>(pl, vp, st);
    if (vp.fro)
        return avec ? launch_v<CN, false, true, true, REALB>(pl, vp, st) : launch_v<CN, false, false, true, REALB>(pl, vp, st);
    return avec ? launch_v<CN, false, true, false, REALB>(pl, vp, st) : launch_v<CN, false, false, false, REALB>(pl, vp, st);
}
template <int CN>
hipError_t launch_v_cn(const VPlan& pl, const VParams& vp, bool adj, bool avec, bool realb, hipStream_t st) {
    return realb ? launch_v_cr<CN, true>(pl, vp, adj, avec, st) : launch_v_cr<CN, false>(pl, vp, adj, avec, st);
}

hipError_t launch_view(const QgemmDesc& d, void* scratch, hipStream_t st) {
    const VPlan pl = make_vplan(d);
    if (!scratch) return hipErrorInvalidValue;
    float* Bt = (float*)scratch;
    float* part = (float*)((char*)scratch + vplan_thin_bytes(pl));
    hipLaunchKernelGGL(k_thin_t, dim3((unsigned)((pl.Kp + 15) / 16), (unsigned)((pl.Np + 63) / 64), d.b_real ? 1 : 4),
                       dim3(256), 0, st,
                       (const float*)d.B, d.ldb, d.bps, d.K, d.N, Bt, pl.Np, pl.Kp, d.skip_flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    VParams vp{};
    vp.A = (const float*)d.A; vp.lda = d.lda; vp.aps = d.aps;
    vp.Bt = Bt; vp.kp = pl.Kp; vp.bps = pl.Np * pl.Kp;
    vp.C = (float*)d.C; vp.ldc = d.ldc; vp.cps = d.cps;
    vp.M = d.M; vp.N = d.N; vp.K = d.K;
    vp.kchunk = pl.kchunk; vp.splits = (int)pl.splits; vp.kw = pl.kw;
    vp.tiles = pl.tiles; vp.gy = pl.gy;
    vp.part = part; vp.Mp = pl.Mp; vp.Np = pl.Np;
    vp.store = d.store; vp.skip = d.skip_flag;
    vp.fro = d.op == OP_NN ? d.fro2_part : nullptr;
    const bool adj = d.op == OP_HN;
    const bool avec = ((uintptr_t)d.A % 16) == 0 && d.lda % 4 == 0 && d.aps % 4 == 0;
    const bool realb = d.b_real != 0;
    switch (pl.CN) {
        case 1: return launch_v_cn<1>(pl, vp, adj, avec, realb, st);
        case 2: return launch_v_cn<2>(pl, vp, adj, avec, realb, st);
        case 3: return launch_v_cn<3>(pl, vp, adj, avec, realb, st);
        case 4: return launch_v_cn<4>(pl, vp, adj, avec, realb, st);
        case 5: return launch_v_cn<5>(pl, vp, adj, avec, realb, st);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------------------------------
// Low-precision views: BF16 / FP16 operands, v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulation.
//
// Both operands are in MFMA operand order before the product starts.  A fragment is 16 rows (or
// columns) by 32 reduction elements of one plane, 1 KB, lane l holding row (column) l % 16 and
// reduction elements 8 (l / 16) .. + 7:
//  - A: the low-precision copy laid out as the rows of the output (A itself for A B, the
//    transposed copy A^T for A^H B) in the tiled order of lowp_copy_launch.  Every A element is
//    used by exactly one wave, so its fragments go from HBM straight into registers.
//  - the thin operand: converted once per launch (k_lp_thin) into fragments ordered by K step,
//    plane, column tile and half step, so that the fragments of one K step, one plane and a
//    workgroup's column tiles are one contiguous run.
// A workgroup is four waves; each owns 16 rows of the output and all of the workgroup's CN column
// tiles in the four planes.  The thin fragments of a K step go from global memory into LDS by
// direct loads (global_load_lds_dwordx4: 1 KB per instruction, no registers), into one of two
// stage buffers: the copy of step s + 1 is in flight during the MFMAs of step s, and one barrier
// per step both publishes it and frees step s's buffer.  The A fragments of step s + 2 are loaded
// (into the ping-pong register sets aX, aY) once step s's MFMAs are issued.  The signs of eq. (1)
// go on a negated copy of the A fragments, made once per step.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <class TL>
struct LpMma;
template <>
struct LpMma<__bf16> {
    using v8 = bf16x8;
    static __device__ __forceinline__ f32x4 mma(v8 a, v8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct LpMma<_Float16> {
    using v8 = f16x8;
    static __device__ __forceinline__ f32x4 mma(v8 a, v8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// flip the sign bit of eight 16-bit values
template <class V>
__device__ __forceinline__ V neg8(V v) {
    u32x4 u = __builtin_bit_cast(u32x4, v);
    u ^= 0x80008000u;
    return __builtin_bit_cast(V, u);
}

constexpr int LBK = 64;        // K per step: two MFMA k-blocks of 32
constexpr int LBM = 64;        // output rows per workgroup (16 per wave)
constexpr int LKS = 2 * LBK;   // K per loop iteration (two steps); K chunks and padding are multiples

struct LpParams {
    const void* A; int64_t akt, art;      // tiled copy: reduction tiles per row tile, row tiles
    const void* Bt; int64_t bnt;          // thin operand in fragment order: column tiles of 16
    const void* A2;                       // split form: the residual copy of A (same tiling)
    const void* Bt2;                      // split form: the residual of the thin operand
    float* C; int64_t ldc, cps;
    int64_t M, N, K;
    int64_t kchunk;
    int splits;
    float* part;
    int64_t Mp, Np;
    const int* skip;
    const float* cscale;
};

// The thin operand in fragment order.  Fragment (s, p, n, h) (K step s, plane p, column tile n
// of NT, half step h) starts at element 512 (((s * 4 + p) * NT + n) * 2 + h); lane l's eight
// elements are B_p(64 s + 32 h + 8 (l / 16) + i, 16 n + l % 16), i = 0..7, zero outside K x N.
// RES: the rounded residual B - (float)(TL)B instead (the split form).  One thread per lane of
// a fragment; S K steps.
template <class TL, bool RES>
__global__ __launch_bounds__(256) void k_lp_thin(const float* __restrict__ B, int64_t ldb, int64_t bps, int64_t K,
                                                 int64_t N, TL* __restrict__ Bt, int64_t NT, int64_t S) {
    using v8 = typename LpMma<TL>::v8;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S * 4 * NT * 128) return;
    const int l = (int)(e & 63);
    const int64_t f = e >> 6;
    const int h = (int)(f & 1);
    const int64_t n = (f >> 1) % NT, sp = (f >> 1) / NT;
    const int p = (int)(sp & 3);
    const int64_t s = sp >> 2;
    const int64_t c = 16 * n + (l & 15), k0 = 64 * s + 32 * h + 8 * (l >> 4);
    v8 out;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int64_t k = k0 + i;
        const float x = (k < K && c < N) ? B[p * bps + k * ldb + c] : 0.0f;
        out[i] = RES ? (TL)(x - (float)(TL)x) : (TL)x;
    }
    *reinterpret_cast<v8*>(Bt + 8 * e) = out;
}

// 16 bytes per lane from global memory straight into LDS: lane l's bytes land at dst + 16 l
// (dst uniform over the wave); counted by vmcnt like any vector load
typedef __attribute__((address_space(1))) const void* global_cptr;
typedef __attribute__((address_space(3))) void* lds_ptr;
__device__ __forceinline__ void lds_copy16(const void* src, void* dst) {
    __builtin_amdgcn_global_load_lds((global_cptr)src, (lds_ptr)dst, 16, 0, 0);
}

// s_waitcnt bounding only the vector-memory count (vmcnt in bits 3:0 and 15:14; expcnt and
// lgkmcnt at their maxima)
constexpr int vmcnt_imm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14); }

// SPL (the split form fused): the residual copies of A and of the thin operand come along; the
// residual fragments are staged next to the value fragments, and every step issues the three
// products A_hi B_hi + A_hi B_lo + A_lo B_hi into the same accumulators.
template <class TL, bool ADJ, int CN, bool SPL>
__global__ __launch_bounds__(256, SPL ? 1 : 2) void k_qgemm_lp(LpParams P) {
    using L = LpMma<TL>;
    using v8 = typename L::v8;
    constexpr int NTILE = SPL ? 2 : 1;           // the value, and the residual
    constexpr int SLAB = 2 * CN;                 // fragments of one plane of one copy per K step
    constexpr int STAGE = NTILE * 4 * SLAB;      // fragments per K step
    constexpr int NA = NTILE * 8;                // A fragment loads per K step and wave
    static_assert(2 * STAGE * 1024 <= 163840, "two stages within LDS");
    __shared__ __attribute__((aligned(16))) v8 sB0[STAGE * 64];
    __shared__ __attribute__((aligned(16))) v8 sB1[STAGE * 64];
    if (P.skip && *P.skip == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int split = blockIdx.z;
    const int64_t kb = (int64_t)split * P.kchunk;
    const int64_t ke = kb + P.kchunk < P.K ? kb + P.kchunk : P.K;
    if (kb >= ke) return;   // uniform: an empty split (no partial tile is read for it)
    // steps [s0, s1): an even number, within the padded thin operand (kb is a multiple of LKS)
    const int64_t s0 = kb / LBK, s1 = s0 + 2 * ((ke - kb + LKS - 1) / LKS);
    const int64_t rt = (int64_t)blockIdx.x * (LBM / 16) + wave;   // this wave's row tile
    const int64_t rbase = 16 * rt;
    const int64_t n0 = (int64_t)blockIdx.y * CN;                   // the workgroup's first column tile
    // a row tile past the copy reads the last one: its rows are never stored
    const int64_t aoff = (rt < P.art ? rt : P.art - 1) * P.akt * 4096 + 8 * lane;
    const TL* __restrict__ Abase[2] = {(const TL*)P.A + aoff, SPL ? (const TL*)P.A2 + aoff : nullptr};
    const TL* __restrict__ Btile[2] = {(const TL*)P.Bt, SPL ? (const TL*)P.Bt2 : nullptr};
    const int64_t kt_last = P.akt - 1;

    // the A fragments of step s: a[t][q][h] for copy t (a step past the copy reads its last
    // reduction tile, which meets zero rows of the padded thin operand)
    auto load_a = [&](int64_t s, v8 (&a)[NTILE][4][2]) {
        const int64_t kt = s < kt_last ? s : kt_last;
#pragma unroll
        for (int t = 0; t < NTILE; t++) {
            const TL* src = Abase[t] + kt * 4096;
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int h = 0; h < 2; h++) a[t][q][h] = *reinterpret_cast<const v8*>(src + q * 1024 + h * 512);
        }
    };
    // this wave's share of step s's thin fragments into a stage: slab wave * NTILE + u (copy t,
    // plane p), fragment 2 j + h of a slab for column tile n0 + j, half h
    auto copy_b = [&](int64_t s, v8* stage) {
#pragma unroll
        for (int u = 0; u < NTILE; u++) {
            const int sig = wave * NTILE + u, t = sig >> 2, p = sig & 3;
            const TL* src = Btile[t] + (((s * 4 + p) * P.bnt + n0) * 128 + lane) * 8;
            v8* dst = stage + sig * SLAB * 64;
#pragma unroll
            for (int i = 0; i < SLAB; i++) lds_copy16(src + i * 512, dst + i * 64);
        }
    };

    f32x4 acc[4][CN];
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int j = 0; j < CN; j++) acc[p][j] = f32x4{0, 0, 0, 0};

    // the MFMAs of one step: for each half step and column tile, the four thin fragments of
    // each copy from LDS, then (value, value), (value, residual), (residual, value) products;
    // consecutive MFMAs update different accumulators
    auto step = [&](const v8 (&a)[NTILE][4][2], const v8* stage) {
        v8 na[NTILE][4][2];
#pragma unroll
        for (int t = 0; t < NTILE; t++)
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int h = 0; h < 2; h++) na[t][q][h] = neg8(a[t][q][h]);
        const v8* sb = stage + lane;
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int j = 0; j < CN; j++) {
                v8 b[NTILE][4];
#pragma unroll
                for (int t = 0; t < NTILE; t++)
#pragma unroll
                    for (int r = 0; r < 4; r++) b[t][r] = sb[((t * 4 + r) * SLAB + 2 * j + h) * 64];
#pragma unroll
                for (int x = 0; x < (SPL ? 3 : 1); x++) {
                    const int ta = x == 2 ? 1 : 0, tb = x == 1 ? 1 : 0;
#pragma unroll
                    for (int q = 0; q < 4; q++)
#pragma unroll
                        for (int p = 0; p < 4; p++)
                            acc[p][j] = L::mma(term_sign<ADJ>(p, q) > 0 ? a[ta][q][h] : na[ta][q][h], b[tb][p ^ q],
                                               acc[p][j]);
                }
            }
    };

    // prologue: A(s0), the thin copy of s0, A(s0 + 1); the wait leaves A(s0 + 1) in flight, the
    // same loads as at the end of every iteration (so the loop head sees one state)
    v8 aX[NTILE][4][2], aY[NTILE][4][2];
    load_a(s0, aX);
    __builtin_amdgcn_sched_barrier(0);
    copy_b(s0, sB0);
    __builtin_amdgcn_sched_barrier(0);
    load_a(s0 + 1, aY);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(NA));   // this wave's copy of step s0 has landed,
    __builtin_amdgcn_s_barrier();                // and every other wave's
    __builtin_amdgcn_sched_barrier(0);
    // Issue order per step: the next step's thin copy, this step's MFMAs, the A loads of the
    // step after next; then a wait that leaves only those A loads in flight, and the barrier.
    // The order is pinned (sched_barrier): the wait counts rely on it.
    for (int64_t s = s0; s < s1; s += 2) {
        copy_b(s + 1, sB1);
        __builtin_amdgcn_sched_barrier(0);
        step(aX, sB0);
        __builtin_amdgcn_sched_barrier(0);
        load_a(s + 2, aX);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(NA));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (s + 2 < s1) copy_b(s + 2, sB0);
        __builtin_amdgcn_sched_barrier(0);
        step(aY, sB1);
        __builtin_amdgcn_sched_barrier(0);
        load_a(s + 3, aY);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(NA));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    const float sc = P.cscale ? *P.cscale : 1.0f;
#pragma unroll
    for (int j = 0; j < CN; j++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t r = rbase + 4 * (lane >> 4) + i;
            const int64_t c = (n0 + j) * 16 + (lane & 15);
            if (P.splits == 1) {
                if (r < P.M && c < P.N)
#pragma unroll
                    for (int p = 0; p < 4; p++) P.C[p * P.cps + r * P.ldc + c] = acc[p][j][i] * sc;
            } else {
#pragma unroll
                for (int p = 0; p < 4; p++)
                    P.part[(((int64_t)split * 4 + p) * P.Mp + r) * P.Np + c] = acc[p][j][i] * sc;
            }
        }
    }
}

struct LpPlan {
    int CN;                 // column tiles of 16 per workgroup
    int64_t gx, gy, splits, kchunk, Mp, Np, Kp;
};

// up to 80 columns per workgroup (wider thin blocks: column tiles as even as possible): two
// stages of 80 columns take 80 KB of LDS, so two workgroups share a CU (two waves per SIMD)
constexpr int kLpMaxCols = 80;

// the split form stages the value and the residual fragments together: up to 80 columns
constexpr int kLpMaxColsSplit = 80;

LpPlan make_lp_plan(const QgemmDesc& d) {
    LpPlan p{};
    const bool split = d.math == MATH_BF16X3 || d.math == MATH_F16X3;
    const int64_t cap = split ? kLpMaxColsSplit : kLpMaxCols;
    const int64_t gy0 = std::max<int64_t>(1, (d.N + cap - 1) / cap);
    p.CN = (int)std::max<int64_t>(1, (d.N + 16 * gy0 - 1) / (16 * gy0));
    p.gy = (d.N + 16 * p.CN - 1) / (16 * p.CN);
    p.Np = p.gy * 16 * (int64_t)p.CN;
    p.gx = (d.M + LBM - 1) / LBM;
    p.Mp = p.gx * LBM;
    p.Kp = ((d.K + LKS - 1) / LKS) * LKS;
    // split K so that every CU gets a workgroup, each over at least 2 K steps; no more splits than
    // that, since the partial tiles (splits x the output) add traffic next to A
    const int64_t tiles = p.gx * p.gy;
    int64_t splits = 1;
    if (tiles < kCUs) splits = std::min<int64_t>((kCUs + tiles - 1) / tiles, (d.K + 2 * LBK - 1) / (2 * LBK));
    splits = std::max<int64_t>(splits, 1);
    int64_t kchunk = (d.K + splits - 1) / splits;
    kchunk = ((kchunk + LKS - 1) / LKS) * LKS;
    p.splits = (d.K + kchunk - 1) / kchunk;
    if (p.splits < 1) p.splits = 1;
    p.kchunk = kchunk;
    return p;
}

size_t lp_thin_bytes(const LpPlan& p) { return (size_t)4 * p.Np * p.Kp * 2; }
size_t lp_part_bytes(const LpPlan& p) { return p.splits > 1 ? (size_t)p.splits * 4 * p.Mp * p.Np * sizeof(float) : 0; }

// The thin operand(s) in fragment order, the product, then (when K is split) the ordered sum of
// the partial tiles.  Scratch: the converted thin operand (and its residual for the split form),
// then the partial tiles.  The split form is one launch with the residual copies (SPL).
size_t lp_scratch_bytes(const LpPlan& p, bool split) {
    return (split ? 2 : 1) * ((lp_thin_bytes(p) + 255) & ~size_t(255)) + lp_part_bytes(p);
}

// the product kernel for CN column tiles (false: no such variant)
template <class TL, bool ADJ, int CN, bool SPL>
bool lp_product_cn(int cn, dim3 grid, const LpParams& P, hipStream_t st) {
    if (cn != CN) return false;
    hipLaunchKernelGGL((k_qgemm_lp<TL, ADJ, CN, SPL>), grid, dim3(256), 0, st, P);
    return true;
}
template <class TL, bool ADJ, bool SPL>
bool lp_product(int cn, dim3 g, const LpParams& P, hipStream_t st) {
    static_assert(kLpMaxCols == 80 && kLpMaxColsSplit == 80, "variants up to 5 column tiles");
    return lp_product_cn<TL, ADJ, 1, SPL>(cn, g, P, st) || lp_product_cn<TL, ADJ, 2, SPL>(cn, g, P, st) ||
           lp_product_cn<TL, ADJ, 3, SPL>(cn, g, P, st) || lp_product_cn<TL, ADJ, 4, SPL>(cn, g, P, st) ||
           lp_product_cn<TL, ADJ, 5, SPL>(cn, g, P, st);
}

template <class TL, bool ADJ, bool SPL>
hipError_t launch_lp(const QgemmDesc& d, const LpPlan& pl, void* scratch, hipStream_t st) {
    char* base = (char*)scratch;
    const size_t tb = (lp_thin_bytes(pl) + 255) & ~size_t(255);
    TL* Bhi = (TL*)base;
    TL* Blo = SPL ? (TL*)(base + tb) : nullptr;
    float* part = (float*)(base + (SPL ? 2 : 1) * tb);
    const int64_t NT = pl.Np / 16, S = pl.Kp / LBK;
    const unsigned tg = (unsigned)((S * 4 * NT * 128 + 255) / 256);
    hipLaunchKernelGGL((k_lp_thin<TL, false>), dim3(tg), dim3(256), 0, st, (const float*)d.B, d.ldb, d.bps, d.K, d.N,
                       Bhi, NT, S);
    if (SPL)
        hipLaunchKernelGGL((k_lp_thin<TL, true>), dim3(tg), dim3(256), 0, st, (const float*)d.B, d.ldb, d.bps, d.K,
                           d.N, Blo, NT, S);
    LpParams P{};
    P.A = d.A; P.A2 = SPL ? d.A_lo : nullptr; P.akt = (d.K + LBK - 1) / LBK; P.art = (d.M + 15) / 16;
    P.Bt = Bhi; P.Bt2 = Blo; P.bnt = NT;
    P.C = (float*)d.C; P.ldc = d.ldc; P.cps = d.cps;
    P.M = d.M; P.N = d.N; P.K = d.K;
    P.kchunk = pl.kchunk; P.splits = (int)pl.splits;
    P.part = part; P.Mp = pl.Mp; P.Np = pl.Np;
    P.skip = d.skip_flag;
    P.cscale = d.cscale;
    dim3 grid((unsigned)pl.gx, (unsigned)pl.gy, (unsigned)pl.splits);
    if (!lp_product<TL, ADJ, SPL>(pl.CN, grid, P, st)) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || pl.splits == 1) return e;
    return reduce_f32(part, (int)pl.splits, pl.Mp, pl.Np, (float*)d.C, d.ldc, d.cps, d.M, d.N, (int)ST_SET,
                      d.skip_flag, st);
}

bool vec_ok(const void* p, int64_t ld, int64_t ps, size_t el) {
    return ((uintptr_t)p % 16) == 0 && ld % 4 == 0 && ps % 4 == 0 && (el == 4 || el == 8);
}

}  // namespace

size_t qgemm_partial_bytes(const QgemmDesc& d) {
    if (d.math == MATH_BF16X3 || d.math == MATH_F16X3) return lp_scratch_bytes(make_lp_plan(d), true);
    if (d.math == MATH_BF16 || d.math == MATH_F16) return lp_scratch_bytes(make_lp_plan(d), false);
    if (d.math == MATH_F32) {
        const VPlan vp = make_vplan(d);
        return vplan_thin_bytes(vp) + vplan_part_bytes(vp);
    }
    const Plan p = make_plan(d);
    if (p.splits <= 1) return 0;
    const size_t el = sizeof(double);
    return (size_t)p.splits * 4 * (size_t)p.Mp * (size_t)p.Np * el;
}

size_t qgemm_counter_count(const QgemmDesc&) { return 0; }

size_t fro2_slots(const QgemmDesc& d) { return d.math == MATH_F32 ? vplan_slots(make_vplan(d)) : 0; }

hipError_t qgemm_launch(const QgemmDesc& d, const QgemmScratch& s, hipStream_t st) {
    if (d.M <= 0 || d.N <= 0) return hipSuccess;
    if (d.math == MATH_BF16X3 || d.math == MATH_F16X3) {
        if (d.b_f64 || d.c_f64 || d.store != ST_SET || !s.partial || !d.A_lo) return hipErrorInvalidValue;
        const LpPlan lp = make_lp_plan(d);
        if (d.math == MATH_BF16X3)
            return d.op == OP_HN ? launch_lp<__bf16, true, true>(d, lp, s.partial, st)
                                 : launch_lp<__bf16, false, true>(d, lp, s.partial, st);
        return d.op == OP_HN ? launch_lp<_Float16, true, true>(d, lp, s.partial, st)
                             : launch_lp<_Float16, false, true>(d, lp, s.partial, st);
    }
    if (d.math == MATH_BF16 || d.math == MATH_F16) {
        if (d.b_f64 || d.c_f64 || d.store != ST_SET || !s.partial) return hipErrorInvalidValue;
        const LpPlan lp = make_lp_plan(d);
        if (d.math == MATH_BF16)
            return d.op == OP_HN ? launch_lp<__bf16, true, false>(d, lp, s.partial, st)
                                 : launch_lp<__bf16, false, false>(d, lp, s.partial, st);
        return d.op == OP_HN ? launch_lp<_Float16, true, false>(d, lp, s.partial, st)
                             : launch_lp<_Float16, false, false>(d, lp, s.partial, st);
    }
    if (d.math == MATH_F32) {
        if (d.a_f64 || d.b_f64 || d.c_f64) return hipErrorInvalidValue;
        return launch_view(d, s.partial, st);
    }
    const Plan pl = make_plan(d);
    KParams kp{};
    kp.A = d.A; kp.lda = d.lda; kp.aps = d.aps;
    kp.B = d.B; kp.ldb = d.ldb; kp.bps = d.bps;
    kp.C = d.C; kp.ldc = d.ldc; kp.cps = d.cps;
    kp.M = d.M; kp.N = d.N; kp.K = d.K;
    kp.kchunk = pl.kchunk; kp.splits = (int)pl.splits;
    kp.part = s.partial; kp.Mp = pl.Mp; kp.Np = pl.Np;
    kp.store = d.store;
    kp.skip = d.skip_flag;
    kp.avec = vec_ok(d.A, d.lda, d.aps, d.a_f64 ? 8 : 4);
    kp.bvec = vec_ok(d.B, d.ldb, d.bps, d.b_f64 ? 8 : 4);
    kp.sym = is_sym_gram(d) ? 1 : 0;
    kp.b_upper = d.b_upper;
    if (pl.splits > 1 && !s.partial) return hipErrorInvalidValue;
    // FP64 arithmetic
    if (d.op == OP_HN) {
        if (!d.a_f64 && !d.b_f64 && d.c_f64) return launch_hn(pl, kp, st);
        if (d.a_f64 && d.b_f64 && d.c_f64)
            return launch_t<double, 2, 2, 1, 1, 16, true, double, double, double>(pl, kp, st);
        return hipErrorInvalidValue;
    }
    const bool square = pl.WN == 2;
    if (nn_direct(d)) return launch_nn(pl, kp, st);
    if (!d.a_f64 && d.b_f64 && !d.c_f64)
        return square ? launch_t<double, 2, 2, 1, 1, 16, false, float, double, float>(pl, kp, st)
                      : launch_t<double, 1, 4, 1, 1, 16, false, float, double, float>(pl, kp, st);
    if (d.a_f64 && d.b_f64 && d.c_f64)
        return square ? launch_t<double, 2, 2, 1, 1, 16, false, double, double, double>(pl, kp, st)
                      : launch_t<double, 1, 4, 1, 1, 16, false, double, double, double>(pl, kp, st);
    return hipErrorInvalidValue;
}

}  // namespace qlra_impl
