// Tall-skinny quaternion products on MFMA (Sec. 2: eq. (1) and the conjugate transpose).
//
// A view multiplies the big matrix A (four FP32 planes) by a thin quaternion block B:
//   C = A B      C_p = sum_q s(p, q) A_q B_{p^q}
//   C = A^H B    C_p = sum_q s(p, q) e_q A_q^T B_{p^q},   e = (+1, -1, -1, -1)
// where e_q e_{p^q} = s(p, q) e_p is the Hamilton product of the units (eq. (1)).  All 16
// plane products are real GEMMs that share operands: each A_q fragment feeds four output
// planes and each B_r fragment feeds four, so one pass over A computes the whole quaternion
// product with A read once.  Signs are applied to the thin operand (a negated register copy),
// never to A.
//
// Tiling (gfx950, wave64): a workgroup of 4 waves owns a BM x BN tile of all four output
// planes; wave (wm, wn) owns RM x CN MFMA sub-tiles of 16 x 16 in every plane.  Per K step
// the four planes of an A tile and of a B tile are staged through LDS with coalesced loads;
// the MFMA A operand always comes from the A tile, so the same kernel serves A B (A tile stored
// row-major) and A^H B (A tile stored k-major, i.e. transposed through LDS).  When there are
// too few output tiles to fill 256 CUs, K is split across workgroups; partial tiles go to
// scratch and the last workgroup of a tile (counter in scratch, reset after use) adds them in
// split order, so results are deterministic.
//
// math = MATH_F32: FP32 operands, v_mfma_f32_16x16x4f32, FP32 accumulation.
// math = MATH_F64: operands converted to FP64 in LDS (exact for FP32 data),
//                  v_mfma_f64_16x16x4f64; used for Gram matrices and small triangular products.
#include "common.h"

#include <algorithm>

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
    unsigned* counters;
    int store;
    const int* skip;
};

template <class T, int WM, int WN, int RM, int CN, int BK, bool ADJ, class TA, class TB, class TC>
__global__ __launch_bounds__(256) void k_qgemm(KParams P) {
    static_assert(WM * WN == 4, "four waves");
    constexpr int BM = WM * RM * 16, BN = WN * CN * 16;
    constexpr int AROWS = ADJ ? BK : BM;      // A tile rows in LDS
    constexpr int AST = ADJ ? BM + 4 : BK + 4; // A tile row stride (elements)
    constexpr int BST = BN + 4;
    __shared__ T sA[4 * AROWS * AST];
    __shared__ T sB[4 * BK * BST];
    __shared__ int s_last;

    if (P.skip && *P.skip == 0) return;
    using M_ = Mma<T>;
    using acc_t = typename M_::acc_t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t row0 = (int64_t)blockIdx.x * BM, col0 = (int64_t)blockIdx.y * BN;
    const int split = blockIdx.z;
    const int64_t kb = (int64_t)split * P.kchunk;
    const int64_t ke = P.K < kb + P.kchunk ? P.K : kb + P.kchunk;
    const TA* __restrict__ A = (const TA*)P.A;
    const TB* __restrict__ B = (const TB*)P.B;

    acc_t acc[RM][CN][4];
#pragma unroll
    for (int rm = 0; rm < RM; rm++)
#pragma unroll
        for (int cn = 0; cn < CN; cn++)
#pragma unroll
            for (int p = 0; p < 4; p++) acc[rm][cn][p] = acc_t{0, 0, 0, 0};

    const int g = lane >> 4, r16 = lane & 15;
    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();
        // ---- stage the four planes of the A tile
        if (!ADJ) {
            // A (M x K, k contiguous): LDS [q][r][kk]
            for (int e = tid; e < 4 * BM * BK; e += 256) {
                const int q = e / (BM * BK), rem = e % (BM * BK), r = rem / BK, kk = rem % BK;
                const int64_t gr = row0 + r, gk = k0 + kk;
                T v = 0;
                if (gr < P.M && gk < ke) v = (T)A[q * P.aps + gr * P.lda + gk];
                sA[(q * AROWS + r) * AST + kk] = v;
            }
        } else {
            // A stored K x M (row of C = column of A, contiguous): LDS [q][kk][r]
            for (int e = tid; e < 4 * BM * BK; e += 256) {
                const int q = e / (BM * BK), rem = e % (BM * BK), kk = rem / BM, r = rem % BM;
                const int64_t gr = row0 + r, gk = k0 + kk;
                T v = 0;
                if (gr < P.M && gk < ke) v = (T)A[q * P.aps + gk * P.lda + gr];
                sA[(q * AROWS + kk) * AST + r] = v;
            }
        }
        // ---- stage the four planes of the B tile (K x N, n contiguous): LDS [q][kk][c]
        for (int e = tid; e < 4 * BK * BN; e += 256) {
            const int q = e / (BK * BN), rem = e % (BK * BN), kk = rem / BN, c = rem % BN;
            const int64_t gk = k0 + kk, gc = col0 + c;
            T v = 0;
            if (gk < ke && gc < P.N) v = (T)B[q * P.bps + gk * P.ldb + gc];
            sB[(q * BK + kk) * BST + c] = v;
        }
        __syncthreads();
        // ---- 16 plane products per (row sub-tile, column sub-tile), 4 k per MFMA
#pragma unroll 2
        for (int ks = 0; ks < BK; ks += 4) {
            T a[4][RM];
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int rm = 0; rm < RM; rm++) {
                    const int r = (wm * RM + rm) * 16 + r16, kk = ks + g;
                    a[q][rm] = ADJ ? sA[(q * AROWS + kk) * AST + r] : sA[(q * AROWS + r) * AST + kk];
                }
#pragma unroll
            for (int cn = 0; cn < CN; cn++) {
                const int c = (wn * CN + cn) * 16 + r16;
                T b[4], nb[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    b[q] = sB[(q * BK + ks + g) * BST + c];
                    nb[q] = -b[q];
                }
#pragma unroll
                for (int rm = 0; rm < RM; rm++)
#pragma unroll
                    for (int p = 0; p < 4; p++)
#pragma unroll
                        for (int q = 0; q < 4; q++)
                            acc[rm][cn][p] = M_::mma(a[q][rm], term_sign<ADJ>(p, q) > 0 ? b[p ^ q] : nb[p ^ q],
                                                     acc[rm][cn][p]);
            }
        }
    }

    TC* __restrict__ C = (TC*)P.C;
    if (P.splits == 1) {
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
                        }
                    }
                }
        return;
    }

    // ---- split K: publish the partial tile, the last workgroup of the tile reduces
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
    __threadfence();
    __syncthreads();
    const int tile = blockIdx.y * gridDim.x + blockIdx.x;
    if (tid == 0) {
        const unsigned prev = atomicAdd(&P.counters[tile], 1u);
        s_last = (prev == (unsigned)(P.splits - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int e = tid; e < 4 * BM * BN; e += 256) {
        const int p = e / (BM * BN), rem = e % (BM * BN), rr = rem / BN, cc = rem % BN;
        const int64_t r = row0 + rr, c = col0 + cc;
        if (r >= P.M || c >= P.N) continue;
        T s = 0;
        for (int sp = 0; sp < P.splits; sp++) s += part[(((int64_t)sp * 4 + p) * P.Mp + r) * P.Np + c];
        TC* dst = C + p * P.cps + r * P.ldc + c;
        *dst = P.store == ST_SUB ? (TC)((T)*dst - s) : (TC)s;
    }
    if (tid == 0) P.counters[tile] = 0u;
}

// ------------------------------------------------------------------------------------------
// configuration choice

struct Plan {
    int WM, WN, RM, CN, BK;
    int64_t gx, gy, splits, kchunk, Mp, Np;
};

constexpr int kCUs = 256;

Plan make_plan(const QgemmDesc& d) {
    Plan p{};
    if (d.math == MATH_F32) {
        p.WM = 4; p.WN = 1; p.BK = 32;
        const int64_t cn_needed = (std::min<int64_t>(d.N, 80) + 15) / 16;
        p.CN = (int)std::max<int64_t>(1, cn_needed);
        const int64_t gy = (d.N + 16 * p.CN - 1) / (16 * p.CN);
        p.RM = ((d.M + 127) / 128) * gy >= kCUs ? 2 : 1;
    } else {
        p.BK = 16;
        if (d.op == OP_HN) { p.WM = 2; p.WN = 2; p.RM = 1; p.CN = 2; }   // Gram-like: small M, N
        else { p.WM = 1; p.WN = 4; p.RM = 1; p.CN = 1; }                 // tall times small
    }
    const int64_t BM = p.WM * p.RM * 16, BN = p.WN * p.CN * 16;
    p.gx = (d.M + BM - 1) / BM;
    p.gy = (d.N + BN - 1) / BN;
    p.Mp = p.gx * BM;
    p.Np = p.gy * BN;
    const int64_t tiles = p.gx * p.gy;
    int64_t splits = 1;
    if (tiles < kCUs && d.K > 4 * p.BK) {
        splits = std::min<int64_t>((2 * kCUs + tiles - 1) / tiles, (d.K + 4 * p.BK - 1) / (4 * p.BK));
        splits = std::max<int64_t>(splits, 1);
    }
    int64_t kchunk = (d.K + splits - 1) / splits;
    kchunk = ((kchunk + p.BK - 1) / p.BK) * p.BK;
    if (kchunk < p.BK) kchunk = p.BK;
    splits = (d.K + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    p.splits = splits;
    p.kchunk = kchunk;
    return p;
}

template <class T, int WM, int WN, int RM, int CN, int BK, bool ADJ, class TA, class TB, class TC>
hipError_t launch_t(const Plan& pl, const KParams& kp, hipStream_t st) {
    dim3 grid((unsigned)pl.gx, (unsigned)pl.gy, (unsigned)pl.splits);
    hipLaunchKernelGGL((k_qgemm<T, WM, WN, RM, CN, BK, ADJ, TA, TB, TC>), grid, dim3(256), 0, st, kp);
    return hipGetLastError();
}

template <bool ADJ>
hipError_t launch_f32(const Plan& pl, const KParams& kp, hipStream_t st) {
#define QL_F32(RM_, CN_) \
    if (pl.RM == RM_ && pl.CN == CN_) return launch_t<float, 4, 1, RM_, CN_, 32, ADJ, float, float, float>(pl, kp, st);
    QL_F32(1, 1) QL_F32(1, 2) QL_F32(1, 3) QL_F32(1, 4) QL_F32(1, 5)
    QL_F32(2, 1) QL_F32(2, 2) QL_F32(2, 3) QL_F32(2, 4) QL_F32(2, 5)
#undef QL_F32
    return hipErrorInvalidValue;
}

}  // namespace

size_t qgemm_partial_bytes(const QgemmDesc& d) {
    const Plan p = make_plan(d);
    if (p.splits <= 1) return 0;
    const size_t el = d.math == MATH_F32 ? sizeof(float) : sizeof(double);
    return (size_t)p.splits * 4 * (size_t)p.Mp * (size_t)p.Np * el;
}

size_t qgemm_counter_count(const QgemmDesc& d) {
    const Plan p = make_plan(d);
    return p.splits <= 1 ? 0 : (size_t)(p.gx * p.gy);
}

hipError_t qgemm_launch(const QgemmDesc& d, const QgemmScratch& s, hipStream_t st) {
    if (d.M <= 0 || d.N <= 0) return hipSuccess;
    const Plan pl = make_plan(d);
    KParams kp{};
    kp.A = d.A; kp.lda = d.lda; kp.aps = d.aps;
    kp.B = d.B; kp.ldb = d.ldb; kp.bps = d.bps;
    kp.C = d.C; kp.ldc = d.ldc; kp.cps = d.cps;
    kp.M = d.M; kp.N = d.N; kp.K = d.K;
    kp.kchunk = pl.kchunk; kp.splits = (int)pl.splits;
    kp.part = s.partial; kp.Mp = pl.Mp; kp.Np = pl.Np;
    kp.counters = s.counters;
    kp.store = d.store;
    kp.skip = d.skip_flag;
    if (pl.splits > 1 && (!s.partial || !s.counters)) return hipErrorInvalidValue;
    if (d.math == MATH_F32) {
        if (d.a_f64 || d.b_f64 || d.c_f64) return hipErrorInvalidValue;
        return d.op == OP_HN ? launch_f32<true>(pl, kp, st) : launch_f32<false>(pl, kp, st);
    }
    // FP64 arithmetic
    if (d.op == OP_HN) {
        if (!d.a_f64 && !d.b_f64 && d.c_f64)
            return launch_t<double, 2, 2, 1, 2, 16, true, float, float, double>(pl, kp, st);
        if (d.a_f64 && d.b_f64 && d.c_f64)
            return launch_t<double, 2, 2, 1, 2, 16, true, double, double, double>(pl, kp, st);
        return hipErrorInvalidValue;
    }
    if (!d.a_f64 && d.b_f64 && !d.c_f64)
        return launch_t<double, 1, 4, 1, 1, 16, false, float, double, float>(pl, kp, st);
    if (d.a_f64 && d.b_f64 && d.c_f64)
        return launch_t<double, 1, 4, 1, 1, 16, false, double, double, double>(pl, kp, st);
    return hipErrorInvalidValue;
}

}  // namespace qlra_impl
