// Low-precision copies of A for the reduced-precision views (the precision form of the
// method: the intermediate views run in BF16 / FP16 with FP32 accumulation, the last two views
// and all Gram, Cholesky and QSVD steps keep their precision).  For the split form the residual
// copies (s a - (s a rounded), rounded) are written in the same pass, in the same layout.
//
// Both orientations are written once per solve, Alo from A (rows m, reduction n) and Alo_t from
// A^T (rows n, reduction m), in the order the view kernel's MFMA A operand is consumed: tiles
// of 16 rows x 64 reduction elements, the four planes of a tile adjacent, and inside a tile
// [half h][quarter kq][row r][8 elements] so that lane l = 16 kq + r of a wave reads the 16
// bytes at h * 1024 + 16 l: every load instruction of the kernel reads 1 KB contiguous and a
// wave's K step reads 8 KB contiguous.  Padding rows and elements are zero.  The transpose goes
// through a 64 x 64 LDS tile so that reads of A and writes of both copies are coalesced.  FP16
// uses a power-of-two scale s derived from ||A||_F (exact, undone on the FP32 results); BF16
// has the FP32 exponent range and uses s = 1.
#include <cmath>

#include "common.h"

namespace qlra_impl {
namespace {

constexpr int kT = 64;

// element (row, k) of plane p in the tiled layout with KT reduction tiles per row tile
__device__ __forceinline__ int64_t tiled_index(int64_t row, int64_t k, int p, int64_t KT) {
    const int64_t rt = row >> 4, kt = k >> 6;
    const int r = (int)(row & 15), kk = (int)(k & 63);
    return ((rt * KT + kt) * 4 + p) * 1024 + (kk >> 5) * 512 + ((kk >> 3) & 3) * 128 + r * 8 + (kk & 7);
}

// one 64 x 64 tile of A (rows r0.., columns c0..), one plane at a time through a 16.6 KB LDS
// tile; the grid covers the padded extents (multiples of 64) so that padding is written as zeros.
// MODE 0: the copies Alo / Alo_t; 1: also the residual copies (x - (float)(TL)x, rounded) into
// Ar / Ar_t in the same pass; 2: the residual copies alone (into Ar / Ar_t).  fro (optional): the
// tile's sum of squares of A (FP64, the values before scaling) into fro[blockIdx.y * gridDim.x +
// blockIdx.x], so that the pass also yields ||A||_F^2.
template <class TL>
struct Vec8;
template <>
struct Vec8<__bf16> { typedef __bf16 type __attribute__((ext_vector_type(8))); };
template <>
struct Vec8<_Float16> { typedef _Float16 type __attribute__((ext_vector_type(8))); };

template <class TL, int MODE>
__global__ __launch_bounds__(256) void k_lowp_copy(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                   int64_t aps, TL* __restrict__ Alo, TL* __restrict__ Alo_t,
                                                   TL* __restrict__ Ar, TL* __restrict__ Ar_t,
                                                   const float* __restrict__ scale, double* __restrict__ fro) {
    using V8 = typename Vec8<TL>::type;
    __shared__ float tile[kT][kT + 1];
    __shared__ double red[4];
    const int64_t r0 = (int64_t)blockIdx.y * kT, c0 = (int64_t)blockIdx.x * kT;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;   // 64 x 4
    const float s = scale ? *scale : 1.0f;
    double sq = 0.0;
    const int64_t KTn = (n + 63) / 64, KTm = (m + 63) / 64;      // reduction tiles of Alo, Alo_t
    const int rtiles_m = (int)(((m + 15) >> 4) - (r0 >> 4)) < 4 ? (int)(((m + 15) >> 4) - (r0 >> 4)) : 4;
    const int rtiles_n = (int)(((n + 15) >> 4) - (c0 >> 4)) < 4 ? (int)(((n + 15) >> 4) - (c0 >> 4)) : 4;
    for (int p = 0; p < 4; p++) {
        if (p) __syncthreads();                                  // the previous plane is written out
        float v[kT / 4];
#pragma unroll
        for (int u = 0; u < kT / 4; u++) {
            const int64_t r = r0 + ty + 4 * u, c = c0 + tx;
            const float a = (r < m && c < n) ? A[p * aps + r * lda + c] : 0.0f;
            if (fro) sq += (double)a * (double)a;
            v[u] = a * s;
        }
#pragma unroll
        for (int u = 0; u < kT / 4; u++) tile[ty + 4 * u][tx] = v[u];
        __syncthreads();
        // Alo: row tiles r0/16 .. +3, reduction tile c0/64; each (row tile, plane) block of 1024
        // elements is contiguous, and a lane's 8 elements (t = 0..7) are 16 contiguous bytes:
        // one thread per 8 elements, one 16-byte store each
        for (int q8 = tid; q8 < rtiles_m * 128; q8 += 256) {
            const int rq = q8 >> 7, o8 = q8 & 127;
            const int h = o8 >> 6, kq = (o8 >> 4) & 3, r = o8 & 15;
            const int il = rq * 16 + r, kl = h * 32 + kq * 8;
            V8 hi, lo;
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const float x = tile[il][kl + t];
                hi[t] = (TL)x;
                lo[t] = (TL)(x - (float)hi[t]);
            }
            const int64_t at = tiled_index(r0 + il, c0 + kl, p, KTn);
            if constexpr (MODE != 2) *reinterpret_cast<V8*>(Alo + at) = hi;
            if constexpr (MODE != 0) *reinterpret_cast<V8*>(Ar + at) = lo;
        }
        // Alo_t: rows = columns of A (c0 ..), reduction = rows of A (r0 ..)
        for (int q8 = tid; q8 < rtiles_n * 128; q8 += 256) {
            const int rq = q8 >> 7, o8 = q8 & 127;
            const int h = o8 >> 6, kq = (o8 >> 4) & 3, r = o8 & 15;
            const int il = rq * 16 + r, kl = h * 32 + kq * 8;   // il: column of A, kl: row of A
            V8 hi, lo;
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const float x = tile[kl + t][il];
                hi[t] = (TL)x;
                lo[t] = (TL)(x - (float)hi[t]);
            }
            const int64_t at = tiled_index(c0 + il, r0 + kl, p, KTm);
            if constexpr (MODE != 2) *reinterpret_cast<V8*>(Alo_t + at) = hi;
            if constexpr (MODE != 0) *reinterpret_cast<V8*>(Ar_t + at) = lo;
        }
    }
    if (fro) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = sq;
        __syncthreads();
        if (tid == 0) fro[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    }
}

__global__ void k_lowp_scale(const double* __restrict__ nA2, int fp16, float* __restrict__ scale,
                             float* __restrict__ inv) {
    if (threadIdx.x != 0) return;
    int e = 0;
    if (fp16) {
        const double na = sqrt(*nA2);
        if (na > 0.0 && na < 1e300) {
            int ex;
            frexp(na, &ex);            // na < 2^ex
            e = 14 - ex;
            e = e < -120 ? -120 : (e > 120 ? 120 : e);
        }
    }
    *scale = ldexpf(1.0f, e);
    *inv = ldexpf(1.0f, -e);
}

}  // namespace

size_t lowp_copy_fro_slots(int64_t m, int64_t n) { return (size_t)((n + kT - 1) / kT) * ((m + kT - 1) / kT); }

hipError_t lowp_copy_launch(const float* A, int64_t m, int64_t n, int64_t lda, int64_t aps, int prec, void* Alo,
                            void* Alo_t, const float* scale, hipStream_t st, void* Ar, void* Ar_t, double* fro) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if ((Ar == nullptr) != (Ar_t == nullptr) || (Alo == nullptr) != (Alo_t == nullptr) || (!Alo && !Ar))
        return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + kT - 1) / kT), (unsigned)((m + kT - 1) / kT), 1);
    const int mode = !Ar ? 0 : (Alo ? 1 : 2);
#define QL_COPY(TL_, M_) \
    hipLaunchKernelGGL((k_lowp_copy<TL_, M_>), grid, dim3(256), 0, st, A, m, n, lda, aps, (TL_*)Alo, (TL_*)Alo_t, \
                       (TL_*)Ar, (TL_*)Ar_t, scale, fro)
    if (prec == QLRA_BF16 || prec == QLRA_BF16_SPLIT) {
        if (mode == 0) QL_COPY(__bf16, 0);
        else if (mode == 1) QL_COPY(__bf16, 1);
        else QL_COPY(__bf16, 2);
    } else if (prec == QLRA_FP16 || prec == QLRA_FP16_SPLIT) {
        if (mode == 0) QL_COPY(_Float16, 0);
        else if (mode == 1) QL_COPY(_Float16, 1);
        else QL_COPY(_Float16, 2);
    } else {
        return hipErrorInvalidValue;
    }
#undef QL_COPY
    return hipGetLastError();
}

size_t lowp_copy_elems(int64_t rows, int64_t k) { return (size_t)((rows + 15) / 16) * ((k + 63) / 64) * 4 * 1024; }

hipError_t lowp_scale_launch(const double* nA2, int prec, float* scale, float* inv, hipStream_t st) {
    hipLaunchKernelGGL(k_lowp_scale, dim3(1), dim3(64), 0, st, nA2, (prec == QLRA_FP16 || prec == QLRA_FP16_SPLIT) ? 1 : 0,
                       scale, inv);
    return hipGetLastError();
}

}  // namespace qlra_impl
