// Low-precision copies of A for the reduced-precision views (the precision form of the
// method: the intermediate views run in BF16 / FP16 with FP32 accumulation, the last two views
// and all Gram, Cholesky and QSVD steps keep their precision).
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

// one 64 x 64 tile of A (rows r0.., columns c0..), all four planes; the grid covers the
// padded extents (multiples of 64) so that padding is written as zeros
template <class TL>
__global__ __launch_bounds__(256) void k_lowp_copy(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                   int64_t aps, TL* __restrict__ Alo, TL* __restrict__ Alo_t,
                                                   const float* __restrict__ scale) {
    __shared__ float tile[4][kT][kT + 1];
    const int64_t r0 = (int64_t)blockIdx.y * kT, c0 = (int64_t)blockIdx.x * kT;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;   // 64 x 4
    const float s = scale ? *scale : 1.0f;
    const int64_t KTn = (n + 63) / 64, KTm = (m + 63) / 64;      // reduction tiles of Alo, Alo_t
    for (int p = 0; p < 4; p++)
        for (int i = ty; i < kT; i += 4) {
            const int64_t r = r0 + i, c = c0 + tx;
            tile[p][i][tx] = (r < m && c < n) ? A[p * aps + r * lda + c] * s : 0.0f;
        }
    __syncthreads();
    // Alo: row tiles r0/16 .. +3, reduction tile c0/64; each (row tile, plane) block of 1024
    // elements is contiguous: thread tid writes offsets tid, tid + 256, ...
    const int rtiles_m = (int)(((m + 15) >> 4) - (r0 >> 4)) < 4 ? (int)(((m + 15) >> 4) - (r0 >> 4)) : 4;
    for (int b = 0; b < 4 * rtiles_m; b++) {
        const int rq = b >> 2, p = b & 3;                          // row tile within the 64, plane
        for (int o = tid; o < 1024; o += 256) {
            const int h = o >> 9, kq = (o >> 7) & 3, r = (o >> 3) & 15, t = o & 7;
            const int il = rq * 16 + r, kl = h * 32 + kq * 8 + t;
            Alo[tiled_index(r0 + il, c0 + kl, p, KTn)] = (TL)tile[p][il][kl];
        }
    }
    // Alo_t: rows = columns of A (c0 ..), reduction = rows of A (r0 ..)
    const int rtiles_n = (int)(((n + 15) >> 4) - (c0 >> 4)) < 4 ? (int)(((n + 15) >> 4) - (c0 >> 4)) : 4;
    for (int b = 0; b < 4 * rtiles_n; b++) {
        const int rq = b >> 2, p = b & 3;
        for (int o = tid; o < 1024; o += 256) {
            const int h = o >> 9, kq = (o >> 7) & 3, r = (o >> 3) & 15, t = o & 7;
            const int il = rq * 16 + r, kl = h * 32 + kq * 8 + t;   // il: column of A, kl: row of A
            Alo_t[tiled_index(c0 + il, r0 + kl, p, KTm)] = (TL)tile[p][kl][il];
        }
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

hipError_t lowp_copy_launch(const float* A, int64_t m, int64_t n, int64_t lda, int64_t aps, int prec, void* Alo,
                            void* Alo_t, const float* scale, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + kT - 1) / kT), (unsigned)((m + kT - 1) / kT), 1);
    if (prec == QLRA_BF16)
        hipLaunchKernelGGL(k_lowp_copy<__bf16>, grid, dim3(256), 0, st, A, m, n, lda, aps, (__bf16*)Alo,
                           (__bf16*)Alo_t, scale);
    else if (prec == QLRA_FP16)
        hipLaunchKernelGGL(k_lowp_copy<_Float16>, grid, dim3(256), 0, st, A, m, n, lda, aps, (_Float16*)Alo,
                           (_Float16*)Alo_t, scale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t lowp_copy_elems(int64_t rows, int64_t k) { return (size_t)((rows + 15) / 16) * ((k + 63) / 64) * 4 * 1024; }

hipError_t lowp_scale_launch(const double* nA2, int prec, float* scale, float* inv, hipStream_t st) {
    hipLaunchKernelGGL(k_lowp_scale, dim3(1), dim3(64), 0, st, nA2, prec == QLRA_FP16 ? 1 : 0, scale, inv);
    return hipGetLastError();
}

}  // namespace qlra_impl
