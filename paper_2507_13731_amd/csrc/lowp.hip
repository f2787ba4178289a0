// Low-precision copies of A for the reduced-precision views (the precision form of the
// method: the intermediate views run in BF16 / FP16 with FP32 accumulation, the last two views
// and all Gram, Cholesky and QSVD steps keep their precision).
//
// Both orientations are written once per solve: Alo = s A (m x n) and Alo_t = s A^T (n x m),
// each plane row-major, so that the view kernel's A operand is always a row of its own output
// (eight consecutive reduction elements per lane, one 16-byte load).  The transpose goes through
// a 64 x 64 LDS tile so that reads of A and writes of both copies are coalesced.  FP16 uses a
// power-of-two scale s derived from ||A||_F (exact, undone on the FP32 results); BF16 has the
// FP32 exponent range and uses s = 1.
#include <cmath>

#include "common.h"

namespace qlra_impl {
namespace {

constexpr int kT = 64;

template <class TL>
__global__ __launch_bounds__(256) void k_lowp_copy(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                   int64_t aps, TL* __restrict__ Alo, TL* __restrict__ Alo_t,
                                                   const float* __restrict__ scale) {
    __shared__ float tile[kT][kT + 1];
    const int p = blockIdx.z;
    const int64_t r0 = (int64_t)blockIdx.y * kT, c0 = (int64_t)blockIdx.x * kT;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4
    const float s = scale ? *scale : 1.0f;
    const float* Ap = A + p * aps;
    TL* Lp = Alo + p * m * n;
    TL* Tp = Alo_t + p * m * n;
    for (int i = ty; i < kT; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        float v = 0.0f;
        if (r < m && c < n) {
            v = Ap[r * lda + c] * s;
            Lp[r * n + c] = (TL)v;
        }
        tile[i][tx] = v;
    }
    __syncthreads();
    for (int i = ty; i < kT; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;   // Alo_t row c, column r
        if (c < n && r < m) Tp[c * m + r] = (TL)tile[tx][i];
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
    dim3 grid((unsigned)((n + kT - 1) / kT), (unsigned)((m + kT - 1) / kT), 4);
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

hipError_t lowp_scale_launch(const double* nA2, int prec, float* scale, float* inv, hipStream_t st) {
    hipLaunchKernelGGL(k_lowp_scale, dim3(1), dim3(64), 0, st, nA2, prec == QLRA_FP16 ? 1 : 0, scale, inv);
    return hipGetLastError();
}

}  // namespace qlra_impl
