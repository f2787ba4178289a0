// Element-wise helpers: gated plane copies and fills used instead of memsets (they stay valid
// inside captured HIP graphs).
#include <algorithm>

#include "common.h"

namespace qlra_impl {
namespace {

__global__ __launch_bounds__(256) void k_copy_planes(const float* __restrict__ src, int64_t lds, int64_t sps,
                                                     float* __restrict__ dst, int64_t ldd, int64_t dps,
                                                     int64_t rows, int64_t cols, const int* gate) {
    if (gate && *gate == 0) return;
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / cols, c = e - r * cols;
#pragma unroll
        for (int p = 0; p < 4; p++) dst[p * dps + r * ldd + c] = src[p * sps + r * lds + c];
    }
}

__global__ __launch_bounds__(256) void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst,
                                                  int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) dst[e] = src[e];
}

__global__ __launch_bounds__(256) void k_fill_int(int* p, int64_t count, int value) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = value;
}

// The set-up of a solve in one launch: status words and counters cleared, *nan_at (if given)
// set to NaN.
__global__ __launch_bounds__(256) void k_solve_prologue(int* status, int nstatus, unsigned* counters, int64_t ncnt,
                                                        double* nan_at) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nstatus) status[e] = 0;
    if (e < ncnt) counters[e] = 0u;
    if (e == 0 && nan_at) *nan_at = __builtin_nan("");
}

}  // namespace

hipError_t copy_planes_launch(const float* src, int64_t lds, int64_t sps, float* dst, int64_t ldd, int64_t dps,
                              int64_t rows, int64_t cols, const int* gate, hipStream_t st) {
    const int64_t total = rows * cols;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy_planes, dim3((unsigned)blocks), dim3(256), 0, st, src, lds, sps, dst, ldd, dps,
                       rows, cols, gate);
    return hipGetLastError();
}

hipError_t copy_f64_launch(const double* src, double* dst, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

hipError_t fill_int_launch(int* p, int64_t count, int value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

hipError_t solve_prologue_launch(int* status, int nstatus, unsigned* counters, int64_t ncnt, double* nan_at,
                                 hipStream_t st) {
    const int64_t n = std::max<int64_t>(std::max<int64_t>(nstatus, ncnt), 1);
    hipLaunchKernelGGL(k_solve_prologue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, status, nstatus, counters,
                       ncnt, nan_at);
    return hipGetLastError();
}

}  // namespace qlra_impl
