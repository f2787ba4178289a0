// Small FP64 kernels of the quaternion CholeskyQR (eq. (QQR) computed as Y = Q R with
// R^H R = Y^H Y): the Hermitian quaternion Cholesky with a shifted retry, the triangular
// inverse, and products of triangular factors.  One workgroup per factorization: the
// matrices are l x l with l = k + p, tiny next to a pass over A; the latency chain, not the
// arithmetic, is what costs here.
#include "common.h"

namespace qlra_impl {
namespace {

struct Q4 {
    double w, x, y, z;
};
__device__ __forceinline__ Q4 qmul(Q4 a, Q4 b) {   // eq. (1)
    return Q4{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
              a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
              a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
              a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
__device__ __forceinline__ Q4 qconj(Q4 a) { return Q4{a.w, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ Q4 ld4(const double* P, int64_t ps, int64_t i) {
    return Q4{P[i], P[ps + i], P[2 * ps + i], P[3 * ps + i]};
}
__device__ __forceinline__ void st4(double* P, int64_t ps, int64_t i, Q4 v) {
    P[i] = v.w; P[ps + i] = v.x; P[2 * ps + i] = v.y; P[3 * ps + i] = v.z;
}

constexpr int kThreads = 1024;

// G (w x w Hermitian, full storage, FP64 planes) -> R upper triangular with real positive
// diagonal, G + shift I = R^H R; Rinv = R^{-1}.  Right-looking: row j of R is row j of the
// updated G divided by sqrt(pivot); the trailing block loses conj(R_ja) R_jb.
__global__ __launch_bounds__(kThreads) void k_chol(const double* __restrict__ G, int w,
                                                    double* __restrict__ R, double* __restrict__ Rinv,
                                                    double* __restrict__ W, int* status,
                                                    int* shift_out, const int* gate, int allow_shift,
                                                    double shift_scale) {
    __shared__ int s_fail;
    __shared__ double s_trace;
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x;
    const int64_t ps = (int64_t)w * w;
    double shift = 0.0;
    int shifted = 0, failed = 0;
    for (int attempt = 0; attempt < 2; attempt++) {
        for (int64_t e = tid; e < ps; e += kThreads) {
            const int a = (int)(e / w), b = (int)(e % w);
            Q4 v = (b >= a) ? ld4(G, ps, e) : Q4{0, 0, 0, 0};
            if (a == b) { v.w += shift; v.x = v.y = v.z = 0.0; }
            st4(W, ps, e, v);
        }
        if (tid == 0) s_fail = 0;
        __syncthreads();
        for (int j = 0; j < w; j++) {
            const double d = W[(int64_t)j * w + j];
            if (!(d > 0.0) || !(d < 1e300)) {   // breakdown or non-finite pivot
                if (tid == 0) s_fail = 1;
                __syncthreads();
                break;
            }
            const double rjj = sqrt(d), inv = 1.0 / rjj;
            __syncthreads();
            for (int c = j + 1 + tid; c < w; c += kThreads) {
                const int64_t e = (int64_t)j * w + c;
                Q4 v = ld4(W, ps, e);
                v.w *= inv; v.x *= inv; v.y *= inv; v.z *= inv;
                st4(W, ps, e, v);
            }
            if (tid == 0) st4(W, ps, (int64_t)j * w + j, Q4{rjj, 0, 0, 0});
            __syncthreads();
            const int t = w - j - 1;
            for (int64_t e = tid; e < (int64_t)t * t; e += kThreads) {
                const int a = j + 1 + (int)(e / t), b = j + 1 + (int)(e % t);
                if (b < a) continue;
                const Q4 ra = qconj(ld4(W, ps, (int64_t)j * w + a));
                const Q4 rb = ld4(W, ps, (int64_t)j * w + b);
                const Q4 pr = qmul(ra, rb);
                Q4 v = ld4(W, ps, (int64_t)a * w + b);
                v.w -= pr.w; v.x -= pr.x; v.y -= pr.y; v.z -= pr.z;
                if (a == b) v.x = v.y = v.z = 0.0;
                st4(W, ps, (int64_t)a * w + b, v);
            }
            __syncthreads();
        }
        __syncthreads();
        if (!s_fail) break;
        if (!allow_shift || attempt == 1) { failed = 1; break; }
        // Shifted CholeskyQR (Fukaya et al.): add s = shift_scale * trace(G) to the diagonal.
        if (tid == 0) {
            double tr = 0.0;
            for (int i = 0; i < w; i++) tr += G[(int64_t)i * w + i];
            s_trace = tr;
        }
        __syncthreads();
        shift = shift_scale * s_trace;
        if (!(shift > 0.0)) shift = 1e-300;
        shifted = 1;
        __syncthreads();
    }
    if (tid == 0) {
        if (shift_out) *shift_out = shifted;
        if (failed) atomicOr(status, 2);
    }
    // R = upper(W)
    for (int64_t e = tid; e < ps; e += kThreads) {
        const int a = (int)(e / w), b = (int)(e % w);
        st4(R, ps, e, b >= a ? ld4(W, ps, e) : Q4{0, 0, 0, 0});
    }
    __syncthreads();
    if (!Rinv) return;
    // Rinv: rows from the bottom; Rinv_ii = 1 / r_ii, Rinv_ic = -(1/r_ii) sum_{t=i+1}^{c} R_it Rinv_tc.
    for (int64_t e = tid; e < ps; e += kThreads) st4(Rinv, ps, e, Q4{0, 0, 0, 0});
    __syncthreads();
    for (int i = w - 1; i >= 0; i--) {
        const double rii = R[(int64_t)i * w + i];
        const double inv = rii > 0.0 ? 1.0 / rii : 0.0;
        for (int c = i + tid; c < w; c += kThreads) {
            if (c == i) {
                Rinv[(int64_t)i * w + i] = inv;
                continue;
            }
            Q4 s{0, 0, 0, 0};
            for (int t = i + 1; t <= c; t++) {
                const Q4 pr = qmul(ld4(R, ps, (int64_t)i * w + t), ld4(Rinv, ps, (int64_t)t * w + c));
                s.w += pr.w; s.x += pr.x; s.y += pr.y; s.z += pr.z;
            }
            st4(Rinv, ps, (int64_t)i * w + c, Q4{-inv * s.w, -inv * s.x, -inv * s.y, -inv * s.z});
        }
        __syncthreads();
    }
}

// Rout = R2 * R1 for upper triangular factors (only the upper triangle is formed).
__global__ __launch_bounds__(256) void k_rmul(const double* __restrict__ R2, const double* __restrict__ R1,
                                              double* __restrict__ Rout, int w, const int* gate) {
    if (gate && *gate == 0) return;
    const int64_t ps = (int64_t)w * w;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ps) return;
    const int a = (int)(e / w), b = (int)(e % w);
    Q4 s{0, 0, 0, 0};
    for (int t = a; t <= b; t++) {
        const Q4 pr = qmul(ld4(R2, ps, (int64_t)a * w + t), ld4(R1, ps, (int64_t)t * w + b));
        s.w += pr.w; s.x += pr.x; s.y += pr.y; s.z += pr.z;
    }
    if (a == b) s.x = s.y = s.z = 0.0;   // the product of real diagonals is real
    st4(Rout, ps, e, s);
}

__global__ __launch_bounds__(256) void k_rcopy(const double* __restrict__ src, double* __restrict__ dst,
                                               int64_t count, const int* gate) {
    if (gate && *gate == 0) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) dst[e] = src[e];
}

}  // namespace

hipError_t chol_launch(const double* G, int64_t w, double* R, double* Rinv, double* work, int* status,
                       int* shift_out, const int* gate, int allow_shift, double shift_scale, hipStream_t st) {
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kThreads), 0, st, G, (int)w, R, Rinv, work, status, shift_out,
                       gate, allow_shift, shift_scale);
    return hipGetLastError();
}

hipError_t rmul_launch(const double* R2, const double* R1, double* Rout, int64_t w, const int* gate,
                       hipStream_t st) {
    const int64_t n = w * w;
    hipLaunchKernelGGL(k_rmul, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, R2, R1, Rout, (int)w, gate);
    return hipGetLastError();
}

hipError_t rcopy_launch(const double* src, double* dst, int64_t w, const int* gate, hipStream_t st) {
    const int64_t n = 4 * w * w;
    hipLaunchKernelGGL(k_rcopy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n, gate);
    return hipGetLastError();
}

}  // namespace qlra_impl
