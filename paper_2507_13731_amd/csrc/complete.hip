// Quaternion matrix completion (Sec. 7): the device side of one iteration after the low-rank
// step.  Given the rank-R factors U, S, V of C^(t), one fused kernel per iteration
//   - rebuilds X = U diag(S) V^H on an output tile plus a halo of `radius` rows and columns
//     (edge indices replicated), from U and S V staged in LDS, FP32 FMA accumulation,
//   - smooths it with the separable Gaussian (along rows, then columns) in LDS,
//   - writes C^(t+1) = mask . M + (1 - mask) . X and, on the last iteration, X itself,
//   - and leaves per-workgroup sums of mask . |X - M|^2 and mask . |M|^2 (FP64),
// and a one-workgroup kernel turns the sums into the relative misfit of the iteration and
// advances the device-side iteration counter, so that the same launches (or a captured graph of
// them) serve every iteration.
//
// The reconstruction is a rank-R outer-product sum (16 R flops per quaternion entry) over a
// region of 48 x 48 entries per workgroup: vector-ALU work at R = 30 and far below the HBM
// stream of M, mask and C only for small R; each thread holds a 3 x 3 micro-tile (stride 16)
// so that every LDS operand read feeds 3 quaternion products.
#include <cmath>

#include "common.h"

namespace qlra_impl {
namespace {

constexpr int kZ = 48;        // region side: output tile + 2 * radius
constexpr int kRC = 16;       // rank chunk staged per round
constexpr int kZP = kZ + 1;   // padded LDS row of the region

struct StepArgs {
    const float* U; int64_t ldu, ups;
    const double* S;
    const float* V; int64_t ldv, vps;
    int R;
    const float* M; int64_t ldm, mps;
    const unsigned char* mask; int64_t ldk;
    float* C; int64_t ldc, cps;
    float* X; int64_t ldx, xps;
    int64_t m, n;
    float w[2 * kCompleteMaxRadius + 1];
    const int* iter; int iters;
    double* part;
};

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// H: smoothing radius (0: none); output tile T = kZ - 2H, region kZ x kZ around it
template <int H>
__global__ __launch_bounds__(256) void k_complete_step(StepArgs a) {
    constexpr int T = kZ - 2 * H, TAPS = 2 * H + 1;
    static_assert(T >= 16 && (kRC * kZ) % 256 == 0, "tile");
    __shared__ f32x4 su[kRC][kZ];
    __shared__ f32x4 sv[kRC][kZ];
    __shared__ float z[H > 0 ? 4 : 1][H > 0 ? kZ : 1][H > 0 ? kZP : 1];
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t oi = (int64_t)blockIdx.y * T, oj = (int64_t)blockIdx.x * T;   // output tile origin
    const int64_t ri = oi - H, rj = oj - H;                                     // region origin

    float acc[3][3][4];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int p = 0; p < 4; p++) acc[i][j][p] = 0.f;

    for (int r0 = 0; r0 < a.R; r0 += kRC) {
        __syncthreads();
        // stage rows of U and of S V (16 consecutive ranks of a row per 16 threads), zero past R;
        // all loads of the round issued before the first store
        f32x4 u[kRC * kZ / 256], v[kRC * kZ / 256];
#pragma unroll
        for (int s = 0; s < kRC * kZ / 256; s++) {
            const int e = tid + 256 * s;
            const int r = e % kRC, t = e / kRC;
            const int rr = r0 + r;
            u[s] = f32x4{0.f, 0.f, 0.f, 0.f};
            v[s] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (rr < a.R) {
                const float* up = a.U + clampi(ri + t, a.m - 1) * a.ldu + rr;
                const float* vp = a.V + clampi(rj + t, a.n - 1) * a.ldv + rr;
                const float sc = (float)a.S[rr];
                u[s] = f32x4{up[0], up[a.ups], up[2 * a.ups], up[3 * a.ups]};
                v[s] = f32x4{sc * vp[0], sc * vp[a.vps], sc * vp[2 * a.vps], sc * vp[3 * a.vps]};
            }
        }
#pragma unroll
        for (int s = 0; s < kRC * kZ / 256; s++) {
            const int e = tid + 256 * s;
            su[e % kRC][e / kRC] = u[s];
            sv[e % kRC][e / kRC] = v[s];
        }
        __syncthreads();
#pragma unroll 1
        for (int r = 0; r < kRC; r++) {
            f32x4 uu[3], vv[3];
#pragma unroll
            for (int i = 0; i < 3; i++) uu[i] = su[r][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 3; j++) vv[j] = sv[r][tx + 16 * j];
            // x += p * conj(q): the Hamilton product with q's imaginary parts negated
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    const f32x4 p = uu[i], q = vv[j];
                    float* x = acc[i][j];
                    x[0] = fmaf(p[0], q[0], x[0]); x[0] = fmaf(p[1], q[1], x[0]);
                    x[0] = fmaf(p[2], q[2], x[0]); x[0] = fmaf(p[3], q[3], x[0]);
                    x[1] = fmaf(p[1], q[0], x[1]); x[1] = fmaf(-p[0], q[1], x[1]);
                    x[1] = fmaf(-p[2], q[3], x[1]); x[1] = fmaf(p[3], q[2], x[1]);
                    x[2] = fmaf(p[2], q[0], x[2]); x[2] = fmaf(-p[0], q[2], x[2]);
                    x[2] = fmaf(p[1], q[3], x[2]); x[2] = fmaf(-p[3], q[1], x[2]);
                    x[3] = fmaf(p[3], q[0], x[3]); x[3] = fmaf(-p[0], q[3], x[3]);
                    x[3] = fmaf(-p[1], q[2], x[3]); x[3] = fmaf(p[2], q[1], x[3]);
                }
        }
    }

    // observed values and mask bits of this thread's outputs, loaded before the smoothing
    float mv[3][3][4];
    bool obs[3][3], out[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const int rw = ty + 16 * i, cl = tx + 16 * j;
            const int64_t gi = oi + rw, gj = oj + cl;
            out[i][j] = rw < T && cl < T && gi < a.m && gj < a.n;
            obs[i][j] = out[i][j] && a.mask[gi * a.ldk + gj] != 0;
#pragma unroll
            for (int p = 0; p < 4; p++) mv[i][j][p] = obs[i][j] ? a.M[p * a.mps + gi * a.ldm + gj] : 0.f;
        }

    if constexpr (H > 0) {
        // separable Gaussian: along rows (column index moves), then along columns
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
#pragma unroll
                for (int p = 0; p < 4; p++) z[p][ty + 16 * i][tx + 16 * j] = acc[i][j][p];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const int rw = ty + 16 * i, cl = tx + 16 * j;
                if (cl < T)
#pragma unroll
                    for (int p = 0; p < 4; p++) {
                        float s = 0.f;
#pragma unroll
                        for (int t = 0; t < TAPS; t++) s = fmaf(a.w[t], z[p][rw][cl + t], s);
                        acc[i][j][p] = s;
                    }
            }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                if (tx + 16 * j < T)
#pragma unroll
                    for (int p = 0; p < 4; p++) z[p][ty + 16 * i][tx + 16 * j] = acc[i][j][p];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const int rw = ty + 16 * i, cl = tx + 16 * j;
                if (rw < T && cl < T)
#pragma unroll
                    for (int p = 0; p < 4; p++) {
                        float s = 0.f;
#pragma unroll
                        for (int t = 0; t < TAPS; t++) s = fmaf(a.w[t], z[p][rw + t][cl], s);
                        acc[i][j][p] = s;
                    }
            }
    }

    // masked update and misfit sums
    const bool last = *a.iter == a.iters - 1;
    double mis = 0.0, ref = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (!out[i][j]) continue;
            const int64_t gi = oi + ty + 16 * i, gj = oj + tx + 16 * j;
#pragma unroll
            for (int p = 0; p < 4; p++) {
                const float x = acc[i][j][p];
                a.C[p * a.cps + gi * a.ldc + gj] = obs[i][j] ? mv[i][j][p] : x;
                if (last) a.X[p * a.xps + gi * a.ldx + gj] = x;
                if (obs[i][j]) {
                    const double d = (double)x - (double)mv[i][j][p];
                    mis += d * d;
                    ref += (double)mv[i][j][p] * (double)mv[i][j][p];
                }
            }
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mis += __shfl_down(mis, off, 64);
        ref += __shfl_down(ref, off, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = mis;
        red[1][tid >> 6] = ref;
    }
    __syncthreads();
    if (tid == 0) {
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        a.part[2 * b] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        a.part[2 * b + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// fit[it] = sqrt(sum mis / sum ref) over the workgroup sums (fixed order), then it += 1.
__global__ __launch_bounds__(256) void k_complete_fit(const double* part, int64_t nb, double* fit, int* iter,
                                                      int iters) {
    __shared__ double sm[2][256];
    const int tid = threadIdx.x;
    double mis = 0.0, ref = 0.0;
    for (int64_t b = tid; b < nb; b += 256) {
        mis += part[2 * b];
        ref += part[2 * b + 1];
    }
    sm[0][tid] = mis;
    sm[1][tid] = ref;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sm[0][tid] += sm[0][tid + s];
            sm[1][tid] += sm[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int t = *iter;
        if (fit && t >= 0 && t < iters) fit[t] = sqrt(sm[0][0] / sm[1][0]);
        *iter = t + 1;
    }
}

// C = mask . M (zero where unobserved); status and iteration counter cleared.
__global__ __launch_bounds__(256) void k_complete_init(const float* M, int64_t ldm, int64_t mps,
                                                       const unsigned char* mask, int64_t ldk, int64_t m, int64_t n,
                                                       float* C, int64_t ldc, int64_t cps, int* iter, int* status) {
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e0 == 0) {
        *iter = 0;
        status[0] = 0;
    }
    for (int64_t e = e0; e < m * n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        const bool obs = mask[i * ldk + j] != 0;
#pragma unroll
        for (int p = 0; p < 4; p++) C[p * cps + i * ldc + j] = obs ? M[p * mps + i * ldm + j] : 0.f;
    }
}

// dst[0] |= src[0] (the sticky status bits of an iteration's solve).
__global__ void k_status_or(int* dst, const int* src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] |= src[0];
}

}  // namespace

int complete_radius(double sigma) {
    if (!(sigma > 0.0)) return 0;
    return (int)std::ceil(3.0 * sigma);
}

int complete_tile(int radius) { return kZ - 2 * radius; }

int64_t complete_blocks(int64_t m, int64_t n, int radius) {
    const int64_t T = complete_tile(radius);
    return ((m + T - 1) / T) * ((n + T - 1) / T);
}

hipError_t complete_init_launch(const float* M, int64_t ldm, int64_t mps, const unsigned char* mask, int64_t ldk,
                                int64_t m, int64_t n, float* C, int64_t ldc, int64_t cps, int* iter, int* status,
                                hipStream_t st) {
    int64_t blocks = (m * n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_complete_init, dim3((unsigned)blocks), dim3(256), 0, st, M, ldm, mps, mask, ldk, m, n, C, ldc,
                       cps, iter, status);
    return hipGetLastError();
}

hipError_t complete_step_launch(const CompleteStep& s, hipStream_t st) {
    const int h = complete_radius(s.sigma);
    if (h > kCompleteMaxRadius || s.R < 1 || s.m < 1 || s.n < 1) return hipErrorInvalidValue;
    StepArgs a{};
    a.U = s.U; a.ldu = s.ldu; a.ups = s.ups;
    a.S = s.S;
    a.V = s.V; a.ldv = s.ldv; a.vps = s.vps;
    a.R = s.R;
    a.M = s.M; a.ldm = s.ldm; a.mps = s.mps;
    a.mask = s.mask; a.ldk = s.ldk;
    a.C = s.C; a.ldc = s.ldc; a.cps = s.cps;
    a.X = s.X; a.ldx = s.ldx; a.xps = s.xps;
    a.m = s.m; a.n = s.n;
    // normalised taps exp(-t^2 / (2 sigma^2)), t = -h .. h, summed in FP64
    double w[2 * kCompleteMaxRadius + 1] = {0.0}, sum = 0.0;
    for (int t = -h; t <= h; t++) sum += (w[t + h] = h ? std::exp(-(double)t * t / (2.0 * s.sigma * s.sigma)) : 1.0);
    for (int t = 0; t <= 2 * h; t++) a.w[t] = (float)(w[t] / sum);
    a.iter = s.iter; a.iters = s.iters;
    a.part = s.part;
    const int T = complete_tile(h);
    const int64_t gx = (s.n + T - 1) / T, gy = (s.m + T - 1) / T;
    if (gx > 0x7fffffff || gy > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)gx, (unsigned)gy);
    switch (h) {
        case 0: hipLaunchKernelGGL(k_complete_step<0>, grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL(k_complete_step<1>, grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL(k_complete_step<2>, grid, dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL(k_complete_step<3>, grid, dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL(k_complete_step<4>, grid, dim3(256), 0, st, a); break;
        case 5: hipLaunchKernelGGL(k_complete_step<5>, grid, dim3(256), 0, st, a); break;
        case 6: hipLaunchKernelGGL(k_complete_step<6>, grid, dim3(256), 0, st, a); break;
        case 7: hipLaunchKernelGGL(k_complete_step<7>, grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL(k_complete_step<8>, grid, dim3(256), 0, st, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_complete_fit, dim3(1), dim3(256), 0, st, (const double*)s.part, gx * gy, s.fit, s.iter,
                       s.iters);
    return hipGetLastError();
}

hipError_t status_or_launch(int* dst, const int* src, hipStream_t st) {
    hipLaunchKernelGGL(k_status_or, dim3(1), dim3(64), 0, st, dst, src);
    return hipGetLastError();
}

}  // namespace qlra_impl
