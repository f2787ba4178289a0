// Small FP64 quaternion SVD (eq. (qsvd)) and the per-solve epilogue kernels.
//
// The QSVD is one-sided (Hestenes) Jacobi on the columns of X.  In the complex adjoint
// chi(X) = [[Xa, Xb], [-conj Xb, conj Xa]] every quaternion column x is the pair of complex
// columns (first column of chi(x), its partner J conj(.)); two quaternion columns a, b are
// orthogonal exactly when both complex inner products of those pairs vanish, i.e. when the
// quaternion a^H b = 0.  The structure-preserving rotation that achieves it: with
// g = a^H b = |g| phi, replace b by b conj(phi) (a unitary column scaling, making a^H b real)
// and apply the real rotation that diagonalises [[|a|^2, |g|], [|g|, |b|^2]].  Working on the
// quaternion form keeps chi's pairing exact and stores half the numbers.
// Columns are held column-major in scratch (one column contiguous) and swept in round-robin
// (tournament) order: all w/2 pairs of a round are disjoint and run in parallel, one wave
// per pair; a sweep is w-1 rounds; sweeps stop when no pair needs a rotation.
#include "common.h"

namespace qlra_impl {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Pair `idx` of round `r` in the circle method for `np` (even) players.
__device__ __forceinline__ void rr_pair(int r, int idx, int np, int* a, int* b) {
    const int n1 = np - 1;
    if (idx == 0) {
        *a = 0;
        *b = 1 + r;
    } else {
        *a = 1 + (r + idx) % n1;
        *b = 1 + (r - idx + n1) % n1;
    }
}

// X (w x w row-major planes) -> S (descending), U (left vectors), V (right vectors).
// work: Mt [4][w][w] column-major copy, Vt [4][w][w], sig [w], rank [w] (as doubles).
__global__ __launch_bounds__(kThreads) void k_qsvd(const double* __restrict__ X, int w,
                                                    double* __restrict__ U, double* __restrict__ S,
                                                    double* __restrict__ V, double* __restrict__ work,
                                                    int want_vectors) {
    __shared__ int s_rot;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ps = (int64_t)w * w;
    double* Mt = work;                 // Mt[p*ps + col*w + row]
    double* Vt = work + 4 * ps;
    double* sig = work + 8 * ps;
    for (int64_t e = tid; e < ps; e += kThreads) {
        const int r = (int)(e / w), c = (int)(e % w);
        for (int p = 0; p < 4; p++) {
            Mt[p * ps + (int64_t)c * w + r] = X[p * ps + e];
            if (want_vectors) Vt[p * ps + (int64_t)c * w + r] = (p == 0 && r == c) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    const int np = w + (w & 1);
    const double tol = (double)w * 2.220446049250313e-16;
    for (int sweep = 0; sweep < 40; sweep++) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r = 0; r < np - 1; r++) {
            for (int idx = wave; idx < np / 2; idx += kWaves) {
                int a, b;
                rr_pair(r, idx, np, &a, &b);
                if (a >= w || b >= w) continue;
                double al = 0, be = 0, g0 = 0, g1 = 0, g2 = 0, g3 = 0;
                for (int i = lane; i < w; i += 64) {
                    const double a0 = Mt[(int64_t)a * w + i], a1 = Mt[ps + (int64_t)a * w + i];
                    const double a2 = Mt[2 * ps + (int64_t)a * w + i], a3 = Mt[3 * ps + (int64_t)a * w + i];
                    const double b0 = Mt[(int64_t)b * w + i], b1 = Mt[ps + (int64_t)b * w + i];
                    const double b2 = Mt[2 * ps + (int64_t)b * w + i], b3 = Mt[3 * ps + (int64_t)b * w + i];
                    al += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
                    be += b0 * b0 + b1 * b1 + b2 * b2 + b3 * b3;
                    // conj(a) b, eq. (1) with a -> conj(a)
                    g0 += a0 * b0 + a1 * b1 + a2 * b2 + a3 * b3;
                    g1 += a0 * b1 - a1 * b0 - a2 * b3 + a3 * b2;
                    g2 += a0 * b2 + a1 * b3 - a2 * b0 - a3 * b1;
                    g3 += a0 * b3 - a1 * b2 + a2 * b1 - a3 * b0;
                }
                al = wave_sum(al); be = wave_sum(be);
                g0 = wave_sum(g0); g1 = wave_sum(g1); g2 = wave_sum(g2); g3 = wave_sum(g3);
                const double ag = sqrt(g0 * g0 + g1 * g1 + g2 * g2 + g3 * g3);
                if (!(ag > tol * sqrt(al * be)) || !(ag > 0.0)) continue;
                if (lane == 0) s_rot = 1;
                // phi = g / |g|; b <- b conj(phi); real rotation on (a, b).
                const double p0 = g0 / ag, p1 = -g1 / ag, p2 = -g2 / ag, p3 = -g3 / ag;  // conj(phi)
                const double zeta = (be - al) / (2.0 * ag);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int pass = 0; pass < (want_vectors ? 2 : 1); pass++) {
                    double* Z = pass ? Vt : Mt;
                    for (int i = lane; i < w; i += 64) {
                        const int64_t ia = (int64_t)a * w + i, ib = (int64_t)b * w + i;
                        const double a0 = Z[ia], a1 = Z[ps + ia], a2 = Z[2 * ps + ia], a3 = Z[3 * ps + ia];
                        const double x0 = Z[ib], x1 = Z[ps + ib], x2 = Z[2 * ps + ib], x3 = Z[3 * ps + ib];
                        // bt = b conj(phi)
                        const double b0 = x0 * p0 - x1 * p1 - x2 * p2 - x3 * p3;
                        const double b1 = x0 * p1 + x1 * p0 + x2 * p3 - x3 * p2;
                        const double b2 = x0 * p2 - x1 * p3 + x2 * p0 + x3 * p1;
                        const double b3 = x0 * p3 + x1 * p2 - x2 * p1 + x3 * p0;
                        Z[ia] = cs * a0 - sn * b0; Z[ps + ia] = cs * a1 - sn * b1;
                        Z[2 * ps + ia] = cs * a2 - sn * b2; Z[3 * ps + ia] = cs * a3 - sn * b3;
                        Z[ib] = sn * a0 + cs * b0; Z[ps + ib] = sn * a1 + cs * b1;
                        Z[2 * ps + ib] = sn * a2 + cs * b2; Z[3 * ps + ib] = sn * a3 + cs * b3;
                    }
                }
            }
            __syncthreads();
        }
        __syncthreads();
        if (s_rot == 0) break;
        __syncthreads();
    }
    // singular values = column norms; order by descending value (ties: lower index first)
    for (int c = wave; c < w; c += kWaves) {
        double s = 0;
        for (int i = lane; i < w; i += 64)
            for (int p = 0; p < 4; p++) {
                const double v = Mt[p * ps + (int64_t)c * w + i];
                s += v * v;
            }
        s = wave_sum(s);
        if (lane == 0) sig[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = tid; c < w; c += kThreads) {
        const double sc = sig[c];
        int rank = 0;
        for (int o = 0; o < w; o++) {
            const double so = sig[o];
            rank += (so > sc) || (so == sc && o < c);
        }
        S[rank] = sc;
        sig[w + c] = (double)rank;
    }
    __syncthreads();
    if (!U && !V) return;
    for (int64_t e = tid; e < ps; e += kThreads) {
        const int c = (int)(e / w), i = (int)(e % w);    // column c, row i
        const int rank = (int)sig[w + c];
        const double sc = sig[c];
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        for (int p = 0; p < 4; p++) {
            if (U) U[p * ps + (int64_t)i * w + rank] = Mt[p * ps + e] * inv;
            if (V && want_vectors) V[p * ps + (int64_t)i * w + rank] = Vt[p * ps + e];
        }
    }
}

__global__ void k_estimate(const double* S, int k, const double* nA2, double* e) {
    if (threadIdx.x != 0) return;
    double top = 0.0;
    for (int j = 0; j < k; j++) top += S[j] * S[j];
    const double a = *nA2;
    const double r = a - top;
    *e = a > 0.0 ? sqrt((r > 0.0 ? r : 0.0) / a) : 0.0;
}

// ||A||_F^2: block b sums rows [b*rows_per, ...) of all four planes in FP64.
__global__ __launch_bounds__(256) void k_fro2_part(const float* __restrict__ A, int64_t m, int64_t n,
                                                   int64_t lda, int64_t aps, int64_t rows_per,
                                                   double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per;
    const int64_t r1 = r0 + rows_per < m ? r0 + rows_per : m;
    double s = 0.0;
    for (int p = 0; p < 4; p++)
        for (int64_t r = r0; r < r1; r++)
            for (int64_t c = threadIdx.x; c < n; c += 256) {
                const double v = A[p * aps + r * lda + c];
                s += v * v;
            }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_fro2_final(const double* __restrict__ part, int nb, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Phase normalisation of the returned singular vectors: column j of U and V is right-multiplied
// by conj(nu / |nu|), nu the entry of largest modulus of V(:, j) (lowest row on ties).  Two
// coalesced passes: partial arg-max over row blocks of V (64 columns per block, a row read
// whole), then each apply block combines the partials of its 64 columns (the order on modulus
// and row is strict, so the scan order does not change the pick) and rotates its 16 rows of U
// and V, all loads of a thread issued before its stores.
struct PhasePart {
    double val;
    int64_t idx;
    float q[4];
};

__device__ __forceinline__ bool phase_better(double v, int64_t i, double bv, int64_t bi) {
    return v > bv || (v == bv && i < bi);
}

__global__ __launch_bounds__(256) void k_phase_part(const float* __restrict__ V, int64_t n, int64_t ldv, int64_t vps,
                                                    int k, int64_t rows_per, PhasePart* __restrict__ part) {
    __shared__ double sv[4][64];
    __shared__ int64_t si[4][64];
    const int c = threadIdx.x & 63, rs = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.y * 64 + c;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per;
    const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
    double best = -1.0;
    int64_t bi = r0;
    if (j < k) {
        for (int64_t i = r0 + rs; i < r1; i += 4) {
            const float* v = V + i * ldv + j;
            const double a = (double)v[0] * v[0] + (double)v[vps] * v[vps] + (double)v[2 * vps] * v[2 * vps] +
                             (double)v[3 * vps] * v[3 * vps];
            if (a > best) { best = a; bi = i; }
        }
    }
    sv[rs][c] = best;
    si[rs][c] = bi;
    __syncthreads();
    if (rs == 0 && j < k) {
        for (int t = 1; t < 4; t++)
            if (phase_better(sv[t][c], si[t][c], best, bi)) { best = sv[t][c]; bi = si[t][c]; }
        PhasePart pp;
        pp.val = best;
        pp.idx = bi;
        const bool ok = best >= 0.0;
        for (int t = 0; t < 4; t++) pp.q[t] = ok ? V[t * vps + bi * ldv + j] : 0.0f;
        part[(int64_t)blockIdx.x * k + j] = pp;
    }
}

template <int RPT>
__global__ __launch_bounds__(256) void k_phase_apply(float* U, int64_t m, int64_t ldu, int64_t ups, float* V, int64_t n,
                                                     int64_t ldv, int64_t vps, int k, const PhasePart* __restrict__ part,
                                                     int nparts) {
    __shared__ double sv[4][64];
    __shared__ int64_t si[4][64];
    __shared__ int sf[4][64];
    __shared__ double ph[4][64];
    __shared__ int okf[64];
    const int c = threadIdx.x & 63, rs = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.y * 64 + c;
    {
        // the four row groups scan interleaved quarters of the partial arg-maxes: the values and
        // rows of eight partials are read together, then compared in order
        double best = -1.0;
        int64_t bi = 0;
        int bt = -1;
        if (j < k) {
            for (int t0 = rs; t0 < nparts; t0 += 32) {
                double pv[8];
                int64_t pi[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int t = t0 + 4 * u;
                    pv[u] = t < nparts ? part[(int64_t)t * k + j].val : -1.0;
                    pi[u] = t < nparts ? part[(int64_t)t * k + j].idx : 0;
                }
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (pv[u] >= 0.0 && phase_better(pv[u], pi[u], best, bi)) { best = pv[u]; bi = pi[u]; bt = t0 + 4 * u; }
            }
        }
        sv[rs][c] = best;
        si[rs][c] = bi;
        sf[rs][c] = bt;
    }
    __syncthreads();
    if (rs == 0) {
        double best = sv[0][c];
        int64_t bi = si[0][c];
        int from = sf[0][c];
        for (int t = 1; t < 4; t++)
            if (sv[t][c] >= 0.0 && phase_better(sv[t][c], si[t][c], best, bi)) { best = sv[t][c]; bi = si[t][c]; from = sf[t][c]; }
        const bool ok = best > 0.0 && from >= 0 && j < k;
        const double nrm = ok ? sqrt(best) : 1.0;
        float q[4] = {0, 0, 0, 0};
        if (ok) {
            const PhasePart& pp = part[(int64_t)from * k + j];
            q[0] = pp.q[0]; q[1] = pp.q[1]; q[2] = pp.q[2]; q[3] = pp.q[3];
        }
        // conj(phase)
        ph[0][c] = q[0] / nrm; ph[1][c] = -q[1] / nrm;
        ph[2][c] = -q[2] / nrm; ph[3][c] = -q[3] / nrm;
        okf[c] = ok;
    }
    __syncthreads();
    if (j >= k || !okf[c]) return;
    const double p0 = ph[0][c], p1 = ph[1][c], p2 = ph[2][c], p3 = ph[3][c];
    // RPT rows per thread (rows t0 + rs + 4 u of U, then of V): all loads, then all stores
    const int64_t t0 = (int64_t)blockIdx.x * 4 * RPT;
    float xv[RPT][4];
#pragma unroll
    for (int u = 0; u < RPT; u++) {
        const int64_t t = t0 + rs + 4 * u;
        if (t < m + n) {
            const bool on_u = t < m;
            const float* x = on_u ? U + t * ldu + j : V + (t - m) * ldv + j;
            const int64_t ps = on_u ? ups : vps;
            xv[u][0] = x[0]; xv[u][1] = x[ps]; xv[u][2] = x[2 * ps]; xv[u][3] = x[3 * ps];
        }
    }
#pragma unroll
    for (int u = 0; u < RPT; u++) {
        const int64_t t = t0 + rs + 4 * u;
        if (t < m + n) {
            const bool on_u = t < m;
            float* x = on_u ? U + t * ldu + j : V + (t - m) * ldv + j;
            const int64_t ps = on_u ? ups : vps;
            const double x0 = xv[u][0], x1 = xv[u][1], x2 = xv[u][2], x3 = xv[u][3];
            x[0] = (float)(x0 * p0 - x1 * p1 - x2 * p2 - x3 * p3);
            x[ps] = (float)(x0 * p1 + x1 * p0 + x2 * p3 - x3 * p2);
            x[2 * ps] = (float)(x0 * p2 - x1 * p3 + x2 * p0 + x3 * p1);
            x[3 * ps] = (float)(x0 * p3 + x1 * p2 - x2 * p1 + x3 * p0);
        }
    }
}

int64_t phase_rows_per(int64_t n) {
    const int64_t r = (n + 255) / 256;
    return r < 32 ? 32 : r;
}

}  // namespace

size_t qsvd_work_doubles(int64_t w) {
    const size_t jac = (size_t)(8 * w * w + 2 * w);
    const size_t gram = qsvd_gram_work_doubles(w);
    return jac > gram ? jac : gram;
}

hipError_t qsvd_launch(const double* X, int64_t w, double* U, double* S, double* V, double* work,
                       int want_vectors, hipStream_t st) {
    if (w <= heig_max()) {
        // eigendecomposition of X^H X (Householder tridiagonalisation, multisection, twisted
        // factorisations): O(w) dependent steps instead of O(sweeps * w) Jacobi rounds
        return qsvd_gram_launch(X, w, want_vectors ? U : nullptr, S, want_vectors ? V : nullptr, work, st);
    } else {
        hipLaunchKernelGGL(k_qsvd, dim3(1), dim3(kThreads), 0, st, X, (int)w, U, S, V, work, want_vectors);
    }
    return hipGetLastError();
}

hipError_t estimate_launch(const double* S, int k, const double* nA2, double* e, hipStream_t st) {
    hipLaunchKernelGGL(k_estimate, dim3(1), dim3(64), 0, st, S, k, nA2, e);
    return hipGetLastError();
}


hipError_t fro2_launch(const float* A, int64_t m, int64_t n, int64_t lda, int64_t aps, double* partial,
                       double* out, hipStream_t st) {
    const int64_t nb = m < 1024 ? m : 1024;
    const int64_t rows_per = (m + nb - 1) / nb;
    const int64_t blocks = (m + rows_per - 1) / rows_per;
    hipLaunchKernelGGL(k_fro2_part, dim3((unsigned)blocks), dim3(256), 0, st, A, m, n, lda, aps, rows_per,
                       partial);
    hipLaunchKernelGGL(k_fro2_final, dim3(1), dim3(256), 0, st, partial, (int)blocks, out);
    return hipGetLastError();
}

hipError_t fro2_final_launch(const double* partial, int64_t nb, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_fro2_final, dim3(1), dim3(256), 0, st, partial, (int)nb, out);
    return hipGetLastError();
}

size_t phase_work_bytes(int64_t n, int k) {
    const int64_t rp = phase_rows_per(n);
    return (size_t)((n + rp - 1) / rp) * (size_t)k * sizeof(PhasePart);
}

hipError_t phase_launch(float* U, int64_t m, int64_t ldu, int64_t ups, float* V, int64_t n, int64_t ldv,
                        int64_t vps, int k, void* work, hipStream_t st) {
    if (k <= 0 || n <= 0) return hipSuccess;
    const int64_t rp = phase_rows_per(n);
    const int64_t nparts = (n + rp - 1) / rp;
    const unsigned gyc = (unsigned)((k + 63) / 64);
    PhasePart* part = (PhasePart*)work;
    hipLaunchKernelGGL(k_phase_part, dim3((unsigned)nparts, gyc), dim3(256), 0, st, V, n, ldv, vps, k, rp, part);
    constexpr int kRpt = 4;                      // rows per thread; 16 rows per workgroup
    const int64_t rb = 4 * kRpt;
    hipLaunchKernelGGL(k_phase_apply<kRpt>, dim3((unsigned)((m + n + rb - 1) / rb), gyc), dim3(256), 0, st, U, m, ldu,
                       ups, V, n, ldv, vps, k, (const PhasePart*)part, (int)nparts);
    return hipGetLastError();
}

}  // namespace qlra_impl
