// Hermitian quaternion eigendecomposition of a small Gram matrix G = X^H X (w x w), used for the
// small QSVD (eq. (qsvd)) of a triangular factor R: with G = R^H R = V S^2 V^H the right
// singular vectors of R are the eigenvectors of G, sigma = sqrt(lambda), and the left vectors
// are R V S^{-1}.  The per-pass estimates need only sum_{j<=k} sigma_j^2, i.e. the k largest
// eigenvalues of the Gram that the CholeskyQR of the view already formed.
//
// Algorithm (one workgroup, FP64):
//  1. Householder tridiagonalisation with quaternion reflectors H = I - tau v v^H (the
//     two-sided update G <- H G H = G - v q^H - q v^H, q = p - K v, p = tau G v,
//     K = tau/2 v^H p, needs only the lower triangle).  The subdiagonal is quaternion; a
//     unitary diagonal scaling D makes it real, so T = D^H Q^H G Q D is real symmetric
//     tridiagonal (the structure-preserving counterpart of reducing the complex adjoint).
//  2. Eigenvalues of T by multisection with Sturm counts from the division-free three-term
//     recurrence of the characteristic polynomials (rescaled to stay in range).
//  3. Eigenvectors of T from twisted factorisations (forward and backward pivots of T - mu,
//     twist index of least |gamma|; inverse iteration with a tridiagonal LU for widths above
//     the LDS limit), re-orthogonalised inside clusters of close eigenvalues.
//  4. Back-transformation y = Q D x with the stored reflectors.
// Storage: the lower triangle of G, packed by rows, four planes; in LDS for w <= kHeigLds,
// otherwise in the caller's scratch (L2 resident).  Reflector v_j overwrites column j below
// the subdiagonal.
#include "common.h"

namespace qlra_impl {
namespace {

constexpr int HT = 1024;
constexpr int kHeigLds = 64;
constexpr int kLdsPacked = kHeigLds * (kHeigLds + 1) / 2;

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
__device__ __forceinline__ Q4 qadd(Q4 a, Q4 b) { return Q4{a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ Q4 qsub(Q4 a, Q4 b) { return Q4{a.w - b.w, a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Q4 qscale(Q4 a, double s) { return Q4{a.w * s, a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double qn2(Q4 a) { return a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z; }
__device__ __forceinline__ double qdot(Q4 a, Q4 b) { return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z; }

// Lower triangle packed by rows: (i, t), t <= i, at i (i + 1) / 2 + t.
struct Low {
    double* p;
    int np;
    __device__ __forceinline__ int idx(int i, int t) const { return i * (i + 1) / 2 + t; }
    __device__ __forceinline__ Q4 get(int i, int t) const {
        const int k = idx(i, t);
        return Q4{p[k], p[np + k], p[2 * np + k], p[3 * np + k]};
    }
    __device__ __forceinline__ void set(int i, int t, Q4 v) {
        const int k = idx(i, t);
        p[k] = v.w; p[np + k] = v.x; p[2 * np + k] = v.y; p[3 * np + k] = v.z;
    }
    // G(i, t) of the Hermitian matrix from its lower triangle
    __device__ __forceinline__ Q4 herm(int i, int t) const { return t <= i ? get(i, t) : qconj(get(t, i)); }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup (all threads must call it).
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0;
    for (int i = 0; i < HT / 64; i++) s += red[i];
    return s;
}

// Number of eigenvalues of the real symmetric tridiagonal (d, b) below x: sign changes of the
// Sturm sequence p_0 = 1, p_1 = d_0 - x, p_i = (d_{i-1} - x) p_{i-1} - b_{i-2}^2 p_{i-2}.
__device__ int sturm_count(const double* d, const double* b2, int w, double x) {
    double pm = 1.0, pc = d[0] - x;
    int cnt = pc < 0.0;
    int prev_neg = pc < 0.0;
    for (int i = 1; i < w; i++) {
        double pn = (d[i] - x) * pc - b2[i - 1] * pm;
        pm = pc;
        pc = pn;
        const double a = fabs(pc);
        if (a > 1e150) { pc *= 1e-150; pm *= 1e-150; }
        else if (a < 1e-150 && fabs(pm) < 1e-150) { pc *= 1e150; pm *= 1e150; }
        const int neg = pc < 0.0 ? 1 : (pc > 0.0 ? 0 : prev_neg);
        cnt += (neg != prev_neg);
        prev_neg = neg;
    }
    return cnt;
}

// Scratch of the eigensolver (w <= kHeigLds): everything the dependent steps touch is in LDS.
struct HeigLds {
    double G[4 * kLdsPacked];          // lower triangle, reflectors below the subdiagonal
    double P[4 * kHeigLds];            // p, then q
    double tau[kHeigLds], sq[4 * kHeigLds], ph[4 * kHeigLds];
    double dg[kHeigLds], b[kHeigLds], b2[kHeigLds], lasc[kHeigLds];
    double X[kHeigLds * kHeigLds];     // eigenvectors of T, column k at X + k * kHeigLds
    double piv[kHeigLds * kHeigLds];   // forward pivots of the twisted factorisations
    double red[HT / 64];
    double bnd[2];
};

// Eigendecomposition for w <= kHeigLds, all scratch in LDS.
__global__ __launch_bounds__(HT) void k_heig_lds(const double* __restrict__ Gin, int w, double* __restrict__ lam,
                                                 double* __restrict__ E) {
    __shared__ HeigLds L;
    const int tid = threadIdx.x;
    const int ty = tid >> 5, tx = tid & 31;
    const int grp8 = tid >> 3, sub8 = tid & 7;
    const int np = w * (w + 1) / 2;
    Low G{L.G, np};
    double* P = L.P;
    const int64_t gps = (int64_t)w * w;
    for (int i = ty; i < w; i += 32)
        for (int t = tx; t <= i; t += 32) {
            const int64_t e = (int64_t)i * w + t;
            Q4 v{Gin[e], Gin[gps + e], Gin[2 * gps + e], Gin[3 * gps + e]};
            if (i == t) v.x = v.y = v.z = 0.0;
            G.set(i, t, v);
        }
    __syncthreads();

    // ---- 1. tridiagonalisation
    for (int j = 0; j + 2 < w; j++) {
        double part = 0.0;
        for (int i = j + 1 + tid; i < w; i += HT) part += qn2(G.get(i, j));
        const double alpha2 = block_sum(part, L.red);
        const Q4 x1 = G.get(j + 1, j);
        const double ax1 = sqrt(qn2(x1));
        const double alpha = sqrt(alpha2);
        const Q4 phi = ax1 > 0.0 ? qscale(x1, 1.0 / ax1) : Q4{1, 0, 0, 0};
        const bool live = alpha > 0.0;
        const double tj = live ? 2.0 / (2.0 * alpha * (alpha + ax1)) : 0.0;
        __syncthreads();                           // everyone has read x1 before v_0 replaces it
        if (tid == 0) {
            L.tau[j] = tj;
            const Q4 s = qscale(phi, -alpha);      // H x = -alpha phi e_1
            L.sq[j] = s.w; L.sq[kHeigLds + j] = s.x; L.sq[2 * kHeigLds + j] = s.y; L.sq[3 * kHeigLds + j] = s.z;
            if (live) G.set(j + 1, j, qadd(x1, qscale(phi, alpha)));
        }
        __syncthreads();
        if (!live) continue;                       // uniform: alpha is a block-wide value
        // p_i = tau sum_t G22(i, t) v_t over i, t in [j+1, w); 8 lanes per row
        for (int i = j + 1 + grp8; i < w; i += HT / 8) {
            Q4 s{0, 0, 0, 0};
            for (int t = j + 1 + sub8; t < w; t += 8) s = qadd(s, qmul(G.herm(i, t), G.get(t, j)));
#pragma unroll
            for (int o = 4; o > 0; o >>= 1) {
                s.w += __shfl_xor(s.w, o, 64); s.x += __shfl_xor(s.x, o, 64);
                s.y += __shfl_xor(s.y, o, 64); s.z += __shfl_xor(s.z, o, 64);
            }
            if (sub8 == 0) {
                P[i] = tj * s.w; P[kHeigLds + i] = tj * s.x; P[2 * kHeigLds + i] = tj * s.y; P[3 * kHeigLds + i] = tj * s.z;
            }
        }
        __syncthreads();
        double kp = 0.0;
        for (int i = j + 1 + tid; i < w; i += HT)
            kp += qdot(G.get(i, j), Q4{P[i], P[kHeigLds + i], P[2 * kHeigLds + i], P[3 * kHeigLds + i]});
        const double K = 0.5 * tj * block_sum(kp, L.red);
        for (int i = j + 1 + tid; i < w; i += HT) {
            const Q4 v = G.get(i, j);
            P[i] -= K * v.w; P[kHeigLds + i] -= K * v.x; P[2 * kHeigLds + i] -= K * v.y; P[3 * kHeigLds + i] -= K * v.z;
        }
        __syncthreads();
        // G22 -= v q^H + q v^H on the lower triangle
        for (int i = j + 1 + ty; i < w; i += 32) {
            const Q4 vi = G.get(i, j), qi{P[i], P[kHeigLds + i], P[2 * kHeigLds + i], P[3 * kHeigLds + i]};
            for (int t = j + 1 + tx; t <= i; t += 32) {
                const Q4 vt = G.get(t, j), qt{P[t], P[kHeigLds + t], P[2 * kHeigLds + t], P[3 * kHeigLds + t]};
                Q4 g = qsub(qsub(G.get(i, t), qmul(vi, qconj(qt))), qmul(qi, qconj(vt)));
                if (i == t) g.x = g.y = g.z = 0.0;
                G.set(i, t, g);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (w >= 2) {
            const Q4 s = G.get(w - 1, w - 2);
            L.sq[w - 2] = s.w; L.sq[kHeigLds + w - 2] = s.x; L.sq[2 * kHeigLds + w - 2] = s.y;
            L.sq[3 * kHeigLds + w - 2] = s.z;
            L.tau[w - 2] = 0.0;
        }
        L.tau[w - 1] = 0.0;
        Q4 pj{1, 0, 0, 0};
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < w; i++) {
            L.dg[i] = G.get(i, i).w;
            L.ph[i] = pj.w; L.ph[kHeigLds + i] = pj.x; L.ph[2 * kHeigLds + i] = pj.y; L.ph[3 * kHeigLds + i] = pj.z;
            double bl = 0.0, br = 0.0;
            L.b[i] = 0.0; L.b2[i] = 0.0;
            if (i + 1 < w) {
                const Q4 s{L.sq[i], L.sq[kHeigLds + i], L.sq[2 * kHeigLds + i], L.sq[3 * kHeigLds + i]};
                const double bs = sqrt(qn2(s));
                L.b[i] = bs;
                L.b2[i] = bs * bs;
                br = bs;
                pj = bs > 0.0 ? qscale(qmul(s, pj), 1.0 / bs) : Q4{1, 0, 0, 0};
            }
            if (i > 0) bl = L.b[i - 1];
            lo = fmin(lo, L.dg[i] - bl - br);
            hi = fmax(hi, L.dg[i] + bl + br);
        }
        const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
        L.bnd[0] = lo - pad;
        L.bnd[1] = hi + pad;
    }
    __syncthreads();

    // ---- 2. eigenvalues: 16 lanes per eigenvalue, 17-section per round
    {
        const int g16 = tid >> 4, s16 = tid & 15;
        const int k = g16;                         // ascending index, w <= 64 = HT / 16
        double a = L.bnd[0], bb = L.bnd[1];
        for (int round = 0; round < 20; round++) {
            const double x = a + (bb - a) * (double)(s16 + 1) / 17.0;
            const int c = k < w ? sturm_count(L.dg, L.b2, w, x) : 0;
            const unsigned long long m = __ballot(c > k);
            const unsigned grpmask = (unsigned)((m >> ((tid & 63) & ~15)) & 0xFFFFull);
            const int first = grpmask ? __builtin_ctz(grpmask) : 16;
            const double xa = first == 0 ? a : a + (bb - a) * (double)first / 17.0;
            const double xb = first == 16 ? bb : a + (bb - a) * (double)(first + 1) / 17.0;
            a = xa;
            bb = xb;
        }
        if (k < w && s16 == 0) L.lasc[k] = 0.5 * (a + bb);
    }
    __syncthreads();
    for (int k = tid; k < w; k += HT) lam[k] = L.lasc[w - 1 - k];    // descending
    if (!E) return;

    // ---- 3. eigenvectors of T by twisted factorisations, one thread per eigenvalue:
    // forward pivots D+ from the top, backward pivots D- from the bottom, twist index r with
    // minimal |gamma_r| = |D+_r + D-_r - (d_r - mu)|, then x_r = 1 propagated both ways.
    const double tnorm = fmax(fabs(L.bnd[0]), fabs(L.bnd[1])) + 1e-300;
    const double tiny = 1e-300 + 2.220446049250313e-16 * tnorm * 1e-3;
    if (tid < w) {
        const int k = tid;
        const double mu = L.lasc[k];
        double* dp = L.piv + k * kHeigLds;
        double* x = L.X + k * kHeigLds;
        // forward: dp_0 = d_0 - mu, dp_i = d_i - mu - b_{i-1}^2 / dp_{i-1}
        double prev = L.dg[0] - mu;
        if (fabs(prev) < tiny) prev = -tiny;
        dp[0] = prev;
        for (int i = 1; i < w; i++) {
            double v = (L.dg[i] - mu) - L.b2[i - 1] / prev;
            if (fabs(v) < tiny) v = -tiny;
            dp[i] = v;
            prev = v;
        }
        // backward pivots (kept in x temporarily) and the twist index
        double dm = L.dg[w - 1] - mu;
        if (fabs(dm) < tiny) dm = -tiny;
        x[w - 1] = dm;
        int r = w - 1;
        double best = fabs(dp[w - 1]);            // gamma_{w-1} = dp_{w-1}
        for (int i = w - 2; i >= 0; i--) {
            double v = (L.dg[i] - mu) - L.b2[i] / dm;
            if (fabs(v) < tiny) v = -tiny;
            x[i] = v;
            dm = v;
            const double gam = fabs(dp[i] + v - (L.dg[i] - mu));
            if (gam < best) { best = gam; r = i; }
        }
        // downward from r: x_{i+1} = -b_i x_i / dm_{i+1}; upward: x_{i-1} = -b_{i-1} x_i / dp_{i-1}
        double xv = 1.0;
        double nrm = 1.0;
        for (int i = r; i + 1 < w; i++) {
            const double nx = -L.b[i] * xv / x[i + 1];
            x[i + 1] = nx;
            xv = nx;
            nrm += nx * nx;
        }
        xv = 1.0;
        for (int i = r; i > 0; i--) {
            const double nx = -L.b[i - 1] * xv / dp[i - 1];
            x[i - 1] = nx;
            xv = nx;
            nrm += nx * nx;
        }
        x[r] = 1.0;
        nrm = 1.0 / sqrt(nrm);
        for (int i = 0; i < w; i++) x[i] *= nrm;
    }
    __syncthreads();
    // clusters of close eigenvalues: modified Gram-Schmidt, ascending order (one wave)
    if (tid < 64) {
        int c0 = 0;
        for (int k = 1; k <= w; k++) {
            if (k < w && L.lasc[k] - L.lasc[k - 1] <= 1e-10 * tnorm) continue;
            for (int a = c0 + 1; a < k; a++) {
                double* xa = L.X + a * kHeigLds;
                for (int bq = c0; bq < a; bq++) {
                    const double* xb = L.X + bq * kHeigLds;
                    double dot = 0.0;
                    for (int i = tid; i < w; i += 64) dot += xa[i] * xb[i];
                    dot = wave_sum(dot);
                    for (int i = tid; i < w; i += 64) xa[i] -= dot * xb[i];
                }
                double nr2 = 0.0;
                for (int i = tid; i < w; i += 64) nr2 += xa[i] * xa[i];
                nr2 = wave_sum(nr2);
                const double inv = nr2 > 0.0 ? 1.0 / sqrt(nr2) : 0.0;
                for (int i = tid; i < w; i += 64) xa[i] *= inv;
            }
            c0 = k;
        }
    }
    __syncthreads();
    // ---- 4. back-transformation y = H_0 ... H_{w-3} D x, one 16-lane group per eigenvector,
    // y in registers (lane s16 holds rows s16, s16 + 16, s16 + 32, s16 + 48)
    {
        const int g16 = tid >> 4, s16 = tid & 15;
        const int kk = g16;                        // output column, descending order
        const bool act = kk < w;
        const double* xk = L.X + (act ? (w - 1 - kk) : 0) * kHeigLds;
        Q4 y[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int i = s16 + 16 * u;
            const double xv = (act && i < w) ? xk[i] : 0.0;
            y[u] = i < w ? Q4{L.ph[i] * xv, L.ph[kHeigLds + i] * xv, L.ph[2 * kHeigLds + i] * xv,
                              L.ph[3 * kHeigLds + i] * xv}
                         : Q4{0, 0, 0, 0};
        }
        for (int j = w - 3; j >= 0; j--) {
            const double tj = L.tau[j];
            if (tj == 0.0) continue;               // uniform
            Q4 s{0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int i = s16 + 16 * u;
                if (i > j && i < w) s = qadd(s, qmul(qconj(G.get(i, j)), y[u]));
            }
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) {
                s.w += __shfl_xor(s.w, o, 64); s.x += __shfl_xor(s.x, o, 64);
                s.y += __shfl_xor(s.y, o, 64); s.z += __shfl_xor(s.z, o, 64);
            }
            s = qscale(s, tj);
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int i = s16 + 16 * u;
                if (i > j && i < w) y[u] = qsub(y[u], qmul(G.get(i, j), s));
            }
        }
        if (act) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int i = s16 + 16 * u;
                if (i < w) {
                    const int64_t o = (int64_t)i * w + kk;
                    E[o] = y[u].w; E[gps + o] = y[u].x; E[2 * gps + o] = y[u].y; E[3 * gps + o] = y[u].z;
                }
            }
        }
    }
}

template <bool SH>
__global__ __launch_bounds__(HT) void k_heig(const double* __restrict__ Gin, int w, double* __restrict__ lam,
                                             double* __restrict__ E, double* __restrict__ work) {
    __shared__ double shG[SH ? 4 * kLdsPacked : 4];
    __shared__ double red[HT / 64];
    __shared__ double s_bnd[2];
    const int tid = threadIdx.x;
    const int ty = tid >> 5, tx = tid & 31;
    const int grp8 = tid >> 3, sub8 = tid & 7;
    const int np = w * (w + 1) / 2;
    // scratch layout (doubles): [packed G if !SH] tau[w] s[4w] ph[4w] d[w] b2[w] lasc[w] P[4w] X[w*w] lu[5w*w]
    double* wk = work;
    Low G{SH ? shG : wk, np};
    if (!SH) wk += 4 * (size_t)np;
    double* tau = wk; wk += w;
    double* sq = wk; wk += 4 * w;        // quaternion subdiagonal s_j, planes of length w
    double* ph = wk; wk += 4 * w;        // phases of D
    double* dg = wk; wk += w;
    double* b2 = wk; wk += w;            // squared real subdiagonal
    double* lasc = wk; wk += w;          // eigenvalues ascending
    double* P = wk; wk += 4 * w;         // p, then q, planes of length w
    double* X = wk; wk += (size_t)w * w; // eigenvectors of T, column k at X + k*w
    double* LU = wk;                     // per-eigenvector elimination scratch, 5w each

    const int64_t gps = (int64_t)w * w;
    for (int i = ty; i < w; i += 32)
        for (int t = tx; t <= i; t += 32) {
            const int64_t e = (int64_t)i * w + t;
            Q4 v{Gin[e], Gin[gps + e], Gin[2 * gps + e], Gin[3 * gps + e]};
            if (i == t) v.x = v.y = v.z = 0.0;
            G.set(i, t, v);
        }
    __syncthreads();

    // ---- 1. tridiagonalisation
    for (int j = 0; j + 2 < w; j++) {
        double part = 0.0;
        for (int i = j + 1 + tid; i < w; i += HT) part += qn2(G.get(i, j));
        const double alpha2 = block_sum(part, red);
        const Q4 x1 = G.get(j + 1, j);
        const double ax1 = sqrt(qn2(x1));
        const double alpha = sqrt(alpha2);
        const Q4 phi = ax1 > 0.0 ? qscale(x1, 1.0 / ax1) : Q4{1, 0, 0, 0};
        const bool live = alpha > 0.0;
        const double tj = live ? 2.0 / (2.0 * alpha * (alpha + ax1)) : 0.0;
        __syncthreads();                           // everyone has read x1 before v_0 replaces it
        if (tid == 0) {
            tau[j] = tj;
            const Q4 s = qscale(phi, -alpha);     // H x = -alpha phi e_1
            sq[j] = s.w; sq[w + j] = s.x; sq[2 * w + j] = s.y; sq[3 * w + j] = s.z;
            if (live) G.set(j + 1, j, qadd(x1, qscale(phi, alpha)));   // v_0; v_i = x_i otherwise
        }
        __syncthreads();
        if (!live) continue;                       // uniform: alpha is a block-wide value
        // p_i = tau sum_t G22(i, t) v_t, i, t in [j+1, w); 8 lanes per row
        for (int i = j + 1 + grp8; i < w; i += HT / 8) {
            Q4 s{0, 0, 0, 0};
            for (int t = j + 1 + sub8; t < w; t += 8) s = qadd(s, qmul(G.herm(i, t), G.get(t, j)));
#pragma unroll
            for (int o = 4; o > 0; o >>= 1) {
                s.w += __shfl_xor(s.w, o, 64); s.x += __shfl_xor(s.x, o, 64);
                s.y += __shfl_xor(s.y, o, 64); s.z += __shfl_xor(s.z, o, 64);
            }
            if (sub8 == 0) { P[i] = tj * s.w; P[w + i] = tj * s.x; P[2 * w + i] = tj * s.y; P[3 * w + i] = tj * s.z; }
        }
        __syncthreads();
        // K = tau/2 Re(v^H p)
        double kp = 0.0;
        for (int i = j + 1 + tid; i < w; i += HT) kp += qdot(G.get(i, j), Q4{P[i], P[w + i], P[2 * w + i], P[3 * w + i]});
        const double K = 0.5 * tj * block_sum(kp, red);
        for (int i = j + 1 + tid; i < w; i += HT) {
            const Q4 v = G.get(i, j);
            P[i] -= K * v.w; P[w + i] -= K * v.x; P[2 * w + i] -= K * v.y; P[3 * w + i] -= K * v.z;
        }
        __syncthreads();
        // G22 -= v q^H + q v^H on the lower triangle
        for (int i = j + 1 + ty; i < w; i += 32) {
            const Q4 vi = G.get(i, j), qi{P[i], P[w + i], P[2 * w + i], P[3 * w + i]};
            for (int t = j + 1 + tx; t <= i; t += 32) {
                const Q4 vt = G.get(t, j), qt{P[t], P[w + t], P[2 * w + t], P[3 * w + t]};
                Q4 g = qsub(qsub(G.get(i, t), qmul(vi, qconj(qt))), qmul(qi, qconj(vt)));
                if (i == t) g.x = g.y = g.z = 0.0;
                G.set(i, t, g);
            }
        }
        __syncthreads();
    }
    // diagonal, the last subdiagonal entry, phases and the real tridiagonal
    if (tid == 0) {
        if (w >= 2) {
            const Q4 s = G.get(w - 1, w - 2);
            sq[w - 2] = s.w; sq[w + w - 2] = s.x; sq[2 * w + w - 2] = s.y; sq[3 * w + w - 2] = s.z;
            tau[w - 2] = 0.0;
        }
        tau[w - 1] = 0.0;
        Q4 pj{1, 0, 0, 0};
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < w; i++) {
            dg[i] = G.get(i, i).w;
            ph[i] = pj.w; ph[w + i] = pj.x; ph[2 * w + i] = pj.y; ph[3 * w + i] = pj.z;
            double bl = 0.0, br = 0.0;
            if (i + 1 < w) {
                const Q4 s{sq[i], sq[w + i], sq[2 * w + i], sq[3 * w + i]};
                const double bs = sqrt(qn2(s));
                b2[i] = bs * bs;
                br = bs;
                pj = bs > 0.0 ? qscale(qmul(s, pj), 1.0 / bs) : Q4{1, 0, 0, 0};
            }
            if (i > 0) bl = sqrt(b2[i - 1]);
            lo = fmin(lo, dg[i] - bl - br);
            hi = fmax(hi, dg[i] + bl + br);
        }
        const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
        s_bnd[0] = lo - pad;
        s_bnd[1] = hi + pad;
    }
    __syncthreads();

    // ---- 2. eigenvalues: 4 lanes per eigenvalue, 5-section per round
    {
        const int g4 = tid >> 2, s4 = tid & 3;
        for (int kb = 0; kb < w; kb += HT / 4) {
            const int k = kb + g4;                 // ascending index
            double a = s_bnd[0], b = s_bnd[1];
            for (int round = 0; round < 40; round++) {
                const double x = a + (b - a) * (double)(s4 + 1) / 5.0;
                const int c = k < w ? sturm_count(dg, b2, w, x) : 0;
                // first of the 4 points with more than k eigenvalues below it
                const int flag = c > k;
                int first = 4;
#pragma unroll
                for (int q = 3; q >= 0; q--) {
                    const int fq = __shfl(flag, (threadIdx.x & ~3) + q, 64);
                    if (fq) first = q;
                }
                const double xa = first == 0 ? a : a + (b - a) * (double)first / 5.0;
                const double xb = first == 4 ? b : a + (b - a) * (double)(first + 1) / 5.0;
                a = xa;
                b = xb;
                if (b - a <= 2.220446049250313e-16 * fmax(fabs(a), fabs(b)) + 1e-300) break;
            }
            if (k < w && s4 == 0) lasc[k] = 0.5 * (a + b);
        }
    }
    __syncthreads();
    for (int k = tid; k < w; k += HT) lam[k] = lasc[w - 1 - k];    // descending
    if (!E) return;

    // ---- 3. eigenvectors of T by inverse iteration, one thread per eigenvalue
    const double tnorm = fmax(fabs(s_bnd[0]), fabs(s_bnd[1])) + 1e-300;
    for (int k = tid; k < w; k += HT) {
        // perturb the shift off the exact eigenvalue
        const double mu = lasc[k] + 1e-13 * tnorm * ((k & 1) ? 1.0 : -1.0);
        double* xk = X + (size_t)k * w;
        double* dd = LU + (size_t)k * 5 * w;      // diag, super, super2, multiplier, pivot flag
        double* du = dd + w;
        double* du2 = du + w;
        double* ml = du2 + w;
        double* pv = ml + w;
        // LU of T - mu I with partial pivoting (LAPACK dgttrf-style)
        for (int i = 0; i < w; i++) { dd[i] = dg[i] - mu; du[i] = i + 1 < w ? sqrt(b2[i]) : 0.0; du2[i] = 0.0; }
        double sub_i = w > 1 ? sqrt(b2[0]) : 0.0;
        for (int i = 0; i + 1 < w; i++) {
            const double nextsub = i + 2 < w ? sqrt(b2[i + 1]) : 0.0;
            if (fabs(dd[i]) >= fabs(sub_i)) {
                pv[i] = 0.0;
                const double f = dd[i] != 0.0 ? sub_i / dd[i] : 0.0;
                ml[i] = f;
                dd[i + 1] -= f * du[i];
            } else {
                pv[i] = 1.0;
                const double f = dd[i] / sub_i;
                ml[i] = f;
                dd[i] = sub_i;
                const double t = du[i];
                du[i] = dd[i + 1];
                dd[i + 1] = t - f * dd[i + 1];
                if (i + 2 < w) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
            }
            sub_i = nextsub;
        }
        for (int i = 0; i < w; i++) if (dd[i] == 0.0) dd[i] = 1e-300 + 1e-16 * tnorm;
        for (int i = 0; i < w; i++) xk[i] = 1.0;
        for (int it = 0; it < 3; it++) {
            // forward: apply the row interchanges and multipliers
            for (int i = 0; i + 1 < w; i++) {
                if (pv[i] == 0.0) xk[i + 1] -= ml[i] * xk[i];
                else { const double t = xk[i]; xk[i] = xk[i + 1]; xk[i + 1] = t - ml[i] * xk[i + 1]; }
            }
            // back substitution with U (diag dd, super du, super2 du2)
            for (int i = w - 1; i >= 0; i--) {
                double s = xk[i];
                if (i + 1 < w) s -= du[i] * xk[i + 1];
                if (i + 2 < w) s -= du2[i] * xk[i + 2];
                xk[i] = s / dd[i];
            }
            double nrm = 0.0;
            for (int i = 0; i < w; i++) nrm += xk[i] * xk[i];
            nrm = 1.0 / sqrt(nrm);
            for (int i = 0; i < w; i++) xk[i] *= nrm;
        }
    }
    __syncthreads();
    // clusters of close eigenvalues: modified Gram-Schmidt, in ascending order
    if (tid == 0) {
        int c0 = 0;
        for (int k = 1; k <= w; k++) {
            if (k < w && lasc[k] - lasc[k - 1] <= 1e-10 * tnorm) continue;
            for (int a = c0 + 1; a < k; a++) {
                double* xa = X + (size_t)a * w;
                for (int b = c0; b < a; b++) {
                    const double* xb = X + (size_t)b * w;
                    double dot = 0.0;
                    for (int i = 0; i < w; i++) dot += xa[i] * xb[i];
                    for (int i = 0; i < w; i++) xa[i] -= dot * xb[i];
                }
                double nrm = 0.0;
                for (int i = 0; i < w; i++) nrm += xa[i] * xa[i];
                nrm = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
                for (int i = 0; i < w; i++) xa[i] *= nrm;
            }
            c0 = k;
        }
    }
    __syncthreads();
    // ---- 4. back-transformation: y = H_0 H_1 ... H_{w-3} D x, 16 lanes per eigenvector
    {
        const int g16 = tid >> 4, s16 = tid & 15;
        for (int kb = 0; kb < w; kb += HT / 16) {
            const int kk = kb + g16;               // output column (descending order)
            const bool act = kk < w;
            const double* xk = X + (size_t)(act ? (w - 1 - kk) : 0) * w;
            // y = D x into the output column kk
            for (int i = s16; i < w; i += 16) {
                if (!act) break;
                const double xv = xk[i];
                const int64_t o = (int64_t)i * w + kk;
                E[o] = ph[i] * xv; E[gps + o] = ph[w + i] * xv; E[2 * gps + o] = ph[2 * w + i] * xv;
                E[3 * gps + o] = ph[3 * w + i] * xv;
            }
            for (int j = w - 3; j >= 0; j--) {
                const double tj = tau[j];
                Q4 s{0, 0, 0, 0};
                if (act && tj != 0.0) {
                    for (int i = j + 1 + s16; i < w; i += 16) {
                        const int64_t o = (int64_t)i * w + kk;
                        s = qadd(s, qmul(qconj(G.get(i, j)), Q4{E[o], E[gps + o], E[2 * gps + o], E[3 * gps + o]}));
                    }
                }
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) {
                    s.w += __shfl_xor(s.w, o, 64); s.x += __shfl_xor(s.x, o, 64);
                    s.y += __shfl_xor(s.y, o, 64); s.z += __shfl_xor(s.z, o, 64);
                }
                if (act && tj != 0.0) {
                    s = qscale(s, tj);
                    for (int i = j + 1 + s16; i < w; i += 16) {
                        const int64_t o = (int64_t)i * w + kk;
                        const Q4 y = qsub(Q4{E[o], E[gps + o], E[2 * gps + o], E[3 * gps + o]}, qmul(G.get(i, j), s));
                        E[o] = y.w; E[gps + o] = y.x; E[2 * gps + o] = y.y; E[3 * gps + o] = y.z;
                    }
                }
            }
        }
    }
}

// G = X^H X for a small square X (w x w FP64 planes), full Hermitian storage.
__global__ __launch_bounds__(256) void k_gram_small(const double* __restrict__ X, int w, double* __restrict__ G) {
    const int64_t ps = (int64_t)w * w;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ps) return;
    const int a = (int)(e / w), b = (int)(e % w);
    Q4 s{0, 0, 0, 0};
    for (int i = 0; i < w; i++) {
        const int64_t ia = (int64_t)i * w + a, ib = (int64_t)i * w + b;
        s = qadd(s, qmul(qconj(Q4{X[ia], X[ps + ia], X[2 * ps + ia], X[3 * ps + ia]}),
                         Q4{X[ib], X[ps + ib], X[2 * ps + ib], X[3 * ps + ib]}));
    }
    if (a == b) s.x = s.y = s.z = 0.0;
    G[e] = s.w; G[ps + e] = s.x; G[2 * ps + e] = s.y; G[3 * ps + e] = s.z;
}

// sigma = sqrt(max(lambda, 0)) and U = X V diag(1/sigma) (left vectors) for the QSVD of X.
__global__ __launch_bounds__(256) void k_left_vectors(const double* __restrict__ X, int w,
                                                      const double* __restrict__ lam, const double* __restrict__ V,
                                                      double* __restrict__ S, double* __restrict__ U) {
    const int64_t ps = (int64_t)w * w;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < w) S[e] = sqrt(fmax(lam[e], 0.0));
    if (e >= ps || !U) return;
    const int i = (int)(e / w), c = (int)(e % w);
    const double sc = sqrt(fmax(lam[c], 0.0));
    const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
    Q4 s{0, 0, 0, 0};
    for (int t = 0; t < w; t++) {
        const int64_t it = (int64_t)i * w + t, tc = (int64_t)t * w + c;
        s = qadd(s, qmul(Q4{X[it], X[ps + it], X[2 * ps + it], X[3 * ps + it]},
                         Q4{V[tc], V[ps + tc], V[2 * ps + tc], V[3 * ps + tc]}));
    }
    U[e] = s.w * inv; U[ps + e] = s.x * inv; U[2 * ps + e] = s.y * inv; U[3 * ps + e] = s.z * inv;
}

}  // namespace

size_t heig_work_doubles(int64_t w) {
    const int64_t np = w * (w + 1) / 2;
    return (size_t)(4 * np + 16 * w + 6 * w * w + 64);
}

hipError_t heig_launch(const double* G, int64_t w, double* lam, double* E, double* work, hipStream_t st) {
    if (w <= kHeigLds)
        hipLaunchKernelGGL(k_heig_lds, dim3(1), dim3(HT), 0, st, G, (int)w, lam, E);
    else
        hipLaunchKernelGGL(k_heig<false>, dim3(1), dim3(HT), 0, st, G, (int)w, lam, E, work);
    return hipGetLastError();
}

// QSVD of a small square X through the eigendecomposition of X^H X: S descending, V right
// vectors, U left vectors (U, V may be null).  work: heig_work_doubles(w) + 5 w^2 doubles.
hipError_t qsvd_gram_launch(const double* X, int64_t w, double* U, double* S, double* V, double* work,
                            hipStream_t st) {
    const int64_t ps = w * w;
    double* G = work;
    double* lam = G + 4 * ps;
    double* Vt = lam + w;
    double* hw = Vt + 4 * ps;
    double* Vout = V ? V : Vt;
    hipLaunchKernelGGL(k_gram_small, dim3((unsigned)((ps + 255) / 256)), dim3(256), 0, st, X, (int)w, G);
    hipError_t e = heig_launch(G, w, lam, (U || V) ? Vout : nullptr, hw, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_left_vectors, dim3((unsigned)((ps + 255) / 256)), dim3(256), 0, st, X, (int)w, lam,
                       Vout, S, U);
    return hipGetLastError();
}

size_t qsvd_gram_work_doubles(int64_t w) { return (size_t)(8 * w * w + w) + heig_work_doubles(w); }

}  // namespace qlra_impl
