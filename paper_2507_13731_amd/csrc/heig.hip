// Hermitian quaternion eigendecomposition of a small Gram matrix G = X^H X (w x w, w <= 64),
// used for the small QSVD (Alg. 2 and Alg. 4, final truncated QSVD of R) and for the per-pass
// error estimates.  With G = R^H R = V S^2 V^H the right singular vectors of R are the
// eigenvectors of G, sigma = sqrt(lambda), and the left vectors are R V S^{-1}.  An estimate
// needs only sum_{j<=k} sigma_j^2, the k largest eigenvalues of the Gram that the CholeskyQR of
// the view formed anyway, so it skips the vectors.
//
// Pipeline (FP64), one record of kTriStride doubles per problem in global scratch:
//  k_tridiag   one workgroup per problem, the matrix in registers (1024 threads x 2 x 2
//              entries): Householder tridiagonalisation with quaternion reflectors
//              H = I - tau v v^H, applied two-sided as G <- G - v q^H - q v^H with p = tau G v,
//              K = tau/2 v^H p, q = p - K v.  The quaternion subdiagonal s_j is made real by a
//              unitary diagonal D (phases), so T = D^H Q^H G Q D is real symmetric tridiagonal:
//              the structure-preserving counterpart of reducing the complex adjoint.
//  k_eigvals   eigenvalues of T by multisection with Sturm counts (one wave per eigenvalue,
//              64 section points per round, 4 eigenvalues per workgroup, any number of
//              problems in one launch).
//  k_eigvecs   eigenvectors of T from twisted factorisations (forward and backward pivots of
//              T - mu, twist index of least |gamma|), modified Gram-Schmidt inside clusters of
//              close eigenvalues, and the back-transformation y = Q D x with the stored
//              reflectors; 16 eigenvectors per workgroup.
#include <algorithm>

#include "common.h"

namespace qlra_impl {
namespace {

constexpr int kW = 96;                          // largest order
constexpr int kPacked = kW * (kW + 1) / 2;      // packed lower triangle, (i, t) at i (i + 1) / 2 + t
constexpr int ET = 256;                         // eigenvalue / eigenvector workgroups
constexpr int kPer = ET / 64;                   // eigenvalues per workgroup, one wave each
constexpr int kRounds = 10;                     // 65-section rounds: width shrinks by 65^10 > 1e18

// record layout (doubles)
constexpr int OFF_D = 0, OFF_B = kW, OFF_B2 = 2 * kW, OFF_TAU = 3 * kW, OFF_PH = 4 * kW, OFF_BND = 8 * kW,
              OFF_LAM = 8 * kW + 8, OFF_REFL = 9 * kW + 8;
constexpr int kTriStride = OFF_REFL + 4 * kPacked;

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
// acc + a b and acc - a b (eq. (1)) as four chains of fused multiply-adds into acc
__device__ __forceinline__ Q4 qfma(Q4 acc, Q4 a, Q4 b) {
    return Q4{fma(-a.z, b.z, fma(-a.y, b.y, fma(-a.x, b.x, fma(a.w, b.w, acc.w)))),
              fma(-a.z, b.y, fma(a.y, b.z, fma(a.x, b.w, fma(a.w, b.x, acc.x)))),
              fma(a.z, b.x, fma(a.y, b.w, fma(-a.x, b.z, fma(a.w, b.y, acc.y)))),
              fma(a.z, b.w, fma(-a.y, b.x, fma(a.x, b.y, fma(a.w, b.z, acc.z))))};
}
__device__ __forceinline__ Q4 qfms(Q4 acc, Q4 a, Q4 b) {
    return Q4{fma(a.z, b.z, fma(a.y, b.y, fma(a.x, b.x, fma(-a.w, b.w, acc.w)))),
              fma(a.z, b.y, fma(-a.y, b.z, fma(-a.x, b.w, fma(-a.w, b.x, acc.x)))),
              fma(-a.z, b.x, fma(-a.y, b.w, fma(a.x, b.z, fma(-a.w, b.y, acc.y)))),
              fma(-a.z, b.w, fma(a.y, b.x, fma(-a.x, b.y, fma(-a.w, b.z, acc.z))))};
}
__device__ __forceinline__ double qdot(Q4 a, Q4 b) { return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z; }

// quaternion vectors stored as four planes of stride S
template <int S>
__device__ __forceinline__ Q4 ldq(const double* p, int i) { return Q4{p[i], p[S + i], p[2 * S + i], p[3 * S + i]}; }
template <int S>
__device__ __forceinline__ void stq(double* p, int i, Q4 v) {
    p[i] = v.w; p[S + i] = v.x; p[2 * S + i] = v.y; p[3 * S + i] = v.z;
}

// quaternion vectors with the four components of an entry side by side (16-byte aligned)
__device__ __forceinline__ void sti(double* p, int i, Q4 v) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    reinterpret_cast<d2*>(p)[2 * i] = d2{v.w, v.x};
    reinterpret_cast<d2*>(p)[2 * i + 1] = d2{v.y, v.z};
}
__device__ __forceinline__ Q4 ldi(const double* p, int i) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 lo = reinterpret_cast<const d2*>(p)[2 * i], hi = reinterpret_cast<const d2*>(p)[2 * i + 1];
    return Q4{lo[0], lo[1], hi[0], hi[1]};
}

template <bool SIDE>
__device__ __forceinline__ Q4 ldv(const double* p, int i) {
    if constexpr (SIDE) return ldi(p, i);
    else return ldq<kW>(p, i);
}
template <bool SIDE>
__device__ __forceinline__ void stv(double* p, int i, Q4 v) {
    if constexpr (SIDE) sti(p, i, v);
    else stq<kW>(p, i, v);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// lane i's value of v, broadcast (i uniform)
__device__ __forceinline__ double bcast(double v, int i) {
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffll), i);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), i);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ------------------------------------------------------------------------------------------
// cross-lane sums on the VALU (DPP), all lanes active

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// sum over the 4 lanes of a quad
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp<0xB1>(v);       // quad_perm [1, 0, 3, 2]
    v += dpp<0x4E>(v);       // quad_perm [2, 3, 0, 1]
    return v;
}
// sum over the 16 lanes of a row
__device__ __forceinline__ double row_sum(double v) {
    v = quad_sum(v);
    v += dpp<0x141>(v);      // row_half_mirror
    v += dpp<0x140>(v);      // row_mirror
    return v;
}
// sum over the wave (uniform result)
__device__ __forceinline__ double wave_total(double v) {
    v = row_sum(v);
    return bcast(v, 0) + bcast(v, 16) + bcast(v, 32) + bcast(v, 48);
}

// ------------------------------------------------------------------------------------------
// 1. tridiagonalisation
//
// Row r of G is held by LPR consecutive lanes (one DPP row of 16, or half of one), lane s owning
// the columns c = s + LPR kk (kk < NCOL): 1024 threads x 4 columns for w <= 64, 768 threads x
// 12 columns for w <= 96.  Matrix-vector products reduce on the VALU and every step skips the
// column blocks and waves that lie left of / above the active part.  Step j: the wave holding
// row j forms the reflector from that row (the column below the diagonal by Hermitian
// symmetry); barrier; p = tau G v per row with the wave's share of K = tau/2 v^H p; barrier; the
// rank-2 update.  v, p and the K shares are double-buffered, so the next reflector needs no
// third barrier.

// sum over groups of LPR consecutive lanes (LPR = 8 or 16)
template <int LPR>
__device__ __forceinline__ double lpr_sum(double v) {
    v = quad_sum(v);
    v += dpp<0x141>(v);      // row_half_mirror: 8 lanes
    if constexpr (LPR == 16) v += dpp<0x140>(v);   // row_mirror: 16 lanes
    return v;
}

template <int LPR, int NCOL, int NT>
__global__ __launch_bounds__(NT)
void k_tridiag(const double* __restrict__ Gall, int64_t gstride, int w, double* __restrict__ triall, int store_refl) {
    static_assert(NT / LPR == LPR * NCOL, "the thread grid covers a square of rows x columns");
    constexpr int RPW = 64 / LPR;           // rows per wave
    constexpr int TW = NT / 64;             // waves
    // x (column j below the diagonal), v (the reflector, zero outside rows j+1 .. w-1) and
    // p = tau G v; in the 1024-thread form the four components of an entry lie side by side
    // (two 16-byte accesses), the 768-thread form keeps planes (its registers are full)
    __shared__ __attribute__((aligned(16))) double xb[4 * kW];
    __shared__ __attribute__((aligned(16))) double vb[2][4 * kW];
    __shared__ __attribute__((aligned(16))) double pb[2][4 * kW];
    __shared__ double kr[2][TW];            // per-wave shares of v^H p
    __shared__ double tb[2];
    __shared__ double sq[4 * kW];           // quaternion subdiagonal s_j
    __shared__ double dg[kW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr bool kSide = NCOL <= 4;
    const int r = tid / LPR, s = tid % LPR;
    const double* G = Gall + (int64_t)blockIdx.x * gstride;
    double* tri = triall + (int64_t)blockIdx.x * kTriStride;
    const int64_t gps = (int64_t)w * w;

    Q4 g[NCOL];
#pragma unroll
    for (int kk = 0; kk < NCOL; kk++) {
        const int c = s + LPR * kk;
        Q4 v{0, 0, 0, 0};
        if (r < w && c < w) {
            const int64_t e = (int64_t)r * w + c;
            v = Q4{G[e], G[gps + e], G[2 * gps + e], G[3 * gps + e]};
            if (r == c) v.x = v.y = v.z = 0.0;
        }
        g[kk] = v;
    }

    for (int j = 0; j + 2 < w; j++) {
        const int bsel = j & 1;
        double* vbj = vb[bsel];
        double* pbj = pb[bsel];
        if (wave == j / RPW) {
            // the row-j lanes publish x_c = G(c, j) = conj(G(j, c)), c > j
            if (r == j) {
#pragma unroll
                for (int kk = 0; kk < NCOL; kk++) {
                    const int c = s + LPR * kk;
                    if (LPR * kk + LPR - 1 <= j) continue;     // uniform
                    if (c > j && c < w) stv<kSide>(xb, c, qconj(g[kk]));
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // lane handles entries lane and lane + 64
            const int c1 = lane + 64;
            const Q4 x = (lane > j && lane < w) ? ldv<kSide>(xb, lane) : Q4{0, 0, 0, 0};
            const Q4 x2 = (c1 > j && c1 < w) ? ldv<kSide>(xb, c1) : Q4{0, 0, 0, 0};
            const double alpha = sqrt(wave_total(qn2(x) + qn2(x2)));
            const Q4 x1 = ldv<kSide>(xb, j + 1);
            const double ax1 = sqrt(qn2(x1));
            const Q4 phi = ax1 > 0.0 ? qscale(x1, 1.0 / ax1) : Q4{1, 0, 0, 0};
            const double tau = alpha > 0.0 ? 1.0 / (alpha * (alpha + ax1)) : 0.0;
            Q4 v = x, v2 = x2;
            if (lane == j + 1) v = qadd(x, qscale(phi, alpha));   // H x = -alpha phi e_1
            if (c1 == j + 1) v2 = qadd(x2, qscale(phi, alpha));
            stv<kSide>(vbj, lane, v);
            if (c1 < kW) stv<kSide>(vbj, c1, v2);
            if (store_refl && lane > j && lane < w) stq<kPacked>(tri + OFF_REFL, lane * (lane + 1) / 2 + j, v);
            if (store_refl && c1 > j && c1 < w) stq<kPacked>(tri + OFF_REFL, c1 * (c1 + 1) / 2 + j, v2);
            if (lane == 0) {
                tb[bsel] = tau;
                stq<kW>(sq, j, qscale(phi, -alpha));
                tri[OFF_TAU + j] = tau;
            }
        }
        __syncthreads();
        const double tau = tb[bsel];
        const bool wave_live = RPW * wave + RPW - 1 > j;        // some row of this wave is active
        if (wave_live) {
            Q4 acc{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < NCOL; kk++) {
                if (LPR * kk + LPR - 1 <= j) continue;          // v vanishes there
                acc = qfma(acc, g[kk], ldv<kSide>(vbj, s + LPR * kk));
            }
            acc.w = lpr_sum<LPR>(acc.w); acc.x = lpr_sum<LPR>(acc.x);
            acc.y = lpr_sum<LPR>(acc.y); acc.z = lpr_sum<LPR>(acc.z);
            const Q4 p = qscale(acc, tau);
            double kp = 0.0;
            if (s == 0 && r < w) {
                stv<kSide>(pbj, r, p);
                if (r > j) kp = qdot(ldv<kSide>(vbj, r), p);
            }
            double ks = 0.0;
#pragma unroll
            for (int q = 0; q < RPW; q++) ks += bcast(kp, q * LPR);
            if (lane == 0) kr[bsel][wave] = ks;
        } else if (lane == 0) {
            kr[bsel][wave] = 0.0;
        }
        __syncthreads();
        if (wave_live) {
            double kq = 0.0;
            for (int q = s; q < TW; q += LPR) kq += kr[bsel][q];
            const double K = 0.5 * tau * lpr_sum<LPR>(kq);
            const bool row_live = r > j && r < w;
            const Q4 vr = ldv<kSide>(vbj, r);
            const Q4 qr = qsub(ldv<kSide>(pbj, r), qscale(vr, K));
#pragma unroll
            for (int kk = 0; kk < NCOL; kk++) {
                const int c = s + LPR * kk;
                if (LPR * kk + LPR - 1 <= j) continue;          // uniform
                const Q4 vc = ldv<kSide>(vbj, c);
                const Q4 qc = qsub(ldv<kSide>(pbj, c), qscale(vc, K));
                if (row_live && c > j && c < w) {
                    Q4 t = qfms(qfms(g[kk], vr, qconj(qc)), qr, qconj(vc));
                    if (r == c) t.x = t.y = t.z = 0.0;
                    g[kk] = t;
                }
            }
        }
    }
    // diagonal and the last subdiagonal entry s_{w-2} = G(w-1, w-2)
#pragma unroll
    for (int kk = 0; kk < NCOL; kk++) {
        const int c = s + LPR * kk;
        if (r < w && c == r) dg[r] = g[kk].w;
        if (w >= 2 && r == w - 1 && c == w - 2) stq<kW>(sq, w - 2, g[kk]);
    }
    __syncthreads();
    if (tid == 0) {
        // D: ph_0 = 1, ph_{j+1} = s_j ph_j / |s_j| turns s_j into the real b_j = |s_j|
        Q4 pj{1, 0, 0, 0};
        double lo = 1e300, hi = -1e300, bl = 0.0;
        for (int i = 0; i < w; i++) {
            const double d = dg[i];
            tri[OFF_D + i] = d;
            stq<kW>(tri + OFF_PH, i, pj);
            double br = 0.0;
            if (i + 1 < w) {
                const Q4 sj = ldq<kW>(sq, i);
                br = sqrt(qn2(sj));
                pj = br > 0.0 ? qscale(qmul(sj, pj), 1.0 / br) : Q4{1, 0, 0, 0};
            }
            tri[OFF_B + i] = br;
            tri[OFF_B2 + i] = br * br;
            lo = fmin(lo, d - bl - br);
            hi = fmax(hi, d + bl + br);
            bl = br;
        }
        if (w >= 2) tri[OFF_TAU + w - 2] = 0.0;
        tri[OFF_TAU + w - 1] = 0.0;
        const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
        tri[OFF_BND] = lo - pad;
        tri[OFF_BND + 1] = hi + pad;
    }
}

// ------------------------------------------------------------------------------------------
// 2. eigenvalues

// Number of eigenvalues of T below x: sign changes of the Sturm sequence p_0 = 1,
// p_1 = d_0 - x, p_i = (d_{i-1} - x) p_{i-1} - b_{i-2}^2 p_{i-2}.  Lane i of the wave holds d_i
// and b_i^2 in (dv, b2v) and d_{64+i}, b_{64+i}^2 in (dv2, b2v2), scaled so that |d_i - x| <= 2
// and b_i^2 <= 4: |p| grows at most 6-fold per step, so a rescale every fourth step keeps it in
// range, and only one FMA per step is on the chain.
__device__ __forceinline__ void sturm_step(double di, double bi, double x, double& pm, double& pc, int& prev,
                                           int& cnt) {
    const double pn = fma(di - x, pc, -bi * pm);
    pm = pc;
    pc = pn;
    // the sign of p_i (an exact zero keeps the previous sign), without branches
    int neg = pn < 0.0;
    neg = pn == 0.0 ? prev : neg;
    cnt += neg ^ prev;
    prev = neg;
}

__device__ __forceinline__ void sturm_rescale(double& pm, double& pc) {
    const double a = fmax(fabs(pc), fabs(pm));
    const double sc = a > 1e150 ? 1e-150 : (a < 1e-150 ? 1e150 : 1.0);
    pc *= sc;
    pm *= sc;
}

__device__ int sturm_count(double dv, double dv2, double b2v, double b2v2, int w, double x) {
    double pm = 1.0, pc = bcast(dv, 0) - x;
    int prev = pc < 0.0 ? 1 : 0;
    int cnt = prev;
    const int w1 = w < 64 ? w : 64;
    int i = 1;
    for (; i + 3 < w1; i += 4) {
#pragma unroll
        for (int u = 0; u < 4; u++) sturm_step(bcast(dv, i + u), bcast(b2v, i + u - 1), x, pm, pc, prev, cnt);
        sturm_rescale(pm, pc);
    }
    for (; i < w1; i++) sturm_step(bcast(dv, i), bcast(b2v, i - 1), x, pm, pc, prev, cnt);
    if (w > 64) {
        sturm_rescale(pm, pc);
        sturm_step(bcast(dv2, 0), bcast(b2v, 63), x, pm, pc, prev, cnt);
        i = 65;
        for (; i + 3 < w; i += 4) {
#pragma unroll
            for (int u = 0; u < 4; u++)
                sturm_step(bcast(dv2, i + u - 64), bcast(b2v2, i + u - 65), x, pm, pc, prev, cnt);
            sturm_rescale(pm, pc);
        }
        for (; i < w; i++) sturm_step(bcast(dv2, i - 64), bcast(b2v2, i - 65), x, pm, pc, prev, cnt);
    }
    return cnt;
}

// grid (ceil(w / kPer), problems); lam_out (optional): descending eigenvalues of problem b at
// lam_out + b * lam_stride, or with lam_prob >= 0 those of problem lam_prob alone at lam_out.  The
// ascending ones go to the record.
__global__ __launch_bounds__(ET) void k_eigvals(double* __restrict__ triall, int w, double* __restrict__ lam_out,
                                                int64_t lam_stride, int lam_prob) {
    double* tri = triall + (int64_t)blockIdx.y * kTriStride;
    const int tid = threadIdx.x, lane = tid & 63;
    // exact power-of-two scaling: |bounds| <= 1 afterwards
    int ex;
    frexp(fmax(fabs(tri[OFF_BND]), fabs(tri[OFF_BND + 1])), &ex);
    const double dv = lane < w ? ldexp(tri[OFF_D + lane], -ex) : 0.0;
    const double b2v = lane < w ? ldexp(tri[OFF_B2 + lane], -2 * ex) : 0.0;
    const double dv2 = lane + 64 < w ? ldexp(tri[OFF_D + 64 + lane], -ex) : 0.0;
    const double b2v2 = lane + 64 < w ? ldexp(tri[OFF_B2 + 64 + lane], -2 * ex) : 0.0;
    const int k = blockIdx.x * kPer + (tid >> 6);          // ascending index
    double a = ldexp(tri[OFF_BND], -ex), bb = ldexp(tri[OFF_BND + 1], -ex);
    for (int round = 0; round < kRounds; round++) {
        const double x = a + (bb - a) * (double)(lane + 1) / 65.0;
        const int c = sturm_count(dv, dv2, b2v, b2v2, w, x);
        const unsigned long long m = __ballot(c > k);
        const int first = m ? __builtin_ctzll(m) : 64;     // first section point above eigenvalue k
        const double xa = first == 0 ? a : a + (bb - a) * (double)first / 65.0;
        const double xb = first == 64 ? bb : a + (bb - a) * (double)(first + 1) / 65.0;
        a = xa;
        bb = xb;
    }
    a = ldexp(a, ex);
    bb = ldexp(bb, ex);
    if (k < w && lane == 0) {
        const double lam = 0.5 * (a + bb);
        tri[OFF_LAM + k] = lam;
        if (lam_out && (lam_prob < 0 || (int)blockIdx.y == lam_prob))
            lam_out[(lam_prob < 0 ? (int64_t)blockIdx.y * lam_stride : 0) + (w - 1 - k)] = lam;
    }
}

// ------------------------------------------------------------------------------------------
// 3. eigenvectors

struct VecLds {
    double ph[4 * kW];
    double dg[kW], b[kW], b2[kW], lam[kW], tau[kW];
    double X[kW * kW];        // eigenvectors of T, ascending index k at X + k * kW
    alignas(16) double dm[kW * kW];   // backward pivots of the twisted factorisations; then staging
    double bnd[2];
};

constexpr int kVecPer = ET / 64;   // eigenvectors per workgroup, one wave each

// x / y from the hardware reciprocal refined by two Newton steps (a few ulp; the twisted
// factorisation only needs pivots to working accuracy)
__device__ __forceinline__ double fdiv(double x, double y) {
    double r = __builtin_amdgcn_rcp(y);
    r = fma(r, fma(-y, r, 1.0), r);
    r = fma(r, fma(-y, r, 1.0), r);
    return x * r;
}

// grid ceil(w / kVecPer): workgroup g returns the eigenvectors of ascending indices
// [g kVecPer, g kVecPer + kVecPer) as columns w - 1 - k of E (descending order).  Clusters
// reaching across the slice are recomputed whole (the same arithmetic in every workgroup).
__global__ __launch_bounds__(ET) void k_eigvecs(const double* __restrict__ tri, int w, double* __restrict__ E) {
    __shared__ VecLds L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < w; i += ET) {
        L.dg[i] = tri[OFF_D + i];
        L.b[i] = tri[OFF_B + i];
        L.b2[i] = tri[OFF_B2 + i];
        L.lam[i] = tri[OFF_LAM + i];
        L.tau[i] = tri[OFF_TAU + i];
#pragma unroll
        for (int p = 0; p < 4; p++) L.ph[p * kW + i] = tri[OFF_PH + p * kW + i];
    }
    if (tid < 2) L.bnd[tid] = tri[OFF_BND + tid];
    __syncthreads();

    const double tnorm = fmax(fabs(L.bnd[0]), fabs(L.bnd[1])) + 1e-300;
    const double ctol = 1e-10 * tnorm;
    const int k0 = blockIdx.x * kVecPer, k1 = min(k0 + kVecPer, w);
    int c0 = k0, c1 = k1;
    while (c0 > 0 && L.lam[c0] - L.lam[c0 - 1] <= ctol) c0--;
    while (c1 < w && L.lam[c1] - L.lam[c1 - 1] <= ctol) c1++;

    // twisted factorisation of T - mu for each eigenvalue mu in [c0, c1): forward pivots
    // dp_0 = d_0 - mu, dp_i = d_i - mu - b_{i-1}^2 / dp_{i-1} and backward pivots
    // dm_{w-1} = d_{w-1} - mu, dm_i = d_i - mu - b_i^2 / dm_{i+1} (the two recurrences
    // interleaved); twist r with the least |gamma_r| = |dp_r + dm_r - (d_r - mu)|; x_r = 1,
    // x_{i+1} = -b_i x_i / dm_{i+1} below r and x_{i-1} = -b_{i-1} x_i / dp_{i-1} above.
    const double tiny = 1e-300 + 2.220446049250313e-16 * tnorm * 1e-3;
    for (int k = c0 + tid; k < c1; k += ET) {
        const double mu = L.lam[k];
        double* x = L.X + k * kW;          // forward pivots first, the vector at the end
        double* dm = L.dm + k * kW;
        double fp = L.dg[0] - mu, bp = L.dg[w - 1] - mu;
        if (fabs(fp) < tiny) fp = -tiny;
        if (fabs(bp) < tiny) bp = -tiny;
        x[0] = fp;
        dm[w - 1] = bp;
        for (int i = 1; i < w; i++) {
            const int ib = w - 1 - i;
            double f = (L.dg[i] - mu) - fdiv(L.b2[i - 1], fp);
            double g = (L.dg[ib] - mu) - fdiv(L.b2[ib], bp);
            if (fabs(f) < tiny) f = -tiny;
            if (fabs(g) < tiny) g = -tiny;
            x[i] = f;
            dm[ib] = g;
            fp = f;
            bp = g;
        }
        int r = w - 1;
        double best = fabs(x[w - 1]);
        for (int i = w - 2; i >= 0; i--) {
            const double gam = fabs(x[i] + dm[i] - (L.dg[i] - mu));
            if (gam < best) { best = gam; r = i; }
        }
        // both propagations from r at once: downward writes x[i > r], upward reads the
        // forward pivots x[i < r] before overwriting them
        double xd = 1.0, xu = 1.0, nrm = 1.0;
        const int steps = max(w - 1 - r, r);
        for (int t = 1; t <= steps; t++) {
            const int id = r + t, iu = r - t;
            if (id < w) {
                xd = -fdiv(L.b[id - 1] * xd, dm[id]);
                x[id] = xd;
                nrm += xd * xd;
            }
            if (iu >= 0) {
                xu = -fdiv(L.b[iu] * xu, x[iu]);
                x[iu] = xu;
                nrm += xu * xu;
            }
        }
        x[r] = 1.0;
        nrm = 1.0 / sqrt(nrm);
        for (int i = 0; i < w; i++) x[i] *= nrm;
    }
    __syncthreads();
    // modified Gram-Schmidt inside each cluster, ascending order (one wave)
    if (tid < 64) {
        int cs = c0;
        for (int k = c0 + 1; k <= c1; k++) {
            if (k < c1 && L.lam[k] - L.lam[k - 1] <= ctol) continue;
            for (int a = cs + 1; a < k; a++) {
                double* xa = L.X + a * kW;
                for (int bq = cs; bq < a; bq++) {
                    const double* xb = L.X + bq * kW;
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
            cs = k;
        }
    }
    __syncthreads();
    // back-transformation y = H_0 ... H_{w-3} D x: one wave per eigenvector, lane i holding rows
    // i and i + 64.  The reflectors come from the record (written by another workgroup) in chunks
    // of kChunk steps, loaded by the whole workgroup into LDS (the backward pivots' space, dead
    // by now) with many loads in flight, then applied from LDS.
    const int k = k0 + wave;
    const bool act = k < k1;                               // uniform per wave
    const int i = lane, i2 = lane + 64;
    Q4 y{0, 0, 0, 0}, y2{0, 0, 0, 0};
    if (act && i < w) y = qscale(ldq<kW>(L.ph, i), L.X[k * kW + i]);
    if (act && i2 < w) y2 = qscale(ldq<kW>(L.ph, i2), L.X[k * kW + i2]);
    const double* refl = tri + OFF_REFL;
    constexpr int kChunk = 16;                             // kChunk x kW entries fit in L.dm
    static_assert(4 * kChunk * kW <= kW * kW, "staging area");
    double* stage = L.dm;
    for (int jhi = w - 3; jhi >= 0; jhi -= kChunk) {
        const int jlo = jhi - kChunk + 1 > 0 ? jhi - kChunk + 1 : 0;
        const int n = (jhi - jlo + 1) * w;                 // entries (step jhi - t, row) at t * w + row
        __syncthreads();                                   // the previous chunk is consumed
        for (int base = tid; base < n; base += 4 * ET) {
            Q4 t[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int e = base + u * ET;
                const int jj = jhi - e / w, row = e % w;
                t[u] = (e < n && row > jj) ? ldq<kPacked>(refl, row * (row + 1) / 2 + jj) : Q4{0, 0, 0, 0};
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int e = base + u * ET;
                if (e < n) sti(stage, (e / w) * kW + e % w, t[u]);
            }
        }
        __syncthreads();
        if (act) {
            for (int j = jhi; j >= jlo; j--) {
                const int o = (jhi - j) * kW;
                const Q4 v = i < w ? ldi(stage, o + i) : Q4{0, 0, 0, 0};
                const Q4 v2 = i2 < w ? ldi(stage, o + i2) : Q4{0, 0, 0, 0};
                const double tj = L.tau[j];
                Q4 s = qfma(qmul(qconj(v), y), qconj(v2), y2);
                s.w = wave_total(s.w); s.x = wave_total(s.x); s.y = wave_total(s.y); s.z = wave_total(s.z);
                s = qscale(s, tj);
                y = qfms(y, v, s);
                y2 = qfms(y2, v2, s);
            }
        }
    }
    if (!act) return;
    const int64_t gps = (int64_t)w * w;
    const int col = w - 1 - k;
    if (i < w) {
        const int64_t o = (int64_t)i * w + col;
        E[o] = y.w; E[gps + o] = y.x; E[2 * gps + o] = y.y; E[3 * gps + o] = y.z;
    }
    if (i2 < w) {
        const int64_t o = (int64_t)i2 * w + col;
        E[o] = y2.w; E[gps + o] = y2.x; E[2 * gps + o] = y2.y; E[3 * gps + o] = y2.z;
    }
}

// ------------------------------------------------------------------------------------------
// Gram, left vectors, estimates

// G = X^H X for a small square X (w x w FP64 planes), full Hermitian storage: one 16 x 16 tile
// of G per workgroup, the two column strips of X staged in LDS.
__global__ __launch_bounds__(256) void k_gram_small(const double* __restrict__ X, int w, double* __restrict__ G) {
    __shared__ double sa[4 * kW * 16], sb[4 * kW * 16];   // [p][i][col]
    const int64_t ps = (int64_t)w * w;
    const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
    const int tid = threadIdx.x;
    const int n = w * 16;
    for (int base = 0; base < n; base += 4 * 256) {
        double va[4][4], vb[4][4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = min(base + u * 256 + tid, n - 1);
            const int i = e >> 4, cc = e & 15;
#pragma unroll
            for (int p = 0; p < 4; p++) {
                va[u][p] = X[p * ps + (int64_t)i * w + min(a0 + cc, w - 1)];
                vb[u][p] = X[p * ps + (int64_t)i * w + min(b0 + cc, w - 1)];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = base + u * 256 + tid;
            if (e >= n) continue;
            const int cc = e & 15;
#pragma unroll
            for (int p = 0; p < 4; p++) {
                sa[p * kW * 16 + e] = a0 + cc < w ? va[u][p] : 0.0;
                sb[p * kW * 16 + e] = b0 + cc < w ? vb[u][p] : 0.0;
            }
        }
    }
    __syncthreads();
    const int aa = tid >> 4, bq = tid & 15;
    const int a = a0 + aa, b = b0 + bq;
    Q4 s{0, 0, 0, 0};
    for (int i = 0; i < w; i++)
        s = qadd(s, qmul(qconj(ldq<kW * 16>(sa, i * 16 + aa)), ldq<kW * 16>(sb, i * 16 + bq)));
    if (a < w && b < w) {
        if (a == b) s.x = s.y = s.z = 0.0;
        const int64_t e = (int64_t)a * w + b;
        G[e] = s.w; G[ps + e] = s.x; G[2 * ps + e] = s.y; G[3 * ps + e] = s.z;
    }
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

// From the eigendecomposition G = E diag(lam) E^H of a view's Gram Y^H Y (lam descending):
// S_j = sqrt(max(lam_j, 0)) and W = E_k diag(1 / S) (w x k, ld k; zero columns where S_j is at
// or below kDegenerate S_0, flagged in *degen).
__global__ __launch_bounds__(256) void k_svals(const double* __restrict__ lam, const double* __restrict__ E,
                                               int64_t lde, int w, int k, double* __restrict__ S,
                                               double* __restrict__ Wk, const double* __restrict__ nA2,
                                               double* __restrict__ est, int* degen) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double s0 = sqrt(fmax(lam[0], 0.0));
    if (e < k) S[e] = sqrt(fmax(lam[e], 0.0));
    if (degen && e == 0) {
        // nonzero: re-orthonormalise the factor Y W (a steep spectrum, or degenerate columns)
        int any = !(sqrt(fmax(lam[k - 1], 0.0)) >= 0.015625 * s0);
        for (int j = 0; j < k; j++) any |= !(sqrt(fmax(lam[j], 0.0)) > kDegenerate * s0);
        *degen = any;
    }
    if (est && e == 0) {
        // the estimate of this pass, sqrt(max(0, ||A||^2 - sum_{j<k} S_j^2) / ||A||^2)
        double top = 0.0;
        for (int j = 0; j < k; j++) {
            const double sj = sqrt(fmax(lam[j], 0.0));
            top += sj * sj;
        }
        const double a = *nA2, r = a - top;
        *est = a > 0.0 ? sqrt((r > 0.0 ? r : 0.0) / a) : 0.0;
    }
    if (!E || e >= (int64_t)w * k) return;
    const int i = (int)(e / k), j = (int)(e % k);
    const double sj = sqrt(fmax(lam[j], 0.0));
    const double inv = sj > kDegenerate * s0 ? 1.0 / sj : 0.0;
    const int64_t eps = (int64_t)w * lde, wps = (int64_t)w * k, src = (int64_t)i * lde + j;
#pragma unroll
    for (int p = 0; p < 4; p++) Wk[p * wps + e] = E[p * eps + src] * inv;
}

// Degenerate columns of a factor Y E_k S^{-1}: a fixed pseudo-random vector (any vector with a
// component outside the kept columns will do; the re-orthonormalisation that follows makes it a
// unit vector orthogonal to them).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // the 32-bit finaliser of MurmurHash3 (Appleby)
    x ^= x >> 16; x *= 0x85ebca6bu; x ^= x >> 13; x *= 0xc2b2ae35u; x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(256) void k_fill_degenerate(float* __restrict__ X, int64_t rows, int k, int64_t ldx,
                                                         int64_t xps, const double* __restrict__ S,
                                                         const int* __restrict__ flag) {
    if (*flag == 0) return;
    const double s0 = S[0];
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * k; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / k;
        const int j = (int)(e - i * k);
        if (S[j] > kDegenerate * s0) continue;
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const uint32_t h = mix32((uint32_t)(e * 4 + p) ^ mix32((uint32_t)(e >> 30) + 0x9e3779b9u));
            X[p * xps + i * ldx + j] = (float)((double)h * (1.0 / 2147483648.0) - 1.0);
        }
    }
}

// e_b = sqrt(max(0, ||A||^2 - sum of the k largest max(lambda, 0)) / ||A||^2) per problem b.
__global__ void k_estimate_batch(const double* __restrict__ triall, int nprob, int w, int k,
                                 const double* __restrict__ nA2, double* __restrict__ e) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    const double* lam = triall + (int64_t)b * kTriStride + OFF_LAM;
    double top = 0.0;
    for (int j = 0; j < k && j < w; j++) top += fmax(lam[w - 1 - j], 0.0);
    const double a = *nA2;
    const double r = a - top;
    e[b] = a > 0.0 ? sqrt((r > 0.0 ? r : 0.0) / a) : 0.0;
}

}  // namespace

int heig_max() { return kW; }

size_t heig_work_doubles(int64_t nprob) { return (size_t)nprob * kTriStride; }

hipError_t heig_launch(const double* G, int64_t w, double* lam, double* E, double* work, hipStream_t st) {
    if (w < 1 || w > kW) return hipErrorInvalidValue;
    if (w <= 64)
        hipLaunchKernelGGL((k_tridiag<16, 4, 1024>), dim3(1), dim3(1024), 0, st, G, (int64_t)0, (int)w, work, E ? 1 : 0);
    else
        hipLaunchKernelGGL((k_tridiag<8, 12, 768>), dim3(1), dim3(768), 0, st, G, (int64_t)0, (int)w, work, E ? 1 : 0);
    const unsigned slices = (unsigned)((w + kPer - 1) / kPer);
    hipLaunchKernelGGL(k_eigvals, dim3(slices, 1), dim3(ET), 0, st, work, (int)w, lam, (int64_t)0, -1);
    if (E)
        hipLaunchKernelGGL(k_eigvecs, dim3((unsigned)((w + kVecPer - 1) / kVecPer)), dim3(ET), 0, st,
                           (const double*)work, (int)w, E);
    return hipGetLastError();
}

hipError_t estimate_batch_launch(const double* G, int64_t gstride, int64_t w, int nprob, int k, const double* nA2,
                                 double* e, double* work, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    if (w < 1 || w > kW) return hipErrorInvalidValue;
    if (w <= 64)
        hipLaunchKernelGGL((k_tridiag<16, 4, 1024>), dim3((unsigned)nprob), dim3(1024), 0, st, G, gstride, (int)w, work, 0);
    else
        hipLaunchKernelGGL((k_tridiag<8, 12, 768>), dim3((unsigned)nprob), dim3(768), 0, st, G, gstride, (int)w, work, 0);
    const unsigned slices = (unsigned)((w + kPer - 1) / kPer);
    hipLaunchKernelGGL(k_eigvals, dim3(slices, (unsigned)nprob), dim3(ET), 0, st, work, (int)w, (double*)nullptr,
                       (int64_t)0, -1);
    hipLaunchKernelGGL(k_estimate_batch, dim3((unsigned)((nprob + 63) / 64)), dim3(64), 0, st, (const double*)work,
                       nprob, (int)w, k, nA2, e);
    return hipGetLastError();
}

hipError_t heig_with_estimates_launch(const double* G, int64_t gstride, int64_t w, int nest, int k, const double* nA2,
                                      double* e, double* lam, double* E, double* work, hipStream_t st) {
    if (w < 1 || w > kW || nest < 0) return hipErrorInvalidValue;
    const unsigned np = (unsigned)nest + 1;
    if (w <= 64)
        hipLaunchKernelGGL((k_tridiag<16, 4, 1024>), dim3(np), dim3(1024), 0, st, G, gstride, (int)w, work, 1);
    else
        hipLaunchKernelGGL((k_tridiag<8, 12, 768>), dim3(np), dim3(768), 0, st, G, gstride, (int)w, work, 1);
    const unsigned slices = (unsigned)((w + kPer - 1) / kPer);
    hipLaunchKernelGGL(k_eigvals, dim3(slices, np), dim3(ET), 0, st, work, (int)w, lam, (int64_t)0, nest);
    if (E)
        hipLaunchKernelGGL(k_eigvecs, dim3((unsigned)((w + kVecPer - 1) / kVecPer)), dim3(ET), 0, st,
                           (const double*)(work + (size_t)nest * kTriStride), (int)w, E);
    if (nest > 0)
        hipLaunchKernelGGL(k_estimate_batch, dim3((unsigned)((nest + 63) / 64)), dim3(64), 0, st, (const double*)work,
                           nest, (int)w, k, nA2, e);
    return hipGetLastError();
}

// QSVD of a small square X through the eigendecomposition of X^H X: S descending, V right
// vectors, U left vectors (U, V may be null).  work: qsvd_gram_work_doubles(w).
hipError_t qsvd_gram_launch(const double* X, int64_t w, double* U, double* S, double* V, double* work,
                            hipStream_t st) {
    if (w < 1 || w > kW) return hipErrorInvalidValue;
    const int64_t ps = w * w;
    double* G = work;
    double* lam = G + 4 * ps;
    double* Vt = lam + w;
    double* hw = Vt + 4 * ps;
    double* Vout = V ? V : Vt;
    const unsigned tiles = (unsigned)((w + 15) / 16);
    hipLaunchKernelGGL(k_gram_small, dim3(tiles, tiles), dim3(256), 0, st, X, (int)w, G);
    hipError_t e = heig_launch(G, w, lam, (U || V) ? Vout : nullptr, hw, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_left_vectors, dim3((unsigned)((ps + 255) / 256)), dim3(256), 0, st, X, (int)w, lam,
                       Vout, S, U);
    return hipGetLastError();
}

hipError_t svals_launch(const double* lam, const double* E, int64_t lde, int64_t w, int k, double* S, double* Wk,
                        hipStream_t st, const double* nA2, double* est, int* degen) {
    const int64_t n = std::max<int64_t>(w * k, k);
    hipLaunchKernelGGL(k_svals, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lam, E, lde, (int)w, k, S, Wk,
                       nA2, est, degen);
    return hipGetLastError();
}

hipError_t fill_degenerate_launch(float* X, int64_t rows, int k, int64_t ldx, int64_t xps, const double* S,
                                  const int* flag, hipStream_t st) {
    if (rows < 1 || k < 1) return hipSuccess;
    int64_t g = (rows * k + 255) / 256;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_fill_degenerate, dim3((unsigned)g), dim3(256), 0, st, X, rows, k, ldx, xps, S, flag);
    return hipGetLastError();
}

size_t qsvd_gram_work_doubles(int64_t w) { return (size_t)(8 * w * w + w) + heig_work_doubles(1); }

}  // namespace qlra_impl
