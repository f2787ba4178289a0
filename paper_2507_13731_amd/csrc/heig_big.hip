// Hermitian quaternion eigendecomposition for orders above the single-workgroup solver (the
// Gram of a wide block-Krylov final view, Alg. 4: W = (number of stacked blocks) x l columns).
// Same method as the small solver (Householder tridiagonalisation with quaternion reflectors
// made real by a diagonal of phases, Sturm multisection, twisted factorisations, the
// back-transformation), spread over many workgroups:
//  - tridiagonalisation: the working matrix stays in global memory (L2 resident); each step is
//    two launches over row blocks of 16 rows: (a) every block forms the reflector v from column
//    j (redundantly), its rows' p = tau G v and a share of K = tau/2 v^H p; (b) every block
//    forms q = p - K v and updates its rows, G <- G - v q^H - q v^H.
//  - eigenvalues: 16 lanes per eigenvalue, the tridiagonal in LDS.
//  - eigenvectors: only the wanted ones (the largest), one wave each, the reflectors read from
//    the record.
#include <algorithm>

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
__device__ __forceinline__ Q4 qadd(Q4 a, Q4 b) { return Q4{a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ Q4 qsub(Q4 a, Q4 b) { return Q4{a.w - b.w, a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Q4 qscale(Q4 a, double s) { return Q4{a.w * s, a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double qn2(Q4 a) { return a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z; }
__device__ __forceinline__ double qdot(Q4 a, Q4 b) { return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ Q4 ld(const double* p, int64_t ps, int64_t i) {
    return Q4{p[i], p[ps + i], p[2 * ps + i], p[3 * ps + i]};
}
__device__ __forceinline__ void st(double* p, int64_t ps, int64_t i, Q4 v) {
    p[i] = v.w; p[ps + i] = v.x; p[2 * ps + i] = v.y; p[3 * ps + i] = v.z;
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    return v;
}
__device__ __forceinline__ double bcast(double v, int i) {
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffll), i);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), i);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_total(double v) {
    v = row16_sum(v);
    return bcast(v, 0) + bcast(v, 16) + bcast(v, 32) + bcast(v, 48);
}
// sum over the workgroup (256 threads); every thread receives it
__device__ double block_total(double v, double* red) {
    v = wave_total(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

constexpr int RB = 16;        // rows per workgroup in the tridiagonalisation (16 lanes each)
constexpr int BT = 256;

// Record for order W (doubles): the working matrix, then the results.
struct BigRec {
    int64_t W;
    double* Gw;     // 4 W^2, full storage
    double* d;      // W
    double* b;      // W
    double* b2;     // W
    double* tau;    // W
    double* ph;     // 4 W
    double* bnd;    // 2 (+ pad)
    double* lam;    // W, ascending
    double* refl;   // 4 W (W + 1) / 2, (i, j) at i (i + 1) / 2 + j
    double* P;      // 4 W: p of the current step
    double* KP;     // ceil(W / RB) shares of v^H p
    double* X;      // W x nvec eigenvectors of T (vector t at X + t W)
    double* DM;     // W x nvec backward pivots
};

__host__ __device__ inline BigRec big_rec(double* base, int64_t W, int64_t nvec) {
    BigRec r;
    r.W = W;
    double* p = base;
    r.Gw = p; p += 4 * W * W;
    r.d = p; p += W;
    r.b = p; p += W;
    r.b2 = p; p += W;
    r.tau = p; p += W;
    r.ph = p; p += 4 * W;
    r.bnd = p; p += 8;
    r.lam = p; p += W;
    r.refl = p; p += 4 * (W * (W + 1) / 2);
    r.P = p; p += 4 * W;
    r.KP = p; p += (W + RB - 1) / RB;
    r.X = p; p += W * nvec;
    r.DM = p; p += W * nvec;
    return r;
}
__host__ __device__ inline int64_t big_rec_doubles(int64_t W, int64_t nvec) {
    return 4 * W * W + 9 * W + 8 + 4 * (W * (W + 1) / 2) + 4 * W + (W + RB - 1) / RB + 2 * W * nvec;
}

__global__ __launch_bounds__(BT) void k_big_copy(const double* __restrict__ G, double* __restrict__ Gw, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (e < n) Gw[e] = G[e];
}

// step j, part (a): reflector from column j (every block), p for this block's rows, K share
__global__ __launch_bounds__(BT) void k_big_a(double* __restrict__ base, int W, int nvec, int j) {
    __shared__ double vs[4 * 1024];   // v, W <= 1024
    __shared__ double red[4];
    BigRec R = big_rec(base, W, nvec);
    const int64_t ps = (int64_t)W * W;
    const int tid = threadIdx.x;
    double part = 0.0;
    for (int r = j + 1 + tid; r < W; r += BT) part += qn2(ld(R.Gw, ps, (int64_t)r * W + j));
    const double alpha = sqrt(block_total(part, red));
    const Q4 x1 = ld(R.Gw, ps, (int64_t)(j + 1) * W + j);
    const double ax1 = sqrt(qn2(x1));
    const Q4 phi = ax1 > 0.0 ? qscale(x1, 1.0 / ax1) : Q4{1, 0, 0, 0};
    const double tau = alpha > 0.0 ? 1.0 / (alpha * (alpha + ax1)) : 0.0;
    for (int r = tid; r < W; r += BT) {
        Q4 v{0, 0, 0, 0};
        if (r > j) {
            v = ld(R.Gw, ps, (int64_t)r * W + j);        // G(r, j), the column below the diagonal
            if (r == j + 1) v = qadd(v, qscale(phi, alpha));
            if (blockIdx.x == 0) st(R.refl, W * (W + 1) / 2, (int64_t)r * (r + 1) / 2 + j, v);
        }
        vs[r] = v.w; vs[1024 + r] = v.x; vs[2048 + r] = v.y; vs[3072 + r] = v.z;
    }
    if (blockIdx.x == 0 && tid == 0) {
        R.tau[j] = tau;
        const Q4 sj = qscale(phi, -alpha);               // H x = -alpha phi e_1
        R.ph[j] = sj.w; R.ph[W + j] = sj.x; R.ph[2 * W + j] = sj.y; R.ph[3 * W + j] = sj.z;   // s_j, for now
    }
    __syncthreads();
    // p_r = tau sum_{c > j} G(r, c) v_c, 16 lanes per row
    const int rl = tid >> 4, s = tid & 15;
    const int r = blockIdx.x * RB + rl;
    Q4 acc{0, 0, 0, 0};
    if (r > j && r < W)
        for (int c = j + 1 + s; c < W; c += 16)
            acc = qadd(acc, qmul(ld(R.Gw, ps, (int64_t)r * W + c), Q4{vs[c], vs[1024 + c], vs[2048 + c], vs[3072 + c]}));
    acc.w = row16_sum(acc.w); acc.x = row16_sum(acc.x); acc.y = row16_sum(acc.y); acc.z = row16_sum(acc.z);
    const Q4 p = qscale(acc, tau);
    double kp = 0.0;
    if (s == 0 && r < W) {
        st(R.P, W, r, p);
        if (r > j) kp = qdot(Q4{vs[r], vs[1024 + r], vs[2048 + r], vs[3072 + r]}, p);
    }
    const double kt = block_total(kp, red);
    if (tid == 0) R.KP[blockIdx.x] = kt;
}

// step j, part (b): q = p - K v, update this block's rows
__global__ __launch_bounds__(BT) void k_big_b(double* __restrict__ base, int W, int nvec, int j) {
    __shared__ double vs[4 * 1024], qs[4 * 1024];
    __shared__ double red[4];
    BigRec R = big_rec(base, W, nvec);
    const int64_t ps = (int64_t)W * W;
    const int tid = threadIdx.x;
    const int nb = (W + RB - 1) / RB;
    double part = 0.0;
    for (int i = tid; i < nb; i += BT) part += R.KP[i];
    const double tau = R.tau[j];
    const double K = 0.5 * tau * block_total(part, red);
    const int64_t pps = (int64_t)W * (W + 1) / 2;
    for (int c = tid; c < W; c += BT) {
        Q4 v{0, 0, 0, 0}, q{0, 0, 0, 0};
        if (c > j) {
            v = ld(R.refl, pps, (int64_t)c * (c + 1) / 2 + j);
            q = qsub(ld(R.P, W, c), qscale(v, K));
        }
        vs[c] = v.w; vs[1024 + c] = v.x; vs[2048 + c] = v.y; vs[3072 + c] = v.z;
        qs[c] = q.w; qs[1024 + c] = q.x; qs[2048 + c] = q.y; qs[3072 + c] = q.z;
    }
    __syncthreads();
    const int rl = tid >> 4, s = tid & 15;
    const int r = blockIdx.x * RB + rl;
    if (r <= j || r >= W) return;
    const Q4 vr{vs[r], vs[1024 + r], vs[2048 + r], vs[3072 + r]};
    const Q4 qr{qs[r], qs[1024 + r], qs[2048 + r], qs[3072 + r]};
    for (int c = j + 1 + s; c < W; c += 16) {
        const Q4 vc{vs[c], vs[1024 + c], vs[2048 + c], vs[3072 + c]};
        const Q4 qc{qs[c], qs[1024 + c], qs[2048 + c], qs[3072 + c]};
        const int64_t e = (int64_t)r * W + c;
        Q4 t = qsub(qsub(ld(R.Gw, ps, e), qmul(vr, qconj(qc))), qmul(qr, qconj(vc)));
        if (r == c) t.x = t.y = t.z = 0.0;
        st(R.Gw, ps, e, t);
    }
}

// diagonal, real subdiagonal b_j = |s_j|, phases ph_{j+1} = s_j ph_j / |s_j|, bounds
__global__ void k_big_fin(double* __restrict__ base, int W, int nvec) {
    if (threadIdx.x != 0) return;
    BigRec R = big_rec(base, W, nvec);
    const int64_t ps = (int64_t)W * W;
    if (W >= 2) {
        const Q4 sl = ld(R.Gw, ps, (int64_t)(W - 1) * W + (W - 2));
        R.ph[W - 2] = sl.w; R.ph[W + W - 2] = sl.x; R.ph[2 * W + W - 2] = sl.y; R.ph[3 * W + W - 2] = sl.z;
        R.tau[W - 2] = 0.0;
    }
    R.tau[W - 1] = 0.0;
    Q4 pj{1, 0, 0, 0};
    double lo = 1e300, hi = -1e300, bl = 0.0;
    for (int i = 0; i < W; i++) {
        const double dd = R.Gw[(int64_t)i * W + i];
        R.d[i] = dd;
        double br = 0.0;
        Q4 sj{0, 0, 0, 0};
        if (i + 1 < W) sj = Q4{R.ph[i], R.ph[W + i], R.ph[2 * W + i], R.ph[3 * W + i]};
        R.ph[i] = pj.w; R.ph[W + i] = pj.x; R.ph[2 * W + i] = pj.y; R.ph[3 * W + i] = pj.z;
        if (i + 1 < W) {
            br = sqrt(qn2(sj));
            pj = br > 0.0 ? qscale(qmul(sj, pj), 1.0 / br) : Q4{1, 0, 0, 0};
        }
        R.b[i] = br;
        R.b2[i] = br * br;
        lo = fmin(lo, dd - bl - br);
        hi = fmax(hi, dd + bl + br);
        bl = br;
    }
    const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
    R.bnd[0] = lo - pad;
    R.bnd[1] = hi + pad;
}

// Sturm count with the (scaled) tridiagonal in LDS
__device__ int sturm_lds(const double* d, const double* b2, int W, double x) {
    double pm = 1.0, pc = d[0] - x;
    int prev = pc < 0.0 ? 1 : 0;
    int cnt = prev;
    for (int i = 1; i < W; i++) {
        const double pn = fma(d[i] - x, pc, -b2[i - 1] * pm);
        pm = pc;
        pc = pn;
        int neg = pn < 0.0;
        neg = pn == 0.0 ? prev : neg;
        cnt += neg ^ prev;
        prev = neg;
        if ((i & 3) == 0) {
            const double a = fmax(fabs(pc), fabs(pm));
            const double sc = a > 1e150 ? 1e-150 : (a < 1e-150 ? 1e150 : 1.0);
            pc *= sc;
            pm *= sc;
        }
    }
    return cnt;
}

// eigenvalues: grid ceil(W / 16), 16 lanes per eigenvalue, 17-section rounds; lam_out descending
__global__ __launch_bounds__(BT) void k_big_eigvals(double* __restrict__ base, int W, int nvec,
                                                    double* __restrict__ lam_out) {
    extern __shared__ double sh[];
    double* d = sh;
    double* b2 = sh + W;
    BigRec R = big_rec(base, W, nvec);
    const int tid = threadIdx.x, lane = tid & 63, s16 = tid & 15;
    int ex;
    frexp(fmax(fabs(R.bnd[0]), fabs(R.bnd[1])), &ex);
    for (int i = tid; i < W; i += BT) {
        d[i] = ldexp(R.d[i], -ex);
        b2[i] = ldexp(R.b2[i], -2 * ex);
    }
    __syncthreads();
    const int k = blockIdx.x * 16 + (tid >> 4);
    double a = ldexp(R.bnd[0], -ex), bb = ldexp(R.bnd[1], -ex);
    for (int round = 0; round < 14; round++) {
        const double x = a + (bb - a) * (double)(s16 + 1) / 17.0;
        const int c = sturm_lds(d, b2, W, x);
        const unsigned long long m = __ballot(c > k);
        const unsigned grp = (unsigned)((m >> (lane & ~15)) & 0xFFFFull);
        const int first = grp ? __builtin_ctz(grp) : 16;
        const double xa = first == 0 ? a : a + (bb - a) * (double)first / 17.0;
        const double xb = first == 16 ? bb : a + (bb - a) * (double)(first + 1) / 17.0;
        a = xa;
        bb = xb;
    }
    if (k < W && s16 == 0) {
        const double lam = ldexp(0.5 * (a + bb), ex);
        R.lam[k] = lam;
        if (lam_out) lam_out[W - 1 - k] = lam;
    }
}

__device__ __forceinline__ double fdiv(double x, double y) {
    double r = __builtin_amdgcn_rcp(y);
    r = fma(r, fma(-y, r, 1.0), r);
    r = fma(r, fma(-y, r, 1.0), r);
    return x * r;
}

// eigenvectors of T for the ascending indices [c0, W) (c0 = W - nvec extended down to the start
// of its cluster, computed on the host side of the launch by every block alike): twisted
// factorisations, one thread each
__global__ __launch_bounds__(BT) void k_big_twisted(double* __restrict__ base, int W, int nvec, int kfirst) {
    BigRec R = big_rec(base, W, nvec);
    const double tnorm = fmax(fabs(R.bnd[0]), fabs(R.bnd[1])) + 1e-300;
    const double tiny = 1e-300 + 2.220446049250313e-16 * tnorm * 1e-3;
    const int t = blockIdx.x * BT + threadIdx.x;     // vector slot
    const int k = kfirst + t;
    if (t >= nvec || k >= W) return;
    const double mu = R.lam[k];
    double* x = R.X + (int64_t)t * W;
    double* dm = R.DM + (int64_t)t * W;
    double fp = R.d[0] - mu, bp = R.d[W - 1] - mu;
    if (fabs(fp) < tiny) fp = -tiny;
    if (fabs(bp) < tiny) bp = -tiny;
    x[0] = fp;
    dm[W - 1] = bp;
    for (int i = 1; i < W; i++) {
        const int ib = W - 1 - i;
        double f = (R.d[i] - mu) - fdiv(R.b2[i - 1], fp);
        double g = (R.d[ib] - mu) - fdiv(R.b2[ib], bp);
        if (fabs(f) < tiny) f = -tiny;
        if (fabs(g) < tiny) g = -tiny;
        x[i] = f;
        dm[ib] = g;
        fp = f;
        bp = g;
    }
    int r = W - 1;
    double best = fabs(x[W - 1]);
    for (int i = W - 2; i >= 0; i--) {
        const double gam = fabs(x[i] + dm[i] - (R.d[i] - mu));
        if (gam < best) { best = gam; r = i; }
    }
    double xd = 1.0, xu = 1.0, nrm = 1.0;
    const int steps = max(W - 1 - r, r);
    for (int s = 1; s <= steps; s++) {
        const int id = r + s, iu = r - s;
        if (id < W) {
            xd = -fdiv(R.b[id - 1] * xd, dm[id]);
            x[id] = xd;
            nrm += xd * xd;
        }
        if (iu >= 0) {
            xu = -fdiv(R.b[iu] * xu, x[iu]);
            x[iu] = xu;
            nrm += xu * xu;
        }
    }
    x[r] = 1.0;
    nrm = 1.0 / sqrt(nrm);
    for (int i = 0; i < W; i++) x[i] *= nrm;
}

// modified Gram-Schmidt inside clusters of close eigenvalues among the computed vectors (one wave)
__global__ void k_big_mgs(double* __restrict__ base, int W, int nvec, int kfirst, int kcount) {
    BigRec R = big_rec(base, W, nvec);
    const int lane = threadIdx.x;
    const double tnorm = fmax(fabs(R.bnd[0]), fabs(R.bnd[1])) + 1e-300;
    const double ctol = 1e-10 * tnorm;
    int cs = 0;
    for (int t = 1; t <= kcount; t++) {
        if (t < kcount && R.lam[kfirst + t] - R.lam[kfirst + t - 1] <= ctol) continue;
        for (int a = cs + 1; a < t; a++) {
            double* xa = R.X + (int64_t)a * W;
            for (int bq = cs; bq < a; bq++) {
                const double* xb = R.X + (int64_t)bq * W;
                double dot = 0.0;
                for (int i = lane; i < W; i += 64) dot += xa[i] * xb[i];
                dot = wave_total(dot);
                for (int i = lane; i < W; i += 64) xa[i] -= dot * xb[i];
            }
            double nr2 = 0.0;
            for (int i = lane; i < W; i += 64) nr2 += xa[i] * xa[i];
            nr2 = wave_total(nr2);
            const double inv = nr2 > 0.0 ? 1.0 / sqrt(nr2) : 0.0;
            for (int i = lane; i < W; i += 64) xa[i] *= inv;
        }
        cs = t;
    }
}

// back-transformation y = H_0 ... H_{W-3} D x for the nout largest eigenvalues, one wave each,
// lane holding rows lane + 64 u; E (W x nout, ld nout) gets them in descending order
constexpr int kBigRows = 16;   // rows per lane: W <= 1024
__global__ __launch_bounds__(BT) void k_big_back(double* __restrict__ base, int W, int nvec, int kfirst, int nout,
                                                 double* __restrict__ E) {
    BigRec R = big_rec(base, W, nvec);
    const int lane = threadIdx.x & 63;
    const int o = blockIdx.x * (BT / 64) + (threadIdx.x >> 6);   // output column
    if (o >= nout) return;
    const int k = W - 1 - o;                                    // ascending index
    const double* xk = R.X + (int64_t)(k - kfirst) * W;
    const int64_t pps = (int64_t)W * (W + 1) / 2;
    Q4 y[kBigRows];
#pragma unroll
    for (int u = 0; u < kBigRows; u++) {
        const int i = lane + 64 * u;
        y[u] = i < W ? qscale(Q4{R.ph[i], R.ph[W + i], R.ph[2 * W + i], R.ph[3 * W + i]}, xk[i]) : Q4{0, 0, 0, 0};
    }
    for (int j = W - 3; j >= 0; j--) {
        const double tj = R.tau[j];
        if (tj == 0.0) continue;
        Q4 s{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < kBigRows; u++) {
            const int i = lane + 64 * u;
            if (64 * u < W && i > j && i < W)                    // the first test is uniform
                s = qadd(s, qmul(qconj(ld(R.refl, pps, (int64_t)i * (i + 1) / 2 + j)), y[u]));
        }
        s.w = wave_total(s.w); s.x = wave_total(s.x); s.y = wave_total(s.y); s.z = wave_total(s.z);
        s = qscale(s, tj);
#pragma unroll
        for (int u = 0; u < kBigRows; u++) {
            const int i = lane + 64 * u;
            if (64 * u < W && i > j && i < W) y[u] = qsub(y[u], qmul(ld(R.refl, pps, (int64_t)i * (i + 1) / 2 + j), s));
        }
    }
    const int64_t eps = (int64_t)W * nout;
#pragma unroll
    for (int u = 0; u < kBigRows; u++) {
        const int i = lane + 64 * u;
        if (i < W) st(E, eps, (int64_t)i * nout + o, y[u]);
    }
}

}  // namespace

int heig_big_max() { return 1024; }

size_t heig_big_work_doubles(int64_t W, int64_t nvec) { return (size_t)big_rec_doubles(W, nvec); }

// lam: W eigenvalues, descending.  E (optional): the nout eigenvectors of the largest
// eigenvalues as columns, descending (W x nout, ld nout).  nvec: vector slots of the record
// (>= nout plus the cluster extension; the caller passes W to be safe or nout + margin).
hipError_t heig_big_launch(const double* G, int64_t W, double* lam, double* E, int64_t nout, double* work,
                           int64_t nvec, hipStream_t st) {
    if (W < 1 || W > heig_big_max() || nout < 0 || nout > W || (E && nvec < nout)) return hipErrorInvalidValue;
    BigRec R = big_rec(work, W, nvec);
    const int64_t n = 4 * W * W;
    hipLaunchKernelGGL(k_big_copy, dim3((unsigned)((n + BT - 1) / BT)), dim3(BT), 0, st, G, R.Gw, n);
    const unsigned nb = (unsigned)((W + RB - 1) / RB);
    for (int j = 0; j + 2 < W; j++) {
        hipLaunchKernelGGL(k_big_a, dim3(nb), dim3(BT), 0, st, work, (int)W, (int)nvec, j);
        hipLaunchKernelGGL(k_big_b, dim3(nb), dim3(BT), 0, st, work, (int)W, (int)nvec, j);
    }
    hipLaunchKernelGGL(k_big_fin, dim3(1), dim3(64), 0, st, work, (int)W, (int)nvec);
    hipLaunchKernelGGL(k_big_eigvals, dim3((unsigned)((W + 15) / 16)), dim3(BT), (size_t)(2 * W * sizeof(double)), st,
                       work, (int)W, (int)nvec, lam);
    if (!E || nout == 0) return hipGetLastError();
    // vectors of ascending indices [W - nvec, W): the top nout plus room below for a cluster
    const int kfirst = (int)(W - nvec);
    hipLaunchKernelGGL(k_big_twisted, dim3((unsigned)((nvec + BT - 1) / BT)), dim3(BT), 0, st, work, (int)W,
                       (int)nvec, kfirst);
    hipLaunchKernelGGL(k_big_mgs, dim3(1), dim3(64), 0, st, work, (int)W, (int)nvec, kfirst, (int)nvec);
    hipLaunchKernelGGL(k_big_back, dim3((unsigned)((nout + 3) / 4)), dim3(BT), 0, st, work, (int)W, (int)nvec, kfirst,
                       (int)nout, E);
    return hipGetLastError();
}

}  // namespace qlra_impl
