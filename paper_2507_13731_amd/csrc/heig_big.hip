// Hermitian quaternion eigendecomposition for orders above the single-workgroup solver (the
// Gram of a wide block-Krylov final view, Alg. 4: W = (number of stacked blocks) x l columns,
// and the Grams of views wider than that solver for the per-pass estimates).  Same method as the
// small solver (Householder tridiagonalisation with quaternion reflectors made real by a
// diagonal of phases, Sturm multisection, twisted factorisations, the back-transformation),
// spread over many workgroups:
//  - tridiagonalisation: the working matrix stays in global memory (L2 / MALL resident), one
//    launch per reflector over row blocks of 4 rows (one wave per row).  Launch j applies the
//    update of reflector j, G <- G - v q^H - q v^H with q = p - K v, to its rows and, in the same
//    sweep, forms p = tau' G v' of the next reflector v' for them.  Every block forms v' itself
//    from column j+1 after the update, which it computes from a copy of that column taken by the
//    previous launch (so no block reads rows another block is writing); p, the shares of
//    v'^H p and the column copies are double-buffered between launches.  Several problems of one
//    order go in one launch (grid y), so the estimates of all views cost one launch sequence.
//  - eigenvalues: 16 lanes per eigenvalue, the tridiagonal in LDS.
//  - eigenvectors: only the wanted ones (the largest), by twisted factorisations of the
//    tridiagonal, then the back-transformation with the reflectors in blocks of four (compact
//    WY form: one cross-lane sum per block instead of one per reflector), one workgroup per
//    vector with its rows split over its four waves.
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
// sum over a workgroup of NW waves (red: NW doubles of LDS); every thread receives it
template <int NW = 4>
__device__ double block_total(double v, double* red) {
    v = wave_total(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = red[0];
#pragma unroll
    for (int i = 1; i < NW; i++) t += red[i];
    return t;
}

constexpr int SRB = 4;        // rows per workgroup in the tridiagonalisation (one wave each)
constexpr int SBT = 64 * SRB; // threads of the tridiagonalisation's workgroups
constexpr int BT = 256;

__host__ __device__ inline int64_t step_blocks(int64_t W) { return (W + SRB - 1) / SRB; }

// packed strictly-lower storage of the reflectors by columns: column j (rows j+1 .. W-1) starts
// at j (2 W - j - 1) / 2, so that a reflector is one contiguous run (coalesced reads)
__host__ __device__ inline int64_t refl_at(int64_t W, int64_t i, int64_t j) { return j * (2 * W - j - 1) / 2 + (i - j - 1); }

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
    double* refl;   // 4 W (W + 1) / 2, reflector j's entry i > j at refl_at(W, i, j): columns contiguous
    double* P;      // 2 x 4 W: p = tau G v of a reflector (the two buffers alternate by step parity)
    double* KP;     // 2 x SRB step_blocks(W) shares of v^H p (one per row wave)
    double* CB;     // 2 x 4 W: copy of the column of the next reflector, taken before its update
    double* X;      // W x nvec eigenvectors of T (entry i of vector t at X[i nvec + t])
    double* wyT;    // 16 (W + 4) doubles: the T factors of the WY blocks of the reflectors
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
    r.P = p; p += 8 * W;
    r.KP = p; p += 2 * SRB * step_blocks(W);
    r.CB = p; p += 8 * W;
    r.X = p; p += W * nvec;
    r.wyT = p; p += 16 * (W + 4);
    return r;
}
__host__ __device__ inline int64_t big_rec_doubles(int64_t W, int64_t nvec) {
    return 4 * W * W + 9 * W + 8 + 4 * (W * (W + 1) / 2) + 16 * W + 2 * SRB * step_blocks(W) + W * nvec +
           16 * (W + 4);
}

// The reflector of a column x (entries r > j0 below the diagonal held in vn[r], zero elsewhere):
// alpha = |x|, phi = x_{j0+1} / |x_{j0+1}|, v = x + alpha phi e_{j0+1} (H x = -alpha phi e_{j0+1}),
// tau = 1 / (alpha (alpha + |x_{j0+1}|)).  vn is left as x: v differs from it only in entry j0 + 1,
// which every thread gets in v1 (so no thread rewrites LDS that others read).  Every thread
// returns tau; block 0 stores v (rows > j0) in the record's column j0, tau and s = -alpha phi.
// part: this thread's share of |x|^2.
__device__ double make_reflector(const double* vn, int W, int j0, double part, double* red, const BigRec& R, bool store,
                                 Q4& v1) {
    const double alpha = sqrt(block_total<SRB>(part, red));
    const Q4 x1 = j0 + 1 < W ? Q4{vn[j0 + 1], vn[W + j0 + 1], vn[2 * W + j0 + 1], vn[3 * W + j0 + 1]}
                             : Q4{0, 0, 0, 0};
    const double ax1 = sqrt(qn2(x1));
    const Q4 phi = ax1 > 0.0 ? qscale(x1, 1.0 / ax1) : Q4{1, 0, 0, 0};
    const double tau = alpha > 0.0 ? 1.0 / (alpha * (alpha + ax1)) : 0.0;
    v1 = qadd(x1, qscale(phi, alpha));
    if (store) {
        const int64_t pps = (int64_t)W * (W + 1) / 2;
        for (int r = j0 + 1 + (int)threadIdx.x; r < W; r += SBT)
            st(R.refl, pps, refl_at(W, r, j0), r == j0 + 1 ? v1 : Q4{vn[r], vn[W + r], vn[2 * W + r], vn[3 * W + r]});
        if (threadIdx.x == 0) {
            R.tau[j0] = tau;
            const Q4 sj = qscale(phi, -alpha);
            R.ph[j0] = sj.w; R.ph[W + j0] = sj.x; R.ph[2 * W + j0] = sj.y; R.ph[3 * W + j0] = sj.z;   // s_j, for now
        }
    }
    return tau;
}

// entry c of the reflector held as x in vn with its entry j0 + 1 in v1
__device__ __forceinline__ Q4 refl_entry(const double* vn, int W, int c, int j0, Q4 v1) {
    return c == j0 + 1 ? v1 : Q4{vn[c], vn[W + c], vn[2 * W + c], vn[3 * W + c]};
}

// Start of the tridiagonalisation of problem blockIdx.y: copy its rows of G into the record,
// reflector 0 from column 0 (every block), p = tau G v for its rows, its share of v^H p, and the
// copy of column 1.  Grid (step_blocks(W), problems).
__global__ __launch_bounds__(SBT) void k_big_start(const double* __restrict__ G0, int64_t gstride, double* base0,
                                                  int64_t rstride, int W, int nvec) {
    __shared__ double vn[4 * 1024];                       // W <= 1024
    __shared__ double red[SRB];
    const double* G = G0 + blockIdx.y * gstride;
    BigRec R = big_rec(base0 + blockIdx.y * rstride, W, nvec);
    const int64_t ps = (int64_t)W * W;
    const int tid = threadIdx.x;
    const int nbs = (int)step_blocks(W);
    const bool refl = W >= 3;
    double tau = 0.0;
    Q4 v1{0, 0, 0, 0};
    if (refl) {
        double part = 0.0;
        for (int r = tid; r < W; r += SBT) {
            const Q4 x = r > 0 ? ld(G, ps, (int64_t)r * W) : Q4{0, 0, 0, 0};
            vn[r] = x.w; vn[W + r] = x.x; vn[2 * W + r] = x.y; vn[3 * W + r] = x.z;
            part += qn2(x);
        }
        tau = make_reflector(vn, W, 0, part, red, R, blockIdx.x == 0, v1);
    }
    const int wave = tid >> 6, lane = tid & 63;
    const int r = blockIdx.x * SRB + wave;
    double kp = 0.0;
    if (r < W) {
        Q4 acc{0, 0, 0, 0};
        for (int c = lane; c < W; c += 64) {
            const int64_t e = (int64_t)r * W + c;
            const Q4 g = ld(G, ps, e);
            st(R.Gw, ps, e, g);
            if (refl && c > 0) acc = qadd(acc, qmul(g, refl_entry(vn, W, c, 0, v1)));
            if (c == 1 && r > 1) st(R.CB, W, r, g);
        }
        if (refl) {
            acc.w = wave_total(acc.w); acc.x = wave_total(acc.x); acc.y = wave_total(acc.y); acc.z = wave_total(acc.z);
            const Q4 p = qscale(acc, tau);
            if (lane == 0 && r > 0) {
                st(R.P, W, r, p);
                kp = qdot(refl_entry(vn, W, r, 0, v1), p);
            }
        }
    }
    if (lane == 0) R.KP[blockIdx.x * SRB + wave] = kp;   // this wave's share of v^H p
    (void)nbs;
}

// Step j of the tridiagonalisation of problem blockIdx.y (0 <= j <= W - 3): q = p - K v for
// reflector j; the next reflector (j + 1 <= W - 3) from column j + 1 after this step's update
// (the copy taken before it, updated here), formed by every block; then this block's rows:
// G <- G - v q^H - q v^H, p' = tau' G v' of the next reflector, the copy of column j + 2.
// Grid (step_blocks(W), problems).
__global__ __launch_bounds__(SBT) void k_big_step(double* base0, int64_t rstride, int W, int nvec, int j) {
    __shared__ double sh[12 * 1024];                      // W <= 1024
    double* vs = sh;            // v of reflector j
    double* qs = sh + 4 * W;    // q of reflector j
    double* vn = sh + 8 * W;    // v of reflector j + 1
    __shared__ double red[SRB];
    BigRec R = big_rec(base0 + blockIdx.y * rstride, W, nvec);
    const int64_t ps = (int64_t)W * W, pps = (int64_t)W * (W + 1) / 2;
    const int tid = threadIdx.x;
    const int nbs = (int)step_blocks(W);
    const int cur = j & 1, nxt = cur ^ 1;
    const double* Pc = R.P + (int64_t)cur * 4 * W;
    double* Pn = R.P + (int64_t)nxt * 4 * W;
    const double* CBc = R.CB + (int64_t)cur * 4 * W;
    double* CBn = R.CB + (int64_t)nxt * 4 * W;
    const int wave = tid >> 6, lane = tid & 63;
    const int r = blockIdx.x * SRB + wave;
    const int nks = SRB * nbs;
    double part = 0.0;
    for (int i = tid; i < nks; i += SBT) part += R.KP[cur * nks + i];
    const double tau = R.tau[j];
    const double K = 0.5 * tau * block_total<SRB>(part, red);
    for (int c = tid; c < W; c += SBT) {
        Q4 v{0, 0, 0, 0}, q{0, 0, 0, 0};
        if (c > j) {
            v = ld(R.refl, pps, refl_at(W, c, j));
            q = qsub(ld(Pc, W, c), qscale(v, K));
        }
        vs[c] = v.w; vs[W + c] = v.x; vs[2 * W + c] = v.y; vs[3 * W + c] = v.z;
        qs[c] = q.w; qs[W + c] = q.x; qs[2 * W + c] = q.y; qs[3 * W + c] = q.z;
    }
    __syncthreads();
    const int j1 = j + 1;
    const bool more = j1 <= W - 3;
    double tau1 = 0.0;
    Q4 v1n{0, 0, 0, 0};
    if (more) {
        // column j1 after this step's update, rows below the diagonal (the same arithmetic as the
        // row update below, so v' is exactly the updated column)
        const Q4 vj{vs[j1], vs[W + j1], vs[2 * W + j1], vs[3 * W + j1]};
        const Q4 qj{qs[j1], qs[W + j1], qs[2 * W + j1], qs[3 * W + j1]};
        const Q4 cvj = qconj(vj), cqj = qconj(qj);
        double p2 = 0.0;
        for (int r = tid; r < W; r += SBT) {
            Q4 x{0, 0, 0, 0};
            if (r > j1) {
                const Q4 vr{vs[r], vs[W + r], vs[2 * W + r], vs[3 * W + r]};
                const Q4 qr{qs[r], qs[W + r], qs[2 * W + r], qs[3 * W + r]};
                x = qsub(qsub(ld(CBc, W, r), qmul(vr, cqj)), qmul(qr, cvj));
                p2 += qn2(x);
            }
            vn[r] = x.w; vn[W + r] = x.x; vn[2 * W + r] = x.y; vn[3 * W + r] = x.z;
        }
        tau1 = make_reflector(vn, W, j1, p2, red, R, blockIdx.x == 0, v1n);
    }
    double kp = 0.0;
    if (r > j && r < W) {
        const Q4 vr{vs[r], vs[W + r], vs[2 * W + r], vs[3 * W + r]};
        const Q4 qr{qs[r], qs[W + r], qs[2 * W + r], qs[3 * W + r]};
        Q4 acc{0, 0, 0, 0};
        for (int c = j + 1 + lane; c < W; c += 64) {
            const Q4 vc{vs[c], vs[W + c], vs[2 * W + c], vs[3 * W + c]};
            const Q4 qc{qs[c], qs[W + c], qs[2 * W + c], qs[3 * W + c]};
            const int64_t e = (int64_t)r * W + c;
            Q4 t = qsub(qsub(ld(R.Gw, ps, e), qmul(vr, qconj(qc))), qmul(qr, qconj(vc)));
            if (r == c) t.x = t.y = t.z = 0.0;
            st(R.Gw, ps, e, t);
            if (more) acc = qadd(acc, qmul(t, refl_entry(vn, W, c, j1, v1n)));
            if (c == j + 2 && r > j + 2) st(CBn, W, r, t);
        }
        if (more) {
            acc.w = wave_total(acc.w); acc.x = wave_total(acc.x); acc.y = wave_total(acc.y); acc.z = wave_total(acc.z);
            const Q4 p = qscale(acc, tau1);
            if (lane == 0 && r > j1) {
                st(Pn, W, r, p);
                kp = qdot(refl_entry(vn, W, r, j1, v1n), p);
            }
        }
    }
    if (lane == 0) R.KP[nxt * nks + blockIdx.x * SRB + wave] = kp;   // this wave's share of v'^H p'
}

// diagonal, real subdiagonal b_j = |s_j|, phases ph_{j+1} = s_j ph_j / |s_j|, bounds (problem
// blockIdx.x): the diagonal of the working matrix and the s_j are staged in LDS by the whole wave
// (independent loads), which also forms b_j, 1 / b_j and the Gershgorin bounds and writes d, b
// and b^2; one lane runs only the chain of phases, into LDS, and the wave writes them out.
__global__ __launch_bounds__(64) void k_big_fin(double* __restrict__ base0, int64_t rstride, int W, int nvec) {
    __shared__ double sd[1024], ss[4 * 1024], sbr[1024], sinv[1024], sph[4 * 1024];   // W <= 1024
    BigRec R = big_rec(base0 + blockIdx.x * rstride, W, nvec);
    const int64_t ps = (int64_t)W * W;
    const int lane = threadIdx.x;
    for (int i = lane; i < W; i += 64) {
        sd[i] = R.Gw[(int64_t)i * W + i];
        Q4 sj{0, 0, 0, 0};
        if (i + 2 < W) sj = Q4{R.ph[i], R.ph[W + i], R.ph[2 * W + i], R.ph[3 * W + i]};
        else if (i + 2 == W) sj = ld(R.Gw, ps, (int64_t)(W - 1) * W + (W - 2));   // the last subdiagonal entry
        ss[i] = sj.w; ss[W + i] = sj.x; ss[2 * W + i] = sj.y; ss[3 * W + i] = sj.z;
        const double br = i + 1 < W ? sqrt(qn2(sj)) : 0.0;
        sbr[i] = br;
        sinv[i] = br > 0.0 ? 1.0 / br : 0.0;
    }
    __syncthreads();
    double lo = 1e300, hi = -1e300;
    for (int i = lane; i < W; i += 64) {
        const double dd = sd[i], br = sbr[i], bl = i > 0 ? sbr[i - 1] : 0.0;
        R.d[i] = dd;
        R.b[i] = br;
        R.b2[i] = br * br;
        lo = fmin(lo, dd - bl - br);
        hi = fmax(hi, dd + bl + br);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) {
        if (W >= 2) R.tau[W - 2] = 0.0;
        R.tau[W - 1] = 0.0;
        const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
        R.bnd[0] = lo - pad;
        R.bnd[1] = hi + pad;
    }
    // The phases: step i maps ph_i to ph_{i+1} = (s_i / b_i) ph_i, or to 1 where b_i = 0, and
    // ph_0 = 1.  Such maps (left multiplication by a quaternion, or a constant) compose
    // associatively: every lane composes the steps of its run of C = ceil(W / 64) entries, a scan
    // over the wave gives each lane the phase at the start of its run, and the lane replays its
    // run from there (about 2 C + 6 dependent products instead of W).
    const int C = (W + 63) / 64;
    const int i0 = lane * C, i1 = min(i0 + C, W);                 // this lane's entries
    auto step = [&](int i, Q4 p) -> Q4 {                          // ph_{i+1} from ph_i
        const Q4 sj{ss[i], ss[W + i], ss[2 * W + i], ss[3 * W + i]};
        return sbr[i] > 0.0 ? qscale(qmul(sj, p), sinv[i]) : Q4{1, 0, 0, 0};
    };
    // the composite of steps i0 .. i1 - 1 (those below W - 1): p -> M p, or the constant M
    Q4 M{1, 0, 0, 0};
    bool cst = false;
    for (int i = i0; i < i1 && i + 1 < W; i++) {
        if (sbr[i] > 0.0) {
            const Q4 sj{ss[i], ss[W + i], ss[2 * W + i], ss[3 * W + i]};
            M = qmul(qscale(sj, sinv[i]), M);
        } else {
            M = Q4{1, 0, 0, 0};
            cst = true;
        }
    }
    // inclusive scan: lane l composes the runs of lanes <= l (the later map applied after)
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const Q4 Mo{__shfl_up(M.w, o, 64), __shfl_up(M.x, o, 64), __shfl_up(M.y, o, 64), __shfl_up(M.z, o, 64)};
        const bool co = __shfl_up((int)cst, o, 64) != 0;
        if (lane >= o && !cst) {
            M = qmul(M, Mo);
            cst = co;
        }
    }
    // the phase at the start of this lane's run: the runs of the lanes before it applied to 1
    Q4 p{__shfl_up(M.w, 1, 64), __shfl_up(M.x, 1, 64), __shfl_up(M.y, 1, 64), __shfl_up(M.z, 1, 64)};
    if (lane == 0) p = Q4{1, 0, 0, 0};
    for (int i = i0; i < i1; i++) {
        sph[i] = p.w; sph[W + i] = p.x; sph[2 * W + i] = p.y; sph[3 * W + i] = p.z;
        if (i + 1 < W) p = step(i, p);
    }
    __syncthreads();
    for (int i = lane; i < W; i += 64) {
        R.ph[i] = sph[i]; R.ph[W + i] = sph[W + i]; R.ph[2 * W + i] = sph[2 * W + i]; R.ph[3 * W + i] = sph[3 * W + i];
    }
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

// eigenvalues: grid (ceil(W / 4), problems), one wave per eigenvalue, 65-section rounds (six bits
// of the interval a round, ten rounds: a width of 65^-10 of the Gershgorin bounds, about 7e-19);
// lam_out (problem 0 only) descending
__global__ __launch_bounds__(BT) void k_big_eigvals(double* __restrict__ base0, int64_t rstride, int W, int nvec,
                                                    double* __restrict__ lam_out) {
    extern __shared__ double sh[];
    double* d = sh;
    double* b2 = sh + W;
    BigRec R = big_rec(base0 + blockIdx.y * rstride, W, nvec);
    if (blockIdx.y != 0) lam_out = nullptr;
    const int tid = threadIdx.x, lane = tid & 63;
    int ex;
    frexp(fmax(fabs(R.bnd[0]), fabs(R.bnd[1])), &ex);
    for (int i = tid; i < W; i += BT) {
        d[i] = ldexp(R.d[i], -ex);
        b2[i] = ldexp(R.b2[i], -2 * ex);
    }
    __syncthreads();
    const int k = blockIdx.x * (BT / 64) + (tid >> 6);
    double a = ldexp(R.bnd[0], -ex), bb = ldexp(R.bnd[1], -ex);
    for (int round = 0; round < 10; round++) {
        const double x = a + (bb - a) * (double)(lane + 1) / 65.0;
        const int c = sturm_lds(d, b2, W, x);
        const unsigned long long m = __ballot(c > k);
        const int first = m ? __builtin_ctzll(m) : 64;
        const double xa = first == 0 ? a : a + (bb - a) * (double)first / 65.0;
        const double xb = first == 64 ? bb : a + (bb - a) * (double)(first + 1) / 65.0;
        a = xa;
        bb = xb;
    }
    if (k < W && lane == 0) {
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
// factorisations, one workgroup of one wave per vector, with the tridiagonal, the forward and
// backward pivots and the vector in LDS.  The two recurrences (the pivots, then the vector
// outward from the twist index) run on lane 0 in their serial order; the twist search and the
// normalisation are spread over the wave.  Vector t's entry i goes to X[i nvec + t].
__global__ __launch_bounds__(64) void k_big_twisted(double* __restrict__ base, int W, int nvec, int kfirst) {
    extern __shared__ double tw[];
    double* sd = tw;                 // W each: d, b, b^2, forward pivots / the vector, backward pivots
    double* sb = tw + W;
    double* sb2 = tw + 2 * W;
    double* xs = tw + 3 * W;
    double* ds = tw + 4 * W;
    BigRec R = big_rec(base, W, nvec);
    const int t = blockIdx.x, k = kfirst + t, lane = threadIdx.x;
    if (t >= nvec || k >= W) return;                   // uniform over the workgroup
    for (int i = lane; i < W; i += 64) {
        sd[i] = R.d[i];
        sb[i] = R.b[i];
        sb2[i] = R.b2[i];
    }
    __syncthreads();
    const double tnorm = fmax(fabs(R.bnd[0]), fabs(R.bnd[1])) + 1e-300;
    const double tiny = 1e-300 + 2.220446049250313e-16 * tnorm * 1e-3;
    const double mu = R.lam[k];
    if (lane == 0) {
        double fp = sd[0] - mu, bp = sd[W - 1] - mu;
        if (fabs(fp) < tiny) fp = -tiny;
        if (fabs(bp) < tiny) bp = -tiny;
        xs[0] = fp;
        ds[W - 1] = bp;
        for (int i = 1; i < W; i++) {
            const int ib = W - 1 - i;
            double f = (sd[i] - mu) - fdiv(sb2[i - 1], fp);
            double g = (sd[ib] - mu) - fdiv(sb2[ib], bp);
            if (fabs(f) < tiny) f = -tiny;
            if (fabs(g) < tiny) g = -tiny;
            xs[i] = f;
            ds[ib] = g;
            fp = f;
            bp = g;
        }
    }
    __syncthreads();
    // the twist index r: the smallest |gamma_i| = |x_i + dm_i - (d_i - mu)| (|x_{W-1}| for the
    // last), the largest i on ties; a non-finite gamma_{W-1} keeps r = W - 1 (the serial scan
    // downwards from W - 1 with a strict comparison)
    double best = __builtin_inf();
    int r = -1;
    for (int i = W - 1 - lane; i >= 0; i -= 64) {
        const double gam = i == W - 1 ? fabs(xs[i]) : fabs(xs[i] + ds[i] - (sd[i] - mu));
        if (gam < best) { best = gam; r = i; }          // descending i: ties keep the larger i
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int orr = __shfl_xor(r, o, 64);
        if (ob < best || (ob == best && orr > r)) { best = ob; r = orr; }
    }
    const double g_last = fabs(xs[W - 1]);
    if (!(g_last == g_last) || r < 0) r = W - 1;
    // x_{r +- s} from x_{r +- (s - 1)}, overwriting the forward pivots as they are used
    __shared__ double nrm_sh;
    if (lane == 0) {
        double xd = 1.0, xu = 1.0, nrm = 1.0;
        const int steps = max(W - 1 - r, r);
        for (int s = 1; s <= steps; s++) {
            const int id = r + s, iu = r - s;
            if (id < W) {
                xd = -fdiv(sb[id - 1] * xd, ds[id]);
                xs[id] = xd;
                nrm += xd * xd;
            }
            if (iu >= 0) {
                xu = -fdiv(sb[iu] * xu, xs[iu]);
                xs[iu] = xu;
                nrm += xu * xu;
            }
        }
        xs[r] = 1.0;
        nrm_sh = 1.0 / sqrt(nrm);
    }
    __syncthreads();
    const double nrm = nrm_sh;
    double* x = R.X + t;
    for (int i = lane; i < W; i += 64) x[(int64_t)i * nvec] = xs[i] * nrm;
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
            double* xa = R.X + a;                       // entry i at xa[i nvec]
            for (int bq = cs; bq < a; bq++) {
                const double* xb = R.X + bq;
                double dot = 0.0;
                for (int i = lane; i < W; i += 64) dot += xa[(int64_t)i * nvec] * xb[(int64_t)i * nvec];
                dot = wave_total(dot);
                for (int i = lane; i < W; i += 64) xa[(int64_t)i * nvec] -= dot * xb[(int64_t)i * nvec];
            }
            double nr2 = 0.0;
            for (int i = lane; i < W; i += 64) nr2 += xa[(int64_t)i * nvec] * xa[(int64_t)i * nvec];
            nr2 = wave_total(nr2);
            const double inv = nr2 > 0.0 ? 1.0 / sqrt(nr2) : 0.0;
            for (int i = lane; i < W; i += 64) xa[(int64_t)i * nvec] *= inv;
        }
        cs = t;
    }
}

// Compact WY form of the back-transformation.  Block m holds reflectors 4 m .. 4 m + 3 (zero past
// W - 3): H_{4m} H_{4m+1} H_{4m+2} H_{4m+3} = I - V T V^H with T upper triangular (quaternion
// entries; the tau are real), built column by column: T_kk = tau_k and, above it,
// -tau_k T (V^H v_k) from the Gram entries v_a^H v_k.  One workgroup per block.
constexpr int WYB = 4;                         // reflectors per block

__host__ __device__ inline int64_t wy_blocks(int64_t W) { return W >= 3 ? (W - 2 + WYB - 1) / WYB : 0; }

__global__ __launch_bounds__(BT) void k_big_wy(double* __restrict__ base, int W, int nvec) {
    __shared__ double red[4];
    BigRec R = big_rec(base, W, nvec);
    const int m = blockIdx.x, j0 = WYB * m, tid = threadIdx.x;
    const int64_t pps = (int64_t)W * (W + 1) / 2;
    // g[a][b] = v_a^H v_b for a < b (six pairs), each thread's share over the rows
    Q4 g[6];
#pragma unroll
    for (int e = 0; e < 6; e++) g[e] = Q4{0, 0, 0, 0};
    for (int i = tid; i < W; i += BT) {
        Q4 v[WYB];
#pragma unroll
        for (int a = 0; a < WYB; a++) {
            const int j = j0 + a;
            v[a] = (j <= W - 3 && i > j) ? ld(R.refl, pps, refl_at(W, i, j)) : Q4{0, 0, 0, 0};
        }
        int e = 0;
#pragma unroll
        for (int a = 0; a < WYB; a++)
#pragma unroll
            for (int b = a + 1; b < WYB; b++) g[e] = qadd(g[e], qmul(qconj(v[a]), v[b])), e++;
    }
#pragma unroll
    for (int e = 0; e < 6; e++) {
        g[e].w = block_total(g[e].w, red); g[e].x = block_total(g[e].x, red);
        g[e].y = block_total(g[e].y, red); g[e].z = block_total(g[e].z, red);
    }
    if (tid != 0) return;
    double tau[WYB];
#pragma unroll
    for (int a = 0; a < WYB; a++) tau[a] = j0 + a <= W - 3 ? R.tau[j0 + a] : 0.0;
    Q4 T[WYB][WYB];
#pragma unroll
    for (int r = 0; r < WYB; r++)
#pragma unroll
        for (int c = 0; c < WYB; c++) T[r][c] = Q4{0, 0, 0, 0};
    auto gram = [&](int a, int b) {   // v_a^H v_b, a < b
        const int e = a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
        return g[e];
    };
    T[0][0] = Q4{tau[0], 0, 0, 0};
#pragma unroll
    for (int k = 1; k < WYB; k++) {
#pragma unroll
        for (int r = 0; r < k; r++) {
            Q4 z{0, 0, 0, 0};
#pragma unroll
            for (int c = r; c < k; c++) z = qadd(z, qmul(T[r][c], gram(c, k)));
            T[r][k] = qscale(z, -tau[k]);
        }
        T[k][k] = Q4{tau[k], 0, 0, 0};
    }
    double* out = R.wyT + (int64_t)m * 4 * WYB * WYB;
#pragma unroll
    for (int r = 0; r < WYB; r++)
#pragma unroll
        for (int c = 0; c < WYB; c++) {
            const int e = 4 * (r * WYB + c);
            out[e] = T[r][c].w; out[e + 1] = T[r][c].x; out[e + 2] = T[r][c].y; out[e + 3] = T[r][c].z;
        }
}

// back-transformation y = H_0 ... H_{W-3} D x for the nout largest eigenvalues by WY blocks, last
// block first: y <- y - V (T (V^H y)).  One workgroup of BWV waves per vector, the waves holding
// row slices of SL = 64 NRS rows (lane l of wave s: rows s SL + l + 64 u); the slices' shares of
// V^H y and the block's T meet in LDS (double-buffered by block parity; the shares summed in
// slice order).  The reflectors of the next block are loaded into the other register set while
// the current block is applied.  E (W x nout, ld nout) gets the vectors in descending order.
constexpr int BWV = 4;                          // waves per vector
template <int NRS>
__global__ __launch_bounds__(64 * BWV) void k_big_back_wy(double* __restrict__ base, int W, int nvec, int kfirst,
                                                          int nout, double* __restrict__ E) {
    constexpr int SL = 64 * NRS;
    __shared__ double part[2][BWV][4 * WYB];
    __shared__ double tb[2][4 * WYB * WYB];
    BigRec R = big_rec(base, W, nvec);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int o = blockIdx.x;                                   // output column
    const int slot = W - 1 - o - kfirst;                        // ascending index W - 1 - o
    const int64_t pps = (int64_t)W * (W + 1) / 2;
    const int nb = (int)wy_blocks(W);
    Q4 y[NRS];
#pragma unroll
    for (int u = 0; u < NRS; u++) {
        const int i = wave * SL + lane + 64 * u;
        y[u] = i < W ? qscale(Q4{R.ph[i], R.ph[W + i], R.ph[2 * W + i], R.ph[3 * W + i]},
                              R.X[(int64_t)i * nvec + slot])
                     : Q4{0, 0, 0, 0};
    }
    auto load_v = [&](int m, Q4 (&v)[WYB][NRS]) {
#pragma unroll
        for (int a = 0; a < WYB; a++) {
            const int j = WYB * m + a;
#pragma unroll
            for (int u = 0; u < NRS; u++) {
                const int i = wave * SL + lane + 64 * u;
                v[a][u] = (j <= W - 3 && i > j && i < W) ? ld(R.refl, pps, refl_at(W, i, j)) : Q4{0, 0, 0, 0};
            }
        }
    };
    auto apply = [&](int m, const Q4 (&v)[WYB][NRS]) {
        const int pb = m & 1;
        if (tid < 4 * WYB * WYB) tb[pb][tid] = R.wyT[(int64_t)m * 4 * WYB * WYB + tid];
        Q4 s[WYB];
#pragma unroll
        for (int a = 0; a < WYB; a++) {
            s[a] = Q4{0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < NRS; u++) s[a] = qadd(s[a], qmul(qconj(v[a][u]), y[u]));
            s[a].w = wave_total(s[a].w); s[a].x = wave_total(s[a].x);
            s[a].y = wave_total(s[a].y); s[a].z = wave_total(s[a].z);
        }
        if (lane == 0)
#pragma unroll
            for (int a = 0; a < WYB; a++) {
                double* q = part[pb][wave] + 4 * a;
                q[0] = s[a].w; q[1] = s[a].x; q[2] = s[a].y; q[3] = s[a].z;
            }
        __syncthreads();
        Q4 S[WYB];
#pragma unroll
        for (int a = 0; a < WYB; a++) {
            S[a] = Q4{0, 0, 0, 0};
#pragma unroll
            for (int w = 0; w < BWV; w++) {
                const double* q = part[pb][w] + 4 * a;
                S[a] = qadd(S[a], Q4{q[0], q[1], q[2], q[3]});
            }
        }
        Q4 U[WYB];
#pragma unroll
        for (int r = 0; r < WYB; r++) {
            U[r] = Q4{0, 0, 0, 0};
#pragma unroll
            for (int c = r; c < WYB; c++) {
                const double* t = tb[pb] + 4 * (r * WYB + c);
                U[r] = qadd(U[r], qmul(Q4{t[0], t[1], t[2], t[3]}, S[c]));
            }
        }
#pragma unroll
        for (int u = 0; u < NRS; u++)
#pragma unroll
            for (int a = 0; a < WYB; a++) y[u] = qsub(y[u], qmul(v[a][u], U[a]));
    };
    Q4 va[WYB][NRS], vb[WYB][NRS];
    int m = nb - 1;
    if (m >= 0) load_v(m, va);
    for (; m >= 1; m -= 2) {
        load_v(m - 1, vb);
        apply(m, va);
        if (m >= 2) load_v(m - 2, va);
        apply(m - 1, vb);
    }
    if (m == 0) apply(0, va);
    const int64_t eps = (int64_t)W * nout;
#pragma unroll
    for (int u = 0; u < NRS; u++) {
        const int i = wave * SL + lane + 64 * u;
        if (i < W) st(E, eps, (int64_t)i * nout + o, y[u]);
    }
}

// e_b = sqrt(max(0, nA2 - sum of the k largest max(lambda, 0)) / nA2) for problem b (thread b).
__global__ void k_big_estimates(const double* __restrict__ base0, int64_t rstride, int W, int nprob, int k,
                                const double* __restrict__ nA2, double* __restrict__ e) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    const BigRec R = big_rec(const_cast<double*>(base0) + b * rstride, W, 0);
    double top = 0.0;
    for (int j = 0; j < k && j < W; j++) top += fmax(R.lam[W - 1 - j], 0.0);
    const double a = *nA2, r = a - top;
    e[b] = a > 0.0 ? sqrt((r > 0.0 ? r : 0.0) / a) : 0.0;
}

// The tridiagonalisation and k_big_fin for nprob problems of order W (problem b's Gram at
// G + b gstride, its record at work + b rstride).
void tridiagonalise(const double* G, int64_t gstride, int64_t W, int nprob, double* work, int64_t rstride,
                    int64_t nvec, hipStream_t st) {
    const dim3 grid((unsigned)step_blocks(W), (unsigned)nprob);
    hipLaunchKernelGGL(k_big_start, grid, dim3(SBT), 0, st, G, gstride, work, rstride, (int)W, (int)nvec);
    for (int j = 0; j + 2 < W; j++)
        hipLaunchKernelGGL(k_big_step, grid, dim3(SBT), 0, st, work, rstride, (int)W, (int)nvec, j);
    hipLaunchKernelGGL(k_big_fin, dim3((unsigned)nprob), dim3(64), 0, st, work, rstride, (int)W, (int)nvec);
}

}  // namespace

int heig_big_max() { return 1024; }

hipError_t heig_big_estimates_launch(const double* G, int64_t gstride, int64_t W, int nprob, int k,
                                     const double* nA2, double* e, double* work, hipStream_t st) {
    if (W < 1 || W > heig_big_max() || nprob < 1) return hipErrorInvalidValue;
    const int64_t rstride = big_rec_doubles(W, 0);
    tridiagonalise(G, gstride, W, nprob, work, rstride, 0, st);
    hipLaunchKernelGGL(k_big_eigvals, dim3((unsigned)((W + 3) / 4), (unsigned)nprob), dim3(BT),
                       (size_t)(2 * W * sizeof(double)), st, work, rstride, (int)W, 0, (double*)nullptr);
    hipLaunchKernelGGL(k_big_estimates, dim3((unsigned)((nprob + 63) / 64)), dim3(64), 0, st, (const double*)work,
                       rstride, (int)W, nprob, k, nA2, e);
    return hipGetLastError();
}

size_t heig_big_work_doubles(int64_t W, int64_t nvec) { return (size_t)big_rec_doubles(W, nvec); }

// lam: W eigenvalues, descending.  E (optional): the nout eigenvectors of the largest
// eigenvalues as columns, descending (W x nout, ld nout).  nvec: vector slots of the record
// (>= nout plus the cluster extension; the caller passes W to be safe or nout + margin).
hipError_t heig_big_launch(const double* G, int64_t W, double* lam, double* E, int64_t nout, double* work,
                           int64_t nvec, hipStream_t st) {
    if (W < 1 || W > heig_big_max() || nout < 0 || nout > W || (E && nvec < nout)) return hipErrorInvalidValue;
    tridiagonalise(G, 0, W, 1, work, 0, nvec, st);
    hipLaunchKernelGGL(k_big_eigvals, dim3((unsigned)((W + 3) / 4), 1), dim3(BT), (size_t)(2 * W * sizeof(double)),
                       st, work, (int64_t)0, (int)W, (int)nvec, lam);
    if (!E || nout == 0) return hipGetLastError();
    // vectors of ascending indices [W - nvec, W): the top nout plus room below for a cluster
    const int kfirst = (int)(W - nvec);
    hipLaunchKernelGGL(k_big_twisted, dim3((unsigned)nvec), dim3(64), (size_t)(5 * W * sizeof(double)), st, work,
                       (int)W, (int)nvec, kfirst);
    hipLaunchKernelGGL(k_big_mgs, dim3(1), dim3(64), 0, st, work, (int)W, (int)nvec, kfirst, (int)nvec);
    const int64_t nb = wy_blocks(W);
    if (nb > 0) hipLaunchKernelGGL(k_big_wy, dim3((unsigned)nb), dim3(BT), 0, st, work, (int)W, (int)nvec);
    const dim3 gb((unsigned)nout);
    if (W <= 64 * BWV)
        hipLaunchKernelGGL(k_big_back_wy<1>, gb, dim3(64 * BWV), 0, st, work, (int)W, (int)nvec, kfirst, (int)nout, E);
    else if (W <= 128 * BWV)
        hipLaunchKernelGGL(k_big_back_wy<2>, gb, dim3(64 * BWV), 0, st, work, (int)W, (int)nvec, kfirst, (int)nout, E);
    else if (W <= 192 * BWV)
        hipLaunchKernelGGL(k_big_back_wy<3>, gb, dim3(64 * BWV), 0, st, work, (int)W, (int)nvec, kfirst, (int)nout, E);
    else
        hipLaunchKernelGGL(k_big_back_wy<4>, gb, dim3(64 * BWV), 0, st, work, (int)W, (int)nvec, kfirst, (int)nout, E);
    return hipGetLastError();
}

}  // namespace qlra_impl
