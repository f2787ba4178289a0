// Small FP64 kernels of the quaternion CholeskyQR (eq. (QQR) computed as Y = Q R with
// R^H R = Y^H Y): the Hermitian quaternion Cholesky with a shifted retry, the triangular
// inverse, and products of triangular factors.  One workgroup per factorization: the matrices
// are l x l with l = k + p, tiny next to a pass over A; the chain of dependent steps is what
// costs, so for l <= kRegMax the factor lives in the registers of one 1024-thread workgroup
// (one barrier per elimination step) and its inverse is formed column by column from a packed
// copy in LDS without barriers.
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
__device__ __forceinline__ Q4 qscale(Q4 a, double s) { return Q4{a.w * s, a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double qn2(Q4 a) { return a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z; }
__device__ __forceinline__ Q4 ld4(const double* P, int64_t ps, int64_t i) {
    return Q4{P[i], P[ps + i], P[2 * ps + i], P[3 * ps + i]};
}
__device__ __forceinline__ void st4(double* P, int64_t ps, int64_t i, Q4 v) {
    P[i] = v.w; P[ps + i] = v.x; P[2 * ps + i] = v.y; P[3 * ps + i] = v.z;
}

constexpr int kThreads = 1024;

// c ? a : b, component by component (a select of values, kept in registers)
__device__ __forceinline__ Q4 qsel(bool c, Q4 a, Q4 b) {
    return Q4{c ? a.w : b.w, c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}
// acc - a b (eq. (1)), as four chains of fused multiply-adds into acc
__device__ __forceinline__ Q4 qfms(Q4 acc, Q4 a, Q4 b) {
    return Q4{fma(a.z, b.z, fma(a.y, b.y, fma(a.x, b.x, fma(-a.w, b.w, acc.w)))),
              fma(a.z, b.y, fma(-a.y, b.z, fma(-a.x, b.w, fma(-a.w, b.x, acc.x)))),
              fma(-a.z, b.x, fma(-a.y, b.w, fma(a.x, b.z, fma(-a.w, b.y, acc.y)))),
              fma(-a.z, b.w, fma(a.y, b.x, fma(-a.x, b.y, fma(-a.w, b.z, acc.z))))};
}

// upper triangle of order w packed by rows: (t, c), c >= t
__device__ __forceinline__ int upk(int t, int c, int w) { return t * (2 * w - t + 1) / 2 + (c - t); }
// ------------------------------------------------------------------------------------------
// Factors of order w <= kRegMax: the matrix in registers (1024 threads, NB x NB entries each:
// rows ty + 32 i, columns tx + 32 j; NB = 2 up to 64, 3 up to 96), one barrier per elimination
// step.
constexpr int kRegMax = 96;

__device__ __forceinline__ Q4 qadd(Q4 a, Q4 b) { return Q4{a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }
template <int S>
__device__ __forceinline__ Q4 ldp(const double* p, int i) { return Q4{p[i], p[S + i], p[2 * S + i], p[3 * S + i]}; }
template <int S>
__device__ __forceinline__ void stp(double* p, int i, Q4 v) {
    p[i] = v.w; p[S + i] = v.x; p[2 * S + i] = v.y; p[3 * S + i] = v.z;
}

// lane i's value of v (i uniform)
__device__ __forceinline__ double bcast(double v, int i) {
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffll), i);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), i);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sqrt(d) and 1 / sqrt(d) for a positive finite d: the hardware reciprocal square root refined
// by two Newton steps (each doubles the correct bits: a short dependent chain next to a
// square root followed by a division); tiny d take the plain route.
__device__ __forceinline__ void sqrt_rsqrt(double d, double& s, double& r) {
    if (d < 1e-280) {
        s = sqrt(d);
        r = 1.0 / s;
        return;
    }
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const double e = fma(-(d * y), y, 1.0);     // 1 - d y^2
        y = fma(0.5 * y, e, y);
    }
    r = y;
    s = d * y;
}

// the pivot row in LDS with the four components of an entry side by side (two 16-byte accesses)
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

// Right-looking Cholesky G + shift I = R^H R (R upper triangular with real positive diagonal):
// step j scales row j by 1 / r_jj (the half wave that owns row j, double-buffered row in LDS),
// then every owner of an entry (a, b), j < a <= b, subtracts conj(r_ja) r_jb.
template <int NB, int H>
__device__ __forceinline__ void chol_row(Q4 (&g)[NB][NB], int j, int w, int tx, double* rb, double rjj, double inv) {
#pragma unroll
    for (int ci = H; ci < NB; ci++) {
        const int c = tx + 32 * ci;
        if (c == j) g[H][ci] = Q4{rjj, 0, 0, 0};
        else if (c > j && c < w) {
            const Q4 r = qscale(g[H][ci], inv);
            g[H][ci] = r;
            sti(rb, c, r);
        }
    }
}

template <int NB, int H = 0>
__device__ __forceinline__ void chol_row_at(Q4 (&g)[NB][NB], int jh, int j, int w, int tx, double* rb, double rjj,
                                            double inv) {
    if constexpr (H < NB) {
        if (jh == H) chol_row<NB, H>(g, j, w, tx, rb, rjj, inv);
        else chol_row_at<NB, H + 1>(g, jh, j, w, tx, rb, rjj, inv);
    }
}

constexpr int kFlag = 4 * kRegMax;                     // breakdown flag behind the pivot row
typedef double RowBuf[4 * kRegMax + 2];                  // pivot row, components side by side

// The factorization of G + shift I (G w x w Hermitian, FP64 planes with row stride ldg and plane
// stride gps; w <= 32 NB) into the registers of a 1024-thread workgroup: thread (ty, tx) holds the
// entries (ty + 32 i, tx + 32 j), j >= i, and ends with those of R.  A breakdown (or non-finite
// pivot) with allow_shift set is redone once with shift = shift_scale * trace(G) (shifted = 1);
// one that remains sets failed = 1.
template <int NB>
__device__ void chol_factor(Q4 (&g)[NB][NB], const double* __restrict__ G, int64_t ldg, int64_t gps, int w,
                            int allow_shift, double shift_scale, RowBuf* rowb, int& shifted, int& failed) {
    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
    double shift = 0.0;
    shifted = 0;
    failed = 0;
    for (int attempt = 0; attempt < 2; attempt++) {
#pragma unroll
        for (int ri = 0; ri < NB; ri++)
#pragma unroll
            for (int ci = 0; ci < NB; ci++) {
                if (ci < ri) continue;                 // blocks below the diagonal hold no entry a <= b
                const int a = ty + 32 * ri, b = tx + 32 * ci;
                Q4 v{0, 0, 0, 0};
                if (a < w && b < w && b >= a) {
                    v = ld4(G, gps, (int64_t)a * ldg + b);
                    if (a == b) { v.w += shift; v.x = v.y = v.z = 0.0; }
                }
                g[ri][ci] = v;
            }
        bool fail = false;
        // the pivot row j (the half wave that owns row j, into rowb[j & 1]) is formed during step
        // j - 1, as soon as that half wave has updated its own row block: the other rows' updates
        // of step j - 1 overlap it, and the wave runs at raised priority until it is done
        auto pivot = [&](int j) {
            const int jr = j & 31, jh = j >> 5;
            double* rb = rowb[j & 1];
            if (ty == jr) {
                // the pivot (j, j) is register g[jh][jh] of lane (ty & 1) * 32 + jr of this wave
                double piv = 0.0;
#pragma unroll
                for (int h = 0; h < NB; h++)
                    if (h == jh) piv = g[h][h].w;
                const double d = bcast(piv, ((ty & 1) << 5) | jr);
                const bool bad = !(d > 0.0) || !(d < 1e300);     // breakdown or non-finite pivot
                if (tx == 0) rb[kFlag] = bad ? 1.0 : 0.0;
                if (!bad) {
                    double rjj, inv;
                    sqrt_rsqrt(d, rjj, inv);
                    chol_row_at<NB>(g, jh, j, w, tx, rb, rjj, inv);
                }
            }
        };
        pivot(0);
        for (int j = 0; j < w; j++) {
            __syncthreads();
            double* rb = rowb[j & 1];
            const int jn = j + 1, hn = jn >> 5;
            const bool next_owner = (ty >> 1) == ((jn & 31) >> 1);   // uniform over the wave
            if (next_owner) __builtin_amdgcn_s_setprio(2);
            // the pivot row's entries of this thread's rows and columns and the flag in one round
            // of LDS reads (indices stay below kRegMax; entries of rows and columns that are not
            // live are read and not used); at NB = 3 the row entries are read per row block, which
            // keeps the register count within what 16 waves of 128 registers hold
            Q4 rjb[NB], rja_all[NB];
#pragma unroll
            for (int i = 0; i < NB; i++) {
                rjb[i] = ldi(rb, tx + 32 * i);
                if constexpr (NB <= 2) rja_all[i] = qconj(ldi(rb, ty + 32 * i));
            }
            if (rb[kFlag] != 0.0) { fail = true; break; }    // uniform
            // row blocks in ascending order: rows a <= j do nothing, so the block of row j + 1 is
            // the first one updated; the next pivot follows it at once
#pragma unroll
            for (int ri = 0; ri < NB; ri++) {
                const int a = ty + 32 * ri;
                if (a > j && a < w) {
                    Q4 rja;
                    if constexpr (NB <= 2) rja = rja_all[ri];
                    else rja = qconj(ldi(rb, a));
#pragma unroll
                    for (int ci = 0; ci < NB; ci++) {
                        if (ci < ri) continue;
                        const int b = tx + 32 * ci;
                        if (b < a || b >= w) continue;
                        Q4 v = qfms(g[ri][ci], rja, rjb[ci]);
                        if (ri == ci && a == b) v.x = v.y = v.z = 0.0;
                        g[ri][ci] = v;
                    }
                }
                if (ri == hn && jn < w) {
                    pivot(jn);
                    if (next_owner) __builtin_amdgcn_s_setprio(0);
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        if (!fail) break;
        if (!allow_shift || attempt == 1) { failed = 1; break; }
        // shifted CholeskyQR (Fukaya et al.): add shift_scale * trace(G) to the diagonal
        double tr = 0.0;
        for (int i = 0; i < w; i++) tr += G[(int64_t)i * ldg + i];
        shift = shift_scale * tr;
        if (!(shift > 0.0)) shift = 1e-300;
        shifted = 1;
        __syncthreads();
    }
}

template <int NB>
__global__ __launch_bounds__(kThreads) void k_chol_reg(const double* __restrict__ G, int w, double* __restrict__ Rout,
                                                        double* __restrict__ Rpk, int* status, int* shift_out,
                                                        const int* gate, int allow_shift, double shift_scale,
                                                        int* gate_out, double gate_tol) {
    __shared__ __attribute__((aligned(16))) RowBuf rowb[2];
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
    const int64_t ps = (int64_t)w * w;
    if (gate_out) {
        // the gate of a second CholeskyQR round, formed here: *gate_out = 1 when max |G - I|
        // exceeds gate_tol or is not finite (then factor), else 0 (and nothing more to do)
        __shared__ double gred[kThreads / 64];
        double mx = 0.0;
        for (int64_t e = tid; e < ps; e += kThreads) {
            const Q4 v = ld4(G, ps, e);
            const double d = (e / w == e % w) ? v.w - 1.0 : v.w;
            const double a = fmax(fmax(fabs(d), fabs(v.x)), fmax(fabs(v.y), fabs(v.z)));
            mx = (a > mx || a != a) ? a : mx;     // a NaN sticks
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double t = __shfl_xor(mx, o, 64);
            mx = (t > mx || t != t) ? t : mx;
        }
        if ((tid & 63) == 0) gred[tid >> 6] = mx;
        __syncthreads();
        double m = gred[0];
        for (int i = 1; i < kThreads / 64; i++) m = (gred[i] > m || gred[i] != gred[i]) ? gred[i] : m;
        const int go = (m <= gate_tol) ? 0 : 1;
        if (tid == 0) *gate_out = go;
        if (!go) return;                           // uniform
    }
    Q4 g[NB][NB];
    int shifted, failed;
    chol_factor<NB>(g, G, w, ps, w, allow_shift, shift_scale, rowb, shifted, failed);
    if (tid == 0) {
        if (shift_out) *shift_out = shifted;
        if (failed) atomicOr(status, 2);
    }
    // R in planes, and its upper triangle packed by rows with the four components of an entry
    // side by side (the layout the triangular solve stages)
    typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int ri = 0; ri < NB; ri++)
#pragma unroll
        for (int ci = 0; ci < NB; ci++) {
            const int a = ty + 32 * ri, b = tx + 32 * ci;
            if (a >= w || b >= w) continue;
            const bool up = ci >= ri && b >= a;
            st4(Rout, ps, (int64_t)a * w + b, up ? g[ri][ci] : Q4{0, 0, 0, 0});
            if (up) {
                d2* o = reinterpret_cast<d2*>(Rpk) + 2 * upk(a, b, w);
                o[0] = d2{g[ri][ci].w, g[ri][ci].x};
                o[1] = d2{g[ri][ci].y, g[ri][ci].z};
            }
        }
}

// Cholesky of order w <= 32 NB in place inside larger matrices: G (row stride ldg, plane stride
// gps), G + shift I = R^H R, R into Rout (row stride ldr, plane stride rps) with zeros below the
// diagonal; with band_w > 0 the block sits at column band_off of a row band of width band_w,
// whose other columns (rows 0 .. w-1 of the block) are set to zero in Rout and in Rinv (ldx, xps),
// the band of the inverse that k_tri_inv fills at the block's columns.  The factor comes from
// chol_factor.
template <int NB>
__global__ __launch_bounds__(kThreads) void k_chol_fac(const double* __restrict__ G, int64_t ldg, int64_t gps, int w,
                                                        double* __restrict__ Rout, int64_t ldr, int64_t rps,
                                                        double* __restrict__ Rinv, int64_t ldx, int64_t xps,
                                                        int64_t band_off, int64_t band_w, int* status, int* shift_out,
                                                        const int* gate, int allow_shift, double shift_scale) {
    __shared__ __attribute__((aligned(16))) RowBuf rowb[2];
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
    Q4 g[NB][NB];
    int shifted, failed;
    chol_factor<NB>(g, G, ldg, gps, w, allow_shift, shift_scale, rowb, shifted, failed);
    if (tid == 0) {
        if (shift_out) *shift_out = shifted;
        if (failed) atomicOr(status, 2);
    }
#pragma unroll
    for (int ri = 0; ri < NB; ri++)
#pragma unroll
        for (int ci = 0; ci < NB; ci++) {
            const int a = ty + 32 * ri, b = tx + 32 * ci;
            if (a >= w || b >= w) continue;
            const bool up = ci >= ri && b >= a;
            st4(Rout, rps, (int64_t)a * ldr + b, up ? g[ri][ci] : Q4{0, 0, 0, 0});
        }
    // the rest of the row band
    if (band_w > 0) {
        const int64_t other = band_w - w;
        for (int64_t e = tid; e < (int64_t)w * other; e += kThreads) {
            const int64_t a = e / other, o = e - a * other;
            const int64_t cb = o < band_off ? o - band_off : o - band_off + w;   // column relative to the block
            st4(Rout, rps, a * ldr + cb, Q4{0, 0, 0, 0});
            st4(Rinv, xps, a * ldx + cb, Q4{0, 0, 0, 0});
        }
    }
}

// R^{-1} of an upper triangular R of order w <= kRegMax (row stride ldr, plane stride rps) into
// Rinv (ldx, xps), zeros below the diagonal.  Column c = 4 blockIdx.x + (wave) is the back
// substitution R x = e_c in one wave, whose lanes hold rows i = lane and lane + 64: step t (c down
// to 0, the same for every lane) finishes x_t = acc_t / r_tt on lane t and reads it on every lane,
// and the rows i < t take r_it x_t off.  No lane of a wave idles on another's column, and the
// columns run on ceil(w / 4) workgroups.  A workgroup first stages columns 0 .. (its last column)
// of R in LDS, packed by columns with the four components of an entry side by side.  A zero or
// negative diagonal entry (a failed factorization) takes 0 for its reciprocal.
__global__ __launch_bounds__(256) void k_tri_inv(const double* __restrict__ R, int64_t ldr, int64_t rps, int w,
                                                 double* __restrict__ Rinv, int64_t ldx, int64_t xps, const int* gate) {
    constexpr int NP = kRegMax * (kRegMax + 1) / 2;
    __shared__ __attribute__((aligned(16))) double sR[4 * NP];
    __shared__ double sdi[kRegMax];
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int c0 = 4 * (int)blockIdx.x;
    const int n = (c0 + 4 < w ? c0 + 4 : w);                 // columns 0 .. n-1 of R are read
    // consecutive threads read along a row of R; four entries per thread are in flight at once
    for (int e0 = 0; e0 < n * n; e0 += 4 * 256) {
        Q4 v[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int e = e0 + q * 256 + tid;
            const int a = e / n, t = e - a * n;
            const int64_t o = (e < n * n && t >= a) ? (int64_t)a * ldr + t : 0;
            v[q] = Q4{R[o], R[rps + o], R[2 * rps + o], R[3 * rps + o]};
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int e = e0 + q * 256 + tid;
            const int a = e / n, t = e - a * n;
            if (e < n * n && t >= a) {
                sti(sR, t * (t + 1) / 2 + a, v[q]);
                if (t == a) sdi[a] = v[q].w > 0.0 ? 1.0 / v[q].w : 0.0;
            }
        }
    }
    __syncthreads();
    const int c = c0 + wave;
    if (c >= w) return;                                      // uniform over the wave
    Q4 acc0 = lane == c ? Q4{1, 0, 0, 0} : Q4{0, 0, 0, 0};
    Q4 acc1 = lane + 64 == c ? Q4{1, 0, 0, 0} : Q4{0, 0, 0, 0};
    // the LDS operands of step t - 1 are read during step t
    const Q4 zero{0, 0, 0, 0};
    auto col = [&](int t, int i) { return ldi(sR, t * (t + 1) / 2 + (i < t ? i : t)); };
    double dn = sdi[c];
    Q4 r0n = col(c, lane), r1n = c >= 64 ? col(c, lane + 64) : zero;
    for (int t = c; t >= 0; t--) {
        const double d = dn;
        const Q4 r0 = r0n, r1 = r1n;
        if (t > 0) {
            dn = sdi[t - 1];
            r0n = col(t - 1, lane);
            if (t - 1 >= 64) r1n = col(t - 1, lane + 64);
        }
        const Q4 v = qsel(t < 64, acc0, acc1);
        const int src = t & 63;
        const Q4 x{bcast(v.w, src) * d, bcast(v.x, src) * d, bcast(v.y, src) * d, bcast(v.z, src) * d};
        acc0 = qsel(lane < t, qfms(acc0, r0, x), qsel(lane == t, x, acc0));
        if (t >= 64) acc1 = qsel(lane + 64 < t, qfms(acc1, r1, x), qsel(lane + 64 == t, x, acc1));
    }
    // rows past c hold zeros
    if (lane < w) st4(Rinv, xps, (int64_t)lane * ldx + c, acc0);
    if (lane + 64 < w) st4(Rinv, xps, (int64_t)(lane + 64) * ldx + c, acc1);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// lane n of each 16-lane row, to the whole row (DPP row_newbcast)
template <int N>
__device__ __forceinline__ Q4 row_bcast(Q4 q) {
    return Q4{dpp<0x150 + N>(q.w), dpp<0x150 + N>(q.x), dpp<0x150 + N>(q.y), dpp<0x150 + N>(q.z)};
}

// Q = Y R^{-1} by forward substitution along each row (q R = y): R upper triangular FP64
// (w x w planes, ld w, w <= kRegMax), Y and Q FP32 planes (Q may alias Y).  One 16-lane group
// per row, lane s owning columns s + 16 u (u < NU); the finished q_t is broadcast to the group
// and subtracted, times row t of R, from the later columns (16 fused multiply-adds per
// quaternion).  R's upper triangle is staged in LDS packed by rows with the four components of
// an entry side by side (two 16-byte reads per entry; dynamic size, w (w + 1) / 2 entries).
constexpr int kTrsmRows = 16;   // rows per 256-thread workgroup
__device__ __forceinline__ Q4 ldr(const double* sR, int i) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 lo = reinterpret_cast<const d2*>(sR)[2 * i], hi = reinterpret_cast<const d2*>(sR)[2 * i + 1];
    return Q4{lo[0], lo[1], hi[0], hi[1]};
}
// columns t = 16 TB + TT of the substitution: q_t = acc_t / r_tt on lane TT, broadcast over the
// row's 16 lanes, then acc_c -= q_t r_tc for the later columns c > t.  Branch-free, so that the
// LDS reads of a step are issued together: the later blocks (u > TB) update every lane (lanes
// past w read row t at column w - 1 and hold values that are never stored or broadcast), and
// block TB keeps its finished columns by a select.
template <int NU, int TB, int TT>
__device__ __forceinline__ void trsm_step(Q4 (&acc)[NU], const double* sR, const double* sinv, int s, int w) {
    constexpr int t = 16 * TB + TT;
    Q4 r[NU];
#pragma unroll
    for (int u = TB; u < NU; u++) r[u] = ldr(sR, upk(t, min(s + 16 * u, w - 1), w));
    const Q4 q = row_bcast<TT>(qscale(acc[TB], sinv[t]));
    const Q4 nb = qfms(acc[TB], q, r[TB]);
    acc[TB] = qsel(s > TT, nb, qsel(s == TT, q, acc[TB]));
#pragma unroll
    for (int u = TB + 1; u < NU; u++) acc[u] = qfms(acc[u], q, r[u]);
}
template <int NU, int TB, int TT = 0>
__device__ __forceinline__ void trsm_block(Q4 (&acc)[NU], const double* sR, const double* sinv, int s, int w) {
    if constexpr (TT < 16) {
        if (16 * TB + TT >= w) return;
        trsm_step<NU, TB, TT>(acc, sR, sinv, s, w);
        trsm_block<NU, TB, TT + 1>(acc, sR, sinv, s, w);
    }
}
template <int NU, int TB = 0>
__device__ __forceinline__ void trsm_all(Q4 (&acc)[NU], const double* sR, const double* sinv, int s, int w) {
    if constexpr (TB < NU) {
        trsm_block<NU, TB>(acc, sR, sinv, s, w);
        trsm_all<NU, TB + 1>(acc, sR, sinv, s, w);
    }
}

template <int NU>
__global__ __launch_bounds__(256) void k_trsm(const float* Y, int64_t ldy, int64_t yps, float* Q, int64_t ldq,
                                              int64_t qps, const double* __restrict__ Rpk, int w, int64_t rows,
                                              const int* gate) {
    extern __shared__ __attribute__((aligned(16))) double dyn[];
    const int pps = w * (w + 1) / 2;
    double* sR = dyn;               // pps entries of four components
    double* sinv = dyn + 4 * pps;   // w
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x, s = tid & 15;
    // staging: a straight copy of the packed triangle, sixteen 16-byte loads in flight per
    // thread (one round for w <= 63)
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* src = reinterpret_cast<const d2*>(Rpk);
    d2* dst = reinterpret_cast<d2*>(sR);
    const int n2 = 2 * pps;
    for (int base = 0; base < n2; base += 16 * 256) {
        d2 v[16];
#pragma unroll
        for (int u = 0; u < 16; u++) v[u] = src[min(base + u * 256 + tid, n2 - 1)];
#pragma unroll
        for (int u = 0; u < 16; u++)
            if (base + u * 256 + tid < n2) dst[base + u * 256 + tid] = v[u];
    }
    for (int t = tid; t < w; t += 256) sinv[t] = 1.0 / Rpk[4 * upk(t, t, w)];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * kTrsmRows + (tid >> 4);
    const bool act = row < rows;
    Q4 acc[NU];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int c = s + 16 * u;
        acc[u] = Q4{0, 0, 0, 0};
        if (act && c < w) {
            const int64_t o = row * ldy + c;
            acc[u] = Q4{(double)Y[o], (double)Y[yps + o], (double)Y[2 * yps + o], (double)Y[3 * yps + o]};
        }
    }
    trsm_all<NU>(acc, sR, sinv, s, w);
    if (act) {
#pragma unroll
        for (int u = 0; u < NU; u++) {
            const int c = s + 16 * u;
            if (c < w) {
                const int64_t o = row * ldq + c;
                Q[o] = (float)acc[u].w; Q[qps + o] = (float)acc[u].x;
                Q[2 * qps + o] = (float)acc[u].y; Q[3 * qps + o] = (float)acc[u].z;
            }
        }
    }
}

// Rout = R2 R1 for upper triangular factors of order w <= kRegMax: one 16 x 16 tile per
// workgroup, the row strip of R2 and the column strip of R1 staged in LDS.
__global__ __launch_bounds__(256) void k_rmul_tile(const double* __restrict__ R2, const double* __restrict__ R1,
                                                   double* __restrict__ Rout, int w, const int* gate) {
    __shared__ double sa[4 * 16 * kRegMax];   // sa[p][r][t] rows a0.. of R2
    __shared__ double sb[4 * kRegMax * 16];   // sb[p][t][c] columns b0.. of R1
    if (gate && *gate == 0) return;
    const int64_t ps = (int64_t)w * w;
    const int a0 = blockIdx.y * 16, b0 = blockIdx.x * 16;
    const int tid = threadIdx.x, aa = tid >> 4, bq = tid & 15;
    const int a = a0 + aa, b = b0 + bq;
    if (a0 > b0 + 15) {                       // tile below the diagonal
        if (a < w && b < w) st4(Rout, ps, (int64_t)a * w + b, Q4{0, 0, 0, 0});
        return;
    }
    const int n = 16 * w;
    for (int base = 0; base < n; base += 4 * 256) {
        Q4 va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = min(base + u * 256 + tid, n - 1);
            const int r = e / w, t = e - r * w;       // sa: row a0 + r, column t
            va[u] = ld4(R2, ps, (int64_t)min(a0 + r, w - 1) * w + t);
            const int t2 = e >> 4, c = e & 15;        // sb: row t2, column b0 + c
            vb[u] = ld4(R1, ps, (int64_t)t2 * w + min(b0 + c, w - 1));
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = base + u * 256 + tid;
            if (e >= n) continue;
            const int r = e / w, t = e - r * w;
            stp<16 * kRegMax>(sa, r * kRegMax + t, a0 + r < w ? va[u] : Q4{0, 0, 0, 0});
            const int t2 = e >> 4, c = e & 15;
            stp<16 * kRegMax>(sb, t2 * 16 + c, b0 + c < w ? vb[u] : Q4{0, 0, 0, 0});
        }
    }
    __syncthreads();
    if (a >= w || b >= w) return;
    Q4 acc{0, 0, 0, 0};
    for (int t = a; t <= b; t++)
        acc = qadd(acc, qmul(ldp<16 * kRegMax>(sa, aa * kRegMax + t), ldp<16 * kRegMax>(sb, t * 16 + bq)));
    if (a == b) acc.x = acc.y = acc.z = 0.0;   // the product of real diagonals is real
    st4(Rout, ps, (int64_t)a * w + b, acc);
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

// ------------------------------------------------------------------------------------------
// Pieces of the blocked factorization of orders above kRegMax (the block steps are driven from
// the host side of the library: diagonal blocks by k_chol_fac and k_tri_inv, the rest as FP64 products).

// W = G with a real diagonal, plus shift I where shift = shift_scale * trace(G) (at least 1e-300)
// when `shifted`; nothing when gate && *gate == 0.
__global__ __launch_bounds__(256) void k_chol_prep(const double* __restrict__ G, int w, double* __restrict__ W,
                                                   const int* gate, int shifted, double shift_scale) {
    if (gate && *gate == 0) return;
    double shift = 0.0;
    if (shifted) {
        double tr = 0.0;
        for (int i = 0; i < w; i++) tr += G[(int64_t)i * w + i];
        shift = shift_scale * tr;
        if (!(shift > 0.0)) shift = 1e-300;
    }
    const int64_t ps = (int64_t)w * w;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < ps; e += (int64_t)gridDim.x * 256) {
        Q4 v = ld4(G, ps, e);
        if (e / w == e % w) { v.w += shift; v.x = v.y = v.z = 0.0; }
        st4(W, ps, e, v);
    }
}

// dst (rows x cols FP64 planes) = src; nothing when gate && *gate == 0.
__global__ __launch_bounds__(256) void k_copy_f64_planes(const double* __restrict__ src, int64_t lds, int64_t sps,
                                                         double* __restrict__ dst, int64_t ldd, int64_t dps,
                                                         int64_t rows, int64_t cols, const int* gate) {
    if (gate && *gate == 0) return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / cols, c = e - r * cols;
        st4(dst, dps, r * ldd + c, ld4(src, sps, r * lds + c));
    }
}

__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ p, int64_t count, const int* gate) {
    if (gate && *gate == 0) return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) p[e] = 0.0;
}

// *gate_out = 1 when max |G - I| over the four planes of a w x w Gram exceeds tol (or is not
// finite), else 0; always 0 when gate_in is given and *gate_in == 0.  *gate_not (if given) is
// the opposite.  One workgroup.
__global__ __launch_bounds__(1024) void k_orth_gate(const double* __restrict__ G, int w, double tol, int* gate_out,
                                                   const int* gate_in, int* gate_not) {
    __shared__ double red[16];
    const int tid = threadIdx.x;
    if (gate_in && *gate_in == 0) {
        if (tid == 0) {
            *gate_out = 0;
            if (gate_not) *gate_not = 1;
        }
        return;
    }
    const int64_t ps = (int64_t)w * w;
    double mx = 0.0;
    auto visit = [&](const Q4& v, bool diag) {
        const double d = diag ? v.w - 1.0 : v.w;
        const double a = fmax(fmax(fabs(d), fabs(v.x)), fmax(fabs(v.y), fabs(v.z)));
        mx = (a > mx || a != a) ? a : mx;     // a NaN sticks
    };
    if (ps < ((int64_t)1 << 31)) {
        // 32-bit indices (a 64-bit division per entry cost more than the loads)
        for (int e = tid; e < (int)ps; e += 1024) {
            const int r = e / w;
            visit(ld4(G, ps, e), e == r * w + r);
        }
    } else {
        for (int64_t e = tid; e < ps; e += 1024) visit(ld4(G, ps, e), e / w == e % w);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(mx, o, 64);
        mx = (t > mx || t != t) ? t : mx;
    }
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = red[0];
        for (int i = 1; i < 16; i++) m = (red[i] > m || red[i] != red[i]) ? red[i] : m;
        *gate_out = (m <= tol) ? 0 : 1;
        if (gate_not) *gate_not = (m <= tol) ? 1 : 0;
    }
}

__global__ void k_flag_nonzero(int* dst, const int* src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src != 0 ? 1 : 0;
}

}  // namespace

int chol_lds_max() { return kRegMax; }
int chol_reg_max() { return kRegMax; }

hipError_t chol_reg_launch(const double* G, int64_t w, double* R, double* Rpk, int* status, int* shift_out,
                           const int* gate, int allow_shift, double shift_scale, hipStream_t st, int* gate_out,
                           double gate_tol) {
    if (w < 1 || w > kRegMax) return hipErrorInvalidValue;
    if (w <= 64)
        hipLaunchKernelGGL(k_chol_reg<2>, dim3(1), dim3(kThreads), 0, st, G, (int)w, R, Rpk, status, shift_out, gate,
                           allow_shift, shift_scale, gate_out, gate_tol);
    else
        hipLaunchKernelGGL(k_chol_reg<3>, dim3(1), dim3(kThreads), 0, st, G, (int)w, R, Rpk, status, shift_out, gate,
                           allow_shift, shift_scale, gate_out, gate_tol);
    return hipGetLastError();
}

hipError_t trsm_launch(const float* Y, int64_t ldy, int64_t yps, float* Q, int64_t ldq, int64_t qps,
                       const double* Rpk, int64_t w, int64_t rows, const int* gate, hipStream_t st) {
    if (w < 1 || w > kRegMax || rows < 0) return hipErrorInvalidValue;
    if (rows == 0) return hipSuccess;
    const int64_t blocks = (rows + kTrsmRows - 1) / kTrsmRows;
    const size_t lds = (size_t)(4 * (w * (w + 1) / 2) + w) * sizeof(double);
    if (w <= 64)
        hipLaunchKernelGGL(k_trsm<4>, dim3((unsigned)blocks), dim3(256), lds, st, Y, ldy, yps, Q, ldq, qps, Rpk, (int)w,
                           rows, gate);
    else
        hipLaunchKernelGGL(k_trsm<6>, dim3((unsigned)blocks), dim3(256), lds, st, Y, ldy, yps, Q, ldq, qps, Rpk, (int)w,
                           rows, gate);
    return hipGetLastError();
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 1024) g = 1024;
    return (unsigned)(g < 1 ? 1 : g);
}

hipError_t chol_prep_launch(const double* G, int64_t w, double* W, const int* gate, int shifted, double shift_scale,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_chol_prep, dim3(grid_for(w * w)), dim3(256), 0, st, G, (int)w, W, gate, shifted, shift_scale);
    return hipGetLastError();
}

hipError_t copy_f64_planes_launch(const double* src, int64_t lds, int64_t sps, double* dst, int64_t ldd, int64_t dps,
                                  int64_t rows, int64_t cols, const int* gate, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f64_planes, dim3(grid_for(rows * cols)), dim3(256), 0, st, src, lds, sps, dst, ldd, dps,
                       rows, cols, gate);
    return hipGetLastError();
}

hipError_t zero_f64_launch(double* p, int64_t count, const int* gate, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(count)), dim3(256), 0, st, p, count, gate);
    return hipGetLastError();
}


hipError_t orth_gate_launch(const double* G, int64_t w, double tol, int* gate_out, const int* gate_in,
                            hipStream_t st, int* gate_not) {
    if (w < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_orth_gate, dim3(1), dim3(1024), 0, st, G, (int)w, tol, gate_out, gate_in, gate_not);
    return hipGetLastError();
}

hipError_t flag_nonzero_launch(int* dst, const int* src, hipStream_t st) {
    hipLaunchKernelGGL(k_flag_nonzero, dim3(1), dim3(64), 0, st, dst, src);
    return hipGetLastError();
}

hipError_t chol_inv_launch(const double* G, int64_t ldg, int64_t gps, int64_t w, double* R, int64_t ldr, int64_t rps,
                           double* Rinv, int64_t ldi, int64_t ips, int64_t band_off, int64_t band_w, int* status,
                           int* shift_out, const int* gate, int allow_shift, double shift_scale, hipStream_t st) {
    if (w < 1 || w > kRegMax || !R || !Rinv || (band_w > 0 && (band_off < 0 || band_off + w > band_w)))
        return hipErrorInvalidValue;
    if (w <= 64)
        hipLaunchKernelGGL(k_chol_fac<2>, dim3(1), dim3(kThreads), 0, st, G, ldg, gps, (int)w, R, ldr, rps, Rinv, ldi,
                           ips, band_off, band_w, status, shift_out, gate, allow_shift, shift_scale);
    else
        hipLaunchKernelGGL(k_chol_fac<3>, dim3(1), dim3(kThreads), 0, st, G, ldg, gps, (int)w, R, ldr, rps, Rinv, ldi,
                           ips, band_off, band_w, status, shift_out, gate, allow_shift, shift_scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tri_inv, dim3((unsigned)((w + 3) / 4)), dim3(256), 0, st, (const double*)R, ldr, rps, (int)w,
                       Rinv, ldi, ips, gate);
    return hipGetLastError();
}

hipError_t chol_launch(const double* G, int64_t w, double* R, double* Rinv, const double* Rprev, double* work,
                       int* status, int* shift_out, const int* gate, int allow_shift, double shift_scale,
                       hipStream_t st) {
    if (w < 1 || w > kRegMax) return hipErrorInvalidValue;   // larger orders: the blocked factorization
    // with an earlier factor: the new factor goes to `work`, then R = work * Rprev
    double* Rnew = Rprev ? work : R;
    const int64_t ps = w * w;
    hipError_t e = chol_inv_launch(G, w, ps, w, Rnew, w, ps, Rinv ? Rinv : work + 4 * ps, w, ps, 0, 0, status,
                                   shift_out, gate, allow_shift, shift_scale, st);
    if (e != hipSuccess || !Rprev) return e;
    const int64_t n = w * w;
    hipLaunchKernelGGL(k_rmul, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const double*)Rnew, Rprev, R,
                       (int)w, gate);
    return hipGetLastError();
}

hipError_t rmul_launch(const double* R2, const double* R1, double* Rout, int64_t w, const int* gate,
                       hipStream_t st) {
    if (w <= kRegMax) {
        const unsigned t = (unsigned)((w + 15) / 16);
        hipLaunchKernelGGL(k_rmul_tile, dim3(t, t), dim3(256), 0, st, R2, R1, Rout, (int)w, gate);
        return hipGetLastError();
    }
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
