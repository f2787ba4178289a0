// Gaussian quaternion sketch Omega (Sec. 2, Def. of a Gaussian quaternion matrix).
//
// Entry (i, j) is a pure function of (seed, i, j): Philox4x32-10 (Salmon et al., SC'11) at
// counter (i, j, 0, 0) under key (seed mod 2^32, seed div 2^32) gives four 32-bit words; each
// becomes u = (2 (x >> 9) + 1) 2^-24 in (0, 1) (exact), and two Box-Muller pairs give the four
// planes.  The transcendental functions are evaluated in FP64 from their series with a fixed
// sequence of IEEE operations (explicit fma, contraction off), so that any correct
// implementation of the same definition on any IEEE machine produces the same FP32 values.
// One thread per entry; the work is ALU-bound and tiny next to a pass over A.
#include <cmath>

#include "common.h"

namespace qlra_impl {
namespace {

#pragma clang fp contract(off)

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// 1 / d for d in [1.5, 2.5]: Newton y <- y + y (1 - d y) from 0.5, five steps.
__device__ __forceinline__ double recip_near2(double d) {
    double y = 0.5;
#pragma unroll
    for (int it = 0; it < 5; it++) {
        const double e = __builtin_fma(-d, y, 1.0);
        y = __builtin_fma(y, e, y);
    }
    return y;
}

// ln u for u in (0, 1]: u = m 2^e, m in [1, 2), folded to m in (0.707, 1.414]; then
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), by the odd series up to s^25.
__device__ __forceinline__ double log_unit(double u) {
    const uint64_t b = __double_as_longlong(u);
    int64_t e = (int64_t)((b >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    const double f = m - 1.0;
    const double s = f * recip_near2(2.0 + f);
    const double z = s * s;
    double p = 1.0 / 25.0;
    p = __builtin_fma(p, z, 1.0 / 23.0);
    p = __builtin_fma(p, z, 1.0 / 21.0);
    p = __builtin_fma(p, z, 1.0 / 19.0);
    p = __builtin_fma(p, z, 1.0 / 17.0);
    p = __builtin_fma(p, z, 1.0 / 15.0);
    p = __builtin_fma(p, z, 1.0 / 13.0);
    p = __builtin_fma(p, z, 1.0 / 11.0);
    p = __builtin_fma(p, z, 1.0 / 9.0);
    p = __builtin_fma(p, z, 1.0 / 7.0);
    p = __builtin_fma(p, z, 1.0 / 5.0);
    p = __builtin_fma(p, z, 1.0 / 3.0);
    const double two_s = 2.0 * s;
    const double zp = z * p;
    const double l1p = __builtin_fma(two_s, zp, two_s);
    return __builtin_fma((double)e, 0.6931471805599453, l1p);
}

// sqrt x for x > 0: Newton on 1/sqrt(x) from an exponent-halving integer guess, then one
// Newton correction of s = x y.
__device__ __forceinline__ double sqrt_pos(double x) {
    double y = __longlong_as_double(0x5FE6EB50C7B537A9ll - (__double_as_longlong(x) >> 1));
    const double h = 0.5 * x;
#pragma unroll
    for (int it = 0; it < 5; it++) {
        const double t = y * y;
        const double r = h * t;
        const double c = 1.5 - r;
        y = y * c;
    }
    const double s = x * y;
    const double res = __builtin_fma(-s, s, x);
    const double hy = 0.5 * y;
    return __builtin_fma(hy, res, s);
}

// sin, cos of 2 pi u, u in [0, 1) with at most 24 significant bits: quadrant q = round(4u),
// exact remainder r = u - q/4, theta = 2 pi r; Taylor to theta^19 / theta^20.
__device__ __forceinline__ void sincos_2pi(double u, double* sn_out, double* cs_out) {
    const double q = floor(4.0 * u + 0.5);
    const double r = u - 0.25 * q;
    const double t = r * 6.283185307179586;
    const double z = t * t;
    double ps = -1.0 / 121645100408832000.0;
    ps = __builtin_fma(ps, z, 1.0 / 355687428096000.0);
    ps = __builtin_fma(ps, z, -1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, z, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, z, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, z, 1.0 / 362880.0);
    ps = __builtin_fma(ps, z, -1.0 / 5040.0);
    ps = __builtin_fma(ps, z, 1.0 / 120.0);
    ps = __builtin_fma(ps, z, -1.0 / 6.0);
    const double tz = t * z;
    const double sn = __builtin_fma(tz, ps, t);
    double pc = 1.0 / 2432902008176640000.0;
    pc = __builtin_fma(pc, z, -1.0 / 6402373705728000.0);
    pc = __builtin_fma(pc, z, 1.0 / 20922789888000.0);
    pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);
    pc = __builtin_fma(pc, z, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, z, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, z, 1.0 / 40320.0);
    pc = __builtin_fma(pc, z, -1.0 / 720.0);
    pc = __builtin_fma(pc, z, 1.0 / 24.0);
    pc = __builtin_fma(pc, z, -1.0 / 2.0);
    const double cs = __builtin_fma(z, pc, 1.0);
    switch (((int)q) & 3) {
        case 0: *sn_out = sn; *cs_out = cs; break;
        case 1: *sn_out = cs; *cs_out = -sn; break;
        case 2: *sn_out = -sn; *cs_out = -cs; break;
        default: *sn_out = -cs; *cs_out = sn; break;
    }
}

__device__ __forceinline__ double unit_open(uint32_t x) {
    return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0);
}

__global__ __launch_bounds__(256) void k_omega(uint32_t k0, uint32_t k1, int64_t n, int64_t l,
                                               float* Om, int64_t ld, int64_t ps, int real_only) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * l) return;
    const int64_t i = idx / l, j = idx - i * l;
    uint32_t c[4] = {(uint32_t)i, (uint32_t)j, 0u, 0u};
    philox4x32_10(c, k0, k1);
    float z[4];
#pragma unroll
    for (int pair = 0; pair < 2; pair++) {
        const double ua = unit_open(c[2 * pair]), ub = unit_open(c[2 * pair + 1]);
        const double rad = sqrt_pos(-2.0 * log_unit(ua));
        double sn, cs;
        sincos_2pi(ub, &sn, &cs);
        const double z0 = rad * cs, z1 = rad * sn;
        z[2 * pair] = (float)z0;
        z[2 * pair + 1] = (float)z1;
    }
    float* o = Om + i * ld + j;
    o[0] = z[0];
    o[ps] = real_only ? 0.0f : z[1];
    o[2 * ps] = real_only ? 0.0f : z[2];
    o[3 * ps] = real_only ? 0.0f : z[3];
}

// The structured sketch: a subsampled randomized Hadamard transform D H S / sqrt(l) (real plane;
// the others zero).  d_i = -1 when bit 0 of word 0 of Philox at counter (i, 0, 2, 0) is set, else
// +1; column j samples column s_j = pi(j) of the +-1 Hadamard matrix of order n_pad (entry
// (-1)^popcount(i & s_j)), pi a keyed four-round Feistel permutation on 2h bits (round r maps
// (L, R) to (R, L xor F), F = word 0 of Philox at counter (R, r, 3, 0) masked to h bits) with
// cycle walking back into [0, n_pad).
__device__ __forceinline__ uint32_t feistel4(uint32_t v, int h, uint32_t mask, uint32_t k0, uint32_t k1) {
    uint32_t L = v >> h, R = v & mask;
#pragma unroll
    for (uint32_t r = 0; r < 4; r++) {
        uint32_t c[4] = {R, r, 3u, 0u};
        philox4x32_10(c, k0, k1);
        const uint32_t t = L ^ (c[0] & mask);
        L = R;
        R = t;
    }
    return (L << h) | R;
}

__global__ __launch_bounds__(256) void k_omega_srht(uint32_t k0, uint32_t k1, int64_t n, int64_t l, uint32_t n_pad,
                                                    int h, float scale, float* __restrict__ Om, int64_t ld,
                                                    int64_t ps) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * l) return;
    const int64_t i = e / l, j = e - i * l;
    const uint32_t mask = (1u << h) - 1u;
    // the permutation's cycle through j returns below n_pad within 2^(2h) applications
    uint32_t sj = feistel4((uint32_t)j, h, mask, k0, k1);
    for (uint32_t walk = 0; sj >= n_pad && walk < (1u << (2 * h)); walk++) sj = feistel4(sj, h, mask, k0, k1);
    uint32_t c[4] = {(uint32_t)i, 0u, 2u, 0u};
    philox4x32_10(c, k0, k1);
    const bool neg = ((c[0] & 1u) != 0) != ((__builtin_popcount((uint32_t)i & sj) & 1) != 0);
    const int64_t o = i * ld + j;
    Om[o] = neg ? -scale : scale;
    Om[ps + o] = 0.0f;
    Om[2 * ps + o] = 0.0f;
    Om[3 * ps + o] = 0.0f;
}

}  // namespace

hipError_t omega_srht_launch(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t ps, hipStream_t st) {
    const int64_t total = n * l;
    if (total == 0) return hipSuccess;
    if (n > (int64_t)1 << 30 || l > n) return hipErrorInvalidValue;
    uint32_t n_pad = 1;
    int bits = 0;
    while ((int64_t)n_pad < n) {
        n_pad <<= 1;
        bits++;
    }
    const int h = (bits + 1) / 2;
    const float scale = (float)(1.0 / std::sqrt((double)l));
    hipLaunchKernelGGL(k_omega_srht, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), n, l, n_pad, h, scale, Om, ld, ps);
    return hipGetLastError();
}

hipError_t omega_launch(uint64_t seed, int64_t n, int64_t l, float* Om, int64_t ld, int64_t ps,
                        hipStream_t st, int real_only) {
    const int64_t total = n * l;
    if (total == 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_omega, dim3((unsigned)blocks), dim3(256), 0, st,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), n, l, Om, ld, ps, real_only);
    return hipGetLastError();
}

}  // namespace qlra_impl
