/*
 * qlra_oracle.c -- plain FP64 CPU oracle for the pass-efficient randomized
 * low-rank approximation of quaternion matrices (arXiv 2507.13731).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  It is written to be
 * read against the paper, not to be fast: plain loops over quaternion structs,
 * FP64 everywhere, OpenMP only over independent output rows.  Build with
 * -ffp-contract=off so the Gaussian generator's operation sequence is exactly
 * the one written here.
 *
 * What each part follows, and what pins it (tests/test_oracle_*.py):
 *   q_mul ............ Sec. 2, eq. (1).  Pinned by the unit rules i^2=j^2=k^2=ijk=-1
 *                      and by the complex-adjoint homomorphism chi(AB)=chi(A)chi(B)
 *                      against numpy complex matmul.
 *   qo_qgemm(_adj) ... Sec. 2 (matrix product, conjugate transpose).  Same pins.
 *   qo_philox4x32_10 . Philox4x32-10 as published by Salmon et al. (SC'11).
 *                      Pinned by the published known-answer vectors.
 *   qo_log_unit, qo_sqrt_pos, qo_sincos_2pi
 *                      series written from their Taylor/atanh expansions and
 *                      Newton's method.  Pinned against libm within a few ulp.
 *   qo_omega ......... Sec. 2, Def. (Gaussian quaternion matrix) + Box-Muller.
 *                      Pinned by moments/independence of the planes.
 *   qo_qr ............ eq. (QQR) by Householder reflections.  Pinned by
 *                      Q^H Q = I, QR = Y, triangularity, real diagonal >= 0.
 *   qo_qsvd .......... eq. (qsvd) through the complex adjoint chi(R), one-sided
 *                      Jacobi.  Pinned by numpy's LAPACK SVD of chi(R).
 *   Alg. 1-4 ......... Sec. 3 (Alg. 1, Alg. 2) and Sec. 5 (Alg. 3, Alg. 4).
 *                      Pinned by planted-rank exact recovery, Eckart-Young lower
 *                      bounds, the full QSVD optimum on tiny inputs, the
 *                      equivalences Alg2(v=2q+2)=Alg1(q), Alg4(v<4)=Alg2,
 *                      Alg4(v=2q+2)=Alg3(q), range inclusion (Sec. 5 Lemma),
 *                      and the error bound of Thm. (flex-Krylov) on averages.
 *   per-pass error ... not in the paper; the identity
 *                      ||A - Q1 [R]_k Q2^H||_F^2 = ||A||_F^2 - sum_{j<=k} sigma_j(R)^2
 *                      holds whenever the view's input basis is orthonormal.
 *                      Pinned against the directly computed residual.
 */
#include "qlra_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Quaternions (Sec. 2)                                                      */
/* ------------------------------------------------------------------------ */

typedef struct { double w, x, y, z; } quat;   /* w + x i + y j + z k */

static const quat QZERO = {0.0, 0.0, 0.0, 0.0};

/* Hamilton product, eq. (1). */
static quat q_mul(quat a, quat b) {
    quat r;
    r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    r.x = a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y;
    r.y = a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x;
    r.z = a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w;
    return r;
}
static quat q_add(quat a, quat b) { quat r = {a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static quat q_sub(quat a, quat b) { quat r = {a.w - b.w, a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static quat q_conj(quat a) { quat r = {a.w, -a.x, -a.y, -a.z}; return r; }
static quat q_scale(quat a, double s) { quat r = {a.w * s, a.x * s, a.y * s, a.z * s}; return r; }
static double q_norm2(quat a) { return a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z; }
static double q_abs(quat a) { return sqrt(q_norm2(a)); }

/* A quaternion matrix, row-major array of structs. */
typedef struct { int64_t r, c; quat* d; } qmat;

static qmat qm_new(int64_t r, int64_t c) {
    qmat M; M.r = r; M.c = c;
    M.d = (quat*)calloc((size_t)(r * c > 0 ? r * c : 1), sizeof(quat));
    return M;
}
static void qm_free(qmat* M) { free(M->d); M->d = NULL; }
#define QM(M, i, j) ((M).d[(int64_t)(i) * (M).c + (j)])

static qmat qm_from_planes(const double* P, int64_t r, int64_t c) {
    qmat M = qm_new(r, c);
    const int64_t ps = r * c;
    for (int64_t i = 0; i < r; i++)
        for (int64_t j = 0; j < c; j++) {
            quat q = {P[i * c + j], P[ps + i * c + j], P[2 * ps + i * c + j], P[3 * ps + i * c + j]};
            QM(M, i, j) = q;
        }
    return M;
}
static void qm_to_planes(const qmat M, double* P) {
    const int64_t ps = M.r * M.c;
    for (int64_t i = 0; i < M.r; i++)
        for (int64_t j = 0; j < M.c; j++) {
            quat q = QM(M, i, j);
            P[i * M.c + j] = q.w; P[ps + i * M.c + j] = q.x;
            P[2 * ps + i * M.c + j] = q.y; P[3 * ps + i * M.c + j] = q.z;
        }
}

/* C = A B. */
static qmat qm_mul(const qmat A, const qmat B) {
    qmat C = qm_new(A.r, B.c);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A.r; i++)
        for (int64_t t = 0; t < A.c; t++) {
            quat a = QM(A, i, t);
            for (int64_t j = 0; j < B.c; j++) QM(C, i, j) = q_add(QM(C, i, j), q_mul(a, QM(B, t, j)));
        }
    return C;
}

/* C = A^H B, with (A^H)_{ji} = conj(A_{ij}) (Sec. 2). */
static qmat qm_adj_mul(const qmat A, const qmat B) {
    qmat C = qm_new(A.c, B.c);
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < A.c; j++)
        for (int64_t i = 0; i < A.r; i++) {
            quat a = q_conj(QM(A, i, j));
            for (int64_t t = 0; t < B.c; t++) QM(C, j, t) = q_add(QM(C, j, t), q_mul(a, QM(B, i, t)));
        }
    return C;
}

static double qm_fro2(const qmat A) {
    double s = 0.0;
    for (int64_t i = 0; i < A.r * A.c; i++) s += q_norm2(A.d[i]);
    return s;
}

/* Columns [c0, c0+w) of A. */
static qmat qm_cols(const qmat A, int64_t c0, int64_t w) {
    qmat C = qm_new(A.r, w);
    for (int64_t i = 0; i < A.r; i++)
        for (int64_t j = 0; j < w; j++) QM(C, i, j) = QM(A, i, c0 + j);
    return C;
}

/* ------------------------------------------------------------------------ */
/* Counter-based Gaussian generator                                          */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
 * published multipliers, the key bumped by the published Weyl constants
 * between rounds. */
void qo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint64_t d2u(double x) { uint64_t u; memcpy(&u, &x, 8); return u; }
static double u2d(uint64_t u) { double x; memcpy(&x, &u, 8); return x; }

/* 1/d for d in [1.5, 2.5] by Newton's iteration y <- y + y(1 - d y) from 0.5;
 * the error squares each step (0.25^32 after five). */
static double recip_1p5_2p5(double d) {
    double y = 0.5;
    for (int it = 0; it < 5; it++) {
        double e = fma(-d, y, 1.0);
        y = fma(y, e, y);
    }
    return y;
}

/* ln u, u in (0, 1] normal.  u = m 2^e with m in [1, 2); if m > sqrt 2 use
 * m/2 and e+1 so that f = m - 1 lies in [-0.293, 0.415].  Then
 * ln(1+f) = 2 atanh(s), s = f/(2+f), |s| < 0.172, by its odd series
 * 2 (s + s^3/3 + s^5/5 + ...), truncated after s^25 (< 1e-19 relative). */
double qo_log_unit(double u) {
    uint64_t b = d2u(u);
    int64_t e = (int64_t)((b >> 52) & 0x7ff) - 1023;
    double m = u2d((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > 1.4142135623730951) { m = m * 0.5; e = e + 1; }
    double f = m - 1.0;
    double s = f * recip_1p5_2p5(2.0 + f);
    double z = s * s;
    double p = 1.0 / 25.0;
    p = fma(p, z, 1.0 / 23.0);
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    double two_s = 2.0 * s;
    double l1p = fma(two_s, z * p, two_s);
    return fma((double)e, 0.6931471805599453, l1p);
}

/* sqrt x, x > 0 normal: reciprocal square root by Newton's iteration
 * y <- y (3/2 - (x/2) y^2) from an exponent-halving integer estimate, then one
 * Newton step on s = x y. */
double qo_sqrt_pos(double x) {
    double y = u2d(0x5FE6EB50C7B537A9ull - (d2u(x) >> 1));
    double h = 0.5 * x;
    for (int it = 0; it < 5; it++) {
        double t = y * y;
        double r = h * t;
        double c = 1.5 - r;
        y = y * c;
    }
    double s = x * y;
    double res = fma(-s, s, x);
    return fma(0.5 * y, res, s);
}

/* sin and cos of 2 pi u for u in [0, 1).  Quadrant q = round(4u) and the exact
 * remainder r = u - q/4 (|r| <= 1/8, exact because u carries at most 24
 * significant bits here); theta = 2 pi r in [-pi/4, pi/4]; Taylor series to
 * theta^19 (sin) and theta^20 (cos); then rotate by q quarter turns. */
void qo_sincos_2pi(double u, double* s_out, double* c_out) {
    double q = floor(4.0 * u + 0.5);
    double r = u - 0.25 * q;
    double t = r * 6.283185307179586;
    double z = t * t;
    double ps = -1.0 / 121645100408832000.0;          /* -1/19! */
    ps = fma(ps, z, 1.0 / 355687428096000.0);         /*  1/17! */
    ps = fma(ps, z, -1.0 / 1307674368000.0);          /* -1/15! */
    ps = fma(ps, z, 1.0 / 6227020800.0);              /*  1/13! */
    ps = fma(ps, z, -1.0 / 39916800.0);               /* -1/11! */
    ps = fma(ps, z, 1.0 / 362880.0);                  /*  1/9!  */
    ps = fma(ps, z, -1.0 / 5040.0);                   /* -1/7!  */
    ps = fma(ps, z, 1.0 / 120.0);                     /*  1/5!  */
    ps = fma(ps, z, -1.0 / 6.0);                      /* -1/3!  */
    double sn = fma(t * z, ps, t);
    double pc = 1.0 / 2432902008176640000.0;          /*  1/20! */
    pc = fma(pc, z, -1.0 / 6402373705728000.0);       /* -1/18! */
    pc = fma(pc, z, 1.0 / 20922789888000.0);          /*  1/16! */
    pc = fma(pc, z, -1.0 / 87178291200.0);            /* -1/14! */
    pc = fma(pc, z, 1.0 / 479001600.0);               /*  1/12! */
    pc = fma(pc, z, -1.0 / 3628800.0);                /* -1/10! */
    pc = fma(pc, z, 1.0 / 40320.0);                   /*  1/8!  */
    pc = fma(pc, z, -1.0 / 720.0);                    /* -1/6!  */
    pc = fma(pc, z, 1.0 / 24.0);                      /*  1/4!  */
    pc = fma(pc, z, -1.0 / 2.0);                      /* -1/2!  */
    double cs = fma(z, pc, 1.0);
    int qi = ((int)q) & 3;
    switch (qi) {
        case 0: *s_out = sn; *c_out = cs; break;
        case 1: *s_out = cs; *c_out = -sn; break;
        case 2: *s_out = -sn; *c_out = -cs; break;
        default: *s_out = -cs; *c_out = sn; break;
    }
}

/* 32-bit word -> uniform in (0, 1): (2 (x >> 9) + 1) 2^-24, exact. */
static double unit_open(uint32_t x) { return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0); }

/* Gaussian quaternion test matrix (Sec. 2, Def. of a Gaussian random matrix):
 * entry (i, j) takes Philox4x32-10 at counter (i, j, 0, 0) under key
 * (seed low 32 bits, seed high 32 bits); the four uniforms feed two Box-Muller
 * pairs: (u0, u1) -> planes 0, 1 and (u2, u3) -> planes 2, 3, each
 * (sqrt(-2 ln ua) cos(2 pi ub), sqrt(-2 ln ua) sin(2 pi ub)), rounded to FP32. */
void qo_omega(uint64_t seed, int64_t n, int64_t l, float* Om) {
    const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    const int64_t ps = n * l;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < l; j++) {
            uint32_t ctr[4] = {(uint32_t)i, (uint32_t)j, 0u, 0u}, x[4];
            qo_philox4x32_10(ctr, key, x);
            double z[4];
            for (int pair = 0; pair < 2; pair++) {
                double ua = unit_open(x[2 * pair]), ub = unit_open(x[2 * pair + 1]);
                double rad = qo_sqrt_pos(-2.0 * qo_log_unit(ua));
                double sn, cs;
                qo_sincos_2pi(ub, &sn, &cs);
                z[2 * pair] = rad * cs;
                z[2 * pair + 1] = rad * sn;
            }
            for (int pl = 0; pl < 4; pl++) Om[pl * ps + i * l + j] = (float)z[pl];
        }
}

/* ------------------------------------------------------------------------ */
/* Householder QR (eq. (QQR); Householder reflections as in Bunse-Gerstner    */
/* et al., cited in Sec. 2)                                                  */
/* ------------------------------------------------------------------------ */

/* Thin QR of Y (m x w, m >= w): Q (m x w) orthonormal, R (w x w) upper
 * triangular with real nonnegative diagonal.
 * Column j: x = Y[j:, j], alpha = ||x||, phi = x_1/|x_1| (1 if x_1 = 0),
 * v = x + alpha phi e_1.  H = I - 2 v v^H / (v^H v) is unitary and Hermitian
 * and maps x to -alpha phi e_1 (v^H x = alpha^2 + alpha |x_1| is real).  The
 * phase d_j = -phi is then moved from R's row j into Q's column j so that the
 * diagonal of R is alpha >= 0. */
static void qm_qr(const qmat Y, qmat* Qout, qmat* Rout) {
    const int64_t m = Y.r, w = Y.c;
    qmat W = qm_new(m, w);
    memcpy(W.d, Y.d, sizeof(quat) * (size_t)(m * w));
    qmat Vs = qm_new(m, w);            /* Householder vectors, column j holds v_j in rows j.. */
    double* tau = (double*)calloc((size_t)w + 1, sizeof(double));
    quat* dph = (quat*)calloc((size_t)w + 1, sizeof(quat));
    for (int64_t j = 0; j < w; j++) {
        double a2 = 0.0;
        for (int64_t i = j; i < m; i++) a2 += q_norm2(QM(W, i, j));
        double alpha = sqrt(a2);
        quat x1 = QM(W, j, j);
        double ax1 = q_abs(x1);
        quat phi = {1.0, 0.0, 0.0, 0.0};
        if (ax1 > 0.0) phi = q_scale(x1, 1.0 / ax1);
        dph[j] = q_scale(phi, -1.0);
        if (alpha == 0.0) { tau[j] = 0.0; continue; }
        for (int64_t i = j; i < m; i++) QM(Vs, i, j) = QM(W, i, j);
        QM(Vs, j, j) = q_add(x1, q_scale(phi, alpha));
        double vv = 2.0 * alpha * (alpha + ax1);
        tau[j] = 2.0 / vv;
        /* W <- H W on columns j..w-1: W_c -= v tau (v^H W_c). */
        for (int64_t c = j; c < w; c++) {
            quat s = QZERO;
            for (int64_t i = j; i < m; i++) s = q_add(s, q_mul(q_conj(QM(Vs, i, j)), QM(W, i, c)));
            s = q_scale(s, tau[j]);
            for (int64_t i = j; i < m; i++) QM(W, i, c) = q_sub(QM(W, i, c), q_mul(QM(Vs, i, j), s));
        }
    }
    /* R = D^H W[:w, :], upper triangular; the diagonal becomes alpha_j. */
    qmat R = qm_new(w, w);
    for (int64_t i = 0; i < w; i++)
        for (int64_t c = i; c < w; c++) QM(R, i, c) = q_mul(q_conj(dph[i]), QM(W, i, c));
    for (int64_t i = 0; i < w; i++) { QM(R, i, i).x = 0.0; QM(R, i, i).y = 0.0; QM(R, i, i).z = 0.0; }
    /* Q = H_0 H_1 ... H_{w-1} E D, E the first w columns of the identity. */
    qmat Q = qm_new(m, w);
    for (int64_t i = 0; i < w; i++) QM(Q, i, i).w = 1.0;
    for (int64_t j = w - 1; j >= 0; j--) {
        if (tau[j] == 0.0) continue;
        for (int64_t c = 0; c < w; c++) {
            quat s = QZERO;
            for (int64_t i = j; i < m; i++) s = q_add(s, q_mul(q_conj(QM(Vs, i, j)), QM(Q, i, c)));
            s = q_scale(s, tau[j]);
            for (int64_t i = j; i < m; i++) QM(Q, i, c) = q_sub(QM(Q, i, c), q_mul(QM(Vs, i, j), s));
        }
    }
    for (int64_t i = 0; i < m; i++)
        for (int64_t c = 0; c < w; c++) QM(Q, i, c) = q_mul(QM(Q, i, c), dph[c]);
    qm_free(&W); qm_free(&Vs); free(tau); free(dph);
    *Qout = Q; *Rout = R;
}

/* ------------------------------------------------------------------------ */
/* QSVD through the complex adjoint (eq. (qsvd); Zhang 1997, cited in Sec. 2) */
/* ------------------------------------------------------------------------ */

/* chi(X) = [[Xa, Xb], [-conj(Xb), conj(Xa)]] with X = Xa + Xb j,
 * Xa = X0 + X1 i, Xb = X2 + X3 i.  chi is an injective homomorphism, so the
 * singular values of chi(X) are those of X, each twice, and a complex singular
 * vector [x; y] of chi(X) is the first column of chi(q) for the quaternion
 * vector q = x - conj(y) j, i.e. planes (Re x, Im x, -Re y, Im y). */
typedef double complex cplx;

/* chi(R) as a (2r) x (2c) complex row-major array. */
static cplx* chi_of(const qmat R) {
    const int64_t r = R.r, c = R.c;
    cplx* C = (cplx*)calloc((size_t)(4 * r * c), sizeof(cplx));
    const int64_t ld = 2 * c;
    for (int64_t i = 0; i < r; i++)
        for (int64_t j = 0; j < c; j++) {
            quat q = QM(R, i, j);
            cplx a = q.w + q.x * I, b = q.y + q.z * I;
            C[i * ld + j] = a;
            C[i * ld + c + j] = b;
            C[(r + i) * ld + j] = -conj(b);
            C[(r + i) * ld + c + j] = conj(a);
        }
    return C;
}

static quat quat_of_cvec(cplx x, cplx y) {
    quat q = {creal(x), cimag(x), -creal(y), cimag(y)};
    return q;
}

/* One-sided (Hestenes) Jacobi on the N columns (length M) of a complex matrix
 * C: rotate column pairs until all are mutually orthogonal.  The column norms
 * are then the singular values, the normalised columns the left vectors, and
 * the accumulated rotations Vc (N x N) the right vectors. */
static void cjacobi(cplx* C, int64_t M, int64_t N, cplx* Vc) {
    for (int64_t i = 0; i < N * N; i++) Vc[i] = 0.0;
    for (int64_t i = 0; i < N; i++) Vc[i * N + i] = 1.0;
    for (int sweep = 0; sweep < 80; sweep++) {
        int rotated = 0;
        for (int64_t a = 0; a < N - 1; a++)
            for (int64_t b = a + 1; b < N; b++) {
                double al = 0.0, be = 0.0;
                cplx g = 0.0;
                for (int64_t i = 0; i < M; i++) {
                    al += creal(C[i * N + a] * conj(C[i * N + a]));
                    be += creal(C[i * N + b] * conj(C[i * N + b]));
                    g += conj(C[i * N + a]) * C[i * N + b];
                }
                double ag = cabs(g);
                if (ag == 0.0 || ag <= 1e-15 * sqrt(al * be)) continue;
                rotated = 1;
                /* With b~ = b conj(ph), ph = g/|g|, the pair (a, b~) has the real
                 * inner product |g|; the real rotation with t = tan(theta),
                 * t^2 + 2 zeta t - 1 = 0, zeta = (||b||^2 - ||a||^2)/(2|g|),
                 * makes the rotated pair orthogonal. */
                cplx ph = g / ag;
                double zeta = (be - al) / (2.0 * ag);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int64_t i = 0; i < M; i++) {
                    cplx ca = C[i * N + a], cb = C[i * N + b] * conj(ph);
                    C[i * N + a] = cs * ca - sn * cb;
                    C[i * N + b] = sn * ca + cs * cb;
                }
                for (int64_t i = 0; i < N; i++) {
                    cplx va = Vc[i * N + a], vb = Vc[i * N + b] * conj(ph);
                    Vc[i * N + a] = cs * va - sn * vb;
                    Vc[i * N + b] = sn * va + cs * vb;
                }
            }
        if (!rotated) break;
    }
}

/* Quaternion inner product X(:, a)^H Y(:, b). */
static quat col_dot(const qmat X, int64_t a, const qmat Y, int64_t b) {
    quat s = QZERO;
    for (int64_t i = 0; i < X.r; i++) s = q_add(s, q_mul(q_conj(QM(X, i, a)), QM(Y, i, b)));
    return s;
}

/* Y(:, b) -= X(:, a) cf. */
static void col_axpy(qmat* Y, int64_t b, const qmat X, int64_t a, quat cf) {
    for (int64_t i = 0; i < Y->r; i++) QM(*Y, i, b) = q_sub(QM(*Y, i, b), q_mul(QM(X, i, a), cf));
}

/* Thin QSVD of a tall quaternion matrix X (r x c, r >= c):
 * X = Uh diag(S) Vh^H, Uh r x c, Vh c x c, S descending (eq. (qsvd)).
 * The 2c complex singular triplets of chi(X) are taken in descending order of
 * sigma and mapped to quaternion vectors.  A candidate is orthogonalised
 * (quaternion Gram-Schmidt, right coefficients, applied alike to the u and v
 * sides so that X^H u = sigma v is kept) against the accepted vectors of the
 * same singular value (relative gap <= 1e-10) and dropped if less than half of
 * it remains; this discards the second member of each chi pair.  For a
 * negligible singular value (below 4 (2r) eps sigma_max, i.e. rank deficiency)
 * the right vector comes from the rotations alone and the left vector is any
 * unit vector orthogonal to the accepted ones, taken from the canonical basis. */
static void qm_qsvd(const qmat X, qmat* Uh_out, double* S, qmat* Vh_out) {
    const int64_t r = X.r, c = X.c, M = 2 * r, N = 2 * c;
    cplx* C = chi_of(X);
    cplx* Vc = (cplx*)calloc((size_t)(N * N), sizeof(cplx));
    cjacobi(C, M, N, Vc);
    double* sig = (double*)calloc((size_t)N, sizeof(double));
    int64_t* ord = (int64_t*)calloc((size_t)N, sizeof(int64_t));
    for (int64_t j = 0; j < N; j++) {
        double s = 0.0;
        for (int64_t i = 0; i < M; i++) s += creal(C[i * N + j] * conj(C[i * N + j]));
        sig[j] = sqrt(s); ord[j] = j;
    }
    for (int64_t a = 1; a < N; a++) {   /* insertion sort, descending, stable */
        int64_t t = ord[a]; int64_t b = a - 1;
        while (b >= 0 && sig[ord[b]] < sig[t]) { ord[b + 1] = ord[b]; b--; }
        ord[b + 1] = t;
    }
    qmat Uh = qm_new(r, c), Vh = qm_new(c, c);
    qmat cu = qm_new(r, 1), cv = qm_new(c, 1);
    const double smax = sig[ord[0]] > 0.0 ? sig[ord[0]] : 1.0;
    /* below this a singular value is rounding noise of a rank-deficient X */
    const double negl = 4.0 * (double)M * 2.220446049250313e-16 * smax;
    int64_t nacc = 0, next_unit = 0;
    for (int64_t t = 0; t < N && nacc < c; t++) {
        const int64_t j = ord[t];
        const double sj = sig[j];
        for (int64_t i = 0; i < c; i++) QM(cv, i, 0) = quat_of_cvec(Vc[i * N + j], Vc[(c + i) * N + j]);
        if (sj > negl) {
            for (int64_t i = 0; i < r; i++) QM(cu, i, 0) = quat_of_cvec(C[i * N + j] / sj, C[(r + i) * N + j] / sj);
            for (int64_t a = 0; a < nacc; a++) {
                if (fabs(S[a] - sj) > 1e-10 * smax) continue;
                quat cf = col_dot(Uh, a, cu, 0);
                col_axpy(&cu, 0, Uh, a, cf);
                col_axpy(&cv, 0, Vh, a, cf);
            }
            double nu = sqrt(qm_fro2(cu));
            if (nu < 0.5) continue;
            for (int64_t i = 0; i < r; i++) QM(Uh, i, nacc) = q_scale(QM(cu, i, 0), 1.0 / nu);
            for (int64_t i = 0; i < c; i++) QM(Vh, i, nacc) = q_scale(QM(cv, i, 0), 1.0 / nu);
        } else {
            for (int64_t a = 0; a < nacc; a++) {
                if (S[a] > negl) continue;
                quat cf = col_dot(Vh, a, cv, 0);
                col_axpy(&cv, 0, Vh, a, cf);
            }
            double nv = sqrt(qm_fro2(cv));
            if (nv < 0.5) continue;
            for (int64_t i = 0; i < c; i++) QM(Vh, i, nacc) = q_scale(QM(cv, i, 0), 1.0 / nv);
            double nu = 0.0;
            while (nu < 0.5 && next_unit < r) {
                for (int64_t i = 0; i < r; i++) QM(cu, i, 0) = QZERO;
                QM(cu, next_unit, 0).w = 1.0;
                next_unit++;
                for (int pass = 0; pass < 2; pass++)
                    for (int64_t a = 0; a < nacc; a++) col_axpy(&cu, 0, Uh, a, col_dot(Uh, a, cu, 0));
                nu = sqrt(qm_fro2(cu));
            }
            for (int64_t i = 0; i < r; i++) QM(Uh, i, nacc) = q_scale(QM(cu, i, 0), 1.0 / nu);
        }
        S[nacc] = sj;
        nacc++;
    }
    free(C); free(Vc); free(sig); free(ord);
    qm_free(&cu); qm_free(&cv);
    *Uh_out = Uh; *Vh_out = Vh;
}

/* Canonical phase of a singular pair (a reading: the paper leaves it free):
 * right-multiply column j of U and V by conj(phi), phi = nu/|nu| with nu the
 * entry of largest modulus in V[:, j] (lowest row on ties), so that this entry
 * becomes real positive.  U S V^H is unchanged. */
static void canon_phase(qmat* U, qmat* V, int64_t k) {
    for (int64_t j = 0; j < k; j++) {
        int64_t best = 0; double bm = -1.0;
        for (int64_t i = 0; i < V->r; i++) {
            double a = q_norm2(QM(*V, i, j));
            if (a > bm) { bm = a; best = i; }
        }
        if (bm <= 0.0) continue;
        quat nu = QM(*V, best, j);
        quat ph = q_conj(q_scale(nu, 1.0 / sqrt(bm)));
        for (int64_t i = 0; i < V->r; i++) QM(*V, i, j) = q_mul(QM(*V, i, j), ph);
        for (int64_t i = 0; i < U->r; i++) QM(*U, i, j) = q_mul(QM(*U, i, j), ph);
    }
}

/* ------------------------------------------------------------------------ */
/* The algorithms (Sec. 3 and Sec. 5)                                        */
/* ------------------------------------------------------------------------ */

/* Per-pass error estimate for a view whose input basis is orthonormal:
 * sqrt(max(0, ||A||_F^2 - sum_{j<=k} sigma_j(R)^2) / ||A||_F^2). */
static double pass_estimate(const qmat R, int k, double nA2) {
    qmat Uh, Vh;
    const int64_t w = R.r;
    double* S = (double*)calloc((size_t)w, sizeof(double));
    qm_qsvd(R, &Uh, S, &Vh);
    double top = 0.0;
    for (int64_t j = 0; j < k && j < w; j++) top += S[j] * S[j];
    qm_free(&Uh); qm_free(&Vh); free(S);
    double r = nA2 - top;
    if (r < 0.0) r = 0.0;
    return nA2 > 0.0 ? sqrt(r / nA2) : 0.0;
}

/* TSVD step shared by all algorithms: given the final bases Q1 (m x w),
 * Q2 (n x w) and the triangular R of the last view, with
 * even ("R = R2", A^H Q1 = Q2 R2): R2 = Vh S Uh^H;
 * odd  ("R = R1", A Q2 = Q1 R1):   R1 = Uh S Vh^H;
 * and U = Q1 Uh(:, 1:k), V = Q2 Vh(:, 1:k) (Alg. 2 last lines). */
static void finish_tsvd(const qmat Q1, const qmat Q2, const qmat R, int r_is_r2, int k,
                        qmat* U, double* S, qmat* V) {
    qmat Lh, Rh;
    const int64_t w = R.r;
    double* Sw = (double*)calloc((size_t)w, sizeof(double));
    qm_qsvd(R, &Lh, Sw, &Rh);
    qmat Uh = qm_cols(r_is_r2 ? Rh : Lh, 0, k);
    qmat Vh = qm_cols(r_is_r2 ? Lh : Rh, 0, k);
    *U = qm_mul(Q1, Uh);
    *V = qm_mul(Q2, Vh);
    for (int j = 0; j < k; j++) S[j] = Sw[j];
    canon_phase(U, V, k);
    qm_free(&Lh); qm_free(&Rh); qm_free(&Uh); qm_free(&Vh); free(Sw);
}

/* Alg. 2: Q2 = Omega; for i = 1..v: odd i: [Q1, R1] = QR(A Q2); even i:
 * [Q2, R2] = QR(A^H Q1); then the TSVD of R2 (v even) or R1 (v odd). */
static void alg2(const qmat A, const qmat Om, int k, int v, double nA2,
                 qmat* U, double* S, qmat* V, double* err, qmat* Q1o, qmat* Q2o) {
    qmat Q2 = qm_new(Om.r, Om.c);
    memcpy(Q2.d, Om.d, sizeof(quat) * (size_t)(Om.r * Om.c));
    qmat Q1 = qm_new(0, 0), R = qm_new(0, 0);
    for (int i = 1; i <= v; i++) {
        qm_free(&R);
        if (i % 2 == 1) {
            qmat Y = qm_mul(A, Q2);
            qm_free(&Q1);
            qm_qr(Y, &Q1, &R);
            qm_free(&Y);
        } else {
            qmat W = qm_adj_mul(A, Q1);
            qm_free(&Q2);
            qm_qr(W, &Q2, &R);
            qm_free(&W);
        }
        err[i - 1] = (i == 1) ? NAN : pass_estimate(R, k, nA2);
    }
    finish_tsvd(Q1, Q2, R, v % 2 == 0, k, U, S, V);
    qm_free(&R);
    *Q1o = Q1; *Q2o = Q2;
}

/* Alg. 1 with q = (v-2)/2: QR(A Omega), q times {QR(A^H Q1), QR(A Q2)},
 * then [Q2, R] = QR(A^H Q1) and TSVD(R). */
static void alg1(const qmat A, const qmat Om, int k, int v, double nA2,
                 qmat* U, double* S, qmat* V, double* err, qmat* Q1o, qmat* Q2o) {
    const int q = (v - 2) / 2;
    qmat R, Q1, Q2;
    int view = 0;
    { qmat Y = qm_mul(A, Om); qm_qr(Y, &Q1, &R); qm_free(&Y); err[view++] = NAN; qm_free(&R); }
    Q2 = qm_new(0, 0);
    for (int it = 0; it < q; it++) {
        qmat W = qm_adj_mul(A, Q1); qm_free(&Q2); qm_qr(W, &Q2, &R); qm_free(&W);
        err[view++] = pass_estimate(R, k, nA2); qm_free(&R);
        qmat Y = qm_mul(A, Q2); qm_free(&Q1); qm_qr(Y, &Q1, &R); qm_free(&Y);
        err[view++] = pass_estimate(R, k, nA2); qm_free(&R);
    }
    { qmat W = qm_adj_mul(A, Q1); qm_free(&Q2); qm_qr(W, &Q2, &R); qm_free(&W); }
    err[view++] = pass_estimate(R, k, nA2);
    finish_tsvd(Q1, Q2, R, 1, k, U, S, V);
    qm_free(&R);
    *Q1o = Q1; *Q2o = Q2;
}

/* [B_1 ... B_s] clamped to its first `cap` columns. */
static qmat stack_cols(qmat* blocks, int nb, int64_t cap) {
    int64_t rows = blocks[0].r, tot = 0;
    for (int b = 0; b < nb; b++) tot += blocks[b].c;
    if (tot > cap) tot = cap;
    qmat K = qm_new(rows, tot);
    int64_t c0 = 0;
    for (int b = 0; b < nb && c0 < tot; b++)
        for (int64_t j = 0; j < blocks[b].c && c0 < tot; j++, c0++)
            for (int64_t i = 0; i < rows; i++) QM(K, i, c0) = QM(blocks[b], i, j);
    return K;
}

/* Alg. 4: s = floor((v-1)/2); for j = 1..s: Q1_j = QR(A Q2_{j-1}).Q,
 * Q2_j = QR(A^H Q1_j).Q with Q2_0 = Omega; if v even, Q1_{s+1} = QR(A Q2_s).Q,
 * stack K1 = [Q1_1 .. Q1_{v/2}], Q1 = QR(K1).Q, [Q2, R2] = QR(A^H Q1),
 * TSVD(R2); if v odd, stack K2 = [Q2_1 .. Q2_s], Q2 = QR(K2).Q,
 * [Q1, R1] = QR(A Q2), TSVD(R1).  The stack is clamped to min(m, n) columns
 * (a reading; the paper does not treat a stack wider than the matrix). */
static void alg4(const qmat A, const qmat Om, int k, int v, double nA2,
                 qmat* U, double* S, qmat* V, double* err, qmat* Q1o, qmat* Q2o) {
    const int s = (v - 1) / 2;
    const int64_t cap = A.r < A.c ? A.r : A.c;
    qmat* Q1b = (qmat*)calloc((size_t)s + 2, sizeof(qmat));
    qmat* Q2b = (qmat*)calloc((size_t)s + 2, sizeof(qmat));
    Q2b[0] = qm_new(Om.r, Om.c);
    memcpy(Q2b[0].d, Om.d, sizeof(quat) * (size_t)(Om.r * Om.c));
    int view = 0;
    qmat R;
    for (int j = 1; j <= s; j++) {
        qmat Y = qm_mul(A, Q2b[j - 1]); qm_qr(Y, &Q1b[j], &R); qm_free(&Y);
        err[view] = view == 0 ? NAN : pass_estimate(R, k, nA2); view++; qm_free(&R);
        qmat W = qm_adj_mul(A, Q1b[j]); qm_qr(W, &Q2b[j], &R); qm_free(&W);
        err[view] = pass_estimate(R, k, nA2); view++; qm_free(&R);
    }
    qmat Q1, Q2;
    if (v % 2 == 0) {
        qmat Y = qm_mul(A, Q2b[s]); qm_qr(Y, &Q1b[s + 1], &R); qm_free(&Y);
        err[view] = view == 0 ? NAN : pass_estimate(R, k, nA2); view++; qm_free(&R);
        qmat K1 = stack_cols(&Q1b[1], v / 2, cap);
        qmat Rk; qm_qr(K1, &Q1, &Rk); qm_free(&Rk); qm_free(&K1);
        qmat W = qm_adj_mul(A, Q1); qm_qr(W, &Q2, &R); qm_free(&W);
        err[view] = pass_estimate(R, k, nA2); view++;
        finish_tsvd(Q1, Q2, R, 1, k, U, S, V);
    } else {
        qmat K2 = stack_cols(&Q2b[1], s, cap);
        qmat Rk; qm_qr(K2, &Q2, &Rk); qm_free(&Rk); qm_free(&K2);
        qmat Y = qm_mul(A, Q2); qm_qr(Y, &Q1, &R); qm_free(&Y);
        err[view] = pass_estimate(R, k, nA2); view++;
        finish_tsvd(Q1, Q2, R, 0, k, U, S, V);
    }
    qm_free(&R);
    for (int j = 0; j <= s + 1; j++) { if (Q1b[j].d) qm_free(&Q1b[j]); if (Q2b[j].d) qm_free(&Q2b[j]); }
    free(Q1b); free(Q2b);
    *Q1o = Q1; *Q2o = Q2;
}

/* Alg. 3 with q = (v-2)/2: K_0 = A Omega, K_i = (A A^H) K_{i-1} (not
 * normalised, as written), K = [K_0 .. K_q], [Q, ~] = QR(K), Y~ = Q^H A,
 * SVD(Y~) = U_Y S_Y V_Y^H, U = Q U_Y(:, 1:k), V = V_Y(:, 1:k).  The SVD of
 * the wide Y~ is taken as the thin QSVD of its conjugate transpose
 * Y~^H = A^H Q = Uh S Vh^H, so U_Y = Vh and V_Y = Uh.  Only the final view
 * has an orthonormal input basis, so only its estimate is defined. */
static void alg3(const qmat A, const qmat Om, int k, int v, double nA2,
                 qmat* U, double* S, qmat* V, double* err, qmat* Q1o, qmat* Q2o) {
    const int q = (v - 2) / 2;
    const int64_t cap = A.r < A.c ? A.r : A.c;
    qmat* Kb = (qmat*)calloc((size_t)q + 1, sizeof(qmat));
    int view = 0;
    Kb[0] = qm_mul(A, Om); err[view++] = NAN;
    for (int i = 1; i <= q; i++) {
        qmat T = qm_adj_mul(A, Kb[i - 1]); err[view++] = NAN;
        Kb[i] = qm_mul(A, T); err[view++] = NAN;
        qm_free(&T);
    }
    qmat K = stack_cols(Kb, q + 1, cap);
    qmat Q1, Rk; qm_qr(K, &Q1, &Rk); qm_free(&Rk); qm_free(&K);
    qmat Yh = qm_adj_mul(A, Q1);                       /* Y~^H, n x w */
    const int64_t w = Yh.c;
    qmat Uh, Vh;
    double* Sw = (double*)calloc((size_t)w, sizeof(double));
    qm_qsvd(Yh, &Uh, Sw, &Vh);
    double top = 0.0;
    for (int j = 0; j < k; j++) top += Sw[j] * Sw[j];
    err[view++] = nA2 > 0.0 ? sqrt((nA2 - top > 0.0 ? nA2 - top : 0.0) / nA2) : 0.0;
    qmat Uy = qm_cols(Vh, 0, k), Vy = qm_cols(Uh, 0, k);
    *U = qm_mul(Q1, Uy);
    *V = Vy;
    for (int j = 0; j < k; j++) S[j] = Sw[j];
    canon_phase(U, V, k);
    /* The co-range basis of this construction is Y~^H's left factor. */
    qmat Q2 = qm_new(Yh.r, w);
    memcpy(Q2.d, Uh.d, sizeof(quat) * (size_t)(Yh.r * w));
    qm_free(&Yh); qm_free(&Uh); qm_free(&Vh); qm_free(&Uy); free(Sw);
    for (int i = 0; i <= q; i++) qm_free(&Kb[i]);
    free(Kb);
    *Q1o = Q1; *Q2o = Q2;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

int qo_qgemm(const double* A, int64_t m, int64_t n, const double* B, int64_t w, double* C) {
    if (!A || !B || !C || m < 0 || n < 0 || w < 0) return -1;
    qmat a = qm_from_planes(A, m, n), b = qm_from_planes(B, n, w);
    qmat c = qm_mul(a, b);
    qm_to_planes(c, C);
    qm_free(&a); qm_free(&b); qm_free(&c);
    return 0;
}

int qo_qgemm_adj(const double* A, int64_t m, int64_t n, const double* B, int64_t w, double* C) {
    if (!A || !B || !C || m < 0 || n < 0 || w < 0) return -1;
    qmat a = qm_from_planes(A, m, n), b = qm_from_planes(B, m, w);
    qmat c = qm_adj_mul(a, b);
    qm_to_planes(c, C);
    qm_free(&a); qm_free(&b); qm_free(&c);
    return 0;
}

int qo_qr(const double* Y, int64_t m, int64_t w, double* Q, double* R) {
    if (!Y || !Q || !R || m < w || w < 1) return -1;
    qmat y = qm_from_planes(Y, m, w), q, r;
    qm_qr(y, &q, &r);
    qm_to_planes(q, Q); qm_to_planes(r, R);
    qm_free(&y); qm_free(&q); qm_free(&r);
    return 0;
}

int qo_qsvd(const double* R, int64_t w, double* Uh, double* S, double* Vh) {
    if (!R || !Uh || !S || !Vh || w < 1) return -1;
    qmat r = qm_from_planes(R, w, w), u, vv;
    qm_qsvd(r, &u, S, &vv);
    qm_to_planes(u, Uh); qm_to_planes(vv, Vh);
    qm_free(&r); qm_free(&u); qm_free(&vv);
    return 0;
}

int qo_qlra_sketch(const double* A, int64_t m, int64_t n, int k, int p, int v, int scheme,
                   const double* Om, double* U, double* S, double* V, double* pass_err,
                   double* Q1p, int64_t* wq1, double* Q2p, int64_t* wq2) {
    const int64_t l = (int64_t)k + p;
    if (!A || !Om || !U || !S || !V || !pass_err) return -1;
    if (k < 1 || p < 0 || v < 2 || l > m || l > n) return -1;
    if ((scheme == 2 || scheme == 3) && (v % 2) != 0) return -1;
    if (scheme < 0 || scheme > 3) return -1;
    qmat a = qm_from_planes(A, m, n), om = qm_from_planes(Om, n, l);
    const double nA2 = qm_fro2(a);
    qmat u, vv, q1, q2;
    switch (scheme) {
        case 0: alg2(a, om, k, v, nA2, &u, S, &vv, pass_err, &q1, &q2); break;
        case 1: alg4(a, om, k, v, nA2, &u, S, &vv, pass_err, &q1, &q2); break;
        case 2: alg1(a, om, k, v, nA2, &u, S, &vv, pass_err, &q1, &q2); break;
        default: alg3(a, om, k, v, nA2, &u, S, &vv, pass_err, &q1, &q2); break;
    }
    /* The last estimate equals the residual of the returned U S V^H. */
    qm_to_planes(u, U); qm_to_planes(vv, V);
    if (Q1p) qm_to_planes(q1, Q1p);
    if (wq1) *wq1 = q1.c;
    if (Q2p) qm_to_planes(q2, Q2p);
    if (wq2) *wq2 = q2.c;
    qm_free(&a); qm_free(&om); qm_free(&u); qm_free(&vv); qm_free(&q1); qm_free(&q2);
    return 0;
}

int qo_qlra(const double* A, int64_t m, int64_t n, int k, int p, int v, int scheme,
            uint64_t seed, double* U, double* S, double* V, double* pass_err) {
    const int64_t l = (int64_t)k + p;
    if (k < 1 || p < 0 || v < 2 || l > m || l > n) return -1;
    float* omf = (float*)malloc(sizeof(float) * (size_t)(4 * n * l));
    double* omd = (double*)malloc(sizeof(double) * (size_t)(4 * n * l));
    if (!omf || !omd) { free(omf); free(omd); return -2; }
    qo_omega(seed, n, l, omf);
    for (int64_t i = 0; i < 4 * n * l; i++) omd[i] = (double)omf[i];
    int rc = qo_qlra_sketch(A, m, n, k, p, v, scheme, omd, U, S, V, pass_err, NULL, NULL, NULL, NULL);
    free(omf); free(omd);
    return rc;
}
