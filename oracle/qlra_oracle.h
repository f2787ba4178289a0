/*
 * qlra_oracle.h -- plain FP64 CPU oracle for the pass-efficient randomized
 * low-rank approximation of quaternion matrices (arXiv 2507.13731).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * (include/qlra.h) against a slow, obviously correct implementation of the
 * same method.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header or constant with
 * the GPU path; the two sides only ever see the same seeded inputs.
 *
 * Conventions (all functions):
 *   - A quaternion matrix X = X0 + X1 i + X2 j + X3 k (Sec. 2) is passed as four
 *     real planes, plane p at X + p*plane_stride, each plane row-major with
 *     leading dimension ld.  All buffers are host memory owned by the caller.
 *   - Internally the oracle works on an array of quaternion structs, a layout
 *     deliberately unlike the GPU path's plane layout.
 *   - Return value: 0 on success, negative on a bad argument (-1) or an
 *     allocation failure (-2).
 *
 * Parity status of each function is stated in qlra_oracle.c's header.
 */
#ifndef QLRA_ORACLE_H
#define QLRA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 block (Salmon et al., SC'11): ctr[4], key[2] -> out[4]. */
void qo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Elementary functions written from their series, used by the Gaussian
 * generator.  Exposed so the tests can compare them with libm. */
double qo_log_unit(double u);          /* ln u for u in (0, 1]                */
double qo_sqrt_pos(double x);          /* sqrt x for x > 0                    */
void   qo_sincos_2pi(double u, double* s, double* c); /* sin/cos(2 pi u), u in [0,1) */

/* Quaternion Gaussian test matrix (Sec. 2, Def. "Gaussian random matrix"):
 * four independent N(0,1) planes, n x l, written as FP32 planes
 * Om[p*n*l + i*l + j].  Entry (i, j) depends only on (seed, i, j). */
void qo_omega(uint64_t seed, int64_t n, int64_t l, float* Om);

/* C = A * B (Hamilton product, eq. (1)); A m x n, B n x w, C m x w. */
int qo_qgemm(const double* A, int64_t m, int64_t n, const double* B, int64_t w, double* C);
/* C = A^H * B (conjugate transpose, Sec. 2); A m x n, B m x w, C n x w. */
int qo_qgemm_adj(const double* A, int64_t m, int64_t n, const double* B, int64_t w, double* C);

/* Thin quaternion QR (eq. (QQR)) by Householder reflections; Q m x w has
 * orthonormal columns, R w x w upper triangular with a real nonnegative
 * diagonal.  Requires m >= w. */
int qo_qr(const double* Y, int64_t m, int64_t w, double* Q, double* R);

/* Full QSVD of a square w x w quaternion matrix through its complex adjoint:
 * R = Uh diag(S) Vh^H with S descending (eq. (qsvd)).  Uh, Vh are w x w. */
int qo_qsvd(const double* R, int64_t w, double* Uh, double* S, double* Vh);

/* Algorithms.  scheme 0 = Alg. 2 (subspace, any v >= 2), 1 = Alg. 4 (block
 * Krylov, any v >= 2), 2 = Alg. 1 with q = (v-2)/2 (v even), 3 = Alg. 3 with
 * q = (v-2)/2 (v even).  Outputs: U m x k, S k, V n x k, pass_err v entries
 * (NaN where undefined).  Omega is generated from `seed` as qo_omega does.
 * A is given in FP64 planes (m x n). */
int qo_qlra(const double* A, int64_t m, int64_t n, int k, int p, int v, int scheme,
            uint64_t seed, double* U, double* S, double* V, double* pass_err);

/* Same as qo_qlra but with an explicit sketch Om (FP64 planes, n x (k+p))
 * instead of the seed, and optional outputs of the final bases:
 * Q1 (m x wq1), Q2 (n x wq2); the widths are returned through wq1/wq2.
 * Pass NULL to skip.  Q1/Q2 must hold m*min(m,(v/2+1)(k+p)) resp.
 * n*min(n,(v/2+1)(k+p)) quaternions per plane. */
int qo_qlra_sketch(const double* A, int64_t m, int64_t n, int k, int p, int v, int scheme,
                   const double* Om, double* U, double* S, double* V, double* pass_err,
                   double* Q1, int64_t* wq1, double* Q2, int64_t* wq2);

#ifdef __cplusplus
}
#endif
#endif
