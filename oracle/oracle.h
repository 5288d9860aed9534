/*
 * CPU oracle for the sketch Y = A * Omega(seed) with a generated random operand.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares
 * no code, header, constant or table with it.
 *
 * Every function here is written for obvious correctness, not speed: plain
 * loops, products formed exactly in FP64, sums accumulated in FP64.
 *
 * Paper: "Communication Lower Bounds and Algorithms for Sketching with Random
 * Dense Matrices" (SPAA '26).  Problem statement B = A*Omega with Omega an
 * n2 x r random matrix (Sec. 4, first paragraph); each processor generates
 * the block of a global Omega it needs from a shared seed (Alg. 1,
 * GenRandom; Sec. 6.3); the generator is the counter-based Philox of
 * Salmon et al. (Sec. 6.3, citing SC'11).
 */
#ifndef SKETCH_ORACLE_H
#define SKETCH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds, key bumped between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Batched form: out[4i..4i+3] = Philox4x32-10(ctr[4i..4i+3], key), i < N. */
void oracle_philox_raw(const uint32_t* ctr, const uint32_t key[2], uint32_t* out, int64_t N);

/* Distribution of Omega's entries. */
enum { ORACLE_DIST_NORMAL = 0, ORACLE_DIST_UNIFORM = 1, ORACLE_DIST_RADEMACHER = 2 };

/* Omega entry (global row j, global column c) as the FP32 value the method
 * defines: Box-Muller over the Philox uniforms, evaluated with the fixed FP32
 * operation sequence documented in oracle.c. */
float oracle_omega_value(uint64_t seed, int64_t row, int64_t col);
/* The entry under another distribution: ORACLE_DIST_UNIFORM gives the uniform
 * u = (2 (r >> 9) + 1) 2^-24 of the entry's own Philox word r, in (0, 1);
 * ORACLE_DIST_RADEMACHER gives +1 if r < 2^31, else -1. */
float oracle_omega_value_dist(uint64_t seed, int64_t row, int64_t col, int dist);
/* The FP32 Box-Muller step alone: from the Philox words (r_even, r_odd) to
 * (rho cos theta, rho sin theta) with u = (2 (r >> 9) + 1) 2^-24,
 * rho = sqrt(-2 ln u_even), theta = 2 pi u_odd. */
void oracle_normal_pair(uint32_t r_even, uint32_t r_odd, float* z_cos, float* z_sin);
/* The same over N word pairs. */
void oracle_normal_pairs(const uint32_t* r_even, const uint32_t* r_odd, float* z_cos,
                         float* z_sin, int64_t N);
/* The two FP32 pieces of that step for odd integers mo in [1, 2^24),
 * u = mo 2^-24: ln u, and (cos 2 pi u, sin 2 pi u). */
void oracle_spec_log_batch(const uint32_t* mo, float* out, int64_t N);
void oracle_spec_cossin_batch(const uint32_t* mo, float* c_out, float* s_out, int64_t N);
/* Same entry through FP64 libm (log, sqrt, cos, sin) of the same uniforms;
 * pins the FP32 sequence's accuracy. */
double oracle_omega_f64ref(uint64_t seed, int64_t row, int64_t col);
/* Omega[row0:row0+n, col0:col0+k] as an n x k row-major FP32 block. */
void oracle_omega_block(uint64_t seed, int64_t row0, int64_t n, int64_t col0, int64_t k,
                        float* out);
void oracle_omega_block_dist(uint64_t seed, int64_t row0, int64_t n, int64_t col0, int64_t k,
                             int dist, float* out);

/* Y (m x k, row-major, FP64) = A (m x n, row-major, leading dim lda, FP32)
 *                              * Omega(seed)[row0:row0+n, col0:col0+k]. */
void oracle_gen_matmul_f64(const float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                           int64_t row0, int64_t col0, int64_t k, double* Y);
void oracle_gen_matmul_dist_f64(const float* A, int64_t m, int64_t n, int64_t lda,
                                uint64_t seed, int64_t row0, int64_t col0, int64_t k, int dist,
                                double* Y);

/* Contraction split with reduction: Y = sum_b A_b * Omega[row0_b : row0_b+n_b, col0:col0+k],
 * blocks summed in order b = 0..P-1 in FP64. */
void oracle_gen_matmul_reduce_f64(const float* const* A_b, int64_t P, int64_t m,
                                  const int64_t* n_b, const int64_t* lda_b,
                                  const int64_t* row0_b, uint64_t seed, int64_t col0,
                                  int64_t k, double* Y);
void oracle_gen_matmul_reduce_dist_f64(const float* const* A_b, int64_t P, int64_t m,
                                       const int64_t* n_b, const int64_t* lda_b,
                                       const int64_t* row0_b, uint64_t seed, int64_t col0,
                                       int64_t k, int dist, double* Y);

/* Column-major A (element (i, j) at A[j * lda + i]): Y (m x k row-major FP64) =
 * A * Omega(seed, dist)[row0:row0+n, col0:col0+k]. */
void oracle_gen_matmul_cm_f64(const float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                              int64_t row0, int64_t col0, int64_t k, int dist, double* Y);
/* Alg. 2's second product: C (k x p row-major FP64) =
 * Omega(seed, dist)[row0:row0+n, col0:col0+k]^T * B (B row-major n x p, leading dim ldb). */
void oracle_gen_tmatmul_f64(const float* B, int64_t n, int64_t p, int64_t ldb, uint64_t seed,
                            int64_t row0, int64_t col0, int64_t k, int dist, double* C);

/* Product with an explicit Omega (n x k row-major FP32, leading dim ldo). */
void oracle_matmul_f64(const float* A, int64_t m, int64_t n, int64_t lda, const float* Om,
                       int64_t ldo, int64_t k, double* Y);

/* ---- low-precision storage of A ---- */
/* bfloat16, round to nearest even. */
void oracle_bf16_encode(const float* x, uint16_t* out, int64_t N);
double oracle_bf16_decode(uint16_t b);
/* OCP FP8 E4M3FN (bias 7, no infinities, max 448), round to nearest even,
 * saturating at +-448. */
uint8_t oracle_fp8e4m3_encode(double x);
double oracle_fp8e4m3_decode(uint8_t b);
/* Per-128-row-block power-of-two scales: s_b = smallest 2^E with
 * amax_b <= 448 * 2^E (s_b = 1 when the block is all zero); codes
 * q(i,j) = fp8(A(i,j) / s_b). */
void oracle_quantize_fp8_rows128(const float* A, int64_t m, int64_t n, int64_t lda,
                                 uint8_t* Q, int64_t ldq, float* scales);
/* Y = dequant(Aq) * Omega in FP64; dtype 1 = bf16 codes, 2 = fp8 codes;
 * scales may be NULL (all ones). */
void oracle_gen_matmul_q_f64(const void* Aq, int dtype, int64_t m, int64_t n, int64_t lda,
                             const float* scales, uint64_t seed, int64_t row0, int64_t col0,
                             int64_t k, double* Y);

/* Threads the oracle's parallel loops use (OpenMP). */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
