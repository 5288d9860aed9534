/*
 * sketch.h -- C ABI of the MI355X (gfx950) library for the sketch
 *
 *     Y = A * Omega(seed)
 *
 * where Omega is a dense N(0,1) random matrix that is never communicated or
 * kept between calls: every call regenerates the entries it needs from a
 * 64-bit seed with a counter-based Philox4x32-10 generator on the device,
 * inside the multiply kernel or, on the matrix-core routes whose row tiles
 * share Omega chunks, once per call into the call's workspace.
 *
 * Paper: "Communication Lower Bounds and Algorithms for Sketching with Random
 * Dense Matrices" (SPAA '26).
 *   - Problem: B = A*Omega, A n1 x n2, Omega n2 x r random, r < n2 (Sec. 4).
 *   - Alg. 1 (RandMatMul): processor (i,j,k) generates the (j,k) block of the
 *     global Omega (GenRandom), multiplies its A block by it, and the partial
 *     products of a contraction split are summed (Reduce-Scatter).
 *   - Sec. 4.3 Case 1 (row split, p1 = P): no communication at all; every
 *     process regenerates the whole Omega from the shared seed (Sec. 6.3/6.4).
 *   - Sec. 6.3: Omega is produced by the counter-based Philox generator
 *     (Salmon et al., SC'11) rather than communicated.
 *
 * Omega is defined entry by entry (readings of the paper documented with the
 * library): Omega(j, c) for global row j and column c is word (j mod 4) of
 * Philox4x32-10 applied to the counter (q mod 2^32, q div 2^32, c, 0) with
 * q = j div 4 and key (seed mod 2^32, seed div 2^32); each word r gives
 * u = (2 (r >> 9) + 1) 2^-24, words (0,1) and (2,3) are Box-Muller pairs
 * (rho cos, rho sin) with rho from the even word and angle 2 pi u from the
 * odd word, evaluated by a fixed FP32 operation sequence so that the values
 * are reproducible bit for bit on any IEEE machine.
 *
 * Conventions for every call below:
 *   - Matrices are row-major: element (i, j) of A sits at A + i*lda + j
 *     (in elements of A's storage type); Y(i, c) sits at Y + i*ldy + c.
 *   - All buffer pointers are DEVICE pointers unless stated, owned by the
 *     caller; the library never allocates or frees memory in these calls.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls only
 *     enqueue work; they never synchronise the host.
 *   - Argument errors are detected on the host before anything is enqueued;
 *     on such an error nothing is written.  SK_EHIP reports a failed launch.
 *   - Results do not depend on the launch configuration: for a given A,
 *     seed, offsets and k, Y is bitwise reproducible run to run, and equal
 *     between a call on a row block and the matching rows of a call on the
 *     whole matrix.
 */
#ifndef SKETCH_H
#define SKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SKETCH_ABI_VERSION 7

enum sk_status {
    SK_OK = 0,
    SK_EINVAL = -1,        /* bad size, pointer, leading dimension or flag       */
    SK_EDTYPE = -2,        /* unknown element type                                */
    SK_EALIGN = -3,        /* A or lda not aligned to 16 bytes (see below)        */
    SK_EWORKSPACE = -4,    /* workspace missing or smaller than required          */
    SK_EHIP = -5,          /* HIP runtime reported an error at launch             */
    SK_ENOMEM = -6,        /* (serving) device memory exhausted                   */
    SK_EUNSUPPORTED = -7,  /* valid request this build does not handle            */
    SK_EBUDGET = -8,       /* (serving) request larger than the memory budget     */
    SK_EQUEUE = -9,        /* (serving) queue full or unknown ticket              */
    SK_ETIMEOUT = -10,     /* (serving) wait ended before the request finished    */
    SK_ESCRATCH = -11      /* call needs more than the library's static scratch   */
};

/* Storage type of A. */
enum sk_adtype {
    SK_A_F32 = 0,          /* IEEE binary32                                       */
    SK_A_BF16 = 1,         /* bfloat16                                            */
    SK_A_FP8_E4M3 = 2      /* OCP FP8 E4M3FN, with per-128-row-block scales       */
};

/* Storage type of Y.  The reduction over column strips and blocks is carried
 * out in FP64 and rounded once to the output type. */
enum sk_ydtype { SK_Y_F32 = 0, SK_Y_F64 = 1 };

/* Distribution of Omega's entries, all from the same Philox word of the entry
 * (word j mod 4 of counter (j div 4, c, 0) under key seed):
 *   SK_DIST_NORMAL      Box-Muller N(0,1) (the definition above; the default);
 *   SK_DIST_UNIFORM     u = (2 (r >> 9) + 1) 2^-24 in (0, 1), exact in FP32 (the
 *                       paper's experiments draw uniform entries, Sec. 6.3);
 *   SK_DIST_RADEMACHER  +1 if r < 2^31, else -1. */
enum sk_dist { SK_DIST_NORMAL = 0, SK_DIST_UNIFORM = 1, SK_DIST_RADEMACHER = 2 };

/* Version of this ABI (SKETCH_ABI_VERSION of the built library). */
int sketch_abi_version(void);

/* Static text for a status code. */
const char* sketch_status_string(int status);

/* Width (columns of A) of the contraction strips a call with this storage
 * type and sketch width sums in FP32 before the FP64 strip sum; 0 for
 * invalid arguments.  The result of a call depends on the strip boundaries
 * only (never on m, the grid or other launch choices). */
int64_t sketch_strip_width(int a_dtype, int64_t k);

/* Bytes of device workspace a call needs (0 if none).  The workspace holds
 * the FP32 partial sums of the column strips between the product kernel and
 * the FP64 reduction kernel of one call (more than one strip), and, on the
 * matrix-core routes that multiply every strip's Omega chunks in several row
 * tiles, the call's Omega formed once by the call itself, at a 256-byte
 * aligned offset after the partials:
 *   BF16 or FP8 A with k > 16: two BF16 planes (the hi and lo terms of each
 *     entry), 2 * S * 4096 * kpad values, kpad = k rounded up to a multiple
 *     of 32 for k <= 32, of 64 beyond;
 *   FP32 A with k > 32 (op 0 and 1), and column-major FP32 A with k > 32, or
 *     with k > 16 and m <= 64 (op 2): one FP32 plane of S * 2048 * kpad
 *     values, kpad = k rounded up to a multiple of 16 * nt, nt = 1, 2, 4, 8
 *     for k <= 16, 32, 64 and beyond;
 * S the call's strips.  Its contents need no preparation.
 * One workspace serves one call at a time: calls that may run concurrently
 * (different streams) need separate workspaces.
 *   op = 0: sketch_gen_matmul / sketch_matmul_omega with an n-column A;
 *   op = 1: sketch_gen_matmul_reduce over P blocks whose widths sum to n.
 *   op = 2: sketch_gen_matmul_cm with an m x n column-major FP32 A (for
 *           sketch_gen_tmatmul pass m = p, the columns of B).
 * The size depends only on (op, a_dtype, m, n, k, P); for op = 1 it is an
 * upper bound valid for any split of n into P blocks.  Returns 0 for
 * invalid arguments. */
size_t sketch_workspace_size(int op, int a_dtype, int64_t m, int64_t n, int64_t k, int64_t P);

/*
 * The local product of one process's share (Alg. 1, local multiplication with
 * GenRandom; Sec. 4.3 Case 1 for a row block):
 *
 *   Y[0:m, 0:k] (=|+=) A[0:m, 0:n] * Omega(seed)[row0 : row0+n, col0 : col0+k]
 *
 *   A          device, m x n, storage a_dtype, leading dim lda (elements).
 *              Alignment: A and lda*sizeof(element) must be multiples of 16 B.
 *   a_scales   device, ceil(m/128) FP32 scales for SK_A_FP8_E4M3 (row i uses
 *              a_scales[i/128]); NULL for F32/BF16 (scale 1).
 *   seed       the shared seed of the global Omega.
 *   omega_row0 global row of Omega matching column 0 of A (0 <= row0, row0+n <= 2^62).
 *   omega_col0 global column of Omega matching column 0 of Y (col0+k <= 2^32).
 *   k          sketch width, 1 <= k <= 1024.
 *   Y          device, m x k, storage y_dtype, leading dim ldy >= k.
 *   beta       0: Y = A*Omega;  1: Y = Y + A*Omega (old Y added in FP64).
 *   workspace  device, >= sketch_workspace_size(0, a_dtype, m, n, k, 1) bytes,
 *              16-B aligned; may be NULL if that size is 0.
 * m == 0 or k == 0: nothing to do.  n == 0: Y = 0 (beta 0) or unchanged.
 */
int sketch_gen_matmul(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                      const float* a_scales, uint64_t seed, int64_t omega_row0,
                      int64_t omega_col0, int64_t k, void* Y, int y_dtype, int64_t ldy,
                      int beta, void* workspace, size_t workspace_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * sketch_gen_matmul without a workspace argument.  What the workspace would
 * hold (strip partials, packed Omega) goes to a fixed device array inside the
 * library, SKETCH_NOALLOC_SCRATCH_BYTES bytes
 * per GPU, held from the first call on that GPU until the process ends; the
 * call itself allocates nothing.  Arguments, results and errors are those of
 * sketch_gen_matmul (same kernels, bitwise the same Y), plus SK_ESCRATCH when
 * sketch_workspace_size(0, a_dtype, m, n, k, 1) exceeds
 * SKETCH_NOALLOC_SCRATCH_BYTES (checked on the host, nothing enqueued).
 * `stream` must belong to the current device.  Every call on one GPU uses
 * the same array and leaves its contents behind (each call writes all it
 * reads, so nothing needs clearing): calls that may overlap on one GPU --
 * other streams, other host threads -- race and must be serialised by the
 * caller.
 */
#define SKETCH_NOALLOC_SCRATCH_BYTES (32u << 20)
int sketch_gen_matmul_noalloc(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                              const float* a_scales, uint64_t seed, int64_t omega_row0,
                              int64_t omega_col0, int64_t k, void* Y, int y_dtype, int64_t ldy,
                              int beta, void* stream);

/* sketch_gen_matmul with Omega drawn from the distribution `dist` (sk_dist;
 * SK_EINVAL otherwise).  Results obey every rule stated for sketch_gen_matmul. */
int sketch_gen_matmul_dist(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                           const float* a_scales, uint64_t seed, int dist, int64_t omega_row0,
                           int64_t omega_col0, int64_t k, void* Y, int y_dtype, int64_t ldy,
                           int beta, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Contraction split with on-device reduction (Alg. 1 on a (1, P, 1) grid: the
 * local products of P column blocks followed by the sum that Reduce-Scatter /
 * AllReduce performs across processes, Sec. 4.3 and Sec. 6.6), done in one
 * launch on one device:
 *
 *   Y (=|+=) sum_{b=0}^{P-1} A_b[0:m, 0:n_b] * Omega(seed)[row0_b : row0_b+n_b, col0 : col0+k]
 *
 *   A_b, n_b, lda_b, row0_b, a_scales_b  HOST arrays of length P describing the
 *              blocks (device pointers A_b[b]; a_scales_b may be NULL, or hold
 *              NULL entries, for F32/BF16).  1 <= P <= 64.
 *   The partial products are summed in FP64 in block order b = 0..P-1 and
 *   rounded once to y_dtype.  Other arguments as for sketch_gen_matmul; the
 *   workspace must hold sketch_workspace_size(1, a_dtype, m, sum n_b, k, P).
 * When each block's width is a multiple of sketch_strip_width(a_dtype, k) and
 * row0_b = row0_0 + the block's column offset, the result equals bitwise that
 * of sketch_gen_matmul on the concatenated A.
 */
int sketch_gen_matmul_reduce(const void* const* A_b, int64_t P, int a_dtype, int64_t m,
                             const int64_t* n_b, const int64_t* lda_b, const int64_t* row0_b,
                             const float* const* a_scales_b, uint64_t seed, int64_t omega_col0,
                             int64_t k, void* Y, int y_dtype, int64_t ldy, int beta,
                             void* workspace, size_t workspace_bytes, void* stream);

/* sketch_gen_matmul_reduce with Omega drawn from the distribution `dist`. */
int sketch_gen_matmul_reduce_dist(const void* const* A_b, int64_t P, int a_dtype, int64_t m,
                                  const int64_t* n_b, const int64_t* lda_b,
                                  const int64_t* row0_b, const float* const* a_scales_b,
                                  uint64_t seed, int dist, int64_t omega_col0, int64_t k,
                                  void* Y, int y_dtype, int64_t ldy, int beta, void* workspace,
                                  size_t workspace_bytes, void* stream);

/*
 * Column-major A (the paper's storage order, Secs. 6.5 and 6.6), FP32:
 *
 *   Y (=|+=) A * Omega(seed, dist)[row0 : row0+n, col0 : col0+k]
 *
 *   A       device, element (i, j) at A + j*lda + i, lda >= m; A and lda*4 must
 *           be multiples of 16 bytes.
 *   y_trans 0: Y row-major m x k (element (i, c) at Y + i*ldy + c, ldy >= k);
 *           1: Y stored transposed, i.e. the k x m matrix Omega^T A^T row-major
 *           (element (i, c) at Y + c*ldy + i, ldy >= m) -- the transposed form
 *           of the product (Sec. 4.1 transposition remark).
 *   Other arguments as for sketch_gen_matmul_dist; workspace:
 *   sketch_workspace_size(2, SK_A_F32, m, n, k, 1).  The FP32 sums run over
 *   strips of columns with FP64 strip sums, as in the row-major calls; for
 *   k > 16 (matrix cores) they are the row-major call's sums in the same order,
 *   so Y equals sketch_gen_matmul's result on the row-major copy of A bit for
 *   bit, and a row's result does not depend on m.
 */
int sketch_gen_matmul_cm(const float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                         int dist, int64_t omega_row0, int64_t omega_col0, int64_t k, void* Y,
                         int y_dtype, int64_t ldy, int y_trans, int beta, void* workspace,
                         size_t workspace_bytes, void* stream);

/*
 * The second product of the Nystrom approximation (Alg. 2: B = A Omega, then
 * C = Omega^T B with the same generated Omega):
 *
 *   C (=|+=) Omega(seed, dist)[row0 : row0+n, col0 : col0+k]^T * B
 *
 *   B   device, n x p row-major FP32, leading dim ldb (B and ldb*4 multiples of
 *       16 bytes); C device, k x p row-major (ldc >= p), storage c_dtype.
 *   Computed as (B^T Omega)^T by sketch_gen_matmul_cm (B row-major is B^T
 *   column-major); workspace: sketch_workspace_size(2, SK_A_F32, p, n, k, 1).
 */
int sketch_gen_tmatmul(const float* B, int64_t n, int64_t p, int64_t ldb, uint64_t seed, int dist,
                       int64_t omega_row0, int64_t omega_col0, int64_t k, void* C, int c_dtype,
                       int64_t ldc, int beta, void* workspace, size_t workspace_bytes,
                       void* stream);

/*
 * Per-phase timing (instrumentation; the paper times each phase separately,
 * Sec. 6): arms the NEXT product call made by this host thread
 * (sketch_gen_matmul, sketch_gen_matmul_reduce or sketch_matmul_omega) to
 * record the given HIP events (hipEvent_t, created by the caller) on its
 * stream: ev_begin before the streaming kernel, ev_mid after it, ev_end after
 * the FP64 reduction (ev_mid and ev_end are recorded together when no
 * reduction is needed).  Each pointer may be NULL.  The arming is consumed by
 * that call (also when it fails validation); pass three NULLs to disarm.
 */
int sketch_trace_events(void* ev_begin, void* ev_mid, void* ev_end);

/*
 * Materialise Omega(seed)[row0 : row0+n, col0 : col0+k] into device memory
 * (n x k FP32, leading dim ldo >= k).  This is the "communicate Omega"
 * alternative of Sec. 6.3 on one device (the operand stored in HBM instead of
 * regenerated); the generated-operand calls above never use it.
 */
int sketch_gen_omega(uint64_t seed, int64_t row0, int64_t n, int64_t col0, int64_t k,
                     float* Omega, int64_t ldo, void* stream);
/* sketch_gen_omega with Omega drawn from the distribution `dist`. */
int sketch_gen_omega_dist(uint64_t seed, int dist, int64_t row0, int64_t n, int64_t col0,
                          int64_t k, float* Omega, int64_t ldo, void* stream);

/*
 * Y (=|+=) A * Omega for an explicit Omega in device memory (n x k FP32,
 * leading dim ldo >= k): the stored-operand counterpart of sketch_gen_matmul
 * (Sec. 6.3), with the same blocking and summation order, so that it returns
 * bitwise the same Y when Omega holds the generated values.  Arguments as for
 * sketch_gen_matmul (workspace op = 0).
 */
int sketch_matmul_omega(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                        const float* a_scales, const float* Omega, int64_t ldo, int64_t k,
                        void* Y, int y_dtype, int64_t ldy, int beta, void* workspace,
                        size_t workspace_bytes, void* stream);

/*
 * Raw Philox4x32-10 stream (Sec. 6.3 generator): out[4i .. 4i+3] =
 * Philox4x32-10(ctr[4i .. 4i+3], key = (seed mod 2^32, seed div 2^32)),
 * 0 <= i < N.  ctr and out are device arrays of 4N uint32.
 */
int sketch_philox_raw(const uint32_t* ctr, uint64_t seed, uint32_t* out, int64_t N,
                      void* stream);

/*
 * The generator's normal transform alone (Sec. 6.3 generator, Box-Muller step
 * of the Omega definition above): for 0 <= i < N,
 *   (out[2i], out[2i+1]) = (rho cos theta, rho sin theta) of the word pair
 *   (words[2i], words[2i+1]), rho from the even word, theta from the odd one,
 * bit for bit the values the product kernels form.  words and out are device
 * arrays of 2N uint32 / floats, 8-byte aligned.  For exhaustive checks of the
 * transform over all 2^23 uniforms of each word.
 */
int sketch_normal_raw(const uint32_t* words, float* out, int64_t N, void* stream);

/*
 * Low-precision storage of A (precision form; untimed preprocessing):
 *   dst_dtype SK_A_BF16: Aq = bf16(A), round to nearest even; scales unused.
 *   dst_dtype SK_A_FP8_E4M3: for each 128-row block b, s_b = the smallest
 *     power of two 2^E with max|A(block)| <= 448 2^E and E >= -149
 *     (the smallest FP32 power of two; 1 for an all-zero
 *     block); Aq(i, j) = e4m3(A(i, j) / s_b), round to nearest even,
 *     saturating at +-448; scales[b] = s_b (ceil(m/128) floats).
 *   ldq in elements of the destination type; Aq and ldq*size 16-B aligned.
 */
int sketch_quantize(const float* A, int64_t m, int64_t n, int64_t lda, int dst_dtype, void* Aq,
                    int64_t ldq, float* scales, void* stream);

/*
 * Nystrom approximation (Sec. 5, Alg. 2): for a symmetric positive semidefinite
 * n x n A, B = A Omega (sketch_gen_matmul) and the core C = Omega^T B
 * (sketch_gen_tmatmul) give A~ = B C^+ B^T.  The three calls below finish it
 * on the device, in FP64.  Unlike the product calls they run several kernels;
 * they still only enqueue work.
 *
 * sketch_core_pinv: the pseudo-inverse of the core, as the paper forms it
 * (eigenvalues below a relative tolerance dropped; Sec. 6.2 uses 1e-12):
 *   S = (C + C^T) / 2 = V diag(lambda) V^T by a parallel block Jacobi
 *   eigensolver (cyclic sweeps of 2x2 rotations over 16-row block pairs, stopped
 *   when the off-diagonal Frobenius norm of the rotated S is at most
 *   8 Rp 2^-53 ||S||_F, Rp = r rounded up to a multiple of 32, or after
 *   max_sweeps sweeps), then
 *   Cp = V diag(mu) V^T, mu_i = 1 / lambda_i if |lambda_i| > tol max_j |lambda_j|,
 *   else 0.
 *   C     device, r x r row-major, leading dim ldc >= r, storage c_dtype
 *         (SK_Y_F32 or SK_Y_F64); only read.
 *   r     0 <= r <= 1024 (r = 0: nothing is done).
 *   tol   relative eigenvalue cut, 0 <= tol <= 1.
 *   max_sweeps  1 .. 100 (about 6 to 14 are needed for r <= 1024).
 *   Cp    device, r x r FP64 row-major, leading dim ldcp >= r; exactly
 *         symmetric.
 *   eigvals  device FP64 array of r (the lambda_i, unsorted) or NULL.
 *   info  device int32[2] or NULL: (sweeps run, 1 if converged else 0).
 *   workspace  device, at least sketch_core_pinv_workspace(r) bytes
 *         (16-byte aligned); its contents on entry do not matter.
 *   Errors: SK_EDTYPE, SK_EINVAL (sizes, tol, max_sweeps, NULL buffers),
 *   SK_EALIGN, SK_EWORKSPACE, SK_EHIP.
 */
size_t sketch_core_pinv_workspace(int64_t r);
int sketch_core_pinv(const void* C, int c_dtype, int64_t r, int64_t ldc, double tol,
                     int max_sweeps, double* Cp, int64_t ldcp, double* eigvals, int32_t* info,
                     void* workspace, size_t workspace_bytes, void* stream);

/*
 * Reconstruction from the factors (Table 2's relative error and rows of A~):
 *   B   device, n x r FP32 row-major, leading dim ldb >= r (1 <= r <= 1024);
 *   Cp  device, r x r FP64 (symmetric, e.g. from sketch_core_pinv), ldcp >= r.
 *   W = B Cp is formed in FP64 in the workspace, then A~(i, j) = W(i, :) B(j, :)^T,
 *   every sum in FP64 in a fixed order.
 * sketch_nystrom_error: sums (device FP64[3]) = (||A - A~||_F^2, ||A||_F^2,
 *   their ratio's square root, 0 if ||A|| = 0) for A device n x n FP32
 *   row-major, lda >= n.  n = 0: nothing is written.
 * sketch_nystrom_rows: out (device FP64, mr x n row-major, ldo >= n) = rows
 *   [row0, row0 + mr) of A~, 0 <= row0 <= n - mr.
 * workspace: sketch_nystrom_workspace(n, r) bytes (both calls), 16-byte
 * aligned.  n is limited to 64 * 65535 (SK_EUNSUPPORTED beyond).
 */
size_t sketch_nystrom_workspace(int64_t n, int64_t r);
int sketch_nystrom_error(const float* A, int64_t n, int64_t lda, const float* B, int64_t r,
                         int64_t ldb, const double* Cp, int64_t ldcp, double* sums,
                         void* workspace, size_t workspace_bytes, void* stream);
int sketch_nystrom_rows(const float* B, int64_t n, int64_t r, int64_t ldb, const double* Cp,
                        int64_t ldcp, int64_t row0, int64_t mr, double* out, int64_t ldo,
                        void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SKETCH_H */
