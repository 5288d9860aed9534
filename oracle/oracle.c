/*
 * CPU oracle for Y = A * Omega(seed).  TEST INFRASTRUCTURE ONLY: loaded by the
 * test suite, the smoke check and the benchmark's CPU-baseline leg, never by
 * the product path.  Shares no code with the GPU library.
 *
 * What the method computes (paper, Sec. 4 problem statement and Alg. 1):
 * B = A * Omega where Omega is a dense random n2 x r matrix that any process
 * can regenerate from a shared seed (Alg. 1 GenRandom, Sec. 6.3), using the
 * counter-based Philox generator (Sec. 6.3, Salmon et al.).  The local
 * product of a process is an ordinary matrix product of its A block with
 * the matching block of the global Omega, so the oracle is that product
 * written out: products of FP32 inputs are exact in FP64, sums are FP64.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *  - generator: Philox4x32-10; key = (seed lo, seed hi); Omega(j, c) takes
 *    output word (j mod 4) of the counter (q lo, q hi, c, 0), q = j div 4;
 *  - uniform: the top 23 bits x of a word give u = (2x + 1) * 2^-24;
 *  - normal: Box-Muller, word pair (0,1) -> (rho cos, rho sin) for words
 *    0 and 1, pair (2,3) likewise for words 2 and 3, where the radius comes
 *    from the even word and the angle 2*pi*u from the odd word;
 *  - the FP32 value of each normal is fixed by the operation sequence in
 *    oracle_normal_pair() below (fma-only series, correctly rounded div/sqrt).
 *  - other distributions of Omega (the paper's experiments draw uniform
 *    entries, Sec. 6.3): "uniform" is the u of the entry's own word, in (0, 1);
 *    "Rademacher" is +1 when the word's top bit is 0, else -1.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 */

#include "oracle.h"

#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 3 / Table 2). */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* key schedule: Weyl sequence, bumped before rounds 2..10 */
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void oracle_philox_raw(const uint32_t* ctr, const uint32_t key[2], uint32_t* out, int64_t N)
{
    for (int64_t i = 0; i < N; ++i) oracle_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

static void omega_words(uint64_t seed, int64_t row, int64_t col, uint32_t r[4])
{
    uint64_t q = (uint64_t)row >> 2;
    uint32_t ctr[4] = {(uint32_t)q, (uint32_t)(q >> 32), (uint32_t)col, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, r);
}

/* ------------------------------------------------------------------ */
/* FP32 normal: constants derived here from their mathematical values.  */
/* ------------------------------------------------------------------ */
static float SIN_C[5];  /* (-1)^i (pi/2)^(2i+1) / (2i+1)!, i = 0..4 */
static float COS_C[6];  /* (-1)^i (pi/2)^(2i)   / (2i)!,   i = 0..5 */
static float ATANH_C[6]; /* 1/(2i+1), i = 0..5 (series of atanh(w)/w) */
static float LN2_F;

__attribute__((constructor)) static void derive_constants(void)
{
    const long double pi = acosl(-1.0L);
    const long double h = pi / 2.0L;
    long double pw = h, fact = 1.0L;
    for (int i = 0; i < 5; ++i) {           /* odd powers 1,3,5,7,9 */
        int n = 2 * i + 1;
        if (i > 0) { pw *= h * h; fact *= (long double)(n - 1) * (long double)n; }
        long double v = pw / fact;
        SIN_C[i] = (float)((i & 1) ? -v : v);
    }
    pw = 1.0L; fact = 1.0L;
    for (int i = 0; i < 6; ++i) {           /* even powers 0,2,...,10 */
        int n = 2 * i;
        if (i > 0) { pw *= h * h; fact *= (long double)(n - 1) * (long double)n; }
        long double v = pw / fact;
        COS_C[i] = (float)((i & 1) ? -v : v);
    }
    for (int i = 0; i < 6; ++i) ATANH_C[i] = (float)(1.0L / (long double)(2 * i + 1));
    LN2_F = (float)logl(2.0L);
}

/* Natural log of u = mo * 2^-24 for an odd integer mo in [1, 2^24).
 * Split u = 2^e * f with f in [sqrt(1/2), sqrt(2)) using integer arithmetic,
 * then ln f = 2 atanh(w), w = (f-1)/(f+1), by its power series in w^2
 * truncated after the w^10 term (|w| <= 0.1716, so the tail is < 1e-10
 * relative).  ln u = e*ln2 + ln f. */
static float spec_log_u(uint32_t mo)
{
    int b = 31 - __builtin_clz(mo);                  /* 2^b <= mo < 2^(b+1) */
    if ((uint64_t)mo * (uint64_t)mo >= (1ull << (2 * b + 1))) b += 1;  /* mo/2^b >= sqrt 2 */
    int e = b - 24;
    float f = ldexpf((float)mo, -b);                 /* exact: mo < 2^24 */
    float s = f - 1.0f;                              /* exact (Sterbenz) */
    float d = f + 1.0f;
    float w = s / d;
    float w2 = w * w;
    float p = ATANH_C[5];
    p = fmaf(p, w2, ATANH_C[4]);
    p = fmaf(p, w2, ATANH_C[3]);
    p = fmaf(p, w2, ATANH_C[2]);
    p = fmaf(p, w2, ATANH_C[1]);
    p = fmaf(p, w2, ATANH_C[0]);
    float lnf = (w + w) * p;
    return fmaf((float)e, LN2_F, lnf);
}

/* cos and sin of 2*pi*u for u = mo * 2^-24, mo odd in [1, 2^24).
 * 4u = nq + f with nq the nearest integer (no ties: mo is odd) and
 * f in [-1/2, 1/2], both found exactly in integers.  With x = (pi/2) f:
 * sin x and cos x by their Taylor series in f (through f^9 and f^10), then
 * rotated by the quadrant nq. */
static void spec_cos_sin_2pi(uint32_t mo, float* c_out, float* s_out)
{
    uint32_t nq = (mo + (1u << 21)) >> 22;           /* 0..4 */
    int32_t fi = (int32_t)mo - (int32_t)(nq << 22);  /* odd, |fi| <= 2^21 */
    float f = ldexpf((float)fi, -22);                /* exact */
    float f2 = f * f;
    float ps = SIN_C[4];
    ps = fmaf(ps, f2, SIN_C[3]);
    ps = fmaf(ps, f2, SIN_C[2]);
    ps = fmaf(ps, f2, SIN_C[1]);
    ps = fmaf(ps, f2, SIN_C[0]);
    float sn = ps * f;
    float pc = COS_C[5];
    pc = fmaf(pc, f2, COS_C[4]);
    pc = fmaf(pc, f2, COS_C[3]);
    pc = fmaf(pc, f2, COS_C[2]);
    pc = fmaf(pc, f2, COS_C[1]);
    float cs = fmaf(pc, f2, COS_C[0]);
    switch (nq & 3u) {
    case 0: *c_out = cs;  *s_out = sn;  break;
    case 1: *c_out = -sn; *s_out = cs;  break;
    case 2: *c_out = -cs; *s_out = -sn; break;
    default: *c_out = sn; *s_out = -cs; break;
    }
}

void oracle_spec_log_batch(const uint32_t* mo, float* out, int64_t N)
{
    for (int64_t i = 0; i < N; ++i) out[i] = spec_log_u(mo[i]);
}

void oracle_spec_cossin_batch(const uint32_t* mo, float* c_out, float* s_out, int64_t N)
{
    for (int64_t i = 0; i < N; ++i) spec_cos_sin_2pi(mo[i], &c_out[i], &s_out[i]);
}

static uint32_t odd24(uint32_t r) { return ((r >> 9) << 1) | 1u; }

/* Box-Muller on the word pair (r_even, r_odd): returns (rho cos, rho sin). */
void oracle_normal_pair(uint32_t r_even, uint32_t r_odd, float* z_cos, float* z_sin)
{
    float L = spec_log_u(odd24(r_even));
    float rho = sqrtf(-2.0f * L);
    float c, s;
    spec_cos_sin_2pi(odd24(r_odd), &c, &s);
    *z_cos = rho * c;
    *z_sin = rho * s;
}

/* oracle_normal_pair over N word pairs (even[i], odd[i]) -> (zc[i], zs[i]). */
void oracle_normal_pairs(const uint32_t* r_even, const uint32_t* r_odd, float* z_cos,
                         float* z_sin, int64_t N)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) oracle_normal_pair(r_even[i], r_odd[i], &z_cos[i], &z_sin[i]);
}

float oracle_omega_value_dist(uint64_t seed, int64_t row, int64_t col, int dist)
{
    uint32_t r[4];
    omega_words(seed, row, col, r);
    int t = (int)(row & 3);
    if (dist == ORACLE_DIST_UNIFORM) return (float)ldexp((double)odd24(r[t]), -24);
    if (dist == ORACLE_DIST_RADEMACHER) return (r[t] >> 31) ? -1.0f : 1.0f;
    float z[4];
    oracle_normal_pair(r[0], r[1], &z[0], &z[1]);
    oracle_normal_pair(r[2], r[3], &z[2], &z[3]);
    return z[t];
}

float oracle_omega_value(uint64_t seed, int64_t row, int64_t col)
{
    return oracle_omega_value_dist(seed, row, col, ORACLE_DIST_NORMAL);
}

double oracle_omega_f64ref(uint64_t seed, int64_t row, int64_t col)
{
    uint32_t r[4];
    omega_words(seed, row, col, r);
    int t = (int)(row & 3);
    int pair = t >> 1;
    double ue = ldexp((double)odd24(r[2 * pair]), -24);
    double uo = ldexp((double)odd24(r[2 * pair + 1]), -24);
    double rho = sqrt(-2.0 * log(ue));
    double th = 2.0 * M_PI * uo;
    return (t & 1) ? rho * sin(th) : rho * cos(th);
}

void oracle_omega_block_dist(uint64_t seed, int64_t row0, int64_t n, int64_t col0, int64_t k,
                             int dist, float* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t c = 0; c < k; ++c)
            out[j * k + c] = oracle_omega_value_dist(seed, row0 + j, col0 + c, dist);
}

void oracle_omega_block(uint64_t seed, int64_t row0, int64_t n, int64_t col0, int64_t k,
                        float* out)
{
    oracle_omega_block_dist(seed, row0, n, col0, k, ORACLE_DIST_NORMAL, out);
}

/* ------------------------------------------------------------------ */
/* Products (FP64 accumulation, sequential in the contraction index).   */
/* ------------------------------------------------------------------ */
void oracle_matmul_f64(const float* A, int64_t m, int64_t n, int64_t lda, const float* Om,
                       int64_t ldo, int64_t k, double* Y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j)
                acc += (double)A[i * lda + j] * (double)Om[j * ldo + c];
            Y[i * k + c] = acc;
        }
    }
}

void oracle_gen_matmul_dist_f64(const float* A, int64_t m, int64_t n, int64_t lda,
                                uint64_t seed, int64_t row0, int64_t col0, int64_t k, int dist,
                                double* Y)
{
    if (m <= 0 || k <= 0) return;
    if (n <= 0) { memset(Y, 0, sizeof(double) * (size_t)(m * k)); return; }
    float* Om = (float*)malloc(sizeof(float) * (size_t)(n * k));
    oracle_omega_block_dist(seed, row0, n, col0, k, dist, Om);
    oracle_matmul_f64(A, m, n, lda, Om, k, k, Y);
    free(Om);
}

void oracle_gen_matmul_f64(const float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                           int64_t row0, int64_t col0, int64_t k, double* Y)
{
    oracle_gen_matmul_dist_f64(A, m, n, lda, seed, row0, col0, k, ORACLE_DIST_NORMAL, Y);
}

void oracle_gen_matmul_reduce_dist_f64(const float* const* A_b, int64_t P, int64_t m,
                                       const int64_t* n_b, const int64_t* lda_b,
                                       const int64_t* row0_b, uint64_t seed, int64_t col0,
                                       int64_t k, int dist, double* Y)
{
    if (m <= 0 || k <= 0) return;
    memset(Y, 0, sizeof(double) * (size_t)(m * k));
    double* part = (double*)malloc(sizeof(double) * (size_t)(m * k));
    for (int64_t b = 0; b < P; ++b) {
        oracle_gen_matmul_dist_f64(A_b[b], m, n_b[b], lda_b[b], seed, row0_b[b], col0, k, dist,
                                   part);
        if (n_b[b] <= 0) continue;
        for (int64_t i = 0; i < m * k; ++i) Y[i] += part[i];
    }
    free(part);
}

void oracle_gen_matmul_reduce_f64(const float* const* A_b, int64_t P, int64_t m,
                                  const int64_t* n_b, const int64_t* lda_b,
                                  const int64_t* row0_b, uint64_t seed, int64_t col0,
                                  int64_t k, double* Y)
{
    oracle_gen_matmul_reduce_dist_f64(A_b, P, m, n_b, lda_b, row0_b, seed, col0, k,
                                      ORACLE_DIST_NORMAL, Y);
}

/* ------------------------------------------------------------------ */
/* Column-major A, and the second Nystrom product.                     */
/* ------------------------------------------------------------------ */
/* Y = A * Omega[row0:row0+n, col0:col0+k] with A column-major: element
 * (i, j) at A[j * lda + i]; Y row-major m x k (FP64). */
void oracle_gen_matmul_cm_f64(const float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                              int64_t row0, int64_t col0, int64_t k, int dist, double* Y)
{
    if (m <= 0 || k <= 0) return;
    memset(Y, 0, sizeof(double) * (size_t)(m * k));
    if (n <= 0) return;
    float* Om = (float*)malloc(sizeof(float) * (size_t)(n * k));
    oracle_omega_block_dist(seed, row0, n, col0, k, dist, Om);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j)
                acc += (double)A[j * lda + i] * (double)Om[j * k + c];
            Y[i * k + c] = acc;
        }
    free(Om);
}

/* Alg. 2's second product: C (k x p, row-major, FP64) =
 * Omega[row0:row0+n, col0:col0+k]^T * B, B row-major n x p (leading dim ldb). */
void oracle_gen_tmatmul_f64(const float* B, int64_t n, int64_t p, int64_t ldb, uint64_t seed,
                            int64_t row0, int64_t col0, int64_t k, int dist, double* C)
{
    if (k <= 0 || p <= 0) return;
    memset(C, 0, sizeof(double) * (size_t)(k * p));
    if (n <= 0) return;
    float* Om = (float*)malloc(sizeof(float) * (size_t)(n * k));
    oracle_omega_block_dist(seed, row0, n, col0, k, dist, Om);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < k; ++a)
        for (int64_t b = 0; b < p; ++b) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j)
                acc += (double)Om[j * k + a] * (double)B[j * ldb + b];
            C[a * p + b] = acc;
        }
    free(Om);
}

/* ------------------------------------------------------------------ */
/* Low-precision storage formats.                                      */
/* ------------------------------------------------------------------ */
void oracle_bf16_encode(const float* x, uint16_t* out, int64_t N)
{
    for (int64_t i = 0; i < N; ++i) {
        uint32_t u;
        memcpy(&u, &x[i], 4);
        if ((u & 0x7fffffffu) > 0x7f800000u) { out[i] = (uint16_t)((u >> 16) | 0x40u); continue; }
        uint32_t hi = u >> 16, rem = u & 0xffffu;
        /* nearest of the two neighbouring bf16 values; ties go to the even one */
        if (rem > 0x8000u || (rem == 0x8000u && (hi & 1u))) hi += 1u;
        out[i] = (uint16_t)hi;
    }
}

double oracle_bf16_decode(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* E4M3FN: sign, 4 exponent bits (bias 7), 3 mantissa bits.  Normal values
 * 2^(E-7) (1 + M/8) for E = 1..15 except E=15,M=7 (NaN); subnormals
 * 2^-6 (M/8).  Largest finite value 448. */
double oracle_fp8e4m3_decode(uint8_t b)
{
    int s = b >> 7, E = (b >> 3) & 15, M = b & 7;
    if (E == 15 && M == 7) return NAN;
    double v = (E == 0) ? ldexp((double)M / 8.0, -6) : ldexp(1.0 + (double)M / 8.0, E - 7);
    return s ? -v : v;
}

uint8_t oracle_fp8e4m3_encode(double x)
{
    if (isnan(x)) return 0x7f;
    uint8_t sign = (x < 0 || (x == 0 && signbit(x))) ? 0x80 : 0x00;
    double a = fabs(x);
    if (a >= 448.0) return (uint8_t)(sign | 0x7e);       /* saturate */
    /* spacing of the grid around a: 2^-9 below 2^-6, else 2^(floor(log2 a) - 3) */
    double step;
    if (a < ldexp(1.0, -6)) {
        step = ldexp(1.0, -9);
    } else {
        int e;
        frexp(a, &e);                                     /* a = m 2^e, m in [0.5,1) */
        step = ldexp(1.0, (e - 1) - 3);
    }
    double qd = a / step;                                 /* exact: power-of-two step */
    double fl = floor(qd);
    double frac = qd - fl;
    double qi = fl;
    if (frac > 0.5 || (frac == 0.5 && fmod(fl, 2.0) != 0.0)) qi = fl + 1.0;
    double v = qi * step;
    if (v >= 448.0) return (uint8_t)(sign | 0x7e);
    if (v == 0.0) return sign;
    /* encode v exactly */
    if (v < ldexp(1.0, -6)) {
        int M = (int)(v / ldexp(1.0, -9));
        return (uint8_t)(sign | M);
    }
    int e;
    double mfr = frexp(v, &e);                            /* v = mfr 2^e, mfr in [0.5,1) */
    int E = (e - 1) + 7;
    int M = (int)((mfr * 2.0 - 1.0) * 8.0);
    return (uint8_t)(sign | (E << 3) | M);
}

void oracle_quantize_fp8_rows128(const float* A, int64_t m, int64_t n, int64_t lda,
                                 uint8_t* Q, int64_t ldq, float* scales)
{
    for (int64_t b = 0; b * 128 < m; ++b) {
        int64_t i0 = b * 128, i1 = (i0 + 128 < m) ? i0 + 128 : m;
        double amax = 0.0;
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double a = fabs((double)A[i * lda + j]);
                if (a > amax) amax = a;
            }
        int E = 0;
        if (amax > 0.0) {
            int ea;
            double ma = frexp(amax, &ea);                 /* amax = ma 2^ea */
            /* smallest E with amax <= 448 2^E = 0.875 2^(9+E) */
            E = ea - 9 + (ma > 0.875 ? 1 : 0);
            /* the scale is stored as FP32: its smallest power of two is 2^-149 */
            if (E < -149) E = -149;
        }
        double s = ldexp(1.0, E);
        scales[b] = (float)s;
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t j = 0; j < n; ++j)
                Q[i * ldq + j] = oracle_fp8e4m3_encode((double)A[i * lda + j] / s);
    }
}

void oracle_gen_matmul_q_f64(const void* Aq, int dtype, int64_t m, int64_t n, int64_t lda,
                             const float* scales, uint64_t seed, int64_t row0, int64_t col0,
                             int64_t k, double* Y)
{
    if (m <= 0 || k <= 0) return;
    if (n <= 0) { memset(Y, 0, sizeof(double) * (size_t)(m * k)); return; }
    float* Om = (float*)malloc(sizeof(float) * (size_t)(n * k));
    oracle_omega_block(seed, row0, n, col0, k, Om);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double s = scales ? (double)scales[i / 128] : 1.0;
        for (int64_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double a = (dtype == 1) ? oracle_bf16_decode(((const uint16_t*)Aq)[i * lda + j])
                                        : oracle_fp8e4m3_decode(((const uint8_t*)Aq)[i * lda + j]);
                acc += a * s * (double)Om[j * k + c];
            }
            Y[i * k + c] = acc;
        }
    }
    free(Om);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
