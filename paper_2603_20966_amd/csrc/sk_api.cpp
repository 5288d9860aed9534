// C ABI of the sketch library: argument validation and dispatch.  Every
// argument error is returned before anything is enqueued.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "../../include/sketch.h"
#include "sk_check.hpp"
#include "sk_internal.hpp"

namespace {

using namespace sk::check;

int from_hip(hipError_t e) { return e == hipSuccess ? SK_OK : SK_EHIP; }

// Events armed by sketch_trace_events for the next product call of this thread.
thread_local sk::TraceEvents g_trace;

sk::TraceEvents take_trace() {
    sk::TraceEvents t = g_trace;
    g_trace = sk::TraceEvents{};
    return t;
}

size_t workspace_for(int op, int adtype, int64_t m, int64_t n, int64_t k, int64_t P) {
    const int64_t C = sk::strip_width_for(adtype, k);
    const int64_t S = (op == 0) ? (n + C - 1) / C : n / C + P;
    return sk::product_workspace_bytes(adtype, m, S, k);
}

int check_workspace(size_t need, const void* ws, size_t bytes) {
    if (need == 0) return SK_OK;
    if (ws == nullptr || bytes < need) return SK_EWORKSPACE;
    if (!aligned16(ws)) return SK_EALIGN;
    return SK_OK;
}

int run_product(sk::GemmLaunch& g, int64_t n_total) {
    if (g.m == 0 || g.k == 0 || n_total == 0) {
        const sk::TraceEvents& t = g.trace;
        for (hipEvent_t e : {t.begin, t.mid}) if (e) (void)hipEventRecord(e, g.stream);
        if (g.m > 0 && g.k > 0 && !g.beta) {
            const int st = from_hip(sk::launch_zero_matrix(g.Y, g.y_f64, g.m, g.k, g.ldy, g.stream));
            if (st != SK_OK) return st;
        }
        if (t.end) (void)hipEventRecord(t.end, g.stream);
        return SK_OK;
    }
    if (sk::use_mfma(g.adtype, g.k)) return from_hip(sk::launch_gemm_mfma(g));
    if (sk::use_mfma_lp(g.adtype, g.k)) return from_hip(sk::launch_gemm_mfma_lp(g));
    return from_hip(sk::launch_gemm_stream(g));
}

}  // namespace

extern "C" {

int sketch_abi_version(void) { return SKETCH_ABI_VERSION; }

const char* sketch_status_string(int status) {
    switch (status) {
    case SK_OK: return "ok";
    case SK_EINVAL: return "invalid argument (size, pointer, leading dimension or flag)";
    case SK_EDTYPE: return "unknown element type";
    case SK_EALIGN: return "misaligned pointer or leading dimension (16 bytes needed)";
    case SK_EWORKSPACE: return "workspace missing or too small";
    case SK_EHIP: return "HIP runtime error";
    case SK_ENOMEM: return "out of device memory";
    case SK_EUNSUPPORTED: return "unsupported request";
    case SK_EBUDGET: return "request exceeds the memory budget";
    case SK_EQUEUE: return "queue full or unknown ticket";
    case SK_ETIMEOUT: return "wait timed out before the request finished";
    case SK_ESCRATCH: return "call needs more workspace than the library's static scratch holds";
    default: return "unknown status";
    }
}

int64_t sketch_strip_width(int a_dtype, int64_t k) {
    if (!adtype_ok(a_dtype) || k < 1 || k > kMaxK) return 0;
    return sk::strip_width_for(a_dtype, k);
}

size_t sketch_workspace_size(int op, int a_dtype, int64_t m, int64_t n, int64_t k, int64_t P) {
    if ((op != 0 && op != 1 && op != 2) || !adtype_ok(a_dtype) || m < 0 || n < 0 || k < 0 ||
        k > kMaxK)
        return 0;
    if (op == 2) {   // column-major A (sketch_gen_matmul_cm; sketch_gen_tmatmul with m = p)
        if (a_dtype != SK_A_F32 || m == 0 || k == 0 || n == 0) return 0;
        return sk::cm_workspace_bytes(m, n, k);
    }
    if (op == 0) P = 1;
    if (P < 1 || P > sk::kMaxBlocks || m == 0 || k == 0 || n == 0) return 0;
    return workspace_for(op, a_dtype, m, n, k, P);
}

int sketch_trace_events(void* ev_begin, void* ev_mid, void* ev_end) {
    g_trace.begin = static_cast<hipEvent_t>(ev_begin);
    g_trace.mid = static_cast<hipEvent_t>(ev_mid);
    g_trace.end = static_cast<hipEvent_t>(ev_end);
    return SK_OK;
}

}  // extern "C"

namespace sk {

// Host-side checks of a sketch_gen_matmul-style call (explicit Omega when
// Omega != nullptr or ldo != 0); on success *need holds the workspace bytes
// the call requires.  Makes no HIP call.
int gen_matmul_validate(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                        const float* a_scales, int dist, int64_t omega_row0, int64_t omega_col0,
                        const float* Omega, int64_t ldo, int64_t k, const void* Y, int y_dtype,
                        int64_t ldy, int beta, size_t* need) {
    *need = 0;
    if (!dist_ok(dist)) return SK_EINVAL;
    int st = check_common(a_dtype, m, k, omega_col0, Y, y_dtype, ldy, beta);
    if (st != SK_OK) return st;
    st = check_block(A, a_dtype, m, n, lda, omega_row0, a_scales);
    if (st != SK_OK) return st;
    if (m == 0 || k == 0) return SK_OK;
    if (Omega != nullptr || ldo != 0) {
        if (n > 0 && (Omega == nullptr || ldo < k)) return SK_EINVAL;
        if (((uintptr_t)Omega & 3u) != 0) return SK_EALIGN;
    }
    *need = n > 0 ? workspace_for(0, a_dtype, m, n, k, 1) : 0;
    return SK_OK;
}

void drop_trace() { (void)take_trace(); }

int gen_matmul_impl(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                    const float* a_scales, uint64_t seed, int dist, int64_t omega_row0,
                    int64_t omega_col0, const float* Omega, int64_t ldo, int64_t k, void* Y,
                    int y_dtype, int64_t ldy, int beta, void* workspace, size_t workspace_bytes,
                    void* stream) {
    const sk::TraceEvents trace = take_trace();
    size_t need = 0;
    int st = gen_matmul_validate(A, a_dtype, m, n, lda, a_scales, dist, omega_row0, omega_col0,
                                 Omega, ldo, k, Y, y_dtype, ldy, beta, &need);
    if (st != SK_OK) return st;
    if (m == 0 || k == 0) return SK_OK;
    st = check_workspace(need, workspace, workspace_bytes);
    if (st != SK_OK) return st;
    sk::GemmLaunch g{};
    g.adtype = a_dtype;
    g.m = m;
    g.P = 1;
    g.blk[0] = sk::BlockDesc{A, n, lda, omega_row0, a_scales};
    g.k = k;
    g.col0 = (uint32_t)omega_col0;
    g.seed = seed;
    g.dist = dist;
    g.omega = Omega;
    g.ldo = ldo;
    g.Y = Y;
    g.y_f64 = (y_dtype == SK_Y_F64);
    g.ldy = ldy;
    g.beta = beta;
    g.workspace = workspace;
    g.workspace_bytes = workspace_bytes;
    g.stream = static_cast<hipStream_t>(stream);
    g.trace = trace;
    return run_product(g, n);
}

}  // namespace sk

extern "C" {

int sketch_gen_matmul(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                      const float* a_scales, uint64_t seed, int64_t omega_row0,
                      int64_t omega_col0, int64_t k, void* Y, int y_dtype, int64_t ldy,
                      int beta, void* workspace, size_t workspace_bytes, void* stream) {
    return sk::gen_matmul_impl(A, a_dtype, m, n, lda, a_scales, seed, SK_DIST_NORMAL, omega_row0,
                           omega_col0, nullptr, 0, k, Y, y_dtype, ldy, beta, workspace,
                           workspace_bytes, stream);
}

int sketch_gen_matmul_dist(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                           const float* a_scales, uint64_t seed, int dist, int64_t omega_row0,
                           int64_t omega_col0, int64_t k, void* Y, int y_dtype, int64_t ldy,
                           int beta, void* workspace, size_t workspace_bytes, void* stream) {
    return sk::gen_matmul_impl(A, a_dtype, m, n, lda, a_scales, seed, dist, omega_row0, omega_col0,
                           nullptr, 0, k, Y, y_dtype, ldy, beta, workspace, workspace_bytes,
                           stream);
}

int sketch_matmul_omega(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                        const float* a_scales, const float* Omega, int64_t ldo, int64_t k,
                        void* Y, int y_dtype, int64_t ldy, int beta, void* workspace,
                        size_t workspace_bytes, void* stream) {
    if (n > 0 && m > 0 && k > 0 && (Omega == nullptr || ldo < k)) return SK_EINVAL;
    return sk::gen_matmul_impl(A, a_dtype, m, n, lda, a_scales, 0, SK_DIST_NORMAL, 0, 0, Omega,
                           ldo < 1 ? 1 : ldo, k, Y, y_dtype, ldy, beta, workspace,
                           workspace_bytes, stream);
}

static int gen_matmul_reduce_impl(const void* const* A_b, int64_t P, int a_dtype, int64_t m,
                                  const int64_t* n_b, const int64_t* lda_b,
                                  const int64_t* row0_b, const float* const* a_scales_b,
                                  uint64_t seed, int dist, int64_t omega_col0, int64_t k, void* Y,
                                  int y_dtype, int64_t ldy, int beta, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    const sk::TraceEvents trace = take_trace();
    if (!dist_ok(dist)) return SK_EINVAL;
    int st = check_common(a_dtype, m, k, omega_col0, Y, y_dtype, ldy, beta);
    if (st != SK_OK) return st;
    if (P < 1 || P > sk::kMaxBlocks) return SK_EINVAL;
    if (A_b == nullptr || n_b == nullptr || lda_b == nullptr || row0_b == nullptr)
        return SK_EINVAL;
    int64_t n_total = 0;
    for (int64_t b = 0; b < P; ++b) {
        const float* sc = a_scales_b ? a_scales_b[b] : nullptr;
        st = check_block(A_b[b], a_dtype, m, n_b[b], lda_b[b], row0_b[b], sc);
        if (st != SK_OK) return st;
        n_total += n_b[b];
    }
    if (m == 0 || k == 0) return SK_OK;
    sk::GemmLaunch g{};
    g.adtype = a_dtype;
    g.m = m;
    g.P = (int)P;
    for (int64_t b = 0; b < P; ++b)
        g.blk[b] = sk::BlockDesc{A_b[b], n_b[b], lda_b[b], row0_b[b],
                                 a_scales_b ? a_scales_b[b] : nullptr};
    g.k = k;
    g.col0 = (uint32_t)omega_col0;
    g.seed = seed;
    g.dist = dist;
    g.omega = nullptr;
    g.Y = Y;
    g.y_f64 = (y_dtype == SK_Y_F64);
    g.ldy = ldy;
    g.beta = beta;
    g.workspace = workspace;
    g.workspace_bytes = workspace_bytes;
    g.stream = static_cast<hipStream_t>(stream);
    g.trace = trace;
    const int64_t S = sk::count_strips(g);
    st = check_workspace(n_total > 0 ? sk::product_workspace_bytes(a_dtype, m, S, k) : 0,
                         workspace, workspace_bytes);
    if (st != SK_OK) return st;
    return run_product(g, n_total);
}

int sketch_gen_matmul_reduce(const void* const* A_b, int64_t P, int a_dtype, int64_t m,
                             const int64_t* n_b, const int64_t* lda_b, const int64_t* row0_b,
                             const float* const* a_scales_b, uint64_t seed, int64_t omega_col0,
                             int64_t k, void* Y, int y_dtype, int64_t ldy, int beta,
                             void* workspace, size_t workspace_bytes, void* stream) {
    return gen_matmul_reduce_impl(A_b, P, a_dtype, m, n_b, lda_b, row0_b, a_scales_b, seed,
                                  SK_DIST_NORMAL, omega_col0, k, Y, y_dtype, ldy, beta,
                                  workspace, workspace_bytes, stream);
}

int sketch_gen_matmul_reduce_dist(const void* const* A_b, int64_t P, int a_dtype, int64_t m,
                                  const int64_t* n_b, const int64_t* lda_b,
                                  const int64_t* row0_b, const float* const* a_scales_b,
                                  uint64_t seed, int dist, int64_t omega_col0, int64_t k,
                                  void* Y, int y_dtype, int64_t ldy, int beta, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    return gen_matmul_reduce_impl(A_b, P, a_dtype, m, n_b, lda_b, row0_b, a_scales_b, seed, dist,
                                  omega_col0, k, Y, y_dtype, ldy, beta, workspace,
                                  workspace_bytes, stream);
}

int sketch_gen_omega_dist(uint64_t seed, int dist, int64_t row0, int64_t n, int64_t col0,
                          int64_t k, float* Omega, int64_t ldo, void* stream) {
    if (!dist_ok(dist)) return SK_EINVAL;
    if (n < 0 || k < 0 || row0 < 0 || row0 > kMaxRow - n || col0 < 0 || col0 + k > kMaxCol)
        return SK_EINVAL;
    if (n == 0 || k == 0) return SK_OK;
    if (Omega == nullptr || ldo < k) return SK_EINVAL;
    if (((uintptr_t)Omega & 3u) != 0) return SK_EALIGN;
    return from_hip(sk::launch_gen_omega(seed, dist, row0, n, col0, k, Omega, ldo,
                                         static_cast<hipStream_t>(stream)));
}

int sketch_gen_omega(uint64_t seed, int64_t row0, int64_t n, int64_t col0, int64_t k,
                     float* Omega, int64_t ldo, void* stream) {
    return sketch_gen_omega_dist(seed, SK_DIST_NORMAL, row0, n, col0, k, Omega, ldo, stream);
}

int sketch_gen_matmul_cm(const float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                         int dist, int64_t omega_row0, int64_t omega_col0, int64_t k, void* Y,
                         int y_dtype, int64_t ldy, int y_trans, int beta, void* workspace,
                         size_t workspace_bytes, void* stream) {
    if (!dist_ok(dist) || (y_trans != 0 && y_trans != 1)) return SK_EINVAL;
    if (!ydtype_ok(y_dtype)) return SK_EDTYPE;
    if (m < 0 || n < 0 || k < 0 || k > kMaxK || (beta != 0 && beta != 1)) return SK_EINVAL;
    if (omega_col0 < 0 || omega_col0 + k > kMaxCol) return SK_EINVAL;
    if (omega_row0 < 0 || omega_row0 > kMaxRow - n) return SK_EINVAL;
    if (m == 0 || k == 0) return SK_OK;
    if (Y == nullptr || ldy < (y_trans ? m : k)) return SK_EINVAL;
    if (((uintptr_t)Y & (y_dtype == SK_Y_F64 ? 7u : 3u)) != 0) return SK_EALIGN;
    if (n > 0) {
        if (A == nullptr || lda < m) return SK_EINVAL;
        if (!aligned16(A) || (lda * 4) % 16 != 0) return SK_EALIGN;
    }
    const int64_t S = n > 0 ? sk::cm_strips(n, k) : 0;
    const int64_t tiles = S * ((m + 255) / 256) * ((k + sk::kColGroup - 1) / sk::kColGroup);
    if (tiles > ((int64_t)1 << 31) - 8) return SK_EUNSUPPORTED;
    int st = check_workspace(n > 0 ? sk::cm_workspace_bytes(m, n, k) : 0, workspace,
                             workspace_bytes);
    if (st != SK_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0) {
        if (beta) return SK_OK;
        if (!y_trans) return from_hip(sk::launch_zero_matrix(Y, y_dtype == SK_Y_F64, m, k, ldy, s));
        return from_hip(sk::launch_zero_matrix(Y, y_dtype == SK_Y_F64, k, m, ldy, s));
    }
    sk::CmLaunch g{};
    g.A = A;
    g.m = m;
    g.n = n;
    g.lda = lda;
    g.row0 = omega_row0;
    g.seed = seed;
    g.dist = dist;
    g.col0 = (uint32_t)omega_col0;
    g.k = k;
    g.Y = Y;
    g.ldy = ldy;
    g.y_trans = y_trans;
    g.y_f64 = (y_dtype == SK_Y_F64);
    g.beta = beta;
    g.workspace = workspace;
    g.stream = s;
    return from_hip(sk::launch_gemm_cm(g));
}

int sketch_gen_tmatmul(const float* B, int64_t n, int64_t p, int64_t ldb, uint64_t seed, int dist,
                       int64_t omega_row0, int64_t omega_col0, int64_t k, void* C, int c_dtype,
                       int64_t ldc, int beta, void* workspace, size_t workspace_bytes,
                       void* stream) {
    // C (k x p) = Omega^T B = (B^T Omega)^T: B row-major n x p is B^T column-major
    // (p x n, leading dim ldb), and C row-major is (B^T Omega) stored transposed.
    if (ldc < p && p > 0 && k > 0) return SK_EINVAL;
    return sketch_gen_matmul_cm(B, p, n, ldb, seed, dist, omega_row0, omega_col0, k, C, c_dtype,
                                ldc, 1, beta, workspace, workspace_bytes, stream);
}

int sketch_philox_raw(const uint32_t* ctr, uint64_t seed, uint32_t* out, int64_t N,
                      void* stream) {
    if (N < 0) return SK_EINVAL;
    if (N == 0) return SK_OK;
    if (ctr == nullptr || out == nullptr) return SK_EINVAL;
    if (!aligned16(ctr) || !aligned16(out)) return SK_EALIGN;
    return from_hip(sk::launch_philox_raw(ctr, seed, out, N, static_cast<hipStream_t>(stream)));
}

int sketch_normal_raw(const uint32_t* words, float* out, int64_t N, void* stream) {
    if (N < 0) return SK_EINVAL;
    if (N == 0) return SK_OK;
    if (words == nullptr || out == nullptr) return SK_EINVAL;
    if (((uintptr_t)words & 7u) != 0 || ((uintptr_t)out & 7u) != 0) return SK_EALIGN;
    return from_hip(sk::launch_normal_raw(words, out, N, static_cast<hipStream_t>(stream)));
}

int sketch_quantize(const float* A, int64_t m, int64_t n, int64_t lda, int dst_dtype, void* Aq,
                    int64_t ldq, float* scales, void* stream) {
    if (dst_dtype != SK_A_BF16 && dst_dtype != SK_A_FP8_E4M3) return SK_EDTYPE;
    if (m < 0 || n < 0) return SK_EINVAL;
    if (m == 0) return SK_OK;
    if (dst_dtype == SK_A_FP8_E4M3 && scales == nullptr) return SK_EINVAL;
    if (scales && ((uintptr_t)scales & 3u)) return SK_EALIGN;
    if (n > 0) {
        if (A == nullptr || Aq == nullptr || lda < n || ldq < n) return SK_EINVAL;
        if (((uintptr_t)A & 3u) != 0) return SK_EALIGN;
        if (!aligned16(Aq) || (ldq * elem_size(dst_dtype)) % 16 != 0) return SK_EALIGN;
    }
    if (m > kMaxGridY) return SK_EUNSUPPORTED;
    return from_hip(sk::launch_quantize(A, m, n, lda, dst_dtype, Aq, ldq, scales,
                                        static_cast<hipStream_t>(stream)));
}

size_t sketch_core_pinv_workspace(int64_t r) {
    if (r < 0 || r > sk::kPinvMaxR) return 0;
    return sk::pinv_workspace_bytes(r);
}

int sketch_core_pinv(const void* C, int c_dtype, int64_t r, int64_t ldc, double tol,
                     int max_sweeps, double* Cp, int64_t ldcp, double* eigvals, int32_t* info,
                     void* workspace, size_t workspace_bytes, void* stream) {
    if (c_dtype != SK_Y_F32 && c_dtype != SK_Y_F64) return SK_EDTYPE;
    if (r < 0 || r > sk::kPinvMaxR) return SK_EINVAL;
    if (!(tol >= 0.0) || tol > 1.0 || max_sweeps < 1 || max_sweeps > 100) return SK_EINVAL;
    if (r == 0) return SK_OK;
    if (C == nullptr || Cp == nullptr || ldc < r || ldcp < r) return SK_EINVAL;
    const uintptr_t cal = c_dtype == SK_Y_F64 ? 7u : 3u;
    if (((uintptr_t)C & cal) || ((uintptr_t)Cp & 7u) || ((uintptr_t)eigvals & 7u) ||
        ((uintptr_t)info & 3u))
        return SK_EALIGN;
    const int st = check_workspace(sk::pinv_workspace_bytes(r), workspace, workspace_bytes);
    if (st != SK_OK) return st;
    return from_hip(sk::launch_core_pinv(C, c_dtype == SK_Y_F64, r, ldc, tol, max_sweeps, Cp, ldcp,
                                         eigvals, info, workspace,
                                         static_cast<hipStream_t>(stream)));
}

size_t sketch_nystrom_workspace(int64_t n, int64_t r) {
    if (n < 0 || r < 0 || r > sk::kPinvMaxR) return 0;
    return sk::nystrom_workspace_bytes(n, r);
}

namespace {
int check_nystrom(const float* B, int64_t n, int64_t r, int64_t ldb, const double* Cp,
                  int64_t ldcp, const void* ws, size_t wsb) {
    if (n < 0 || r < 1 || r > sk::kPinvMaxR) return SK_EINVAL;
    if (n == 0) return SK_OK;
    if (B == nullptr || Cp == nullptr || ldb < r || ldcp < r) return SK_EINVAL;
    if (((uintptr_t)B & 3u) || ((uintptr_t)Cp & 7u)) return SK_EALIGN;
    if ((n + 63) / 64 > kMaxGridY) return SK_EUNSUPPORTED;
    return check_workspace(sk::nystrom_workspace_bytes(n, r), ws, wsb);
}
}  // namespace

int sketch_nystrom_error(const float* A, int64_t n, int64_t lda, const float* B, int64_t r,
                         int64_t ldb, const double* Cp, int64_t ldcp, double* sums,
                         void* workspace, size_t workspace_bytes, void* stream) {
    int st = check_nystrom(B, n, r, ldb, Cp, ldcp, workspace, workspace_bytes);
    if (st != SK_OK || n == 0) return st;
    if (A == nullptr || sums == nullptr || lda < n) return SK_EINVAL;
    if (((uintptr_t)A & 3u) || ((uintptr_t)sums & 7u)) return SK_EALIGN;
    return from_hip(sk::launch_nystrom(A, lda, B, n, r, ldb, Cp, ldcp, 0, n, nullptr, 0, sums,
                                       workspace, static_cast<hipStream_t>(stream)));
}

int sketch_nystrom_rows(const float* B, int64_t n, int64_t r, int64_t ldb, const double* Cp,
                        int64_t ldcp, int64_t row0, int64_t mr, double* out, int64_t ldo,
                        void* workspace, size_t workspace_bytes, void* stream) {
    int st = check_nystrom(B, n, r, ldb, Cp, ldcp, workspace, workspace_bytes);
    if (st != SK_OK) return st;
    if (row0 < 0 || mr < 0 || row0 > n - mr) return SK_EINVAL;
    if (n == 0 || mr == 0) return SK_OK;
    if (out == nullptr || ldo < n) return SK_EINVAL;
    if ((uintptr_t)out & 7u) return SK_EALIGN;
    return from_hip(sk::launch_nystrom(nullptr, 0, B, n, r, ldb, Cp, ldcp, row0, mr, out, ldo,
                                       nullptr, workspace, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
