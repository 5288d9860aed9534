// Argument checks shared by the direct calls and the request server: every
// argument error is found on the host before anything is enqueued.
#pragma once

#include <stdint.h>

#include "../../include/sketch.h"
#include "sk_internal.hpp"

namespace sk {
namespace check {

constexpr int64_t kMaxRow = (int64_t)1 << 62;
constexpr int64_t kMaxCol = (int64_t)1 << 32;
constexpr int64_t kMaxK = 1024;
constexpr int64_t kMaxGridY = 65535;

inline int elem_size(int a_dtype) { return a_dtype == SK_A_F32 ? 4 : a_dtype == SK_A_BF16 ? 2 : 1; }
inline bool adtype_ok(int t) { return t == SK_A_F32 || t == SK_A_BF16 || t == SK_A_FP8_E4M3; }
inline bool ydtype_ok(int t) { return t == SK_Y_F32 || t == SK_Y_F64; }
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
inline bool dist_ok(int d) { return d == SK_DIST_NORMAL || d == SK_DIST_UNIFORM || d == SK_DIST_RADEMACHER; }

// Checks of the output side and sizes, shared by every product call.
inline int check_common(int a_dtype, int64_t m, int64_t k, int64_t col0, const void* Y,
                        int y_dtype, int64_t ldy, int beta) {
    if (!adtype_ok(a_dtype) || !ydtype_ok(y_dtype)) return SK_EDTYPE;
    if (m < 0 || k < 0 || k > kMaxK) return SK_EINVAL;
    if (beta != 0 && beta != 1) return SK_EINVAL;
    if (col0 < 0 || col0 + k > kMaxCol) return SK_EINVAL;
    if (m == 0 || k == 0) return SK_OK;
    if (Y == nullptr || ldy < k) return SK_EINVAL;
    if (((uintptr_t)Y & (y_dtype == SK_Y_F64 ? 7u : 3u)) != 0) return SK_EALIGN;
    // grid: rows per workgroup are at most 1024 (streaming kernel), exactly
    // kMfmaRows (FP32 matrix-core kernel) or at least 256 (low-precision
    // matrix-core kernel); row blocks at most 65535
    const int64_t rows = sk::use_mfma(a_dtype, k) ? sk::kMfmaRows
                         : sk::use_mfma_lp(a_dtype, k) ? 256 : 1024;
    if (m > kMaxGridY * rows) return SK_EUNSUPPORTED;
    return SK_OK;
}

// Checks of one A block (device memory).
inline int check_block(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                       int64_t row0, const float* scales) {
    if (n < 0 || row0 < 0 || row0 > kMaxRow - n) return SK_EINVAL;
    if (n == 0 || m == 0) return SK_OK;
    if (A == nullptr || lda < n) return SK_EINVAL;
    if (!aligned16(A) || (lda * elem_size(a_dtype)) % 16 != 0) return SK_EALIGN;
    if (a_dtype == SK_A_FP8_E4M3 && scales == nullptr) return SK_EINVAL;
    if (scales && ((uintptr_t)scales & 3u)) return SK_EALIGN;
    return SK_OK;
}

}  // namespace check
}  // namespace sk
