// Column-major A: Y = A * Omega(seed) with A stored by columns (element (i, j)
// at A + j*lda + i), the paper's storage order (Secs. 6.5 and 6.6), and optionally Y
// stored transposed (the form Omega^T A^T of the transposition remark in
// Sec. 4.1).  The same kernel computes Alg. 2's second product C = Omega^T B:
// a row-major B (n x p) is B^T stored by columns, and C = (B^T Omega)^T.
//
// Tile of one workgroup (256 threads = 4 waves): 256 rows x one strip of
// columns x <= 16 sketch columns.  Lane l of every wave owns rows 4l .. 4l+3 of
// the tile; a column of the tile is one contiguous 1 KB run that a wave reads
// with one 16-byte load per lane.  The four waves take the strip's columns
// round-robin, each accumulating its own partial sums in registers (no
// cross-lane reduction: a lane's rows are its own), and Omega's row for a
// column is a broadcast read from LDS.  At the end waves 1..3 hand their sums
// to wave 0 through LDS, which adds them in wave order and writes the strip
// partial.  The FP64 strip sum is the shared reduction kernel, so results do
// not depend on the tile grid.  This kernel serves k <= 16; wider sketches go
// to the matrix cores (k_gemm_cm_mfma), which read A once for all k.
#include <algorithm>

#include "sk_device.hpp"
#include "sk_internal.hpp"

#pragma clang fp contract(off)

namespace sk {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kCmRows = 256;   // rows per tile: 64 lanes x 4 rows
constexpr int kCmUnroll = 8;   // columns per wave per step (loads in flight)

struct CmArgs {
    const float* A;
    int64_t m, n, lda;
    int64_t row0;
    uint32_t key0, key1, col0;
    int dist;
    int64_t k;
    void* Y;
    int64_t ldy;
    int y_trans, y_f64, beta;
    float* partials;
    int S;                // strips
    int num_rb;           // row tiles
    int64_t tiles, tiles8;
};

__device__ __forceinline__ void lds_barrier_c() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int K>
__global__ __launch_bounds__(256) void k_gemm_cm(const CmArgs a) {
    constexpr int C = cm_strip_width(K);
    constexpr int KP = (K + 3) / 4 * 4;      // Omega row padded to whole float4s
    // the Omega strip, reused at the end for the hand-off of waves 1..3
    constexpr int kLdsRows = C > 3 * kCmRows ? C : 3 * kCmRows;
    __shared__ __attribute__((aligned(16))) float om[kLdsRows * KP];

    const int64_t id = blockIdx.x;
    const int64_t t = (id % 8) * a.tiles8 + id / 8;     // XCD-grouped tile order
    if (t >= a.tiles) return;
    const int strip = (int)(t % a.S);
    const int rb = (int)((t / a.S) % a.num_rb);
    const int cg = (int)(t / ((int64_t)a.S * a.num_rb));
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t col_begin = (int64_t)strip * C;
    const int w = (int)min<int64_t>(C, a.n - col_begin);
    const int c_base = cg * kColGroup;
    const int kg = (int)min<int64_t>(kColGroup, a.k - c_base);
    const int64_t r = (int64_t)rb * kCmRows + 4 * lane;   // first row of the lane

    // ---- Omega rows of the strip -> LDS (om[j*KP + c]) ----------------------------
    {
        const int64_t g0 = a.row0 + col_begin;
        const int64_t q_lo = g0 >> 2;
        const int nq = (int)(((g0 + w - 1) >> 2) - q_lo + 1);
        for (int it = tid; it < nq * kg; it += 256) {
            const int qi = it / kg;
            const int c = it - qi * kg;
            const float4 z = omega4_dist((uint64_t)(q_lo + qi), a.col0 + (uint32_t)(c_base + c),
                                         a.key0, a.key1, a.dist);
            const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = 4 * (q_lo + qi) + u - g0;
                if (j >= 0 && j < w) om[j * KP + c] = zz[u];
            }
        }
        for (int it = tid; it < w * KP; it += 256)
            if (it % KP >= kg) om[it] = 0.0f;
    }
    lds_barrier_c();

    // ---- stream the columns of the strip: wave w takes j = w, w + 4, ... ----------
    const bool full = r + 3 < a.m;
    const int nrow = full ? 4 : (int)max<int64_t>(0, a.m - r);
    const float* base = a.A + col_begin * a.lda + r;
    auto load = [&](int j) -> v4f {
        const float* p = base + (int64_t)j * a.lda;
        if (full) return __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
        v4f v = {0.f, 0.f, 0.f, 0.f};
        for (int e = 0; e < nrow; ++e) v[e] = p[e];
        return v;
    };
    float acc[4][K];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < K; ++c) acc[e][c] = 0.0f;

    auto fma_col = [&](const v4f x, int j) {
        float wv[KP];
#pragma unroll
        for (int q = 0; q < KP / 4; ++q) {
            const v4f o = *reinterpret_cast<const v4f*>(&om[j * KP + 4 * q]);
            wv[4 * q] = o[0];
            wv[4 * q + 1] = o[1];
            wv[4 * q + 2] = o[2];
            wv[4 * q + 3] = o[3];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < K; ++c) acc[e][c] = __builtin_fmaf(x[e], wv[c], acc[e][c]);
    };

    constexpr int STEP = 4 * kCmUnroll;      // columns per workgroup step
    const int nfull = w / STEP;
    v4f buf[2][kCmUnroll];
    auto issue = [&](v4f* b, int s) {
#pragma unroll
        for (int u = 0; u < kCmUnroll; ++u) b[u] = load(s * STEP + wave + 4 * u);
    };
    auto consume = [&](const v4f* b, int s) {
#pragma unroll
        for (int u = 0; u < kCmUnroll; ++u) fma_col(b[u], s * STEP + wave + 4 * u);
    };
    if (nrow > 0) {
        if (nfull > 0) issue(buf[0], 0);
        for (int s = 0; s < nfull; s += 2) {
            if (s + 1 < nfull) issue(buf[1], s + 1);
            consume(buf[0], s);
            if (s + 1 < nfull) {
                if (s + 2 < nfull) issue(buf[0], s + 2);
                consume(buf[1], s + 1);
            }
        }
        for (int j = nfull * STEP + wave; j < w; j += 4) fma_col(load(j), j);
    }

    // ---- waves 1..3 hand their sums to wave 0 (LDS reused), added in wave order ----
    lds_barrier_c();
    if (wave > 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < K; ++c) om[((wave - 1) * kCmRows + 4 * lane + e) * KP + c] = acc[e][c];
    }
    lds_barrier_c();
    if (wave != 0) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t row = r + e;
        if (row >= a.m) continue;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            if (c >= kg) continue;
            float v = acc[e][c];
#pragma unroll
            for (int q = 0; q < 3; ++q) v += om[(q * kCmRows + 4 * lane + e) * KP + c];
            const int64_t col = c_base + c;
            if (a.S == 1) {
                const int64_t off = a.y_trans ? col * a.ldy + row : row * a.ldy + col;
                double y = (double)v;
                if (a.y_f64) {
                    double* Yp = static_cast<double*>(a.Y) + off;
                    if (a.beta) y += *Yp;
                    *Yp = y;
                } else {
                    float* Yp = static_cast<float*>(a.Y) + off;
                    if (a.beta) y += (double)*Yp;
                    *Yp = (float)y;
                }
            } else {
                a.partials[((int64_t)strip * a.m + row) * a.k + col] = v;
            }
        }
    }
}

// Few rows (m <= kSkinnyRows; e.g. B^T of the Nystrom second product with a
// narrow sketch): the tile above would leave all but m/4 lanes of one wave
// idle and walk each wave's 256 columns of a strip one load round at a time.
// Here a workgroup takes one strip and one group of sketch columns; all its
// kSkinnyThreads threads stage the strip's 1024 columns of A (room for 8 rows when
// m <= 8 and k <= 8, else 16) and their Omega rows in LDS at once, and thread
// (w, i, c) runs the chain that wave w of the tile kernel runs for row i and
// sketch column c (waves 0..3): columns j = w, w + 4, ... of
// the strip in order, FP32 fma, then the four chains added in wave order.  Every
// sum is the tile kernel's, bit for bit.  The other twelve waves only help stage:
// with four waves the Philox work of a strip (1280 quads at k = 5) ran five quads
// deep per thread with nothing to hide its latency.
constexpr int kSkinnyRows = 16;
constexpr int kSkinnyThreads = 1024;

// SUB strip columns staged per step, MP rows (LDS pitch of a column).
template <int K, int SUB, int MP>
__global__ __launch_bounds__(kSkinnyThreads) void k_gemm_cm_skinny(const CmArgs a) {
    constexpr int C = cm_strip_width(K);
    constexpr int KP = (K + 3) / 4 * 4;
    constexpr int CQ = (K + 3) / 4;                    // sketch columns per thread
    static_assert(MP <= kSkinnyRows && C % SUB == 0 && SUB % 4 == 0, "staging geometry");
    // Staged by chain: column j of the step sits in the block of wave j % 4, at
    // position j / 4 of a row of pitch PJ (4 floats of padding keep the rows of one
    // wave's reads on different banks), so a chain's 8 columns of a batch are two
    // 16-byte LDS reads
    constexpr int PJ = SUB / 4 + 4;
    __shared__ __attribute__((aligned(16))) float om[4 * KP * PJ];   // [j % 4][c][j / 4]
    __shared__ __attribute__((aligned(16))) float as[4 * MP * PJ];   // [j % 4][i][j / 4] = A(i, j)
    __shared__ float hand[3][MP][4 * CQ];

    const int strip = (int)(blockIdx.x % a.S);
    const int cg = (int)(blockIdx.x / a.S);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;                         // chain (waves 0..3): columns j = wave (mod 4)
    const bool chain = wave < 4;
    const int i = (tid & 63) >> 2;                     // row
    const int cq = tid & 3;                            // sketch columns cq, cq + 4, ...
    const int64_t col_begin = (int64_t)strip * C;
    const int w = (int)min<int64_t>(C, a.n - col_begin);
    const int c_base = cg * kColGroup;
    const int kg = (int)min<int64_t>(kColGroup, a.k - c_base);
    const int m = (int)a.m;

    float acc[CQ];
#pragma unroll
    for (int u = 0; u < CQ; ++u) acc[u] = 0.0f;

    for (int js = 0; js < w; js += SUB) {
        const int sw = min(SUB, w - js);
        // Omega rows js .. js + sw - 1 of the strip (quads cut by the step edges are
        // generated by both steps; each entry is written from one of them)
        const int64_t g0 = a.row0 + col_begin + js;
        const int64_t q_lo = g0 >> 2;
        const int nq = (int)(((g0 + sw - 1) >> 2) - q_lo + 1);
        for (int it = tid; it < nq * kg; it += kSkinnyThreads) {
            const int qi = it / kg;
            const int c = it - qi * kg;
            const float4 z = omega4_dist((uint64_t)(q_lo + qi), a.col0 + (uint32_t)(c_base + c),
                                         a.key0, a.key1, a.dist);
            const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = 4 * (q_lo + qi) + u - g0;
                if (j >= 0 && j < sw) om[((j & 3) * KP + c) * PJ + (j >> 2)] = zz[u];
            }
        }
        for (int e = tid; e < sw * m; e += kSkinnyThreads) {
            const int j = e / m, r = e - j * m;
            as[((j & 3) * MP + r) * PJ + (j >> 2)] = a.A[(col_begin + js + j) * a.lda + r];
        }
        lds_barrier_c();
        if (chain && i < m) {
            // the chain over columns j = wave (mod 4) of this step, in order (js is a
            // multiple of 4); a batch of 8 columns is read before its fmas
            const float* xa = &as[(wave * MP + i) * PJ];
            const float* oa[CQ];
#pragma unroll
            for (int u = 0; u < CQ; ++u) oa[u] = &om[(wave * KP + min(cq + 4 * u, KP - 1)) * PJ];
            auto step = [&](int j) {
                const float x = xa[j >> 2];
#pragma unroll
                for (int u = 0; u < CQ; ++u) {
                    const int c = cq + 4 * u;
                    if (c < kg) acc[u] = __builtin_fmaf(x, oa[u][j >> 2], acc[u]);
                }
            };
            int j = wave;
            for (; j + 28 < sw; j += 32) {
                const int b = j >> 2;                  // a multiple of 8 (wave < 4)
                float x[8], o[8][CQ];
                const v4f x0 = *reinterpret_cast<const v4f*>(xa + b);
                const v4f x1 = *reinterpret_cast<const v4f*>(xa + b + 4);
#pragma unroll
                for (int t = 0; t < 4; ++t) { x[t] = x0[t]; x[t + 4] = x1[t]; }
#pragma unroll
                for (int u = 0; u < CQ; ++u) {
                    const v4f o0 = *reinterpret_cast<const v4f*>(oa[u] + b);
                    const v4f o1 = *reinterpret_cast<const v4f*>(oa[u] + b + 4);
#pragma unroll
                    for (int t = 0; t < 4; ++t) { o[t][u] = o0[t]; o[t + 4][u] = o1[t]; }
                }
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int u = 0; u < CQ; ++u)
                        if (cq + 4 * u < kg) acc[u] = __builtin_fmaf(x[t], o[t][u], acc[u]);
            }
            for (; j < sw; j += 4) step(j);
        }
        lds_barrier_c();
    }

    if (chain && wave > 0 && i < m) {
#pragma unroll
        for (int u = 0; u < CQ; ++u) hand[wave - 1][i][cq + 4 * u] = acc[u];
    }
    lds_barrier_c();
    if (wave != 0 || i >= m) return;
    const int64_t row = i;
#pragma unroll
    for (int u = 0; u < CQ; ++u) {
        const int c = cq + 4 * u;
        if (c >= kg) continue;
        float v = acc[u];
#pragma unroll
        for (int q = 0; q < 3; ++q) v += hand[q][i][c];
        const int64_t col = c_base + c;
        if (a.S == 1) {
            const int64_t off = a.y_trans ? col * a.ldy + row : row * a.ldy + col;
            double y = (double)v;
            if (a.y_f64) {
                double* Yp = static_cast<double*>(a.Y) + off;
                if (a.beta) y += *Yp;
                *Yp = y;
            } else {
                float* Yp = static_cast<float*>(a.Y) + off;
                if (a.beta) y += (double)*Yp;
                *Yp = (float)y;
            }
        } else {
            a.partials[((int64_t)strip * a.m + row) * a.k + col] = v;
        }
    }
}

template <int K>
hipError_t launch_cm_k(const CmArgs& a, hipStream_t s) {
    if (a.m <= kSkinnyRows) {
        const dim3 grid((unsigned)(a.S * ((a.k + kColGroup - 1) / kColGroup)));
        if constexpr (K <= 8) {
            if (a.m <= 8) {
                hipLaunchKernelGGL((k_gemm_cm_skinny<K, cm_strip_width(K), 8>), grid, dim3(kSkinnyThreads),
                                   0, s, a);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_gemm_cm_skinny<K, cm_strip_width(K), kSkinnyRows>), grid,
                           dim3(kSkinnyThreads), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_gemm_cm<K>), dim3((unsigned)(8 * a.tiles8)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// Matrix-core kernel for k > 16 (sk_mfma.hip): one pass over A, strips of
// kMfmaStrip columns.
hipError_t launch_gemm_cm_mfma(const CmLaunch& g);

int64_t cm_strips(int64_t n, int64_t k) {
    const int64_t C = k > kColGroup ? kMfmaStrip
                                    : cm_strip_width(k_class((int)std::min<int64_t>(k, kColGroup)));
    return (n + C - 1) / C;
}

hipError_t launch_gemm_cm(const CmLaunch& g) {
    if (g.k > kColGroup) return launch_gemm_cm_mfma(g);
    const int kc = k_class((int)std::min<int64_t>(g.k, kColGroup));
    const int64_t S = cm_strips(g.n, g.k);
    const int64_t ncg = (g.k + kColGroup - 1) / kColGroup;
    CmArgs a{};
    a.A = g.A;
    a.m = g.m;
    a.n = g.n;
    a.lda = g.lda;
    a.row0 = g.row0;
    a.key0 = (uint32_t)g.seed;
    a.key1 = (uint32_t)(g.seed >> 32);
    a.col0 = g.col0;
    a.dist = g.dist;
    a.k = g.k;
    a.Y = g.Y;
    a.ldy = g.ldy;
    a.y_trans = g.y_trans;
    a.y_f64 = g.y_f64;
    a.beta = g.beta;
    a.partials = S > 1 ? static_cast<float*>(g.workspace) : nullptr;
    a.S = (int)S;
    a.num_rb = (int)((g.m + kCmRows - 1) / kCmRows);
    a.tiles = S * a.num_rb * ncg;
    a.tiles8 = (a.tiles + 7) / 8;
    hipError_t e;
    switch (kc) {
    case 1: e = launch_cm_k<1>(a, g.stream); break;
    case 2: e = launch_cm_k<2>(a, g.stream); break;
    case 3: e = launch_cm_k<3>(a, g.stream); break;
    case 4: e = launch_cm_k<4>(a, g.stream); break;
    case 5: e = launch_cm_k<5>(a, g.stream); break;
    case 6: e = launch_cm_k<6>(a, g.stream); break;
    case 8: e = launch_cm_k<8>(a, g.stream); break;
    case 12: e = launch_cm_k<12>(a, g.stream); break;
    default: e = launch_cm_k<16>(a, g.stream); break;
    }
    if (e != hipSuccess || S == 1) return e;
    return launch_reduce_partials_t(a.partials, (int)S, g.m, g.k, g.Y, g.y_f64, g.ldy, g.beta,
                                    g.y_trans, g.stream);
}

}  // namespace sk
