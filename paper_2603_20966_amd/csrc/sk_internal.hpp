// Host-side interfaces between the C ABI layer and the kernel translation
// units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sk {

constexpr int kMaxBlocks = 64;     // contraction blocks per reduce call
constexpr int kColGroup = 16;      // Omega columns handled by one workgroup
constexpr int kStreamWaves = 8;                  // waves per workgroup of the streaming kernel
constexpr int kWgThreads = 64 * kStreamWaves;    // its threads
constexpr int kRowQuantum = 8 * kStreamWaves;    // rows per workgroup pass (8 rows per wave)

// Register-tile class (template K of the streaming kernel) for a group of
// kg Omega columns.
constexpr int k_class(int kg) { return kg <= 6 ? kg : kg <= 8 ? 8 : kg <= 12 ? 12 : 16; }

// Strip width (columns of A per FP32 partial sum) of the streaming kernel:
// 4096 columns for FP32 and BF16 A at every k <= 16.  A function of the
// storage type only, so results never depend on m or on the launch shape.
// The partial sums' HBM writes slow the read stream far beyond their share of
// the bytes (scattered writes in the middle of a read stream): 1024-column
// strips cost about 10% of the A stream at k = 5, so the strips are as wide
// as the 4096-column blocks of a contraction split of 32768 columns over 8
// processes, whose bitwise agreement with the row layout needs the block
// width to be a multiple of the strip width.
constexpr int strip_width(int /*kclass*/, int /*adtype*/) { return 4096; }

// A strip is streamed as chunks of 1024 columns: each chunk's Omega slice
// (kclass x chunk floats) sits in one half of a double-buffered LDS ring, the
// next chunk's slice being generated while the current one is multiplied.
// The 64-lane sums close each chunk; a strip's FP32 partial is the sum of its
// chunk sums in chunk order.  A function of the tile class only.
constexpr int chunk_width(int /*kclass*/) { return 1024; }

// Most rows one streaming tile covers (the per-pass strip sums of a wave live
// in LDS: 16 passes of 8 rows per wave).
constexpr int stream_max_rows(int /*kclass*/) { return 16 * 8 * kStreamWaves; }

// The matrix-core kernel takes FP32 A from k = 9 on: past 8 sketch columns
// the non-packed FP32 FMAs of the streaming kernel (4k per 16 bytes of A)
// approach the vector ALU's rate at HBM speed, and its registers no longer
// hold 8 rows of k accumulators.  Its strips are 2048 columns.
constexpr int kMfmaStrip = 2048;
constexpr int kMfmaRows = 512;     // rows of a matrix-core tile
constexpr int kStreamMaxK = 8;     // widest sketch of the streaming kernel (FP32 A)
constexpr int kStreamMaxKBf16 = 6; // ... for BF16 A (its unpacked elements take 32 more registers)
constexpr int kMfmaMinK = kStreamMaxK + 1;
constexpr bool use_mfma(int adtype, int64_t k) { return adtype == 0 && k >= kMfmaMinK; }

// Low-precision A on the BF16 matrix cores: FP8 at every k (on the VALU path
// its conversions and 5 FMAs per byte cap k = 5 at 2.6 TB/s, against 3.2 TB/s
// here), BF16 from k = 7 on, where the streaming kernel's registers no longer
// hold 8 rows of unpacked BF16 and k accumulators (at k = 5 both paths
// measured the same speed, and the VALU path sums with FP32 Omega: 1e-7
// against 2.5e-6 relative arithmetic error).  Strips of 4096 columns.
constexpr int kLpStrip = 4096;
constexpr int kLpBatchWaves = 8;                  // waves per tile in batched launches
constexpr int kLpBatchRows = 64 * kLpBatchWaves;  // rows per tile in batched launches
constexpr bool use_mfma_lp(int adtype, int64_t k) {
    return adtype == 2 || (adtype == 1 && k > kStreamMaxKBf16);
}

// Strip width used for a sketch of width k with A stored as adtype.
constexpr int64_t strip_width_for(int adtype, int64_t k) {
    return use_mfma(adtype, k)      ? kMfmaStrip
           : use_mfma_lp(adtype, k) ? kLpStrip
                                    : strip_width(k_class((int)(k < kStreamMaxK ? k : kStreamMaxK)), adtype);
}

struct BlockDesc {
    const void* A;        // device pointer to the block's first element
    int64_t n;            // columns of the block
    int64_t lda;          // leading dimension (elements)
    int64_t row0;         // global Omega row of the block's column 0
    const float* scales;  // per-128-row scales or nullptr
};

struct TraceEvents {
    hipEvent_t begin = nullptr, mid = nullptr, end = nullptr;
};

struct GemmLaunch {
    int adtype;               // 0 f32, 1 bf16, 2 fp8
    int64_t m;
    int P;
    BlockDesc blk[kMaxBlocks];
    int64_t k;
    uint32_t col0;
    uint64_t seed;
    int dist;                 // Omega's distribution: 0 normal, 1 uniform, 2 Rademacher
    const float* omega;       // explicit Omega (n x k) or nullptr to generate
    int64_t ldo;
    void* Y;
    int y_f64;
    int64_t ldy;
    int beta;
    void* workspace;
    size_t workspace_bytes;
    hipStream_t stream;
    TraceEvents trace;
};

// One request of a serving batch: one A block with its own output.  Tiles of
// request q are [tile_begin, tile_begin + strips*rowblocks*colgroups); its
// outputs (for the batched strip sum) are [out_begin, out_begin + m*k).
constexpr int kMaxBatch = 16;
struct BatchReq {
    const void* A;
    int64_t n, lda, row0;
    const float* scales;
    int64_t m, k;
    void* Y;
    int64_t ldy;
    float* partials;        // [strips][m][k] (unused when strips == 1)
    uint64_t seed;
    uint32_t col0;
    int32_t dist;
    int32_t y_f64, beta;
    int32_t rows_per_wg, strips, rowblocks;
    int64_t tile_begin, out_begin;
};
struct BatchArgs {
    int count;
    int64_t total_tiles;
    int64_t total_outputs;   // outputs of requests with more than one strip
    BatchReq req[kMaxBatch];
};

// Number of FP32 strip partials of a launch.
int64_t count_strips(const GemmLaunch& g);
size_t gemm_workspace_bytes(int64_t m, int64_t strips, int64_t k);
// Workspace of a product call over `strips` strips: the strip partials, and on
// the low-precision matrix-core route the call's packed Omega after them.
size_t product_workspace_bytes(int adtype, int64_t m, int64_t strips, int64_t k);
// Workspace of a column-major product call (m rows, n contraction columns).
size_t cm_workspace_bytes(int64_t m, int64_t n, int64_t k);

// Column-major A (element (i, j) at A + j*lda + i), FP32, generated Omega; Y
// row-major or transposed (element (i, c) at Y + c*ldy + i).  Strips of
// cm_strip_width(kclass) columns (1024 at every k <= 16: with 512 at k = 9 ..
// 16 the doubled partial sums cost 8-10% on 32768^2); partials [S][m][k] as
// for the other kernels.
constexpr int cm_strip_width(int) { return 1024; }
struct CmLaunch {
    const float* A;
    int64_t m, n, lda, row0;
    uint64_t seed;
    int dist;
    uint32_t col0;
    int64_t k;
    void* Y;
    int64_t ldy;
    int y_trans, y_f64, beta;
    void* workspace;
    hipStream_t stream;
};
int64_t cm_strips(int64_t n, int64_t k);
hipError_t launch_gemm_cm(const CmLaunch& g);

hipError_t launch_gemm_stream(const GemmLaunch& g);
// Streaming-kernel batch: all requests share the tile class (kclass, adtype);
// followed by the batched FP64 strip sums.  grid <= 0: one resident round of
// workgroups (occupancy x compute units), at most one per tile.
hipError_t launch_gemm_batch(const BatchArgs& a, int kclass, int adtype, int grid, hipStream_t s);
hipError_t launch_reduce_batch(const BatchArgs& a, hipStream_t s);
hipError_t launch_gemm_mfma(const GemmLaunch& g);
// Matrix-core batch (FP32 A, generated Omega): every request has the same N-tile
// count nt; BatchReq.rowblocks counts kMfmaRows-row tiles, strips kMfmaStrip columns.
hipError_t launch_gemm_mfma_batch(const BatchArgs& a, int nt, int grid, hipStream_t s);
int mfma_ntiles(int64_t k);
// Low-precision A (BF16 / FP8) on the BF16 matrix cores; batches use
// kLpBatchRows-row tiles and kLpStrip-column strips.
hipError_t launch_gemm_mfma_lp(const GemmLaunch& g);
hipError_t launch_gemm_mfma_lp_batch(const BatchArgs& a, int nt, int adtype, int grid,
                                     hipStream_t s);
int lp_ntiles(int64_t k);
// Persistent grid for total_tiles tiles of a kernel holding per_cu workgroups
// per compute unit (grid > 0: that size, capped at the tile count); a
// multiple of 8.
int batch_grid(int per_cu, int64_t total_tiles, int grid);
// Compute units of the current device; rows per streaming tile for m rows,
// `strips` strips and ncg column groups.
int device_cus();
int64_t rows_per_tile(int64_t m, int64_t strips, int64_t ncg, int64_t max_rows);
// A[i][j] ~ N(0,1) for a synthetic request: Philox4x32-10 on counters
// (j/4, i, 0, 1) (the last word keeps the stream apart from Omega's, whose
// last word is 0), Box-Muller with the hardware transcendentals.
hipError_t launch_fill_normal(float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                              hipStream_t s);
hipError_t launch_reduce_partials(const float* partials, int S, int64_t m, int64_t k, void* Y,
                                  int y_f64, int64_t ldy, int beta, hipStream_t s);
// The same with Y transposed when y_trans (element (i, c) at Y + c*ldy + i).
hipError_t launch_reduce_partials_t(const float* partials, int S, int64_t m, int64_t k, void* Y,
                                    int y_f64, int64_t ldy, int beta, int y_trans, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_zero_matrix(void* Y, int f64, int64_t m, int64_t k, int64_t ldy, hipStream_t s);
hipError_t launch_philox_raw(const uint32_t* ctr, uint64_t seed, uint32_t* out, int64_t N,
                             hipStream_t s);
// out[2i], out[2i+1] = the generator's FP32 Box-Muller pair of words[2i], words[2i+1].
hipError_t launch_normal_raw(const uint32_t* words, float* out, int64_t N, hipStream_t s);
hipError_t launch_gen_omega(uint64_t seed, int dist, int64_t row0, int64_t n, int64_t col0,
                            int64_t k, float* Om, int64_t ldo, hipStream_t s);
hipError_t launch_quantize(const float* A, int64_t m, int64_t n, int64_t lda, int dst, void* Aq,
                           int64_t ldq, float* scales, hipStream_t s);

// Nystrom core and reconstruction (FP64, sk_nystrom.hip).
constexpr int64_t kPinvMaxR = 1024;
size_t pinv_workspace_bytes(int64_t r);
hipError_t launch_core_pinv(const void* C, int c_f64, int64_t r, int64_t ldc, double tol,
                            int max_sweeps, double* Cp, int64_t ldcp, double* eig, int32_t* info,
                            void* ws, hipStream_t s);
size_t nystrom_workspace_bytes(int64_t n, int64_t r);
hipError_t launch_nystrom(const float* A, int64_t lda, const float* B, int64_t n, int64_t r,
                          int64_t ldb, const double* Cp, int64_t ldcp, int64_t row0, int64_t mr,
                          double* out, int64_t ldo, double* sums, void* ws, hipStream_t s);

// The C ABI's sketch_gen_matmul path, shared by the entry points that bring
// their own workspace and by the one that uses the library's static scratch.
// gen_matmul_validate makes no HIP call; *need receives the workspace bytes.
int gen_matmul_validate(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                        const float* a_scales, int dist, int64_t omega_row0, int64_t omega_col0,
                        const float* Omega, int64_t ldo, int64_t k, const void* Y, int y_dtype,
                        int64_t ldy, int beta, size_t* need);
int gen_matmul_impl(const void* A, int a_dtype, int64_t m, int64_t n, int64_t lda,
                    const float* a_scales, uint64_t seed, int dist, int64_t omega_row0,
                    int64_t omega_col0, const float* Omega, int64_t ldo, int64_t k, void* Y,
                    int y_dtype, int64_t ldy, int beta, void* workspace, size_t workspace_bytes,
                    void* stream);
// Consumes the events armed by sketch_trace_events for this thread.
void drop_trace();

}  // namespace sk
