// Streaming kernel for Y = A * Omega(seed) on gfx950 (small sketch width).
//
// The local product of Alg. 1 (GenRandom + local multiplication) and, for a
// contraction split, the sum of the partial products (the Reduce-Scatter of
// Alg. 1, done on the device), in one launch.
//
// Work decomposition (one workgroup = one tile):
//   * a strip of C consecutive columns of one A block (C = strip_width(kg))
//     times a range of R rows, for a group of kg <= 16 Omega columns;
//   * the workgroup first builds its C x kg slice of Omega in LDS (generated
//     from the seed, or copied from an explicit Omega for the stored-operand
//     variant), so Omega never exists in HBM on the generated path;
//   * each wave then streams passes of 8 rows (32 rows apart between the
//     four waves): all 64 lanes read one row segment per step, 16 contiguous
//     bytes per lane (1 KB per load instruction), and multiply them by the
//     matching Omega values from LDS with FP32 FMAs into per-lane
//     accumulators (8 rows x kg columns per lane);
//   * the first loads of A are issued before the Omega slice is generated,
//     and each wave keeps two steps of nontemporal loads in flight across
//     its passes;
//   * at the end of a pass the 64 lanes' accumulators are summed by a fixed
//     reduce-scatter (permlane32 and permlane16 swaps, then a DPP butterfly
//     inside 16-lane rows), giving the FP32 partial of (row, strip, column);
//     partials go to the workspace;
//   * a second small kernel sums the partials of all strips in FP64, in strip
//     order, adds beta * Y, rounds once and writes Y.  (No cross-workgroup
//     synchronisation inside the streaming kernel: device-scope release /
//     acquire would write back and invalidate the L2 of an XCD under every
//     streaming wave.)
// The summation order depends only on the strip boundaries, never on m, R or
// the grid, so results are bitwise reproducible and layout independent.
#include "sk_device.hpp"
#include "sk_internal.hpp"

#pragma clang fp contract(off)

namespace sk {
namespace {

constexpr int kLanesPerRow = 64;  // a whole wave reads one row segment (1 KB per instruction)
constexpr int kRowGroups = 8;     // rows per wave pass
constexpr int kDepth = 2;         // steps of A loads in flight per wave

typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

// 16-byte load of A marked nontemporal: A is streamed once, so it should not
// displace other lines (measured: +10% streaming bandwidth on gfx950).
__device__ __forceinline__ uint4 load_a16(const unsigned char* p) {
    const v4u32 v = __builtin_nontemporal_load(reinterpret_cast<const v4u32*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

struct KArgs {
    int64_t m;
    int64_t k;
    int64_t ldy;
    int64_t ldo;
    const float* omega;
    void* Y;
    float* partials;
    uint32_t key0, key1;
    uint32_t col0;
    int dist;
    int P;
    int S_total;
    int rows_per_wg;
    int num_rb;
    int64_t tiles;    // strips x row blocks x column groups
    int64_t tiles8;   // ceil(tiles / 8)
    int y_f64;
    int beta;
    BlockDesc blk[kMaxBlocks];
};

template <int ADT>
struct Elem;
template <>
struct Elem<0> {
    static constexpr int size = 4;
};
template <>
struct Elem<1> {
    static constexpr int size = 2;
};
template <>
struct Elem<2> {
    static constexpr int size = 1;
};

// 16 raw bytes of A -> EPL floats.
template <int ADT>
__device__ __forceinline__ void unpack16(const uint4 raw, float* out) {
    if constexpr (ADT == 0) {
        out[0] = __uint_as_float(raw.x);
        out[1] = __uint_as_float(raw.y);
        out[2] = __uint_as_float(raw.z);
        out[3] = __uint_as_float(raw.w);
    } else if constexpr (ADT == 1) {
        const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            out[2 * i] = __uint_as_float(w[i] << 16);
            out[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
        }
    } else {
        const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
            out[4 * i + 0] = lo[0];
            out[4 * i + 1] = lo[1];
            out[4 * i + 2] = hi[0];
            out[4 * i + 3] = hi[1];
        }
    }
}

// Load up to 16 bytes at p of which only `nvalid` elements exist; the rest
// read as zero.  Used for the ragged last step of a strip.
template <int ADT>
__device__ __forceinline__ uint4 load_tail(const unsigned char* p, int nvalid) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    constexpr int es = Elem<ADT>::size;
    for (int e = 0; e < 16 / es; ++e) {
        if (e < nvalid) {
            uint32_t v;
            if constexpr (es == 4) v = *reinterpret_cast<const uint32_t*>(p + 4 * e);
            else if constexpr (es == 2) v = *reinterpret_cast<const uint16_t*>(p + 2 * e);
            else v = p[e];
            const int byte = e * es;
            w[byte >> 2] |= v << (8 * (byte & 3));
        }
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Sum over the 16 lanes of a DPP row with a fixed butterfly; every lane of
// the row receives the same bits.
__device__ __forceinline__ float row16_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
    return v;
}

// Workgroup barrier ordering LDS only: outstanding global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Everything one workgroup needs for one tile (strip x row range x column
// group) of one A block and its output.
struct Tile {
    const unsigned char* A;   // first element of the A block
    int64_t lda;              // elements
    int64_t n;                // columns of the block
    int64_t row0;             // global Omega row of the block's column 0
    const float* scales;      // per-128-row scales or nullptr
    int64_t m, k;             // rows of A and Y, sketch width
    int64_t col_begin;        // first block column of the strip
    int64_t row_begin, row_end;
    int c_base, kg;           // sketch columns [c_base, c_base + kg)
    uint32_t key0, key1, col0;
    int dist;                 // Omega's distribution (0 normal, 1 uniform, 2 Rademacher)
    const float* omega;       // stored operand (n x k, ldo) when not generated
    int64_t ldo;
    void* Y;
    int64_t ldy;
    int y_f64, beta;
    float* partials;          // [S][m][k] of the output, or nullptr
    int64_t strip_index;      // row of this strip in the partial array
    bool single;              // the output has one strip: write Y directly
};

// One tile: issue the first A loads, build the Omega slice in LDS, stream the
// rows, write the strip partials (or Y).  All threads of the workgroup call it.
template <int K, int ADT, bool GEN>
__device__ __forceinline__ void tile_body(const Tile& tl, float (*om)[strip_width(K, ADT)]) {
    constexpr int es = Elem<ADT>::size;
    constexpr int EPL = 16 / es;                 // elements per lane step
    constexpr int C = strip_width(K, ADT);       // columns per strip
    constexpr int STEP = kLanesPerRow * EPL;     // columns per wave step
    constexpr int T = C / STEP;                  // steps per full strip
    static_assert(C % STEP == 0, "strip must hold whole steps");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int kg = tl.kg;
    const int c_base = tl.c_base;
    const int64_t col_begin = tl.col_begin;
    const int w = (int)min<int64_t>(C, tl.n - col_begin);
    const int64_t row_end = tl.row_end;

    // ---- this wave's rows: passes of 8 rows, 32 rows apart ------------------
    const int64_t lda_bytes = tl.lda * es;
    const bool full = (w == C);
    const int Tr = full ? T : (w + STEP - 1) / STEP;    // steps per pass
    const int64_t first_pb = tl.row_begin + wave * kRowGroups;
    const int npass = first_pb < row_end ? (int)((row_end - first_pb + kRowQuantum - 1) / kRowQuantum) : 0;
    const unsigned char* lane_col = tl.A + (col_begin + lane * EPL) * es;

    // Steps run pass by pass (8 rows), column step by column step; loads are
    // issued kDepth steps ahead of the FMAs that consume them.
    int ip = 0, it_ = 0;   // next step to load: pass, column step
    int cp = 0, ct = 0;    // next step to consume
    auto issue = [&](uint4* buf) {
        if (ip >= npass) return;
        const int p = ip;
        const int t = it_;
        if (++it_ == Tr) {
            it_ = 0;
            ++ip;
        }
        const int64_t pb = first_pb + (int64_t)p * kRowQuantum;
        const int cl = t * STEP + lane * EPL;
#pragma unroll
        for (int i = 0; i < kRowGroups; ++i) {
            const int64_t r = min<int64_t>(pb + i, tl.m - 1);
            const unsigned char* ptr = lane_col + r * lda_bytes + (int64_t)t * STEP * es;
            if (full || w - cl >= EPL) buf[i] = load_a16(ptr);
            else buf[i] = load_tail<ADT>(ptr, w - cl);
        }
    };

    uint4 bufs[kDepth][kRowGroups];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) issue(bufs[d]);

    // ---- Omega slice for this strip -> LDS (overlaps the first loads) --------
    if constexpr (GEN) {
        const int64_t g0 = tl.row0 + col_begin;            // global Omega row of column 0
        const int64_t q_lo = g0 >> 2;
        const int64_t q_hi = (g0 + w - 1) >> 2;
        const int nq = (int)(q_hi - q_lo + 1);
        const int items = nq * kg;
        const bool aligned = (g0 & 3) == 0;
        for (int it = tid; it < items; it += kWgThreads) {
            const int qi = it / kg;
            const int c = it - qi * kg;
            const float4 z = omega4_dist((uint64_t)(q_lo + qi), tl.col0 + (uint32_t)(c_base + c),
                                         tl.key0, tl.key1, tl.dist);
            const int64_t p0 = 4 * (q_lo + qi) - g0;       // local column of z.x
            if (aligned && p0 + 3 < w) {
                *reinterpret_cast<float4*>(&om[c][p0]) = z;
            } else {
                const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int64_t p = p0 + t;
                    if (p >= 0 && p < w) om[c][p] = zz[t];
                }
            }
        }
    } else {
        for (int it = tid; it < w * kg; it += kWgThreads) {
            const int jl = it / kg;
            const int c = it - jl * kg;
            om[c][jl] = tl.omega[(col_begin + jl) * tl.ldo + c_base + c];
        }
    }
    // zero the unused part of the slice (ragged strip, unused columns)
    for (int it = tid; it < K * C; it += kWgThreads) {
        const int c = it / C;
        const int jl = it - c * C;
        if (c >= kg || jl >= w) om[c][jl] = 0.0f;
    }
    lds_barrier();

    // ---- stream: FMA each step, 64-lane sums at the end of each pass ---------
    float acc[kRowGroups][K];
#pragma unroll
    for (int i = 0; i < kRowGroups; ++i)
#pragma unroll
        for (int c = 0; c < K; ++c) acc[i][c] = 0.0f;

    auto consume = [&](const uint4* raw) {
        const int p = cp;
        const int t = ct;
        if (++ct == Tr) {
            ct = 0;
            ++cp;
        }
        float a[kRowGroups][EPL];
#pragma unroll
        for (int i = 0; i < kRowGroups; ++i) unpack16<ADT>(raw[i], a[i]);
        const int cl = t * STEP + lane * EPL;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            float wv[EPL];
#pragma unroll
            for (int v = 0; v < EPL / 4; ++v) {
                const float4 q = *reinterpret_cast<const float4*>(&om[c][cl + 4 * v]);
                wv[4 * v + 0] = q.x;
                wv[4 * v + 1] = q.y;
                wv[4 * v + 2] = q.z;
                wv[4 * v + 3] = q.w;
            }
#pragma unroll
            for (int i = 0; i < kRowGroups; ++i)
#pragma unroll
                for (int e = 0; e < EPL; ++e) acc[i][c] = __builtin_fmaf(a[i][e], wv[e], acc[i][c]);
        }
        if (t != Tr - 1) return;
        // End of pass: sum each of the V = 8K accumulators over the 64 lanes as a
        // reduce-scatter.  permlane32_swap exchanges rows {2,3} of one register
        // with rows {0,1} of another, so one swap + add halves the values per
        // lane (lanes 0-31 keep the first half, lanes 32-63 the second);
        // permlane16_swap does the same between rows 0|1 and 2|3; a 4-stage DPP
        // butterfly finishes each value inside its 16-lane row.  Row r then
        // holds values [r*V/4, (r+1)*V/4); every addition order is fixed.
        const int64_t pb = first_pb + (int64_t)p * kRowQuantum;
        constexpr int V = kRowGroups * K;
        constexpr int H = V / 2;
        constexpr int Q = V / 4;
        float hv[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int i0 = j / K, c0 = j % K, i1 = (j + H) / K, c1 = (j + H) % K;
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[i0][c0]),
                                                             __float_as_uint(acc[i1][c1]), false, false);
            hv[j] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
        }
        float qv[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(hv[j]),
                                                             __float_as_uint(hv[j + Q]), false, false);
            qv[j] = row16_sum(__uint_as_float(sw[0]) + __uint_as_float(sw[1]));
        }
        const int row16 = lane >> 4;
        const int vbase = (row16 >> 1) * H + (row16 & 1) * Q;
        const int sig = lane & 15;
#pragma unroll
        for (int base = 0; base < Q; base += 16) {
            float mine = 0.0f;
#pragma unroll
            for (int j = base; j < base + 16 && j < Q; ++j)
                if (sig == j - base) mine = qv[j];
            const int v = vbase + base + sig;        // accumulator index i*K + c
            const int wi = v / K;
            const int wc = v - wi * K;
            const int64_t r = pb + wi;
            if (base + sig < Q && r < row_end && wc < kg) {
                if (tl.scales) mine *= tl.scales[r >> 7];
                if (tl.single) {
                    double y = (double)mine;
                    if (tl.y_f64) {
                        double* Yp = static_cast<double*>(tl.Y) + r * tl.ldy + c_base + wc;
                        if (tl.beta) y += *Yp;
                        *Yp = y;
                    } else {
                        float* Yp = static_cast<float*>(tl.Y) + r * tl.ldy + c_base + wc;
                        if (tl.beta) y += (double)*Yp;
                        *Yp = (float)y;
                    }
                } else {
                    tl.partials[(tl.strip_index * tl.m + r) * tl.k + c_base + wc] = mine;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kRowGroups; ++i)
#pragma unroll
            for (int c = 0; c < K; ++c) acc[i][c] = 0.0f;
    };

    while (cp < npass) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d) {
            if (cp < npass) {
                consume(bufs[d]);
                issue(bufs[d]);
            }
        }
    }
}

// One call: grid (strips of all blocks, row blocks, column groups), one tile
// per workgroup; the blocks share the output (contraction split).
// Tile of a workgroup in an XCD-grouped order: workgroups are handed to the 8
// XCDs round-robin, so XCD x receives ids x, x+8, ...; giving it the
// contiguous tile range [x*T8, (x+1)*T8) (strips fastest, then row blocks)
// makes each XCD stream whole rows of A at a time.
__device__ __forceinline__ int64_t xcd_tile(int64_t id, int64_t T8) {
    return (id % 8) * T8 + id / 8;
}

template <int K, int ADT, bool GEN>
__global__ __launch_bounds__(kWgThreads) void k_gemm_stream(const KArgs args) {
    constexpr int C = strip_width(K, ADT);
    __shared__ float om[K][C];
    const int64_t t = xcd_tile(blockIdx.x, args.tiles8);
    if (t >= args.tiles) return;
    const int strip = (int)(t % args.S_total);
    const int64_t rbt = t / args.S_total;
    const int rb = (int)(rbt % args.num_rb);
    const int cg = (int)(rbt / args.num_rb);
    int b = 0;
    int64_t strip_in_block = strip;
    for (; b < args.P; ++b) {
        const int64_t sb = (args.blk[b].n + C - 1) / C;
        if (strip_in_block < sb) break;
        strip_in_block -= sb;
    }
    const BlockDesc& blk = args.blk[b];
    Tile tl;
    tl.A = static_cast<const unsigned char*>(blk.A);
    tl.lda = blk.lda;
    tl.n = blk.n;
    tl.row0 = blk.row0;
    tl.scales = blk.scales;
    tl.m = args.m;
    tl.k = args.k;
    tl.col_begin = strip_in_block * C;
    tl.row_begin = (int64_t)rb * args.rows_per_wg;
    tl.row_end = min<int64_t>(tl.row_begin + args.rows_per_wg, args.m);
    tl.c_base = cg * kColGroup;
    tl.kg = (int)min<int64_t>(kColGroup, args.k - tl.c_base);
    tl.key0 = args.key0;
    tl.key1 = args.key1;
    tl.col0 = args.col0;
    tl.dist = args.dist;
    tl.omega = args.omega;
    tl.ldo = args.ldo;
    tl.Y = args.Y;
    tl.ldy = args.ldy;
    tl.y_f64 = args.y_f64;
    tl.beta = args.beta;
    tl.partials = args.partials;
    tl.strip_index = strip;
    tl.single = (args.S_total == 1);
    tile_body<K, ADT, GEN>(tl, om);
}

// A batch of independent requests (serving): the same tiles as one call per
// request, walked by a fixed grid; each request keeps its own seed, offsets,
// output and partial array, so its result does not depend on the batch.
template <int K, int ADT>
__global__ __launch_bounds__(kWgThreads) void k_gemm_batch(const BatchArgs args) {
    constexpr int C = strip_width(K, ADT);
    __shared__ float om[K][C];
    bool first = true;
    const int64_t T8 = (args.total_tiles + 7) / 8;
    for (int64_t v = blockIdx.x; v < 8 * T8; v += gridDim.x) {   // gridDim.x is a multiple of 8
        const int64_t t = xcd_tile(v, T8);
        if (t >= args.total_tiles) continue;
        int q = 0;
        while (q + 1 < args.count && t >= args.req[q + 1].tile_begin) ++q;
        const BatchReq& rq = args.req[q];
        const int64_t lt = t - rq.tile_begin;
        const int64_t strip = lt % rq.strips;
        const int64_t rb = (lt / rq.strips) % rq.rowblocks;
        const int cg = (int)(lt / ((int64_t)rq.strips * rq.rowblocks));
        Tile tl;
        tl.A = static_cast<const unsigned char*>(rq.A);
        tl.lda = rq.lda;
        tl.n = rq.n;
        tl.row0 = rq.row0;
        tl.scales = rq.scales;
        tl.m = rq.m;
        tl.k = rq.k;
        tl.col_begin = strip * C;
        tl.row_begin = rb * rq.rows_per_wg;
        tl.row_end = min<int64_t>(tl.row_begin + rq.rows_per_wg, rq.m);
        tl.c_base = cg * kColGroup;
        tl.kg = (int)min<int64_t>(kColGroup, rq.k - tl.c_base);
        tl.key0 = (uint32_t)rq.seed;
        tl.key1 = (uint32_t)(rq.seed >> 32);
        tl.col0 = rq.col0;
        tl.dist = rq.dist;
        tl.omega = nullptr;
        tl.ldo = 0;
        tl.Y = rq.Y;
        tl.ldy = rq.ldy;
        tl.y_f64 = rq.y_f64;
        tl.beta = rq.beta;
        tl.partials = rq.partials;
        tl.strip_index = strip;
        tl.single = (rq.strips == 1);
        if (!first) lds_barrier();   // every wave is done with the previous slice
        first = false;
        tile_body<K, ADT, true>(tl, om);
    }
}

// Y (=|+=) sum over strips of the FP32 partials, in FP64, strip order fixed;
// one thread per output element, loads issued 32 at a time.
__global__ void k_reduce_partials(const float* __restrict__ partials, int S, int64_t m, int64_t k,
                                  void* Y, int y_f64, int64_t ldy, int beta, int y_trans) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= m * k) return;
    const int64_t r = o / k;
    const int64_t c = o - r * k;
    const float* p = partials + o;
    const int64_t sstride = m * k;
    double y = 0.0;
    int s = 0;
    for (; s + 32 <= S; s += 32) {
        float v[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = __builtin_nontemporal_load(p + (int64_t)(s + j) * sstride);
#pragma unroll
        for (int j = 0; j < 32; ++j) y += (double)v[j];
    }
    for (; s < S; ++s) y += (double)p[(int64_t)s * sstride];
    const int64_t off = y_trans ? c * ldy + r : r * ldy + c;
    if (y_f64) {
        double* Yp = static_cast<double*>(Y) + off;
        if (beta) y += *Yp;
        *Yp = y;
    } else {
        float* Yp = static_cast<float*>(Y) + off;
        if (beta) y += (double)*Yp;
        *Yp = (float)y;
    }
}

// Batched FP64 strip sums: one thread per output element of every request
// with more than one strip, in strip order.
__global__ void k_reduce_batch(const BatchArgs args) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= args.total_outputs) return;
    int q = 0;
    while (q + 1 < args.count && o >= args.req[q + 1].out_begin) ++q;
    const BatchReq& rq = args.req[q];
    if (rq.strips == 1) return;
    const int64_t lo = o - rq.out_begin;
    const int64_t r = lo / rq.k;
    const int64_t c = lo - r * rq.k;
    const float* p = rq.partials + lo;
    const int64_t sstride = rq.m * rq.k;
    double y = 0.0;
    int s = 0;
    for (; s + 16 <= rq.strips; s += 16) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = __builtin_nontemporal_load(p + (int64_t)(s + j) * sstride);
#pragma unroll
        for (int j = 0; j < 16; ++j) y += (double)v[j];
    }
    for (; s < rq.strips; ++s) y += (double)p[(int64_t)s * sstride];
    if (rq.y_f64) {
        double* Yp = static_cast<double*>(rq.Y) + r * rq.ldy + c;
        if (rq.beta) y += *Yp;
        *Yp = y;
    } else {
        float* Yp = static_cast<float*>(rq.Y) + r * rq.ldy + c;
        if (rq.beta) y += (double)*Yp;
        *Yp = (float)y;
    }
}

template <int K, int ADT, bool GEN>
hipError_t launch_k(const KArgs& a, dim3 grid, hipStream_t s, const TraceEvents& tr) {
    if (tr.begin) (void)hipEventRecord(tr.begin, s);
    hipLaunchKernelGGL((k_gemm_stream<K, ADT, GEN>), grid, dim3(kWgThreads), 0, s, a);
    if (tr.mid) (void)hipEventRecord(tr.mid, s);
    if (a.S_total > 1)
        (void)launch_reduce_partials(a.partials, a.S_total, a.m, a.k, a.Y, a.y_f64, a.ldy, a.beta,
                                     s);
    if (tr.end) (void)hipEventRecord(tr.end, s);
    return hipGetLastError();
}

template <int ADT, bool GEN>
hipError_t dispatch_k(int kc, const KArgs& a, dim3 grid, hipStream_t s, const TraceEvents& tr) {
    switch (kc) {
    case 1: return launch_k<1, ADT, GEN>(a, grid, s, tr);
    case 2: return launch_k<2, ADT, GEN>(a, grid, s, tr);
    case 3: return launch_k<3, ADT, GEN>(a, grid, s, tr);
    case 4: return launch_k<4, ADT, GEN>(a, grid, s, tr);
    case 5: return launch_k<5, ADT, GEN>(a, grid, s, tr);
    case 6: return launch_k<6, ADT, GEN>(a, grid, s, tr);
    case 8: return launch_k<8, ADT, GEN>(a, grid, s, tr);
    case 12: return launch_k<12, ADT, GEN>(a, grid, s, tr);
    default: return launch_k<16, ADT, GEN>(a, grid, s, tr);
    }
}

}  // namespace

// Compute units of the current device (cached per device).
int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) dev = 0;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n < 1)
            n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

// Rows per tile: a multiple of 32 giving about two tiles per compute unit,
// at most 512 rows (measured best on the 4096 x 32768 share and on the
// 32768 x 32768 column layout).  SKETCH_ROWS_PER_TILE overrides it for tuning.
int64_t rows_per_tile(int64_t m, int64_t strips, int64_t ncg) {
    static const int64_t forced = [] {
        const char* e = getenv("SKETCH_ROWS_PER_TILE");
        const long long v = e ? atoll(e) : 0;
        return (int64_t)(v > 0 ? v : 0);
    }();
    const int64_t want = 2 * (int64_t)device_cus();
    int64_t R = forced > 0 ? forced : (m * strips * ncg + want - 1) / want;
    R = (R + kRowQuantum - 1) / kRowQuantum * kRowQuantum;
    if (forced == 0) R = std::min<int64_t>(R, 512);
    return std::max<int64_t>(kRowQuantum, R);
}

int64_t count_strips(const GemmLaunch& g) {
    const int64_t C = strip_width_for(g.adtype, g.k);
    int64_t s = 0;
    for (int b = 0; b < g.P; ++b) s += (g.blk[b].n + C - 1) / C;
    return s;
}

size_t gemm_workspace_bytes(int64_t m, int64_t strips, int64_t k) {
    if (strips <= 1) return 0;
    return (size_t)strips * (size_t)m * (size_t)k * sizeof(float);
}

hipError_t launch_reduce_partials_t(const float* partials, int S, int64_t m, int64_t k, void* Y,
                                    int y_f64, int64_t ldy, int beta, int y_trans, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((m * k + 255) / 256)), dim3(256), 0, s,
                       partials, S, m, k, Y, y_f64, ldy, beta, y_trans);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* partials, int S, int64_t m, int64_t k, void* Y,
                                  int y_f64, int64_t ldy, int beta, hipStream_t s) {
    return launch_reduce_partials_t(partials, S, m, k, Y, y_f64, ldy, beta, 0, s);
}

hipError_t launch_gemm_stream(const GemmLaunch& g) {
    const int64_t ncg = (g.k + kColGroup - 1) / kColGroup;
    const int kg0 = (int)std::min<int64_t>(g.k, kColGroup);
    const int kc = k_class(kg0);
    const int64_t S = count_strips(g);
    KArgs a{};
    a.m = g.m;
    a.k = g.k;
    a.ldy = g.ldy;
    a.ldo = g.ldo;
    a.omega = g.omega;
    a.Y = g.Y;
    a.key0 = (uint32_t)g.seed;
    a.key1 = (uint32_t)(g.seed >> 32);
    a.col0 = g.col0;
    a.dist = g.dist;
    a.P = g.P;
    a.S_total = (int)S;
    a.y_f64 = g.y_f64;
    a.beta = g.beta;
    for (int b = 0; b < g.P; ++b) a.blk[b] = g.blk[b];
    const bool gen = (g.omega == nullptr);
    const int64_t R = rows_per_tile(g.m, S, ncg);
    const int64_t nrb = (g.m + R - 1) / R;
    a.rows_per_wg = (int)R;
    a.num_rb = (int)nrb;
    a.tiles = S * nrb * ncg;
    a.tiles8 = (a.tiles + 7) / 8;
    if (S > 1) a.partials = static_cast<float*>(g.workspace);
    dim3 grid((unsigned)(8 * a.tiles8));
    const TraceEvents& tr = g.trace;
    switch (g.adtype) {
    case 0: return gen ? dispatch_k<0, true>(kc, a, grid, g.stream, tr) : dispatch_k<0, false>(kc, a, grid, g.stream, tr);
    case 1: return gen ? dispatch_k<1, true>(kc, a, grid, g.stream, tr) : dispatch_k<1, false>(kc, a, grid, g.stream, tr);
    default: return gen ? dispatch_k<2, true>(kc, a, grid, g.stream, tr) : dispatch_k<2, false>(kc, a, grid, g.stream, tr);
    }
}

hipError_t launch_reduce_batch(const BatchArgs& a, hipStream_t s) {
    if (a.total_outputs > 0)
        hipLaunchKernelGGL(k_reduce_batch, dim3((unsigned)((a.total_outputs + 255) / 256)),
                           dim3(256), 0, s, a);
    return hipGetLastError();
}

namespace {

// Persistent grid of a batch: the workgroups one resident round holds
// (occupancy x compute units), at most one per tile, a multiple of 8 so that
// every workgroup stays on one XCD's tile range.
int resident_grid(int per_cu, int64_t total_tiles, int grid) {
    if (grid <= 0) grid = std::max(1, per_cu) * device_cus();
    const int64_t cap = (total_tiles + 7) / 8 * 8;
    grid = (int)std::min<int64_t>(grid, cap);
    return std::max(8, (grid + 7) / 8 * 8);
}

template <int K, int ADT>
hipError_t run_batch(const BatchArgs& a, int grid, hipStream_t s) {
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_batch<K, ADT>, kWgThreads, 0) !=
            hipSuccess)
            n = 1;
        return n;
    }();
    grid = resident_grid(per_cu, a.total_tiles, grid);
    hipLaunchKernelGGL((k_gemm_batch<K, ADT>), dim3((unsigned)grid), dim3(kWgThreads), 0, s, a);
    return hipGetLastError();
}

template <int ADT>
hipError_t run_batch_k(int kclass, const BatchArgs& a, int grid, hipStream_t s) {
    switch (kclass) {
    case 1: return run_batch<1, ADT>(a, grid, s);
    case 2: return run_batch<2, ADT>(a, grid, s);
    case 3: return run_batch<3, ADT>(a, grid, s);
    case 4: return run_batch<4, ADT>(a, grid, s);
    case 5: return run_batch<5, ADT>(a, grid, s);
    case 6: return run_batch<6, ADT>(a, grid, s);
    case 8: return run_batch<8, ADT>(a, grid, s);
    case 12: return run_batch<12, ADT>(a, grid, s);
    case 16: return run_batch<16, ADT>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int batch_grid(int per_cu, int64_t total_tiles, int grid) {
    return resident_grid(per_cu, total_tiles, grid);
}

hipError_t launch_gemm_batch(const BatchArgs& a, int kclass, int adtype, int grid,
                             hipStream_t s) {
    if (a.count == 0 || a.total_tiles == 0) return hipSuccess;
    hipError_t e = adtype == 0   ? run_batch_k<0>(kclass, a, grid, s)
                   : adtype == 1 ? run_batch_k<1>(kclass, a, grid, s)
                                 : run_batch_k<2>(kclass, a, grid, s);
    if (e != hipSuccess) return e;
    return launch_reduce_batch(a, s);
}

}  // namespace sk
