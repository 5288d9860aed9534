// Streaming kernel for Y = A * Omega(seed) on gfx950 (small sketch width).
//
// The local product of Alg. 1 (GenRandom + local multiplication) and, for a
// contraction split, the sum of the partial products (the Reduce-Scatter of
// Alg. 1, done on the device).
//
// Work decomposition (one workgroup of 8 waves = one tile):
//   * a strip of C = 4096 consecutive columns of one A block times a range of
//     R rows, for all k <= 8 Omega columns;
//   * the strip is streamed in chunks of 1024 columns whose Omega slices live
//     in a double-buffered LDS ring:
//     generated from the seed (or copied from an explicit Omega for the
//     stored-operand variant) one chunk ahead, so Omega never exists in HBM
//     on the generated path and only the first chunk's generation is exposed;
//   * each wave streams passes of 8 rows (64 rows apart between the eight
//     waves): all 64 lanes read one row segment per step, 16 contiguous bytes
//     per lane (1 KB per load instruction), and multiply them by the matching
//     Omega values from LDS with FP32 FMAs into per-lane accumulators (8 rows
//     x kg columns per lane); two steps of nontemporal loads stay in flight
//     across passes and chunks;
//   * at the end of a pass the 64 lanes' accumulators are summed by a fixed
//     reduce-scatter (permlane32 and permlane16 swaps, then a DPP butterfly
//     inside 16-lane rows) and added, chunk after chunk, to the pass's FP32
//     strip sums; after the last chunk they go to the workspace (or to Y);
//   * a second small kernel sums the strip partials in FP64, in strip order,
//     adds beta * Y, rounds once and writes Y.  (No cross-workgroup
//     synchronisation inside the streaming kernel: device-scope release /
//     acquire would write back and invalidate the L2 of an XCD under every
//     streaming wave.)
// The summation order depends only on the strip and chunk boundaries, never
// on m, R or the grid, so results are bitwise reproducible and layout
// independent.
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

// The same 16-byte nontemporal load through a buffer descriptor: `row` is a
// wave-uniform address (scalar registers), voff the lane's byte offset, soff a
// wave-uniform byte offset, so no vector instruction forms the address.
__device__ __forceinline__ uint4 load_a16_row(const unsigned char* row, uint32_t voff,
                                              uint32_t soff) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<unsigned char*>(row), (short)0, (int)0xFFFFFFFFu, 0x00020000);
    const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 2 /* nt */);
    return make_uint4(v.x, v.y, v.z, v.w);
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

// LDS of one streaming workgroup: the double-buffered ring of Omega chunks and
// every thread's running strip sums (one slot per pass and reduced value).
template <int K>
struct StreamLds {
    static constexpr int CH = chunk_width(K);
    static constexpr int Q = 2 * K;                   // reduced values per 16-lane row and pass
    static constexpr int VPL = (Q + 15) / 16;         // reduced values per lane and pass
    static constexpr int NP = stream_max_rows(K) / kRowQuantum;   // passes per wave
    float om[2][K][CH];
    float sacc[NP * VPL][kWgThreads];
};

// Sum each of the V = 8K accumulators of a pass over the 64 lanes as a
// reduce-scatter.  permlane32_swap exchanges rows {2,3} of one register with
// rows {0,1} of another, so one swap + add halves the values per lane (lanes
// 0-31 keep the first half, lanes 32-63 the second); permlane16_swap does the
// same between rows 0|1 and 2|3; a 4-stage DPP butterfly finishes each value
// inside its 16-lane row.  Row r then holds values [r*V/4, (r+1)*V/4), lane
// sig of the row value 16*b + sig of that range in mine[b]; every addition
// order is fixed.
template <int K>
__device__ __forceinline__ void lane_reduce(const float (&acc)[kRowGroups][K], int lane,
                                            float (&mine)[StreamLds<K>::VPL]) {
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
    const int sig = lane & 15;
#pragma unroll
    for (int b = 0; b < StreamLds<K>::VPL; ++b) {
        float m = 0.0f;
#pragma unroll
        for (int j = 16 * b; j < 16 * b + 16 && j < Q; ++j)
            if (sig == j - 16 * b) m = qv[j];
        mine[b] = m;
    }
}

// One tile: a range of rows times one strip.  The strip is streamed chunk by
// chunk; all threads generate the next chunk's Omega slice into the other half
// of the LDS ring, a few quads at the start of each of their passes, while the
// current chunk's loads are in flight; one LDS-only barrier per chunk.  Each
// wave streams passes of 8 rows (64 rows apart between the eight waves): all 64
// lanes read one row segment per step, 16 contiguous bytes per lane (1 KB per
// load instruction), and multiply them by the matching Omega values from LDS
// with FP32 FMAs into per-lane accumulators; loads run two steps ahead across
// pass and chunk boundaries.  At the end of a pass the 64 lanes' accumulators
// are reduced (lane_reduce) and added, in chunk order, to the pass's running
// FP32 strip sums in LDS; after the last chunk the strip sums go to the
// workspace (or to Y when the call has one strip).  All threads call it.
template <int K, int ADT, bool GEN>
__device__ __forceinline__ void tile_body(const Tile& tl, StreamLds<K>& L) {
    constexpr int es = Elem<ADT>::size;
    constexpr int EPL = 16 / es;                 // elements per lane step
    constexpr int C = strip_width(K, ADT);       // columns per strip
    constexpr int CH = StreamLds<K>::CH;         // columns per chunk
    constexpr int STEP = kLanesPerRow * EPL;     // columns per wave step
    constexpr int TS = CH / STEP;                // steps per chunk
    constexpr int KD = TS >= kDepth ? kDepth : 1;
    constexpr int VPL = StreamLds<K>::VPL;
    constexpr int Q = StreamLds<K>::Q;
    static_assert(C % CH == 0 && CH % STEP == 0 && TS % KD == 0, "strip = whole chunks = whole steps");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // wave-uniform, so that row indices and row addresses live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kg = tl.kg;
    const int c_base = tl.c_base;
    const int64_t col_begin = tl.col_begin;
    const int w = (int)min<int64_t>(C, tl.n - col_begin);   // columns of this strip
    const int nch = (w + CH - 1) / CH;
    const int64_t row_end = tl.row_end;
    const int64_t lda_bytes = tl.lda * es;
    const int64_t first_pb = tl.row_begin + wave * kRowGroups;
    const int npass = first_pb < row_end ? (int)((row_end - first_pb + kRowQuantum - 1) / kRowQuantum) : 0;
    const unsigned char* strip_base = tl.A + col_begin * es;
    const int m_last = __builtin_amdgcn_readfirstlane((int)(tl.m - 1));
    const uint32_t lane_off = (uint32_t)lane * 16u;       // bytes

    // ---- A loads: step (chunk j, pass p, step t) reads 8 rows of this wave at
    //      strip columns j*CH + t*STEP + [lane*EPL, lane*EPL + EPL); the row
    //      address is wave-uniform, the lane offset a 32-bit vector offset ------
    int ij = npass > 0 ? 0 : nch, ip = 0, it_ = 0;   // next step to load
    auto issue = [&](uint4* buf) {
        if (ij >= nch) return;
        const int64_t pb = first_pb + (int64_t)ip * kRowQuantum;
        const int off = ij * CH + it_ * STEP;
        const unsigned char* colp = strip_base + (int64_t)off * es;
        if (off + STEP <= w) {
            // rows are below 2^31 (the host checks bound m); every quantity here is wave-uniform
            const int pr = __builtin_amdgcn_readfirstlane((int)pb);
#pragma unroll
            for (int i = 0; i < kRowGroups; ++i) {
                const int r = min(pr + i, m_last);
                buf[i] = load_a16_row(strip_base + (int64_t)r * lda_bytes, lane_off,
                                      (uint32_t)(off * es));
            }
        } else {
            // ragged end of the strip: only the valid elements are read
            const int left = w - off - lane * EPL;      // valid elements from this lane's first
#pragma unroll
            for (int i = 0; i < kRowGroups; ++i) {
                const unsigned char* ptr = colp + min<int64_t>(pb + i, tl.m - 1) * lda_bytes + lane_off;
                buf[i] = left >= EPL ? load_a16(ptr)
                         : left > 0  ? load_tail<ADT>(ptr, left)
                                     : make_uint4(0u, 0u, 0u, 0u);
            }
        }
        if (++it_ == TS) {
            it_ = 0;
            if (++ip == npass) {
                ip = 0;
                ++ij;
            }
        }
    };

    // ---- Omega chunk j -> L.om[j & 1]: items [i0, i1) of this thread's list ----
    // Generated: item = (Philox quad qi, column c), four consecutive Omega rows;
    // stored operand: item = (column jl of the chunk, Omega column c).
    const int64_t g0 = tl.row0 + col_begin;                  // global Omega row of strip column 0
    auto chunk_items = [&](int j) {
        const int wj = min(CH, w - j * CH);
        if constexpr (GEN) {
            const int64_t gj = g0 + (int64_t)j * CH;
            return (int)(((gj + wj - 1) >> 2) - (gj >> 2) + 1) * kg;
        } else {
            return wj * kg;
        }
    };
    auto gen_items = [&](int j, int i0, int i1) {
        float (*om)[CH] = L.om[j & 1];
        const int wj = min(CH, w - j * CH);
        const int items = chunk_items(j);
        const int64_t gj = g0 + (int64_t)j * CH;
        for (int i = i0; i < i1; ++i) {
            const int it = tid + i * kWgThreads;
            if (it >= items) break;
            if constexpr (GEN) {
                const int64_t q_lo = gj >> 2;
                const int qi = it / kg;
                const int c = it - qi * kg;
                const float4 z = omega4_dist((uint64_t)(q_lo + qi), tl.col0 + (uint32_t)(c_base + c),
                                             tl.key0, tl.key1, tl.dist);
                const int64_t p0 = 4 * (q_lo + qi) - gj;          // chunk column of z.x
                if ((gj & 3) == 0 && p0 + 3 < wj) {
                    *reinterpret_cast<float4*>(&om[c][p0]) = z;
                } else {
                    const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int64_t p = p0 + t;
                        if (p >= 0 && p < wj) om[c][p] = zz[t];
                    }
                }
            } else {
                const int jl = it / kg;
                const int c = it - jl * kg;
                om[c][jl] = tl.omega[(col_begin + (int64_t)j * CH + jl) * tl.ldo + c_base + c];
            }
        }
    };
    // zero what a ragged chunk or a partial column group leaves unwritten
    auto zero_unused = [&](int j) {
        const int wj = min(CH, w - j * CH);
        if (wj == CH && kg == K) return;
        float (*om)[CH] = L.om[j & 1];
        for (int it = tid; it < K * CH; it += kWgThreads) {
            const int c = it / CH;
            const int jl = it - c * CH;
            if (c >= kg || jl >= wj) om[c][jl] = 0.0f;
        }
    };

    uint4 bufs[KD][kRowGroups];
#pragma unroll
    for (int d = 0; d < KD; ++d) issue(bufs[d]);

    // chunk 0 while the first loads are in flight
    gen_items(0, 0, (chunk_items(0) + kWgThreads - 1) / kWgThreads);
    zero_unused(0);
    lds_barrier();

    // This thread's share of chunk j + 1 (cnt items), spread over the wave's
    // steps of chunk j: ips items after each step's load is issued.
    int cnt = 0, ips = 0, gi = 0;
    auto plan_next = [&](int j) {
        cnt = j + 1 < nch ? (chunk_items(j + 1) + kWgThreads - 1) / kWgThreads : 0;
        const int steps = npass * TS;
        ips = steps > 0 ? (cnt + steps - 1) / steps : cnt;
        gi = 0;
    };

    if (npass == 0) {
        // no rows for this wave: it only helps to build the chunks
        for (int j = 0; j + 1 < nch; ++j) {
            plan_next(j);
            gen_items(j + 1, 0, cnt);
            zero_unused(j + 1);
            lds_barrier();
        }
    } else {
        plan_next(0);
    }

    float acc[kRowGroups][K];
#pragma unroll
    for (int i = 0; i < kRowGroups; ++i)
#pragma unroll
        for (int c = 0; c < K; ++c) acc[i][c] = 0.0f;

    int cj = 0, cp = 0, ct = 0;   // next step to consume: chunk, pass, step
    auto fma_step = [&](const uint4* raw) {
        const float (*om)[CH] = L.om[cj & 1];
        float a[kRowGroups][EPL];
#pragma unroll
        for (int i = 0; i < kRowGroups; ++i) unpack16<ADT>(raw[i], a[i]);
        const int cl = ct * STEP + lane * EPL;
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
    };
    // after a step: a slice of the next chunk, then the pass / chunk bookkeeping
    auto advance = [&]() {
        if (gi < cnt) {
            gen_items(cj + 1, gi, min(cnt, gi + ips));
            gi += ips;
        }
        if (++ct < TS) return;
        // end of a pass: 64-lane sums, added to the pass's strip sums in chunk order
        ct = 0;
        float mine[VPL];
        lane_reduce<K>(acc, lane, mine);
#pragma unroll
        for (int b = 0; b < VPL; ++b) {
            float& sv = L.sacc[cp * VPL + b][tid];
            sv = (cj == 0) ? mine[b] : sv + mine[b];
        }
#pragma unroll
        for (int i = 0; i < kRowGroups; ++i)
#pragma unroll
            for (int c = 0; c < K; ++c) acc[i][c] = 0.0f;
        if (++cp < npass) return;
        // end of a chunk: the next one is complete once every wave is here
        cp = 0;
        if (cj + 1 < nch) {
            if (gi < cnt) gen_items(cj + 1, gi, cnt);
            zero_unused(cj + 1);
            lds_barrier();
        }
        ++cj;
        plan_next(cj);
    };

    if (npass > 0) {
        while (cj < nch) {
#pragma unroll
            for (int d = 0; d < KD; ++d) {
                if (cj < nch) {
                    fma_step(bufs[d]);
                    issue(bufs[d]);
                    advance();
                }
            }
        }
    }

    // ---- strip sums -> workspace (or Y) ----------------------------------------
    const int row16 = lane >> 4;
    const int sig = lane & 15;
    const int vbase = (row16 >> 1) * (kRowGroups * K / 2) + (row16 & 1) * Q;
    for (int p = 0; p < npass; ++p) {
        const int64_t pb = first_pb + (int64_t)p * kRowQuantum;
#pragma unroll
        for (int b = 0; b < VPL; ++b) {
            const int v = vbase + 16 * b + sig;        // accumulator index i*K + c
            const int wi = v / K;
            const int wc = v - wi * K;
            const int64_t r = pb + wi;
            if (16 * b + sig >= Q || r >= row_end || wc >= kg) continue;
            float val = L.sacc[p * VPL + b][tid];
            if (tl.scales) val *= tl.scales[r >> 7];
            if (tl.single) {
                double y = (double)val;
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
                tl.partials[(tl.strip_index * tl.m + r) * tl.k + c_base + wc] = val;
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
    __shared__ StreamLds<K> lds;
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
    tile_body<K, ADT, GEN>(tl, lds);
}

// A batch of independent requests (serving): the same tiles as one call per
// request, walked by a fixed grid; each request keeps its own seed, offsets,
// output and partial array, so its result does not depend on the batch.
template <int K, int ADT>
__global__ __launch_bounds__(kWgThreads) void k_gemm_batch(const BatchArgs args) {
    constexpr int C = strip_width(K, ADT);
    __shared__ StreamLds<K> lds;
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
        if (!first) lds_barrier();   // every wave is done with the previous tile's LDS
        first = false;
        tile_body<K, ADT, true>(tl, lds);
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
    for (; s + 8 <= S; s += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = __builtin_nontemporal_load(p + (int64_t)(s + j) * sstride);
#pragma unroll
        for (int j = 0; j < 8; ++j) y += (double)v[j];
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
    default:
        if constexpr (ADT == 0) return launch_k<8, ADT, GEN>(a, grid, s, tr);
        return hipErrorInvalidValue;   // BF16 past 6 columns runs on the matrix cores
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

// Rows per tile: a multiple of the pass height giving about one tile (one
// workgroup of 8 waves, the most that the kernel's registers let a compute
// unit hold) per compute unit, or two when that would leave tiles of fewer
// than 256 rows (a 4096 x 32768 share: 64-row tiles in two rounds measured
// 93 us against 129 us for one round of 128-row tiles, whose per-unit
// bandwidth spread then sets the end), at most max_rows (the per-pass strip
// sums of a tile live in LDS).  SKETCH_ROWS_PER_TILE overrides it for tuning
// (still capped at max_rows).
int64_t rows_per_tile(int64_t m, int64_t strips, int64_t ncg, int64_t max_rows) {
    static const int64_t forced = [] {
        const char* e = getenv("SKETCH_ROWS_PER_TILE");
        const long long v = e ? atoll(e) : 0;
        return (int64_t)(v > 0 ? v : 0);
    }();
    const int64_t cus = (int64_t)device_cus();
    const int64_t work = m * strips * ncg;
    int64_t R = (work + cus - 1) / cus;
    if (R < 256) R = (work + 2 * cus - 1) / (2 * cus);
    if (forced > 0) R = forced;
    R = (R + kRowQuantum - 1) / kRowQuantum * kRowQuantum;
    return std::max<int64_t>(kRowQuantum, std::min<int64_t>(R, max_rows));
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
    if (g.k > kStreamMaxK) return hipErrorInvalidValue;   // wider sketches run on the matrix cores
    const int64_t ncg = 1;
    const int kc = k_class((int)g.k);
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
    const int64_t R = rows_per_tile(g.m, S, ncg, stream_max_rows(kc));
    const int64_t nrb = (g.m + R - 1) / R;
    a.rows_per_wg = (int)R;
    a.num_rb = (int)nrb;
    a.tiles = S * nrb * ncg;
    a.tiles8 = (a.tiles + 7) / 8;
    if (S > 1) a.partials = static_cast<float*>(g.workspace);
    dim3 grid((unsigned)(8 * a.tiles8));
    const TraceEvents& tr = g.trace;
    // FP8 A always runs on the low-precision matrix-core kernel
    switch (g.adtype) {
    case 0: return gen ? dispatch_k<0, true>(kc, a, grid, g.stream, tr) : dispatch_k<0, false>(kc, a, grid, g.stream, tr);
    case 1: return gen ? dispatch_k<1, true>(kc, a, grid, g.stream, tr) : dispatch_k<1, false>(kc, a, grid, g.stream, tr);
    default: return hipErrorInvalidValue;
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
    case 8:
        if constexpr (ADT == 0) return run_batch<8, ADT>(a, grid, s);
        return hipErrorInvalidValue;
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
                                 : hipErrorInvalidValue;   // FP8: matrix-core batches only
    if (e != hipSuccess) return e;
    return launch_reduce_batch(a, s);
}

}  // namespace sk
