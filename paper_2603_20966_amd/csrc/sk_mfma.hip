// Matrix-core kernel for Y = A * Omega(seed) with a wide sketch (k > 16) on gfx950.
//
// Once k is large the product is a dense contraction (2k flops per A element;
// non-packed FP32 VALU FMAs reach their ridge near k = 20), so the local
// multiplication of Alg. 1 runs on the MFMA units: v_mfma_f32_16x16x4f32,
// FP32 in, FP32 accumulate.
//
// Tile of one workgroup (512 threads = 8 waves): 512 rows of A x a strip of
// kMfmaStrip contraction columns x BN = 16*NT sketch columns.  Each wave owns
// 64 rows (4 M-tiles of 16) x NT N-tiles, i.e. 4*NT accumulator tiles.  Eight
// waves share each generated Omega chunk, which halves the generation work per
// A element against four (measured: 109 vs 75 TFLOP/s at k = 256).
//
// Contraction in chunks of KC = 32 columns:
//   * A goes straight from HBM into the MFMA A-operand layout: lane (g, i)
//     (g = lane/16, i = lane%16) loads the KC/4 contiguous floats
//     A[row i][kc + g*KC/4 ...] of each M-tile as KC/16 back-to-back 16-byte
//     loads, so each 128-byte line of a row is requested at once; component s of
//     load v feeds one MFMA, whose contraction index g then stands for column
//     kc + g*KC/4 + 4v + s.  Any order of the contraction is a valid product, so
//     no shuffle is needed.  Plain (temporal) loads: the lines of a row are
//     shared by the four lanes of a row (measured faster than nontemporal).
//   * Omega for the chunk (KC x BN) is generated from the seed into one half of
//     a double-buffered LDS tile, laid out [column][KC + 4 pad] so that lane
//     (g, j) reads Omega[kc + g*KC/4 ...][j] as ds_read_b128s: exactly the B
//     operands of the same MFMAs.
//   * The next chunk's Omega is generated while this chunk's MFMAs run (VALU
//     and matrix cores work in parallel); one LDS-only barrier per chunk.
// Strip partials are FP32 in [S][m][k]; the FP64 strip sum is the shared
// reduction kernel.  The order of every sum depends only on the strip
// boundaries, so results are layout independent and reproducible.
#include <algorithm>

#include "sk_device.hpp"
#include "sk_internal.hpp"

#pragma clang fp contract(off)

namespace sk {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int kTM = 4;                  // M-tiles (16 rows) per wave
constexpr int kWaves = 8;               // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kBM = kWaves * kTM * 16;  // rows per workgroup
static_assert(kBM == kMfmaRows, "tile rows");
// contraction columns per chunk, and floats per LDS column (chunk + 4 pad):
// 32 at every N-tile count, so a chunk takes 128 bytes of each row (with 16
// columns every 128-byte line of A was fetched twice: 16 GiB instead of 8 for
// a two-block k = 256 sketch of 32768^2, rocprofv3 FETCH_SIZE).  With 8
// N-tiles the A operands are single-buffered (the accumulators take 128
// registers): a chunk's 256 MFMAs cover the next chunk's load.
constexpr int chunk_cols(int) { return 32; }
constexpr bool single_a(int nt) { return nt >= 8; }
constexpr int lds_row(int nt) { return chunk_cols(nt) + 4; }

struct MArgs {
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
    int y_f64;
    int beta;
    const uint16_t* opack;    // low-precision path: packed Omega, hi plane
    const uint16_t* opack_lo; // and lo plane
    int64_t kpad;             // sketch columns per packed chunk (k rounded up to the N-tile)
    int64_t nrt;              // row tiles
    int nblk;                 // sketch-column blocks
    const float* fpack;       // FP32 path with 4+ N-tiles: the call's packed Omega
    BlockDesc blk[kMaxBlocks];
};

// Tile of this workgroup in a one-dimensional grid of 8 * ceil(T / 8)
// workgroups over T = nblk * S_total * nrt tiles.
// XCD (low-precision kernel): workgroups are handed to the 8 XCDs
// round-robin, so XCD x runs ids x, x + 8, ...; mapping them to the contiguous
// tile range [x * T8, (x + 1) * T8), ordered sketch-column block fastest, then
// strip, then row tile, makes each XCD read whole rows of A (every strip of a
// row tile at once) and keeps the column blocks of one (strip, row tile) in
// one L2.  Measured on 32768^2 FP8 at k = 64: 290 us against 371 with the
// strip index fastest across XCDs.
// Otherwise (FP32 kernel, measured 2-3% faster so at k = 64): the id is the
// tile, strip fastest, then row tile, then column block.
// Returns false for the padding ids past T.
struct TileId {
    int strip;
    int64_t rtile;
    int nb;
};
template <bool XCD>
__device__ __forceinline__ bool mfma_tile_id(const MArgs& a, TileId& id) {
    const int64_t T = (int64_t)a.nblk * a.S_total * a.nrt;
    const int64_t v = blockIdx.x;
    if constexpr (XCD) {
        const int64_t T8 = (T + 7) / 8;
        const int64_t t = (v % 8) * T8 + v / 8;
        if (t >= T) return false;
        id.nb = (int)(t % a.nblk);
        const int64_t r = t / a.nblk;
        id.strip = (int)(r % a.S_total);
        id.rtile = r / a.S_total;
    } else {
        if (v >= T) return false;
        id.strip = (int)(v % a.S_total);
        const int64_t r = v / a.S_total;
        id.rtile = r % a.nrt;
        id.nb = (int)(r / a.nrt);
    }
    return true;
}

dim3 mfma_grid(const MArgs& a) {
    const int64_t T = (int64_t)a.nblk * a.S_total * a.nrt;
    return dim3((unsigned)(8 * ((T + 7) / 8)));
}

__device__ __forceinline__ void lds_barrier_m() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One tile: rows [block_row, block_row + 512) of a block, one strip of its
// columns, sketch columns [n_base, n_base + 16*NT).
struct MTile {
    const unsigned char* A;   // the block's A
    int64_t lda, n, row0;     // the block's ld, width, first Omega row
    const float* scales;
    int64_t m, k;
    int64_t col_begin;        // first column of the strip inside the block
    int64_t block_row;        // first row of the workgroup (before the wave offset)
    int n_base;
    uint32_t key0, key1, col0;
    int dist;                 // Omega's distribution (0 normal, 1 uniform, 2 Rademacher)
    const float* omega;
    int64_t ldo;
    void* Y;
    int64_t ldy;
    int y_f64, beta;
    float* partials;
    int64_t strip;            // strip index in the partial array
    bool single;
    const uint16_t* opack;    // packed Omega of the call (low-precision path), hi plane
    const uint16_t* opack_lo; // and lo plane
    int64_t kpad;
    const float* fpack;       // packed Omega of the call (FP32 path), or nullptr
};

// Arguments of the kernels that form a call's Omega once, before the product
// (k_f32_pack: one FP32 plane at hi; k_lp_pack: BF16 hi and lo planes).
struct PackArgs {
    void* hi;
    void* lo;
    int64_t k, kpad;
    uint32_t key0, key1, col0;
    int dist;
    const float* omega;       // stored Omega (n x k, ldo), or nullptr: generated
    int64_t ldo;
    int P;
    BlockDesc blk[kMaxBlocks];
};

// Write a wave's accumulators: lane (g, j) holds rows 4g..4g+3 and column j of
// each 16 x 16 tile.  The per-128-row scale (FP8 storage) is applied to each
// strip partial; a single-strip call writes Y directly (old Y added in FP64).
template <int NT>
__device__ __forceinline__ void store_tile(const MTile& t, const v4f (&acc)[kTM][NT],
                                           int64_t row_base, int kb, int g, int i16) {
#pragma unroll
    for (int tm = 0; tm < kTM; ++tm) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int cn = nt * 16 + i16;
            if (cn >= kb) continue;
            const int64_t col = t.n_base + cn;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int64_t r = row_base + tm * 16 + 4 * g + rr;
                if (r >= t.m) continue;
                float v = acc[tm][nt][rr];
                if (t.scales) v *= t.scales[r >> 7];
                if (t.single) {
                    double y = (double)v;
                    if (t.y_f64) {
                        double* Yp = static_cast<double*>(t.Y) + r * t.ldy + col;
                        if (t.beta) y += *Yp;
                        *Yp = y;
                    } else {
                        float* Yp = static_cast<float*>(t.Y) + r * t.ldy + col;
                        if (t.beta) y += (double)*Yp;
                        *Yp = (float)y;
                    }
                } else {
                    t.partials[(t.strip * t.m + r) * t.k + col] = v;
                }
            }
        }
    }
}

// Columns past k of both LDS halves (BN sketch columns x KC + 4 floats) are
// zeroed once: generation never writes them.
template <int BN, int KC>
__device__ __forceinline__ void omega_zero_pad(float (*om)[BN][KC + 4], int kb) {
    for (int it = threadIdx.x; it < 2 * BN * (KC + 4); it += kThreads) {
        const int n = (it / (KC + 4)) % BN;
        if (n >= kb) (&om[0][0][0])[it] = 0.0f;
    }
}

// Omega rows of chunk c of the tile's strip (kvalid of them; zeros past the
// strip's end) for sketch columns n_base .. n_base + kb - 1 -> LDS half c & 1,
// laid out [column][contraction]; generated from the seed, or read from a
// stored Omega.
template <int BN, int kKC, bool GEN>
__device__ __forceinline__ void omega_chunk(const MTile& t, float (*om)[BN][kKC + 4], int c, int w,
                                            int kb) {
    const int tid = threadIdx.x;
    const int nthr = kThreads;
    const int buf = c & 1;
    const int kvalid = min(kKC, w - c * kKC);
    if constexpr (GEN) {
        const int64_t g0 = t.row0 + t.col_begin + (int64_t)c * kKC;  // global Omega row of local 0
        const int64_t q_lo = g0 >> 2;
        const int nq = (int)(((g0 + kKC - 1) >> 2) - q_lo + 1);       // KC/4, or one more if unaligned
        const int items = nq * kb;
        for (int it = tid; it < items; it += nthr) {
            const int qi = it / kb;
            const int n = it - qi * kb;
            const float4 z = omega4_dist((uint64_t)(q_lo + qi), t.col0 + (uint32_t)(t.n_base + n),
                                         t.key0, t.key1, t.dist);
            const int kl0 = (int)(4 * (q_lo + qi) - g0);
            if (kl0 >= 0 && (kl0 & 3) == 0 && kl0 + 3 < kvalid) {
                *reinterpret_cast<float4*>(&om[buf][n][kl0]) = z;
            } else {
                const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int kl = kl0 + u;
                    if (kl >= 0 && kl < kKC) om[buf][n][kl] = (kl < kvalid) ? zz[u] : 0.0f;
                }
            }
        }
    } else {
        for (int it = tid; it < kKC * kb; it += nthr) {
            const int kl = it / kb;
            const int n = it - kl * kb;
            om[buf][n][kl] = (kl < kvalid)
                                 ? t.omega[(t.col_begin + (int64_t)c * kKC + kl) * t.ldo + t.n_base + n]
                                 : 0.0f;
        }
    }
}

// Chunks c0 .. c0 + G - 1 (those below nchunks) of the tile's strip, generated
// together into LDS slots slot0 .. slot0 + G - 1 (each laid out as above): with
// few sketch columns one chunk has too few Philox quads to occupy the
// workgroup, G of them do.  A chunk's first Omega row is aligned as the strip's
// (chunk widths are multiples of 4), so every chunk has the same quad count.
template <int BN, int kKC, int G>
__device__ __forceinline__ void omega_group(const MTile& t, float (*om)[BN][kKC + 4], int slot0,
                                            int c0, int nchunks, int w, int kb) {
    const int64_t gb = t.row0 + t.col_begin;                       // Omega row of strip column 0
    const int nq = (int)(((gb + kKC - 1) >> 2) - (gb >> 2) + 1);   // quads per chunk
    const int per = nq * kb;
    const int cnt = min(G, nchunks - c0);
    for (int it = threadIdx.x; it < cnt * per; it += kThreads) {
        const int ci = it / per;
        const int r = it - ci * per;
        const int qi = r / kb;
        const int n = r - qi * kb;
        const int c = c0 + ci;
        const int64_t g0 = gb + (int64_t)c * kKC;
        const int kvalid = min(kKC, w - c * kKC);
        const int64_t q = (g0 >> 2) + qi;
        const float4 z = omega4_dist((uint64_t)q, t.col0 + (uint32_t)(t.n_base + n), t.key0, t.key1,
                                     t.dist);
        const int kl0 = (int)(4 * q - g0);
        float* dst = om[slot0 + ci][n];
        if (kl0 >= 0 && (kl0 & 3) == 0 && kl0 + 3 < kvalid) {
            *reinterpret_cast<float4*>(&dst[kl0]) = z;
        } else {
            const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kl = kl0 + u;
                if (kl >= 0 && kl < kKC) dst[kl] = (kl < kvalid) ? zz[u] : 0.0f;
            }
        }
    }
}

// ---- Omega of a whole call for the FP32 tiles (four or more N-tiles) ---------
// As for the low-precision route: every 512-row tile of a strip multiplies the
// same Omega chunks, so the call forms them once.  One FP32 plane, chunk
// gc = strip * (kMfmaStrip / 32) + c, then sketch column n in [0, kpad), then
// contraction column kl in [0, 32): element (gc * kpad + n) * 32 + kl; the
// values (zeros past the strip's end and for n >= k) are those omega_chunk
// writes into LDS, so the sums are the same bit for bit.
constexpr int kF32PackRows = 16;   // sketch columns per packing workgroup
constexpr bool mfma_packed(int nt) { return nt >= 4; }

// grid (chunks of all strips / kF32PackChunks, ceil(kpad / 16)); 256 threads.
// A workgroup forms kF32PackChunks consecutive chunks of one strip (a strip is
// 64 chunks), so that its threads have Philox quads enough to keep busy.
constexpr int kF32PackChunks = 4;

template <bool GEN>
__global__ __launch_bounds__(256) void k_f32_pack(const PackArgs a) {
    constexpr int KC = chunk_cols(4);
    constexpr int CPS = kMfmaStrip / KC;
    constexpr int G = kF32PackChunks;
    static_assert(CPS % G == 0, "groups of chunks inside a strip");
    __shared__ __attribute__((aligned(16))) float sh[G][kF32PackRows][KC + 4];
    const int tid = threadIdx.x;
    const int64_t gc0 = (int64_t)blockIdx.x * G;          // first chunk of the group
    const int64_t strip = gc0 / CPS;
    const int c0 = (int)(gc0 - strip * CPS);
    int b = 0;
    int64_t sib = strip;
    for (; b < a.P; ++b) {
        const int64_t sb = (a.blk[b].n + kMfmaStrip - 1) / kMfmaStrip;
        if (sib < sb) break;
        sib -= sb;
    }
    const int64_t col_begin = sib * kMfmaStrip;
    const int w = (int)min<int64_t>(kMfmaStrip, a.blk[b].n - col_begin);
    const int nc = min(G, (w - c0 * KC + KC - 1) / KC);   // chunks of the group inside the strip
    if (nc <= 0) return;                                  // past the strip's end: never read
    const int nb0 = blockIdx.y * kF32PackRows;
    const int kb = (int)min<int64_t>(kF32PackRows, a.k - nb0);   // <= 0: all zero
    for (int it = tid; it < G * kF32PackRows * (KC + 4); it += 256) (&sh[0][0][0])[it] = 0.0f;
    __syncthreads();
    if constexpr (GEN) {
        // every chunk starts at the same offset within a Philox quad (KC is a multiple of 4)
        const int64_t gs = a.blk[b].row0 + col_begin + (int64_t)c0 * KC;
        const int nq = (int)(((gs + KC - 1) >> 2) - (gs >> 2) + 1);
        const int per = kb > 0 ? nq * kb : 0;
        for (int it = tid; it < nc * per; it += 256) {
            const int ci = it / per;
            const int r = it - ci * per;
            const int qi = r / kb;
            const int n = r - qi * kb;
            const int64_t g0 = gs + (int64_t)ci * KC;
            const int kvalid = min(KC, w - (c0 + ci) * KC);
            const int64_t q_lo = g0 >> 2;
            const float4 z = omega4_dist((uint64_t)(q_lo + qi), a.col0 + (uint32_t)(nb0 + n),
                                         a.key0, a.key1, a.dist);
            const int kl0 = (int)(4 * (q_lo + qi) - g0);
            const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kl = kl0 + u;
                if (kl >= 0 && kl < kvalid) sh[ci][n][kl] = zz[u];
            }
        }
    } else {
        const int per = kb > 0 ? KC * kb : 0;
        for (int it = tid; it < nc * per; it += 256) {
            const int ci = it / per;
            const int r = it - ci * per;
            const int kl = r / kb;
            const int n = r - kl * kb;
            if (kl < min(KC, w - (c0 + ci) * KC))
                sh[ci][n][kl] = a.omega[(col_begin + (int64_t)(c0 + ci) * KC + kl) * a.ldo + nb0 + n];
        }
    }
    __syncthreads();
    const int rows = (int)min<int64_t>(kF32PackRows, a.kpad - nb0);
    const int ppc = rows * (KC / 4);                      // 16-byte pieces per chunk
    float* out = static_cast<float*>(a.hi);
    for (int it = tid; it < nc * ppc; it += 256) {
        const int ci = it / ppc;
        const int pc = it - ci * ppc;
        const int n = pc / (KC / 4);
        const int kl4 = (pc - n * (KC / 4)) * 4;
        *reinterpret_cast<v4f*>(out + (((gc0 + ci) * a.kpad + nb0 + n) * KC + kl4)) =
            *reinterpret_cast<const v4f*>(&sh[ci][n][kl4]);
    }
}

// FULL: every chunk of the launch is whole (block widths multiples of the chunk
// width).  Then every lane issues the same A loads every chunk, unconditionally
// (a load past the strip's end re-reads its last chunk, never used), and the
// compiler waits for the chunk being multiplied alone; with the per-lane tail
// path present it waits for every load in flight, including the next chunk's,
// which undoes the double buffering.
// PK: Omega chunks copied from the call's packed Omega (k_f32_pack); the copy of
// chunk c + 2 is issued ahead of the A loads issued after it, so waiting for
// it leaves those in flight.
template <int NT, bool GEN, bool FULL = false, bool PK = false>
__device__ __forceinline__ void mfma_tile(const MTile& t, float (*om)[16 * NT][lds_row(NT)]) {
    constexpr int BN = 16 * NT;
    constexpr int kKC = chunk_cols(NT);
    constexpr int kLV = kKC / 16;   // 16-byte A loads per lane per M-tile per chunk
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = lane >> 4;      // contraction group of the lane (A and B operands)
    const int i16 = lane & 15;    // row (A operand) / column (B operand) within a tile

    const int w = (int)min<int64_t>(kMfmaStrip, t.n - t.col_begin);
    const int nchunks = (w + kKC - 1) / kKC;
    const int64_t row_base = t.block_row + wave * (kTM * 16);
    const int n_base = t.n_base;
    const int kb = (int)min<int64_t>(BN, t.k - n_base);

    // ---- A operand loads ----------------------------------------------------------
    const int64_t lda4 = t.lda * 4;
    const unsigned char* arow[kTM];
#pragma unroll
    for (int tm = 0; tm < kTM; ++tm) {
        const int64_t r = min<int64_t>(row_base + tm * 16 + i16, t.m - 1);
        arow[tm] = t.A + r * lda4 + (t.col_begin + 4 * kLV * g) * 4;
    }
    auto load_a = [&](v4f (*a)[kLV], int c) {
        if constexpr (FULL) {
            const int cc = c < nchunks ? c : nchunks - 1;
#pragma unroll
            for (int tm = 0; tm < kTM; ++tm) {
                const unsigned char* p = arow[tm] + (int64_t)cc * kKC * 4;
#pragma unroll
                for (int v = 0; v < kLV; ++v) a[tm][v] = *reinterpret_cast<const v4f*>(p + 16 * v);
            }
            return;
        }
        if (c >= nchunks) return;
        const int kl = c * kKC + 4 * kLV * g;               // local column of component 0
#pragma unroll
        for (int tm = 0; tm < kTM; ++tm) {
            const unsigned char* p = arow[tm] + (int64_t)c * kKC * 4;
            if (kl + 4 * kLV - 1 < w) {
#pragma unroll
                for (int v = 0; v < kLV; ++v) a[tm][v] = *reinterpret_cast<const v4f*>(p + 16 * v);
            } else {
                const float* pf = reinterpret_cast<const float*>(p);
#pragma unroll
                for (int v = 0; v < kLV; ++v) {
                    v4f x = {0.f, 0.f, 0.f, 0.f};
                    for (int e = 0; e < 4; ++e)
                        if (kl + 4 * v + e < w) x[e] = pf[4 * v + e];
                    a[tm][v] = x;
                }
            }
        }
    };

    // ---- Omega chunk -> LDS ----------------------------------------------------------
    if constexpr (!PK) omega_zero_pad<BN, kKC>(om, kb);
    auto make_chunk = [&](int c) { omega_chunk<BN, kKC, GEN>(t, om, c, w, kb); };
    // packed route: 16-byte pieces of the tile's run of a chunk, OPT per thread;
    // chunk indices past the last are clamped (a re-read of valid memory whose
    // copy lands in the LDS half no step reads next)
    constexpr int PPL = BN * kKC / 4;
    constexpr int OPT = (PPL + kThreads - 1) / kThreads;
    auto om_load = [&](v4f* r, int c) {
        const int cc = c < nchunks ? c : nchunks - 1;
        const float* src = t.fpack + ((t.strip * (kMfmaStrip / kKC) + cc) * t.kpad + n_base) * kKC;
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int p = min(tid + j * kThreads, PPL - 1);
            r[j] = *reinterpret_cast<const v4f*>(src + 4 * p);
        }
    };
    auto om_store = [&](const v4f* r, int c) {
        const int buf = c & 1;
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int p = min(tid + j * kThreads, PPL - 1);
            const int n = p / (kKC / 4);
            const int kl4 = (p - n * (kKC / 4)) * 4;
            *reinterpret_cast<v4f*>(&om[buf][n][kl4]) = r[j];
        }
    };

    v4f acc[kTM][NT];
#pragma unroll
    for (int tm = 0; tm < kTM; ++tm)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[tm][nt] = v4f{0.f, 0.f, 0.f, 0.f};

    v4f a0[kTM][kLV], a1[kTM][kLV];
    v4f orr[PK ? OPT : 1];
    if constexpr (PK) {
        load_a(a0, 0);
        om_load(orr, 0);
        om_store(orr, 0);
        if constexpr (!single_a(NT)) {
            om_load(orr, 1);
            __builtin_amdgcn_sched_barrier(0);
            load_a(a1, 1);
        }
    } else {
        load_a(a0, 0);
        if constexpr (!single_a(NT)) load_a(a1, 1);
        make_chunk(0);
    }
    lds_barrier_m();

    auto compute = [&](v4f (*a)[kLV], int c) {
        const int buf = c & 1;
#pragma unroll
        for (int v = 0; v < kLV; ++v) {
            v4f bop[NT];   // Omega operands of load v, read as they are used
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                bop[nt] = *reinterpret_cast<const v4f*>(&om[buf][nt * 16 + i16][4 * kLV * g + 4 * v]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int tm = 0; tm < kTM; ++tm)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[tm][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            a[tm][v][s], bop[nt][s], acc[tm][nt], 0, 0, 0);
        }
    };

    if constexpr (PK && single_a(NT)) {
        // one A buffer (the accumulators leave no room for more): step c runs
        // chunk c's MFMAs, then issues chunk c + 1's A and Omega loads and
        // stores the Omega copy (its registers are never live across MFMAs);
        // the next step needs those A loads at once either way
        for (int c = 0; c < nchunks; ++c) {
            compute(a0, c);
            load_a(a0, c + 1);
            om_load(orr, c + 1);
            om_store(orr, c + 1);
            lds_barrier_m();
        }
    } else if constexpr (PK) {
        for (int c = 0; c < nchunks; c += 2) {
            om_store(orr, c + 1);
            om_load(orr, c + 2);
            __builtin_amdgcn_sched_barrier(0);
            compute(a0, c);
            load_a(a0, c + 2);
            if constexpr (FULL) __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
            om_store(orr, c + 2);
            om_load(orr, c + 3);
            __builtin_amdgcn_sched_barrier(0);
            if (c + 1 < nchunks) compute(a1, c + 1);
            load_a(a1, c + 3);
            if constexpr (FULL) __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
        }
    } else if constexpr (single_a(NT)) {
        for (int c = 0; c < nchunks; ++c) {
            if (c + 1 < nchunks) make_chunk(c + 1);
            compute(a0, c);
            load_a(a0, c + 1);
            lds_barrier_m();
        }
    } else {
        for (int c = 0; c < nchunks; c += 2) {
            if (c + 1 < nchunks) make_chunk(c + 1);
            compute(a0, c);
            load_a(a0, c + 2);
            lds_barrier_m();
            if (c + 1 < nchunks) {
                if (c + 2 < nchunks) make_chunk(c + 2);
                compute(a1, c + 1);
                load_a(a1, c + 3);
                lds_barrier_m();
            }
        }
    }

    store_tile<NT>(t, acc, row_base, kb, g, i16);
}

// One call: one workgroup per (strip of any block, 512-row tile, sketch-column
// block), strip fastest.
template <int NT, bool GEN, bool FULL>
__global__ __launch_bounds__(kThreads) void k_gemm_mfma(const MArgs args) {
    __shared__ float om[2][16 * NT][lds_row(NT)];
    TileId id;
    if (!mfma_tile_id<false>(args, id)) return;
    const int strip = id.strip;
    int b = 0;
    int64_t sib = strip;
    for (; b < args.P; ++b) {
        const int64_t sb = (args.blk[b].n + kMfmaStrip - 1) / kMfmaStrip;
        if (sib < sb) break;
        sib -= sb;
    }
    const BlockDesc& blk = args.blk[b];
    MTile t;
    t.A = static_cast<const unsigned char*>(blk.A);
    t.lda = blk.lda;
    t.n = blk.n;
    t.row0 = blk.row0;
    t.scales = blk.scales;
    t.m = args.m;
    t.k = args.k;
    t.col_begin = sib * kMfmaStrip;
    t.block_row = id.rtile * kBM;
    t.n_base = id.nb * 16 * NT;
    t.key0 = args.key0;
    t.key1 = args.key1;
    t.col0 = args.col0;
    t.dist = args.dist;
    t.omega = args.omega;
    t.ldo = args.ldo;
    t.Y = args.Y;
    t.ldy = args.ldy;
    t.y_f64 = args.y_f64;
    t.beta = args.beta;
    t.partials = args.partials;
    t.strip = strip;
    t.single = (args.S_total == 1);
    t.opack = nullptr;
    t.opack_lo = nullptr;
    t.kpad = args.kpad;
    t.fpack = args.fpack;
    mfma_tile<NT, GEN, FULL, mfma_packed(NT)>(t, om);
}

// A batch of independent requests (serving): the tiles of each request are the
// ones a call for that request alone would run, walked by a fixed grid in an
// XCD-grouped order, so each result does not depend on the batch.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_gemm_mfma_batch(const BatchArgs args) {
    __shared__ float om[2][16 * NT][lds_row(NT)];
    const int64_t T8 = (args.total_tiles + 7) / 8;
    bool first = true;
    for (int64_t v = blockIdx.x; v < 8 * T8; v += gridDim.x) {   // gridDim.x is a multiple of 8
        const int64_t tt = (v % 8) * T8 + v / 8;
        if (tt >= args.total_tiles) continue;
        int q = 0;
        while (q + 1 < args.count && tt >= args.req[q + 1].tile_begin) ++q;
        const BatchReq& rq = args.req[q];
        const int64_t lt = tt - rq.tile_begin;
        const int64_t strip = lt % rq.strips;
        const int64_t rb = (lt / rq.strips) % rq.rowblocks;
        const int nb = (int)(lt / ((int64_t)rq.strips * rq.rowblocks));
        MTile t;
        t.A = static_cast<const unsigned char*>(rq.A);
        t.lda = rq.lda;
        t.n = rq.n;
        t.row0 = rq.row0;
        t.scales = rq.scales;
        t.m = rq.m;
        t.k = rq.k;
        t.col_begin = strip * kMfmaStrip;
        t.block_row = rb * kBM;
        t.n_base = nb * 16 * NT;
        t.key0 = (uint32_t)rq.seed;
        t.key1 = (uint32_t)(rq.seed >> 32);
        t.col0 = rq.col0;
        t.dist = rq.dist;
        t.omega = nullptr;
        t.ldo = 0;
        t.Y = rq.Y;
        t.ldy = rq.ldy;
        t.y_f64 = rq.y_f64;
        t.beta = rq.beta;
        t.partials = rq.partials;
        t.strip = strip;
        t.single = (rq.strips == 1);
        t.opack = nullptr;
        t.opack_lo = nullptr;
        t.kpad = 0;
        t.fpack = nullptr;
        if (!first) lds_barrier_m();   // every wave is done with the previous tile's LDS
        first = false;
        mfma_tile<NT, true>(t, om);
    }
}

// ---------------------------------------------------------------------------
// Column-major A (element (i, j) at A + j*lda + i, the paper's storage order) on
// the same matrix cores, for k > 16.  The tile computes the transposed product
// Y^T = Omega^T A^T: the Omega chunk in LDS (same layout and same reads as the
// B operand above) is the A operand, and A enters as the B operand straight
// from HBM.  Lane (g, j) loads 16 bytes, rows 4j .. 4j + 3 of one column (a
// wave reads 256 contiguous bytes of each of four columns per load); component
// q of the load feeds the MFMA of row set {4j + q}, so a wave holds four 16 x 16
// accumulator tiles of Y^T per N-tile, covering 64 rows.  Step s of a chunk
// reads column kc + g*KC/4 + s, the column that contraction index g of step s
// stands for in the row-major kernel: both kernels form the same products in
// the same order, and every A element is read once for all k sketch columns.
struct CmMArgs {
    const float* A;
    int64_t m, n, lda, row0;
    uint32_t key0, key1, col0;
    int dist;
    int64_t k;
    void* Y;
    int64_t ldy;
    int y_trans, y_f64, beta;
    float* partials;
    int S;                 // strips of kMfmaStrip columns
    int num_rb;            // 512-row tiles
    int64_t tiles, tiles8;
    const float* fpack;    // four or more N-tiles: the call's packed Omega (k_f32_pack)
    int64_t kpad;
};

// KC = the row-major kernel's chunk for this k (chunk_cols(mfma_ntiles(k))),
// whatever N-tile count the launch picked, so that the sums are the same.
// FULL (m a multiple of 4, whole chunks): every lane of every wave issues the same
// loads each chunk from a valid address (a lane or wave without rows reads row 0;
// its sums are never stored; a load past the strip's end re-reads its last chunk),
// so the compiler waits for the chunk in use alone (see mfma_tile).
// Packed Omega on the column-major tiles: four or more N-tiles, except eight
// without whole chunks (that kernel's registers have no room for the copy).
constexpr bool cm_packed(int nt, bool full) { return mfma_packed(nt) && (full || nt < 8); }

template <int NT, int kKC, bool FULL>
__global__ __launch_bounds__(kThreads) void k_gemm_cm_mfma(const CmMArgs a) {
    constexpr int BN = 16 * NT;
    constexpr int kNS = kKC / 4;     // MFMA steps (and 16-byte loads per lane) per chunk
    constexpr int kLV = kKC / 16;    // 16-byte Omega reads per lane and N-tile per chunk
    // chunks generated per barrier: enough quads for every thread (1 when BN*KC/4 >= 512)
    constexpr int kG = kThreads / (kNS * BN) > 1 ? kThreads / (kNS * BN) : 1;
    static_assert(kG == 1 || kG % 2 == 0, "chunk pairs per generation group");
    __shared__ float om[2 * kG][BN][kKC + 4];

    const int64_t id = blockIdx.x;
    const int64_t tt = (id % 8) * a.tiles8 + id / 8;       // XCD-grouped tile order
    if (tt >= a.tiles) return;
    const int strip = (int)(tt % a.S);
    const int rb = (int)((tt / a.S) % a.num_rb);
    const int nb = (int)(tt / ((int64_t)a.S * a.num_rb));

    MTile t{};
    t.row0 = a.row0;
    t.col_begin = (int64_t)strip * kMfmaStrip;
    t.n_base = nb * BN;
    t.key0 = a.key0;
    t.key1 = a.key1;
    t.col0 = a.col0;
    t.dist = a.dist;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int j = lane & 15;
    const int w = (int)min<int64_t>(kMfmaStrip, a.n - t.col_begin);
    const int nchunks = (w + kKC - 1) / kKC;
    const int kb = (int)min<int64_t>(BN, a.k - t.n_base);
    const int64_t r0 = (int64_t)rb * kBM + wave * 64;      // first row of the wave
    const int64_t rl = r0 + 4 * j;                          // first row of the lane
    const bool active = r0 < a.m;                           // the wave has rows
    const bool full_rows = rl + 3 < a.m;

    // ---- A loads: step s of chunk c is column col_begin + c*KC + g*KC/4 + s --------
    const float* acol = a.A + (t.col_begin + g * kNS) * a.lda + (FULL && rl >= a.m ? 0 : rl);
    auto load_a = [&](v4f* x, int c) {
        if constexpr (FULL) {
            const int cc = c < nchunks ? c : nchunks - 1;
#pragma unroll
            for (int s = 0; s < kNS; ++s)
                x[s] = *reinterpret_cast<const v4f*>(acol + (int64_t)(cc * kKC + s) * a.lda);
            return;
        }
        if (!active || c >= nchunks) return;
        const int kl = c * kKC + g * kNS;
#pragma unroll
        for (int s = 0; s < kNS; ++s) {
            const float* p = acol + (int64_t)(c * kKC + s) * a.lda;
            if (full_rows && kl + s < w) {
                x[s] = *reinterpret_cast<const v4f*>(p);
            } else {
                v4f v = {0.f, 0.f, 0.f, 0.f};
                if (kl + s < w)
                    for (int q = 0; q < 4; ++q)
                        if (rl + q < a.m) v[q] = p[q];
                x[s] = v;
            }
        }
    };

    // packed route (as mfma_tile): 16-byte pieces of the tile's run of a chunk
    constexpr bool PK = cm_packed(NT, FULL);
    constexpr int PPL = BN * kKC / 4;
    constexpr int OPT = (PPL + kThreads - 1) / kThreads;
    const int tid = threadIdx.x;
    auto om_load = [&](v4f* r, int c) {
        const int cc = c < nchunks ? c : nchunks - 1;
        const float* src = a.fpack + (((int64_t)strip * (kMfmaStrip / kKC) + cc) * a.kpad + t.n_base) * kKC;
#pragma unroll
        for (int i = 0; i < OPT; ++i) {
            const int p = min(tid + i * kThreads, PPL - 1);
            r[i] = *reinterpret_cast<const v4f*>(src + 4 * p);
        }
    };
    auto om_store = [&](const v4f* r, int slot) {
#pragma unroll
        for (int i = 0; i < OPT; ++i) {
            const int p = min(tid + i * kThreads, PPL - 1);
            const int n = p / (kKC / 4);
            const int kl4 = (p - n * (kKC / 4)) * 4;
            *reinterpret_cast<v4f*>(&om[slot][n][kl4]) = r[i];
        }
    };

    if constexpr (!PK) omega_zero_pad<BN, kKC>(om, kb);
    v4f acc[4][NT];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[q][nt] = v4f{0.f, 0.f, 0.f, 0.f};

    v4f a0[kNS], a1[kNS];
    v4f orr[PK ? OPT : 1];
    if constexpr (PK) {
        static_assert(!PK || kG == 1, "one chunk per barrier on the packed route");
        load_a(a0, 0);
        om_load(orr, 0);
        om_store(orr, 0);
        if constexpr (!single_a(NT)) {
            om_load(orr, 1);
            __builtin_amdgcn_sched_barrier(0);
            load_a(a1, 1);
        }
    } else {
        load_a(a0, 0);
        if constexpr (!single_a(NT)) load_a(a1, 1);
        omega_group<BN, kKC, kG>(t, om, 0, 0, nchunks, w, kb);
    }
    lds_barrier_m();

    auto compute = [&](const v4f* x, int buf) {
        if (!active) return;
        v4f wop[NT][kLV];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < kLV; ++v)
                wop[nt][v] = *reinterpret_cast<const v4f*>(&om[buf][nt * 16 + j][4 * kLV * g + 4 * v]);
#pragma unroll
        for (int v = 0; v < kLV; ++v)
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[q][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            wop[nt][v][s], x[4 * v + s][q], acc[q][nt], 0, 0, 0);
    };

    if constexpr (PK && single_a(NT)) {
        // the order of mfma_tile's packed loops (Omega copies never live across MFMAs here)
        for (int c = 0; c < nchunks; ++c) {
            compute(a0, c & 1);
            load_a(a0, c + 1);
            om_load(orr, c + 1);
            om_store(orr, (c + 1) & 1);
            lds_barrier_m();
        }
    } else if constexpr (PK) {
        for (int c = 0; c < nchunks; c += 2) {
            om_store(orr, 1);
            om_load(orr, c + 2);
            __builtin_amdgcn_sched_barrier(0);
            compute(a0, 0);
            load_a(a0, c + 2);
            if constexpr (FULL) __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
            om_store(orr, 0);
            om_load(orr, c + 3);
            __builtin_amdgcn_sched_barrier(0);
            if (c + 1 < nchunks) compute(a1, 1);
            load_a(a1, c + 3);
            if constexpr (FULL) __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
        }
    } else if constexpr (single_a(NT)) {
        for (int c = 0; c < nchunks; ++c) {
            if (c + 1 < nchunks) omega_group<BN, kKC, 1>(t, om, (c + 1) & 1, c + 1, nchunks, w, kb);
            compute(a0, c & 1);
            load_a(a0, c + 1);
            lds_barrier_m();
        }
    } else if constexpr (kG == 1) {
        for (int c = 0; c < nchunks; c += 2) {
            if (c + 1 < nchunks) omega_group<BN, kKC, 1>(t, om, 1, c + 1, nchunks, w, kb);
            compute(a0, 0);
            load_a(a0, c + 2);
            lds_barrier_m();
            if (c + 1 < nchunks) {
                if (c + 2 < nchunks) omega_group<BN, kKC, 1>(t, om, 0, c + 2, nchunks, w, kb);
                compute(a1, 1);
                load_a(a1, c + 3);
                lds_barrier_m();
            }
        }
    } else {
        // group u of kG chunks sits in slots (u & 1) kG ..; the next group is generated
        // into the other half while this one is consumed, one barrier per group
        for (int cb = 0; cb < nchunks; cb += kG) {
            const int half = (cb / kG) & 1;
            if (cb + kG < nchunks) omega_group<BN, kKC, kG>(t, om, (half ^ 1) * kG, cb + kG, nchunks, w, kb);
#pragma unroll
            for (int i = 0; i < kG; i += 2) {
                if (cb + i < nchunks) {
                    compute(a0, half * kG + i);
                    load_a(a0, cb + i + 2);
                }
                if (cb + i + 1 < nchunks) {
                    compute(a1, half * kG + i + 1);
                    load_a(a1, cb + i + 3);
                }
            }
            lds_barrier_m();
        }
    }
    if (!active) return;

    // ---- lane l holds Y^T rows (sketch columns) 4g .. 4g + 3 of column j of each
    // accumulator tile: Y[rl + q][n_base + 16 nt + 4g + r] = acc[q][nt][r] ---------------
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t row = rl + q;
        if (row >= a.m) continue;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int cn = nt * 16 + 4 * g + r;
                if (cn >= kb) continue;
                const int64_t col = t.n_base + cn;
                const float v = acc[q][nt][r];
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
}

// Few rows (m <= 64; e.g. B^T of the Nystrom second product): the kernel above
// gives a tile's 64 rows to one wave, which runs all 4 x NT accumulator chains
// while the other seven idle.  Here a workgroup takes one strip and one N-tile of
// 16 sketch columns, and its waves split the work: waves 0..3 each run one chain
// (row set q = wave: rows 4j + q of lane j) with the steps, operands and order of
// the kernel above, so the results equal it (and the row-major kernel) bit for
// bit; waves 4..11 stage kSkG chunks at a time, A and the call's packed Omega,
// into the other half of a double-buffered LDS ring, with the loads of the group
// after next in flight while they store the next one.  A chain's step then waits
// on LDS only, not on a global load.  The launch always packs the call's Omega
// for this kernel (a.fpack is set).  Eight staging waves rather than four: the
// staging alone took most of the kernel's time.
constexpr int kSkG = 4;
constexpr int kSkChainThreads = 256;                       // waves 0..3
constexpr int kSkGenThreads = 512;                         // waves 4..11
constexpr int kSkThreads = kSkChainThreads + kSkGenThreads;

template <int kKC, bool ALIGNED>
__global__ __launch_bounds__(kSkThreads) void k_gemm_cm_mfma_skinny(const CmMArgs a) {
    constexpr int BN = 16;
    constexpr int kNS = kKC / 4;
    constexpr int kLV = kKC / 16;
    constexpr int kGenThreads = kSkGenThreads;
    // a staged column of A: row 4j + q at [q][j], 2 floats of padding so that the
    // four lane groups of a chain's read (8 columns apart) fall on different banks
    constexpr int kAP = 66;
    constexpr int kAPieces = kSkG * kKC * 16 / kGenThreads;       // 16-byte pieces of A per thread
    constexpr int kOPieces = kSkG * BN * kKC / 4 / kGenThreads;   // and of Omega
    static_assert(kAPieces * kGenThreads == kSkG * kKC * 16 &&
                  kOPieces * kGenThreads == kSkG * BN * kKC / 4, "whole pieces per thread");
    __shared__ __attribute__((aligned(16))) float om[2 * kSkG][BN][kKC + 4];
    __shared__ float as[2 * kSkG][kKC][kAP];

    const int64_t tt = blockIdx.x;
    if (tt >= a.tiles) return;
    const int strip = (int)(tt % a.S);
    const int nb = (int)(tt / a.S);
    const int64_t col_begin = (int64_t)strip * kMfmaStrip;
    const int n_base = nb * BN;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const bool gen_wave = wave >= 4;
    const int q = wave & 3;
    const int g = lane >> 4;
    const int j = lane & 15;
    const int w = (int)min<int64_t>(kMfmaStrip, a.n - col_begin);
    const int nchunks = (w + kKC - 1) / kKC;
    const int ngroups = (nchunks + kSkG - 1) / kSkG;
    const int kb = (int)min<int64_t>(BN, a.k - n_base);
    const int64_t rl = 4 * j;                               // first row of the lane

    // columns past k of every slot are zero (the packed plane holds zeros there too)
    for (int it = threadIdx.x; it < 2 * kSkG * BN * (kKC + 4); it += kSkThreads) {
        const int n = (it / (kKC + 4)) % BN;
        if (n >= kb) (&om[0][0][0])[it] = 0.0f;
    }

    // staging (waves 4..7).  Every load is issued unconditionally from a valid
    // address (chunks past the strip's last re-read it, rows past m read rows 0..3,
    // columns past the strip's end read its last column), so the compiler waits for
    // the older group only; columns past the strip's end are stored as zeros, rows
    // past m are never stored by the chains.
    const int tg = threadIdx.x - kSkChainThreads;
    auto g_load = [&](int gi, v4f* xa, v4f* xo) {
#pragma unroll
        for (int t = 0; t < kAPieces; ++t) {
            const int p = tg + t * kGenThreads;
            const int ci = p / (kKC * 16);
            const int rem = p - ci * (kKC * 16);
            const int col = rem >> 4;
            const int r4 = rem & 15;
            const int c = min(gi * kSkG + ci, nchunks - 1);
            const int64_t colg = col_begin + min(c * kKC + col, w - 1);
            const float* src = a.A + colg * a.lda;
            if constexpr (ALIGNED) {
                xa[t] = *reinterpret_cast<const v4f*>(src + (4 * r4 < a.m ? 4 * r4 : 0));
            } else {
                v4f v = {0.f, 0.f, 0.f, 0.f};
                if (4 * r4 + 3 < a.m) {
                    v = *reinterpret_cast<const v4f*>(src + 4 * r4);
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (4 * r4 + e < a.m) v[e] = src[4 * r4 + e];
                }
                xa[t] = v;
            }
        }
#pragma unroll
        for (int t = 0; t < kOPieces; ++t) {
            const int it = tg + t * kGenThreads;
            constexpr int PPC = BN * kKC / 4;                   // pieces per chunk
            const int ci = it / PPC;
            const int pc = it - ci * PPC;
            const int c = min(gi * kSkG + ci, nchunks - 1);
            const int n = pc / (kKC / 4);
            const int kl4 = (pc - n * (kKC / 4)) * 4;
            xo[t] = *reinterpret_cast<const v4f*>(
                a.fpack + (((int64_t)strip * (kMfmaStrip / kKC) + c) * a.kpad + n_base + n) * kKC + kl4);
        }
    };
    auto g_store = [&](int gi, const v4f* xa, const v4f* xo) {
        const int slot0 = (gi & 1) * kSkG;
#pragma unroll
        for (int t = 0; t < kAPieces; ++t) {
            const int p = tg + t * kGenThreads;
            const int ci = p / (kKC * 16);
            const int rem = p - ci * (kKC * 16);
            const int col = rem >> 4;
            const int r4 = rem & 15;
            const bool inside = (gi * kSkG + ci) * kKC + col < w;
            float* dst = &as[slot0 + ci][col][r4];
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[16 * e] = inside ? xa[t][e] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < kOPieces; ++t) {
            const int it = tg + t * kGenThreads;
            constexpr int PPC = BN * kKC / 4;
            const int ci = it / PPC;
            const int pc = it - ci * PPC;
            const int n = pc / (kKC / 4);
            const int kl4 = (pc - n * (kKC / 4)) * 4;
            *reinterpret_cast<v4f*>(&om[slot0 + ci][n][kl4]) = xo[t];
        }
    };

    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
    auto chain_group = [&](int gi) {
        const int slot0 = (gi & 1) * kSkG;
#pragma unroll
        for (int cc = 0; cc < kSkG; ++cc) {
            if (gi * kSkG + cc < nchunks) {
                const float* ob = &om[slot0 + cc][j][4 * kLV * g];
                v4f wop[kLV];
#pragma unroll
                for (int v = 0; v < kLV; ++v) wop[v] = *reinterpret_cast<const v4f*>(ob + 4 * v);
                const float* ab = &as[slot0 + cc][g * kNS][16 * q + j];
                float x[kNS];
#pragma unroll
                for (int s = 0; s < kNS; ++s) x[s] = ab[s * kAP];
#pragma unroll
                for (int v = 0; v < kLV; ++v)
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wop[v][s], x[4 * v + s], acc, 0, 0, 0);
            }
        }
    };

    v4f ra[kAPieces], ro[kOPieces], rb[kAPieces], rbo[kOPieces];
    if (gen_wave) {
        g_load(0, ra, ro);
        g_store(0, ra, ro);
        g_load(min(1, ngroups - 1), ra, ro);
    }
    lds_barrier_m();
    // group gi: the chains use slot gi & 1; the stagers store group gi + 1 (held in
    // cur) into the other slot after issuing the loads of group gi + 2 into nxt
    auto iter = [&](int gi, v4f* cur_a, v4f* cur_o, v4f* nxt_a, v4f* nxt_o) {
        if (gen_wave) {
            g_load(min(gi + 2, ngroups - 1), nxt_a, nxt_o);
            if (gi + 1 < ngroups) g_store(gi + 1, cur_a, cur_o);
        } else {
            chain_group(gi);
        }
        lds_barrier_m();
    };
    for (int gi = 0; gi < ngroups; gi += 2) {
        iter(gi, ra, ro, rb, rbo);
        if (gi + 1 < ngroups) iter(gi + 1, rb, rbo, ra, ro);
    }
    if (gen_wave) return;

    // lane (g, j) holds Y^T rows (sketch columns) 4g .. 4g + 3 of column j of the tile:
    // Y[rl + q][n_base + 4g + r] = acc[r]
    const int64_t row = rl + q;
    if (row >= a.m) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int cn = 4 * g + r;
        if (cn >= kb) continue;
        const int64_t col = n_base + cn;
        const float v = acc[r];
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

template <int NT, int KC>
hipError_t launch_cm_mfma_nt(const CmMArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)(8 * a.tiles8));
    if (a.m % 4 == 0 && a.n % KC == 0)
        hipLaunchKernelGGL((k_gemm_cm_mfma<NT, KC, true>), grid, dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_gemm_cm_mfma<NT, KC, false>), grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Low-precision A (BF16, or FP8-E4M3 widened to BF16 exactly) on the BF16
// matrix cores: v_mfma_f32_16x16x32_bf16, FP32 accumulate.  Omega is split into
// two BF16 terms, hi = bf16(w) and lo = bf16(w - hi), and each step runs two
// MFMAs (A*hi, then A*lo): |w - hi - lo| <= 2^-16 |w|, far below the storage
// error of A, so the product carries A's quantisation only.  The workgroup
// is W waves x 64 rows sharing each generated Omega chunk (a run of
// contraction columns): the more rows, the less generation per A element, which matters
// because a byte of FP8 holds four times the elements of a byte of FP32.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Contraction columns per chunk: 128 bytes of every row (BF16: 64 columns,
// FP8: 128), 32 bytes per lane, so a row is read in whole 128-byte lines
// (measured: 64-byte runs cost FP8 a quarter of its rate; 256-byte runs gain
// nothing and cost registers).
constexpr int lp_kc(int adt) { return adt == 2 ? 128 : 64; }
constexpr int lp_row(int adt) { return lp_kc(adt) + 8; }   // bf16 per LDS column (+8 pad)
static_assert(64 * kLpBatchWaves == kLpBatchRows, "batch tile rows");

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// Omega value -> (hi, lo) BF16 bit patterns; z - hi is exact in FP32.
__device__ __forceinline__ void split_bf16(float z, uint16_t& hi, uint16_t& lo) {
    const uint32_t h = bf16_rne_bits(z);
    hi = (uint16_t)h;
    lo = (uint16_t)bf16_rne_bits(z - __uint_as_float(h << 16));
}

// 4 FP8-E4M3 codes (one word) -> 4 BF16 in two words, element order kept (exact:
// 4 significant bits).  PACKED: one gfx950 packed conversion per pair (scale 1);
// otherwise through FP32 and a repack.  Both give the same bits; measured on
// 32768^2, the packed form is 3% faster with four N-tiles and 3% slower with
// one (whose kernel sits at the 128-register cap).
template <bool PACKED>
__device__ __forceinline__ void fp8x4_to_bf16(uint32_t w, uint32_t& lo2, uint32_t& hi2) {
    if constexpr (PACKED) {
        lo2 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)w, 1.0f, false));
        hi2 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)w, 1.0f, true));
    } else {
        const auto a = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
        const auto b = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
        lo2 = (__float_as_uint(a[1]) & 0xFFFF0000u) | (__float_as_uint(a[0]) >> 16);
        hi2 = (__float_as_uint(b[1]) & 0xFFFF0000u) | (__float_as_uint(b[0]) >> 16);
    }
}

// ---- Omega of a whole call, split and laid out for the low-precision tiles ----
// Every row tile of a strip multiplies the same Omega chunks, so a call's
// Omega (hi, lo) is formed once, before the product, instead of once per
// 64W-row tile (a 32768-row FP8 call has 64 tiles per strip).  Layout, one
// plane for hi and one for lo: chunk gc = strip * (kLpStrip / KC) + c, then
// sketch column n in [0, kpad), then contraction column kl in [0, KC):
// element ((gc * kpad + n) * KC + kl).  A tile's BN columns of a chunk are
// then one contiguous run of BN * KC values.  Entries past the strip's last
// column and sketch columns >= k hold zero; the values are those the fused
// generation writes into LDS, so both routes give the same sums bit for bit.

// sketch columns per packing workgroup: 16 gives each compute unit several
// workgroups to interleave (the work is a chain of dependent arithmetic)
constexpr int kPackRows = 16;

// grid (chunks of all strips, ceil(kpad / 16)); 256 threads
template <int ADT, bool GEN>
__global__ __launch_bounds__(256) void k_lp_pack(const PackArgs a) {
    constexpr int KC = lp_kc(ADT);
    constexpr int R = lp_row(ADT);
    constexpr int CPS = kLpStrip / KC;
    __shared__ __attribute__((aligned(16))) uint16_t sh[2][kPackRows][R];
    const int tid = threadIdx.x;
    const int64_t gc = blockIdx.x;
    const int64_t strip = gc / CPS;
    const int c = (int)(gc - strip * CPS);
    int b = 0;
    int64_t sib = strip;
    for (; b < a.P; ++b) {
        const int64_t sb = (a.blk[b].n + kLpStrip - 1) / kLpStrip;
        if (sib < sb) break;
        sib -= sb;
    }
    const int64_t col_begin = sib * kLpStrip;
    const int w = (int)min<int64_t>(kLpStrip, a.blk[b].n - col_begin);
    if (c * KC >= w) return;                      // past the strip's end: never read
    const int kvalid = min(KC, w - c * KC);
    const int nb0 = blockIdx.y * kPackRows;
    const int kb = (int)min<int64_t>(kPackRows, a.k - nb0);   // <= 0: all zero
    static_assert((2 * kPackRows * R) % 8 == 0, "whole 16-byte pieces");
    for (int it = tid; it < 2 * kPackRows * R / 8; it += 256)
        reinterpret_cast<v4u*>(&sh[0][0][0])[it] = v4u{0u, 0u, 0u, 0u};
    __syncthreads();
    if constexpr (GEN) {
        const int64_t g0 = a.blk[b].row0 + col_begin + (int64_t)c * KC;
        const int64_t q_lo = g0 >> 2;
        const int nq = (int)(((g0 + KC - 1) >> 2) - q_lo + 1);
        const int items = kb > 0 ? nq * kb : 0;
        for (int it = tid; it < items; it += 256) {
            const int qi = it / kb;
            const int n = it - qi * kb;
            const float4 z = omega4_dist((uint64_t)(q_lo + qi), a.col0 + (uint32_t)(nb0 + n),
                                         a.key0, a.key1, a.dist);
            const int kl0 = (int)(4 * (q_lo + qi) - g0);
            const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kl = kl0 + u;
                if (kl >= 0 && kl < kvalid) split_bf16(zz[u], sh[0][n][kl], sh[1][n][kl]);
            }
        }
    } else {
        const int items = kb > 0 ? kvalid * kb : 0;
        for (int it = tid; it < items; it += 256) {
            const int kl = it / kb;
            const int n = it - kl * kb;
            split_bf16(a.omega[(col_begin + (int64_t)c * KC + kl) * a.ldo + nb0 + n],
                       sh[0][n][kl], sh[1][n][kl]);
        }
    }
    __syncthreads();
    const int rows = (int)min<int64_t>(kPackRows, a.kpad - nb0);
    const int pieces = rows * (KC / 8);           // 16-byte pieces per plane
    for (int it = tid; it < 2 * pieces; it += 256) {
        const int pl = it >= pieces;
        const int q = it - pl * pieces;
        const int n = q / (KC / 8);
        const int kl8 = (q - n * (KC / 8)) * 8;
        uint16_t* dst = static_cast<uint16_t*>(pl ? a.lo : a.hi) + ((gc * a.kpad + nb0 + n) * KC + kl8);
        *reinterpret_cast<v4u*>(dst) = *reinterpret_cast<const v4u*>(&sh[pl][n][kl8]);
    }
}

// FULL: whole chunks only, unconditional A loads (as in mfma_tile).
// PK: Omega chunks copied from the call's packed Omega (k_lp_pack) instead of
// generated or split here; the copy of chunk c + 2 is issued ahead of the A
// loads of chunk c + 2, so waiting for it leaves those in flight.
template <int NT, int ADT, int W, bool GEN, bool FULL = false, bool PK = false>
__device__ __forceinline__ void lp_tile(const MTile& t, uint16_t (*oh)[16 * NT][lp_row(ADT)],
                                        uint16_t (*ol)[16 * NT][lp_row(ADT)]) {
    constexpr int BN = 16 * NT;
    constexpr int TH = 64 * W;
    constexpr int KC = lp_kc(ADT);
    constexpr int KG = KC / 4;            // columns of a lane group per chunk
    constexpr int V = KC / 32;            // MFMA steps per chunk
    constexpr int es = ADT == 1 ? 2 : 1;
    constexpr int RW = 2;                 // 16-byte raw A words per lane and M-tile
    static_assert(KG * es == 16 * RW && kLpStrip % KC == 0, "chunk geometry");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = lane >> 4;
    const int i16 = lane & 15;

    const int w = (int)min<int64_t>(kLpStrip, t.n - t.col_begin);
    const int nchunks = (w + KC - 1) / KC;
    const int64_t row_base = t.block_row + wave * (kTM * 16);
    const int kb = (int)min<int64_t>(BN, t.k - t.n_base);

    // ---- A: lane (g, i) holds columns kc + KG g .. kc + KG g + KG - 1 of row i ------
    const int64_t ldab = t.lda * es;
    const unsigned char* arow[kTM];
#pragma unroll
    for (int tm = 0; tm < kTM; ++tm) {
        const int64_t r = min<int64_t>(row_base + tm * 16 + i16, t.m - 1);
        arow[tm] = t.A + r * ldab + (t.col_begin + KG * g) * es;
    }
    // raw A of a chunk, RW words per lane and M-tile; FP8 is widened to BF16
    // only when the chunk is consumed, so the loads stay in flight behind the
    // current chunk's MFMAs
    auto load_a = [&](v4u (*a)[RW], int c) {
        if constexpr (FULL) {
            const int cc = c < nchunks ? c : nchunks - 1;
#pragma unroll
            for (int tm = 0; tm < kTM; ++tm) {
                const unsigned char* p = arow[tm] + (int64_t)cc * KC * es;
#pragma unroll
                for (int v = 0; v < RW; ++v) a[tm][v] = *reinterpret_cast<const v4u*>(p + 16 * v);
            }
            return;
        }
        if (c >= nchunks) return;
        const int kl = c * KC + KG * g;
#pragma unroll
        for (int tm = 0; tm < kTM; ++tm) {
            const unsigned char* p = arow[tm] + (int64_t)c * KC * es;
            if (kl + KG - 1 < w) {
#pragma unroll
                for (int v = 0; v < RW; ++v) a[tm][v] = *reinterpret_cast<const v4u*>(p + 16 * v);
            } else {
                uint32_t wd[4 * RW];
#pragma unroll
                for (int q = 0; q < 4 * RW; ++q) wd[q] = 0u;
                for (int e = 0; e < KG; ++e) {
                    if (kl + e < w) {
                        const uint32_t v = ADT == 1 ? (uint32_t)reinterpret_cast<const uint16_t*>(p)[e]
                                                    : (uint32_t)p[e];
                        const int byte = e * es;
                        wd[byte >> 2] |= v << (8 * (byte & 3));
                    }
                }
#pragma unroll
                for (int v = 0; v < RW; ++v)
                    a[tm][v] = v4u{wd[4 * v], wd[4 * v + 1], wd[4 * v + 2], wd[4 * v + 3]};
            }
        }
    };
    // the 8-element BF16 operand of MFMA step v (columns KG g + 8v .. + 7 of the lane)
    auto operand = [&](const v4u* raw, int v) -> v4u {
        if constexpr (ADT == 1) {
            return raw[v];
        } else {
            const v4u r = raw[v >> 1];     // 16 FP8 = two steps per word
            const int q = 2 * (v & 1);
            uint32_t o[4];
            fp8x4_to_bf16<(NT > 1)>(r[q], o[0], o[1]);
            fp8x4_to_bf16<(NT > 1)>(r[q + 1], o[2], o[3]);
            return v4u{o[0], o[1], o[2], o[3]};
        }
    };

    // ---- Omega chunk -> LDS as (hi, lo) ------------------------------------------
    if constexpr (!PK) {
        for (int it = tid; it < 2 * BN * lp_row(ADT); it += TH) {
            const int n = (it / lp_row(ADT)) % BN;
            if (n >= kb) {
                (&oh[0][0][0])[it] = 0;
                (&ol[0][0][0])[it] = 0;
            }
        }
    }
    // packed route: 16-byte pieces of the tile's run of a chunk (both planes),
    // OPT per thread; chunk indices past the last are clamped (a re-read of
    // valid memory whose copy lands in the LDS buffer no step reads next)
    constexpr int PPL = BN * KC / 8;              // pieces per plane
    constexpr int OPT = (2 * PPL + TH - 1) / TH;
    auto om_load = [&](v4u* r, int c) {
        const int cc = c < nchunks ? c : nchunks - 1;
        const int64_t off = ((t.strip * (kLpStrip / KC) + cc) * t.kpad + t.n_base) * KC;
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int p = min(tid + j * TH, 2 * PPL - 1);
            const int pl = p >= PPL;
            const uint16_t* src = (pl ? t.opack_lo : t.opack) + off + (p - pl * PPL) * 8;
            r[j] = *reinterpret_cast<const v4u*>(src);
        }
    };
    auto om_store = [&](const v4u* r, int c) {
        const int buf = c & 1;
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int p = min(tid + j * TH, 2 * PPL - 1);
            const int pl = p >= PPL;
            const int q = p - pl * PPL;
            const int n = q / (KC / 8);
            const int kl8 = (q - n * (KC / 8)) * 8;
            *reinterpret_cast<v4u*>(pl ? &ol[buf][n][kl8] : &oh[buf][n][kl8]) = r[j];
        }
    };
    auto make_chunk = [&](int c) {
        const int buf = c & 1;
        const int kvalid = min(KC, w - c * KC);
        if constexpr (GEN) {
            const int64_t g0 = t.row0 + t.col_begin + (int64_t)c * KC;
            const int64_t q_lo = g0 >> 2;
            const int nq = (int)(((g0 + KC - 1) >> 2) - q_lo + 1);
            const int items = nq * kb;
            for (int it = tid; it < items; it += TH) {
                const int qi = it / kb;
                const int n = it - qi * kb;
                const float4 z = omega4_dist((uint64_t)(q_lo + qi), t.col0 + (uint32_t)(t.n_base + n),
                                             t.key0, t.key1, t.dist);
                const int kl0 = (int)(4 * (q_lo + qi) - g0);
                const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int kl = kl0 + u;
                    if (kl >= 0 && kl < KC) {
                        uint16_t h = 0, l = 0;
                        if (kl < kvalid) split_bf16(zz[u], h, l);
                        oh[buf][n][kl] = h;
                        ol[buf][n][kl] = l;
                    }
                }
            }
        } else {
            for (int it = tid; it < KC * kb; it += TH) {
                const int kl = it / kb;
                const int n = it - kl * kb;
                uint16_t h = 0, l = 0;
                if (kl < kvalid)
                    split_bf16(t.omega[(t.col_begin + (int64_t)c * KC + kl) * t.ldo + t.n_base + n],
                               h, l);
                oh[buf][n][kl] = h;
                ol[buf][n][kl] = l;
            }
        }
    };

    v4f acc[kTM][NT];
#pragma unroll
    for (int tm = 0; tm < kTM; ++tm)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[tm][nt] = v4f{0.f, 0.f, 0.f, 0.f};

    v4u a0[kTM][RW], a1[kTM][RW];
    v4u orr[PK ? OPT : 1];
    if constexpr (PK) {
        load_a(a0, 0);
        om_load(orr, 0);
        om_store(orr, 0);
        om_load(orr, 1);
        __builtin_amdgcn_sched_barrier(0);
        load_a(a1, 1);
    } else {
        load_a(a0, 0);
        load_a(a1, 1);
        make_chunk(0);
    }
    lds_barrier_m();

    auto compute = [&](v4u (*a)[RW], int c) {
        const int buf = c & 1;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            v4u op[kTM];
#pragma unroll
            for (int tm = 0; tm < kTM; ++tm) op[tm] = operand(a[tm], v);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const v4u bh = *reinterpret_cast<const v4u*>(&oh[buf][nt * 16 + i16][KG * g + 8 * v]);
                const v4u bl = *reinterpret_cast<const v4u*>(&ol[buf][nt * 16 + i16][KG * g + 8 * v]);
#pragma unroll
                for (int tm = 0; tm < kTM; ++tm) {
                    const v8bf av = __builtin_bit_cast(v8bf, op[tm]);
                    acc[tm][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        av, __builtin_bit_cast(v8bf, bh), acc[tm][nt], 0, 0, 0);
                    acc[tm][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        av, __builtin_bit_cast(v8bf, bl), acc[tm][nt], 0, 0, 0);
                }
            }
        }
    };

    if constexpr (PK) {
        // step c: chunk c + 1's Omega to LDS, chunk c + 2's Omega issued, chunk c's
        // MFMAs, chunk c + 2's A issued (the same summation order as below)
        for (int c = 0; c < nchunks; c += 2) {
            om_store(orr, c + 1);
            om_load(orr, c + 2);
            __builtin_amdgcn_sched_barrier(0);
            compute(a0, c);
            load_a(a0, c + 2);
            if constexpr (FULL) __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
            om_store(orr, c + 2);
            om_load(orr, c + 3);
            __builtin_amdgcn_sched_barrier(0);
            if (c + 1 < nchunks) compute(a1, c + 1);
            load_a(a1, c + 3);
            if constexpr (FULL) __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
        }
    } else if constexpr (FULL) {
        // the same order with every load issued (and kept ahead of the next chunk's work)
        for (int c = 0; c < nchunks; c += 2) {
            if (c + 1 < nchunks) make_chunk(c + 1);
            compute(a0, c);
            load_a(a0, c + 2);
            __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
            if (c + 2 < nchunks) make_chunk(c + 2);
            if (c + 1 < nchunks) compute(a1, c + 1);
            load_a(a1, c + 3);
            __builtin_amdgcn_sched_barrier(0);
            lds_barrier_m();
        }
    } else {
        for (int c = 0; c < nchunks; c += 2) {
            if (c + 1 < nchunks) make_chunk(c + 1);
            compute(a0, c);
            load_a(a0, c + 2);
            lds_barrier_m();
            if (c + 1 < nchunks) {
                if (c + 2 < nchunks) make_chunk(c + 2);
                compute(a1, c + 1);
                load_a(a1, c + 3);
                lds_barrier_m();
            }
        }
    }
    store_tile<NT>(t, acc, row_base, kb, g, i16);
}

// One call: one workgroup per (strip of any block, 64W-row tile, sketch-column
// block), in the XCD-grouped order of mfma_tile_id.
// One-N-tile, 4-wave workgroups are kept within 128 registers so that four of
// them share a compute unit (a 32768-row FP8 launch is exactly four per unit;
// with three, a quarter of the tiles run as a tail on an underfilled chip).
constexpr int lp_min_waves(int nt, int w) { return nt == 1 && w == 4 ? 4 : 1; }

// Omega from the call's packed copy with more than one N-tile; one N-tile
// generates (or splits) its chunks in the tile, as the 128 registers of its
// 4-wave workgroups hold no staging registers besides.
constexpr bool lp_packed(int nt) { return nt > 1; }

template <int NT, int ADT, int W, bool GEN, bool FULL>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(lp_min_waves(NT, W))))
void k_gemm_mfma_lp(const MArgs args) {
    __shared__ __attribute__((aligned(16))) uint16_t oh[2][16 * NT][lp_row(ADT)];
    __shared__ __attribute__((aligned(16))) uint16_t ol[2][16 * NT][lp_row(ADT)];
    TileId id;
    if (!mfma_tile_id<true>(args, id)) return;
    const int strip = id.strip;
    int b = 0;
    int64_t sib = strip;
    for (; b < args.P; ++b) {
        const int64_t sb = (args.blk[b].n + kLpStrip - 1) / kLpStrip;
        if (sib < sb) break;
        sib -= sb;
    }
    const BlockDesc& blk = args.blk[b];
    MTile t;
    t.A = static_cast<const unsigned char*>(blk.A);
    t.lda = blk.lda;
    t.n = blk.n;
    t.row0 = blk.row0;
    t.scales = blk.scales;
    t.m = args.m;
    t.k = args.k;
    t.col_begin = sib * kLpStrip;
    t.block_row = id.rtile * (64 * W);
    t.n_base = id.nb * 16 * NT;
    t.key0 = args.key0;
    t.key1 = args.key1;
    t.col0 = args.col0;
    t.dist = args.dist;
    t.omega = args.omega;
    t.ldo = args.ldo;
    t.Y = args.Y;
    t.ldy = args.ldy;
    t.y_f64 = args.y_f64;
    t.beta = args.beta;
    t.partials = args.partials;
    t.strip = strip;
    t.single = (args.S_total == 1);
    t.opack = args.opack;
    t.opack_lo = args.opack_lo;
    t.kpad = args.kpad;
    t.fpack = nullptr;
    lp_tile<NT, ADT, W, GEN, FULL, lp_packed(NT)>(t, oh, ol);
}

// Batch of requests of one class (serving); rows per tile = kLpBatchRows.
template <int NT, int ADT>
__global__ __launch_bounds__(64 * kLpBatchWaves) void k_gemm_mfma_lp_batch(const BatchArgs args) {
    __shared__ __attribute__((aligned(16))) uint16_t oh[2][16 * NT][lp_row(ADT)];
    __shared__ __attribute__((aligned(16))) uint16_t ol[2][16 * NT][lp_row(ADT)];
    const int64_t T8 = (args.total_tiles + 7) / 8;
    bool first = true;
    for (int64_t v = blockIdx.x; v < 8 * T8; v += gridDim.x) {   // gridDim.x is a multiple of 8
        const int64_t tt = (v % 8) * T8 + v / 8;
        if (tt >= args.total_tiles) continue;
        int q = 0;
        while (q + 1 < args.count && tt >= args.req[q + 1].tile_begin) ++q;
        const BatchReq& rq = args.req[q];
        const int64_t lt = tt - rq.tile_begin;
        const int64_t strip = lt % rq.strips;
        const int64_t rb = (lt / rq.strips) % rq.rowblocks;
        const int nb = (int)(lt / ((int64_t)rq.strips * rq.rowblocks));
        MTile t;
        t.A = static_cast<const unsigned char*>(rq.A);
        t.lda = rq.lda;
        t.n = rq.n;
        t.row0 = rq.row0;
        t.scales = rq.scales;
        t.m = rq.m;
        t.k = rq.k;
        t.col_begin = strip * kLpStrip;
        t.block_row = rb * kLpBatchRows;
        t.n_base = nb * 16 * NT;
        t.key0 = (uint32_t)rq.seed;
        t.key1 = (uint32_t)(rq.seed >> 32);
        t.col0 = rq.col0;
        t.dist = rq.dist;
        t.omega = nullptr;
        t.ldo = 0;
        t.Y = rq.Y;
        t.ldy = rq.ldy;
        t.y_f64 = rq.y_f64;
        t.beta = rq.beta;
        t.partials = rq.partials;
        t.strip = strip;
        t.single = (rq.strips == 1);
        t.opack = nullptr;
        t.opack_lo = nullptr;
        t.kpad = 0;
        t.fpack = nullptr;
        if (!first) lds_barrier_m();
        first = false;
        lp_tile<NT, ADT, kLpBatchWaves, true>(t, oh, ol);
    }
}

template <int NT, int ADT, int W, bool GEN>
hipError_t launch_lp(const MArgs& args, hipStream_t s) {
    MArgs a = args;
    a.nrt = (a.m + 64 * W - 1) / (64 * W);
    const dim3 grid = mfma_grid(a);
    // whole chunks: unconditional loads (one N-tile measured 5-8% slower with them: its
    // 4-wave, 128-register tiles already keep enough loads in flight)
    bool full = NT > 1;
    for (int b = 0; b < a.P; ++b) full = full && a.blk[b].n % lp_kc(ADT) == 0;
    if (full)
        hipLaunchKernelGGL((k_gemm_mfma_lp<NT, ADT, W, GEN, true>), grid, dim3(64 * W), 0, s, a);
    else
        hipLaunchKernelGGL((k_gemm_mfma_lp<NT, ADT, W, GEN, false>), grid, dim3(64 * W), 0, s, a);
    return hipGetLastError();
}

template <int NT, int ADT, bool GEN>
hipError_t dispatch_lp_w(int waves, const MArgs& a, hipStream_t s) {
    return waves == 4 ? launch_lp<NT, ADT, 4, GEN>(a, s) : launch_lp<NT, ADT, 8, GEN>(a, s);
}

// packed tiles do not look at GEN (the packing kernel did): one instantiation
template <int ADT>
hipError_t dispatch_lp(int nt, bool gen, int waves, const MArgs& a, hipStream_t s) {
    static_assert(!lp_packed(1) && lp_packed(2) && lp_packed(4), "routes below");
    switch (nt) {
    case 1: return gen ? dispatch_lp_w<1, ADT, true>(waves, a, s)
                       : dispatch_lp_w<1, ADT, false>(waves, a, s);
    case 2: return dispatch_lp_w<2, ADT, true>(waves, a, s);
    default: return dispatch_lp_w<4, ADT, true>(waves, a, s);
    }
}

template <int NT, bool GEN>
hipError_t launch_m(const MArgs& a, dim3 grid, hipStream_t s) {
    // packed tiles do not look at GEN (the packing kernel did): one instantiation
    constexpr bool G = mfma_packed(NT) || GEN;
    bool full = true;
    for (int b = 0; b < a.P; ++b) full = full && a.blk[b].n % chunk_cols(NT) == 0;
    if (full)
        hipLaunchKernelGGL((k_gemm_mfma<NT, G, true>), grid, dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_gemm_mfma<NT, G, false>), grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <bool GEN>
hipError_t dispatch_m(int nt, const MArgs& a, dim3 grid, hipStream_t s) {
    switch (nt) {
    case 1: return launch_m<1, GEN>(a, grid, s);
    case 2: return launch_m<2, GEN>(a, grid, s);
    case 4: return launch_m<4, GEN>(a, grid, s);
    default: return launch_m<8, GEN>(a, grid, s);
    }
}

}  // namespace

// N-tiles (of 16 sketch columns) per workgroup for a sketch of width k.
int mfma_ntiles(int64_t k) { return k <= 16 ? 1 : k <= 32 ? 2 : k <= 64 ? 4 : 8; }

namespace {

// workspace of a packed route: [strip partials (more than one strip)]
// [256-B aligned: the packed Omega planes]
size_t pack_offset(int64_t m, int64_t strips, int64_t k) {
    return (gemm_workspace_bytes(m, strips, k) + 255) / 256 * 256;
}

int64_t mfma_kpad(int64_t k) {
    const int64_t BN = 16 * mfma_ntiles(k);
    return (k + BN - 1) / BN * BN;
}

size_t f32_plane_elems(int64_t strips, int64_t k) {
    return (size_t)strips * (size_t)kMfmaStrip * (size_t)mfma_kpad(k);
}

}  // namespace

hipError_t launch_gemm_mfma(const GemmLaunch& g) {
    const int nt = mfma_ntiles(g.k);
    const int64_t BN = 16 * nt;
    const int64_t nblk = (g.k + BN - 1) / BN;
    int64_t S = 0;
    for (int b = 0; b < g.P; ++b) S += (g.blk[b].n + kMfmaStrip - 1) / kMfmaStrip;
    PackArgs pk{};
    if (mfma_packed(nt)) {
        pk.hi = static_cast<unsigned char*>(g.workspace) + pack_offset(g.m, S, g.k);
        pk.k = g.k;
        pk.kpad = mfma_kpad(g.k);
        pk.key0 = (uint32_t)g.seed;
        pk.key1 = (uint32_t)(g.seed >> 32);
        pk.col0 = g.col0;
        pk.dist = g.dist;
        pk.omega = g.omega;
        pk.ldo = g.ldo;
        pk.P = g.P;
        for (int b = 0; b < g.P; ++b) pk.blk[b] = g.blk[b];
    }
    MArgs a{};
    a.fpack = static_cast<const float*>(pk.hi);
    a.kpad = pk.kpad;
    a.m = g.m;
    a.k = g.k;
    a.ldy = g.ldy;
    a.ldo = g.ldo;
    a.omega = g.omega;
    a.Y = g.Y;
    a.partials = S > 1 ? static_cast<float*>(g.workspace) : nullptr;
    a.key0 = (uint32_t)g.seed;
    a.key1 = (uint32_t)(g.seed >> 32);
    a.col0 = g.col0;
    a.dist = g.dist;
    a.P = g.P;
    a.S_total = (int)S;
    a.y_f64 = g.y_f64;
    a.beta = g.beta;
    for (int b = 0; b < g.P; ++b) a.blk[b] = g.blk[b];
    a.nrt = (g.m + kBM - 1) / kBM;
    a.nblk = (int)nblk;
    const dim3 grid = mfma_grid(a);
    const TraceEvents& tr = g.trace;
    if (tr.begin) (void)hipEventRecord(tr.begin, g.stream);
    if (mfma_packed(nt)) {
        const dim3 pgrid((unsigned)(S * (kMfmaStrip / chunk_cols(nt)) / kF32PackChunks),
                         (unsigned)((pk.kpad + kF32PackRows - 1) / kF32PackRows));
        if (pk.omega)
            hipLaunchKernelGGL((k_f32_pack<false>), pgrid, dim3(256), 0, g.stream, pk);
        else
            hipLaunchKernelGGL((k_f32_pack<true>), pgrid, dim3(256), 0, g.stream, pk);
        const hipError_t pe = hipGetLastError();
        if (pe != hipSuccess) return pe;
    }
    hipError_t e = (g.omega == nullptr) ? dispatch_m<true>(nt, a, grid, g.stream)
                                        : dispatch_m<false>(nt, a, grid, g.stream);
    if (e != hipSuccess) return e;
    if (tr.mid) (void)hipEventRecord(tr.mid, g.stream);
    if (S > 1) e = launch_reduce_partials(a.partials, (int)S, g.m, g.k, g.Y, g.y_f64, g.ldy,
                                          g.beta, g.stream);
    if (tr.end) (void)hipEventRecord(tr.end, g.stream);
    return e;
}

namespace {

template <int NT>
hipError_t run_mfma_batch(const BatchArgs& a, int grid, hipStream_t s) {
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_mfma_batch<NT>, kThreads, 0) !=
            hipSuccess)
            n = 1;
        return n;
    }();
    grid = batch_grid(per_cu, a.total_tiles, grid);
    hipLaunchKernelGGL((k_gemm_mfma_batch<NT>), dim3((unsigned)grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_mfma_batch(const BatchArgs& a, int nt, int grid, hipStream_t s) {
    if (a.count == 0 || a.total_tiles == 0) return hipSuccess;
    hipError_t e;
    switch (nt) {
    case 1: e = run_mfma_batch<1>(a, grid, s); break;
    case 2: e = run_mfma_batch<2>(a, grid, s); break;
    case 4: e = run_mfma_batch<4>(a, grid, s); break;
    case 8: e = run_mfma_batch<8>(a, grid, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return launch_reduce_batch(a, s);
}

// Column-major A, k > 16: one pass over A for all sketch columns (strips of
// kMfmaStrip columns, FP32 partials [S][m][k], FP64 strip sums).  N-tiles per
// workgroup are halved while the launch has fewer tiles than compute units (a
// few-row A, e.g. the n x p factor of the Nystrom second product, where
// generating Omega is the work): each sketch column's sums are the same for
// any N-tile count (the chunk width stays the one of the row-major kernel for
// this k), only A is re-read per column block.
hipError_t launch_gemm_cm_mfma(const CmLaunch& g) {
    const int64_t S = (g.n + kMfmaStrip - 1) / kMfmaStrip;
    const bool skinny = g.m <= 64;
    const int64_t nrb = skinny ? 1 : (g.m + kBM - 1) / kBM;
    int nt = skinny ? 1 : mfma_ntiles(g.k);
    while (!skinny && nt > 1 && S * nrb * ((g.k + 16 * nt - 1) / (16 * nt)) < device_cus()) nt /= 2;
    const int64_t BN = 16 * nt;
    CmMArgs a{};
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
    a.S = (int)S;
    a.partials = a.S > 1 ? static_cast<float*>(g.workspace) : nullptr;
    a.num_rb = (int)nrb;
    a.tiles = (int64_t)a.S * a.num_rb * ((g.k + BN - 1) / BN);
    a.tiles8 = (a.tiles + 7) / 8;
    hipError_t e;
    constexpr int KCc = chunk_cols(8);
    if (skinny || cm_packed(nt, g.m % 4 == 0 && g.n % KCc == 0)) {
        // the call's Omega, once (the same plane as the row-major call's); the
        // few-row kernel copies it instead of generating in its workgroups
        PackArgs pk{};
        pk.hi = static_cast<unsigned char*>(g.workspace) + pack_offset(g.m, S, g.k);
        pk.k = g.k;
        pk.kpad = mfma_kpad(g.k);
        pk.key0 = a.key0;
        pk.key1 = a.key1;
        pk.col0 = a.col0;
        pk.dist = a.dist;
        pk.P = 1;
        pk.blk[0] = BlockDesc{g.A, g.n, g.lda, g.row0, nullptr};
        const dim3 pgrid((unsigned)(S * (kMfmaStrip / chunk_cols(nt)) / kF32PackChunks),
                         (unsigned)((pk.kpad + kF32PackRows - 1) / kF32PackRows));
        hipLaunchKernelGGL((k_f32_pack<true>), pgrid, dim3(256), 0, g.stream, pk);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        a.fpack = static_cast<const float*>(pk.hi);
        a.kpad = pk.kpad;
    }
    constexpr int KC = chunk_cols(8);
    static_assert(chunk_cols(1) == KC && chunk_cols(2) == KC && chunk_cols(4) == KC,
                  "one chunk width for every N-tile count of the row-major kernel");
    if (skinny) {
        if (g.m % 4 == 0)
            hipLaunchKernelGGL((k_gemm_cm_mfma_skinny<KC, true>), dim3((unsigned)a.tiles),
                               dim3(kSkThreads), 0, g.stream, a);
        else
            hipLaunchKernelGGL((k_gemm_cm_mfma_skinny<KC, false>), dim3((unsigned)a.tiles),
                               dim3(kSkThreads), 0, g.stream, a);
        e = hipGetLastError();
    } else switch (nt) {
    case 1: e = launch_cm_mfma_nt<1, KC>(a, g.stream); break;
    case 2: e = launch_cm_mfma_nt<2, KC>(a, g.stream); break;
    case 4: e = launch_cm_mfma_nt<4, KC>(a, g.stream); break;
    default: e = launch_cm_mfma_nt<8, KC>(a, g.stream); break;
    }
    if (e != hipSuccess || a.S == 1) return e;
    return launch_reduce_partials_t(a.partials, a.S, g.m, g.k, g.Y, g.y_f64, g.ldy, g.beta,
                                    g.y_trans, g.stream);
}

int lp_ntiles(int64_t k) { return k <= 16 ? 1 : k <= 32 ? 2 : 4; }

// Waves per workgroup of the low-precision kernel: 8 (512 rows share each
// Omega chunk), unless that leaves compute units without a tile.  Measured on
// 32768^2 with the XCD-grouped tile order: FP8 k = 5 199-201 us against 207-210
// with 4-wave workgroups, k = 64 299 against 375.  (Before that order, 4-wave
// workgroups had won at k = 5: 3.2 vs 2.6 TB/s.)
int lp_waves(int64_t m, int64_t strips, int64_t nblk, int nt) {
    (void)nt;
    const int64_t tiles8 = strips * ((m + 511) / 512) * nblk;
    return tiles8 >= device_cus() ? 8 : 4;
}

namespace {

int64_t lp_kpad(int64_t k) {
    const int64_t BN = 16 * lp_ntiles(k);
    return (k + BN - 1) / BN * BN;
}

// packed Omega after the partials (pack_offset): hi plane then lo plane,
// strips * kLpStrip * kpad BF16 values each
size_t lp_plane_elems(int64_t strips, int64_t k) {
    return (size_t)strips * (size_t)kLpStrip * (size_t)lp_kpad(k);
}

template <int ADT>
hipError_t launch_lp_pack(const PackArgs& p, int64_t strips, hipStream_t s) {
    const dim3 grid((unsigned)(strips * (kLpStrip / lp_kc(ADT))),
                    (unsigned)((p.kpad + kPackRows - 1) / kPackRows));
    if (p.omega)
        hipLaunchKernelGGL((k_lp_pack<ADT, false>), grid, dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL((k_lp_pack<ADT, true>), grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace

// column-major A: partials, and the packed Omega where a matrix-core kernel
// takes it: the few-row kernel (m <= 64) at every k > 16, the tile kernel at
// k > 32 (whose launch may still run fewer N-tiles and leave it unused)
size_t cm_workspace_bytes(int64_t m, int64_t n, int64_t k) {
    const int64_t S = cm_strips(n, k);
    if (k <= kColGroup) return gemm_workspace_bytes(m, S, k);
    if (m <= 64) return pack_offset(m, S, k) + f32_plane_elems(S, k) * sizeof(float);
    return product_workspace_bytes(0, m, S, k);
}

size_t product_workspace_bytes(int adtype, int64_t m, int64_t strips, int64_t k) {
    if (use_mfma(adtype, k) && mfma_packed(mfma_ntiles(k)))
        return pack_offset(m, strips, k) + f32_plane_elems(strips, k) * sizeof(float);
    if (use_mfma_lp(adtype, k) && lp_packed(lp_ntiles(k)))
        return pack_offset(m, strips, k) + 2 * lp_plane_elems(strips, k) * sizeof(uint16_t);
    return gemm_workspace_bytes(m, strips, k);
}

hipError_t launch_gemm_mfma_lp(const GemmLaunch& g) {
    const int nt = lp_ntiles(g.k);
    const int64_t BN = 16 * nt;
    const int64_t nblk = (g.k + BN - 1) / BN;
    int64_t S = 0;
    for (int b = 0; b < g.P; ++b) S += (g.blk[b].n + kLpStrip - 1) / kLpStrip;
    PackArgs pk{};
    if (lp_packed(nt)) {
        uint16_t* hi = reinterpret_cast<uint16_t*>(static_cast<unsigned char*>(g.workspace) +
                                                   pack_offset(g.m, S, g.k));
        pk.hi = hi;
        pk.lo = hi + lp_plane_elems(S, g.k);
    }
    pk.k = g.k;
    pk.kpad = lp_kpad(g.k);
    pk.key0 = (uint32_t)g.seed;
    pk.key1 = (uint32_t)(g.seed >> 32);
    pk.col0 = g.col0;
    pk.dist = g.dist;
    pk.omega = g.omega;
    pk.ldo = g.ldo;
    pk.P = g.P;
    for (int b = 0; b < g.P; ++b) pk.blk[b] = g.blk[b];
    MArgs a{};
    a.opack = static_cast<const uint16_t*>(pk.hi);
    a.opack_lo = static_cast<const uint16_t*>(pk.lo);
    a.kpad = pk.kpad;
    a.m = g.m;
    a.k = g.k;
    a.ldy = g.ldy;
    a.ldo = g.ldo;
    a.omega = g.omega;
    a.Y = g.Y;
    a.partials = S > 1 ? static_cast<float*>(g.workspace) : nullptr;
    a.key0 = (uint32_t)g.seed;
    a.key1 = (uint32_t)(g.seed >> 32);
    a.col0 = g.col0;
    a.dist = g.dist;
    a.P = g.P;
    a.S_total = (int)S;
    a.y_f64 = g.y_f64;
    a.beta = g.beta;
    for (int b = 0; b < g.P; ++b) a.blk[b] = g.blk[b];
    const int waves = lp_waves(g.m, S, nblk, nt);
    a.nblk = (int)nblk;
    const TraceEvents& tr = g.trace;
    if (tr.begin) (void)hipEventRecord(tr.begin, g.stream);
    hipError_t e = hipSuccess;
    if (lp_packed(nt)) {
        e = g.adtype == 1 ? launch_lp_pack<1>(pk, S, g.stream) : launch_lp_pack<2>(pk, S, g.stream);
        if (e != hipSuccess) return e;
    }
    const bool gen = (g.omega == nullptr);
    e = g.adtype == 1 ? dispatch_lp<1>(nt, gen, waves, a, g.stream)
                      : dispatch_lp<2>(nt, gen, waves, a, g.stream);
    if (e != hipSuccess) return e;
    if (tr.mid) (void)hipEventRecord(tr.mid, g.stream);
    if (S > 1) e = launch_reduce_partials(a.partials, (int)S, g.m, g.k, g.Y, g.y_f64, g.ldy,
                                          g.beta, g.stream);
    if (tr.end) (void)hipEventRecord(tr.end, g.stream);
    return e;
}

namespace {

template <int NT, int ADT>
hipError_t run_lp_batch(const BatchArgs& a, int grid, hipStream_t s) {
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_mfma_lp_batch<NT, ADT>,
                                                         64 * kLpBatchWaves, 0) != hipSuccess)
            n = 1;
        return n;
    }();
    grid = batch_grid(per_cu, a.total_tiles, grid);
    hipLaunchKernelGGL((k_gemm_mfma_lp_batch<NT, ADT>), dim3((unsigned)grid),
                       dim3(64 * kLpBatchWaves), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_mfma_lp_batch(const BatchArgs& a, int nt, int adtype, int grid,
                                     hipStream_t s) {
    if (a.count == 0 || a.total_tiles == 0) return hipSuccess;
    hipError_t e;
    if (adtype == 1) {
        e = nt == 1 ? run_lp_batch<1, 1>(a, grid, s) : nt == 2 ? run_lp_batch<2, 1>(a, grid, s)
                                                              : run_lp_batch<4, 1>(a, grid, s);
    } else {
        e = nt == 1 ? run_lp_batch<1, 2>(a, grid, s) : nt == 2 ? run_lp_batch<2, 2>(a, grid, s)
                                                              : run_lp_batch<4, 2>(a, grid, s);
    }
    if (e != hipSuccess) return e;
    return launch_reduce_batch(a, s);
}

}  // namespace sk
