// Auxiliary kernels: raw Philox stream export, explicit Omega fill (the
// stored-operand alternative of Sec. 6.3), workspace zeroing, and the
// low-precision storage of A (bf16 / fp8 e4m3 with per-128-row scales).
#include "sk_device.hpp"
#include "sk_internal.hpp"

#pragma clang fp contract(off)

namespace sk {
namespace {

__global__ void k_philox_raw(const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint4 c = ctr[i];
    const Words4 r = philox4x32_10(Words4{c.x, c.y, c.z, c.w}, k0, k1);
    out[i] = make_uint4(r.x, r.y, r.z, r.w);
}

// The FP32 Box-Muller pair of each word pair, exactly as the generator forms
// it inside the product kernels.
__global__ void k_normal_raw(const uint2* words, float2* out, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint2 w = words[i];
    float zc, zs;
    box_muller(w.x, w.y, zc, zs);
    out[i] = make_float2(zc, zs);
}

// One thread per (Philox counter q, column c): writes Omega rows 4q..4q+3
// that fall inside [row0, row0+n).
__global__ void k_gen_omega(uint32_t k0, uint32_t k1, int dist, int64_t row0, int64_t n,
                            int64_t col0, int64_t k, float* Om, int64_t ldo, int64_t q_lo,
                            int64_t nq) {
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= nq * k) return;
    const int64_t qi = it / k;
    const int64_t c = it - qi * k;
    const int64_t q = q_lo + qi;
    const float4 z = omega4_dist((uint64_t)q, (uint32_t)(col0 + c), k0, k1, dist);
    const float zz[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t j = 4 * q + t - row0;
        if (j >= 0 && j < n) Om[j * ldo + c] = zz[t];
    }
}

// Synthetic N(0,1) matrix (load generation, not the sketch's operand): thread
// (i, q) writes columns 4q .. 4q+3 of row i from one Philox4x32-10 call on the
// counter (q, i, 0, 1) and two Box-Muller pairs evaluated with the hardware
// transcendentals (v_log_f32 = log2, v_sin_f32 / v_cos_f32 in revolutions,
// v_sqrt_f32): a few instructions per value, deterministic on the device.
__device__ __forceinline__ void fast_pair(uint32_t re, uint32_t ro, float& zc, float& zs) {
    const float ue = (float)(odd24(re)) * 0x1p-24f;   // (0, 1)
    const float uo = (float)(odd24(ro)) * 0x1p-24f;
    const float rho = __builtin_amdgcn_sqrtf(-2.0f * 0x1.62e430p-1f * __builtin_amdgcn_logf(ue));
    zc = rho * __builtin_amdgcn_cosf(uo);
    zs = rho * __builtin_amdgcn_sinf(uo);
}

__global__ void k_fill_normal(float* A, int64_t m, int64_t n, int64_t lda, uint32_t k0,
                              uint32_t k1) {
    const int64_t nq = (n + 3) >> 2;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < m * nq;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = it / nq;
        const int64_t q = it - i * nq;
        Words4 ctr{(uint32_t)q, (uint32_t)i, 0u, 1u};
        const Words4 r = philox4x32_10(ctr, k0, k1);
        float z[4];
        fast_pair(r.x, r.y, z[0], z[1]);
        fast_pair(r.z, r.w, z[2], z[3]);
        float* row = A + i * lda + 4 * q;
        if (4 * q + 3 < n && (lda & 3) == 0 && ((uintptr_t)A & 15) == 0) {
            *reinterpret_cast<float4*>(row) = make_float4(z[0], z[1], z[2], z[3]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * q + t < n) row[t] = z[t];
        }
    }
}

__global__ void k_zero(uint32_t* p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Y[0:m, 0:k] = 0 with leading dimension ldy: a grid-stride loop over the m*k
// elements, so any m fits the one-dimensional grid.
__global__ void k_zero_matrix(void* Y, int f64, int64_t m, int64_t k, int64_t ldy) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * k;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / k;
        const int64_t c = e - i * k;
        if (f64) static_cast<double*>(Y)[i * ldy + c] = 0.0;
        else static_cast<float*>(Y)[i * ldy + c] = 0.0f;
    }
}

__global__ void k_zero_bytes(unsigned char* p, int64_t bytes) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < bytes) p[i] = 0;
}

// bf16 = round-to-nearest-even of the upper half of the FP32 pattern.
__global__ void k_to_bf16(const float* A, int64_t m, int64_t n, int64_t lda, uint16_t* Q,
                          int64_t ldq) {
    const int64_t i = blockIdx.y;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = __float_as_uint(A[i * lda + j]);
        uint16_t h;
        if ((u & 0x7FFFFFFFu) > 0x7F800000u) h = (uint16_t)((u >> 16) | 0x40u);
        else h = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
        Q[i * ldq + j] = h;
    }
}

// max |A| of each 128-row block, as the FP32 bit pattern (monotone for
// non-negative values): block (x, b) scans rows [128b, 128b + 128) over a
// strided set of columns, reduces in registers, the wave and LDS, and issues
// one device-scope atomic max.
__global__ void k_amax_rows128(const float* A, int64_t m, int64_t n, int64_t lda, uint32_t* amax) {
    __shared__ uint32_t wmax[4];
    const int64_t b = blockIdx.y;
    const int64_t r_end = min<int64_t>(m, 128 * (b + 1));
    uint32_t mx = 0u;
    for (int64_t i = 128 * b; i < r_end; ++i)
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
             j += (int64_t)gridDim.x * blockDim.x)
            mx = max(mx, __float_as_uint(A[i * lda + j]) & 0x7FFFFFFFu);
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(&amax[b], max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3])));
}

// amax bits -> power-of-two scale 2^E, the smallest with amax <= 448 * 2^E
// among the powers of two an FP32 scale can hold (E >= -149, the smallest
// subnormal: a block whose amax is at most 448 * 2^-149 gets 2^-149).
__global__ void k_fp8_scales(uint32_t* s, int64_t nb) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const uint32_t bits = s[b];
    float scale = 1.0f;
    if (bits != 0u) {
        const float amax = __uint_as_float(bits);
        int E = -149;
        // 448 * 2^E (exact for E >= -149) doubles per step
        float lim = __builtin_ldexpf(448.0f, E);
        while (lim < amax) {
            ++E;
            lim = __builtin_ldexpf(448.0f, E);
        }
        scale = __builtin_ldexpf(1.0f, E);
    }
    reinterpret_cast<float*>(s)[b] = scale;
}

// E4M3FN code of x (|x| <= 448 after scaling), round to nearest even,
// saturating at +-448, from the FP32 bit pattern.
__device__ __forceinline__ uint8_t e4m3_code(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t sign = (u >> 24) & 0x80u;
    const float a = fabsf(x);
    if (!(a < 448.0f)) return (uint8_t)(sign | 0x7Eu);
    if (a < 0x1p-6f) {
        // subnormal grid, spacing 2^-9; code = M, and M = 8 is exactly 2^-6 (code 8)
        const uint32_t M = (uint32_t)__builtin_rintf(a * 512.0f);
        return (uint8_t)(sign | M);
    }
    const uint32_t ua = __float_as_uint(a);
    int ue = (int)((ua >> 23) & 0xFFu) - 127;          // -6 .. 8
    uint32_t mant = ua & 0x7FFFFFu;
    uint32_t m3 = mant >> 20;
    const uint32_t rem = mant & 0xFFFFFu;
    if (rem > 0x80000u || (rem == 0x80000u && (m3 & 1u))) ++m3;
    if (m3 == 8u) { m3 = 0u; ++ue; }
    uint32_t code = ((uint32_t)(ue + 7) << 3) | m3;
    if (code > 0x7Eu) code = 0x7Eu;
    return (uint8_t)(sign | code);
}

// Exponent E of a power-of-two scale 2^E, -149 <= E <= 127, read from its bits
// (normal: the biased exponent; subnormal: the position of its one set bit).
__device__ __forceinline__ int pow2_exponent(float s) {
    const uint32_t u = __float_as_uint(s);
    if (u >= 0x00800000u) return (int)(u >> 23) - 127;
    return (31 - __clz(u)) - 149;
}

// A / s_b as x * 2^-E: exact (the quotient is at most 448 in magnitude, and a
// result below FP32's normal range lies far under FP8's smallest step), with no
// reciprocal that could overflow for E <= -128.
__global__ void k_to_fp8(const float* A, int64_t m, int64_t n, int64_t lda, const float* scales,
                         uint8_t* Q, int64_t ldq) {
    const int64_t i = blockIdx.y;
    const int negE = -pow2_exponent(scales[i >> 7]);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        Q[i * ldq + j] = e4m3_code(__builtin_ldexpf(A[i * lda + j], negE));
}

}  // namespace

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const int64_t words = (int64_t)(bytes / 4);
    if (words) {
        const int64_t blocks = std::min<int64_t>((words + 255) / 256, 4096);
        hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<uint32_t*>(p), words);
    }
    const int64_t tail = (int64_t)(bytes - 4 * (size_t)words);
    if (tail)
        hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, s,
                           static_cast<unsigned char*>(p) + 4 * words, tail);
    return hipGetLastError();
}

hipError_t launch_zero_matrix(void* Y, int f64, int64_t m, int64_t k, int64_t ldy,
                              hipStream_t s) {
    if (m == 0 || k == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((m * k + 255) / 256, 16384);
    hipLaunchKernelGGL(k_zero_matrix, dim3((unsigned)blocks), dim3(256), 0, s, Y, f64, m, k, ldy);
    return hipGetLastError();
}

hipError_t launch_philox_raw(const uint32_t* ctr, uint64_t seed, uint32_t* out, int64_t N,
                             hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_raw, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(ctr), (uint32_t)seed,
                       (uint32_t)(seed >> 32), reinterpret_cast<uint4*>(out), N);
    return hipGetLastError();
}

hipError_t launch_normal_raw(const uint32_t* words, float* out, int64_t N, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_normal_raw, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint2*>(words), reinterpret_cast<float2*>(out), N);
    return hipGetLastError();
}

hipError_t launch_gen_omega(uint64_t seed, int dist, int64_t row0, int64_t n, int64_t col0,
                            int64_t k, float* Om, int64_t ldo, hipStream_t s) {
    if (n == 0 || k == 0) return hipSuccess;
    const int64_t q_lo = row0 >> 2;
    const int64_t nq = ((row0 + n - 1) >> 2) - q_lo + 1;
    const int64_t items = nq * k;
    hipLaunchKernelGGL(k_gen_omega, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s,
                       (uint32_t)seed, (uint32_t)(seed >> 32), dist, row0, n, col0, k, Om, ldo,
                       q_lo, nq);
    return hipGetLastError();
}

hipError_t launch_fill_normal(float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                              hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    const int64_t items = m * ((n + 3) >> 2);
    const unsigned blocks = (unsigned)std::min<int64_t>((items + 255) / 256, 8 * 1024);
    hipLaunchKernelGGL(k_fill_normal, dim3(blocks), dim3(256), 0, s, A, m, n, lda, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_quantize(const float* A, int64_t m, int64_t n, int64_t lda, int dst, void* Aq,
                           int64_t ldq, float* scales, hipStream_t s) {
    if (m == 0) return hipSuccess;
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 64));
    dim3 grid(gx, (unsigned)m);
    if (dst == 1) {
        if (n == 0) return hipSuccess;
        hipLaunchKernelGGL(k_to_bf16, grid, dim3(256), 0, s, A, m, n, lda,
                           static_cast<uint16_t*>(Aq), ldq);
        return hipGetLastError();
    }
    const int64_t nb = (m + 127) / 128;
    hipError_t e = launch_zero(scales, (size_t)nb * sizeof(float), s);
    if (e != hipSuccess) return e;
    if (n > 0) {
        const dim3 g2((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 64)),
                      (unsigned)nb);
        hipLaunchKernelGGL(k_amax_rows128, g2, dim3(256), 0, s, A, m, n, lda,
                           reinterpret_cast<uint32_t*>(scales));
    }
    hipLaunchKernelGGL(k_fp8_scales, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(scales), nb);
    if (n > 0)
        hipLaunchKernelGGL(k_to_fp8, grid, dim3(256), 0, s, A, m, n, lda, scales,
                           static_cast<uint8_t*>(Aq), ldq);
    return hipGetLastError();
}

}  // namespace sk
