// Device-side generator of the random operand Omega (gfx950).
//
// GenRandom of Alg. 1 as a pure function of (seed, global row, global
// column): the counter-based Philox4x32-10 generator (Sec. 6.3, Salmon et
// al. SC'11) followed by a Box-Muller transform to N(0,1).  The FP32
// operation sequence is fixed (fma-only series, correctly rounded division
// and square root, integer argument reduction) so every entry is
// reproducible bit for bit; FP contraction is disabled in this file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace sk {

struct Words4 {
    uint32_t x, y, z, w;
};

// Philox4x32-10: ten rounds of two 32x32->64 multiplies and xors; the key is
// advanced by the Weyl constants before rounds 2..10.
__device__ __forceinline__ Words4 philox4x32_10(Words4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        Words4 d;
        d.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        d.y = (uint32_t)p1;
        d.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        d.w = (uint32_t)p0;
        c = d;
    }
    return c;
}

// The 23 high bits x of a word as the odd integer 2x+1 < 2^24; the uniform
// variate is u = (2x+1) 2^-24, in (0, 1) and never 0 or 1.
__device__ __forceinline__ uint32_t odd24(uint32_t r) { return ((r >> 9) << 1) | 1u; }

// ln(mo 2^-24), mo odd in [1, 2^24): u = 2^e f with f in [sqrt(1/2), sqrt 2)
// found in integers; ln f = 2 atanh(w), w = (f-1)/(f+1), by the atanh series
// through w^10 (coefficients 1/(2i+1) rounded to FP32).
__device__ __forceinline__ float log_u24(uint32_t mo) {
    int b = 31 - __clz(mo);
    const uint64_t sq = (uint64_t)mo * (uint64_t)mo;
    if (sq >= (1ull << (2 * b + 1))) b += 1;
    const int e = b - 24;
    const float f = __builtin_ldexpf((float)mo, -b);
    const float s = f - 1.0f;
    const float d = f + 1.0f;
    const float w = __fdiv_rn(s, d);
    const float w2 = w * w;
    float p = 0x1.745d18p-4f;                  // 1/11
    p = __builtin_fmaf(p, w2, 0x1.c71c72p-4f);  // 1/9
    p = __builtin_fmaf(p, w2, 0x1.24924ap-3f);  // 1/7
    p = __builtin_fmaf(p, w2, 0x1.99999ap-3f);  // 1/5
    p = __builtin_fmaf(p, w2, 0x1.555556p-2f);  // 1/3
    p = __builtin_fmaf(p, w2, 1.0f);
    const float lnf = (w + w) * p;
    return __builtin_fmaf((float)e, 0x1.62e430p-1f, lnf);  // e ln2 + ln f
}

// (cos, sin) of 2 pi mo 2^-24: 4u = nq + f, nq nearest integer (found in
// integers; no ties since mo is odd), f in [-1/2, 1/2]; sin and cos of
// (pi/2) f by their Taylor series in f (through f^9 / f^10, coefficients
// (pi/2)^n / n! rounded to FP32), then rotated by the quadrant nq mod 4.
__device__ __forceinline__ void cos_sin_2pi_u24(uint32_t mo, float& c_out, float& s_out) {
    const uint32_t nq = (mo + (1u << 21)) >> 22;
    const int32_t fi = (int32_t)mo - (int32_t)(nq << 22);
    const float f = __builtin_ldexpf((float)fi, -22);
    const float f2 = f * f;
    float ps = 0x1.507834p-13f;
    ps = __builtin_fmaf(ps, f2, -0x1.32d2ccp-8f);
    ps = __builtin_fmaf(ps, f2, 0x1.466bc6p-4f);
    ps = __builtin_fmaf(ps, f2, -0x1.4abbcep-1f);
    ps = __builtin_fmaf(ps, f2, 0x1.921fb6p+0f);
    const float sn = ps * f;
    float pc = -0x1.a6d1f2p-16f;
    pc = __builtin_fmaf(pc, f2, 0x1.e1f506p-11f);
    pc = __builtin_fmaf(pc, f2, -0x1.55d3c8p-6f);
    pc = __builtin_fmaf(pc, f2, 0x1.03c1f0p-2f);
    pc = __builtin_fmaf(pc, f2, -0x1.3bd3ccp+0f);
    const float cs = __builtin_fmaf(pc, f2, 1.0f);
    const uint32_t quad = nq & 3u;
    const float a = (quad & 1u) ? sn : cs;   // |cos| of the rotated angle
    const float bb = (quad & 1u) ? cs : sn;  // |sin| of the rotated angle
    c_out = (quad == 1u || quad == 2u) ? -a : a;
    s_out = (quad >= 2u) ? -bb : bb;
}

// Correctly rounded square root of a positive normal x.  The hardware
// estimate s is within one ulp of sqrt(x), so the rounded root is s or one of
// its neighbours s- and s+.  x - s+- * s is formed exactly by an fma before
// its single rounding, so its sign is exact: x <= s- * s means sqrt(x) lies
// below the midpoint of s- and s (the product differs from the squared
// midpoint by a quarter ulp^2, finer than the spacing of x and of the
// products themselves), and x > s+ * s means it lies above the midpoint of s
// and s+.
__device__ __forceinline__ float sqrt_rn(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);
    const float s_dn = __uint_as_float(__float_as_uint(s) - 1u);
    const float s_up = __uint_as_float(__float_as_uint(s) + 1u);
    const float r_dn = __builtin_fmaf(-s_dn, s, x);
    const float r_up = __builtin_fmaf(-s_up, s, x);
    float r = s;
    if (r_dn <= 0.0f) r = s_dn;
    if (r_up > 0.0f) r = s_up;
    return r;
}

// Box-Muller on one word pair: (rho cos theta, rho sin theta) with
// rho = sqrt(-2 ln u_even), theta = 2 pi u_odd.
__device__ __forceinline__ void box_muller(uint32_t r_even, uint32_t r_odd, float& z_cos,
                                           float& z_sin) {
    const float L = log_u24(odd24(r_even));
    const float rho = sqrt_rn(-2.0f * L);  // -2L in [2^-23.9, 33.3]: normal
    float c, s;
    cos_sin_2pi_u24(odd24(r_odd), c, s);
    z_cos = rho * c;
    z_sin = rho * s;
}

// Omega rows 4q .. 4q+3 of global column c, from one Philox call.
__device__ __forceinline__ float4 omega4(uint64_t q, uint32_t c, uint32_t k0, uint32_t k1) {
    Words4 ctr{(uint32_t)q, (uint32_t)(q >> 32), c, 0u};
    const Words4 r = philox4x32_10(ctr, k0, k1);
    float4 z;
    box_muller(r.x, r.y, z.x, z.y);
    box_muller(r.z, r.w, z.z, z.w);
    return z;
}

// Omega entries under another distribution (dist 1: the uniform of each
// word, exact in FP32; dist 2: Rademacher, +1 when the word's top bit is 0);
// dist 0 is the normal of omega4.  dist is uniform across a launch.
__device__ __forceinline__ float4 omega4_dist(uint64_t q, uint32_t c, uint32_t k0, uint32_t k1,
                                              int dist) {
    if (dist == 0) return omega4(q, c, k0, k1);
    Words4 ctr{(uint32_t)q, (uint32_t)(q >> 32), c, 0u};
    const Words4 r = philox4x32_10(ctr, k0, k1);
    if (dist == 1)
        return make_float4((float)odd24(r.x) * 0x1p-24f, (float)odd24(r.y) * 0x1p-24f,
                           (float)odd24(r.z) * 0x1p-24f, (float)odd24(r.w) * 0x1p-24f);
    return make_float4((r.x >> 31) ? -1.0f : 1.0f, (r.y >> 31) ? -1.0f : 1.0f,
                       (r.z >> 31) ? -1.0f : 1.0f, (r.w >> 31) ? -1.0f : 1.0f);
}

}  // namespace sk
