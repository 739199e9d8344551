// Shared device-side types and helpers of libwm (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wm {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr float LOG2E = 1.4426950408889634f;

// float32 -> bfloat16 bits, round to nearest even (NaN kept quiet): the
// gfx950 conversion instruction (v_cvt_pk_bf16_f32) does exactly this.
__device__ __forceinline__ unsigned short f2bf_bits(float f) {
    return __builtin_bit_cast(unsigned short, (bf16)f);
}
// Two floats -> packed bfloat16 pair (lo in bits 0..15), one instruction.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16x2(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}
__device__ __forceinline__ float bf_bits2f(unsigned short b) {
    return __uint_as_float(((unsigned int)b) << 16);
}
__device__ __forceinline__ bf16 f2bf(float f) {
    unsigned short b = f2bf_bits(f);
    return __builtin_bit_cast(bf16, b);
}
__device__ __forceinline__ float bf2f(bf16 b) {
    return bf_bits2f(__builtin_bit_cast(unsigned short, b));
}

// s_waitcnt with vmcnt <= n and no wait on the other counters (gfx9 encoding:
// vmcnt bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Sum over the 4 lanes l, l^16, l^32, l^48 (in the MFMA layouts, the lanes
// that hold the same token or query); every one of them gets the same bits
// (same operand order).
__device__ __forceinline__ float xsum16_32(float v) {
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Four floats -> four OCP e4m3 codes (byte i = value i), round to nearest
// even, saturated at +-448 (the gfx950 conversion instruction rounds; the
// clamp keeps out-of-range values finite).
__device__ __forceinline__ unsigned e4m3x4(float a, float b, float c, float d) {
    const unsigned w = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(fminf(fmaxf(a, -448.0f), 448.0f),
                                                                  fminf(fmaxf(b, -448.0f), 448.0f), 0, false);
    return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(fminf(fmaxf(c, -448.0f), 448.0f),
                                                     fminf(fmaxf(d, -448.0f), 448.0f), (int)w, true);
}

// Loads/stores of element type T as float.
template <typename T> struct Elt;
template <> struct Elt<float> {
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, float v) { *p = v; }
};
template <> struct Elt<bf16> {
    static __device__ __forceinline__ float ld(const bf16 *p) { return bf2f(*p); }
    static __device__ __forceinline__ void st(bf16 *p, float v) { *p = f2bf(v); }
};

// Maximum of floats as one gfx950 v_maximum3_f32 / v_maximum_f32: unlike
// fmaxf it needs no NaN-quieting pass over its operands (a NaN operand
// propagates instead of being dropped).
__device__ __forceinline__ float max2f(float a, float b) { return __builtin_elementwise_maximum(a, b); }
__device__ __forceinline__ float max3f(float a, float b, float c) {
    return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c);
}

// Wave-wide reductions (64 lanes).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
    return v;
}

// GELU(z) = z * Phi(z) = z/2 * (1 + erf(z / sqrt 2)), with erf from the
// approximation of Abramowitz & Stegun, Handbook of Mathematical Functions,
// eq. 7.1.28 (Hastings): for x >= 0,
//   erf(x) = 1 - (1 + a1 x + a2 x^2 + ... + a6 x^6)^-16,  |error| <= 3e-7.
// With x = |z| / sqrt 2 and erf odd, both signs of z collapse to
//   GELU(z) = max(z, 0) - |z|/2 * (1 + a1 x + ... + a6 x^6)^-16,
// one reciprocal and no exponential (transcendentals issue at a quarter of
// the VALU rate); the 1/sqrt 2 powers are folded into the coefficients.
__device__ __forceinline__ float gelu_as(float z) {
    constexpr float r2 = 0.70710678118654752f;
    constexpr float c1 = 0.0705230784f * r2, c2 = 0.0422820123f * r2 * r2, c3 = 0.0092705272f * r2 * r2 * r2,
                    c4 = 0.0001520143f * r2 * r2 * r2 * r2, c5 = 0.0002765672f * r2 * r2 * r2 * r2 * r2,
                    c6 = 0.0000430638f * r2 * r2 * r2 * r2 * r2 * r2;
    const float az = fabsf(z);
    float p = fmaf(c6, az, c5);
    p = fmaf(p, az, c4);
    p = fmaf(p, az, c3);
    p = fmaf(p, az, c2);
    p = fmaf(p, az, c1);
    p = fmaf(p, az, 1.0f);
    float r = __builtin_amdgcn_rcpf(p);
    r *= r;    // ^2
    r *= r;    // ^4
    r *= r;    // ^8
    r *= r;    // ^16
    return fmaf(-0.5f * az, r, fmaxf(z, 0.0f));
}

// The same form with the shorter approximation of eq. 7.1.27: for x >= 0,
//   erf(x) = 1 - (1 + a1 x + a2 x^2 + a3 x^3 + a4 x^4)^-4,  |error| <= 5e-4,
// so GELU(z) = max(z, 0) - |z|/2 * (...)^-4 is within 2.5e-4 |z| of the
// exact GELU: below the rounding of a bf16 (or e4m3) output, at 4 FMAs and
// 2 multiplies instead of 6 and 4 -- the bf16 and e4m3 GEMM epilogues use it
// (the float32 path keeps 7.1.28).
__device__ __forceinline__ float gelu_as4(float z) {
    constexpr float r2 = 0.70710678118654752f;
    constexpr float c1 = 0.278393f * r2, c2 = 0.230389f * r2 * r2, c3 = 0.000972f * r2 * r2 * r2,
                    c4 = 0.078108f * r2 * r2 * r2 * r2;
    const float az = fabsf(z);
    float p = fmaf(c4, az, c3);
    p = fmaf(p, az, c2);
    p = fmaf(p, az, c1);
    p = fmaf(p, az, 1.0f);
    float r = __builtin_amdgcn_rcpf(p);
    r *= r;    // ^2
    r *= r;    // ^4
    return fmaf(-0.5f * az, r, fmaxf(z, 0.0f));
}

// ---------------------------------------------------------------------------
// Neighborhood windows (WeatherMesh-3 Sec. 2.1 NATTEN; App. A.2).  One axis
// of length n with odd window k, r = (k-1)/2.
//   clamped axis (lat, level): the window keeps k entries and shifts inward
//     at the borders: start = min(max(i-r, 0), n-k); keys start+t.
//   periodic axis (lon): keys (i-r+t) mod n.
// The bias-table index of key t is (key - query offset) + k - 1; on a
// periodic axis the offset is t - r.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int win_start(int i, int n, int k, bool periodic) {
    int r = (k - 1) >> 1;
    if (periodic) {
        int s = (i - r) % n;
        return s < 0 ? s + n : s;
    }
    int s = i - r;
    s = s < 0 ? 0 : s;
    return s > n - k ? n - k : s;
}
// Bias index of the first key (t = 0) of position i's window.
__host__ __device__ __forceinline__ int win_bias0(int i, int n, int k, bool periodic) {
    if (periodic) return k - 1 - ((k - 1) >> 1);          // offset -r  ->  -r + k - 1
    return win_start(i, n, k, false) - i + k - 1;
}

}  // namespace wm
