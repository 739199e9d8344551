// FP8 (OCP e4m3, max 448) quantization for the FP8 processor precision.
//
// A tensor quantized per state uses the dequantization scale
//   s = amax / 448   (amax = max |value| over the state's tokens),
// and codes q = RNE(clamp(value * (448 / amax), -448, 448)).  amax values
// are kept as float bits and combined with unsigned atomicMax (|v| >= 0, so
// the bit patterns order like the values).  Producers spread their atomics
// over AMAX_SHARDS copies of each slot (shard = workgroup id mod shards);
// amax_fold then reduces the copies into shard 0, which consumers read.
#include "kernels.hpp"

namespace wm {
namespace {

__device__ __forceinline__ float clamp448(float v) { return fminf(fmaxf(v, -448.0f), 448.0f); }

__device__ __forceinline__ float inv_scale(float amax) { return amax > 0.f ? 448.0f / amax : 1.0f; }

// Fold the shard copies of n amax slots into shard 0.
__global__ void amax_fold_kernel(unsigned *amax, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned m = 0;
    for (int s = 0; s < AMAX_SHARDS; ++s) m = max(m, amax[s * AMAX_STRIDE + i]);
    amax[i] = m;
}

// LayerNorm, then e4m3 codes with one static scale amax/448 for every row
// (`amax`: a device float).  The layout of layernorm_kernel: RPW rows per
// wave, each lane W consecutive channels per chunk (16-byte loads), so a
// lane stores its W codes at once.
template <int VPT, int RPW>
__global__ __launch_bounds__(256) void ln8_kernel(float *x, float *const *xs, unsigned T, UDiv dT,
                                                  const float *__restrict__ gamma,
                                                  const float *__restrict__ beta, int M, float eps,
                                                  const float *__restrict__ amax, unsigned char *__restrict__ out) {
    constexpr int C = VPT * 64;
    constexpr int W = VPT >= 4 ? 4 : VPT;     // channels per lane and chunk
    constexpr int NV = VPT / W;
    const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW;
    if (row0 >= M) return;
    const int lane = threadIdx.x & 63;
    const float inv = inv_scale(*amax);
    float v[RPW][VPT];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const float *xr = state_row(x, xs, T, dT, (unsigned)min(row0 + r, M - 1), C);
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int base = (j * 64 + lane) * W;
            if constexpr (W == 4) {
                const float4 t = *(const float4 *)(xr + base);
                v[r][4 * j] = t.x; v[r][4 * j + 1] = t.y; v[r][4 * j + 2] = t.z; v[r][4 * j + 3] = t.w;
            } else {
                const float2 t = *(const float2 *)(xr + base);
                v[r][2 * j] = t.x; v[r][2 * j + 1] = t.y;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int row = row0 + r;
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < VPT; ++i) s += v[r][i];
        const float mean = wave_sum(s) * (1.0f / C);
        float q = 0.f;
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const float d = v[r][i] - mean;
            q = fmaf(d, d, q);
        }
        const float rstd = 1.0f / sqrtf(wave_sum(q) * (1.0f / C) + eps);
        if (row >= M) continue;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int base = (j * 64 + lane) * W;
            float y[W];
            // explicit FMA: the rounding must not depend on the row's slot in
            // the unrolled row loop (its position depends on the batch)
#pragma unroll
            for (int t = 0; t < W; ++t) y[t] = fmaf((v[r][W * j + t] - mean) * rstd, gamma[base + t], beta[base + t]) * inv;
            unsigned char *o = out + (size_t)row * C + base;
            const unsigned w = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(clamp448(y[0]), clamp448(y[1]), 0, false);
            if constexpr (W == 4)
                *(unsigned *)o = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(clamp448(y[2]), clamp448(y[3]), (int)w, true);
            else
                *(unsigned short *)o = (unsigned short)(w & 0xffffu);
        }
    }
}

// float32 -> e4m3 with one given multiplier (codes = RNE(clamp(x * mul))).
__global__ __launch_bounds__(256) void quant_f32_kernel(const float *__restrict__ in, size_t n, float mul,
                                                        unsigned char *__restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const unsigned w = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(clamp448(in[i] * mul), 0.f, 0, false);
        out[i] = (unsigned char)(w & 0xff);
    }
}

// amax over each state's bf16 elements (8 per lane per step).
__global__ __launch_bounds__(256) void amax_bf16_kernel(const unsigned short *__restrict__ x, size_t per_state,
                                                        unsigned *__restrict__ amax, int amax_stride) {
    const int b = blockIdx.y;
    const unsigned short *xs = x + (size_t)b * per_state;
    float m = 0.f;
    const size_t n8 = per_state / 8;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n8; i += (size_t)gridDim.x * 256) {
        const uint4 u = *(const uint4 *)(xs + 8 * i);
        const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            m = fmaxf(m, fmaxf(fabsf(__uint_as_float(w[q] << 16)), fabsf(__uint_as_float(w[q] & 0xffff0000u))));
    }
    for (size_t i = n8 * 8 + (size_t)blockIdx.x * 256 + threadIdx.x; i < per_state; i += (size_t)gridDim.x * 256)
        m = fmaxf(m, fabsf(__uint_as_float((unsigned)xs[i] << 16)));
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0)
        atomicMax(amax + (blockIdx.x % AMAX_SHARDS) * AMAX_STRIDE + b * amax_stride, __float_as_uint(m));
}

__global__ void zero_u32_kernel(unsigned *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

template <int VPT>
hipError_t ln_fp8_static(const StateRows &x, const float *g, const float *b, int M, float eps, const float *amax,
                         unsigned char *out, hipStream_t s) {
    constexpr int RPW = 2;
    ln8_kernel<VPT, RPW><<<(M + 4 * RPW - 1) / (4 * RPW), 256, 0, s>>>(x.x, x.xs, x.T, udiv_make(x.T), g, b, M, eps,
                                                                      amax, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_layernorm_fp8_static(const StateRows &x, const float *gamma, const float *beta, int M, int C,
                                       float eps, const float *amax, unsigned char *out, hipStream_t stream) {
    if (M <= 0) return hipSuccess;
    if (x.xs && x.T == 0) return hipErrorInvalidValue;
    switch (C) {
    case 128: return ln_fp8_static<2>(x, gamma, beta, M, eps, amax, out, stream);
    case 256: return ln_fp8_static<4>(x, gamma, beta, M, eps, amax, out, stream);
    case 512: return ln_fp8_static<8>(x, gamma, beta, M, eps, amax, out, stream);
    case 1024: return ln_fp8_static<16>(x, gamma, beta, M, eps, amax, out, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_amax_bf16(const void *x, size_t per_state, int B, unsigned *amax, int amax_stride,
                            hipStream_t stream) {
    if (B <= 0 || per_state == 0) return hipSuccess;
    size_t bx = (per_state / 8 + 255) / 256;
    if (bx > 1024) bx = 1024;
    if (bx == 0) bx = 1;
    amax_bf16_kernel<<<dim3((unsigned)bx, (unsigned)B), 256, 0, stream>>>((const unsigned short *)x, per_state, amax,
                                                                         amax_stride);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned *p, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    zero_u32_kernel<<<(unsigned)blocks, 256, 0, stream>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_amax_fold(unsigned *amax, int n, hipStream_t stream) {
    amax_fold_kernel<<<(n + 255) / 256, 256, 0, stream>>>(amax, n);
    return hipGetLastError();
}

hipError_t launch_quant_f32(const float *in, size_t n, float mul, unsigned char *out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    quant_f32_kernel<<<(unsigned)blocks, 256, 0, stream>>>(in, n, mul, out);
    return hipGetLastError();
}

}  // namespace wm
