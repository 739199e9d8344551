// LayerNorm, neighborhood index tables and the float64 error norm.
#include "kernels.hpp"

namespace wm {
namespace {

// One wave per RPW token rows; C = 64 * VPT.  Each lane holds VPT values of
// each row, read as float4 (or float2) chunks interleaved across the wave so
// every load instruction covers one contiguous span of a row; all rows'
// loads are issued before any arithmetic.  Statistics are float32 with a
// two-pass (mean, then centred squares) variance kept in registers.
// Input rows come from one buffer x or from per-state buffers xs
// (StateRows).
template <int VPT, bool OBF, int RPW>
__global__ __launch_bounds__(256) void layernorm_kernel(float *x, float *const *xs, unsigned T, UDiv dT,
                                                        const float *__restrict__ gamma,
                                                        const float *__restrict__ beta,
                                                        void *__restrict__ out, int M, float eps) {
    constexpr int C = VPT * 64;
    constexpr int W = VPT >= 4 ? 4 : VPT;     // vector width
    constexpr int NV = VPT / W;
    const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW;
    if (row0 >= M) return;
    const int lane = threadIdx.x & 63;
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
        const float var = wave_sum(q) * (1.0f / C);
        const float rstd = 1.0f / sqrtf(var + eps);
        if (row >= M) continue;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int base = (j * 64 + lane) * W;
            float y[W];
#pragma unroll
            // explicit FMA: the rounding must not depend on the row's slot in
            // the unrolled row loop (its position depends on the batch)
            for (int t = 0; t < W; ++t) y[t] = fmaf((v[r][W * j + t] - mean) * rstd, gamma[base + t], beta[base + t]);
            if constexpr (OBF) {
                bf16 *o = (bf16 *)out + (size_t)row * C + base;
                if constexpr (W == 4) {
                    uint2 u;
                    u.x = pack_bf16x2(y[0], y[1]);
                    u.y = pack_bf16x2(y[2], y[3]);
                    *(uint2 *)o = u;
                } else {
                    *(unsigned *)o = pack_bf16x2(y[0], y[1]);
                }
            } else {
                float *o = (float *)out + (size_t)row * C + base;
                if constexpr (W == 4) *(float4 *)o = make_float4(y[0], y[1], y[2], y[3]);
                else *(float2 *)o = make_float2(y[0], y[1]);
            }
        }
    }
}

template <int VPT>
hipError_t ln_launch(const StateRows &x, const float *g, const float *b, void *out, bool obf, int M, float eps,
                     hipStream_t s) {
    constexpr int RPW = 2;
    const int grid = (M + 4 * RPW - 1) / (4 * RPW);
    const UDiv dT = udiv_make(x.T);
    if (obf) layernorm_kernel<VPT, true, RPW><<<grid, 256, 0, s>>>(x.x, x.xs, x.T, dT, g, b, out, M, eps);
    else layernorm_kernel<VPT, false, RPW><<<grid, 256, 0, s>>>(x.x, x.xs, x.T, dT, g, b, out, M, eps);
    return hipGetLastError();
}

__global__ void set_ptrs_kernel(float **dst, PtrList ptrs, int n) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = ptrs.p[i];
}

__global__ void nat_indices_kernel(int Z, int Y, int X, int Kz, int Ky, int Kx, unsigned periodic,
                                   int *out) {
    const int n = Z + Y + X;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int pos, N, K;
    bool per;
    if (i < Z) { pos = i; N = Z; K = Kz; per = periodic & 1; }
    else if (i < Z + Y) { pos = i - Z; N = Y; K = Ky; per = (periodic >> 1) & 1; }
    else { pos = i - Z - Y; N = X; K = Kx; per = (periodic >> 2) & 1; }
    out[i] = win_start(pos, N, K, per);
    out[n + i] = win_bias0(pos, N, K, per);
}

__global__ __launch_bounds__(256) void relerr_kernel(const float *__restrict__ y, const double *__restrict__ r,
                                                     size_t n, double *acc) {
    double se = 0.0, sr = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double rv = r[i];
        const double d = (double)y[i] - rv;
        se += d * d;
        sr += rv * rv;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        se += __shfl_xor(se, o, 64);
        sr += __shfl_xor(sr, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(acc, se);
        atomicAdd(acc + 1, sr);
    }
}

// Element-wise float32 <-> bfloat16 copy (RNE on the way down).
template <bool SB, bool DB>
__global__ __launch_bounds__(256) void convert_kernel(const void *__restrict__ src, void *__restrict__ dst,
                                                      size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float v = SB ? bf2f(((const bf16 *)src)[i]) : ((const float *)src)[i];
        if (DB) ((bf16 *)dst)[i] = f2bf(v);
        else ((float *)dst)[i] = v;
    }
}

}  // namespace

hipError_t launch_convert(const void *src, bool src_bf16, void *dst, bool dst_bf16, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (src_bf16 && !dst_bf16) convert_kernel<true, false><<<(unsigned)blocks, 256, 0, stream>>>(src, dst, n);
    else if (!src_bf16 && dst_bf16) convert_kernel<false, true><<<(unsigned)blocks, 256, 0, stream>>>(src, dst, n);
    else if (src_bf16) convert_kernel<true, true><<<(unsigned)blocks, 256, 0, stream>>>(src, dst, n);
    else convert_kernel<false, false><<<(unsigned)blocks, 256, 0, stream>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_layernorm(const StateRows &x, const float *gamma, const float *beta, void *out, bool out_bf16,
                            int M, int C, float eps, hipStream_t stream) {
    if (M <= 0) return hipSuccess;
    if (x.xs && x.T == 0) return hipErrorInvalidValue;
    switch (C) {
    case 128: return ln_launch<2>(x, gamma, beta, out, out_bf16, M, eps, stream);
    case 256: return ln_launch<4>(x, gamma, beta, out, out_bf16, M, eps, stream);
    case 512: return ln_launch<8>(x, gamma, beta, out, out_bf16, M, eps, stream);
    case 1024: return ln_launch<16>(x, gamma, beta, out, out_bf16, M, eps, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_set_ptrs(float **dst, const PtrList &ptrs, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (n > 64) return hipErrorInvalidValue;
    set_ptrs_kernel<<<1, 64, 0, stream>>>(dst, ptrs, n);
    return hipGetLastError();
}

hipError_t launch_nat_indices(int Z, int Y, int X, int Kz, int Ky, int Kx, unsigned periodic, int *out,
                              hipStream_t stream) {
    const int n = Z + Y + X;
    nat_indices_kernel<<<(n + 255) / 256, 256, 0, stream>>>(Z, Y, X, Kz, Ky, Kx, periodic, out);
    return hipGetLastError();
}

hipError_t launch_relerr(const float *y, const double *r, size_t n, double *acc, hipStream_t stream) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    relerr_kernel<<<(unsigned)blocks, 256, 0, stream>>>(y, r, n, acc);
    return hipGetLastError();
}

}  // namespace wm
