// bf16 MFMA GEMM with a 3-stage LDS ring filled by direct buffer->LDS loads.
//
//   D[m][n] = sum_k A[m][k] * W[n][k]      (A: tokens x K, W: [out][in])
//
// Workgroup = 256 threads (4 waves, 2 x 2), tile BM x BN (128 x 128 by
// default: wave tile 64 x 64, 4 x 4 MFMA 16x16x32 tiles, 16 MFMA per
// 32-wide k-step against 8 fragment reads; 256 x 128 also built).  K
// advances in 64-element (128-byte) stages.
// A workgroup owns one token tile and walks several output-feature tiles;
// the stage stream runs on across tile boundaries, so the next tile's first
// loads are in flight while the previous tile's epilogue runs.
// Each stage is written straight from global memory into LDS by
// buffer_load_dwordx4 ... lds (no register staging), issued STAGES-1
// stages ahead; with two stages (64 KB) two workgroups share a CU and hide
// each other's load latency and epilogues.  Rows of
// A past M come back as zeros from the buffer range check, which handles
// the ragged last token tile.  LDS rows are 128 bytes; their 16-byte chunks
// are XOR-swizzled by (row >> 1) & 7 so the 16 rows a fragment read touches
// fall in distinct banks.  The MFMA "A" operand is the weight tile and "B"
// the activation tile, so every lane ends up with four consecutive output
// features of one token for the epilogue.  Tiles go out in an XCD-aware
// order (consecutive ids on one XCD share an activation tile in its L2).
#include <cstdlib>

#include "kernels.hpp"

namespace wm {
namespace glds {

constexpr int NT = 256;
constexpr int BK_BYTES = 128;

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int swz(int row) { return (row >> 1) & 7; }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, unsigned bytes) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(((unsigned long long)hi << 32) | lo), 0, bytes,
                                             0x00020000);
}

__device__ __forceinline__ void store4(float *p, f32x4 v) {
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(bf16 *p, f32x4 v) {
    uint2 u;
    u.x = (unsigned)f2bf_bits(v[0]) | ((unsigned)f2bf_bits(v[1]) << 16);
    u.y = (unsigned)f2bf_bits(v[2]) | ((unsigned)f2bf_bits(v[3]) << 16);
    *(uint2 *)p = u;
}

// Epilogue on four consecutive output features n..n+3 of token m.  For the
// QKV scatter, `qkv_base` is the element offset of (part, head 0, token 0)
// of the tile's part, `hc` the channel within the part and `qs` the Q scale
// (1 for K and V): all but hc are uniform over the tile.
template <int EPI>
__device__ __forceinline__ float epilogue4(const EpiArgs &ep, int M, int N, int m, int n, f32x4 v,
                                           size_t qkv_base, int hc, float qs, float dq) {
    if (m >= M) return 0.f;
    v[0] *= dq; v[1] *= dq; v[2] *= dq; v[3] *= dq;
    const float4 b = *(const float4 *)(ep.bias + n);
    v[0] += b.x; v[1] += b.y; v[2] += b.z; v[3] += b.w;
    if constexpr (EPI == EPI_QKV) {
        v[0] *= qs; v[1] *= qs; v[2] *= qs; v[3] *= qs;
        store4((bf16 *)ep.out + qkv_base + ((size_t)(hc >> 5) * M + m) * 32 + (hc & 31), v);
    } else if constexpr (EPI == EPI_GELU) {
        v[0] = gelu_as(v[0]); v[1] = gelu_as(v[1]); v[2] = gelu_as(v[2]); v[3] = gelu_as(v[3]);
        store4((bf16 *)ep.out + (size_t)m * N + n, v);
    } else if constexpr (EPI == EPI_RESID) {
        float *r = ep.resid + (size_t)m * N + n;
        float4 x = *(const float4 *)r;
        x.x += v[0]; x.y += v[1]; x.z += v[2]; x.w += v[3];
        *(float4 *)r = x;
    } else {
        store4((bf16 *)ep.out + (size_t)m * N + n, v);
    }
    return fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
}

// s_waitcnt with vmcnt <= n and no wait on the other counters (gfx9 encoding:
// vmcnt bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
}

// FP8: operands are e4m3 bytes (128 k-values per 128-byte stage, MFMA
// 16x16x32 fp8 with 8-byte fragments); the epilogue dequantizes per row.
template <int BM, int BN, int STAGES, int EPI, bool FP8>
__global__ __launch_bounds__(NT, (BM == 128 ? 2 : 1)) void gemm_lds_kernel(const void *__restrict__ A, const void *__restrict__ W,
                                                         int M, int N, int K, EpiArgs ep, int tpw) {
#if defined(__HIP_DEVICE_COMPILE__)   // LDS-address-space builtins exist only in the device pass
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int ROWS = BM + BN;                  // LDS rows per stage
    constexpr int STAGE_BYTES = ROWS * BK_BYTES;
    constexpr int LPW = ROWS / 8 / 4;              // load instructions per wave per stage
    static_assert(ROWS % 32 == 0 && BM % 32 == 0, "rows per stage must split over 4 waves x 8 rows");
    extern __shared__ __align__(16) unsigned char smem[];

    const int ntn = N / BN, ntm = (M + BM - 1) / BM;
    const int ngrp = (ntn + tpw - 1) / tpw, total = ngrp * ntm;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    const int tg = id % ngrp, tm = id / ngrp;
    const int m0 = tm * BM;
    const int tn0 = tg * tpw;
    const int nn = min(tpw, ntn - tn0);          // output-feature tiles of this workgroup

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int g = lane >> 4, r16 = lane & 15;
    const unsigned Kb = (unsigned)K * (FP8 ? 1 : 2);
    const __amdgpu_buffer_rsrc_t ars = make_rsrc(A, (unsigned)M * Kb);
    const __amdgpu_buffer_rsrc_t wrs = make_rsrc(W, (unsigned)N * Kb);

    // per-lane global byte offsets of this wave's load instructions
    // Instruction i of wave w fills LDS rows 8(w + 4i) .. +7; since BM is a
    // multiple of 32, rows below BM (activation rows) are exactly i < BM/32.
    unsigned voff[LPW];
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
        const int row = 8 * (wave + 4 * i) + (lane >> 3);
        const int lc = (lane & 7) ^ swz(row);
        voff[i] = i < BM / 32 ? (unsigned)(m0 + row) * Kb + lc * 16
                              : (unsigned)(tn0 * BN + row - BM) * Kb + lc * 16;
    }
    const int nk = K / (FP8 ? 128 : 64);
    // stage s of the stream = k-stage (s % nk) of feature tile (s / nk)
    auto issue = [&](int s, int stage) {
        const int t = s / nk, kt = s - t * nk;
        unsigned char *sbase = smem + stage * STAGE_BYTES;
        const unsigned wsoff = (unsigned)t * BN * Kb + kt * BK_BYTES;
#pragma unroll
        for (int i = 0; i < LPW; ++i) {
            lds_void *dst = (lds_void *)(sbase + 8 * (wave + 4 * i) * BK_BYTES);
            if (i < BM / 32)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ars, dst, 16, voff[i], kt * BK_BYTES, 0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(wrs, dst, 16, voff[i], wsoff, 0, 0);
        }
    };

    f32x4 acc[TN][TM];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};

    // lane-constant fragment offsets inside a stage (swizzle depends on r16
    // only): bf16 k-step ks reads 16 bytes at k = 32ks + 8g; fp8 k-step ks
    // reads 8 bytes at k = 32ks + 8g.
    constexpr int KSTEPS = FP8 ? 4 : 2;
    int aoff[KSTEPS], woff[KSTEPS];
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        const int pc = FP8 ? ((((2 * ks + (g >> 1)) ^ ((r16 >> 1) & 7)) << 4) + 8 * (g & 1))
                           : (((4 * ks + g) ^ ((r16 >> 1) & 7)) << 4);
        aoff[ks] = (wm * WM + r16) * BK_BYTES + pc;
        woff[ks] = (BM + wn * WN + r16) * BK_BYTES + pc;
    }

    const int S = nn * nk;
    constexpr int AHEAD = STAGES - 1;                // stages in flight ahead of the one in use
#pragma unroll
    for (int a = 0; a < AHEAD; ++a)
        if (a < S) issue(a, a);
    for (int t = 0; t < nn; ++t) {
        for (int kt = 0; kt < nk; ++kt) {
            const int st = t * nk + kt;
            // This wave's loads of stage st have landed once at most the LPW
            // loads of stage st + 1 are outstanding; the barrier then makes
            // all waves' parts of stage st visible and frees the stage read
            // in iteration st - 1.  (A bare s_barrier: __syncthreads() would
            // also drain the stage still in flight.)
            if constexpr (AHEAD == 2) {
                if (st + 1 < S) wait_vmcnt<LPW>();
                else wait_vmcnt<0>();
            } else {
                wait_vmcnt<0>();
            }
            __builtin_amdgcn_s_barrier();
            if (st + AHEAD < S) issue(st + AHEAD, (st + AHEAD) % STAGES);
            const unsigned char *sb = smem + (st % STAGES) * STAGE_BYTES;
#pragma unroll
            for (int ks = 0; ks < KSTEPS; ++ks) {
                if constexpr (FP8) {
                    long af[TM], wf[TN];
#pragma unroll
                    for (int i = 0; i < TM; ++i) af[i] = *(const long *)(sb + aoff[ks] + 16 * i * BK_BYTES);
#pragma unroll
                    for (int j = 0; j < TN; ++j) wf[j] = *(const long *)(sb + woff[ks] + 16 * j * BK_BYTES);
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int i = 0; i < TM; ++i)
                            acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(wf[j], af[i], acc[j][i], 0, 0, 0);
                } else {
                    bf16x8 af[TM], wf[TN];
#pragma unroll
                    for (int i = 0; i < TM; ++i) af[i] = *(const bf16x8 *)(sb + aoff[ks] + 16 * i * BK_BYTES);
#pragma unroll
                    for (int j = 0; j < TN; ++j) wf[j] = *(const bf16x8 *)(sb + woff[ks] + 16 * j * BK_BYTES);
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int i = 0; i < TM; ++i)
                            acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[j], af[i], acc[j][i], 0, 0, 0);
                }
            }
        }
        const int n0 = (tn0 + t) * BN;
        // a feature tile never straddles Q/K/V (C is a multiple of BN)
        const int part = EPI == EPI_QKV ? n0 / ep.C : 0;
        const size_t qkv_base = (size_t)part * ep.H * M * 32;
        const float qs = part == 0 ? ep.qscale : 1.0f;
        // per-row dequantization (fp8) and per-state amax of the outputs
        float dq[TM];
        int srow[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int m = min(m0 + wm * WM + 16 * i + r16, M - 1);
            srow[i] = FP8 || ep.out_amax ? (int)(m / ep.T) : 0;
            dq[i] = FP8 ? ep.a_amax[srow[i]] * (1.0f / 448.0f) * ep.w_dequant : 1.0f;
        }
        const int s_lo = ep.out_amax ? (int)(min(m0, M - 1) / ep.T) : 0;
        float mlo = 0.f, mhi = 0.f;
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int m = m0 + wm * WM + 16 * i + r16;
                const int n = n0 + wn * WN + 16 * j + 4 * g;
                const float a = epilogue4<EPI>(ep, M, N, m, n, acc[j][i], qkv_base, n - part * ep.C, qs, dq[i]);
                acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};
                if (ep.out_amax) {
                    if (srow[i] == s_lo) mlo = fmaxf(mlo, a);
                    else if (srow[i] == s_lo + 1) mhi = fmaxf(mhi, a);
                    else if (m < M)
                        atomicMax(ep.out_amax + (blockIdx.x % AMAX_SHARDS) * AMAX_STRIDE + srow[i] * ep.amax_stride + part,
                                  __float_as_uint(a));
                }
            }
        if (ep.out_amax) {
            mlo = wave_max(mlo);
            mhi = wave_max(mhi);
            if (lane == 0) {
                unsigned *sh = ep.out_amax + (blockIdx.x % AMAX_SHARDS) * AMAX_STRIDE;
                atomicMax(sh + s_lo * ep.amax_stride + part, __float_as_uint(mlo));
                if ((long)(s_lo + 1) * ep.T < M)
                    atomicMax(sh + (s_lo + 1) * ep.amax_stride + part, __float_as_uint(mhi));
            }
        }
    }
#endif
}

template <int BM, int BN, int STAGES, bool FP8>
hipError_t launch_cfg(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                      hipStream_t stream) {
    constexpr size_t lds = (size_t)STAGES * (BM + BN) * BK_BYTES;
    static bool attr_set = false;
    if (!attr_set) {
        const void *fns[4] = {(const void *)gemm_lds_kernel<BM, BN, STAGES, EPI_QKV, FP8>,
                              (const void *)gemm_lds_kernel<BM, BN, STAGES, EPI_GELU, FP8>,
                              (const void *)gemm_lds_kernel<BM, BN, STAGES, EPI_RESID, FP8>,
                              (const void *)gemm_lds_kernel<BM, BN, STAGES, EPI_STORE, FP8>};
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        attr_set = true;
    }
    const int ntn = N / BN;
    // Output-feature tiles per workgroup (WM_GEMM_TPW overrides, for tuning).
    static const int tpw_env = [] {
        const char *v = getenv("WM_GEMM_TPW");
        return v ? atoi(v) : 0;
    }();
    const int tpw = tpw_env > 0 ? (tpw_env < ntn ? tpw_env : ntn) : 1;
    const int total = ((ntn + tpw - 1) / tpw) * ((M + BM - 1) / BM);
    const int grid = ((total + 7) >> 3) << 3;
    const void *a = A;
    const void *w = W;
    switch (epi) {
    case EPI_QKV: gemm_lds_kernel<BM, BN, STAGES, EPI_QKV, FP8><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep, tpw); break;
    case EPI_GELU: gemm_lds_kernel<BM, BN, STAGES, EPI_GELU, FP8><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep, tpw); break;
    case EPI_RESID: gemm_lds_kernel<BM, BN, STAGES, EPI_RESID, FP8><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep, tpw); break;
    default: gemm_lds_kernel<BM, BN, STAGES, EPI_STORE, FP8><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep, tpw); break;
    }
    return hipGetLastError();
}

}  // namespace glds

using namespace glds;

bool gemm_lds_applies(int M, int N, int K) {
    return N % 128 == 0 && K % 64 == 0 && (unsigned long long)M * K * 2 < (1ull << 32) &&
           (unsigned long long)N * K * 2 < (1ull << 32);
}

hipError_t launch_gemm_lds(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                           hipStream_t stream) {
    // Default: 128x128 tiles, 2 stages (64 KB of LDS, two workgroups per CU,
    // so one's epilogue overlaps the other's MFMA work).  WM_GEMM_CFG=2
    // selects 256x128 tiles with 3 stages (one workgroup per CU), for tuning.
    static const int cfg = [] {
        const char *v = getenv("WM_GEMM_CFG");
        return v ? atoi(v) : 0;
    }();
    if (cfg == 2) return launch_cfg<256, 128, 3, false>(A, W, M, N, K, epi, ep, stream);
    return launch_cfg<128, 128, 2, false>(A, W, M, N, K, epi, ep, stream);
}

hipError_t launch_gemm_fp8(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                           hipStream_t stream) {
    if (M <= 0) return hipSuccess;
    if (N % 128 || K % 128 || (unsigned long long)M * K >= (1ull << 32)) return hipErrorInvalidValue;
    return launch_cfg<128, 128, 2, true>(A, W, M, N, K, epi, ep, stream);
}

}  // namespace wm
