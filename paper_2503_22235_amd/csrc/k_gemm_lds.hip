// bf16 MFMA GEMM with a 3-stage LDS ring filled by direct buffer->LDS loads.
//
//   D[m][n] = sum_k A[m][k] * W[n][k]      (A: tokens x K, W: [out][in])
//
// Workgroup = 256 threads (4 waves, 2 x 2), tile BM x BN = 256 x 128, wave
// tile 128 x 64 (8 x 4 MFMA 16x16x32 tiles; 32 MFMA per 32-wide k-step
// against 12 fragment reads).  K advances in 64-element (128-byte) stages.
// Each stage is written straight from global memory into LDS by
// buffer_load_dwordx4 ... lds (no register staging), issued two stages
// ahead, so a load has two stages of MFMA work (~1.7 us) to land.  Rows of
// A past M come back as zeros from the buffer range check, which handles
// the ragged last token tile.  LDS rows are 128 bytes; their 16-byte chunks
// are XOR-swizzled by (row >> 1) & 7 so the 16 rows a fragment read touches
// fall in distinct banks.  The MFMA "A" operand is the weight tile and "B"
// the activation tile, so every lane ends up with four consecutive output
// features of one token for the epilogue.  Tiles go out in an XCD-aware
// order (consecutive ids on one XCD share an activation tile in its L2).
#include "kernels.hpp"

namespace wm {
namespace glds {

constexpr int NT = 256;
constexpr int BK_BYTES = 128;
constexpr int STAGES = 3;

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

template <int EPI>
__device__ __forceinline__ void epilogue4(const EpiArgs &ep, int M, int N, int m, int n, f32x4 v) {
    if (m >= M) return;
    const float4 b = *(const float4 *)(ep.bias + n);
    v[0] += b.x; v[1] += b.y; v[2] += b.z; v[3] += b.w;
    if constexpr (EPI == EPI_QKV) {
        const int part = n / ep.C;
        const int hc = n - part * ep.C;
        const int h = hc >> 5, e = hc & 31;
        if (part == 0) { v[0] *= ep.qscale; v[1] *= ep.qscale; v[2] *= ep.qscale; v[3] *= ep.qscale; }
        store4((bf16 *)ep.out + (((size_t)(part * ep.H + h) * M + m) * 32 + e), v);
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
}

// s_waitcnt with vmcnt <= n and no wait on the other counters (gfx9 encoding:
// vmcnt bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int BM, int BN, int EPI>
__global__ __launch_bounds__(NT, 1) void gemm_lds_kernel(const bf16 *__restrict__ A, const bf16 *__restrict__ W,
                                                         int M, int N, int K, EpiArgs ep) {
#if defined(__HIP_DEVICE_COMPILE__)   // LDS-address-space builtins exist only in the device pass
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int ROWS = BM + BN;                  // LDS rows per stage
    constexpr int STAGE_BYTES = ROWS * BK_BYTES;
    constexpr int LPW = ROWS / 8 / 4;              // load instructions per wave per stage
    static_assert(ROWS % 32 == 0 && BM % 32 == 0, "rows per stage must split over 4 waves x 8 rows");
    extern __shared__ __align__(16) unsigned char smem[];

    const int ntn = N / BN, ntm = (M + BM - 1) / BM, total = ntn * ntm;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    const int tn = id % ntn, tm = id / ntn;
    const int m0 = tm * BM, n0 = tn * BN;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int g = lane >> 4, r16 = lane & 15;
    const unsigned Kb = (unsigned)K * 2;
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
        voff[i] = i < BM / 32 ? (unsigned)(m0 + row) * Kb + lc * 16 : (unsigned)(n0 + row - BM) * Kb + lc * 16;
    }
    auto issue = [&](int kt, int stage) {
        unsigned char *sbase = smem + stage * STAGE_BYTES;
#pragma unroll
        for (int i = 0; i < LPW; ++i) {
            lds_void *dst = (lds_void *)(sbase + 8 * (wave + 4 * i) * BK_BYTES);
            if (i < BM / 32)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ars, dst, 16, voff[i], kt * BK_BYTES, 0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(wrs, dst, 16, voff[i], kt * BK_BYTES, 0, 0);
        }
    };

    f32x4 acc[TN][TM];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};

    // lane-constant fragment offsets inside a stage (swizzle depends on r16 only)
    int aoff[2], woff[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int pc = ((4 * ks + g) ^ ((r16 >> 1) & 7)) << 4;
        aoff[ks] = (wm * WM + r16) * BK_BYTES + pc;
        woff[ks] = (BM + wn * WN + r16) * BK_BYTES + pc;
    }

    const int nk = K / 64;
    issue(0, 0);
    if (nk > 1) issue(1, 1);
    for (int kt = 0; kt < nk; ++kt) {
        // This wave's loads of stage kt have landed once at most the LPW
        // loads of stage kt + 1 are outstanding; the barrier then makes all
        // waves' parts of stage kt visible and frees the stage read in
        // iteration kt - 1.  (A bare s_barrier: __syncthreads() would also
        // drain the stage still in flight.)
        if (kt + 1 < nk) wait_vmcnt<LPW>();
        else wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        if (kt + 2 < nk) issue(kt + 2, (kt + 2) % STAGES);
        const unsigned char *sb = smem + (kt % STAGES) * STAGE_BYTES;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
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

#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int m = m0 + wm * WM + 16 * i + r16;
            const int n = n0 + wn * WN + 16 * j + 4 * g;
            epilogue4<EPI>(ep, M, N, m, n, acc[j][i]);
        }
#endif
}

template <int BM, int BN>
hipError_t launch_cfg(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                      hipStream_t stream) {
    constexpr size_t lds = (size_t)STAGES * (BM + BN) * BK_BYTES;
    static bool attr_set = false;
    if (!attr_set) {
        const void *fns[4] = {(const void *)gemm_lds_kernel<BM, BN, EPI_QKV>,
                              (const void *)gemm_lds_kernel<BM, BN, EPI_GELU>,
                              (const void *)gemm_lds_kernel<BM, BN, EPI_RESID>,
                              (const void *)gemm_lds_kernel<BM, BN, EPI_STORE>};
        for (const void *f : fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        attr_set = true;
    }
    const int total = (N / BN) * ((M + BM - 1) / BM);
    const int grid = ((total + 7) >> 3) << 3;
    const bf16 *a = (const bf16 *)A;
    const bf16 *w = (const bf16 *)W;
    switch (epi) {
    case EPI_QKV: gemm_lds_kernel<BM, BN, EPI_QKV><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep); break;
    case EPI_GELU: gemm_lds_kernel<BM, BN, EPI_GELU><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep); break;
    case EPI_RESID: gemm_lds_kernel<BM, BN, EPI_RESID><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep); break;
    default: gemm_lds_kernel<BM, BN, EPI_STORE><<<grid, NT, lds, stream>>>(a, w, M, N, K, ep); break;
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
    return launch_cfg<256, 128>(A, W, M, N, K, epi, ep, stream);
}

}  // namespace wm
