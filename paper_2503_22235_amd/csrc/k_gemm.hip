// MFMA GEMM for the block's linear maps, with fused epilogues.
//
//   D[m][n] = sum_k A[m][k] * W[n][k]
//
// A is the activation (tokens x features, row-major), W the weight stored
// [out][in] (row-major, K contiguous).  The MFMA "A" operand is a W tile
// and the "B" operand an activation tile, so each lane ends up holding
// four consecutive output features of one token: stores and the float32
// residual update are then 8-16 contiguous bytes per lane.
//
// Workgroup: 256 threads = 4 waves in a 2x2 arrangement, tile BM x BN,
// K-tiles of 128 bytes per row (64 bf16 or 32 float32) staged through LDS,
// double-buffered, with the 16-byte chunks of each row XOR-swizzled so the
// per-lane 16-byte fragment reads of a wave spread over the banks.
// Tiles are handed out in an XCD-aware order: consecutive tile ids land on
// the same XCD (the hardware deals workgroups round-robin over the 8 XCDs),
// so the workgroups that share an activation tile share that XCD's L2.
#include "kernels.hpp"

namespace wm {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ int swz(int row) { return (row >> 1) & 7; }

__device__ __forceinline__ void store4(float *p, f32x4 v) {
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(bf16 *p, f32x4 v) {
    uint2 u;
    u.x = pack_bf16x2(v[0], v[1]);
    u.y = pack_bf16x2(v[2], v[3]);
    *(uint2 *)p = u;
}

// Epilogue on four consecutive output features n..n+3 of token m.
template <int EPI, typename TO>
__device__ __forceinline__ void epilogue4(const EpiArgs &ep, int M, int N, int m, int n, f32x4 v) {
    if (m >= M) return;
    const float4 b = *(const float4 *)(ep.bias + n);
    v[0] += b.x; v[1] += b.y; v[2] += b.z; v[3] += b.w;
    if constexpr (epi_qkv(EPI)) {
        const int part = ep.part0 + n / ep.C;
        const int hc = n - (part - ep.part0) * ep.C;
        const int h = hc >> 5, e = hc & 31;
        if (EPI == EPI_QKV_ROPE && part < 2) {
            float r[4] = {v[0], v[1], v[2], v[3]};
            rope_rotate(r, 4, e, m, ep);
            v[0] = r[0]; v[1] = r[1]; v[2] = r[2]; v[3] = r[3];
        }
        if (part == 0) { v[0] *= ep.qscale; v[1] *= ep.qscale; v[2] *= ep.qscale; v[3] *= ep.qscale; }
        TO *dst = (TO *)ep.out + (((size_t)(part * ep.H + h) * M + m) * 32 + e);
        store4(dst, v);
    } else if constexpr (EPI == EPI_GELU) {
        v[0] = gelu_as(v[0]); v[1] = gelu_as(v[1]); v[2] = gelu_as(v[2]); v[3] = gelu_as(v[3]);
        store4((TO *)ep.out + (size_t)m * N + n, v);
    } else if constexpr (EPI == EPI_RESID) {
        float *r = state_row(ep.resid, ep.resid_ptrs, (unsigned)ep.T, ep.dT, (unsigned)m, N) + n;
        float4 x = *(const float4 *)r;
        x.x += v[0]; x.y += v[1]; x.z += v[2]; x.w += v[3];
        *(float4 *)r = x;
    } else {
        store4((TO *)ep.out + (size_t)m * N + n, v);
    }
}

template <typename TA> struct KTile;
template <> struct KTile<bf16> { static constexpr int BK = 64; };
template <> struct KTile<float> { static constexpr int BK = 32; };

template <typename TA, int BM, int BN, int EPI>
__global__ __launch_bounds__(NT) void gemm_kernel(const TA *__restrict__ A, const TA *__restrict__ W,
                                                   int M, int N, int K, EpiArgs ep) {
    constexpr int BK = KTile<TA>::BK;
    constexpr int CPR = 8;                 // 16-byte chunks per 128-byte tile row
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int A_LD = BM * CPR / NT, W_LD = BN * CPR / NT;
    static_assert(A_LD >= 1 && W_LD >= 1, "tile too small");
    __shared__ uint4 sA[2][BM * CPR];
    __shared__ uint4 sW[2][BN * CPR];

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
    const int lc = tid & 7, lr = tid >> 3;

    const char *Ab = (const char *)A;
    const char *Wb = (const char *)W;
    const size_t rowbytes = (size_t)K * sizeof(TA);
    uint4 ra[A_LD], rw[W_LD];

    auto gload = [&](int kt) {
        const size_t kb = (size_t)kt * 128 + lc * 16;
#pragma unroll
        for (int i = 0; i < A_LD; ++i) {
            int gm = m0 + lr + 32 * i;
            gm = gm < M ? gm : M - 1;
            ra[i] = *(const uint4 *)(Ab + (size_t)gm * rowbytes + kb);
        }
#pragma unroll
        for (int i = 0; i < W_LD; ++i) {
            const int gn = n0 + lr + 32 * i;
            rw[i] = *(const uint4 *)(Wb + (size_t)gn * rowbytes + kb);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < A_LD; ++i) {
            const int row = lr + 32 * i;
            sA[buf][row * CPR + (lc ^ swz(row))] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < W_LD; ++i) {
            const int row = lr + 32 * i;
            sW[buf][row * CPR + (lc ^ swz(row))] = rw[i];
        }
    };

    f32x4 acc[TN][TM];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int nk = K / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
        if constexpr (sizeof(TA) == 2) {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int c = 4 * ks + g;
                bf16x8 af[TM], wf[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int row = wm * WM + 16 * i + r16;
                    af[i] = __builtin_bit_cast(bf16x8, sA[cur][row * CPR + (c ^ swz(row))]);
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int row = wn * WN + 16 * j + r16;
                    wf[j] = __builtin_bit_cast(bf16x8, sW[cur][row * CPR + (c ^ swz(row))]);
                }
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int i = 0; i < TM; ++i)
                        acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[j], af[i], acc[j][i], 0, 0, 0);
            }
        } else {
            // float32: lane group g contracts k = 8g + s over the 8 steps s.
            f32x4 af[TM][2], wf[TN][2];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = wm * WM + 16 * i + r16;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    af[i][h] = __builtin_bit_cast(f32x4, sA[cur][row * CPR + ((2 * g + h) ^ swz(row))]);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int row = wn * WN + 16 * j + r16;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    wf[j][h] = __builtin_bit_cast(f32x4, sW[cur][row * CPR + ((2 * g + h) ^ swz(row))]);
            }
#pragma unroll
            for (int s = 0; s < 8; ++s)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int i = 0; i < TM; ++i)
                        acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(wf[j][s >> 2][s & 3], af[i][s >> 2][s & 3],
                                                                        acc[j][i], 0, 0, 0);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    typedef typename std::conditional<sizeof(TA) == 2, bf16, float>::type TO;
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int m = m0 + wm * WM + 16 * i + r16;
            const int n = n0 + wn * WN + 16 * j + 4 * g;
            epilogue4<EPI, TO>(ep, M, N, m, n, acc[j][i]);
        }
}

template <typename TA, int BM, int BN>
hipError_t launch_cfg(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                      hipStream_t stream) {
    const int total = (N / BN) * ((M + BM - 1) / BM);
    const int grid = ((total + 7) >> 3) << 3;
    const TA *a = (const TA *)A;
    const TA *w = (const TA *)W;
    switch (epi) {
    case EPI_QKV: gemm_kernel<TA, BM, BN, EPI_QKV><<<grid, NT, 0, stream>>>(a, w, M, N, K, ep); break;
    case EPI_QKV_ROPE: gemm_kernel<TA, BM, BN, EPI_QKV_ROPE><<<grid, NT, 0, stream>>>(a, w, M, N, K, ep); break;
    case EPI_GELU: gemm_kernel<TA, BM, BN, EPI_GELU><<<grid, NT, 0, stream>>>(a, w, M, N, K, ep); break;
    case EPI_RESID: gemm_kernel<TA, BM, BN, EPI_RESID><<<grid, NT, 0, stream>>>(a, w, M, N, K, ep); break;
    default: gemm_kernel<TA, BM, BN, EPI_STORE><<<grid, NT, 0, stream>>>(a, w, M, N, K, ep); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(const void *A, const void *W, int M, int N, int K, bool a_bf16, EpiKind epi,
                       const EpiArgs &ep, hipStream_t stream) {
    if (M <= 0) return hipSuccess;
    if (a_bf16 && gemm_lds_applies(M, N, K)) return launch_gemm_lds(A, W, M, N, K, epi, ep, stream);
    // permuted W rows and the blocked V layout are the LDS kernels' only
    if (ep.perm || ep.vt || ep.out8 || epi == EPI_RESID_LN) return hipErrorInvalidValue;
    if (a_bf16) {
        if (N % 128 == 0) return launch_cfg<bf16, 128, 128>(A, W, M, N, K, epi, ep, stream);
        return launch_cfg<bf16, 128, 64>(A, W, M, N, K, epi, ep, stream);
    }
    if (N % 128 == 0) return launch_cfg<float, 128, 128>(A, W, M, N, K, epi, ep, stream);
    return launch_cfg<float, 128, 64>(A, W, M, N, K, epi, ep, stream);
}

}  // namespace wm
