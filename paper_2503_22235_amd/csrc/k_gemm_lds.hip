// MFMA GEMM (bf16 or e4m3 operands, float32 accumulation) fed by an LDS
// ring that direct buffer->LDS loads fill.
//
//   D[m][n] = sum_k A[m][k] * W[n][k]      (A: tokens x K, W: [out][in])
//
// A workgroup of WGM x WGN waves computes a BM x BN tile; each wave owns a
// (BM/WGM) x (BN/WGN) sub-tile of 16x16x32 MFMA tiles.  The default for the
// block's shapes is 256 x 256 with 8 waves (wave tile 64 x 128), one
// workgroup per CU; 128 x 128 with 4 waves and two workgroups per CU covers
// N not divisible by 256.  K advances in stages of BKB bytes per row (64
// bf16 or 128 e4m3 values for 128-byte rows).  Each stage is written
// straight from global memory into LDS by buffer_load_dwordx4 ... lds (no
// register staging): the activation tile and the weight tile through rings
// of D slots each, D - 1 stages ahead (D = 2 on the shapes launched here).
// A workgroup
// owns one token tile and walks one or more
// output-feature tiles; the stage stream runs on across tile boundaries, so
// the next tile's first loads are in flight while the previous tile's
// epilogue runs.  Rows of A past M come back as zeros from the buffer range
// check, which handles the ragged last token tile.  16-byte chunks of an LDS
// row are XOR-swizzled so the 16 rows one fragment read touches fall in
// distinct banks.  The MFMA "A" operand is the weight tile and "B" the
// activation tile, so every lane ends up with four consecutive output
// features of one token for the epilogue.  Tiles go out in an XCD-aware
// order (consecutive ids on one XCD share an activation tile in its L2).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "kernels.hpp"

namespace wm {
namespace glds {

typedef __attribute__((address_space(3))) void lds_void;

// XOR swizzle of the 16-byte chunks of an LDS row of BKB bytes: 128-byte rows
// by (row >> 1) & 7, 64-byte rows by (row >> 2) & 3, so the 16 rows that one
// fragment read touches fall in distinct banks.
template <int BKB>
__device__ __forceinline__ int swz(int row) {
    return BKB == 128 ? (row >> 1) & 7 : (row >> 2) & 3;
}

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
    u.x = pack_bf16x2(v[0], v[1]);
    u.y = pack_bf16x2(v[2], v[3]);
    *(uint2 *)p = u;
}

// Epilogue on four consecutive output features n..n+3 of token m.  For the
// QKV scatter, `qkv_base` is the element offset of (part, head 0, token 0)
// of the tile's part, `hc` the channel within the part and `qs` the factor
// of the part (the Q scale or 1, times out_mul[part] when e4m3 codes are
// stored): all but hc are uniform over the tile.
template <int EPI>
__device__ __forceinline__ float epilogue4(const EpiArgs &ep, int N, long m, int n, f32x4 v,
                                           size_t qkv_base, int hc, float qs, float dq, float4 b, float4 rr) {
    // explicit FMAs: the rounding of every element must not depend on how
    // the compiler contracts each unrolled copy (a token's result must not
    // depend on its position in the tile, i.e. on the batch)
    v[0] = fmaf(v[0], dq, b.x); v[1] = fmaf(v[1], dq, b.y); v[2] = fmaf(v[2], dq, b.z); v[3] = fmaf(v[3], dq, b.w);
    if constexpr (epi_qkv(EPI)) {
        if (EPI == EPI_QKV_ROPE && n < 2 * ep.C) {
            float r[4] = {v[0], v[1], v[2], v[3]};
            rope_rotate(r, 4, hc & 31, m, ep);
            v[0] = r[0]; v[1] = r[1]; v[2] = r[2]; v[3] = r[3];
        }
        v[0] *= qs; v[1] *= qs; v[2] *= qs; v[3] *= qs;
        const size_t o = qkv_base + ((size_t)(hc >> 5) * ep.Mtot + m) * 32 + (hc & 31);
        if (ep.out8) *(unsigned *)((unsigned char *)ep.out + o) = e4m3x4(v[0], v[1], v[2], v[3]);
        else store4((bf16 *)ep.out + o, v);
    } else if constexpr (EPI == EPI_GELU) {
        v[0] = gelu_as4(v[0]); v[1] = gelu_as4(v[1]); v[2] = gelu_as4(v[2]); v[3] = gelu_as4(v[3]);
        if (ep.out8) {
            const float om = ep.out_mul[0];
            *(unsigned *)((unsigned char *)ep.out + (size_t)m * N + n) = e4m3x4(v[0] * om, v[1] * om, v[2] * om, v[3] * om);
        } else {
            store4((bf16 *)ep.out + (size_t)m * N + n, v);
        }
    } else if constexpr (EPI == EPI_RESID) {
        // rr: the residual values at (m, n..n+3), loaded by the caller
        *(float4 *)(state_row(ep.resid, ep.resid_ptrs, (unsigned)ep.T, ep.dT, (unsigned)m, N) + n) =
            make_float4(rr.x + v[0], rr.y + v[1], rr.z + v[2], rr.w + v[3]);
    } else {
        store4((bf16 *)ep.out + (size_t)m * N + n, v);
    }
    if (!ep.out_amax) return 0.f;           // amax only feeds FP8 requantization
    return fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
}

__device__ __forceinline__ void store8(bf16 *p, const float *v) {
    uint4 u;
    u.x = pack_bf16x2(v[0], v[1]);
    u.y = pack_bf16x2(v[2], v[3]);
    u.z = pack_bf16x2(v[4], v[5]);
    u.w = pack_bf16x2(v[6], v[7]);
    *(uint4 *)p = u;
}

// Epilogue on eight consecutive output features n..n+7 of (global) token
// mg, from two MFMA tiles of permuted W rows (16-byte stores; 32 bytes for
// the float32 residual).  Same conventions as epilogue4.
template <int EPI>
__device__ __forceinline__ float epilogue8(const EpiArgs &ep, int N, long mg, int n, f32x4 a, f32x4 c,
                                           size_t qkv_base, int hc, float qs, float dq, const float2 *rc,
                                           float4 b0, float4 b1) {
    float v[8] = {a[0], a[1], a[2], a[3], c[0], c[1], c[2], c[3]};
    const float bb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = fmaf(v[i], dq, bb[i]);    // explicit FMA, as in epilogue4
    if constexpr (epi_qkv(EPI)) {
        if (EPI == EPI_QKV_ROPE && n < 2 * ep.C) {
            // rc: (cos, sin) of this row's 4 channel pairs (hc & 31) / 2 ..
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float a0 = v[2 * i], a1 = v[2 * i + 1];
                v[2 * i] = fmaf(a0, rc[i].x, -(a1 * rc[i].y));
                v[2 * i + 1] = fmaf(a0, rc[i].y, a1 * rc[i].x);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] *= qs;
        const size_t o = qkv_base + ((size_t)(hc >> 5) * ep.Mtot + mg) * 32 + (hc & 31);
        if (ep.out8) *(uint2 *)((unsigned char *)ep.out + o) = make_uint2(e4m3x4(v[0], v[1], v[2], v[3]), e4m3x4(v[4], v[5], v[6], v[7]));
        else store8((bf16 *)ep.out + o, v);
    } else if constexpr (EPI == EPI_GELU) {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = gelu_as4(v[i]);
        if (ep.out8) {
            const float om = ep.out_mul[0];
            *(uint2 *)((unsigned char *)ep.out + (size_t)mg * N + n) =
                make_uint2(e4m3x4(v[0] * om, v[1] * om, v[2] * om, v[3] * om), e4m3x4(v[4] * om, v[5] * om, v[6] * om, v[7] * om));
        } else {
            store8((bf16 *)ep.out + (size_t)mg * N + n, v);
        }
    } else if constexpr (EPI == EPI_RESID) {
        float4 *r = (float4 *)(state_row(ep.resid, ep.resid_ptrs, (unsigned)ep.T, ep.dT, (unsigned)mg, N) + n);
        float4 x0 = r[0], x1 = r[1];
        x0.x += v[0]; x0.y += v[1]; x0.z += v[2]; x0.w += v[3];
        x1.x += v[4]; x1.y += v[5]; x1.z += v[6]; x1.w += v[7];
        r[0] = x0;
        r[1] = x1;
    } else {
        store8((bf16 *)ep.out + (size_t)mg * N + n, v);
    }
    if (!ep.out_amax) return 0.f;
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[i]));
    return m;
}

// Wait until at most min(later, D - 2) stages of PER load instructions each
// are still in flight (later: stages issued after the one waited for).
template <int PER, int D>
__device__ __forceinline__ void wait_stages(int later) {
    if constexpr (D >= 5)
        if (later >= 3) return wait_vmcnt<3 * PER>();
    if constexpr (D >= 4)
        if (later >= 2) return wait_vmcnt<2 * PER>();
    if constexpr (D >= 3)
        if (later >= 1) return wait_vmcnt<PER>();
    wait_vmcnt<0>();
}

// The MFMAs of one K stage for a wave's TM x TN tiles.  FIRST: the stage is
// the tile's first, so its first k-step adds to zero instead of acc.
// SWAP: the activation tile is the MFMA "A" operand, so a lane holds four
// consecutive tokens of one output feature (the blocked V layout).
// The bf16 MFMA block of each k-step runs at raised wave priority, so that a
// wave with its operands in registers issues ahead of waves still loading
// from LDS or in their epilogue (measured 1-3% faster on the bf16
// projections; the e4m3 stage, whose weight loads sit between its MFMAs, was
// no faster with it).
template <bool FIRST, bool FP8, int TM, int TN, int KSTEPS, int BKB, bool SWAP = false>
__device__ __forceinline__ void mma_stage(const unsigned char *sa, const unsigned char *sw, const int *aoff,
                                          const int *woff, f32x4 (&acc)[TN][TM]) {
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        if constexpr (FP8) {
            // gfx950 16x16x128 f8f6f4 MFMA (e4m3 x e4m3): a lane holds 32
            // k-values of its row for both operands, the k chunk 32 g .. 32 g
            // + 31 of the stage read as two 16-byte pieces (aoff[2 ks],
            // aoff[2 ks + 1]); both operands use the same k assignment, which
            // is all a contraction over k needs.
            i32x8 af[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const uint4 lo = *(const uint4 *)(sa + aoff[2 * ks] + 16 * i * BKB);
                const uint4 hi = *(const uint4 *)(sa + aoff[2 * ks + 1] + 16 * i * BKB);
                af[i] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const uint4 lo = *(const uint4 *)(sw + woff[2 * ks] + 16 * j * BKB);
                const uint4 hi = *(const uint4 *)(sw + woff[2 * ks + 1] + 16 * j * BKB);
                const i32x8 wf = {(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    acc[j][i] = SWAP ? __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                                           af[i], wf, FIRST && ks == 0 ? zero : acc[j][i], 0, 0, 0, 0, 0, 0)
                                     : __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                                           wf, af[i], FIRST && ks == 0 ? zero : acc[j][i], 0, 0, 0, 0, 0, 0);
            }
        } else {
            bf16x8 af[TM], wf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = *(const bf16x8 *)(sa + aoff[ks] + 16 * i * BKB);
#pragma unroll
            for (int j = 0; j < TN; ++j) wf[j] = *(const bf16x8 *)(sw + woff[ks] + 16 * j * BKB);
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    acc[j][i] = SWAP ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], wf[j], FIRST && ks == 0 ? zero : acc[j][i],
                                                                               0, 0, 0)
                                     : __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[j], af[i], FIRST && ks == 0 ? zero : acc[j][i],
                                                                               0, 0, 0);
            __builtin_amdgcn_s_setprio(0);
        }
    }
}

// Epilogue of a V tile of the QKV projection (swapped operands): acc[j][i]
// holds tokens r0 + 16 i + 4 g + (0..3) (chunk rows) of V feature
// f0 + 16 j + r16 (head f >> 5, channel f & 31; V bias `bias`); each lane
// stores its four tokens' values in the blocked layout (plus the wrapped
// copies near lon 0 and X): 8 bytes of bf16, or (FP8) 4 e4m3 codes of
// value * out_mul[2] after the dequantization acc * a_dequant * w_dequant.
// Rows whose four tokens leave a lat row (X or the state size not a
// multiple of 4) are stored one by one.
template <int TM, int TN, bool FP8>
__device__ __forceinline__ void vt_epilogue(const EpiArgs &ep, const float *bias, int M, int r0, int f0,
                                            const f32x4 (&acc)[TN][TM], int g, int r16) {
    float bv[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) bv[j] = bias[f0 + 16 * j + r16];
    const float dq = FP8 ? ep.a_dequant * ep.w_dequant : 1.0f;
    const float om = FP8 ? ep.out_mul[2] : 1.0f;
    const int X = ep.vX, xp = ep.vxp, YX = ep.vY * ep.vX;
    const bool quad = (X & 3) == 0 && (ep.T & 3) == 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int m4 = r0 + 16 * i + 4 * g;
        if (m4 >= M) continue;
        if (quad) {
            const unsigned mg = (unsigned)(m4 + ep.row0);
            const unsigned b = udiv(mg, ep.dT), tt = mg - b * (unsigned)ep.T;
            const unsigned z = udiv(tt, ep.dYX), rr = tt - z * (unsigned)YX;
            const unsigned y = udiv(rr, ep.dX), x = rr - y * (unsigned)X;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int f = f0 + 16 * j + r16;
                const size_t row = v_blocked_offset(ep.vB, ep.vZ, ep.vY, xp, f >> 5, (int)b, (int)z, (int)y, 0, f & 31);
                const int i0 = (int)x + 4;
                float e[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) e[k] = fmaf(acc[j][i][k], dq, bv[j]);
                if constexpr (FP8) {
                    unsigned char *vt = (unsigned char *)ep.vt + row;
                    const unsigned u = e4m3x4(e[0] * om, e[1] * om, e[2] * om, e[3] * om);
                    *(unsigned *)(vt + (size_t)(i0 >> 2) * 128) = u;
                    if (i0 - X >= 0) *(unsigned *)(vt + (size_t)((i0 - X) >> 2) * 128) = u;
                    if (i0 + X < xp) *(unsigned *)(vt + (size_t)((i0 + X) >> 2) * 128) = u;
                } else {
                    bf16 *vt = (bf16 *)ep.vt + row;
                    uint2 u;
                    u.x = pack_bf16x2(e[0], e[1]);
                    u.y = pack_bf16x2(e[2], e[3]);
                    *(uint2 *)(vt + (size_t)(i0 >> 2) * 128) = u;
                    if (i0 - X >= 0) *(uint2 *)(vt + (size_t)((i0 - X) >> 2) * 128) = u;
                    if (i0 + X < xp) *(uint2 *)(vt + (size_t)((i0 + X) >> 2) * 128) = u;
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (m4 + e >= M) break;
                const unsigned mg = (unsigned)(m4 + e + ep.row0);
                const unsigned b = udiv(mg, ep.dT), tt = mg - b * (unsigned)ep.T;
                const unsigned z = udiv(tt, ep.dYX), rr = tt - z * (unsigned)YX;
                const unsigned y = udiv(rr, ep.dX), x = rr - y * (unsigned)X;
                const int i0 = (int)x + 4;
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int f = f0 + 16 * j + r16;
                    const float val = fmaf(acc[j][i][e], dq, bv[j]);
                    const size_t row = v_blocked_offset(ep.vB, ep.vZ, ep.vY, xp, f >> 5, (int)b, (int)z, (int)y, 0, f & 31);
                    const size_t o0 = (size_t)(i0 >> 2) * 128 + (i0 & 3);
                    const size_t o1 = (size_t)((i0 - X) >> 2) * 128 + ((i0 - X) & 3);
                    const size_t o2 = (size_t)((i0 + X) >> 2) * 128 + ((i0 + X) & 3);
                    if constexpr (FP8) {
                        unsigned char *vt = (unsigned char *)ep.vt + row;
                        const unsigned char c = (unsigned char)(e4m3x4(val * om, 0.f, 0.f, 0.f) & 0xffu);
                        vt[o0] = c;
                        if (i0 - X >= 0) vt[o1] = c;
                        if (i0 + X < xp) vt[o2] = c;
                    } else {
                        bf16 *vt = (bf16 *)ep.vt + row;
                        const bf16 c = (bf16)val;
                        vt[o0] = c;
                        if (i0 - X >= 0) vt[o1] = c;
                        if (i0 + X < xp) vt[o2] = c;
                    }
                }
            }
        }
    }
}

// Workgroup barrier ordering LDS accesses only: the vector-memory loads and
// stores in flight (the next stage's loads) stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Epilogue of EPI_RESID_LN (LayerNorm fused into the residual update, WM3
// Sec. 2.1: a block's second LayerNorm reads the residual stream its
// out-projection has just updated).  The tile spans all N features
// of its rows.  A lane holds features ncol + 16 j + 4 g .. +3 of token
// row0w + 16 i + r16 (tile j, row tile i): the residual update of
// EPI_RESID, kept in acc, then the row statistics, summed in the lane (the
// tiles in order, each tile's 4 values pairwise), over the 4 lanes g
// (xsum16_32) and over the WGN waves of the row block through LDS, the
// same steps for every row, so a row's result does not depend on its
// position in the batch.  Two passes, as the LayerNorm kernel: the mean,
// then the mean square of the deviations.
// On gfx9 a wait for a load also waits for the stores issued before it:
// ln_g and ln_b are loaded before the first store and go through LDS, so
// that the normalized rows' stores wait for nothing (the updated rows are
// stored a pair of feature tiles at a time, as in the EPI_RESID epilogue:
// holding them to the end spills registers).
// `red` (LDS, 2 WGN BM + 2 N floats): row sums, then ln_g and ln_b.
template <int TM, int TN, int WGN, int BM, bool FP8>
__device__ __forceinline__ void resid_ln_epilogue(const EpiArgs &ep, int M, int N, int mt, int row0w, int wn, int ncol,
                                                  int g, int r16, int tid, int nth, f32x4 (&acc)[TN][TM], float *red) {
    const float dq = FP8 ? ep.a_dequant * ep.w_dequant : 1.0f;
    // this thread's share of ln_g and ln_b (N <= 2 nth)
    float lg[2], lb[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = tid + u * nth;
        lg[u] = c < N ? ep.ln_g[c] : 0.f;
        lb[u] = c < N ? ep.ln_b[c] : 0.f;
    }
    float *xr[TM];
    float s[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int m = min(mt + row0w + 16 * i + r16, M - 1);
        xr[i] = state_row(ep.resid, ep.resid_ptrs, (unsigned)ep.T, ep.dT, (unsigned)(m + ep.row0), N);
        s[i] = 0.f;
    }
    // residual update, a pair of feature tiles at a time
#pragma unroll
    for (int j = 0; j < TN; j += 2) {
        const int n = ncol + 16 * j + 4 * g;
        const float4 b0 = *(const float4 *)(ep.bias + n), b1 = *(const float4 *)(ep.bias + n + 16);
        float4 rz[TM][2];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            rz[i][0] = *(const float4 *)(xr[i] + n);
            rz[i][1] = *(const float4 *)(xr[i] + n + 16);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float4 b = h ? b1 : b0, r = rz[i][h];
                f32x4 &a = acc[j + h][i];
                // explicit FMAs, as in epilogue4
                a[0] = r.x + fmaf(a[0], dq, b.x);
                a[1] = r.y + fmaf(a[1], dq, b.y);
                a[2] = r.z + fmaf(a[2], dq, b.z);
                a[3] = r.w + fmaf(a[3], dq, b.w);
                if (mt + row0w + 16 * i + r16 < M) *(float4 *)(xr[i] + n + 16 * h) = make_float4(a[0], a[1], a[2], a[3]);
                s[i] += (a[0] + a[1]) + (a[2] + a[3]);
            }
        }
    }
    // row sums across the lanes g and the waves: red[w][row], then
    // red[WGN + w][row]; ln_g and ln_b at red + 2 WGN BM
    const float invN = 1.0f / (float)N;
    float *const lgb = red + 2 * WGN * BM;
    float mean[TM], rstd[TM];
    lds_barrier();    // every wave is done with the stage slot that `red` lies in
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = tid + u * nth;
        if (c < N) {
            lgb[c] = lg[u];
            lgb[N + c] = lb[u];
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        s[i] = xsum16_32(s[i]);
        if (g == 0) red[wn * BM + row0w + 16 * i + r16] = s[i];
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        float t = red[row0w + 16 * i + r16];
#pragma unroll
        for (int w = 1; w < WGN; ++w) t += red[w * BM + row0w + 16 * i + r16];
        mean[i] = t * invN;
        float q = 0.f;
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float d = acc[j][i][c] - mean[i];
                q = fmaf(d, d, q);
            }
        q = xsum16_32(q);
        if (g == 0) red[(WGN + wn) * BM + row0w + 16 * i + r16] = q;
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        float t = red[WGN * BM + row0w + 16 * i + r16];
#pragma unroll
        for (int w = 1; w < WGN; ++w) t += red[(WGN + w) * BM + row0w + 16 * i + r16];
        rstd[i] = 1.0f / sqrtf(t * invN + ep.ln_eps);
    }
    // normalized rows: bf16, or e4m3 codes at the static scale *ln_amax / 448
    const float inv = FP8 ? (*ep.ln_amax > 0.f ? 448.0f / *ep.ln_amax : 1.0f) : 1.0f;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int n = ncol + 16 * j + 4 * g;
        const float4 gm = *(const float4 *)(lgb + n), bt = *(const float4 *)(lgb + N + n);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int m = mt + row0w + 16 * i + r16;
            if (m >= M) continue;
            const f32x4 a = acc[j][i];
            // explicit FMAs, as in the LayerNorm kernel
            const float y0 = fmaf((a[0] - mean[i]) * rstd[i], gm.x, bt.x) * inv;
            const float y1 = fmaf((a[1] - mean[i]) * rstd[i], gm.y, bt.y) * inv;
            const float y2 = fmaf((a[2] - mean[i]) * rstd[i], gm.z, bt.z) * inv;
            const float y3 = fmaf((a[3] - mean[i]) * rstd[i], gm.w, bt.w) * inv;
            const size_t o = (size_t)(m + ep.row0) * N + n;
            if constexpr (FP8) {
                *(unsigned *)((unsigned char *)ep.ln_out + o) = e4m3x4(y0, y1, y2, y3);
            } else {
                uint2 u;
                u.x = pack_bf16x2(y0, y1);
                u.y = pack_bf16x2(y2, y3);
                *(uint2 *)((bf16 *)ep.ln_out + o) = u;
            }
        }
    }
}

// FP8: operands are e4m3 bytes (128 k-values per 128-byte stage, MFMA
// 16x16x128 f8f6f4, one k-step per stage); the epilogue dequantizes per row.
// WGM x WGN waves tile the BM x BN output; OCC workgroups share a CU.
// The activation and weight tiles of each K stage stream through two rings
// of D slots each, D - 1 stages ahead of the MFMAs.
template <int BM, int BN, int BKB, int D, int WGM, int WGN, int OCC, int EPI, bool FP8>
__global__ __launch_bounds__(64 * WGM * WGN, OCC) void gemm_lds_kernel(const void *__restrict__ A, const void *__restrict__ W,
                                                         int M, int N, int K, EpiArgs ep, int tpw, int rw) {
#if defined(__HIP_DEVICE_COMPILE__)   // LDS-address-space builtins exist only in the device pass
    constexpr int NW = WGM * WGN;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int ABYTES = BM * BKB, WBYTES = BN * BKB;   // one slot of each ring
    constexpr int CPR = BKB / 16;                  // 16-byte chunks per LDS row
    constexpr int RPI = 64 / CPR;                  // rows one load instruction fills
    constexpr int LPA = BM / RPI / NW;             // activation load instructions per wave per stage
    constexpr int LPB = BN / RPI / NW;             // weight load instructions per wave per stage
    static_assert(BKB == 128 || BKB == 64, "stage row bytes");
    static_assert(BM % (RPI * NW) == 0 && BN % (RPI * NW) == 0, "rows per stage must split over the waves");
    static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile");
    static_assert(D >= 2 && D <= 5, "ring depth");
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *const aring = smem, *const wring = smem + D * ABYTES;

    // A workgroup computes nn tiles: feature tiles tn0 .. tn0+nn-1 of row
    // block m0 (rw == 0), or row blocks m0, m0+BM, .. of feature tile tn0
    // (rw == 1: the workgroups sharing a row block are consecutive ids, so
    // they run together on one XCD and read that block once into its L2).
    const int ntn = N / BN, ntm = (M + BM - 1) / BM;
    const int ngrp = rw ? (ntm + tpw - 1) / tpw : (ntn + tpw - 1) / tpw;
    const int total = rw ? ngrp * ntn : ngrp * ntm;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    const int m0 = rw ? (id / ntn) * tpw * BM : (id / ngrp) * BM;
    const int tn0 = rw ? id % ntn : (id % ngrp) * tpw;
    const int nn = rw ? min(tpw, ntm - m0 / BM) : min(tpw, ntn - tn0);
    // per-tile advance of the activation rows and of the weight rows (bytes)
    const unsigned astep = rw ? (unsigned)BM * (unsigned)K * (FP8 ? 1u : 2u) : 0u;
    const unsigned wstep = rw ? 0u : (unsigned)BN * (unsigned)K * (FP8 ? 1u : 2u);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int g = lane >> 4, r16 = lane & 15;
    const unsigned Kb = (unsigned)K * (FP8 ? 1 : 2);
    const __amdgpu_buffer_rsrc_t ars = make_rsrc(A, (unsigned)M * Kb);
    const __amdgpu_buffer_rsrc_t wrs = make_rsrc(W, (unsigned)N * Kb);

    // per-lane global byte offsets of this wave's load instructions:
    // instruction i of wave w fills rows RPI (w + NW i) .. +RPI-1 of a slot
    unsigned voa[LPA], vob[LPB];
#pragma unroll
    for (int i = 0; i < LPA; ++i) {
        const int row = RPI * (wave + NW * i) + lane / CPR;
        voa[i] = (unsigned)(m0 + row) * Kb + (((lane % CPR) ^ swz<BKB>(row)) << 4);
    }
#pragma unroll
    for (int i = 0; i < LPB; ++i) {
        const int row = RPI * (wave + NW * i) + lane / CPR;
        vob[i] = (unsigned)(tn0 * BN + row) * Kb + (((lane % CPR) ^ swz<BKB>(row)) << 4);
    }
    const int nk = K / (FP8 ? BKB : BKB / 2);
    // stage s of the stream = k-stage (s % nk) of tile (s / nk)
    auto issue_a = [&](int s) {
        const int t = s / nk, kt = s - t * nk;
        unsigned char *sbase = aring + (s % D) * ABYTES;
        // the row advance goes into the vector offset: rows past M must fail
        // the buffer range check and read zero
        const unsigned aadv = (unsigned)t * astep;
#pragma unroll
        for (int i = 0; i < LPA; ++i)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ars, (lds_void *)(sbase + RPI * (wave + NW * i) * BKB), 16,
                                                     voa[i] + aadv, kt * BKB, 0, 0);
    };
    auto issue_w = [&](int s) {
        const int t = s / nk, kt = s - t * nk;
        unsigned char *sbase = wring + (s % D) * WBYTES;
        const unsigned wsoff = (unsigned)t * wstep + kt * BKB;
#pragma unroll
        for (int i = 0; i < LPB; ++i)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(wrs, (lds_void *)(sbase + RPI * (wave + NW * i) * BKB), 16,
                                                     vob[i], wsoff, 0, 0);
    };

    constexpr bool ZSTART = !FP8 && EPI != EPI_QKV_ROPE && EPI != EPI_RESID_LN;

    // lane-constant fragment offsets inside a stage (swizzle depends on r16
    // only): bf16 k-step ks reads 16 bytes at k = 32ks + 8g; fp8 k-step ks
    // reads 8 bytes at k = 32ks + 8g.
    // fp8: one 16x16x128 k-step per 128-byte stage; a lane reads chunks
    // 2g and 2g + 1 (k = 32 g .. 32 g + 31) of its row.
    constexpr int KSTEPS = FP8 ? BKB / 128 : BKB / 64;
    constexpr int NOFF = FP8 ? 2 * KSTEPS : KSTEPS;
    static_assert(!FP8 || BKB == 128, "fp8 stages hold one 128-k MFMA step");
    int aoff[NOFF], woff[NOFF];
#pragma unroll
    for (int o = 0; o < NOFF; ++o) {
        const int pc = FP8 ? (((8 * (o >> 1) + 2 * g + (o & 1)) ^ swz<BKB>(r16)) << 4)
                           : (((4 * o + g) ^ swz<BKB>(r16)) << 4);
        aoff[o] = (wm * WM + r16) * BKB + pc;
        woff[o] = (wn * WN + r16) * BKB + pc;
    }

    // Issue order: A(0), W(0), .., A(D-2), W(D-2), then in iteration st
    // A(st+D-1), W(st+D-1).  So when iteration st waits, the loads of stages
    // st+1 .. st+D-2 (those that exist) may stay in flight.
    const int S = nn * nk;
#pragma unroll
    for (int s0 = 0; s0 < D - 1; ++s0)
        if (s0 < S) {
            issue_a(s0);
            issue_w(s0);
        }

    // The tiles of this workgroup.  SWAP (the V tiles of a QKV projection
    // with ep.vt set; a workgroup's tiles are all V or none):
    // swapped MFMA operands and the blocked-layout epilogue.  The two bodies
    // are separate instantiations, so neither carries the other's registers.
    auto body = [&](auto swap_tag) {
    constexpr bool SWAP = decltype(swap_tag)::value;
    f32x4 acc[TN][TM];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < nn; ++t) {
        for (int kt = 0; kt < nk; ++kt) {
            const int st = t * nk + kt;
            // This wave's loads of stage st have landed once at most the
            // loads of the later stages already issued are outstanding (loads
            // return in order); the barrier then makes all waves' parts of
            // stage st visible and frees the slots read in iteration st - 1.  (A bare s_barrier: __syncthreads() would
            // also drain the loads still in flight.)
            wait_stages<LPA + LPB, D>(S - 1 - st);
            __builtin_amdgcn_s_barrier();
            if (st + D - 1 < S) {
                issue_a(st + D - 1);
                issue_w(st + D - 1);
            }
            const unsigned char *sbA = aring + (st % D) * ABYTES, *sbW = wring + (st % D) * WBYTES;
            // ZSTART: a tile's first k-step starts its accumulators from an
            // inline zero operand instead of registers cleared in the previous
            // epilogue (not for the FP8, rotary and LayerNorm variants, whose
            // extra registers would spill with a second copy of the stage code)
            if (ZSTART && kt == 0) mma_stage<ZSTART, FP8, TM, TN, KSTEPS, BKB, SWAP>(sbA, sbW, aoff, woff, acc);
            else mma_stage<false, FP8, TM, TN, KSTEPS, BKB, SWAP>(sbA, sbW, aoff, woff, acc);
        }
        const int n0 = (rw ? tn0 : tn0 + t) * BN;
        const int mt = rw ? m0 + t * BM : m0;    // first row of this tile
        if constexpr (EPI == EPI_RESID_LN) {
            // the launcher checks N == BN; the partial sums go to the
            // activation slot of the tile's last stage, which no load is
            // filling (the next tile's first stage went to the other slot)
            static_assert((2 * WGN * BM + 2 * BN) * 4 <= ABYTES && BN <= 2 * NW * 64, "row sums and ln_g, ln_b fit a stage slot");
            resid_ln_epilogue<TM, TN, WGN, BM, FP8>(ep, M, N, mt, wm * WM, wn, wn * WN, g, r16, tid, NW * 64, acc,
                                                    (float *)(aring + (((t + 1) * nk - 1) % D) * ABYTES));
            if constexpr (!ZSTART) {
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            continue;
        }
        if constexpr (SWAP) {
            vt_epilogue<TM, TN, FP8>(ep, ep.bias + 2 * ep.C, M, mt + wm * WM, n0 - 2 * ep.C + wn * WN, acc, g, r16);
            if constexpr (!ZSTART) {
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            continue;
        }
        // a feature tile never straddles Q/K/V (C is a multiple of BN)
        const int part = epi_qkv(EPI) ? ep.part0 + n0 / ep.C : 0;
        const size_t qkv_base = (size_t)part * ep.H * ep.Mtot * 32;
        const float qs = (part == 0 ? ep.qscale : 1.0f) * (epi_qkv(EPI) && ep.out8 ? ep.out_mul[part] : 1.0f);
        // per-row dequantization (fp8) and per-state amax of the outputs
        float dq[TM];
        int srow[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const long mg = (long)min(mt + wm * WM + 16 * i + r16, M - 1) + ep.row0;
            srow[i] = FP8 || ep.out_amax ? (int)(mg / ep.T) : 0;
            dq[i] = FP8 ? (ep.a_amax ? ep.a_amax[srow[i]] * (1.0f / 448.0f) : ep.a_dequant) * ep.w_dequant : 1.0f;
        }
        const int s_lo = ep.out_amax ? (int)(((long)min(mt, M - 1) + ep.row0) / ep.T) : 0;
        // rotary (cos, sin) of each row's channel pairs 4g .. 4g+3 (the same
        // pairs in every head this lane stores), loaded once per tile
        float2 rc[TM][4];
        if constexpr (EPI == EPI_QKV_ROPE) {
            if (ep.perm && part < 2) {
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const long mg = (long)min(mt + wm * WM + 16 * i + r16, M - 1) + ep.row0;
                    const unsigned tt = (unsigned)(mg % ep.T);
                    const unsigned yx = (unsigned)(ep.rY * ep.rX);
                    const int z = (int)(tt / yx), y = (int)((tt / (unsigned)ep.rX) % (unsigned)ep.rY),
                              x = (int)(tt % (unsigned)ep.rX);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int pr = 4 * g + q;
                        const int row = pr < 4 ? z : (pr < 10 ? ep.rZ + y : ep.rZ + ep.rY + x);
                        rc[i][q] = *(const float2 *)(ep.rope + 2 * (row * 16 + pr));
                    }
                }
            }
        }
        // Bias of the features this lane stores.  On gfx9 a wait for a load
        // also waits for every store issued before it, so a load between the
        // stores puts a store round trip on the path: the bias is loaded
        // before the first store (where registers allow) or once per column
        // pair, together with that pair's residual rows.  Tile j covers
        // features 16j + 4g .. (perm: pair j, j+1 covers 16j + 8g .. +7).
        constexpr bool PRE_B = !FP8 && (EPI == EPI_QKV || EPI == EPI_GELU || EPI == EPI_STORE);
        float4 bz[TN];
        auto load_bias = [&](int j) {
            bz[j] = *(const float4 *)(ep.bias + n0 + wn * WN + 16 * (j & ~1) +
                                      (ep.perm ? 8 * g + 4 * (j & 1) : 4 * g + 16 * (j & 1)));
        };
        if constexpr (PRE_B) {
#pragma unroll
            for (int j = 0; j < TN; ++j) load_bias(j);
        }
        float mlo = 0.f, mhi = 0.f;
#pragma unroll
        for (int j = 0; j < TN; j += 2) {
            if constexpr (!PRE_B) {
                load_bias(j);
                load_bias(j + 1);
            }
            // residual rows of this column pair, loaded RI row groups at a
            // time (one wait per batch; FP8 keeps fewer in registers)
            constexpr int RI = FP8 ? 2 : TM;
            float4 rz[TM][2];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                if constexpr (EPI == EPI_RESID) {
                    if (i % RI == 0) {
#pragma unroll
                        for (int ii = i; ii < i + RI; ++ii) {
                            const int m = min(mt + wm * WM + 16 * ii + r16, M - 1);
                            const float *r = state_row(ep.resid, ep.resid_ptrs, (unsigned)ep.T, ep.dT,
                                                       (unsigned)(m + ep.row0), N) + n0 + wn * WN + 16 * j + 4 * g;
                            rz[ii][0] = *(const float4 *)r;
                            rz[ii][1] = *(const float4 *)(r + 16);
                        }
                    }
                }
                const int m = mt + wm * WM + 16 * i + r16;
                const long mg = (long)m + ep.row0;
                float a = 0.f;
                if (m < M) {
                    if (ep.perm) {
                        const int n = n0 + wn * WN + 16 * j + 8 * g;
                        a = epilogue8<EPI>(ep, N, mg, n, acc[j][i], acc[j + 1][i], qkv_base, n - (part - ep.part0) * ep.C, qs,
                                           dq[i], rc[i], bz[j], bz[j + 1]);
                    } else {
                        const int n = n0 + wn * WN + 16 * j + 4 * g;
                        float4 r0 = {}, r1 = {};
                        if constexpr (EPI == EPI_RESID) {
                            r0 = rz[i][0];
                            r1 = rz[i][1];
                        }
                        a = fmaxf(epilogue4<EPI>(ep, N, mg, n, acc[j][i], qkv_base, n - (part - ep.part0) * ep.C, qs, dq[i],
                                                 bz[j], r0),
                                  epilogue4<EPI>(ep, N, mg, n + 16, acc[j + 1][i], qkv_base, n + 16 - (part - ep.part0) * ep.C,
                                                 qs, dq[i], bz[j + 1], r1));
                    }
                }
                if constexpr (!ZSTART) {
                    acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};
                    acc[j + 1][i] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
                if (ep.out_amax) {
                    if (srow[i] == s_lo) mlo = fmaxf(mlo, a);
                    else if (srow[i] == s_lo + 1) mhi = fmaxf(mhi, a);
                    else if (m < M)
                        atomicMax(ep.out_amax + (blockIdx.x % AMAX_SHARDS) * AMAX_STRIDE + srow[i] * ep.amax_stride + part,
                                  __float_as_uint(a));
                }
            }
        }
        if (ep.out_amax) {
            mlo = wave_max(mlo);
            mhi = wave_max(mhi);
            if (lane == 0) {
                unsigned *sh = ep.out_amax + (blockIdx.x % AMAX_SHARDS) * AMAX_STRIDE;
                atomicMax(sh + s_lo * ep.amax_stride + part, __float_as_uint(mlo));
                if ((long)(s_lo + 1) * ep.T < (long)ep.Mtot)
                    atomicMax(sh + (s_lo + 1) * ep.amax_stride + part, __float_as_uint(mhi));
            }
        }
    }
    };
    if constexpr (epi_qkv(EPI)) {
        if (ep.vt && tn0 * BN >= 2 * ep.C) {
            body(std::true_type{});
            return;
        }
    }
    body(std::false_type{});
#endif
}

// Feature tiles per workgroup for 256-wide tiles: the block's QKV (N = 3C =
// 1536) and MLP1 (N = 4C = 2048) GEMMs at C = 512 run fastest with 3 and 4
// (measured); other N of 1536 or more take 2, smaller N take 1.
inline int wide_tpw(int N) { return N == 1536 ? 3 : (N == 2048 ? 4 : (N >= 1536 ? 2 : 1)); }

// RLN: the instantiation for EPI_RESID_LN alone (its tile spans N), which
// takes no other epilogue.
template <int BM, int BN, int BKB, int D, int WGM, int WGN, int OCC, bool FP8, bool RLN = false>
hipError_t launch_cfg(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                      hipStream_t stream, int tpw_default = 1, int rw_default = 0) {
    constexpr size_t lds = (size_t)D * (BM + BN) * BKB;
    static_assert(lds * OCC <= 160 * 1024, "LDS per CU");
    constexpr int NTH = 64 * WGM * WGN;
    if (RLN != (epi == EPI_RESID_LN) || (RLN && N != BN)) return hipErrorInvalidValue;
    // LDS limit of the variants, set once per process (a local static's
    // initialisation is thread-safe; the server thread launches too)
    static const hipError_t attr_err = [] {
        if constexpr (RLN) {
            return hipFuncSetAttribute((const void *)gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_RESID_LN, FP8>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        } else {
            const void *fns[5] = {(const void *)gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_QKV, FP8>,
                                  (const void *)gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_QKV_ROPE, FP8>,
                                  (const void *)gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_GELU, FP8>,
                                  (const void *)gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_RESID, FP8>,
                                  (const void *)gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_STORE, FP8>};
            for (const void *f : fns) {
                const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
    }();
    if (attr_err != hipSuccess) return attr_err;
    const int ntn = N / BN;
    // Output-feature tiles per workgroup (WM_GEMM_TPW overrides, for tuning).
    static const int tpw_env = [] {
        const char *v = getenv("WM_GEMM_TPW");
        return v ? atoi(v) : 0;
    }();
    const int tpw_req = tpw_env > 0 ? tpw_env : tpw_default;
    // Tile order (WM_GEMM_ORDER overrides, for tuning): 0 walks feature
    // tiles, 1 walks row blocks.
    static const int order_env = [] {
        const char *v = getenv("WM_GEMM_ORDER");
        return v ? atoi(v) : -1;
    }();
    const int rw = order_env >= 0 ? (order_env != 0) : rw_default;
    // A is addressed with 32-bit byte offsets from the chunk's first row:
    // split M into row chunks below 2 GiB of A.
    const size_t row_bytes = (size_t)K * (FP8 ? 1 : 2);
    const int chunk = (int)std::min<size_t>((size_t)M, ((size_t)0x7fffffff / row_bytes) / BM * BM);
    for (int r0 = 0; r0 < M; r0 += chunk) {
        const int Mc = std::min(chunk, M - r0);
        EpiArgs e = ep;
        e.row0 = r0;
        e.Mtot = M;
        const void *Ac = (const unsigned char *)A + (size_t)r0 * row_bytes;
        const int ntm = (Mc + BM - 1) / BM;
        const int tpw = std::max(1, std::min(tpw_req, rw ? ntm : ntn));
        const int total = rw ? ((ntm + tpw - 1) / tpw) * ntn : ((ntn + tpw - 1) / tpw) * ntm;
        const int grid = ((total + 7) >> 3) << 3;
        if constexpr (RLN) {
            gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_RESID_LN, FP8><<<grid, NTH, lds, stream>>>(Ac, W, Mc, N, K, e, tpw, rw);
        } else switch (epi) {
        case EPI_QKV:
            gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_QKV, FP8><<<grid, NTH, lds, stream>>>(Ac, W, Mc, N, K, e, tpw, rw);
            break;
        case EPI_QKV_ROPE:
            gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_QKV_ROPE, FP8><<<grid, NTH, lds, stream>>>(Ac, W, Mc, N, K, e, tpw, rw);
            break;
        case EPI_GELU:
            gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_GELU, FP8><<<grid, NTH, lds, stream>>>(Ac, W, Mc, N, K, e, tpw, rw);
            break;
        case EPI_RESID:
            gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_RESID, FP8><<<grid, NTH, lds, stream>>>(Ac, W, Mc, N, K, e, tpw, rw);
            break;
        default:
            gemm_lds_kernel<BM, BN, BKB, D, WGM, WGN, OCC, EPI_STORE, FP8><<<grid, NTH, lds, stream>>>(Ac, W, Mc, N, K, e, tpw, rw);
            break;
        }
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// 128-byte stages in rings of 2, one stage ahead.  Measured on the block's
// shapes (8x90x180, C = 512): 64-byte stages in rings of 4 or 5 (three or
// four stages ahead) are 8-10% slower, and so are two 4-wave workgroups per
// CU on 128 x 256 or 256 x 128 tiles: the per-stage barrier costs more than
// the load latency that deeper rings hide.
template <int BM, int BN, int WGM, int WGN, int OCC, bool FP8>
hipError_t launch_sa(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                     hipStream_t stream, int tpw_default = 1, int rw_default = 0) {
    return launch_cfg<BM, BN, 128, 2, WGM, WGN, OCC, FP8>(A, W, M, N, K, epi, ep, stream, tpw_default, rw_default);
}

}  // namespace glds

using namespace glds;

bool gemm_lds_applies(int M, int N, int K) {
    (void)M;
    return N % 128 == 0 && K % 64 == 0 && (unsigned long long)N * K * 2 < (1ull << 31);
}

hipError_t launch_gemm_lds(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                           hipStream_t stream) {
    // Default for N a multiple of 256: 256x256 tiles, 8 waves (4 x 2, wave
    // tile 64 x 128), 2 stages of 64 KB, one workgroup per CU; wide outputs
    // (six or more feature tiles) walk several feature tiles per workgroup
    // (wide_tpw) so that each next tile's loads overlap the previous tile's
    // epilogue, and N = 512 walks two row blocks of one feature tile for the
    // same overlap.  Other N: 128x128 tiles, 2 stages, two workgroups per CU.
    // WM_GEMM_CFG selects other shapes for tuning.
    static const int cfg = [] {
        const char *v = getenv("WM_GEMM_CFG");
        return v ? atoi(v) : -1;
    }();
    // EPI_RESID_LN: 128 x 512 tiles (8 waves, 2 x 4, the same 64 x 128
    // wave tile), two stages of 80 KB, two row blocks per workgroup
    if (epi == EPI_RESID_LN) {
        if (!gemm_resid_ln_applies(N) || ep.out8 || ep.out_amax || ep.perm || !ep.ln_g || !ep.ln_b || !ep.ln_out) return hipErrorInvalidValue;
        return launch_cfg<128, 512, 128, 2, 2, 4, 1, false, true>(A, W, M, N, K, epi, ep, stream, 2, 1);
    }
    // (a QKV feature tile must not straddle two of Q, K and V: BN divides C)
    const bool n256 = N % 256 == 0 && (!epi_qkv(epi) || ep.C % 256 == 0);
    switch (cfg) {
    case 0: return launch_sa<128, 128, 2, 2, 2, false>(A, W, M, N, K, epi, ep, stream);
    case 3: return launch_cfg<256, 128, 128, 2, 4, 2, 1, false>(A, W, M, N, K, epi, ep, stream);
    default: break;
    }
    auto wide = [&](int tpw, int rw) -> hipError_t {
        return launch_sa<256, 256, 4, 2, 1, false>(A, W, M, N, K, epi, ep, stream, tpw, rw);
    };
    if (epi_qkv(epi) && ep.vt) {
        // a workgroup's feature tiles must be all V or none: walk 2 when a
        // part (C columns) holds an even number of tiles, else 1
        const int bn = n256 ? 256 : 128, per_part = ep.C / bn;
        if (n256) return wide(per_part % 2 ? 1 : 2, 0);
        return launch_sa<128, 128, 2, 2, 2, false>(A, W, M, N, K, epi, ep, stream, per_part % 2 ? 1 : 2, 0);
    }
    if (n256) {
        // N = 512 (the out-projection and MLP2 at C = 512): two row blocks of
        // one feature tile per workgroup (measured 2-3% faster than one tile
        // per workgroup; walking feature tiles is faster for wide N)
        if (N == 512) return wide(2, 1);
        return wide(wide_tpw(N), 0);
    }
    return launch_sa<128, 128, 2, 2, 2, false>(A, W, M, N, K, epi, ep, stream);
}

hipError_t launch_gemm_fp8(const void *A, const void *W, int M, int N, int K, EpiKind epi, const EpiArgs &ep,
                           hipStream_t stream) {
    if (M <= 0) return hipSuccess;
    if (N % 128 || K % 128 || (unsigned long long)N * K >= (1ull << 31)) return hipErrorInvalidValue;
    static const int cfg = [] {
        const char *v = getenv("WM_GEMM_CFG");
        return v ? atoi(v) : -1;
    }();
    if (epi == EPI_RESID_LN) {
        // as in launch_gemm_lds; one dequantization scale for all rows, and
        // the LayerNorm output as e4m3 codes (out8) at a given scale
        if (!gemm_resid_ln_applies(N) || ep.a_amax || !ep.out8 || !ep.ln_amax || ep.out_amax || ep.perm || !ep.ln_g ||
            !ep.ln_b || !ep.ln_out)
            return hipErrorInvalidValue;
        return launch_cfg<128, 512, 128, 2, 2, 4, 1, true, true>(A, W, M, N, K, epi, ep, stream, 2, 1);
    }
    if (epi_qkv(epi) && ep.vt) {
        if (ep.a_amax) return hipErrorInvalidValue;   // V tiles dequantize with the one scale a_dequant
        // a workgroup's feature tiles must be all V or none (as in launch_gemm_lds)
        const bool n256 = N % 256 == 0 && ep.C % 256 == 0;
        const int per_part = ep.C / (n256 ? 256 : 128);
        if (n256) return launch_sa<256, 256, 4, 2, 1, true>(A, W, M, N, K, epi, ep, stream, per_part % 2 ? 1 : 2, 0);
        return launch_sa<128, 128, 2, 2, 2, true>(A, W, M, N, K, epi, ep, stream, per_part % 2 ? 1 : 2, 0);
    }
    if (N % 256 == 0 && (!epi_qkv(epi) || ep.C % 256 == 0) && cfg != 0) {
        // N = 512 (MLP2 at C = 512): row walk, as in launch_gemm_lds
        if (N == 512) return launch_sa<256, 256, 4, 2, 1, true>(A, W, M, N, K, epi, ep, stream, 2, 1);
        return launch_sa<256, 256, 4, 2, 1, true>(A, W, M, N, K, epi, ep, stream, wide_tpw(N), 0);
    }
    return launch_sa<128, 128, 2, 2, 2, true>(A, W, M, N, K, epi, ep, stream);
}

}  // namespace wm
