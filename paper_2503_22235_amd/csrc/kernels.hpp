// Host-side launchers of the libwm kernels (all enqueue on `stream`).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.hpp"

namespace wm {

// Rows of the float32 residual stream [B*T][C]: one buffer x, or (xs set)
// a device array of B state pointers, row m at xs[m / T] + (m % T) * C (the
// states of a batch in separate buffers, e.g. serving slots).
struct StateRows {
    float *x;
    float *const *xs;
    unsigned T;
};

// --- LayerNorm over the channel axis, float32 statistics -----------------
// out[m][c] = (x[m][c] - mu_m) / sqrt(var_m + eps) * gamma[c] + beta[c]
// with biased variance; out element type is float or bf16.
hipError_t launch_layernorm(const StateRows &x, const float *gamma, const float *beta,
                            void *out, bool out_bf16, int M, int C, float eps,
                            hipStream_t stream);

// --- GEMM D[m][n] = sum_k A[m][k] * W[n][k] with fused epilogues ---------
enum EpiKind : int {
    EPI_QKV = 0,    // +bias; Q columns * qscale; scatter to head-major [3][H][M][32]
    EPI_GELU = 1,   // gelu(+bias) -> out [M][N]
    EPI_RESID = 2,  // resid[m][n] += acc + bias (float32 in place)
    EPI_STORE = 3,  // +bias -> out [M][N]
    EPI_QKV_ROPE = 4, // EPI_QKV with q and k rotated (EpiArgs.rope)
    EPI_RESID_LN = 5  // EPI_RESID, then the LayerNorm of each updated row
                      // (EpiArgs.ln_*); LDS GEMMs with N = 512 only
};
constexpr bool epi_qkv(int e) { return e == EPI_QKV || e == EPI_QKV_ROPE; }
// Division of n < 2^31 by a fixed d >= 1 as a multiply-high and a shift
// (Granlund and Montgomery 1994: with l = ceil(log2 d) and
// m = floor(2^(31+l) / d) + 1, floor(n/d) = floor(n m / 2^(31+l))).
struct UDiv {
    unsigned m;
    int s;          // shift after the multiply-high; -1: d == 1
};
inline UDiv udiv_make(unsigned d) {
    if (d <= 1) return UDiv{0u, -1};
    int l = 0;
    while ((1ull << l) < d) ++l;
    return UDiv{(unsigned)((1ull << (31 + l)) / d + 1), l - 1};
}
__device__ __forceinline__ unsigned udiv(unsigned n, UDiv d) { return d.s < 0 ? n : (__umulhi(n, d.m) >> d.s); }
// Row m (< 2^31) of the residual stream of StateRows x with n columns.
__device__ __forceinline__ float *state_row(float *x, float *const *xs, unsigned T, UDiv dT, unsigned m, int n) {
    if (!xs) return x + (size_t)m * n;
    const unsigned b = udiv(m, dT);
    return xs[b] + (size_t)(m - b * T) * n;
}
struct EpiArgs {
    const float *bias;  // [N]
    void *out;          // EPI_QKV / EPI_GELU / EPI_STORE output
    float *resid;       // EPI_RESID target
    // EPI_RESID on states in separate buffers: row m of the target is
    // resid_ptrs[m / T] + (m % T) * N (T and dT set; resid unused)
    float *const *resid_ptrs;
    int C, H;           // EPI_QKV: model width and heads (d = 32)
    int part0;          // EPI_QKV: part (0 Q, 1 K, 2 V) of output column 0
    float qscale;       // EPI_QKV: factor on Q columns
    // FP8 operands: acc * (a_amax[state of row] / 448) * w_dequant, or
    // acc * a_dequant * w_dequant when a_amax is null (one scale for all rows)
    const float *a_amax;
    float a_dequant;
    float w_dequant;
    long T;             // tokens per state
    // optional: per-state amax of the stored outputs (float bits), index
    // state * amax_stride + (QKV part or 0)
    unsigned *out_amax;
    int amax_stride;
    // W rows permuted within aligned groups of 32 (perm_row), so a lane's
    // two adjacent MFMA tiles hold 8 consecutive output features and store
    // them at once; set for processor weights, not for caller-supplied W
    // (LDS GEMMs only).
    int perm;
    // EPI_QKV with rotary position embedding: table of (cos, sin) per
    // [axis offset + position][pair] (level rows 0..Z-1, lat rows Z..Z+Y-1,
    // lon rows Z+Y..Z+Y+X-1; 16 pairs; see rope_rotate) and the grid; null: none
    const float *rope;
    int rZ, rY, rX;
    // Set by the LDS GEMM launchers when they split M into row chunks: the
    // global row of the chunk's row 0 and the total row count.
    int row0, Mtot;
    // EPI_QKV, bf16 LDS GEMM, vt set: V feature f (head f >> 5, channel
    // f & 31) goes to `vt` in the blocked layout of v_blocked_offset (grid
    // vZ x vY x vX, vxp padded positions, vB states) instead of the
    // head-major scatter; the V rows of W are in natural order (Q and K rows
    // permuted when perm is set).  Divisors of a row index: tokens per state
    // (T), per level, per lat row.
    void *vt;
    int vB, vZ, vY, vX, vxp;
    UDiv dT, dYX, dX;
    // FP8 GEMMs (EPI_QKV / EPI_GELU): out8 set stores e4m3 codes of each
    // output value times out_mul[part] (QKV part 0 Q, 1 K, 2 V; GELU part 0)
    // instead of bf16: the Q/K planes and the blocked V with byte elements,
    // the GELU output as [M][N] bytes.
    int out8;
    float out_mul[3];
    // EPI_RESID_LN: every updated row x' of the target (all N features) is
    // also written layer-normalized to ln_out [M][N]:
    // (x' - mean) / sqrt(var + ln_eps) * ln_g + ln_b, as bf16, or, with out8
    // set, as e4m3 codes of that value times 448 / *ln_amax.
    const float *ln_g, *ln_b, *ln_amax;
    void *ln_out;
    float ln_eps;
};
// Rotary position embedding of cnt consecutive channels e.. (e even) of a
// q or k head row at global row mg (token mg mod T): channel pair p =
// e/2 + i rotates by the angle of its axis (pairs 0-3 level, 4-9 lat, 10-15
// lon) at the token's position, read from the (cos, sin) table.
__device__ __forceinline__ void rope_rotate(float *v, int cnt, int e, long mg, const EpiArgs &ep) {
    const unsigned t = (unsigned)(mg % ep.T);
    const unsigned yx = (unsigned)(ep.rY * ep.rX);
    const int z = (int)(t / yx), y = (int)((t / (unsigned)ep.rX) % (unsigned)ep.rY), x = (int)(t % (unsigned)ep.rX);
    for (int i = 0; i < cnt / 2; ++i) {
        const int p = e / 2 + i;
        const int row = p < 4 ? z : (p < 10 ? ep.rZ + y : ep.rZ + ep.rY + x);
        const float2 cs = *(const float2 *)(ep.rope + 2 * (row * 16 + p));
        const float a = v[2 * i], b = v[2 * i + 1];
        v[2 * i] = fmaf(a, cs.x, -(b * cs.y));      // explicit FMAs: position-independent rounding
        v[2 * i + 1] = fmaf(a, cs.y, b * cs.x);
    }
}

// Output feature stored in W row o when EpiArgs.perm is set: within each
// group of 32 rows, row 16 jj + 4 g + i holds feature 8 g + 4 jj + i.
__host__ __device__ inline int perm_row(int o) {
    const int r = o & 31, jj = r >> 4, rho = r & 15;
    return (o & ~31) + 8 * (rho >> 2) + 4 * jj + (rho & 3);
}
// A: [M][K], W: [N][K], both bf16 (a_bf16) or float32.  Output element
// type follows the operands (bf16 or float) except EPI_RESID (float32).
// Requires N % 128 == 0 (N % 64 for small N) and K % 64 == 0 (bf16) /
// K % 32 == 0 (float32).
hipError_t launch_gemm(const void *A, const void *W, int M, int N, int K, bool a_bf16,
                       EpiKind epi, const EpiArgs &ep, hipStream_t stream);

// The LDS-ring bf16 kernel (taken by launch_gemm when it applies).
bool gemm_lds_applies(int M, int N, int K);
hipError_t launch_gemm_lds(const void *A, const void *W, int M, int N, int K, EpiKind epi,
                           const EpiArgs &ep, hipStream_t stream);
// e4m3 operands (A [M][K], W [N][K] bytes); needs N % 128 == 0, K % 128 == 0.
hipError_t launch_gemm_fp8(const void *A, const void *W, int M, int N, int K, EpiKind epi,
                           const EpiArgs &ep, hipStream_t stream);
// Whether the LDS GEMMs take EPI_RESID_LN for this output width (a
// workgroup's tile must span every feature of its rows).
inline bool gemm_resid_ln_applies(int N) { return N == 512; }

// --- FP8 quantization (OCP e4m3; per-state scale amax / 448) --------------
// amax slots live in AMAX_SHARDS copies AMAX_STRIDE apart; producers write
// any copy, launch_amax_fold reduces slots [0, n) into copy 0.
constexpr int AMAX_SHARDS = 64;
constexpr int AMAX_STRIDE = 512;            // slots per copy (>= 8 per state x 64 states)
// per-state amax of bf16 data: state b covers elements [b*per_state, (b+1)*per_state);
// atomicMax into amax[shard*AMAX_STRIDE + b*amax_stride] (fold afterwards)
hipError_t launch_amax_bf16(const void *x, size_t per_state, int B, unsigned *amax, int amax_stride,
                            hipStream_t stream);
// dst[i] = ptrs[i] for i < n (n <= 64): a batch's state pointers written by
// a kernel, in stream order, with no host buffer to keep alive
struct PtrList {
    float *p[64];
};
hipError_t launch_set_ptrs(float **dst, const PtrList &ptrs, int n, hipStream_t stream);
// zero n 32-bit words (a kernel, so graph capture records no memset node)
hipError_t launch_zero_u32(unsigned *p, size_t n, hipStream_t stream);
hipError_t launch_amax_fold(unsigned *amax, int n, hipStream_t stream);
// LayerNorm + quantize with one static amax (device float at `amax`) for
// every row: a single pass.
hipError_t launch_layernorm_fp8_static(const StateRows &x, const float *gamma, const float *beta, int M, int C,
                                       float eps, const float *amax, unsigned char *out, hipStream_t stream);
// float32 -> e4m3 codes = RNE(clamp(x * mul, +-448))
hipError_t launch_quant_f32(const float *in, size_t n, float mul, unsigned char *out, hipStream_t stream);

// --- 3-D neighborhood attention ------------------------------------------
struct NatArgs {
    const void *q, *k, *v;  // element (b,t,h,e) at base + b*bs + t*ts + h*hs + e
    long bs, ts, hs;        // strides of q/k/v in elements
    void *out;              // element (b,t,h,e) at out + b*obs + t*ots + h*32 + e
    long obs, ots;
    const float *rpb;       // [H][2Kz-1][2Ky-1][2Kx-1]
    float qscale;           // scores: (q.k) * qscale + rpb * bscale, in log2 units
    float bscale;
    int B, Z, Y, X, H;
    int Kz, Ky, Kx;
    unsigned periodic;
    float *tbl_ws;          // device scratch of NAT_TBL_WS_FLOATS * H floats (tiled kernel;
                            // B * H tables for the FP8 variant)
    int tbl_ready;          // bf16 tiled kernel: tbl_ws already holds the prepared
                            // table (see launch_nat_bias_table), skip its preparation
    // FP8 attention: per-state amax of q, k, v (floats at amax[b*amax_stride
    // + 0, 1, 2]); when set and the tiled kernel applies, both contractions
    // run on e4m3 codes with the scales amax/448.
    const float *amax;
    int amax_stride;
    // v is in the blocked layout of v_blocked_offset (vt = 1) with xp padded
    // lon positions per row: bf16 elements with q pre-scaled (qscale = 1),
    // or (amax set) e4m3 bytes from launch_kv8 with k in e4m3 as well
    int vt;
    int xp;
    // e4m3 level-ring kernel (amax and vt set): q8 set, q holds e4m3 codes
    // (same strides, in bytes) instead of bf16; o8 set, out receives e4m3
    // codes at v's scale (the output is a convex combination of v rows, so
    // v's amax bounds it) instead of bf16.
    int q8, o8;
};
// Blocked V layout (bf16), written by the QKV projection of bf16
// processors for the tiled attention kernel: per (head, state, level, lat)
// a row of xp padded lon positions i, position i holding lon (i - 4) mod X,
// in blocks of 4 positions x 32 channels x 4 positions (256 bytes), so that
// the 16 positions 8 tx .. 8 tx + 15 (the halo of query tile tx) are one
// 1 KB run.  Element offset of (head h, state b, level z, lat y, position
// i, channel d):
__host__ __device__ inline size_t v_blocked_offset(int B, int Z, int Y, int xp, int h, int b, int z, int y, int i,
                                                   int d) {
    return ((((size_t)h * B + b) * Z + z) * Y + y) * ((size_t)xp * 32) + (size_t)(i >> 2) * 128 + d * 4 + (i & 3);
}
// padded positions per row: every tile's 16-position halo run plus the wrap
inline int v_blocked_xp(int X) { return 8 * ((X + 7) / 8) + 8; }
constexpr int NAT_TBL_WS_FLOATS = 2048;     // per head, >= padded bias table
// Picks the LDS-tiled bf16 kernel when it applies, else the generic one.
hipError_t launch_nat(const NatArgs &a, bool bf16, hipStream_t stream);
// Writes the tiled bf16 kernel's bias table for a.rpb (already in log2
// units, q pre-scaled: qscale = bscale = 1) to a.tbl_ws, so that launches
// with tbl_ready set skip its preparation.  hipErrorNotSupported for windows
// the tiled kernel does not cover.
hipError_t launch_nat_bias_table(const NatArgs &a, hipStream_t stream);
hipError_t launch_nat_generic(const NatArgs &a, bool bf16, hipStream_t stream);
// LDS bytes of the tiled bf16 kernel for these arguments (0: not applicable).
size_t nat_tile_lds_bytes(const NatArgs &a);
hipError_t launch_nat_tile(const NatArgs &a, hipStream_t stream);
// Copies a.v (bf16, token-major with strides bs, ts, hs) into `out` in the
// blocked layout of v_blocked_offset with a.xp positions per row.
hipError_t launch_v_blocked(const NatArgs &a, void *out, hipStream_t stream);
// FP8: a.k and a.v (bf16, token-major) quantized with each state's scales
// (a.amax, folded) into e4m3: k8 with the same strides (in bytes), v8 in the
// blocked layout with byte elements and a.xp positions per row.
hipError_t launch_kv8(const NatArgs &a, unsigned char *k8, unsigned char *v8, hipStream_t stream);

// --- index tables (same window functions as the attention kernels) ------
hipError_t launch_nat_indices(int Z, int Y, int X, int Kz, int Ky, int Kx,
                              unsigned periodic, int *out, hipStream_t stream);

// --- float64 relative-error partial sums: acc[0] += sum (y-r)^2, acc[1] += sum r^2
hipError_t launch_relerr(const float *y, const double *r, size_t n, double *acc,
                         hipStream_t stream);

// --- float32 <-> bfloat16 element copies (either direction, or plain copy)
hipError_t launch_convert(const void *src, bool src_bf16, void *dst, bool dst_bf16, size_t n,
                          hipStream_t stream);
}  // namespace wm
