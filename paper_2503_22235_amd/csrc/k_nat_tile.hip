// LDS-tiled bf16 neighborhood attention for lon-periodic, lat/level-clamped
// grids (the WeatherMesh-3 setting, Sec. 2.1 NATTEN and App. A.2).
//
// Workgroup = 256 threads, one head, a query tile of 4 levels x 4 lats x
// 8 lons (128 queries = 8 groups of 4x2x2).  The union of the tile's
// windows (the halo: 6 x 10 x 14 tokens at 8 levels with a 5x7x7 window)
// of V is staged once in LDS, transposed (d-major, row stride padded so the
// transposing writes hit distinct banks), and shared by all 8 query groups.
// K fragments are read straight from global memory (buffer loads, one chunk
// ahead; the tile's groups re-read them from L1/L2), which keeps the LDS
// footprint at ~66 KB so two workgroups share a CU and one's loads overlap
// the other's math.  Each wave owns two groups with the same level/lat
// window pattern, so they share the relative-position-bias lookups, which
// come from a per-head table (nat_bias_prep): prepared once per processor
// block when the processor is created, else once per launch.
//
// Per group the halo is walked in chunks of 32 keys = 4 lat rows x 8 lon
// columns at one level.  A chunk costs 5 MFMA:
//   S^T = K . Q^T + B        2 x 16x16x32 (the bias-and-mask tile B is the
//                            accumulator input: masked keys enter as -inf)
//   O^T += V^T . P^T         2 x 16x16x32
//   l   += 1 . P^T           1 x 16x16x32 (sums of the bf16 weights)
// The softmax runs in base 2 with a lazily moved reference maximum: the
// weights are exp2(s - m_ref), and m_ref (with the accumulators) is only
// moved when a chunk's maximum exceeds it by more than 8, so weights stay
// <= 256 and most chunks need no rescaling.  Max and sums are float32.
//
// Layout facts used (lane l, g = l/16, r = l%16) for the gfx950 bf16 MFMA
// 16x16x32: A[r][8g..8g+7], B[8g..8g+7][r], D[4g..4g+3][r].  A lane's
// scores in a chunk are keys {4g+i, 16+4g+i}; the P.V contraction takes its
// k index in that order (k-slot 8g + 4j + i <-> key 16j + 4g + i).  The
// query max is shared by lanes l, l^16, l^32, l^48: two permlane swaps.
#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace wm {
namespace {

constexpr int TZ = 4, TY = 4, TX = 8;    // query tile
constexpr int GX = 2;                     // group lon extent
constexpr int XW = 16;                    // halo lon extent, padded (>= TX + Kx - 1)
constexpr int XT = 9;                     // bias table lon extent: hx - xq_rel + 1
constexpr float TAU = 8.0f;               // lazy rescale threshold (log2 units)
constexpr int LD_BATCH = 4;               // halo items loaded before they are stored
constexpr int NEG_RUN = 64;               // -inf entries after the bias table (>= 6 XT + 4)
constexpr int YR_MIN = 10;                // lat rows per level slab a chunk walk may read (2 + 8)

__device__ __forceinline__ void clamp_range(int a0, int tsize, int N, int K, int &lo, int &n) {
    const int last = min(a0 + tsize - 1, N - 1);
    lo = win_start(a0, N, K, false);
    n = win_start(last, N, K, false) + K - lo;
}

// The workgroup's base pointer, held in scalar registers (it is uniform;
// saying so lets buffer loads take it as a scalar resource).
__device__ __forceinline__ void *uniform_ptr(const void *p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (void *)(((unsigned long long)hi << 32) | lo);
}

// 24-bit unsigned product (v_mul_u32_u24): both operands must be below 2^24.
__device__ __forceinline__ unsigned mul24(unsigned a, unsigned b) { return (a & 0xffffffu) * (b & 0xffffffu); }

__device__ __forceinline__ float xmax16_32(float v) {
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = max2f(__uint_as_float(a[0]), __uint_as_float(a[1]));
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return max2f(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

// Division of a workgroup id by the tile counts and the head count:
// m = ceil(2^32 / d) (0 for d = 1) gives floor(t / d) = mulhi(t, m) exactly
// while t d < 2^32, which the launcher checks.
struct TileDiv { unsigned mx, my, mz, mh; };
__device__ __forceinline__ unsigned mdiv(unsigned t, unsigned m) { return m ? __umulhi(t, m) : t; }
inline unsigned div_magic(unsigned d) { return d <= 1 ? 0u : (unsigned)(((1ull << 32) + d - 1) / d); }
inline TileDiv tile_div(const NatArgs &a) {
    return TileDiv{div_magic((a.X + TX - 1) / TX), div_magic((a.Y + TY - 1) / TY), div_magic((a.Z + TZ - 1) / TZ),
                   div_magic(a.H)};
}

// QSCALED: q already carries the factor log2(e)/sqrt(d) (the block path folds
// it into the QKV projection); otherwise scores are scaled after the MFMA and
// the bias table is stored divided by that scale.
template <int KZ, int KY, int KX>
constexpr int tbl_padded() { return ((2 * KZ - 1) * (2 * KY - 1) * XT + NEG_RUN + 3) & ~3; }

// Per-head bias table in the layout the tile kernel reads: tbl[iz][iy][ixt]
// (ixt = key lon slot - query lon slot + 1), lon validity folded in as
// -inf, followed by a run of NEG_RUN entries of -inf that masked (level,
// lat) rows read.
template <int KZ, int KY, int KX, bool QSCALED>
__global__ void nat_bias_prep(NatArgs p) {
    constexpr int RX = (KX - 1) / 2, BY = 2 * KY - 1, BZ = 2 * KZ - 1;
    constexpr int TBL = BZ * BY * XT, TBLP = tbl_padded<KZ, KY, KX>();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.H * TBLP) return;
    const int h = e / TBLP, i = e - h * TBLP;
    const float bs = QSCALED ? p.bscale : p.bscale / p.qscale;
    float v = -INFINITY;
    if (i < TBL) {
        const int ixt = i % XT, rest = i / XT;
        const int dx = ixt - 1 - RX;
        if (dx >= -RX && dx <= RX) v = p.rpb[((size_t)h * BZ * BY + rest) * (2 * KX - 1) + dx + KX - 1] * bs;
    }
    p.tbl_ws[e] = v;
}

typedef __attribute__((address_space(3))) void lds_void;

// bf16 tile kernel for token-major v.  The V halo sits in LDS as slabs of
// 1 KB, one per (level, lat) halo row: 4 blocks of 4 lon columns x 32
// channels x 4 lon (block q holds halo columns 4q .. 4q+3; halo column c is
// lon 8 tx - 4 + c), transposed through registers while it is staged.
//
// Softmax reference: every query's weights are exp2(s - m) with m its own
// score (the query's key is always in its window), so the chunk walk needs
// no running maximum; its own weight is 1, so the sum is >= 1.  A score far
// above m would overflow: the wave then finds the exact maxima in a second
// pass and runs the walk again from them (the result check is on the sum
// and the accumulators).
template <int KZ, int KY, int KX, bool QSCALED>
__global__ __launch_bounds__(256, 2) void nat_tile_kernel(NatArgs p, int ZWmax, int YR, TileDiv dm) {
    constexpr int RX = (KX - 1) / 2;
    constexpr int BY = 2 * KY - 1;
    constexpr int TBL = (2 * KZ - 1) * BY * XT;    // bias table entries
    constexpr int SX = 4 - RX;                      // query tile tx starts at lon 8 tx - SX
    static_assert(2 + KX - 1 <= 8 && 2 + KY - 1 <= 8, "window too large for the 8-wide group halo");
    static_assert(TX == 8 && XW == 16, "halo slab layout");

    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    extern __shared__ __align__(16) unsigned char smem[];
    float *tbl = (float *)smem;                                  // [BZ][BY][XT] + a run of -inf
    unsigned char *Vh = smem + TBLP * 4;                         // [ZWmax * YR] slabs of 1 KB

    // ---- tile of this workgroup (XCD-aware order over (b, h, tile)) ----
    const int ntz = (p.Z + TZ - 1) / TZ, nty = (p.Y + TY - 1) / TY, ntx = (p.X + TX - 1) / TX;
    const int ntiles = ntz * nty * ntx;
    const int total = ntiles * p.H * p.B;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    unsigned t = (unsigned)id, q;
    q = mdiv(t, dm.mx); const int tx = (int)(t - q * (unsigned)ntx); t = q;
    q = mdiv(t, dm.my); const int ty = (int)(t - q * (unsigned)nty); t = q;
    q = mdiv(t, dm.mz); const int tz = (int)(t - q * (unsigned)ntz); t = q;
    q = mdiv(t, dm.mh); const int h = (int)(t - q * (unsigned)p.H);
    const int b = (int)q;
    const int z0 = tz * TZ, y0 = ty * TY;
    const int x0 = tx * TX - SX;                   // lon of the tile's first query (may wrap)
    const int hx0 = tx * TX - 4;                   // lon of halo column 0 (may wrap)

    int zlo, zn, ylo, yn;
    clamp_range(z0, TZ, p.Z, KZ, zlo, zn);
    clamp_range(y0, TY, p.Y, KY, ylo, yn);

    const bf16 *kb = (const bf16 *)p.k + (size_t)b * p.bs + (size_t)h * p.hs;
    const bf16 *qb = (const bf16 *)p.q + (size_t)b * p.bs + (size_t)h * p.hs;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // ---- V halo slabs: (hz, hy) for hz < zn, hy < YR; rows past the halo
    // repeat its last lat row (finite values: their keys are masked, and
    // 0 x V must stay 0) ----
    {
        // item = (slab, lon block qb4, channel chunk c): 4 tokens x 8 channels,
        // written as 8 runs of (channel, 4 lon)
        const bf16 *vb = (const bf16 *)p.v + (size_t)b * p.bs + (size_t)h * p.hs;
        const int nitem = zn * YR * 16;
        for (int it = tid; it < nitem; it += 256) {
            const int sl = it >> 4, qb4 = (it >> 2) & 3, c = it & 3;
            const int hz = sl / YR, hy = sl - hz * YR;
            const int yy = min(ylo + hy, ylo + yn - 1);
            const long rowt = ((long)(zlo + hz) * p.Y + yy) * p.X;
            uint4 u[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int xc = hx0 + 4 * qb4 + e;
                xc = xc < 0 ? xc + p.X : (xc >= p.X ? xc - p.X : xc);
                u[e] = *(const uint4 *)(vb + (rowt + xc) * p.ts + 8 * c);
            }
            const unsigned w0[4] = {u[0].x, u[0].y, u[0].z, u[0].w}, w1[4] = {u[1].x, u[1].y, u[1].z, u[1].w};
            const unsigned w2[4] = {u[2].x, u[2].y, u[2].z, u[2].w}, w3[4] = {u[3].x, u[3].y, u[3].z, u[3].w};
            uint2 *dst = (uint2 *)(Vh + sl * 1024 + qb4 * 256 + (8 * c) * 8);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                dst[2 * k] = make_uint2(__builtin_amdgcn_perm(w1[k], w0[k], 0x05040100u),
                                        __builtin_amdgcn_perm(w3[k], w2[k], 0x05040100u));
                dst[2 * k + 1] = make_uint2(__builtin_amdgcn_perm(w1[k], w0[k], 0x07060302u),
                                            __builtin_amdgcn_perm(w3[k], w2[k], 0x07060302u));
            }
        }
    }
    // ---- bias table of this head (prepared by nat_bias_prep) ----
    {
        const uint4 *src = (const uint4 *)(p.tbl_ws + (size_t)h * TBLP);
        for (int e = tid; e < TBLP / 4; e += 256) ((uint4 *)tbl)[e] = src[e];
    }

    // ---- per wave: lat group pair (wave & 1), lon groups 2*(wave>>1) + {0,1} ----
    const int g = lane >> 4, r16 = lane & 15;
    const int y0g = y0 + 2 * (wave & 1);
    const int gxa = 2 * (wave >> 1);
    const int zq = z0 + (r16 >> 2), yq = y0g + ((r16 >> 1) & 1);
    const int xrel = r16 & 1;
    const int zc = min(zq, p.Z - 1), yc = min(yq, p.Y - 1);

    int ylg, yng;
    clamp_range(min(y0g, p.Y - 1), 2, p.Y, KY, ylg, yng);
    const int dy = ylg - ylo;
    const int wz = win_start(zc, p.Z, KZ, false) - zlo;
    const int wy = win_start(yc, p.Y, KY, false) - ylg;
    const int zb = zlo - zc + KZ - 1;
    const int yb = ylg - yc + KY - 1;

    // Key (block j, lane slot 4g + i) of a chunk (hz, hf) is lat row
    // 4hf + j + 2(g >> 1) of the group halo and lon column 4(g & 1) + i.
    bool oky[2][2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            oky[hf][j] = (unsigned)(4 * hf + j + 2 * (g >> 1) - wy) < (unsigned)KY;
    const int tb_lane = (zb * BY + yb + 2 * (g >> 1)) * XT + 4 * (g & 1) - xrel + 1;

    // K operand: key 16j + r16 = lat row 4hf + j + 2 (r16 >> 3), lon column
    // r16 & 7 of the group halo, from global memory (byte offsets within level
    // zlo; the level advances through the scalar offset).
    const unsigned utsb = (unsigned)p.ts * 2u;
    const unsigned usrow = (unsigned)p.X * utsb;
    const unsigned urow0 = (unsigned)zlo * ((unsigned)p.Y * usrow) + (unsigned)ylo * usrow;
    const __amdgpu_buffer_rsrc_t krs = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(kb), 0, 0x7ffffffe, 0x00020000);
    const int tsb = (int)p.ts * 2;
    int kofs[4][2];
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int hyk = min(4 * (qq >> 1) + (qq & 1) + 2 * (r16 >> 3) + dy, yn - 1);
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            int xk = hx0 + (r16 & 7) + GX * (gxa + G);
            xk = xk < 0 ? xk + p.X : (xk >= p.X ? xk - p.X : xk);
            kofs[qq][G] = (int)(urow0 + mul24((unsigned)hyk, usrow) + mul24((unsigned)xk, utsb)) + 16 * g;
        }
    }
    const int kslab = p.Y * p.X * tsb;
    // V^T operand: lane base of slab (hz, dy + 2 (g >> 1)), lon block
    // (wave >> 1) + (g & 1), channel r16; group 0 reads lon columns 0..3 of
    // that block, group 1 columns 2, 3 of it and 0, 1 of the next.
    const int vbase = ((dy + 2 * (g >> 1)) * 1024) + ((wave >> 1) + (g & 1)) * 256 + r16 * 8;
    const int vslab = YR * 1024;

    // Q fragments and the queries' own scores
    bf16x8 qf[2];
    long qtok[2];
    bool act[2];
    float mref[2];
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        const int xp_ = x0 + GX * (gxa + G) + xrel;               // query lon before wrapping
        act[G] = zq < p.Z && yq < p.Y && xp_ < p.X - SX;
        const int xc = xp_ < 0 ? xp_ + p.X : (xp_ >= p.X ? xp_ - p.X : xp_);
        qtok[G] = (long)mul24(mul24((unsigned)zc, (unsigned)p.Y) + (unsigned)yc, (unsigned)p.X) + xc;
        qf[G] = *(const bf16x8 *)(qb + qtok[G] * p.ts + 8 * g);
        const bf16x8 ks = *(const bf16x8 *)(kb + qtok[G] * p.ts + 8 * g);
        float sd = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) sd = fmaf(bf2f(qf[G][e]), bf2f(ks[e]), sd);
        mref[G] = xsum16_32(sd);
    }
    __syncthreads();     // V halo (and table) in LDS
    {
        const float tcenter = tbl[((KZ - 1) * BY + KY - 1) * XT + 1 + RX];   // bias at offset (0, 0, 0)
#pragma unroll
        for (int G = 0; G < 2; ++G) mref[G] = QSCALED ? mref[G] + tcenter : (mref[G] + tcenter) * p.qscale;
    }

    // all-ones operand of the row-sum MFMA, kept in vector registers (the
    // empty asm hides the constant, so it is not rematerialized per chunk)
    uint4 ones_u = make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u);
    asm volatile("" : "+v"(ones_u.x), "+v"(ones_u.y), "+v"(ones_u.z), "+v"(ones_u.w));
    const bf16x8 ones = __builtin_bit_cast(bf16x8, ones_u);

    f32x4 oacc[2][2], lacc[2];
    for (int pass = 0;; ++pass) {
#pragma unroll
        for (int G = 0; G < 2; ++G) oacc[G][0] = oacc[G][1] = lacc[G] = f32x4{0.f, 0.f, 0.f, 0.f};
        // K fragments rotate through four register sets, two chunks ahead:
        // chunk (hz, hf) uses kreg[2 (hz & 1) + hf] while chunk (hz + 1, hf)
        // is in flight into kreg[2 (~hz & 1) + hf] (the last level reloads
        // itself).  Levels go two per iteration so the set indices are constants.
        bf16x8 kreg[4][2][2];
#pragma unroll
        for (int G = 0; G < 2; ++G)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                kreg[0][G][j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(krs, kofs[j][G], 0, 0));
                kreg[1][G][j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(krs, kofs[2 + j][G], 0, 0));
            }
        for (int hz0 = 0; hz0 < zn; hz0 += 2)
#pragma unroll
        for (int lv = 0; lv < 2; ++lv) {
            const int hz = hz0 + lv;
            if (hz >= zn) break;                 // uniform
            const bool okz = (unsigned)(hz - wz) < (unsigned)KZ;
            const unsigned char *vz = Vh + vbase + hz * vslab;
            const int tbh = tb_lane + hz * BY * XT;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                const int ks = 2 * lv + hf;
                {   // chunk (hz + 1, hf) into the set of (hz - 1, hf)
                    const int soff = __builtin_amdgcn_readfirstlane(min(hz + 1, zn - 1) * kslab);
#pragma unroll
                    for (int G = 0; G < 2; ++G)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            kreg[ks ^ 2][G][j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(
                                krs, kofs[2 * hf + j][G], soff, 0));
                }
                // bias + mask tile (shared by both groups)
                f32x4 binit[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int a = (okz && oky[hf][j]) ? tbh : TBL;
                    const float *tp = tbl + a + (4 * hf + j) * XT;
#pragma unroll
                    for (int i = 0; i < 4; ++i) binit[j][i] = tp[i];
                }
                bf16x8 pb[2];
#pragma unroll
                for (int G = 0; G < 2; ++G)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        f32x4 sc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kreg[ks][G][j], qf[G], binit[j], 0, 0, 0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float sv = QSCALED ? sc[i] : sc[i] * p.qscale;
                            pb[G][4 * j + i] = (bf16)__builtin_amdgcn_exp2f(sv - mref[G]);
                        }
                    }
                const unsigned char *vr = vz + 4 * hf * 1024;
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) {
                    uint4 w0, w1;
                    {   // group 0: lon columns 0..3 of the lane's block, rows j = 0, 1
                        const uint2 a0 = *(const uint2 *)(vr + 128 * tt);
                        const uint2 a1 = *(const uint2 *)(vr + 128 * tt + 1024);
                        w0 = make_uint4(a0.x, a0.y, a1.x, a1.y);
                    }
                    {   // group 1: columns 2, 3 of the block and 0, 1 of the next
                        const unsigned char *v1 = vr + 128 * tt + 4;
                        w1 = make_uint4(*(const unsigned *)v1, *(const unsigned *)(v1 + 252),
                                        *(const unsigned *)(v1 + 1024), *(const unsigned *)(v1 + 1276));
                    }
                    oacc[0][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, w0), pb[0],
                                                                          oacc[0][tt], 0, 0, 0);
                    oacc[1][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, w1), pb[1],
                                                                          oacc[1][tt], 0, 0, 0);
                }
#pragma unroll
                for (int G = 0; G < 2; ++G)
                    lacc[G] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ones, pb[G], lacc[G], 0, 0, 0);
            }
        }
        // The query's own weight is 1, so the sum is >= 1; a sum above 2^96
        // or a non-finite accumulator means a score far above the reference.
        bool bad = false;
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            bad |= !(lacc[G][0] <= 0x1p96f);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                for (int i = 0; i < 4; ++i) bad |= !__builtin_isfinite(oacc[G][tt][i]);
        }
        if (pass == 1 || !__builtin_amdgcn_ballot_w64(bad)) break;
        // exact maxima of the wave's queries, then the walk again
        float mx[2] = {-INFINITY, -INFINITY};
        for (int hz = 0; hz < zn; ++hz) {
            const bool okz = (unsigned)(hz - wz) < (unsigned)KZ;
            const int tbh = tb_lane + hz * BY * XT;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int a = (okz && oky[hf][j]) ? tbh : TBL;
                    const float *tp = tbl + a + (4 * hf + j) * XT;
                    f32x4 bi;
#pragma unroll
                    for (int i = 0; i < 4; ++i) bi[i] = tp[i];
#pragma unroll
                    for (int G = 0; G < 2; ++G) {
                        const bf16x8 kf = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(
                            krs, kofs[2 * hf + j][G], hz * kslab, 0));
                        const f32x4 sc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kf, qf[G], bi, 0, 0, 0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) mx[G] = max2f(mx[G], QSCALED ? sc[i] : sc[i] * p.qscale);
                    }
                }
            }
        }
#pragma unroll
        for (int G = 0; G < 2; ++G) mref[G] = xmax16_32(mx[G]);
    }

#pragma unroll
    for (int G = 0; G < 2; ++G) {
        if (!act[G]) continue;
        const float inv = 1.0f / lacc[G][0];
        bf16 *ob = (bf16 *)p.out + (size_t)b * p.obs + (size_t)qtok[G] * p.ots + h * 32;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            f32x4 v = oacc[G][tt];
            uint2 u;
            u.x = pack_bf16x2(v[0] * inv, v[1] * inv);
            u.y = pack_bf16x2(v[2] * inv, v[3] * inv);
            *(uint2 *)(ob + 16 * tt + 4 * g) = u;
        }
    }
}

// ---------------------------------------------------------------------------
// bf16 kernel for v in the blocked layout (the block path): the K and V
// halos stream through LDS one level at a time.  A level is 10 lat rows of
// K (16 tokens x 64 bytes per row) and 10 of V (one 1 KB slab per row),
// written by direct buffer -> LDS loads (5 per wave per level); two level
// slots alternate, so level hz+1 loads while level hz is computed, and the
// only vector-memory loads in the walk are those, so a full wait and one
// barrier per level order them.  45 KB of LDS per workgroup: three
// workgroups share a CU.  K rows are token-major with the 16-byte channel
// chunks of token c (halo column) of row R stored at chunk position
// q ^ kswz(R, c), so the 16 lanes of a fragment read hit distinct banks.
// Arithmetic, key order and softmax reference are those of nat_tile_kernel.
constexpr int RING_ROWS = YR_MIN;              // lat rows per level (>= TY + KY - 1)
constexpr int RING_SLOT = 2 * RING_ROWS * 1024;   // K rows, then V rows

__device__ __forceinline__ int kswz(int R, int c) { return ((c >> 2) & 1) | (((R >> 1) & 1) << 1); }

template <int KZ, int KY, int KX, bool QSCALED>
__global__ __launch_bounds__(256, 3) void nat_ring_kernel(NatArgs p, TileDiv dm) {
    constexpr int RX = (KX - 1) / 2;
    constexpr int BY = 2 * KY - 1;
    constexpr int TBL = (2 * KZ - 1) * BY * XT;
    constexpr int SX = 4 - RX;
    static_assert(2 + KX - 1 <= 8 && 2 + KY - 1 <= 8, "window too large for the 8-wide group halo");
    static_assert(TY + KY - 1 <= RING_ROWS, "lat halo rows per level");
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    extern __shared__ __align__(16) unsigned char smem[];
    float *tbl = (float *)smem;
    unsigned char *ring = smem + TBLP * 4;          // [2 slots][K rows | V rows]

    const int ntz = (p.Z + TZ - 1) / TZ, nty = (p.Y + TY - 1) / TY, ntx = (p.X + TX - 1) / TX;
    const int ntiles = ntz * nty * ntx;
    const int total = ntiles * p.H * p.B;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    unsigned t = (unsigned)id, q;
    q = mdiv(t, dm.mx); const int tx = (int)(t - q * (unsigned)ntx); t = q;
    q = mdiv(t, dm.my); const int ty = (int)(t - q * (unsigned)nty); t = q;
    q = mdiv(t, dm.mz); const int tz = (int)(t - q * (unsigned)ntz); t = q;
    q = mdiv(t, dm.mh); const int h = (int)(t - q * (unsigned)p.H);
    const int b = (int)q;
    const int z0 = tz * TZ, y0 = ty * TY;
    const int x0 = tx * TX - SX;
    const int hx0 = tx * TX - 4;

    int zlo, zn, ylo, yn;
    clamp_range(z0, TZ, p.Z, KZ, zlo, zn);
    clamp_range(y0, TY, p.Y, KY, ylo, yn);

    const bf16 *kb = (const bf16 *)p.k + (size_t)b * p.bs + (size_t)h * p.hs;
    const bf16 *qb = (const bf16 *)p.q + (size_t)b * p.bs + (size_t)h * p.hs;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // ---- level staging: row r = wave + 4 u (u < 5) of the 20 (K rows 0..9,
    // V rows 10..19); rows past the halo repeat its last lat row ----
    const unsigned tsb = (unsigned)p.ts * 2u;       // token stride, bytes
    const __amdgpu_buffer_rsrc_t krs = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(kb), 0, 0x7ffffffe, 0x00020000);
    const size_t plane = (size_t)p.Z * p.Y * p.xp * 64;
    const unsigned char *vp = (const unsigned char *)p.v + ((size_t)h * p.B + b) * plane;
    const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(vp), 0, (unsigned)plane, 0x00020000);
    unsigned kcol[3];          // per K row this wave loads: token and chunk byte offset within the row
    {
        const int c = lane >> 2, cq = lane & 3;
        int xk = hx0 + c;
        xk = xk < 0 ? xk + p.X : (xk >= p.X ? xk - p.X : xk);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int r = wave + 4 * u;    // K row (u < 3 covers rows 0..9 of waves 0, 1 and 0..7 of 2, 3)
            kcol[u] = (unsigned)xk * tsb + 16u * (unsigned)(cq ^ kswz(r, c));
        }
    }
    const unsigned vcol = 512u * (unsigned)tx + 16u * (unsigned)lane;
    const unsigned rowb = (unsigned)p.xp * 64u;
    auto stage = [&](int hz, int slot) {
        unsigned char *dst = ring + slot * RING_SLOT;
        const unsigned zr = (unsigned)(zlo + hz) * (unsigned)p.Y;
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int r = wave + 4 * u;
            if (r < RING_ROWS) {
                const unsigned yy = (unsigned)min(ylo + r, ylo + yn - 1);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(krs, (lds_void *)(dst + r * 1024), 16,
                                                         (zr + yy) * (unsigned)p.X * tsb + kcol[u < 3 ? u : 0], 0, 0, 0);
            } else {
                const unsigned yy = (unsigned)min(ylo + r - RING_ROWS, ylo + yn - 1);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(vrs, (lds_void *)(dst + r * 1024), 16, (zr + yy) * rowb + vcol, 0, 0, 0);
            }
        }
    };
    stage(0, 0);
    {
        const uint4 *src = (const uint4 *)(p.tbl_ws + (size_t)h * TBLP);
        for (int e = tid; e < TBLP / 4; e += 256) ((uint4 *)tbl)[e] = src[e];
    }

    // ---- per wave: lat group pair (wave & 1), lon groups 2*(wave>>1) + {0,1} ----
    const int g = lane >> 4, r16 = lane & 15;
    const int y0g = y0 + 2 * (wave & 1);
    const int gxa = 2 * (wave >> 1);
    const int zq = z0 + (r16 >> 2), yq = y0g + ((r16 >> 1) & 1);
    const int xrel = r16 & 1;
    const int zc = min(zq, p.Z - 1), yc = min(yq, p.Y - 1);
    int ylg, yng;
    clamp_range(min(y0g, p.Y - 1), 2, p.Y, KY, ylg, yng);
    const int dy = ylg - ylo;
    const int wz = win_start(zc, p.Z, KZ, false) - zlo;
    const int wy = win_start(yc, p.Y, KY, false) - ylg;
    const int zb = zlo - zc + KZ - 1;
    const int yb = ylg - yc + KY - 1;
    bool oky[2][2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            oky[hf][j] = (unsigned)(4 * hf + j + 2 * (g >> 1) - wy) < (unsigned)KY;
    const int tb_lane = (zb * BY + yb + 2 * (g >> 1)) * XT + 4 * (g & 1) - xrel + 1;
    // K operand (key 16 j + r16 = lat row 4hf + j + 2 (r16 >> 3), lon column
    // r16 & 7 of the group halo): LDS byte offsets within a level slot
    int kaddr[2][2][2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int G = 0; G < 2; ++G) {
                const int R = dy + 4 * hf + j + 2 * (r16 >> 3), c = GX * (gxa + G) + (r16 & 7);
                kaddr[hf][j][G] = R * 1024 + c * 64 + 16 * (g ^ kswz(R, c));
            }
    // V^T operand (as in nat_tile_kernel), within a level's V rows
    const int vbase = RING_ROWS * 1024 + (dy + 2 * (g >> 1)) * 1024 + ((wave >> 1) + (g & 1)) * 256 + r16 * 8;

    bf16x8 qf[2];
    long qtok[2];
    bool act[2];
    float mref[2];
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        const int xp_ = x0 + GX * (gxa + G) + xrel;
        act[G] = zq < p.Z && yq < p.Y && xp_ < p.X - SX;
        const int xc = xp_ < 0 ? xp_ + p.X : (xp_ >= p.X ? xp_ - p.X : xp_);
        qtok[G] = (long)mul24(mul24((unsigned)zc, (unsigned)p.Y) + (unsigned)yc, (unsigned)p.X) + xc;
        qf[G] = *(const bf16x8 *)(qb + qtok[G] * p.ts + 8 * g);
        const bf16x8 ks = *(const bf16x8 *)(kb + qtok[G] * p.ts + 8 * g);
        float sd = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) sd = fmaf(bf2f(qf[G][e]), bf2f(ks[e]), sd);
        mref[G] = xsum16_32(sd);
    }
    __syncthreads();     // bias table and level 0 in LDS
    {
        const float tcenter = tbl[((KZ - 1) * BY + KY - 1) * XT + 1 + RX];
#pragma unroll
        for (int G = 0; G < 2; ++G) mref[G] = QSCALED ? mref[G] + tcenter : (mref[G] + tcenter) * p.qscale;
    }

    uint4 ones_u = make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u);
    asm volatile("" : "+v"(ones_u.x), "+v"(ones_u.y), "+v"(ones_u.z), "+v"(ones_u.w));
    const bf16x8 ones = __builtin_bit_cast(bf16x8, ones_u);

    f32x4 oacc[2][2], lacc[2];
    for (int pass = 0;; ++pass) {
#pragma unroll
        for (int G = 0; G < 2; ++G) oacc[G][0] = oacc[G][1] = lacc[G] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int hz0 = 0; hz0 < zn; hz0 += 2)
#pragma unroll
        for (int lv = 0; lv < 2; ++lv) {          // level hz0 + lv is in slot lv
            const int hz = hz0 + lv;
            if (hz >= zn) break;                  // uniform
            if (hz > 0) __syncthreads();          // level hz landed; level hz - 1 is done with
            if (hz + 1 < zn) stage(hz + 1, lv ^ 1);
            const unsigned char *sl = ring + lv * RING_SLOT;
            const bool okz = (unsigned)(hz - wz) < (unsigned)KZ;
            const int tbh = tb_lane + hz * BY * XT;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                f32x4 binit[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int a = (okz && oky[hf][j]) ? tbh : TBL;
                    const float *tp = tbl + a + (4 * hf + j) * XT;
#pragma unroll
                    for (int i = 0; i < 4; ++i) binit[j][i] = tp[i];
                }
                bf16x8 pb[2];
#pragma unroll
                for (int G = 0; G < 2; ++G)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const bf16x8 kf = *(const bf16x8 *)(sl + kaddr[hf][j][G]);
                        const f32x4 sc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kf, qf[G], binit[j], 0, 0, 0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float sv = QSCALED ? sc[i] : sc[i] * p.qscale;
                            pb[G][4 * j + i] = (bf16)__builtin_amdgcn_exp2f(sv - mref[G]);
                        }
                    }
                const unsigned char *vr = sl + vbase + 4 * hf * 1024;
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) {
                    uint4 w0, w1;
                    {
                        const uint2 a0 = *(const uint2 *)(vr + 128 * tt);
                        const uint2 a1 = *(const uint2 *)(vr + 128 * tt + 1024);
                        w0 = make_uint4(a0.x, a0.y, a1.x, a1.y);
                    }
                    {
                        const unsigned char *v1 = vr + 128 * tt + 4;
                        w1 = make_uint4(*(const unsigned *)v1, *(const unsigned *)(v1 + 252),
                                        *(const unsigned *)(v1 + 1024), *(const unsigned *)(v1 + 1276));
                    }
                    oacc[0][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, w0), pb[0],
                                                                          oacc[0][tt], 0, 0, 0);
                    oacc[1][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, w1), pb[1],
                                                                          oacc[1][tt], 0, 0, 0);
                }
#pragma unroll
                for (int G = 0; G < 2; ++G)
                    lacc[G] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ones, pb[G], lacc[G], 0, 0, 0);
            }
        }
        int bad = 0;
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            bad |= !(lacc[G][0] <= 0x1p96f);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                for (int i = 0; i < 4; ++i) bad |= !__builtin_isfinite(oacc[G][tt][i]);
        }
        // workgroup-uniform decision: the walk has barriers
        if (!__syncthreads_or(bad) || pass == 1) break;
        // exact maxima (K from global memory), then the walk again
        {
            const unsigned usrow = (unsigned)p.X * tsb;
            const unsigned urow0 = (unsigned)zlo * ((unsigned)p.Y * usrow) + (unsigned)ylo * usrow;
            const int kslab = p.Y * p.X * (int)tsb;
            float mx[2] = {-INFINITY, -INFINITY};
            for (int hz = 0; hz < zn; ++hz) {
                const bool okz = (unsigned)(hz - wz) < (unsigned)KZ;
                const int tbh = tb_lane + hz * BY * XT;
#pragma unroll
                for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int a = (okz && oky[hf][j]) ? tbh : TBL;
                        const float *tp = tbl + a + (4 * hf + j) * XT;
                        f32x4 bi;
#pragma unroll
                        for (int i = 0; i < 4; ++i) bi[i] = tp[i];
                        const int hyk = min(4 * hf + j + 2 * (r16 >> 3) + dy, yn - 1);
#pragma unroll
                        for (int G = 0; G < 2; ++G) {
                            int xk = hx0 + (r16 & 7) + GX * (gxa + G);
                            xk = xk < 0 ? xk + p.X : (xk >= p.X ? xk - p.X : xk);
                            const unsigned ko = urow0 + (unsigned)hyk * usrow + (unsigned)xk * tsb + 16u * g;
                            const bf16x8 kf = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(
                                krs, ko, hz * kslab, 0));
                            const f32x4 sc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kf, qf[G], bi, 0, 0, 0);
#pragma unroll
                            for (int i = 0; i < 4; ++i) mx[G] = max2f(mx[G], QSCALED ? sc[i] : sc[i] * p.qscale);
                        }
                    }
            }
#pragma unroll
            for (int G = 0; G < 2; ++G) mref[G] = xmax16_32(mx[G]);
        }
        stage(0, 0);
        __syncthreads();
    }

#pragma unroll
    for (int G = 0; G < 2; ++G) {
        if (!act[G]) continue;
        const float inv = 1.0f / lacc[G][0];
        bf16 *ob = (bf16 *)p.out + (size_t)b * p.obs + (size_t)qtok[G] * p.ots + h * 32;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            f32x4 v = oacc[G][tt];
            uint2 u;
            u.x = pack_bf16x2(v[0] * inv, v[1] * inv);
            u.y = pack_bf16x2(v[2] * inv, v[3] * inv);
            *(uint2 *)(ob + 16 * tt + 4 * g) = u;
        }
    }
}

// ---------------------------------------------------------------------------
// FP8 variant: both contractions run on e4m3 codes (gfx950 MFMA
// 16x16x32 fp8, 8-byte fragments in the bf16 layout).  Q, K and V arrive
// in bf16 with per-(state, tensor) amax values and are quantized with the
// state's scale amax/448 as they are staged: K and V halos go to LDS as
// e4m3 (K token-major with 32 bytes per token, V transposed), Q stays in
// registers.  A score leaves the MFMA in units of c = s_q s_k qscale; the
// bias table (per state and head) is stored divided by c, the reference
// maximum is kept in those raw units, and the weights are
// p = exp2(c (s - m)) <= 2^TAU, quantized with the static scale 1.
// O = (sum_k p_k v_k) s_v / (sum_k p_k), both sums from the same e4m3 p.

__device__ __forceinline__ float dq_scale(float amax) { return amax > 0.f ? amax * (1.0f / 448.0f) : 1.0f; }
__device__ __forceinline__ float q_mul(float amax) { return amax > 0.f ? 448.0f / amax : 1.0f; }
__device__ __forceinline__ float clamp448(float v) { return fminf(fmaxf(v, -448.0f), 448.0f); }

// 8 bf16 values -> 8 e4m3 codes of value * mul (round to nearest even,
// saturated); byte i of the result is value i.
__device__ __forceinline__ uint2 bf16x8_to_e4m3(uint4 u, float mul) {
    const unsigned w[4] = {u.x, u.y, u.z, u.w};
    float f[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[2 * q] = __uint_as_float(w[q] << 16) * mul;
        f[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u) * mul;
    }
    uint2 o;
    unsigned a = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(clamp448(f[0]), clamp448(f[1]), 0, false);
    o.x = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(clamp448(f[2]), clamp448(f[3]), (int)a, true);
    a = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(clamp448(f[4]), clamp448(f[5]), 0, false);
    o.y = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(clamp448(f[6]), clamp448(f[7]), (int)a, true);
    return o;
}

constexpr int KRS = XW * 32 + 16;   // K halo bytes per lat row (16-byte pad against bank conflicts)

// V^T row stride in bytes: >= the halo slots, = 8 mod 128.
__host__ __device__ inline int vt_row_bytes(int zw, int yr) { return (zw * yr * XW + 119) / 128 * 128 + 8; }

// Per-(state, head) bias table divided by that state's score unit c.
template <int KZ, int KY, int KX>
__global__ void nat_bias_prep_fp8(NatArgs p) {
    constexpr int RX = (KX - 1) / 2, BY = 2 * KY - 1, BZ = 2 * KZ - 1;
    constexpr int TBL = BZ * BY * XT, TBLP = tbl_padded<KZ, KY, KX>();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.B * p.H * TBLP) return;
    const int bh = e / TBLP, i = e - bh * TBLP;
    const int b = bh / p.H, h = bh - b * p.H;
    const float c = dq_scale(p.amax[(size_t)b * p.amax_stride]) * dq_scale(p.amax[(size_t)b * p.amax_stride + 1]) *
                    p.qscale;
    float v = -INFINITY;
    if (i < TBL) {
        const int ixt = i % XT, rest = i / XT;
        const int dx = ixt - 1 - RX;
        if (dx >= -RX && dx <= RX) v = p.rpb[((size_t)h * BZ * BY + rest) * (2 * KX - 1) + dx + KX - 1] * p.bscale / c;
    }
    p.tbl_ws[e] = v;
}

// ---------------------------------------------------------------------------
// FP8 level-ring kernel (the FP8 block path): the arithmetic of
// nat_tile_fp8_kernel (e4m3 QK and PV on 16x16x32 fp8 MFMA, scores in units
// of c = s_q s_k, per-(state, head) bias table divided by c, e4m3 softmax
// weights with the static scale 1) on the tiling and level streaming of
// nat_ring_kernel.  K and V arrive already quantized (the kv8 pass, or the
// FP8 QKV projection): K as e4m3 rows of 32 bytes per token, V in the
// blocked layout with byte elements; Q in bf16 (quantized here) or, with
// q8, in e4m3; the output in bf16 or, with o8, as e4m3 codes at v's scale.
// A level is 10 lat rows of K (16 tokens x 32 bytes, the 16-byte halves of
// token c in row R swapped when bit 1 of R is set, against bank conflicts)
// and 10 of V (512 bytes), 10 KB; three slots rotate, so the loads of two
// levels are in flight while one is computed (a wave waits for its own part
// of a level with a vmcnt that leaves the next level's loads in flight, then
// a bare barrier).  35 KB of LDS and 128 VGPRs: four workgroups share a CU
// (the level walk is a loop, not unrolled, to stay within the registers;
// measured 262 -> 239 us per state at 8x90x180 with B = 4 against two slots
// and three workgroups per CU).  Reference: each
// query's own score; the weights are exp2(c (s - m)), and if a score
// exceeds m by more than TAU / c (a weight above 2^TAU, outside what the
// e4m3 weights hold with the static scale) the workgroup finds the exact
// maxima and runs the walk again.
constexpr int RING8_ROWB = 512;                        // bytes per K or V row of a level
constexpr int RING8_SLOT = 2 * RING_ROWS * RING8_ROWB;

template <int BYTE>
__device__ __forceinline__ float e4m3_f32(unsigned w) {
    return __builtin_amdgcn_cvt_f32_fp8((int)w, BYTE);
}
// sum over the 4 bytes of a and b (e4m3 codes) of a_i b_i, added to s
__device__ __forceinline__ float e4m3_dot4(unsigned a, unsigned b, float s) {
    s = fmaf(e4m3_f32<0>(a), e4m3_f32<0>(b), s);
    s = fmaf(e4m3_f32<1>(a), e4m3_f32<1>(b), s);
    s = fmaf(e4m3_f32<2>(a), e4m3_f32<2>(b), s);
    return fmaf(e4m3_f32<3>(a), e4m3_f32<3>(b), s);
}

template <int KZ, int KY, int KX>
__global__ __launch_bounds__(256, 4) void nat_ring_fp8_kernel(NatArgs p, TileDiv dm) {
    constexpr int RX = (KX - 1) / 2;
    constexpr int BY = 2 * KY - 1;
    constexpr int TBL = (2 * KZ - 1) * BY * XT;
    constexpr int SX = 4 - RX;
    static_assert(2 + KX - 1 <= 8 && 2 + KY - 1 <= 8, "window too large for the 8-wide group halo");
    static_assert(TY + KY - 1 <= RING_ROWS, "lat halo rows per level");
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    extern __shared__ __align__(16) unsigned char smem[];
    float *tbl = (float *)smem;
    unsigned char *ring = smem + TBLP * 4;

    const int ntz = (p.Z + TZ - 1) / TZ, nty = (p.Y + TY - 1) / TY, ntx = (p.X + TX - 1) / TX;
    const int ntiles = ntz * nty * ntx;
    const int total = ntiles * p.H * p.B;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    unsigned t = (unsigned)id, q;
    q = mdiv(t, dm.mx); const int tx = (int)(t - q * (unsigned)ntx); t = q;
    q = mdiv(t, dm.my); const int ty = (int)(t - q * (unsigned)nty); t = q;
    q = mdiv(t, dm.mz); const int tz = (int)(t - q * (unsigned)ntz); t = q;
    q = mdiv(t, dm.mh); const int h = (int)(t - q * (unsigned)p.H);
    const int b = (int)q;
    const int z0 = tz * TZ, y0 = ty * TY;
    const int x0 = tx * TX - SX;
    const int hx0 = tx * TX - 4;

    int zlo, zn, ylo, yn;
    clamp_range(z0, TZ, p.Z, KZ, zlo, zn);
    clamp_range(y0, TY, p.Y, KY, ylo, yn);

    const unsigned char *k8 = (const unsigned char *)p.k + (size_t)b * p.bs + (size_t)h * p.hs;
    const size_t qoff = (size_t)b * p.bs + (size_t)h * p.hs;   // elements (bf16) or bytes (q8)
    const float aq = p.amax[(size_t)b * p.amax_stride], ak = p.amax[(size_t)b * p.amax_stride + 1],
                av = p.amax[(size_t)b * p.amax_stride + 2];
    const float c = dq_scale(aq) * dq_scale(ak) * p.qscale;     // score unit, log2 domain
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // ---- level staging: instruction u = wave + 4 k (< 10) moves rows 2u, 2u+1
    // of K (u < 5) or of V (u >= 5); rows past the halo repeat its last lat row
    const unsigned tsb = (unsigned)p.ts;                // K token stride, bytes
    const __amdgpu_buffer_rsrc_t krs = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(k8), 0, 0x7ffffffe, 0x00020000);
    const size_t plane = (size_t)p.Z * p.Y * p.xp * 32;
    const unsigned char *vp = (const unsigned char *)p.v + ((size_t)h * p.B + b) * plane;
    const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(vp), 0, (unsigned)plane, 0x00020000);
    const int lrow = lane >> 5;                        // which of the instruction's two rows
    unsigned kcol[2];
    {
        const int cc = (lane >> 1) & 15, hq = lane & 1;
        int xk = hx0 + cc;
        xk = xk < 0 ? xk + p.X : (xk >= p.X ? xk - p.X : xk);
#pragma unroll
        for (int k = 0; k < 2; ++k) {                  // K instructions of this wave: u = wave + 4 k
            const int r = 2 * (wave + 4 * k) + lrow;
            kcol[k] = (unsigned)xk * tsb + 16u * (unsigned)(hq ^ ((r >> 1) & 1));
        }
    }
    const unsigned vcol = 256u * (unsigned)tx + 16u * (unsigned)(lane & 31);
    const unsigned rowb = (unsigned)p.xp * 32u;
    auto stage = [&](int hz, int slot) {
        unsigned char *dst = ring + slot * RING8_SLOT;
        const unsigned zr = (unsigned)(zlo + hz) * (unsigned)p.Y;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int u = wave + 4 * k;
            if (u < 5) {
                const int r = 2 * u + lrow;
                const unsigned yy = (unsigned)min(ylo + r, ylo + yn - 1);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(krs, (lds_void *)(dst + 2 * u * RING8_ROWB), 16,
                                                         (zr + yy) * (unsigned)p.X * tsb + kcol[k < 2 ? k : 0], 0, 0, 0);
            } else if (u < 10) {
                const int r = 2 * (u - 5) + lrow;
                const unsigned yy = (unsigned)min(ylo + r, ylo + yn - 1);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(vrs, (lds_void *)(dst + (RING_ROWS + 2 * (u - 5)) * RING8_ROWB),
                                                         16, (zr + yy) * rowb + vcol, 0, 0, 0);
            }
        }
    };
    stage(0, 0);
    if (zn > 1) stage(1, 1);
    {
        const uint4 *src = (const uint4 *)(p.tbl_ws + ((size_t)b * p.H + h) * TBLP);
        for (int e = tid; e < TBLP / 4; e += 256) ((uint4 *)tbl)[e] = src[e];
    }

    const int g = lane >> 4, r16 = lane & 15;
    const int y0g = y0 + 2 * (wave & 1);
    const int gxa = 2 * (wave >> 1);
    const int zq = z0 + (r16 >> 2), yq = y0g + ((r16 >> 1) & 1);
    const int xrel = r16 & 1;
    const int zc = min(zq, p.Z - 1), yc = min(yq, p.Y - 1);
    int ylg, yng;
    clamp_range(min(y0g, p.Y - 1), 2, p.Y, KY, ylg, yng);
    const int dy = ylg - ylo;
    const int wz = win_start(zc, p.Z, KZ, false) - zlo;
    const int wy = win_start(yc, p.Y, KY, false) - ylg;
    const int zb = zlo - zc + KZ - 1;
    const int yb = ylg - yc + KY - 1;
    bool oky[2][2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            oky[hf][j] = (unsigned)(4 * hf + j + 2 * (g >> 1) - wy) < (unsigned)KY;
    const int tb_lane = (zb * BY + yb + 2 * (g >> 1)) * XT + 4 * (g & 1) - xrel + 1;
    // K operand (key 16 j + r16 = lat row 4hf + j + 2 (r16 >> 3), lon column
    // r16 & 7 of the group halo; channels 8g .. 8g+7): LDS offsets in a slot
    int kaddr[2][2][2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int G = 0; G < 2; ++G) {
                const int R = dy + 4 * hf + j + 2 * (r16 >> 3), cc = GX * (gxa + G) + (r16 & 7);
                kaddr[hf][j][G] = R * RING8_ROWB + cc * 32 + 8 * (g ^ (((R >> 1) & 1) << 1));
            }
    // V^T operand (channel r16 + 16 tt; keys 4g .. 4g+3 of lat rows R0 and
    // R0 + 1): block (wave >> 1) + (g & 1) of row R0 = dy + 4hf + 2 (g >> 1)
    const int vbase = RING_ROWS * RING8_ROWB + (dy + 2 * (g >> 1)) * RING8_ROWB + ((wave >> 1) + (g & 1)) * 128 + r16 * 4;

    long qf[2];
    long qtok[2];
    bool act[2];
    float mref[2];
    const float mulq = q_mul(aq);
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        const int xp_ = x0 + GX * (gxa + G) + xrel;
        act[G] = zq < p.Z && yq < p.Y && xp_ < p.X - SX;
        const int xc = xp_ < 0 ? xp_ + p.X : (xp_ >= p.X ? xp_ - p.X : xp_);
        qtok[G] = (long)mul24(mul24((unsigned)zc, (unsigned)p.Y) + (unsigned)yc, (unsigned)p.X) + xc;
        const uint2 q8 = p.q8 ? *(const uint2 *)((const unsigned char *)p.q + qoff + qtok[G] * p.ts + 8 * g)
                              : bf16x8_to_e4m3(*(const uint4 *)((const bf16 *)p.q + qoff + qtok[G] * p.ts + 8 * g), mulq);
        qf[G] = (long)(((unsigned long long)q8.y << 32) | q8.x);
        const uint2 ks = *(const uint2 *)(k8 + qtok[G] * p.ts + 8 * g);
        mref[G] = xsum16_32(e4m3_dot4(q8.y, ks.y, e4m3_dot4(q8.x, ks.x, 0.f)));                     // the query's own score, raw units (bias below)
    }
    __syncthreads();     // bias table and levels 0 and 1 in LDS
    {
        const float tcenter = tbl[((KZ - 1) * BY + KY - 1) * XT + 1 + RX];
#pragma unroll
        for (int G = 0; G < 2; ++G) mref[G] += tcenter;
    }
    const float tau_raw = TAU / c;
    const long ones = 0x3838383838383838L;   // e4m3 1.0 in every byte

    f32x4 oacc[2][2], lacc[2];
    for (int pass = 0;; ++pass) {
        float mx[2] = {-INFINITY, -INFINITY}, nmc[2];
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            oacc[G][0] = oacc[G][1] = lacc[G] = f32x4{0.f, 0.f, 0.f, 0.f};
            nmc[G] = -c * mref[G];
        }
        for (int hz = 0, lv = 0; hz < zn; ++hz, lv = lv == 2 ? 0 : lv + 1) {
            if (hz > 0) {
                // this wave's loads of level hz have landed once at most those
                // of level hz + 1 (3 instructions for waves 0 and 1, 2 for
                // waves 2 and 3, issued later) are outstanding; the barrier
                // then makes every wave's part visible and frees the slot of
                // level hz - 1 (levels 0 and 1 were waited for before the walk)
                if (hz > 1) {
                    if (hz + 1 < zn) {
                        if (wave < 2) wait_vmcnt<3>();
                        else wait_vmcnt<2>();
                    } else {
                        wait_vmcnt<0>();
                    }
                }
                __builtin_amdgcn_s_barrier();
            }
            if (hz + 2 < zn) stage(hz + 2, lv == 0 ? 2 : lv - 1);
            const unsigned char *sl = ring + lv * RING8_SLOT;
            const bool okz = (unsigned)(hz - wz) < (unsigned)KZ;
            const int tbh = tb_lane + hz * BY * XT;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                f32x4 binit[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int a = (okz && oky[hf][j]) ? tbh : TBL;
                    const float *tp = tbl + a + (4 * hf + j) * XT;
#pragma unroll
                    for (int i = 0; i < 4; ++i) binit[j][i] = tp[i];
                }
                long pf[2];
#pragma unroll
                for (int G = 0; G < 2; ++G) {
                    float pv[8];
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const long kf = *(const long *)(sl + kaddr[hf][j][G]);
                        const f32x4 sc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(kf, qf[G], binit[j], 0, 0, 0);
                        mx[G] = max3f(mx[G], max3f(sc[0], sc[1], sc[2]), sc[3]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) pv[4 * j + i] = __builtin_amdgcn_exp2f(fmaf(sc[i], c, nmc[G]));
                    }
                    unsigned lo = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[0], pv[1], 0, false);
                    lo = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[2], pv[3], (int)lo, true);
                    unsigned hi = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[4], pv[5], 0, false);
                    hi = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[6], pv[7], (int)hi, true);
                    pf[G] = (long)(((unsigned long long)hi << 32) | lo);
                }
                const unsigned char *vr = sl + vbase + 4 * hf * RING8_ROWB;
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) {
                    const unsigned char *vt = vr + 64 * tt;
                    const unsigned a0 = *(const unsigned *)vt, a1 = *(const unsigned *)(vt + 128);
                    const unsigned b0 = *(const unsigned *)(vt + RING8_ROWB), b1 = *(const unsigned *)(vt + RING8_ROWB + 128);
                    // group 0: lon columns 0..3 of the block; group 1: columns 2, 3 and 0, 1 of the next
                    const long v0 = (long)(((unsigned long long)b0 << 32) | a0);
                    const long v1 = (long)(((unsigned long long)__builtin_amdgcn_alignbyte(b1, b0, 2) << 32) |
                                           __builtin_amdgcn_alignbyte(a1, a0, 2));
                    oacc[0][tt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(v0, pf[0], oacc[0][tt], 0, 0, 0);
                    oacc[1][tt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(v1, pf[1], oacc[1][tt], 0, 0, 0);
                }
#pragma unroll
                for (int G = 0; G < 2; ++G)
                    lacc[G] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ones, pf[G], lacc[G], 0, 0, 0);
            }
        }
        // weights above 2^TAU (or a non-finite result) need the exact maxima
        int bad = 0;
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            bad |= !(mx[G] - mref[G] <= tau_raw);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                for (int i = 0; i < 4; ++i) bad |= !__builtin_isfinite(oacc[G][tt][i]);
        }
        if (!__syncthreads_or(bad) || pass == 1) break;
        {
            const unsigned usrow = (unsigned)p.X * tsb;
            const unsigned urow0 = (unsigned)zlo * ((unsigned)p.Y * usrow) + (unsigned)ylo * usrow;
            const int kslab = p.Y * p.X * (int)tsb;
            float me[2] = {-INFINITY, -INFINITY};
            for (int hz = 0; hz < zn; ++hz) {
                const bool okz = (unsigned)(hz - wz) < (unsigned)KZ;
                const int tbh = tb_lane + hz * BY * XT;
#pragma unroll
                for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int a = (okz && oky[hf][j]) ? tbh : TBL;
                        const float *tp = tbl + a + (4 * hf + j) * XT;
                        f32x4 bi;
#pragma unroll
                        for (int i = 0; i < 4; ++i) bi[i] = tp[i];
                        const int hyk = min(4 * hf + j + 2 * (r16 >> 3) + dy, yn - 1);
#pragma unroll
                        for (int G = 0; G < 2; ++G) {
                            int xk = hx0 + (r16 & 7) + GX * (gxa + G);
                            xk = xk < 0 ? xk + p.X : (xk >= p.X ? xk - p.X : xk);
                            const unsigned ko = urow0 + (unsigned)hyk * usrow + (unsigned)xk * tsb + 8u * g;
                            const long kf = (long)__builtin_bit_cast(unsigned long long,
                                                                   __builtin_amdgcn_raw_buffer_load_b64(krs, ko, hz * kslab, 0));
                            const f32x4 sc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(kf, qf[G], bi, 0, 0, 0);
                            me[G] = max3f(me[G], max3f(sc[0], sc[1], sc[2]), sc[3]);
                        }
                    }
            }
#pragma unroll
            for (int G = 0; G < 2; ++G) mref[G] = xmax16_32(me[G]);
        }
        stage(0, 0);
        if (zn > 1) stage(1, 1);
        __syncthreads();
    }

    // o = s_v (sum p v8) / (sum p); as e4m3 codes at v's scale: (sum p v8) / (sum p)
    const float sv = p.o8 ? 1.0f : dq_scale(av);
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        if (!act[G]) continue;
        const float inv = sv / lacc[G][0];
        const size_t oo = (size_t)b * p.obs + (size_t)qtok[G] * p.ots + h * 32;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            f32x4 v = oacc[G][tt];
            if (p.o8) {
                *(unsigned *)((unsigned char *)p.out + oo + 16 * tt + 4 * g) =
                    e4m3x4(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
            } else {
                uint2 u;
                u.x = pack_bf16x2(v[0] * inv, v[1] * inv);
                u.y = pack_bf16x2(v[2] * inv, v[3] * inv);
                *(uint2 *)((bf16 *)p.out + oo + 16 * tt + 4 * g) = u;
            }
        }
    }
}

// K (bf16, token-major with strides bs, ts, hs) -> e4m3 at the state's
// scale amax_k / 448, same strides in bytes; 8 channels per thread.
__global__ void k8_kernel(const bf16 *__restrict__ k, long bs, long ts, long hs, unsigned char *__restrict__ out,
                          int B, long T, int H, const float *__restrict__ amax, int amax_stride) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)B * T * H * 4;
    if (e >= total) return;
    const int c = (int)(e & 3);
    long r = e >> 2;
    const int h = (int)(r % H); r /= H;
    const long t = r % T;
    const int b = (int)(r / T);
    const size_t off = (size_t)b * bs + (size_t)t * ts + (size_t)h * hs + 8 * c;
    *(uint2 *)(out + off) = bf16x8_to_e4m3(*(const uint4 *)(k + off), q_mul(amax[(size_t)b * amax_stride + 1]));
}

// V (bf16, token-major) -> e4m3 at the state's scale amax_v / 448 in the
// blocked layout with byte elements: one thread per (head, state, level,
// lat, block of 4 positions, 8 channels).
__global__ void v8_blocked_kernel(const bf16 *__restrict__ v, long bs, long ts, long hs, unsigned char *__restrict__ out,
                                  int B, int Z, int Y, int X, int H, int xp, const float *__restrict__ amax,
                                  int amax_stride) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nxb = xp >> 2;
    const long total = (long)H * B * Z * Y * nxb * 4;
    if (e >= total) return;
    const int c = (int)(e & 3);
    long r = e >> 2;
    const int xb = (int)(r % nxb); r /= nxb;
    const long zyb = r;
    const int y = (int)(r % Y); r /= Y;
    const int z = (int)(r % Z); r /= Z;
    const int b = (int)(r % B);
    const int h = (int)(r / B);
    const float mul = q_mul(amax[(size_t)b * amax_stride + 2]);
    uint2 q8[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int x = 4 * xb + k - 4;
        x = ((x % X) + X) % X;
        q8[k] = bf16x8_to_e4m3(*(const uint4 *)(v + (size_t)b * bs + (((size_t)z * Y + y) * X + x) * ts + (size_t)h * hs + 8 * c), mul);
    }
    // channel 8c + i of the 4 positions -> one dword (byte k = position k)
    unsigned *dst = (unsigned *)(out + ((size_t)zyb * nxb + xb) * 128 + (8 * c) * 4);
    const unsigned lo01 = __builtin_amdgcn_perm(q8[1].x, q8[0].x, 0x05010400u);   // p0c0 p1c0 p0c1 p1c1
    const unsigned lo23 = __builtin_amdgcn_perm(q8[3].x, q8[2].x, 0x05010400u);
    const unsigned hi01 = __builtin_amdgcn_perm(q8[1].x, q8[0].x, 0x07030602u);   // c2, c3
    const unsigned hi23 = __builtin_amdgcn_perm(q8[3].x, q8[2].x, 0x07030602u);
    const unsigned lo01b = __builtin_amdgcn_perm(q8[1].y, q8[0].y, 0x05010400u);
    const unsigned lo23b = __builtin_amdgcn_perm(q8[3].y, q8[2].y, 0x05010400u);
    const unsigned hi01b = __builtin_amdgcn_perm(q8[1].y, q8[0].y, 0x07030602u);
    const unsigned hi23b = __builtin_amdgcn_perm(q8[3].y, q8[2].y, 0x07030602u);
    dst[0] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
    dst[1] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
    dst[2] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
    dst[3] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
    dst[4] = __builtin_amdgcn_perm(lo23b, lo01b, 0x05040100u);
    dst[5] = __builtin_amdgcn_perm(lo23b, lo01b, 0x07060302u);
    dst[6] = __builtin_amdgcn_perm(hi23b, hi01b, 0x05040100u);
    dst[7] = __builtin_amdgcn_perm(hi23b, hi01b, 0x07060302u);
}

template <int KZ, int KY, int KX>
__global__ __launch_bounds__(256, 2) void nat_tile_fp8_kernel(NatArgs p, int ZWmax, int YR, TileDiv dm) {
    constexpr int RX = (KX - 1) / 2;
    constexpr int BY = 2 * KY - 1;
    constexpr int TBL = (2 * KZ - 1) * BY * XT;
    static_assert(2 + KX - 1 <= 8 && 2 + KY - 1 <= 8, "window too large for the 8-wide group halo");
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    extern __shared__ __align__(16) unsigned char smem[];
    float *tbl = (float *)smem;
    unsigned char *Ks = smem + TBLP * 4;                     // [ZWmax*YR lat rows][KRS]
    const int VSB = vt_row_bytes(ZWmax, YR);
    unsigned char *Vt = Ks + (size_t)ZWmax * YR * KRS;       // [32][VSB]

    const int ntz = (p.Z + TZ - 1) / TZ, nty = (p.Y + TY - 1) / TY, ntx = (p.X + TX - 1) / TX;
    const int ntiles = ntz * nty * ntx;
    const int total = ntiles * p.H * p.B;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    // (tile x, y, z, head, state) from id by multiply-high divisions on
    // scalar registers (magic numbers from the launcher)
    unsigned t = (unsigned)id, q;
    q = mdiv(t, dm.mx); const int tx = (int)(t - q * (unsigned)ntx); t = q;
    q = mdiv(t, dm.my); const int ty = (int)(t - q * (unsigned)nty); t = q;
    q = mdiv(t, dm.mz); const int tz = (int)(t - q * (unsigned)ntz); t = q;
    q = mdiv(t, dm.mh); const int h = (int)(t - q * (unsigned)p.H);
    const int b = (int)q;
    const int z0 = tz * TZ, y0 = ty * TY, x0 = tx * TX;

    int zlo, zn, ylo, yn;
    clamp_range(z0, TZ, p.Z, KZ, zlo, zn);
    clamp_range(y0, TY, p.Y, KY, ylo, yn);
    const int xlo = x0 - RX;

    const bf16 *kb = (const bf16 *)p.k + (size_t)b * p.bs + (size_t)h * p.hs;
    const bf16 *vb = (const bf16 *)p.v + (size_t)b * p.bs + (size_t)h * p.hs;
    const bf16 *qb = (const bf16 *)p.q + (size_t)b * p.bs + (size_t)h * p.hs;
    const float aq = p.amax[(size_t)b * p.amax_stride], ak = p.amax[(size_t)b * p.amax_stride + 1],
                av = p.amax[(size_t)b * p.amax_stride + 2];
    const float c = dq_scale(aq) * dq_scale(ak) * p.qscale;     // score unit, log2 domain
    const float mulk = q_mul(ak), mulv = q_mul(av);
    const int tid = threadIdx.x;
    // 32-bit byte offsets within the head's K and V planes, 24-bit products
    // (the launcher checks the plane and row sizes)
    const unsigned utsb = (unsigned)p.ts * 2u, usrow = (unsigned)p.X * utsb, uslab = (unsigned)p.Y * usrow;
    const unsigned urow0 = (unsigned)zlo * uslab + (unsigned)ylo * usrow;

    {
        const uint4 *src = (const uint4 *)(p.tbl_ws + ((size_t)b * p.H + h) * TBLP);
        for (int e = tid; e < TBLP / 4; e += 256) ((uint4 *)tbl)[e] = src[e];
    }
    // ---- K halo, token-major e4m3: item = (slot, 16-byte chunk c of 8
    // channels); the 64 items of a halo row go to 64 consecutive threads, so
    // a thread keeps its lon slot and chunk and walks rows 4 apart.
    const int nrows = zn * yn;
    const unsigned ym = (65536u + yn - 1) / yn;              // row / yn == (row * ym) >> 16 (row * yn < 2^16)
    {
        const int cc = tid & 3, hx = (tid >> 2) & 15, rb0 = tid >> 6;
        int xc = xlo + (hx < TX + KX - 1 ? hx : 0);
        xc = xc < 0 ? xc + p.X : (xc >= p.X ? xc - p.X : xc);
        unsigned char *kdst = Ks + hx * 32 + 8 * cc;
        const unsigned kcol = mul24((unsigned)xc, utsb) + 16u * cc;
        const __amdgpu_buffer_rsrc_t krs8 = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(kb), 0, 0x7ffffffe, 0x00020000);
        for (int rb = rb0; rb < nrows; rb += 4 * LD_BATCH) {
            uint4 raw[LD_BATCH];
#pragma unroll
            for (int u = 0; u < LD_BATCH; ++u) {
                const unsigned row = (unsigned)min(rb + 4 * u, nrows - 1);
                const unsigned hz = mul24(row, ym) >> 16, hy = row - mul24(hz, (unsigned)yn);
                raw[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                    krs8, urow0 + hz * uslab + mul24(hy, usrow) + kcol, 0, 0));
            }
#pragma unroll
            for (int u = 0; u < LD_BATCH; ++u) {
                const int row = rb + 4 * u;
                if (row < nrows) {
                    const unsigned hz = mul24((unsigned)row, ym) >> 16, hy = (unsigned)row - mul24(hz, (unsigned)yn);
                    *(uint2 *)(kdst + mul24(mul24(hz, (unsigned)YR) + hy, (unsigned)KRS)) = bf16x8_to_e4m3(raw[u], mulk);
                }
            }
        }
    }
    // ---- V halo, transposed e4m3: item = (4 neighbouring slots, chunk c);
    // the 16 items of a halo row go to 16 consecutive threads (rows 16 apart).
    {
        const int cc = tid & 3, qd = (tid >> 2) & 3, rb0 = tid >> 4;
        int xs[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            int xc = xlo + (4 * qd + w < TX + KX - 1 ? 4 * qd + w : 0);
            xs[w] = xc < 0 ? xc + p.X : (xc >= p.X ? xc - p.X : xc);
        }
        unsigned char *vdst = Vt + (8 * cc) * VSB + 4 * qd;
        unsigned vcol[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) vcol[w] = mul24((unsigned)xs[w], utsb) + 16u * cc;
        const __amdgpu_buffer_rsrc_t vrs8 = __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(vb), 0, 0x7ffffffe, 0x00020000);
        for (int rb = rb0; rb < nrows; rb += 16 * (LD_BATCH / 2)) {
            uint4 raw[LD_BATCH / 2][4];
#pragma unroll
            for (int u = 0; u < LD_BATCH / 2; ++u) {
                const unsigned row = (unsigned)min(rb + 16 * u, nrows - 1);
                const unsigned hz = mul24(row, ym) >> 16, hy = row - mul24(hz, (unsigned)yn);
                const unsigned ro = urow0 + hz * uslab + mul24(hy, usrow);
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    raw[u][w] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(vrs8, ro + vcol[w], 0, 0));
            }
#pragma unroll
            for (int u = 0; u < LD_BATCH / 2; ++u) {
                const int row = rb + 16 * u;
                if (row < nrows) {
                    const unsigned hz = mul24((unsigned)row, ym) >> 16, hy = (unsigned)row - mul24(hz, (unsigned)yn);
                    uint2 cv[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) cv[w] = bf16x8_to_e4m3(raw[u][w], mulv);
                    // 4 tokens x 8 channels of bytes -> 8 dwords of 4 tokens each
                    const unsigned lo01 = __builtin_amdgcn_perm(cv[1].x, cv[0].x, 0x05010400u);  // t0c0 t1c0 t0c1 t1c1
                    const unsigned lo23 = __builtin_amdgcn_perm(cv[3].x, cv[2].x, 0x05010400u);
                    const unsigned hi01 = __builtin_amdgcn_perm(cv[1].x, cv[0].x, 0x07030602u);  // c2, c3
                    const unsigned hi23 = __builtin_amdgcn_perm(cv[3].x, cv[2].x, 0x07030602u);
                    const unsigned lo01b = __builtin_amdgcn_perm(cv[1].y, cv[0].y, 0x05010400u);
                    const unsigned lo23b = __builtin_amdgcn_perm(cv[3].y, cv[2].y, 0x05010400u);
                    const unsigned hi01b = __builtin_amdgcn_perm(cv[1].y, cv[0].y, 0x07030602u);
                    const unsigned hi23b = __builtin_amdgcn_perm(cv[3].y, cv[2].y, 0x07030602u);
                    unsigned char *dst = vdst + mul24(mul24(hz, (unsigned)YR) + hy, (unsigned)XW);
                    *(unsigned *)(dst + 0 * VSB) = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
                    *(unsigned *)(dst + 1 * VSB) = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
                    *(unsigned *)(dst + 2 * VSB) = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
                    *(unsigned *)(dst + 3 * VSB) = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
                    *(unsigned *)(dst + 4 * VSB) = __builtin_amdgcn_perm(lo23b, lo01b, 0x05040100u);
                    *(unsigned *)(dst + 5 * VSB) = __builtin_amdgcn_perm(lo23b, lo01b, 0x07060302u);
                    *(unsigned *)(dst + 6 * VSB) = __builtin_amdgcn_perm(hi23b, hi01b, 0x05040100u);
                    *(unsigned *)(dst + 7 * VSB) = __builtin_amdgcn_perm(hi23b, hi01b, 0x07060302u);
                }
            }
        }
    }
    // ---- zero the lat rows yn .. YR-1 of every level (read for keys outside
    // every window, whose weight is 0; 0 x code must stay 0)
    if (yn < YR) {
        const int kgap = (YR - yn) * KRS / 4;                 // dwords per level (K)
        const unsigned km = 0xffffffffu / (unsigned)kgap + 1u;   // e / kgap == mulhi(e, km) (e * kgap < 2^32)
        for (int e = tid; e < zn * kgap; e += 256) {
            const int hz = (int)__umulhi((unsigned)e, km), o = e - hz * kgap;
            ((unsigned *)(Ks + (hz * YR + yn) * KRS))[o] = 0u;
        }
        const int vgap = (YR - yn) * XW / 4;                  // dwords per level and channel (V)
        const unsigned vm = 0xffffffffu / (unsigned)vgap + 1u;   // col / vgap == mulhi(col, vm) (col * vgap < 2^32)
        for (int e = tid; e < 32 * zn * vgap; e += 256) {
            const int d = e & 31, col = e >> 5;
            const int hz = (int)__umulhi((unsigned)col, vm), o = col - hz * vgap;
            ((unsigned *)(Vt + d * VSB + (hz * YR + yn) * XW))[o] = 0u;
        }
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int y0g = y0 + 2 * (wave & 1);
    const int gxa = 2 * (wave >> 1);
    const int zq = z0 + (r16 >> 2), yq = y0g + ((r16 >> 1) & 1);
    const int xrel = r16 & 1;
    const int zc = min(zq, p.Z - 1), yc = min(yq, p.Y - 1);

    int ylg, yng;
    clamp_range(min(y0g, p.Y - 1), 2, p.Y, KY, ylg, yng);
    const int dy = ylg - ylo;
    const int wz = win_start(zc, p.Z, KZ, false) - zlo;
    const int wy = win_start(yc, p.Y, KY, false) - ylg;
    const int zb = zlo - zc + KZ - 1;
    const int yb = ylg - yc + KY - 1;
    bool oky[2][2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            oky[hf][j] = (unsigned)(4 * hf + 2 * j + (g >> 1) - wy) < (unsigned)KY;
    const int tb_lane = (zb * BY + yb + (g >> 1)) * XT + 4 * (g & 1) - xrel + 1;

    // K fragment (key 16j + r16 = lat row 4hf + 2j + (r16 >> 3), lon column
    // r16 & 7 of the group halo; channels 8g..8g+7): lane base at level 0.
    const int kbase = ((r16 >> 3) + dy) * KRS + ((r16 & 7) + GX * gxa) * 32 + 8 * g;
    // V^T fragment (channel r16; keys 4g..4g+3 of lat row 2j + (g >> 1)):
    // lane base of group 0 at level 0; group 1 sits 2 bytes further and is
    // cut out of the same two dwords.
    const int vbase = r16 * VSB + ((g >> 1) + dy) * XW + 4 * (g & 1) + GX * gxa;

    long qf[2];
    long qtok[2];
    bool act[2];
    const float mulq = q_mul(aq);
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        const int xq = x0 + GX * (gxa + G) + xrel;
        act[G] = zq < p.Z && yq < p.Y && xq < p.X;
        const int xc = min(xq, p.X - 1);
        qtok[G] = (long)mul24(mul24((unsigned)zc, (unsigned)p.Y) + (unsigned)yc, (unsigned)p.X) + xc;
        const uint2 q8 = bf16x8_to_e4m3(*(const uint4 *)(qb + qtok[G] * p.ts + 8 * g), mulq);
        qf[G] = (long)(((unsigned long long)q8.y << 32) | q8.x);
    }

    f32x4 oacc[2][2], lacc[2];
    float mref[2], thr[2], nmc[2];
    const float tau_raw = TAU / c;
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        oacc[G][0] = oacc[G][1] = lacc[G] = f32x4{0.f, 0.f, 0.f, 0.f};
        mref[G] = -1e30f;
        thr[G] = -1e30f;
        nmc[G] = 0.f;
    }
    const long ones = 0x3838383838383838L;   // e4m3 1.0 in every byte

    for (int hz = 0; hz < zn; ++hz) {
        const bool okz = (unsigned)(hz - wz) < (unsigned)KZ;
        const unsigned char *kz = Ks + kbase + hz * YR * KRS;
        const unsigned char *vz0 = Vt + vbase + hz * YR * XW;
        const unsigned char *vz1 = vz0 + 16 * VSB;
        const int tbh = tb_lane + hz * BY * XT;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            f32x4 binit[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int a = (okz && oky[hf][j]) ? tbh : TBL;
                const float *tp = tbl + a + (4 * hf + 2 * j) * XT;
#pragma unroll
                for (int i = 0; i < 4; ++i) binit[j][i] = tp[i];
            }
            f32x4 s[2][2];
            float cm[2];
#pragma unroll
            for (int G = 0; G < 2; ++G)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const long kf = *(const long *)(kz + (4 * hf + 2 * j) * KRS + GX * 32 * G);
                    s[G][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(kf, qf[G], binit[j], 0, 0, 0);
                }
#pragma unroll
            for (int G = 0; G < 2; ++G)
                cm[G] = max3f(max3f(s[G][0][0], s[G][0][1], s[G][0][2]), max3f(s[G][0][3], s[G][1][0], s[G][1][1]),
                              max2f(s[G][1][2], s[G][1][3]));
            if (__builtin_amdgcn_ballot_w64(cm[0] > thr[0] || cm[1] > thr[1])) {
#pragma unroll
                for (int G = 0; G < 2; ++G) {
                    const float mn = max2f(mref[G], xmax16_32(cm[G]));
                    const float al = __builtin_amdgcn_exp2f(c * (mref[G] - mn));
                    mref[G] = mn;
                    thr[G] = mn + tau_raw;
                    nmc[G] = -c * mn;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        oacc[G][0][i] *= al;
                        oacc[G][1][i] *= al;
                        lacc[G][i] *= al;
                    }
                }
            }
            long pf[2];
#pragma unroll
            for (int G = 0; G < 2; ++G) {
                float pv[8];
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) pv[4 * j + i] = __builtin_amdgcn_exp2f(fmaf(s[G][j][i], c, nmc[G]));
                unsigned lo = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[0], pv[1], 0, false);
                lo = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[2], pv[3], (int)lo, true);
                unsigned hi = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[4], pv[5], 0, false);
                hi = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(pv[6], pv[7], (int)hi, true);
                pf[G] = (long)(((unsigned long long)hi << 32) | lo);
            }
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const unsigned char *vz = tt ? vz1 : vz0;
                const unsigned d0 = *(const unsigned *)(vz + (4 * hf) * XW);
                const unsigned d1 = *(const unsigned *)(vz + (4 * hf) * XW + 4);
                const unsigned d2 = *(const unsigned *)(vz + (4 * hf + 2) * XW);
                const unsigned d3 = *(const unsigned *)(vz + (4 * hf + 2) * XW + 4);
                const long v0 = (long)(((unsigned long long)d2 << 32) | d0);
                const long v1 = (long)(((unsigned long long)__builtin_amdgcn_alignbyte(d3, d2, 2) << 32) |
                                       __builtin_amdgcn_alignbyte(d1, d0, 2));
                oacc[0][tt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(v0, pf[0], oacc[0][tt], 0, 0, 0);
                oacc[1][tt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(v1, pf[1], oacc[1][tt], 0, 0, 0);
            }
#pragma unroll
            for (int G = 0; G < 2; ++G)
                lacc[G] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ones, pf[G], lacc[G], 0, 0, 0);
        }
    }

    const float sv = dq_scale(av);
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        if (!act[G]) continue;
        const float inv = sv / lacc[G][0];
        bf16 *ob = (bf16 *)p.out + (size_t)b * p.obs + (size_t)qtok[G] * p.ots + h * 32;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            f32x4 v = oacc[G][tt];
            uint2 u;
            u.x = pack_bf16x2(v[0] * inv, v[1] * inv);
            u.y = pack_bf16x2(v[2] * inv, v[3] * inv);
            *(uint2 *)(ob + 16 * tt + 4 * g) = u;
        }
    }
}

// Largest halo extent of a clamped axis over the tiles of size tsize.
int max_halo(int N, int K, int tsize) {
    int m = 0;
    for (int a0 = 0; a0 < N; a0 += tsize) {
        const int last = std::min(a0 + tsize - 1, N - 1);
        const int lo = win_start(a0, N, K, false);
        m = std::max(m, win_start(last, N, K, false) + K - lo);
    }
    return m;
}

size_t tile_lds(int Kz, int Ky, int zw, int yr) {
    const int tblp = (((2 * Kz - 1) * (2 * Ky - 1) * XT + NEG_RUN + 3) & ~3);
    return (size_t)tblp * 4 + (size_t)zw * yr * 1024;     // table + V halo slabs
}

template <int KZ, int KY, int KX, bool QSCALED>
hipError_t launch_tile_q(const NatArgs &a, hipStream_t stream) {
    const int zw = max_halo(a.Z, KZ, TZ), yr = std::max(max_halo(a.Y, KY, TY), YR_MIN);
    const size_t lds = tile_lds(KZ, KY, zw, yr);
    // set once per process (thread-safe local static initialisation)
    static const hipError_t attr_err = hipFuncSetAttribute((const void *)nat_tile_kernel<KZ, KY, KX, QSCALED>,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr_err != hipSuccess) return attr_err;
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    if (!a.tbl_ready) nat_bias_prep<KZ, KY, KX, QSCALED><<<(a.H * TBLP + 255) / 256, 256, 0, stream>>>(a);
    const int ntiles = ((a.Z + TZ - 1) / TZ) * ((a.Y + TY - 1) / TY) * ((a.X + TX - 1) / TX);
    const long total = (long)ntiles * a.H * a.B;
    const unsigned grid = (unsigned)(((total + 7) >> 3) << 3);
    nat_tile_kernel<KZ, KY, KX, QSCALED><<<grid, 256, lds, stream>>>(a, zw, yr, tile_div(a));
    return hipGetLastError();
}

size_t ring_lds(int Kz, int Ky) {
    const int tblp = (((2 * Kz - 1) * (2 * Ky - 1) * XT + NEG_RUN + 3) & ~3);
    return (size_t)tblp * 4 + 2 * (size_t)RING_SLOT;
}

template <int KZ, int KY, int KX, bool QSCALED>
hipError_t launch_ring(const NatArgs &a, hipStream_t stream) {
    // exactly the dynamic size: the kernel also holds a little static LDS (__syncthreads_or)
    static const hipError_t attr_err = hipFuncSetAttribute((const void *)nat_ring_kernel<KZ, KY, KX, QSCALED>,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                                           (int)ring_lds(KZ, KY));
    if (attr_err != hipSuccess) return attr_err;
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    if (!a.tbl_ready) nat_bias_prep<KZ, KY, KX, QSCALED><<<(a.H * TBLP + 255) / 256, 256, 0, stream>>>(a);
    const int ntiles = ((a.Z + TZ - 1) / TZ) * ((a.Y + TY - 1) / TY) * ((a.X + TX - 1) / TX);
    const long total = (long)ntiles * a.H * a.B;
    const unsigned grid = (unsigned)(((total + 7) >> 3) << 3);
    nat_ring_kernel<KZ, KY, KX, QSCALED><<<grid, 256, ring_lds(KZ, KY), stream>>>(a, tile_div(a));
    return hipGetLastError();
}

// v [B][T][H][32] (strides bs, ts, hs) -> the blocked layout: one thread per
// (head, state, level, lat, block of 4 positions, 8 channels).
__global__ void v_blocked_kernel(const bf16 *__restrict__ v, long bs, long ts, long hs, bf16 *__restrict__ out,
                                 int B, int Z, int Y, int X, int H, int xp) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nxb = xp >> 2;
    const long total = (long)H * B * Z * Y * nxb * 4;
    if (e >= total) return;
    const int c = (int)(e & 3);
    long r = e >> 2;
    const int xb = (int)(r % nxb); r /= nxb;
    const long zyb = r;                          // ((h B + b) Z + z) Y + y
    const int y = (int)(r % Y); r /= Y;
    const int z = (int)(r % Z); r /= Z;
    const int b = (int)(r % B);
    const int h = (int)(r / B);
    uint4 u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int x = 4 * xb + k - 4;
        x = ((x % X) + X) % X;
        u[k] = *(const uint4 *)(v + (size_t)b * bs + (((size_t)z * Y + y) * X + x) * ts + (size_t)h * hs + 8 * c);
    }
    const unsigned w0[4] = {u[0].x, u[0].y, u[0].z, u[0].w}, w1[4] = {u[1].x, u[1].y, u[1].z, u[1].w};
    const unsigned w2[4] = {u[2].x, u[2].y, u[2].z, u[2].w}, w3[4] = {u[3].x, u[3].y, u[3].z, u[3].w};
    uint2 *dst = (uint2 *)(out + ((size_t)zyb * nxb + xb) * 128 + (8 * c) * 4);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dst[2 * k] = make_uint2(__builtin_amdgcn_perm(w1[k], w0[k], 0x05040100u), __builtin_amdgcn_perm(w3[k], w2[k], 0x05040100u));
        dst[2 * k + 1] = make_uint2(__builtin_amdgcn_perm(w1[k], w0[k], 0x07060302u), __builtin_amdgcn_perm(w3[k], w2[k], 0x07060302u));
    }
}

size_t tile_lds_fp8(int Kz, int Ky, int zw, int yr) {
    const int tblp = (((2 * Kz - 1) * (2 * Ky - 1) * XT + NEG_RUN + 3) & ~3);
    return (size_t)tblp * 4 + (size_t)zw * yr * KRS + 32 * (size_t)vt_row_bytes(zw, yr);
}

template <int KZ, int KY, int KX>
hipError_t launch_tile_fp8(const NatArgs &a, hipStream_t stream) {
    const int zw = max_halo(a.Z, KZ, TZ), yr = std::max(max_halo(a.Y, KY, TY), YR_MIN);
    const size_t lds = tile_lds_fp8(KZ, KY, zw, yr);
    // set once per process (thread-safe local static initialisation)
    static const hipError_t attr_err = hipFuncSetAttribute((const void *)nat_tile_fp8_kernel<KZ, KY, KX>,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr_err != hipSuccess) return attr_err;
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    nat_bias_prep_fp8<KZ, KY, KX><<<(a.B * a.H * TBLP + 255) / 256, 256, 0, stream>>>(a);
    const int ntiles = ((a.Z + TZ - 1) / TZ) * ((a.Y + TY - 1) / TY) * ((a.X + TX - 1) / TX);
    const long total = (long)ntiles * a.H * a.B;
    const unsigned grid = (unsigned)(((total + 7) >> 3) << 3);
    nat_tile_fp8_kernel<KZ, KY, KX><<<grid, 256, lds, stream>>>(a, zw, yr, tile_div(a));
    return hipGetLastError();
}

size_t ring8_lds(int Kz, int Ky) {
    const int tblp = (((2 * Kz - 1) * (2 * Ky - 1) * XT + NEG_RUN + 3) & ~3);
    return (size_t)tblp * 4 + 3 * (size_t)RING8_SLOT;
}

template <int KZ, int KY, int KX>
hipError_t launch_ring_fp8(const NatArgs &a, hipStream_t stream) {
    // exactly the dynamic size: the kernel also holds a little static LDS (__syncthreads_or)
    static const hipError_t attr_err = hipFuncSetAttribute((const void *)nat_ring_fp8_kernel<KZ, KY, KX>,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                                           (int)ring8_lds(KZ, KY));
    if (attr_err != hipSuccess) return attr_err;
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    nat_bias_prep_fp8<KZ, KY, KX><<<(a.B * a.H * TBLP + 255) / 256, 256, 0, stream>>>(a);
    const int ntiles = ((a.Z + TZ - 1) / TZ) * ((a.Y + TY - 1) / TY) * ((a.X + TX - 1) / TX);
    const long total = (long)ntiles * a.H * a.B;
    const unsigned grid = (unsigned)(((total + 7) >> 3) << 3);
    nat_ring_fp8_kernel<KZ, KY, KX><<<grid, 256, ring8_lds(KZ, KY), stream>>>(a, tile_div(a));
    return hipGetLastError();
}

template <int KZ, int KY, int KX>
hipError_t launch_tile(const NatArgs &a, hipStream_t stream) {
    if (a.amax && a.vt) return launch_ring_fp8<KZ, KY, KX>(a, stream);
    if (a.q8 || a.o8) return hipErrorInvalidValue;   // e4m3 q / o: the level-ring kernel only
    if (a.amax) return launch_tile_fp8<KZ, KY, KX>(a, stream);
    if (a.vt) {
        if (a.qscale == 1.0f) return launch_ring<KZ, KY, KX, true>(a, stream);
        return launch_ring<KZ, KY, KX, false>(a, stream);
    }
    if (a.qscale == 1.0f) return launch_tile_q<KZ, KY, KX, true>(a, stream);
    return launch_tile_q<KZ, KY, KX, false>(a, stream);
}

}  // namespace

size_t nat_tile_lds_bytes(const NatArgs &a) {
    if (a.periodic != 0x4) return 0;
    const bool known = (a.Kz == 5 && a.Ky == 7 && a.Kx == 7) || (a.Kz == 3 && a.Ky == 5 && a.Kx == 5) ||
                       (a.Kz == 3 && a.Ky == 3 && a.Kx == 3);
    if (!known) return 0;
    if (a.X < TX + a.Kx - 1) return 0;     // the lon halo must not wrap onto itself
    if (!a.tbl_ws) return 0;
    // K and V are addressed with 32-bit byte offsets from the state's base,
    // rows and tokens with 24-bit products
    if ((long)a.Z * a.Y * a.X * a.ts * 2 >= (1L << 31)) return 0;
    if ((long)a.X * a.ts * 2 >= (1L << 24) || (long)a.Z * a.Y >= (1L << 24)) return 0;
    {   // workgroup-id divisions by multiply-high (tile_div) are exact while id * d < 2^32
        const long nt[4] = {(a.X + TX - 1) / TX, (a.Y + TY - 1) / TY, (a.Z + TZ - 1) / TZ, a.H};
        const long total = nt[0] * nt[1] * nt[2] * a.H * a.B;
        for (long d : nt)
            if (total * d >= (1L << 32)) return 0;
    }
    if (a.vt) {
        // blocked V: every halo row must be one in-range run, and a (head,
        // state) plane must be addressable with 32-bit offsets
        if (a.xp < v_blocked_xp(a.X)) return 0;
        if ((long)a.Z * a.Y * a.xp * 64 >= (1L << 31)) return 0;
        if (a.amax && a.B > 64) return 0;
        return a.amax ? ring8_lds(a.Kz, a.Ky) : ring_lds(a.Kz, a.Ky);
    }
    const int zw = max_halo(a.Z, a.Kz, TZ), yr = std::max(max_halo(a.Y, a.Ky, TY), YR_MIN);
    return a.amax ? tile_lds_fp8(a.Kz, a.Ky, zw, yr) : tile_lds(a.Kz, a.Ky, zw, yr);
}

template <int KZ, int KY, int KX>
hipError_t bias_table_only(const NatArgs &a, hipStream_t stream) {
    constexpr int TBLP = tbl_padded<KZ, KY, KX>();
    nat_bias_prep<KZ, KY, KX, true><<<(a.H * TBLP + 255) / 256, 256, 0, stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_nat_bias_table(const NatArgs &a, hipStream_t stream) {
    if (a.qscale != 1.0f || a.bscale != 1.0f || !a.tbl_ws || a.H < 1) return hipErrorInvalidValue;
    if (a.Kz == 5 && a.Ky == 7 && a.Kx == 7) return bias_table_only<5, 7, 7>(a, stream);
    if (a.Kz == 3 && a.Ky == 5 && a.Kx == 5) return bias_table_only<3, 5, 5>(a, stream);
    if (a.Kz == 3 && a.Ky == 3 && a.Kx == 3) return bias_table_only<3, 3, 3>(a, stream);
    return hipErrorNotSupported;
}

hipError_t launch_kv8(const NatArgs &a, unsigned char *k8, unsigned char *v8, hipStream_t stream) {
    if (!a.amax || (a.xp & 3)) return hipErrorInvalidValue;
    const long T = (long)a.Z * a.Y * a.X;
    const long nk = (long)a.B * T * a.H * 4, nv = (long)a.H * a.B * a.Z * a.Y * (a.xp / 4) * 4;
    if (nk > 0x7fffffffL || nv > 0x7fffffffL) return hipErrorInvalidValue;
    if (nk) k8_kernel<<<(unsigned)((nk + 255) / 256), 256, 0, stream>>>((const bf16 *)a.k, a.bs, a.ts, a.hs, k8, a.B, T,
                                                                      a.H, a.amax, a.amax_stride);
    if (nv) v8_blocked_kernel<<<(unsigned)((nv + 255) / 256), 256, 0, stream>>>((const bf16 *)a.v, a.bs, a.ts, a.hs, v8,
                                                                              a.B, a.Z, a.Y, a.X, a.H, a.xp, a.amax,
                                                                              a.amax_stride);
    return hipGetLastError();
}

hipError_t launch_v_blocked(const NatArgs &a, void *out, hipStream_t stream) {
    const long total = (long)a.H * a.B * a.Z * a.Y * (a.xp / 4) * 4;
    if (total == 0) return hipSuccess;
    if ((a.xp & 3) || total > 0x7fffffffL) return hipErrorInvalidValue;
    v_blocked_kernel<<<(unsigned)((total + 255) / 256), 256, 0, stream>>>((const bf16 *)a.v, a.bs, a.ts, a.hs, (bf16 *)out,
                                                                        a.B, a.Z, a.Y, a.X, a.H, a.xp);
    return hipGetLastError();
}

hipError_t launch_nat_tile(const NatArgs &a, hipStream_t stream) {
    if (a.Kz == 5 && a.Ky == 7 && a.Kx == 7) return launch_tile<5, 7, 7>(a, stream);
    if (a.Kz == 3 && a.Ky == 5 && a.Kx == 5) return launch_tile<3, 5, 5>(a, stream);
    if (a.Kz == 3 && a.Ky == 3 && a.Kx == 3) return launch_tile<3, 3, 3>(a, stream);
    return hipErrorNotSupported;
}

}  // namespace wm
