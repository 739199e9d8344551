// LDS-tiled bf16 neighborhood attention for lon-periodic, lat/level-clamped
// grids (the WeatherMesh-3 setting, Sec. 2.1 NATTEN and App. A.2).
//
// Workgroup = 256 threads, one head, a query tile of 4 levels x 4 lats x
// 8 lons (128 queries = 8 groups of 4x2x2).  The union of the tile's
// windows (the halo: <= 6 x 10 x 14 tokens at 8 levels and a 5x7x7 window)
// is staged once in LDS -- K row-major with 16-byte chunks swizzled, V
// transposed (d-major) -- and shared by all 8 query groups.  Each wave owns
// two groups with the same level/lat window pattern, so they share the
// relative-position-bias lookups.
//
// Per group the halo is walked in chunks of 32 keys = 4 lat rows x 8 lon
// columns at one level.  A chunk costs 5 MFMA:
//   S^T = K . Q^T + B        2 x 16x16x32 (the bias-and-mask tile B is the
//                            accumulator input: masked keys enter as -inf)
//   O^T += V^T . P^T         2 x 16x16x32
//   l   += 1 . P^T           1 x 16x16x32 (row sums of the bf16 weights)
// The softmax runs in base 2 with a lazily updated reference maximum:
// the weights are exp2(s - m_ref) and m_ref (with the accumulators) is only
// moved when a chunk's maximum exceeds it by more than 8, so the weights
// stay <= 256 and most chunks need no rescaling.  Max and sums are float32.
//
// Layout facts used (lane l, g = l/16, r = l%16) for the gfx950 bf16 MFMA
// 16x16x32: A[r][8g..8g+7], B[8g..8g+7][r], D[4g..4g+3][r].  A lane's
// scores in a chunk are keys {4g+i, 16+4g+i}; the P.V contraction takes its
// k index in that order (k-slot 8g + 4j + i <-> key 16j + 4g + i).
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

__device__ __forceinline__ int kswz(int row, int x) { return ((x >> 2) ^ row) & 3; }

__device__ __forceinline__ void clamp_range(int a0, int tsize, int N, int K, int &lo, int &n) {
    const int last = min(a0 + tsize - 1, N - 1);
    lo = win_start(a0, N, K, false);
    n = win_start(last, N, K, false) + K - lo;
}

// QSCALED: q already carries the factor log2(e)/sqrt(d) (the block path folds
// it into the QKV projection); otherwise scores are scaled after the MFMA and
// the bias table is stored divided by the scale.
template <int KZ, int KY, int KX, bool QSCALED>
__global__ __launch_bounds__(256, 1) void nat_tile_kernel(NatArgs p, int ZWmax, int YWmax) {
    constexpr int RX = (KX - 1) / 2;
    constexpr int BY = 2 * KY - 1;
    constexpr int BZ = 2 * KZ - 1;
    constexpr int NCH = 2 * (4 + KZ - 1);           // max chunks per group
    constexpr int TBL = BZ * BY * XT;               // bias table entries
    static_assert(2 + KX - 1 <= 8 && 2 + KY - 1 <= 8, "window too large for 8-wide group halo");

    extern __shared__ __align__(16) unsigned char smem[];
    float *tbl = (float *)smem;                                  // [BZ][BY][XT] + 4 of -inf
    const int tbl_bytes = ((TBL + 4) * 4 + 15) & ~15;
    const int nslot_max = ZWmax * YWmax * XW;
    uint4 *Ks = (uint4 *)(smem + tbl_bytes);                     // [slot][4 chunks]
    unsigned short *Vt = (unsigned short *)(smem + tbl_bytes + nslot_max * 64);  // [32][nslot]

    // ---- tile of this workgroup (XCD-aware order over (b, h, tile)) ----
    const int ntz = (p.Z + TZ - 1) / TZ, nty = (p.Y + TY - 1) / TY, ntx = (p.X + TX - 1) / TX;
    const int ntiles = ntz * nty * ntx;
    const int total = ntiles * p.H * p.B;
    const int per = (total + 7) >> 3;
    const int L = blockIdx.x;
    const int id = (L & 7) * per + (L >> 3);
    if (id >= total) return;
    int t = id;
    const int tx = t % ntx; t /= ntx;
    const int ty = t % nty; t /= nty;
    const int tz = t % ntz; t /= ntz;
    const int h = t % p.H;
    const int b = t / p.H;
    const int z0 = tz * TZ, y0 = ty * TY, x0 = tx * TX;

    int zlo, zn, ylo, yn;
    clamp_range(z0, TZ, p.Z, KZ, zlo, zn);
    clamp_range(y0, TY, p.Y, KY, ylo, yn);
    const int xlo = x0 - RX;                       // periodic lon
    const int nslot = zn * yn * XW;

    const bf16 *kb = (const bf16 *)p.k + (size_t)b * p.bs + (size_t)h * p.hs;
    const bf16 *vb = (const bf16 *)p.v + (size_t)b * p.bs + (size_t)h * p.hs;
    const bf16 *qb = (const bf16 *)p.q + (size_t)b * p.bs + (size_t)h * p.hs;
    const int tid = threadIdx.x;

    // ---- bias table: tbl[iz][iy][ixt], lon validity folded in ----
    {
        const float *r = p.rpb + (size_t)h * BZ * BY * (2 * KX - 1);
        const float bs = QSCALED ? p.bscale : p.bscale / p.qscale;
        for (int e = tid; e < TBL + 4; e += 256) {
            float v = -INFINITY;
            if (e < TBL) {
                const int ixt = e % XT, rest = e / XT;
                const int dx = ixt - 1 - RX;              // hx - xq_rel - r
                if (dx >= -RX && dx <= RX) v = r[rest * (2 * KX - 1) + dx + KX - 1] * bs;
            }
            tbl[e] = v;
        }
    }
    // ---- K and V halo: slot = (hz * yn + hy) * XW + hx ----
    for (int e = tid; e < nslot * 4; e += 256) {
        const int slot = e >> 2, c = e & 3;
        const int hx = slot % XW, row = slot / XW;
        const int hy = row % yn, hz = row / yn;
        int xx = (xlo + (hx < TX + KX - 1 ? hx : 0)) % p.X;
        xx = xx < 0 ? xx + p.X : xx;
        const long tok = ((long)(zlo + hz) * p.Y + (ylo + hy)) * p.X + xx;
        const uint4 kv = *(const uint4 *)(kb + tok * p.ts + 8 * c);
        Ks[slot * 4 + (c ^ kswz(row, hx))] = kv;
        const uint4 vv = *(const uint4 *)(vb + tok * p.ts + 8 * c);
        const unsigned w[4] = {vv.x, vv.y, vv.z, vv.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Vt[(8 * c + 2 * q) * nslot + slot] = (unsigned short)(w[q] & 0xffffu);
            Vt[(8 * c + 2 * q + 1) * nslot + slot] = (unsigned short)(w[q] >> 16);
        }
    }
    __syncthreads();

    // ---- per wave: lat group (wave & 1), lon groups 2*(wave>>1) + {0,1} ----
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int y0g = y0 + 2 * (wave & 1);
    const int gxa = 2 * (wave >> 1);
    const int zq = z0 + (r16 >> 2), yq = y0g + ((r16 >> 1) & 1);
    const int xrel = r16 & 1;
    const int zc = min(zq, p.Z - 1), yc = min(yq, p.Y - 1);

    int zlg, zng, ylg, yng;
    clamp_range(z0, 4, p.Z, KZ, zlg, zng);
    clamp_range(min(y0g, p.Y - 1), 2, p.Y, KY, ylg, yng);
    const int nch = 2 * zng;
    const int dz = zlg - zlo, dy = ylg - ylo;
    const int wz = win_start(zc, p.Z, KZ, false) - zlg;
    const int wy = win_start(yc, p.Y, KY, false) - ylg;
    const int zb = zlg - zc + KZ - 1;
    const int yb = ylg - yc + KY - 1;

    // validity of (level row hz, lat row hy) for this lane's query
    unsigned vmask = 0;     // bit 2c + j
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int hz = c >> 1, hy = 4 * (c & 1) + 2 * j + (g >> 1);
            const bool ok = c < nch && (unsigned)(hz - wz) < (unsigned)KZ && (unsigned)(hy - wy) < (unsigned)KY;
            vmask |= (ok ? 1u : 0u) << (2 * c + j);
        }
    const int tb_lane = (zb * BY + yb + (g >> 1)) * XT + 4 * (g & 1) - xrel + 1;

    // lat rows (clamped into the halo) for the K operand and the V operand
    int krow[4], vrow[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int hy_k = 4 * (q >> 1) + 2 * (q & 1) + (r16 >> 3);
        const int hy_v = 4 * (q >> 1) + 2 * (q & 1) + (g >> 1);
        krow[q] = min(hy_k + dy, yn - 1);
        vrow[q] = min(hy_v + dy, yn - 1);
    }

    // Q fragments of the two groups
    bf16x8 qf[2];
    long qtok[2];
    bool act[2];
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        const int xq = x0 + GX * (gxa + G) + xrel;
        act[G] = zq < p.Z && yq < p.Y && xq < p.X;
        const int xc = min(xq, p.X - 1);
        qtok[G] = ((long)zc * p.Y + yc) * p.X + xc;
        qf[G] = *(const bf16x8 *)(qb + qtok[G] * p.ts + 8 * g);
    }

    f32x4 oacc[2][2], lacc[2];
    float mref[2];
#pragma unroll
    for (int G = 0; G < 2; ++G) {
        oacc[G][0] = oacc[G][1] = lacc[G] = f32x4{0.f, 0.f, 0.f, 0.f};
        mref[G] = -1e30f;
    }
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = __builtin_bit_cast(bf16, (unsigned short)0x3f80);

#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (c >= nch) break;
        const int hz = (c >> 1) + dz;
        // bias + mask tile (shared by both groups)
        f32x4 binit[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const bool ok = (vmask >> (2 * c + j)) & 1u;
            const int a = ok ? tb_lane + (c >> 1) * BY * XT + (4 * (c & 1) + 2 * j) * XT : TBL;
#pragma unroll
            for (int i = 0; i < 4; ++i) binit[j][i] = tbl[a + i];
        }
        bf16x8 pb[2];
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            const int xg = GX * (gxa + G);          // group lon offset in the halo
            f32x4 s[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = hz * yn + krow[(c & 1) * 2 + j];
                const int hx = (r16 & 7) + xg;
                const int slot = row * XW + hx;
                const bf16x8 kf = __builtin_bit_cast(bf16x8, Ks[slot * 4 + (g ^ kswz(row, hx))]);
                s[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kf, qf[G], binit[j], 0, 0, 0);
                if constexpr (!QSCALED) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) s[j][i] *= p.qscale;
                }
            }
            float cm = fmaxf(fmaxf(fmaxf(s[0][0], s[0][1]), fmaxf(s[0][2], s[0][3])),
                             fmaxf(fmaxf(s[1][0], s[1][1]), fmaxf(s[1][2], s[1][3])));
            cm = fmaxf(cm, __shfl_xor(cm, 16, 64));
            cm = fmaxf(cm, __shfl_xor(cm, 32, 64));
            if (__builtin_amdgcn_ballot_w64(cm > mref[G] + TAU)) {
                const float mn = fmaxf(mref[G], cm);
                const float al = exp2f(mref[G] - mn);
                mref[G] = mn;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    oacc[G][0][i] *= al;
                    oacc[G][1][i] *= al;
                    lacc[G][i] *= al;
                }
            }
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) pb[G][4 * j + i] = (bf16)exp2f(s[j][i] - mref[G]);
        }
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            const int xg = GX * (gxa + G);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const unsigned short *vrowp = Vt + (16 * tt + r16) * nslot;
                bf16x8 vf;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int slot = (hz * yn + vrow[(c & 1) * 2 + j]) * XW + 4 * (g & 1) + xg;
                    const unsigned w0 = *(const unsigned *)(vrowp + slot);
                    const unsigned w1 = *(const unsigned *)(vrowp + slot + 2);
                    vf[4 * j + 0] = __builtin_bit_cast(bf16, (unsigned short)(w0 & 0xffffu));
                    vf[4 * j + 1] = __builtin_bit_cast(bf16, (unsigned short)(w0 >> 16));
                    vf[4 * j + 2] = __builtin_bit_cast(bf16, (unsigned short)(w1 & 0xffffu));
                    vf[4 * j + 3] = __builtin_bit_cast(bf16, (unsigned short)(w1 >> 16));
                }
                oacc[G][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vf, pb[G], oacc[G][tt], 0, 0, 0);
            }
            lacc[G] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ones, pb[G], lacc[G], 0, 0, 0);
        }
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
            u.x = (unsigned)f2bf_bits(v[0] * inv) | ((unsigned)f2bf_bits(v[1] * inv) << 16);
            u.y = (unsigned)f2bf_bits(v[2] * inv) | ((unsigned)f2bf_bits(v[3] * inv) << 16);
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

size_t tile_lds(int Kz, int Ky, int zw, int yw) {
    const int tbl = (2 * Kz - 1) * (2 * Ky - 1) * XT;
    return (((tbl + 4) * 4 + 15) & ~15) + (size_t)zw * yw * XW * 128;
}

template <int KZ, int KY, int KX, bool QSCALED>
hipError_t launch_tile_q(const NatArgs &a, hipStream_t stream) {
    const int zw = max_halo(a.Z, KZ, TZ), yw = max_halo(a.Y, KY, TY);
    const size_t lds = tile_lds(KZ, KY, zw, yw);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)nat_tile_kernel<KZ, KY, KX, QSCALED>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int ntiles = ((a.Z + TZ - 1) / TZ) * ((a.Y + TY - 1) / TY) * ((a.X + TX - 1) / TX);
    const long total = (long)ntiles * a.H * a.B;
    const unsigned grid = (unsigned)(((total + 7) >> 3) << 3);
    nat_tile_kernel<KZ, KY, KX, QSCALED><<<grid, 256, lds, stream>>>(a, zw, yw);
    return hipGetLastError();
}

template <int KZ, int KY, int KX>
hipError_t launch_tile(const NatArgs &a, hipStream_t stream) {
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
    if ((long)a.Z * a.Y * a.X * a.B > (1L << 30)) return 0;
    return tile_lds(a.Kz, a.Ky, max_halo(a.Z, a.Kz, TZ), max_halo(a.Y, a.Ky, TY));
}

hipError_t launch_nat_tile(const NatArgs &a, hipStream_t stream) {
    if (a.Kz == 5 && a.Ky == 7 && a.Kx == 7) return launch_tile<5, 7, 7>(a, stream);
    if (a.Kz == 3 && a.Ky == 5 && a.Kx == 5) return launch_tile<3, 5, 5>(a, stream);
    if (a.Kz == 3 && a.Ky == 3 && a.Kx == 3) return launch_tile<3, 3, 3>(a, stream);
    return hipErrorNotSupported;
}

}  // namespace wm
