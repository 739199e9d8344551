// 3-D neighborhood attention with relative-position bias on MFMA.
//
// WeatherMesh-3 Sec. 2.1 (NATTEN) and App. A.2: every latent token attends
// to the Kz x Ky x Kx box around it over (level, lat, lon); lon wraps, lat
// and level windows keep their size and shift inward at the borders.
//
// Work split: one wave owns a group of 16 queries -- 4 levels x 2 lats x
// 2 lons -- and one head.  The union of the 16 windows (the group halo) is
// walked in chunks of 32 keys.  Per chunk:
//   S^T[32 keys x 16 queries] = K_chunk . Q^T       (MFMA, d = 32 contracted)
//   mask + bias, online softmax in float32 (base-2 exponent)
//   O^T[32 d x 16 queries] += V^T_chunk . P^T         (MFMA, keys contracted)
// Computing S transposed makes each lane own one query column in both the
// score tile and the output tile, so the softmax state (running max, sum)
// of a query lives in the 4 lanes l, l^16, l^32, l^48.
//
// MFMA lane layouts (16x16 tiles; lane l, g = l/16, r = l%16):
//   bf16 16x16x32: A[r][8g..8g+7], B[8g..8g+7][r], D[4g..4g+3][r]
//   f32  16x16x4 : A[r][g],        B[g][r],        D[4g..4g+3][r]
// A lane's 8 scores in a chunk are keys {4g..4g+3, 16+4g..16+4g+3}; the
// P.V contraction takes its k index in that same order (k-slot 8g + 4j + i
// <-> key 16j + 4g + i), so the score registers feed the second MFMA
// without any data movement.
#include <cmath>

#include "kernels.hpp"

namespace wm {
namespace {

constexpr int GZ = 4, GY = 2, GX = 2;   // query group shape (16 queries)

struct Axis {
    int lo;      // first halo coordinate (may be negative on a periodic axis)
    int n;       // halo length
    int ws;      // this lane's window start, in halo slots
    int boff;    // bias index of halo slot s = s + boff
    int N;       // axis length
    bool per;
};

__device__ __forceinline__ Axis make_axis(int g0, int gsize, int qi, int N, int K, bool per) {
    Axis a;
    a.N = N;
    a.per = per;
    const int r = (K - 1) >> 1;
    if (per) {
        a.lo = g0 - r;
        a.n = gsize + K - 1;
        a.ws = qi - g0;
        a.boff = r - a.ws;
    } else {
        const int last = min(g0 + gsize - 1, N - 1);
        a.lo = win_start(g0, N, K, false);
        a.n = win_start(last, N, K, false) + K - a.lo;
        a.ws = win_start(qi, N, K, false) - a.lo;
        a.boff = a.lo - qi + K - 1;
    }
    return a;
}

__device__ __forceinline__ int coord(const Axis &a, int s) {
    int c = a.lo + s;
    if (a.per) {
        c %= a.N;
        c = c < 0 ? c + a.N : c;
    }
    return c;
}

template <typename T>
__global__ __launch_bounds__(256) void nat_generic_kernel(NatArgs p) {
    const int ngz = (p.Z + GZ - 1) / GZ, ngy = (p.Y + GY - 1) / GY, ngx = (p.X + GX - 1) / GX;
    const long ngroups = (long)ngz * ngy * ngx;
    const long total = ngroups * p.H * p.B;
    const long wid = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= total) return;
    const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;

    long t = wid;
    const int gx = (int)(t % ngx); t /= ngx;
    const int gy = (int)(t % ngy); t /= ngy;
    const int gz = (int)(t % ngz); t /= ngz;
    const int h = (int)(t % p.H); t /= p.H;
    const int b = (int)t;
    const int z0 = gz * GZ, y0 = gy * GY, x0 = gx * GX;

    const int zq = z0 + (r16 >> 2), yq = y0 + ((r16 >> 1) & 1), xq = x0 + (r16 & 1);
    const bool active = zq < p.Z && yq < p.Y && xq < p.X;
    const int zc = min(zq, p.Z - 1), yc = min(yq, p.Y - 1), xc = min(xq, p.X - 1);

    const Axis az = make_axis(z0, GZ, zc, p.Z, p.Kz, p.periodic & 1);
    const Axis ay = make_axis(y0, GY, yc, p.Y, p.Ky, (p.periodic >> 1) & 1);
    const Axis ax = make_axis(x0, GX, xc, p.X, p.Kx, (p.periodic >> 2) & 1);
    const int nxp = (ax.n + 3) & ~3;
    const int nf = az.n * ay.n * nxp;
    const int nchunk = (nf + 31) >> 5;
    const int By = 2 * p.Ky - 1, Bx = 2 * p.Kx - 1;
    const float *rpb = p.rpb + (size_t)h * (2 * p.Kz - 1) * By * Bx;

    const T *qb = (const T *)p.q + (size_t)b * p.bs + (size_t)h * p.hs;
    const T *kb = (const T *)p.k + (size_t)b * p.bs + (size_t)h * p.hs;
    const T *vb = (const T *)p.v + (size_t)b * p.bs + (size_t)h * p.hs;
    const long qtok = ((long)zc * p.Y + yc) * p.X + xc;

    // Q fragment of this lane's query: d in [8g, 8g+8).
    float qf[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) qf[e] = Elt<T>::ld(qb + qtok * p.ts + 8 * g + e);

    const float NEG = -INFINITY;
    float m_run = -1e30f, l_run = 0.f;
    f32x4 o0 = {0.f, 0.f, 0.f, 0.f}, o1 = {0.f, 0.f, 0.f, 0.f};

    for (int c = 0; c < nchunk; ++c) {
        f32x4 sacc[2];
        long ktok[2][4];
        bool kval[2][4];
        // ---- scores S^T = K . Q^T ----
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            // MFMA A operand: key row f_a = 32c + 16j + r16, d in [8g, 8g+8)
            const int fa = 32 * c + 16 * j + r16;
            float kf[8];
            bool ok = fa < nf;
            long kt = 0;
            if (ok) {
                const int sx = fa % nxp, rest = fa / nxp;
                const int sy = rest % ay.n, sz = rest / ay.n;
                ok = sx < ax.n;
                kt = ((long)coord(az, sz) * p.Y + coord(ay, sy)) * p.X + coord(ax, sx);
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) kf[e] = ok ? Elt<T>::ld(kb + kt * p.ts + 8 * g + e) : 0.f;
            sacc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            if constexpr (sizeof(T) == 2) {
                bf16x8 av, bv;
#pragma unroll
                for (int e = 0; e < 8; ++e) { av[e] = f2bf(kf[e]); bv[e] = f2bf(qf[e]); }
                sacc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, sacc[j], 0, 0, 0);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    sacc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(kf[e], qf[e], sacc[j], 0, 0, 0);
            }
        }
        // ---- mask + bias on this lane's 8 keys: f = 32c + 16j + 4g + i ----
        float s[2][4];
        float cmax = NEG;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int f0 = 32 * c + 16 * j + 4 * g;
            const bool qok = f0 < nf;
            const int sx0 = f0 % nxp, rest = f0 / nxp;
            const int sy = rest % ay.n, sz = rest / ay.n;
            const bool zyok = qok && (unsigned)(sz - az.ws) < (unsigned)p.Kz &&
                              (unsigned)(sy - ay.ws) < (unsigned)p.Ky;
            const long rowtok = ((long)coord(az, sz) * p.Y + coord(ay, sy)) * p.X;
            const int bzy = ((sz + az.boff) * By + (sy + ay.boff)) * Bx;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int sx = sx0 + i;
                // The key exists in the halo (its V row feeds every query of
                // the group through the P.V product) ...
                const bool exists = qok && sx < ax.n;
                kval[j][i] = exists;
                ktok[j][i] = exists ? rowtok + coord(ax, sx) : qtok;
                // ... but only scores inside this lane's window count.
                const bool ok = zyok && sx < ax.n && (unsigned)(sx - ax.ws) < (unsigned)p.Kx;
                const float bias = ok ? rpb[bzy + sx + ax.boff] : 0.f;
                s[j][i] = ok ? fmaf(sacc[j][i], p.qscale, bias * p.bscale) : NEG;
                cmax = fmaxf(cmax, s[j][i]);
            }
        }
        cmax = fmaxf(cmax, __shfl_xor(cmax, 16, 64));
        cmax = fmaxf(cmax, __shfl_xor(cmax, 32, 64));
        const float m_new = fmaxf(m_run, cmax);
        const float alpha = exp2f(m_run - m_new);
        m_run = m_new;
        float pv[2][4];
        float psum = 0.f;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                pv[j][i] = exp2f(s[j][i] - m_new);
                psum += pv[j][i];
            }
        l_run = l_run * alpha + psum;
#pragma unroll
        for (int i = 0; i < 4; ++i) { o0[i] *= alpha; o1[i] *= alpha; }
        // ---- O^T += V^T . P^T ----
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int dcol = 16 * tt + r16;
            float vf[2][4];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    vf[j][i] = kval[j][i] ? Elt<T>::ld(vb + ktok[j][i] * p.ts + dcol) : 0.f;
            f32x4 &o = tt ? o1 : o0;
            if constexpr (sizeof(T) == 2) {
                bf16x8 av, bv;
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        av[4 * j + i] = f2bf(vf[j][i]);
                        bv[4 * j + i] = f2bf(pv[j][i]);
                    }
                o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, o, 0, 0, 0);
            } else {
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        o = __builtin_amdgcn_mfma_f32_16x16x4f32(vf[j][i], pv[j][i], o, 0, 0, 0);
            }
        }
    }
    float l_tot = l_run + __shfl_xor(l_run, 16, 64);
    l_tot += __shfl_xor(l_tot, 32, 64);
    const float inv = 1.0f / l_tot;
    if (active) {
        T *ob = (T *)p.out + (size_t)b * p.obs + (size_t)qtok * p.ots + h * 32;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Elt<T>::st(ob + 4 * g + i, o0[i] * inv);
            Elt<T>::st(ob + 16 + 4 * g + i, o1[i] * inv);
        }
    }
}

}  // namespace

hipError_t launch_nat(const NatArgs &a, bool bf16in, hipStream_t stream) {
    if (bf16in) {
        const size_t lds = nat_tile_lds_bytes(a);
        if (lds > 0 && lds <= 160 * 1024) return launch_nat_tile(a, stream);
    }
    // e4m3 contractions exist only in the tiled kernel: never fall back to
    // bf16 arithmetic for a caller that asked for them
    if (a.amax) return hipErrorNotSupported;
    return launch_nat_generic(a, bf16in, stream);
}

hipError_t launch_nat_generic(const NatArgs &a, bool bf16in, hipStream_t stream) {
    if (a.vt || a.q8 || a.o8) return hipErrorInvalidValue;     // reads token-major bf16/f32 q, k, v only
    const long ngroups = (long)((a.Z + GZ - 1) / GZ) * ((a.Y + GY - 1) / GY) * ((a.X + GX - 1) / GX);
    const long waves = ngroups * a.H * a.B;
    if (waves == 0) return hipSuccess;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    if (bf16in) nat_generic_kernel<bf16><<<grid, 256, 0, stream>>>(a);
    else nat_generic_kernel<float><<<grid, 256, 0, stream>>>(a);
    return hipGetLastError();
}

}  // namespace wm
