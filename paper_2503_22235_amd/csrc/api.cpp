// C ABI of libwm: contexts, processors, the block / step / rollout launch
// sequences and the small helpers.  Declarations and contracts: wm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wm.h"
#include "kernels.hpp"
#include "runtime.hpp"

using namespace wm;

namespace wm {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(WM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int validate_grid(const wm_grid *g, bool need_block) {
    if (!g) return fail(WM_EINVAL, "grid is NULL");
    const int N[3] = {g->Z, g->Y, g->X}, K[3] = {g->Kz, g->Ky, g->Kx};
    const char *nm = "ZYX";
    for (int a = 0; a < 3; ++a) {
        if (N[a] < 1) return fail(WM_EINVAL, "axis %c has length %d", nm[a], N[a]);
        if (K[a] < 1 || K[a] % 2 == 0) return fail(WM_EINVAL, "window on %c must be odd (got %d)", nm[a], K[a]);
        if (K[a] > N[a]) return fail(WM_EINVAL, "window %d larger than axis %c (%d)", K[a], nm[a], N[a]);
    }
    if (g->periodic_mask > 7) return fail(WM_EINVAL, "periodic_mask must be within 0..7");
    if (g->heads < 1 || g->C != g->heads * 32) return fail(WM_EINVAL, "head dim must be 32 (C=%d heads=%d)", g->C, g->heads);
    if (need_block && !(g->C == 128 || g->C == 256 || g->C == 512 || g->C == 1024))
        return fail(WM_EINVAL, "C must be 128, 256, 512 or 1024 (got %d)", g->C);
    if ((long long)g->Z * g->Y * g->X > (1LL << 30)) return fail(WM_EINVAL, "grid too large");
    return WM_OK;
}

// Whether the e4m3 attention kernel covers grid g at batch B with token
// stride ts (elements) (the FP8 processors and wm_nat_forward in FP8 have no
// other attention kernel).
bool fp8_attention_applies(const wm_grid *g, int B, long ts) {
    static float dummy_tbl;
    static float dummy_amax;
    NatArgs a{};
    a.ts = ts;
    a.B = B; a.Z = g->Z; a.Y = g->Y; a.X = g->X; a.H = g->heads;
    a.Kz = g->Kz; a.Ky = g->Ky; a.Kx = g->Kx; a.periodic = g->periodic_mask;
    a.tbl_ws = &dummy_tbl;       // only tested for null
    a.amax = &dummy_amax;
    const size_t lds = nat_tile_lds_bytes(a);
    return lds > 0 && lds <= 160 * 1024;
}

bool fp8_ring_applies(const wm_grid *g, int B, long ts) {
    static float dummy_tbl;
    static float dummy_amax;
    NatArgs a{};
    a.ts = ts;
    a.B = B; a.Z = g->Z; a.Y = g->Y; a.X = g->X; a.H = g->heads;
    a.Kz = g->Kz; a.Ky = g->Ky; a.Kx = g->Kx; a.periodic = g->periodic_mask;
    a.tbl_ws = &dummy_tbl;       // only tested for null
    a.amax = &dummy_amax;
    a.vt = 1;
    a.xp = v_blocked_xp(g->X);
    const size_t lds = nat_tile_lds_bytes(a);
    return lds > 0 && lds <= 160 * 1024;
}

// Whether the bf16 attention on v in the blocked layout (the level-ring
// kernel) covers grid g at batch B with q/k token stride ts (elements).
bool ring_attention_applies(const wm_grid *g, int B, long ts) {
    static float dummy_tbl;
    NatArgs a{};
    a.ts = ts;
    a.B = B; a.Z = g->Z; a.Y = g->Y; a.X = g->X; a.H = g->heads;
    a.Kz = g->Kz; a.Ky = g->Ky; a.Kx = g->Kx; a.periodic = g->periodic_mask;
    a.tbl_ws = &dummy_tbl;       // only tested for null
    a.vt = 1;
    a.xp = v_blocked_xp(g->X);
    const size_t lds = nat_tile_lds_bytes(a);
    return lds > 0 && lds <= 160 * 1024;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

int ctx_reserve(wm_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return WM_OK;
    hipError_t e;
    if (ctx->ws) {
        // In-flight work may still use the old buffer.
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    if ((e = hipMalloc(&ctx->ws, bytes)) != hipSuccess) {
        ctx->ws = nullptr;
        (void)hipGetLastError();
        return fail(WM_ENOMEM, "workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    ctx->ws_bytes = bytes;
    return WM_OK;
}


// Argument checks of the attention entry points; *ws_need receives the
// scratch bytes nat_forward_into uses (bias tables, FP8 amax slots).
int nat_forward_check(const wm_grid *g, int B, wm_precision prec, const void *q, const void *k, const void *v,
                      const float *rpb, void *out, bool blocked_v, size_t *ws_need) {
    int rc = validate_grid(g, false);
    if (rc) return rc;
    if (B < 0) return fail(WM_EINVAL, "negative batch");
    if (prec != WM_F32 && prec != WM_BF16 && prec != WM_FP8_E4M3) return fail(WM_EINVAL, "unknown precision");
    const bool fp8 = prec == WM_FP8_E4M3;
    if (fp8 && B > 64) return fail(WM_EINVAL, "FP8 attention takes at most 64 states per call");
    *ws_need = (size_t)(fp8 ? B : 1) * g->heads * NAT_TBL_WS_FLOATS * 4 +
               (fp8 ? (size_t)AMAX_SHARDS * AMAX_STRIDE * 4 : 0);
    if (blocked_v && prec == WM_BF16 && B > 0 && ring_attention_applies(g, B, g->C))
        *ws_need += (size_t)B * g->Z * g->Y * v_blocked_xp(g->X) * g->C * 2;
    if (blocked_v && fp8 && B > 0 && fp8_ring_applies(g, B, g->C))   // e4m3 k, then blocked e4m3 v
        *ws_need = al256(*ws_need) + al256((size_t)B * g->Z * g->Y * g->X * g->C) +
                   (size_t)B * g->Z * g->Y * v_blocked_xp(g->X) * g->C;
    if (B == 0) return WM_OK;
    if (!q || !k || !v || !rpb || !out) return fail(WM_EINVAL, "NULL tensor");
    if (fp8 && !fp8_attention_applies(g, B, g->C))
        return fail(WM_EINVAL, "FP8 attention needs lon-periodic only, a 5x7x7, 3x5x5 or 3x3x3 window "
                               "and lon >= 8 + Kx - 1");
    return WM_OK;
}

// Enqueue the attention of wm_nat_forward (arguments already checked by
// nat_forward_check, B > 0) with its scratch at device address ws.
int nat_forward_into(const wm_grid *g, int B, wm_precision prec, const void *q, const void *k, const void *v,
                     const float *rpb, void *out, bool blocked_v, void *ws, hipStream_t s) {
    const long T = (long)g->Z * g->Y * g->X;
    const bool fp8 = prec == WM_FP8_E4M3;
    const size_t tbl_bytes = (size_t)(fp8 ? B : 1) * g->heads * NAT_TBL_WS_FLOATS * 4;
    NatArgs a{};
    a.q = q; a.k = k; a.v = v;
    a.bs = T * g->C; a.ts = g->C; a.hs = 32;
    a.out = out; a.obs = T * g->C; a.ots = g->C;
    a.rpb = rpb;
    a.qscale = LOG2E / std::sqrt(32.0f);
    a.bscale = LOG2E;
    a.B = B; a.Z = g->Z; a.Y = g->Y; a.X = g->X; a.H = g->heads;
    a.Kz = g->Kz; a.Ky = g->Ky; a.Kx = g->Kx; a.periodic = g->periodic_mask;
    a.tbl_ws = (float *)ws;
    hipError_t e;
    if (fp8) {
        unsigned *amax = (unsigned *)((char *)ws + tbl_bytes);
        if ((e = launch_zero_u32(amax, (size_t)AMAX_SHARDS * AMAX_STRIDE, s)) != hipSuccess) return hip_fail(e, "zero");
        const void *src[3] = {q, k, v};
        for (int i = 0; i < 3; ++i)
            if ((e = launch_amax_bf16(src[i], (size_t)T * g->C, B, amax + i, 3, s)) != hipSuccess)
                return hip_fail(e, "amax");
        if ((e = launch_amax_fold(amax, 3 * B, s)) != hipSuccess) return hip_fail(e, "amax fold");
        a.amax = (const float *)amax;
        a.amax_stride = 3;
    }
    if (blocked_v && fp8 && fp8_ring_applies(g, B, g->C)) {
        // k and v quantized once (k with its strides, v in the blocked layout,
        // after the tables and amax slots), read by the e4m3 level-ring kernel
        const size_t off = al256(tbl_bytes + (size_t)AMAX_SHARDS * AMAX_STRIDE * 4);
        unsigned char *k8 = (unsigned char *)ws + off;
        unsigned char *v8 = k8 + al256((size_t)B * T * g->C);
        a.xp = v_blocked_xp(g->X);
        a.vt = 1;
        if ((e = launch_kv8(a, k8, v8, s)) != hipSuccess) return hip_fail(e, "k, v to e4m3");
        a.k = k8;
        a.v = v8;
    }
    if (blocked_v && prec == WM_BF16 && ring_attention_applies(g, B, g->C)) {
        // v copied to the blocked layout (after the tables), read by the level-ring kernel
        void *vb = (char *)ws + tbl_bytes;
        a.xp = v_blocked_xp(g->X);
        if ((e = launch_v_blocked(a, vb, s)) != hipSuccess) return hip_fail(e, "v to blocked layout");
        a.v = vb;
        a.vt = 1;
    }
    e = launch_nat(a, prec != WM_F32, s);
    return e == hipSuccess ? WM_OK : hip_fail(e, "nat launch");
}
}  // namespace wm

static uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

extern "C" {

const char *wm_last_error(void) { return g_err.c_str(); }

const char *wm_version(void) { return "libwm 0.1 (gfx950)"; }

int wm_ctx_create(int device, wm_ctx **out) {
    if (!out) return fail(WM_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(WM_EINVAL, "device %d out of range (%d devices)", device, n);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    wm_ctx *c = new (std::nothrow) wm_ctx();
    if (!c) return fail(WM_ENOMEM, "context allocation");
    c->device = device;
    if ((e = hipMalloc(&c->small, 4096)) != hipSuccess) {
        delete c;
        return hip_fail(e, "hipMalloc(small)");
    }
    *out = c;
    return WM_OK;
}

void wm_ctx_destroy(wm_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->small) (void)hipFree(ctx->small);
    if (ctx->aux) (void)hipFree(ctx->aux);
    delete ctx;
}

int wm_prof_enable(wm_ctx *ctx, int on) {
    if (!ctx) return fail(WM_EINVAL, "ctx is NULL");
    ctx->prof_mask = on != 0 ? 0xffffffffu : 0u;
    return WM_OK;
}

int wm_prof_select(wm_ctx *ctx, unsigned kinds_mask) {
    if (!ctx) return fail(WM_EINVAL, "ctx is NULL");
    ctx->prof_mask = kinds_mask;
    return WM_OK;
}

int wm_prof_collect(wm_ctx *ctx, double *ms, long long *counts, int nkinds) {
    if (!ctx) return fail(WM_EINVAL, "ctx is NULL");
    if (nkinds < 0) return fail(WM_EINVAL, "negative nkinds");
    hipError_t e;
    int rc = WM_OK;
    for (auto &r : ctx->recs) {
        if (rc == WM_OK) {
            float t = 0.f;
            if ((e = hipEventSynchronize(r.b)) != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
            else if ((e = hipEventElapsedTime(&t, r.a, r.b)) != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
            else if (r.kind < nkinds) {
                if (ms) ms[r.kind] += t;
                if (counts) counts[r.kind] += 1;
            }
        }
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    return rc;
}

int wm_nat_indices(const wm_grid *g, int *dev_out, void *stream) {
    int rc = validate_grid(g, false);
    if (rc) return rc;
    if (!dev_out) return fail(WM_EINVAL, "dev_out is NULL");
    hipError_t e = launch_nat_indices(g->Z, g->Y, g->X, g->Kz, g->Ky, g->Kx, g->periodic_mask, dev_out,
                                      (hipStream_t)stream);
    return e == hipSuccess ? WM_OK : hip_fail(e, "nat_indices launch");
}

int wm_nat_forward(wm_ctx *ctx, const wm_grid *g, int B, wm_precision prec, const void *q, const void *k,
                   const void *v, const float *rpb, void *out, void *stream) {
    size_t need = 0;
    int rc = nat_forward_check(g, B, prec, q, k, v, rpb, out, true, &need);
    if (rc) return rc;
    if (!ctx) return fail(WM_EINVAL, "ctx is NULL");
    if (B == 0) return WM_OK;
    rc = ctx_reserve(ctx, need);
    if (rc) return rc;
    return nat_forward_into(g, B, prec, q, k, v, rpb, out, true, ctx->ws, (hipStream_t)stream);
}

int wm_layernorm(int M, int C, const float *x, const float *gamma, const float *beta, float eps,
                 wm_precision out_prec, void *out, void *stream) {
    if (M < 0) return fail(WM_EINVAL, "negative M");
    if (!(C == 128 || C == 256 || C == 512 || C == 1024)) return fail(WM_EINVAL, "C must be 128/256/512/1024");
    if (out_prec != WM_F32 && out_prec != WM_BF16) return fail(WM_EINVAL, "out precision must be F32 or BF16");
    if (M == 0) return WM_OK;
    if (!x || !gamma || !beta || !out) return fail(WM_EINVAL, "NULL tensor");
    hipError_t e = launch_layernorm(StateRows{const_cast<float *>(x), nullptr, 0}, gamma, beta, out, out_prec == WM_BF16, M, C,
                                    eps, (hipStream_t)stream);
    return e == hipSuccess ? WM_OK : hip_fail(e, "layernorm launch");
}

int wm_linear(int M, int N, int K, wm_precision prec, const void *a, const void *w, const float *bias,
              int epilogue, void *out, void *stream) {
    if (M < 0 || N <= 0 || K <= 0) return fail(WM_EINVAL, "bad GEMM shape");
    if (prec != WM_F32 && prec != WM_BF16) return fail(WM_EINVAL, "precision must be F32 or BF16");
    if (N % 64) return fail(WM_EINVAL, "N must be a multiple of 64");
    if (K % (prec == WM_BF16 ? 64 : 32)) return fail(WM_EINVAL, "K must be a multiple of %d", prec == WM_BF16 ? 64 : 32);
    if (epilogue < 0 || epilogue > 2) return fail(WM_EINVAL, "epilogue must be 0, 1 or 2");
    if (M == 0) return WM_OK;
    if (!a || !w || !bias || !out) return fail(WM_EINVAL, "NULL tensor");
    EpiArgs ep{};
    ep.bias = bias;
    EpiKind kind = EPI_STORE;
    if (epilogue == 1) { kind = EPI_GELU; ep.out = out; }
    else if (epilogue == 2) { kind = EPI_RESID; ep.resid = (float *)out; }
    else ep.out = out;
    hipError_t e = launch_gemm(a, w, M, N, K, prec == WM_BF16, kind, ep, (hipStream_t)stream);
    return e == hipSuccess ? WM_OK : hip_fail(e, "gemm launch");
}

int wm_quantize_fp8(size_t n, const float *x, float mul, unsigned char *out, void *stream) {
    if (n == 0) return WM_OK;
    if (!x || !out) return fail(WM_EINVAL, "NULL tensor");
    hipError_t e = launch_quant_f32(x, n, mul, out, (hipStream_t)stream);
    return e == hipSuccess ? WM_OK : hip_fail(e, "quantize launch");
}

int wm_linear_fp8(int M, int N, int K, const void *a8, float a_dequant, const void *w8, float w_dequant,
                  const float *bias, int epilogue, void *out, void *stream) {
    if (M < 0 || N <= 0 || K <= 0) return fail(WM_EINVAL, "bad GEMM shape");
    if (N % 128 || K % 128) return fail(WM_EINVAL, "N and K must be multiples of 128");
    if (epilogue < 0 || epilogue > 2) return fail(WM_EINVAL, "epilogue must be 0, 1 or 2");
    if (M == 0) return WM_OK;
    if (!a8 || !w8 || !bias || !out) return fail(WM_EINVAL, "NULL tensor");
    hipStream_t s = (hipStream_t)stream;
    EpiArgs ep{};
    ep.bias = bias;
    ep.a_dequant = a_dequant;     // one scale for all rows
    ep.w_dequant = w_dequant;
    ep.T = M;
    EpiKind kind = EPI_STORE;
    if (epilogue == 1) { kind = EPI_GELU; ep.out = out; }
    else if (epilogue == 2) { kind = EPI_RESID; ep.resid = (float *)out; }
    else ep.out = out;
    const hipError_t e = launch_gemm_fp8(a8, w8, M, N, K, kind, ep, s);
    return e == hipSuccess ? WM_OK : hip_fail(e, "gemm launch");
}

int wm_processor_create(wm_ctx *ctx, const wm_grid *g, int n_blocks, int mlp_ratio, wm_precision prec,
                        const float *host_params, wm_processor **out) {
    if (!out) return fail(WM_EINVAL, "out is NULL");
    *out = nullptr;
    // Argument checks come before the context's: they need no device.
    int rc = validate_grid(g, true);
    if (rc) return rc;
    if (n_blocks < 1 || n_blocks > 64) return fail(WM_EINVAL, "n_blocks must be 1..64");
    if (mlp_ratio < 1 || mlp_ratio > 8) return fail(WM_EINVAL, "mlp_ratio must be 1..8");
    if (prec != WM_F32 && prec != WM_BF16 && prec != WM_FP8_E4M3)
        return fail(WM_EINVAL, "processor precision %d not supported", (int)prec);
    // (head-major q, k, v: 32 elements per token)
    if (prec == WM_FP8_E4M3 && !fp8_ring_applies(g, 1, 32))
        return fail(WM_EINVAL, "FP8 processors run QK and PV on e4m3 codes, which needs lon-periodic only "
                               "(periodic_mask 4), a 5x7x7, 3x5x5 or 3x3x3 window and lon >= 8 + Kx - 1");
    if (!host_params) return fail(WM_EINVAL, "host_params is NULL");
    if (!ctx) return fail(WM_EINVAL, "ctx is NULL");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");

    wm_processor *p = new (std::nothrow) wm_processor();
    if (!p) return fail(WM_ENOMEM, "processor allocation");
    p->g = *g;
    p->nb = n_blocks;
    p->mlp = mlp_ratio;
    p->prec = prec;
    p->device = ctx->device;
    const int C = g->C, F = C * mlp_ratio, H = g->heads;
    const size_t nrpb = (size_t)H * (2 * g->Kz - 1) * (2 * g->Ky - 1) * (2 * g->Kx - 1);
    // Bytes per weight element: float32, bfloat16, or (FP8) e4m3.
    const bool fp8 = prec == WM_FP8_E4M3;
    const size_t esz = prec == WM_F32 ? 4 : 2;
    const size_t esz_big = fp8 ? 1 : esz;
    // Device image per block: float32 vectors, then the four transposed weights.
    const size_t nvec = 2 * C + 3 * C + nrpb + C + 2 * C + F + C + 5;
    const size_t nw_bytes = ((size_t)3 * C * C + (size_t)F * C * 2) * esz_big + (size_t)C * C * esz + 4 * 256;
    auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
    // BF16: room for the tiled attention kernel's prepared bias table
    const size_t tbl_bytes = prec == WM_BF16 ? align((size_t)H * NAT_TBL_WS_FLOATS * 4) : 0;
    const size_t blk_bytes = align(nvec * 4) + align(nw_bytes) + 4 * 256 + tbl_bytes;
    p->bytes = blk_bytes * n_blocks;
    if ((e = hipMalloc(&p->mem, p->bytes)) != hipSuccess) {
        delete p;
        (void)hipGetLastError();
        return fail(WM_ENOMEM, "processor weights (%zu bytes): %s", p->bytes, hipGetErrorString(e));
    }
    std::vector<unsigned char> img(blk_bytes);
    const float *src = host_params;
    for (int bI = 0; bI < n_blocks; ++bI) {
        std::memset(img.data(), 0, img.size());
        unsigned char *dev = (unsigned char *)p->mem + blk_bytes * bI;
        BlockWeights &bw = p->blk[bI];
        size_t off = 0;
        auto put_vec = [&](const float *s, size_t n, float scale, const float **dst) {
            float *d = (float *)(img.data() + off);
            for (size_t i = 0; i < n; ++i) d[i] = s[i] * scale;
            *dst = (const float *)(dev + off);
            off += n * 4;
        };
        // source [in][out] -> device [out][in] (bf16 and e4m3 with pr: rows
        // permuted within groups of 32 by perm_row); returns the fp8 dequant
        // scale
        // pr_rows: rows below it are permuted (perm_row), the rest keep their order
        auto put_wt = [&](const float *s, int in, int outn, const void **dst, bool q8, int pr_rows) -> float {
            auto src_col = [&](int o) { return o < pr_rows ? perm_row(o) : o; };
            off = align(off);
            if (q8) {
                float amax = 0.f;
                for (size_t i = 0; i < (size_t)in * outn; ++i) amax = std::max(amax, std::fabs(s[i]));
                const float inv = amax > 0.f ? 448.0f / amax : 1.0f;
                unsigned char *d = img.data() + off;
                for (int o = 0; o < outn; ++o)
                    for (int i = 0; i < in; ++i)
                        d[(size_t)o * in + i] = host_fp8_e4m3(s[(size_t)i * outn + src_col(o)] * inv);
                *dst = dev + off;
                off += (size_t)in * outn;
                return amax > 0.f ? amax / 448.0f : 1.0f;
            }
            if (esz == 2) {
                uint16_t *d = (uint16_t *)(img.data() + off);
                for (int o = 0; o < outn; ++o)
                    for (int i = 0; i < in; ++i) d[(size_t)o * in + i] = host_bf16(s[(size_t)i * outn + src_col(o)]);
            } else {
                float *d = (float *)(img.data() + off);
                for (int o = 0; o < outn; ++o)
                    for (int i = 0; i < in; ++i) d[(size_t)o * in + i] = s[(size_t)i * outn + o];
            }
            *dst = dev + off;
            off += (size_t)in * outn * esz;
            return 1.0f;
        };
        const float *ln1_g = src; src += C;
        const float *ln1_b = src; src += C;
        const float *w_qkv = src; src += (size_t)C * 3 * C;
        const float *b_qkv = src; src += 3 * C;
        const float *rpb = src; src += nrpb;
        const float *w_o = src; src += (size_t)C * C;
        const float *b_o = src; src += C;
        const float *ln2_g = src; src += C;
        const float *ln2_b = src; src += C;
        const float *w_1 = src; src += (size_t)C * F;
        const float *b_1 = src; src += F;
        const float *w_2 = src; src += (size_t)F * C;
        const float *b_2 = src; src += C;
        put_vec(ln1_g, C, 1.f, &bw.ln1_g);
        put_vec(ln1_b, C, 1.f, &bw.ln1_b);
        put_vec(b_qkv, 3 * C, 1.f, &bw.b_qkv);
        put_vec(rpb, nrpb, LOG2E, &bw.rpb_log2);
        put_vec(b_o, C, 1.f, &bw.b_o);
        put_vec(ln2_g, C, 1.f, &bw.ln2_g);
        put_vec(ln2_b, C, 1.f, &bw.ln2_b);
        put_vec(b_1, F, 1.f, &bw.b_1);
        put_vec(b_2, C, 1.f, &bw.b_2);
        if (fp8) {
            // static LayerNorm-output amax: |gamma_c| sqrt(C - 1) + |beta_c| bounds channel c
            auto ln_bound = [&](const float *gm, const float *bt) {
                double m = 0.0;
                for (int c = 0; c < C; ++c)
                    m = std::max(m, std::fabs((double)gm[c]) * std::sqrt((double)(C - 1)) + std::fabs((double)bt[c]));
                return (float)m;
            };
            // bound of output j of a projection [in = C][outn] (source layout
            // [in][out]) fed by LayerNorm (gamma, beta): sum_c |W_jc| L_c + |b_j|
            auto proj_bound = [&](const float *wt, const float *bias, int outn, int j, const float *gm,
                                  const float *bt) {
                double u = std::fabs((double)bias[j]);
                const double r = std::sqrt((double)(C - 1));
                for (int c = 0; c < C; ++c)
                    u += std::fabs((double)wt[(size_t)c * outn + j]) * (std::fabs((double)gm[c]) * r + std::fabs((double)bt[c]));
                return u;
            };
            double part_max[3] = {0.0, 0.0, 0.0};
            for (int j = 0; j < 3 * C; ++j)
                part_max[j / C] = std::max(part_max[j / C], proj_bound(w_qkv, b_qkv, 3 * C, j, ln1_g, ln1_b));
            // q and k: times sqrt 2, so the bound also holds once rotary (set
            // after creation) mixes each channel pair
            const double rot = std::sqrt(2.0);
            const float aq = (float)(part_max[0] * rot * (LOG2E / std::sqrt(32.0)));
            const float ak = (float)(part_max[1] * rot), av = (float)part_max[2];
            double hmax = 0.17;
            for (int j = 0; j < F; ++j) hmax = std::max(hmax, proj_bound(w_1, b_1, F, j, ln2_g, ln2_b));
            const float a5[5] = {ln_bound(ln1_g, ln1_b), ln_bound(ln2_g, ln2_b), aq, ak, av};
            const float *d5 = nullptr;
            put_vec(a5, 5, 1.f, &d5);
            bw.ln1_amax = d5;
            bw.ln2_amax = d5 + 1;
            bw.qkv_amax = d5 + 2;
            bw.ln1_amax_h = a5[0];
            bw.ln2_amax_h = a5[1];
            bw.qkv_amax_h[0] = aq;
            bw.qkv_amax_h[1] = ak;
            bw.qkv_amax_h[2] = av;
            bw.h_amax_h = (float)hmax;
        }
        // QKV and MLP1 rows permuted (their epilogues store 8 features per
        // lane); the residual GEMMs keep the natural order
        // (bf16: the V rows of W_qkv keep their order; the V tiles of the
        // projection write the blocked layout with swapped operands)
        bw.dq_qkv = put_wt(w_qkv, C, 3 * C, &bw.w_qkv, fp8, 2 * C);
        bw.dq_o = put_wt(w_o, C, C, &bw.w_o, fp8, 0);
        bw.dq_1 = put_wt(w_1, C, F, &bw.w_1, fp8, F);
        bw.dq_2 = put_wt(w_2, F, C, &bw.w_2, fp8, 0);
        if ((e = hipMemcpy(dev, img.data(), blk_bytes, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(p->mem);
            delete p;
            return hip_fail(e, "weight upload");
        }
        if (tbl_bytes) {
            // the table depends on the weights only: prepare it once here
            // (same arguments as the block's attention launch)
            NatArgs na{};
            na.rpb = bw.rpb_log2;
            na.qscale = 1.0f;
            na.bscale = 1.0f;
            na.H = H;
            na.Kz = g->Kz; na.Ky = g->Ky; na.Kx = g->Kx;
            na.tbl_ws = (float *)(dev + blk_bytes - tbl_bytes);
            e = launch_nat_bias_table(na, nullptr);
            if (e == hipSuccess) bw.nat_tbl = na.tbl_ws;
            else if (e != hipErrorNotSupported) {   // not supported: a window without a tiled kernel
                (void)hipFree(p->mem);
                delete p;
                return hip_fail(e, "attention bias table");
            }
        }
    }
    if (tbl_bytes && (e = hipStreamSynchronize(nullptr)) != hipSuccess) {
        (void)hipFree(p->mem);
        delete p;
        return hip_fail(e, "attention bias table");
    }
    *out = p;
    return WM_OK;
}

void wm_processor_destroy(wm_processor *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->mem) (void)hipFree(p->mem);
    if (p->rope_tab) (void)hipFree(p->rope_tab);
    delete p;
}

int wm_processor_set_rope(wm_processor *p, int on) {
    if (!p) return fail(WM_EINVAL, "processor is NULL");
    hipError_t e;
    if ((e = hipSetDevice(p->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (!on) {
        if (p->rope_tab) {
            if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
            (void)hipFree(p->rope_tab);
            p->rope_tab = nullptr;
        }
        return WM_OK;
    }
    if (p->rope_tab) return WM_OK;
    const int Z = p->g.Z, Y = p->g.Y, X = p->g.X, rows = Z + Y + X;
    // angle of pair q at position pos of its axis: level pairs 0-3 and lat
    // pairs 4-9 on the frequency ladder 10000^(-j/P), lon pairs 10-15 at
    // the integer frequencies 2 pi (j+1) / X
    std::vector<float> tab((size_t)rows * 16 * 2);
    for (int r = 0; r < rows; ++r) {
        const int axis = r < Z ? 0 : (r < Z + Y ? 1 : 2);
        const int pos = axis == 0 ? r : (axis == 1 ? r - Z : r - Z - Y);
        for (int q = 0; q < 16; ++q) {
            double ang = 0.0;
            if (axis == 0 && q < 4) ang = pos * std::pow(10000.0, -q / 4.0);
            else if (axis == 1 && q >= 4 && q < 10) ang = pos * std::pow(10000.0, -(q - 4) / 6.0);
            else if (axis == 2 && q >= 10) ang = pos * 2.0 * M_PI * (q - 10 + 1) / X;
            tab[((size_t)r * 16 + q) * 2] = (float)std::cos(ang);
            tab[((size_t)r * 16 + q) * 2 + 1] = (float)std::sin(ang);
        }
    }
    float *d = nullptr;
    if ((e = hipMalloc(&d, tab.size() * 4)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(WM_ENOMEM, "rotary table: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(d, tab.data(), tab.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "rotary table copy");
    }
    p->rope_tab = d;
    return WM_OK;
}

int wm_processor_blocks(const wm_processor *p) { return p ? p->nb : fail(WM_EINVAL, "processor is NULL"); }

int wm_processor_block(wm_ctx *ctx, const wm_processor *p, int block, int B, float *x, void *stream) {
    if (!ctx || !p) return fail(WM_EINVAL, "NULL ctx or processor");
    if (block < 0 || block >= p->nb) return fail(WM_EINVAL, "block %d out of range (%d blocks)", block, p->nb);
    if (B < 0) return fail(WM_EINVAL, "negative batch");
    if (B == 0) return WM_OK;
    if (!x) return fail(WM_EINVAL, "x is NULL");
    int rc = reserve_block_workspace(ctx, p, B);
    if (rc) return rc;
    return run_block(ctx, p, block, B, x, nullptr, (hipStream_t)stream);
}

int wm_processor_step(wm_ctx *ctx, const wm_processor *p, int B, float *x, void *stream) {
    if (!ctx || !p) return fail(WM_EINVAL, "NULL ctx or processor");
    if (B < 0) return fail(WM_EINVAL, "negative batch");
    if (B == 0) return WM_OK;
    if (!x) return fail(WM_EINVAL, "x is NULL");
    int rc = reserve_block_workspace(ctx, p, B);
    if (rc) return rc;
    return run_step(ctx, p, B, x, nullptr, (hipStream_t)stream);
}

int wm_processor_step_states(wm_ctx *ctx, const wm_processor *p, int B, float *const *dev_states, void *stream) {
    if (!ctx || !p) return fail(WM_EINVAL, "NULL ctx or processor");
    if (B < 0 || B > 64) return fail(WM_EINVAL, "batch %d outside 0..64", B);
    if (B == 0) return WM_OK;
    if (!dev_states) return fail(WM_EINVAL, "dev_states is NULL");
    int rc = reserve_block_workspace(ctx, p, B);
    if (rc) return rc;
    return run_step(ctx, p, B, nullptr, dev_states, (hipStream_t)stream);
}

int wm_schedule(int lead_hours, int *steps_out, int cap) {
    if (lead_hours < 0) return fail(WM_EINVAL, "negative lead time %d", lead_hours);
    const int n = greedy_schedule(lead_hours, nullptr, 0);
    if (steps_out) {
        if (cap < n) return fail(WM_EINVAL, "schedule needs %d entries, cap is %d", n, cap);
        greedy_schedule(lead_hours, steps_out, cap);
    }
    return n;
}

int wm_rollout(wm_ctx *ctx, const wm_processor *p6, const wm_processor *p1, int B, float *x, int lead_hours,
               void *stream) {
    if (!ctx || !p6 || !p1) return fail(WM_EINVAL, "NULL ctx or processor");
    if (lead_hours < 0) return fail(WM_EINVAL, "negative lead time %d", lead_hours);
    if (B < 0) return fail(WM_EINVAL, "negative batch");
    if (std::memcmp(&p6->g, &p1->g, sizeof(wm_grid)) != 0) return fail(WM_EINVAL, "processors have different grids");
    if (B == 0 || lead_hours == 0) return WM_OK;
    if (!x) return fail(WM_EINVAL, "x is NULL");
    int rc = reserve_block_workspace(ctx, p6, B);
    if (rc) return rc;
    rc = reserve_block_workspace(ctx, p1, B);
    if (rc) return rc;
    std::vector<int> steps(greedy_schedule(lead_hours, nullptr, 0));
    greedy_schedule(lead_hours, steps.data(), (int)steps.size());
    for (int s : steps) {
        rc = run_step(ctx, s == 6 ? p6 : p1, B, x, nullptr, (hipStream_t)stream);
        if (rc) return rc;
    }
    return WM_OK;
}

int wm_forecast_hourly(wm_ctx *ctx, const wm_processor *p6, const wm_processor *p1, const float *x, int hours,
                       float *const *outs, int batch, void *stream) {
    if (!ctx || !p6 || !p1) return fail(WM_EINVAL, "NULL ctx or processor");
    if (hours < 0) return fail(WM_EINVAL, "negative hours %d", hours);
    if (batch < 1 || batch > 64) return fail(WM_EINVAL, "batch must be in 1..64");
    if (std::memcmp(&p6->g, &p1->g, sizeof(wm_grid)) != 0) return fail(WM_EINVAL, "processors have different grids");
    if (hours == 0) return WM_OK;
    if (!x) return fail(WM_EINVAL, "x is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)p6->g.Z * p6->g.Y * p6->g.X * p6->g.C;
    const size_t sb = n * 4;
    int rc = reserve_block_workspace(ctx, p6, 1);
    if (rc) return rc;
    rc = reserve_block_workspace(ctx, p1, batch);
    if (rc) return rc;
    // aux: the six-hour chain state, then `batch` branch states
    const size_t need = sb * (size_t)(1 + batch);
    if (need > ctx->aux_bytes) {
        hipError_t e;
        if (ctx->aux) {
            if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
            (void)hipFree(ctx->aux);
            ctx->aux = nullptr;
            ctx->aux_bytes = 0;
        }
        if ((e = hipMalloc(&ctx->aux, need)) != hipSuccess) {
            ctx->aux = nullptr;
            (void)hipGetLastError();
            return fail(WM_ENOMEM, "forecast states (%zu bytes): %s", need, hipGetErrorString(e));
        }
        ctx->aux_bytes = need;
    }
    float *chain = (float *)ctx->aux;
    float *branch = chain + n;
    hipError_t e;
    auto copy = [&](float *dst, const float *src) -> int {
        if ((e = hipMemcpyAsync(dst, src, sb, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return hip_fail(e, "state copy");
        return WM_OK;
    };
    auto out_of = [&](int lead) -> float * { return outs && lead >= 1 && lead <= hours ? outs[lead - 1] : nullptr; };
    if ((rc = copy(chain, x))) return rc;
    int base[64], nbr = 0;
    // One-hour branches of the gathered six-hour states: j steps give leads base + j.
    auto run_branches = [&]() -> int {
        int jmax = 0;
        for (int i = 0; i < nbr; ++i) jmax = std::max(jmax, std::min(5, hours - base[i]));
        for (int j = 1; j <= jmax; ++j) {
            if ((rc = run_step(ctx, p1, nbr, branch, nullptr, s))) return rc;
            for (int i = 0; i < nbr; ++i)
                if (float *o = base[i] + j <= hours ? out_of(base[i] + j) : nullptr)
                    if ((rc = copy(o, branch + (size_t)i * n))) return rc;
        }
        nbr = 0;
        return WM_OK;
    };
    for (int lead = 0; lead <= hours; lead += 6) {
        if (lead > 0) {
            if ((rc = run_step(ctx, p6, 1, chain, nullptr, s))) return rc;
            if (float *o = out_of(lead))
                if ((rc = copy(o, chain))) return rc;
        }
        if (lead + 1 <= hours) {
            if ((rc = copy(branch + (size_t)nbr * n, chain))) return rc;
            base[nbr++] = lead;
            if (nbr == batch && (rc = run_branches())) return rc;
        }
    }
    if (nbr > 0 && (rc = run_branches())) return rc;
    return WM_OK;
}

double wm_relerr_l2(wm_ctx *ctx, const float *y, const double *y_ref, size_t n, void *stream) {
    if (!ctx || !y || !y_ref) return (double)fail(WM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if ((e = launch_zero_u32((unsigned *)ctx->small, 4, s)) != hipSuccess)
        return (double)hip_fail(e, "zero");
    if ((e = launch_relerr(y, y_ref, n, (double *)ctx->small, s)) != hipSuccess) return (double)hip_fail(e, "relerr");
    double h[2];
    if ((e = hipMemcpyAsync(h, ctx->small, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return (double)hip_fail(e, "copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return (double)hip_fail(e, "sync");
    if (h[1] == 0.0) return h[0] == 0.0 ? 0.0 : INFINITY;
    return std::sqrt(h[0] / h[1]);
}

}  // extern "C"
