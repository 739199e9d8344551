// Launch sequences of a processor block and step, and the greedy schedule.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "runtime.hpp"

namespace wm {

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// FP8 block: the region of the e4m3 q and k planes and the blocked e4m3 v,
// which later holds the e4m3 GELU output [M][F].
static size_t fp8_big_bytes(const wm_processor *p, int B) {
    const size_t M = (size_t)B * p->g.Z * p->g.Y * p->g.X;
    const size_t C = p->g.C, F = C * p->mlp;
    const size_t qkv = al256(2 * M * C) + (size_t)B * p->g.Z * p->g.Y * v_blocked_xp(p->g.X) * C;
    return al256(std::max(qkv, M * F));
}

size_t block_workspace_bytes(const wm_processor *p, int B) {
    const size_t M = (size_t)B * p->g.Z * p->g.Y * p->g.X;
    const size_t C = p->g.C, F = C * p->mlp;
    if (p->prec == WM_FP8_E4M3) {
        // LN codes | q8 k8 v8, then GELU codes | o8 | bias tables
        return al256(M * C) + fp8_big_bytes(p, B) + al256(M * C) + (size_t)B * p->g.heads * NAT_TBL_WS_FLOATS * 4;
    }
    const size_t esz = p->prec == WM_BF16 ? 2 : 4;
    const size_t big = (3 * C > F ? 3 * C : F);
    const size_t act = (M * C * esz + 255) & ~(size_t)255;
    size_t bigb = (M * big * esz + 255) & ~(size_t)255;
    if (p->prec == WM_BF16) {
        // q and k head-major, v in the blocked layout (padded lon)
        const size_t qkv = 2 * M * C * 2 + (size_t)B * p->g.Z * p->g.Y * v_blocked_xp(p->g.X) * C * 2;
        bigb = std::max(bigb, al256(qkv));
    }
    return act + bigb + (size_t)p->g.heads * NAT_TBL_WS_FLOATS * 4;
}

// Bytes from the start of the block workspace to the bias-table scratch.
static size_t block_tbl_offset(const wm_processor *p, int B) {
    return block_workspace_bytes(p, B) - (size_t)p->g.heads * NAT_TBL_WS_FLOATS * 4;
}

int reserve_block_workspace(wm_ctx *ctx, const wm_processor *p, int B) {
    return ctx_reserve(ctx, block_workspace_bytes(p, B));
}

static hipEvent_t pool_get(wm_ctx *ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int prof_begin(wm_ctx *ctx, hipStream_t s, int kind) {
    if (!((ctx->prof_mask >> kind) & 1u)) return WM_OK;
    ProfRec r{kind, pool_get(ctx), pool_get(ctx)};
    if (!r.a || !r.b) return fail(WM_EHIP, "hipEventCreate failed");
    hipError_t e = hipEventRecord(r.a, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ctx->recs.push_back(r);
    ctx->prof_open = true;
    return WM_OK;
}

int prof_end(wm_ctx *ctx, hipStream_t s) {
    if (!ctx->prof_open || ctx->recs.empty()) return WM_OK;
    ctx->prof_open = false;
    hipError_t e = hipEventRecord(ctx->recs.back().b, s);
    return e == hipSuccess ? WM_OK : hip_fail(e, "hipEventRecord");
}

// One pre-norm block on the float32 residual stream x [B*T][C]:
//   u = LN1(x); [q|k|v] = u W_qkv + b (Q pre-scaled by log2(e)/sqrt(d),
//   written head-major); o = NA(q, k, v); x += o W_o + b_o;
//   w = LN2(x); h = GELU(w W_1 + b_1); x += h W_2 + b_2.
// u, o and w share one buffer; qkv and h share the other.
static int run_block_fp8(wm_ctx *ctx, const wm_processor *p, int block, int B, float *x, float *const *xs,
                         hipStream_t s);

bool block_fuses_ln(const wm_processor *p) {
    return (p->prec == WM_BF16 || p->prec == WM_FP8_E4M3) && gemm_resid_ln_applies(p->g.C);
}

int run_block(wm_ctx *ctx, const wm_processor *p, int block, int B, float *x, float *const *xs, hipStream_t s) {
    if (p->prec == WM_FP8_E4M3) return run_block_fp8(ctx, p, block, B, x, xs, s);
    const bool fuse = block_fuses_ln(p);
    const wm_grid &g = p->g;
    const BlockWeights &w = p->blk[block];
    const long T = (long)g.Z * g.Y * g.X;
    const int M = (int)(B * T);
    const int C = g.C, F = C * p->mlp, H = g.heads;
    const bool bf = p->prec == WM_BF16;
    const size_t esz = bf ? 2 : 4;
    char *act = (char *)ctx->ws;
    char *big = act + (((size_t)M * C * esz + 255) & ~(size_t)255);
    float *tbl_ws = (float *)((char *)ctx->ws + block_tbl_offset(p, B));
    hipError_t e;

    // Attention arguments first: bf16 blocks whose grid the tiled kernel
    // covers take v in the blocked layout, straight from the QKV epilogue.
    NatArgs na{};
    const size_t plane = (size_t)H * M * 32 * esz;
    na.q = big;
    na.k = big + plane;
    na.v = big + 2 * plane;
    na.bs = T * 32;
    na.ts = 32;
    na.hs = (long)M * 32;
    na.out = act;
    na.obs = T * C;
    na.ots = C;
    na.rpb = w.rpb_log2;
    na.qscale = 1.0f;
    na.bscale = 1.0f;
    na.B = B; na.Z = g.Z; na.Y = g.Y; na.X = g.X; na.H = H;
    na.Kz = g.Kz; na.Ky = g.Ky; na.Kx = g.Kx; na.periodic = g.periodic_mask;
    na.tbl_ws = w.nat_tbl ? w.nat_tbl : tbl_ws;
    na.tbl_ready = w.nat_tbl != nullptr;
    if (bf) {
        na.vt = 1;
        na.xp = v_blocked_xp(g.X);
        const size_t lds = nat_tile_lds_bytes(na);
        if (lds == 0 || lds > 160 * 1024) na.vt = 0;
    }

    int rc;
#define WM_TIMED(kind, call, what)                                  \
    if ((rc = prof_begin(ctx, s, kind)) != WM_OK) return rc;        \
    if ((e = (call)) != hipSuccess) return hip_fail(e, what);       \
    if ((rc = prof_end(ctx, s)) != WM_OK) return rc;
    const StateRows xr{x, xs, (unsigned)T};
    WM_TIMED(PK_LN1, launch_layernorm(xr, w.ln1_g, w.ln1_b, act, bf, M, C, 1e-5f, s), "LN1")
    EpiArgs ep{};
    ep.bias = w.b_qkv;
    ep.out = big;
    ep.C = C;
    ep.H = H;
    ep.qscale = LOG2E / std::sqrt(32.0f);
    if (p->rope_tab) {
        ep.rope = p->rope_tab;
        ep.rZ = g.Z; ep.rY = g.Y; ep.rX = g.X;
        ep.T = T;
    }
    // bf16: W_qkv holds the Q and K rows permuted by perm_row and the V rows
    // in natural order.  When the attention reads the blocked V layout, one
    // launch writes Q and K head-major and V blocked (its V workgroups swap
    // the MFMA operands); otherwise Q|K and V are two launches.
    auto qkv = [&]() -> hipError_t {
        const EpiKind kqk = p->rope_tab ? EPI_QKV_ROPE : EPI_QKV;
        if (!bf) return launch_gemm(act, w.w_qkv, M, 3 * C, C, false, kqk, ep, s);
        EpiArgs eqk = ep;
        eqk.perm = 1;
        if (na.vt) {
            eqk.vt = (void *)na.v;
            eqk.vB = B; eqk.vZ = g.Z; eqk.vY = g.Y; eqk.vX = g.X; eqk.vxp = na.xp;
            eqk.T = T;
            eqk.dT = udiv_make((unsigned)T);
            eqk.dYX = udiv_make((unsigned)(g.Y * g.X));
            eqk.dX = udiv_make((unsigned)g.X);
            return launch_gemm(act, w.w_qkv, M, 3 * C, C, true, kqk, eqk, s);
        }
        hipError_t err = launch_gemm(act, w.w_qkv, M, 2 * C, C, true, kqk, eqk, s);
        if (err != hipSuccess) return err;
        EpiArgs ev{};
        ev.bias = w.b_qkv + 2 * C;
        ev.out = big;
        ev.C = C;
        ev.H = H;
        ev.qscale = 1.0f;
        ev.part0 = 2;
        return launch_gemm(act, (const unsigned char *)w.w_qkv + (size_t)2 * C * C * 2, M, C, C, true, EPI_QKV, ev, s);
    };
    WM_TIMED(PK_QKV, qkv(), "QKV")

    WM_TIMED(PK_NA, launch_nat(na, bf, s), "NA")

    EpiArgs er{};
    er.bias = w.b_o;
    er.resid = x;
    er.resid_ptrs = xs;
    er.T = T;
    er.dT = udiv_make((unsigned)T);
    if (fuse) {
        // LN2 of each updated row into act, over the projection's own input
        // rows (a workgroup has read all of its rows of A by then)
        er.ln_g = w.ln2_g;
        er.ln_b = w.ln2_b;
        er.ln_out = act;
        er.ln_eps = 1e-5f;
        WM_TIMED(PK_PROJ, launch_gemm(act, w.w_o, M, C, C, bf, EPI_RESID_LN, er, s), "proj + LN2")
    } else {
        WM_TIMED(PK_PROJ, launch_gemm(act, w.w_o, M, C, C, bf, EPI_RESID, er, s), "proj")
        WM_TIMED(PK_LN2, launch_layernorm(xr, w.ln2_g, w.ln2_b, act, bf, M, C, 1e-5f, s), "LN2")
    }
    EpiArgs eg{};
    eg.bias = w.b_1;
    eg.out = big;
    eg.perm = bf;
    WM_TIMED(PK_MLP1, launch_gemm(act, w.w_1, M, F, C, bf, EPI_GELU, eg, s), "MLP1")
    EpiArgs e2{};
    e2.bias = w.b_2;
    e2.resid = x;
    e2.resid_ptrs = xs;
    e2.T = T;
    e2.dT = udiv_make((unsigned)T);
    WM_TIMED(PK_MLP2, launch_gemm(big, w.w_2, M, C, F, bf, EPI_RESID, e2, s), "MLP2")
#undef WM_TIMED
    return WM_OK;
}

// Every GEMM and both attention contractions run on e4m3 operands with
// static per-tensor scales fixed at processor creation from the weights
// (BlockWeights): each producer stores e4m3 codes directly -- the
// LayerNorms, the QKV projection (q and k planes, v in the blocked
// layout), the attention (its output at v's scale) and MLP1 (the GELU
// output) -- and each consumer dequantizes its MFMA sums with the product
// of the two scales.  Softmax, LayerNorm statistics and the residual stream
// stay float32.
static int run_block_fp8(wm_ctx *ctx, const wm_processor *p, int block, int B, float *x, float *const *xs,
                         hipStream_t s) {
    const bool fuse = block_fuses_ln(p);
    const wm_grid &g = p->g;
    const BlockWeights &w = p->blk[block];
    const long T = (long)g.Z * g.Y * g.X;
    const int M = (int)(B * T);
    const int C = g.C, F = C * p->mlp, H = g.heads;
    const int xp = v_blocked_xp(g.X);
    unsigned char *act8 = (unsigned char *)ctx->ws;
    unsigned char *big = act8 + al256((size_t)M * C);
    unsigned char *q8 = big, *k8 = big + (size_t)M * C, *v8 = big + al256(2 * (size_t)M * C);
    unsigned char *h8 = big;                                 // after the attention
    unsigned char *o8 = big + fp8_big_bytes(p, B);
    float *tbl_ws = (float *)(o8 + al256((size_t)M * C));
    hipError_t e;
    int rc;
#define WM_TIMED(kind, call, what)                                  \
    if ((rc = prof_begin(ctx, s, kind)) != WM_OK) return rc;        \
    if ((e = (call)) != hipSuccess) return hip_fail(e, what);       \
    if ((rc = prof_end(ctx, s)) != WM_OK) return rc;
    if (B > 64) return fail(WM_EINVAL, "FP8 processors take at most 64 states per call");
    if (!fp8_ring_applies(&g, B, 32)) return fail(WM_EINVAL, "no e4m3 attention kernel for this grid and batch");
    const StateRows xr{x, xs, (unsigned)T};
    WM_TIMED(PK_LN1, launch_layernorm_fp8_static(xr, w.ln1_g, w.ln1_b, M, C, 1e-5f, w.ln1_amax, act8, s), "LN1")
    EpiArgs ep{};
    ep.bias = w.b_qkv;
    ep.out = q8;
    ep.C = C;
    ep.H = H;
    ep.qscale = LOG2E / std::sqrt(32.0f);
    ep.a_dequant = w.ln1_amax_h / 448.0f;   // static scale of the LN1 codes
    ep.w_dequant = w.dq_qkv;
    ep.T = T;
    ep.perm = 1;   // W_qkv (Q and K rows) and W_1 are stored with permuted rows (perm_row)
    ep.out8 = 1;
    for (int part = 0; part < 3; ++part) ep.out_mul[part] = 448.0f / w.qkv_amax_h[part];
    ep.vt = v8;
    ep.vB = B; ep.vZ = g.Z; ep.vY = g.Y; ep.vX = g.X; ep.vxp = xp;
    ep.dT = udiv_make((unsigned)T);
    ep.dYX = udiv_make((unsigned)(g.Y * g.X));
    ep.dX = udiv_make((unsigned)g.X);
    if (p->rope_tab) {
        ep.rope = p->rope_tab;
        ep.rZ = g.Z; ep.rY = g.Y; ep.rX = g.X;
    }
    WM_TIMED(PK_QKV, launch_gemm_fp8(act8, w.w_qkv, M, 3 * C, C, p->rope_tab ? EPI_QKV_ROPE : EPI_QKV, ep, s), "QKV")
    NatArgs na{};
    na.q = q8;
    na.k = k8;
    na.v = v8;
    na.bs = T * 32;
    na.ts = 32;
    na.hs = (long)M * 32;
    na.out = o8;
    na.obs = T * C;
    na.ots = C;
    na.rpb = w.rpb_log2;
    na.qscale = 1.0f;
    na.bscale = 1.0f;
    na.B = B; na.Z = g.Z; na.Y = g.Y; na.X = g.X; na.H = H;
    na.Kz = g.Kz; na.Ky = g.Ky; na.Kx = g.Kx; na.periodic = g.periodic_mask;
    na.tbl_ws = tbl_ws;
    na.amax = w.qkv_amax;      // the static (aq, ak, av) of every state
    na.amax_stride = 0;
    na.vt = 1;
    na.xp = xp;
    na.q8 = 1;
    na.o8 = 1;
    WM_TIMED(PK_NA, launch_nat(na, true, s), "NA")
    EpiArgs er{};
    er.bias = w.b_o;
    er.resid = x;
    er.resid_ptrs = xs;
    er.T = T;
    er.dT = udiv_make((unsigned)T);
    er.a_dequant = w.qkv_amax_h[2] / 448.0f;   // o is coded at v's scale
    er.w_dequant = w.dq_o;
    er.T = T;
    if (fuse) {
        // LN2 codes of each updated row into act8 (static scale ln2_amax)
        er.ln_g = w.ln2_g;
        er.ln_b = w.ln2_b;
        er.ln_amax = w.ln2_amax;
        er.ln_out = act8;
        er.ln_eps = 1e-5f;
        er.out8 = 1;
        WM_TIMED(PK_PROJ, launch_gemm_fp8(o8, w.w_o, M, C, C, EPI_RESID_LN, er, s), "proj + LN2")
    } else {
        WM_TIMED(PK_PROJ, launch_gemm_fp8(o8, w.w_o, M, C, C, EPI_RESID, er, s), "proj")
        WM_TIMED(PK_LN2, launch_layernorm_fp8_static(xr, w.ln2_g, w.ln2_b, M, C, 1e-5f, w.ln2_amax, act8, s), "LN2")
    }
    EpiArgs eg{};
    eg.bias = w.b_1;
    eg.out = h8;
    eg.a_dequant = w.ln2_amax_h / 448.0f;   // static scale of the LN2 codes
    eg.w_dequant = w.dq_1;
    eg.T = T;
    eg.perm = 1;
    eg.out8 = 1;
    eg.out_mul[0] = 448.0f / w.h_amax_h;
    WM_TIMED(PK_MLP1, launch_gemm_fp8(act8, w.w_1, M, F, C, EPI_GELU, eg, s), "MLP1")
    EpiArgs e2{};
    e2.bias = w.b_2;
    e2.resid = x;
    e2.resid_ptrs = xs;
    e2.T = T;
    e2.dT = udiv_make((unsigned)T);
    e2.a_dequant = w.h_amax_h / 448.0f;
    e2.w_dequant = w.dq_2;
    e2.T = T;
    WM_TIMED(PK_MLP2, launch_gemm_fp8(h8, w.w_2, M, C, F, EPI_RESID, e2, s), "MLP2")
#undef WM_TIMED
    return WM_OK;
}

int run_step(wm_ctx *ctx, const wm_processor *p, int B, float *x, float *const *xs, hipStream_t s) {
    for (int b = 0; b < p->nb; ++b) {
        int rc = run_block(ctx, p, b, B, x, xs, s);
        if (rc) return rc;
    }
    return WM_OK;
}

unsigned char host_fp8_e4m3(float x) {
    const unsigned char sign = std::signbit(x) ? 0x80 : 0x00;
    double a = std::fabs((double)x);
    if (std::isnan(x)) return 0x7f;
    if (a > 448.0) a = 448.0;
    // exponent of the representable grid around a: normals 2^-6 .. 2^8
    int e = a > 0 ? (int)std::floor(std::log2(a)) : -6;
    if (e < -6) e = -6;
    double q = std::nearbyint(a / std::ldexp(1.0, e - 3));   // mantissa units, ties to even
    if (q >= 16.0) {                                           // rounded up into the next binade
        e += 1;
        q = 8.0;
    }
    if (e > 8 || (e == 8 && q > 14.0)) {                      // saturate at 448
        e = 8;
        q = 14.0;
    }
    unsigned char code;
    if (q < 8.0) code = (unsigned char)q;                      // subnormal (e == -6)
    else code = (unsigned char)(((e + 7) << 3) | ((int)q - 8));
    return sign | code;
}

// Sec. 2.1, latent rollout: the six-hour and one-hour processors are called
// until the lead time is reached by a greedy schedule -- as many six-hour
// steps as fit, then one-hour steps.
int greedy_schedule(int lead_hours, int *out, int cap) {
    int n = 0;
    int left = lead_hours;
    const int sizes[2] = {6, 1};
    for (int size : sizes) {
        while (left >= size) {
            if (out && n < cap) out[n] = size;
            ++n;
            left -= size;
        }
    }
    return n;
}

}  // namespace wm
