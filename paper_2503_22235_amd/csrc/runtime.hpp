// Internal objects of libwm and the launch sequences of a block and a step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "../../include/wm.h"
#include "kernels.hpp"

namespace wm {

// Device pointers of one block's parameters (owned by the processor).
struct BlockWeights {
    const float *ln1_g, *ln1_b, *b_qkv, *rpb_log2, *b_o, *ln2_g, *ln2_b, *b_1, *b_2;
    const void *w_qkv, *w_o, *w_1, *w_2;   // [out][in], processor precision
    // FP8 processors: the four weight matrices hold e4m3 codes with these
    // per-tensor dequantization scales (amax / 448).
    float dq_qkv = 1.f, dq_o = 1.f, dq_1 = 1.f, dq_2 = 1.f;
    // FP8 processors: static amax (scale = amax / 448) of every activation
    // tensor, bounds that no input can exceed, from the weights alone:
    //  - LayerNorm output channel c: |gamma_c| sqrt(C - 1) + |beta_c| (a
    //    normalized row has mean 0 and mean square 1, so no entry exceeds
    //    sqrt(C - 1)); ln*_amax is the maximum over c (device float and host
    //    copy);
    //  - projection output j: sum_c |W_jc| L_c + |b_j| with L_c the bound of
    //    its LayerNorm input channel; q stored times its score factor; q and
    //    k times sqrt 2 (rotary, which may be set later, mixes a channel pair);
    //    qkv_amax = (aq, ak, av) on the device, qkv_amax_h on the host;
    //  - attention output: a convex combination of v rows, bounded by av;
    //  - GELU output: max(U, 0.17) for pre-activation bound U (GELU(u) lies
    //    in [-0.17, max(u, 0)]).
    const float *ln1_amax = nullptr, *ln2_amax = nullptr;
    float ln1_amax_h = 0.f, ln2_amax_h = 0.f;
    const float *qkv_amax = nullptr;
    float qkv_amax_h[3] = {0.f, 0.f, 0.f};
    float h_amax_h = 0.f;
    // BF16 processors: the tiled attention kernel's bias table of this
    // block, prepared once at creation (null: prepared per launch)
    float *nat_tbl = nullptr;
};

constexpr int MAX_BLOCKS = 64;

// Kernel kinds of a block, in launch order (timing records).
enum ProfKind : int { PK_LN1 = 0, PK_QKV, PK_NA, PK_PROJ, PK_LN2, PK_MLP1, PK_MLP2, PK_N };

struct ProfRec {
    int kind;
    hipEvent_t a, b;
};

}  // namespace wm

struct wm_ctx {
    int device = 0;
    void *ws = nullptr;       // block intermediates, grown on demand
    size_t ws_bytes = 0;
    void *small = nullptr;    // 4 KiB of device scratch (reductions)
    void *aux = nullptr;      // state copies of the hourly forecast, grown on demand
    size_t aux_bytes = 0;
    unsigned prof_mask = 0;   // bracket block kernels of these kinds (bit k = kind k) with HIP events
    bool prof_open = false;   // a record is waiting for its end event
    std::vector<wm::ProfRec> recs;
    std::vector<hipEvent_t> pool;
};

struct wm_processor {
    wm_grid g{};
    int nb = 0, mlp = 4, device = 0;
    wm_precision prec = WM_F32;
    void *mem = nullptr;
    size_t bytes = 0;
    float *rope_tab = nullptr;   // rotary (cos, sin) table, or null (no rotary embedding)
    wm::BlockWeights blk[wm::MAX_BLOCKS];
};

namespace wm {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int ctx_reserve(wm_ctx *ctx, size_t bytes);
bool fp8_attention_applies(const wm_grid *g, int B, long ts);
// Whether the e4m3 level-ring attention (v in the blocked layout, q and k
// with token stride ts) covers grid g at batch B.
bool fp8_ring_applies(const wm_grid *g, int B, long ts);
// wm_nat_forward in two parts: argument checks (and the scratch bytes
// needed), then the launches with the scratch at a given device address.
// blocked_v: bf16 attention copies v to the blocked layout in the scratch
// and runs the level-ring kernel (else the token-major tile kernel).
int nat_forward_check(const wm_grid *g, int B, wm_precision prec, const void *q, const void *k, const void *v,
                      const float *rpb, void *out, bool blocked_v, size_t *ws_need);
int nat_forward_into(const wm_grid *g, int B, wm_precision prec, const void *q, const void *k, const void *v,
                     const float *rpb, void *out, bool blocked_v, void *ws, hipStream_t s);
bool ring_attention_applies(const wm_grid *g, int B, long ts);


// Bytes of workspace a block of processor p needs for B states.
size_t block_workspace_bytes(const wm_processor *p, int B);
int reserve_block_workspace(wm_ctx *ctx, const wm_processor *p, int B);
// Timing records (no-ops for kinds outside ctx->prof_mask).
int prof_begin(wm_ctx *ctx, hipStream_t s, int kind);
int prof_end(wm_ctx *ctx, hipStream_t s);
// Enqueue one block / one step on `s` (workspace already reserved).
// x: the float32 residual stream [B*T][C] in one buffer, or (xs set, x
// unused) B states in separate buffers whose pointers are in the device
// array xs.
// Blocks whose LN2 runs in the epilogue of the out-projection (bf16 and
// FP8 at C = 512).
bool block_fuses_ln(const wm_processor *p);
int run_block(wm_ctx *ctx, const wm_processor *p, int block, int B, float *x, float *const *xs, hipStream_t s);
int run_step(wm_ctx *ctx, const wm_processor *p, int B, float *x, float *const *xs, hipStream_t s);
// Host OCP e4m3 encoding, round to nearest even, saturating at +-448.
unsigned char host_fp8_e4m3(float x);

// Greedy 6 h / 1 h schedule; writes up to cap entries if out != nullptr and
// returns the number of steps.
int greedy_schedule(int lead_hours, int *out, int cap);

}  // namespace wm
