/*
 * wm.h -- C ABI of the MI355X latent processor library (libwm.so).
 *
 * WeatherMesh-3 (arXiv 2503.22235) forecasts by encoding the weather state
 * into a 2-degree latent grid, running a processor (a stack of
 * neighborhood-attention transformer blocks) on that latent any number of
 * times -- one call advances one hour or six hours -- and decoding
 * (Sec. 2.1, "Encoder-processor-decoder architecture").  The problem it
 * solves is stated there: from a single state, predict the state any integer
 * number of hours later.  This library is the latent part of that path on
 * one GPU: the neighborhood attention (wm_nat_forward), one transformer
 * block (wm_processor_block), one processor step (wm_processor_step), the
 * greedy rollout (wm_schedule, wm_rollout) and a continuous-batching
 * request loop (wm_serve_*).
 *
 * Conventions shared by every entry point:
 *  - Grid axes are (Z = pressure level, Y = latitude, X = longitude); a
 *    state is [B][Z][Y][X][C] float32, channels last, token
 *    t = (z*Y + y)*X + x.  Channel c of an attention head is h*d + e with
 *    d = C / heads (d must be 32).
 *  - Tensor pointers are DEVICE pointers owned by the caller unless a
 *    comment says host.  The library never frees caller memory.
 *  - Streams are hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on that stream; calls return without waiting for the
 *    GPU unless stated otherwise.
 *  - Every int-returning call returns WM_OK (0) or a negative wm_status;
 *    wm_last_error() then holds a message for the calling thread.
 */
#ifndef WM_H
#define WM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WM_OK = 0,
    WM_EINVAL = -1,    /* invalid argument (shape, window, precision, lead) */
    WM_ENOMEM = -2,    /* device or host allocation failed                  */
    WM_EAGAIN = -3,    /* not ready yet (serving: request still running)    */
    WM_EHIP = -4,      /* a HIP runtime call failed                         */
    WM_ENOTFOUND = -5  /* unknown request id                                */
} wm_status;

typedef enum {
    WM_F32 = 0,        /* float32 operands, float32 accumulation            */
    WM_BF16 = 1,       /* bfloat16 operands (RNE), float32 accumulation     */
    WM_FP8_E4M3 = 2    /* OCP e4m3 operands with per-tensor scales          */
} wm_precision;

/* Latent grid and attention window.  Windows are odd and no larger than
 * their axis.  periodic_mask: bit0 = Z, bit1 = Y, bit2 = X; the paper's
 * setting is 0x4 -- longitude wraps around the sphere (its own circular
 * padding), latitude and level windows keep their size and shift inward at
 * the borders (NATTEN's border behaviour) (App. A.2). */
typedef struct {
    int Z, Y, X;
    int C, heads;
    int Kz, Ky, Kx;
    unsigned periodic_mask;
} wm_grid;

typedef struct wm_ctx wm_ctx;
typedef struct wm_processor wm_processor;
typedef struct wm_server wm_server;

/* Message of the last failing call on this thread ("" if none).  The
 * string is owned by the library and valid until the next call. */
const char *wm_last_error(void);

/* Library version string (static storage). */
const char *wm_version(void);

/* Context bound to one HIP device.  It owns a workspace that grows on
 * demand to hold a block's intermediates for the largest batch seen.
 * The caller destroys it after all work enqueued through it has finished.
 * A context serves one thread (and one stream) at a time: work enqueued
 * through it on two streams at once would share its workspace.  A
 * processor is only read by the calls that run it (wm_processor_set_rope
 * aside), so any number of contexts and threads may run it at once. */
int wm_ctx_create(int device, wm_ctx **out);
void wm_ctx_destroy(wm_ctx *ctx);

/* Kernel timing.  While enabled, every kernel a block launches is
 * bracketed by HIP events recorded on the stream it is launched on.
 * wm_prof_collect waits for the recorded events, ADDS each kernel kind's
 * total milliseconds and launch count into ms[kind] and counts[kind]
 * (kinds 0..6: LN1, QKV projection, neighborhood attention, output
 * projection, LN2, MLP1, MLP2; arrays of nkinds entries, either may be
 * NULL) and clears the records.  BF16 and FP8 processors at C = 512 run
 * LN2 inside the output projection's kernel: kind 3 then covers both and
 * kind 4 records no launches. */
int wm_prof_enable(wm_ctx *ctx, int on);
/* Like wm_prof_enable, for the kinds whose bit is set in kinds_mask only
 * (bit k = kind k; 0 turns timing off), so that a timed region carries
 * events around the kernels it reports and no others. */
int wm_prof_select(wm_ctx *ctx, unsigned kinds_mask);
int wm_prof_collect(wm_ctx *ctx, double *ms, long long *counts, int nkinds);

/* Neighborhood index tables of a grid (Sec. 2.1 NATTEN; App. A.2).
 * dev_out: device int32[2*(Z+Y+X)].  Entries [0, Z+Y+X) are, per axis in
 * the order Z, Y, X, the first key coordinate of every position's window
 * (clamped axis: min(max(i-r, 0), N-K); periodic axis: (i-r) mod N); the
 * window is that coordinate plus t = 0..K-1 (mod N when periodic).
 * Entries [Z+Y+X, 2*(Z+Y+X)) are the bias-table index (offset + K - 1) of
 * the first key of that window; it grows by one with t.  Written by a
 * kernel with the same index functions the attention kernels use. */
int wm_nat_indices(const wm_grid *g, int *dev_out, void *stream);

/* 3-D neighborhood attention with relative-position bias (Sec. 2.1 NATTEN;
 * App. A.2 circular padding and bump attention).  For every state b,
 * token n and head h:
 *   s(n,m) = q_h(n).k_h(m) / sqrt(d) + rpb[h][dz+Kz-1][dy+Ky-1][dx+Kx-1]
 *   out_h(n) = sum over m in the window of n of softmax_m(s) v_h(m)
 * with (dz,dy,dx) = key - query offsets (periodic axes: t - r).
 * q, k, v, out: device [B][Z*Y*X][heads][d] in float32 (WM_F32) or
 * bfloat16 (WM_BF16 and WM_FP8_E4M3); rpb: device float32
 * [heads][2Kz-1][2Ky-1][2Kx-1].  Softmax max and sum are float32.
 * WM_FP8_E4M3 runs both contractions on OCP e4m3 codes: q, k and v of each
 * state are quantized with the scale amax/448 of that state's tensor (round
 * to nearest even, saturating), the softmax weights with the static scale 1
 * (they are <= 256 by construction), and the output is dequantized to bf16;
 * it needs a lon-periodic grid (periodic_mask 4), a 5x7x7, 3x5x5 or 3x3x3
 * window, X >= Kx + 7 and B <= 64 (else WM_EINVAL).  Uses the context
 * workspace. */
int wm_nat_forward(wm_ctx *ctx, const wm_grid *g, int B, wm_precision prec,
                   const void *q, const void *k, const void *v,
                   const float *rpb, void *out, void *stream);

/* wm_nat_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, layouts, results and errors as wm_nat_forward, without a
 * context.  It runs on the calling thread's current HIP device, and
 * `stream` must belong to that device.  Its scratch (bias tables, FP8 amax
 * slots) is one fixed array of WM_NAT_NOALLOC_SCRATCH_BYTES in each
 * device's memory, held from the first call on that device until the
 * process ends; it calls no hipMalloc/hipFree.  Calls needing more scratch
 * than that -- heads * 8 KiB for F32/BF16, B * heads * 8 KiB + 128 KiB for
 * WM_FP8_E4M3 -- return WM_EINVAL.  Every call on one device shares that
 * array and rewrites what it reads before reading it, so calls whose work
 * overlaps on one device (two streams, or two threads) race: serialize
 * them. */
#define WM_NAT_NOALLOC_SCRATCH_BYTES (4u << 20)
int wm_nat_forward_noalloc(const wm_grid *g, int B, wm_precision prec,
                           const void *q, const void *k, const void *v,
                           const float *rpb, void *out, void *stream);

/* LayerNorm of M rows of C float32 values, float32 statistics with biased
 * variance (the block's two norms; the pre-norm vision-transformer layout
 * the paper builds on, Sec. 2.1):
 *   out[m][c] = (x[m][c] - mean_m) / sqrt(var_m + eps) * gamma[c] + beta[c]
 * x: device float32 [M][C]; gamma, beta: device float32 [C]; out: device
 * [M][C] float32 (WM_F32) or bfloat16 (WM_BF16).  C in {128,256,512,1024}. */
int wm_layernorm(int M, int C, const float *x, const float *gamma,
                 const float *beta, float eps, wm_precision out_prec,
                 void *out, void *stream);

/* One of the block's linear maps with its fused epilogue:
 *   r[m][n] = sum_k a[m][k] * w[n][k] + bias[n]
 * a: device [M][K], w: device [N][K] (output-major), both float32 (WM_F32)
 * or bfloat16 (WM_BF16), float32 accumulation; bias: device float32 [N].
 * epilogue 0: out[m][n] = r (operand precision); 1: out = GELU(r) with the
 * exact erf form (operand precision); 2: float32 out[m][n] += r (the
 * residual update).  N % 64 == 0; K % 64 == 0 (bf16) or % 32 (float32). */
int wm_linear(int M, int N, int K, wm_precision prec, const void *a,
              const void *w, const float *bias, int epilogue, void *out,
              void *stream);

/* FP8 quantization as the FP8 processors use it (OCP e4m3, max 448):
 * out[i] = RNE(clamp(x[i] * mul, -448, 448)) as e4m3 codes.  x: device
 * float32 [n]; out: device bytes [n]. */
int wm_quantize_fp8(size_t n, const float *x, float mul, unsigned char *out,
                    void *stream);

/* One linear map on e4m3 operands with float32 accumulation:
 *   r[m][n] = a_dequant * w_dequant * sum_k a8[m][k] * w8[n][k] + bias[n]
 * a8 [M][K], w8 [N][K] device e4m3 codes; epilogue and out as wm_linear
 * (0 and 1 write bfloat16).  N % 128 == 0, K % 128 == 0.  Enqueued on
 * `stream`; allocates nothing. */
int wm_linear_fp8(int M, int N, int K, const void *a8, float a_dequant,
                  const void *w8, float w_dequant, const float *bias,
                  int epilogue, void *out, void *stream);

/* A processor: n_blocks pre-norm neighborhood-attention transformer blocks
 * (Sec. 2.1; App. A.2) with MLP width mlp_ratio*C, uploaded from HOST
 * float32 parameters in canonical order, per block:
 *   ln1_g[C] ln1_b[C] w_qkv[C][3C] b_qkv[3C] rpb[H][2Kz-1][2Ky-1][2Kx-1]
 *   w_o[C][C] b_o[C] ln2_g[C] ln2_b[C] w_1[C][F] b_1[F] w_2[F][C] b_2[C]
 * Linear maps are [in][out] (y = x W + b); QKV columns are [Q | K | V].
 * The library copies and converts what it needs (the host array may be
 * freed on return) and owns the device copy until wm_processor_destroy.
 * Requires d = C/heads = 32 and C in {128, 256, 512, 1024}.
 * WM_FP8_E4M3 processors store all four weight matrices as e4m3 with
 * per-tensor scales (amax / 448) and run every GEMM and both attention
 * contractions on e4m3 codes with float32 accumulation.  The activations
 * (LayerNorm outputs, q, k, v, the attention output, the GELU output) are
 * quantized with static per-tensor scales bound / 448, where each bound is
 * computed here from the weights and no input can exceed it: channel c of a
 * LayerNorm output is at most |gamma_c| sqrt(C-1) + |beta_c|; output j of
 * a projection is at most sum_c |W_cj| L_c + |b_j| over the bounds L_c of
 * its input (q and k times sqrt 2, which also covers rotary; q times its
 * score factor 1/sqrt(32)); the attention output is bounded by v's bound;
 * the GELU output by max(U, 0.17) for its pre-activation bound U.
 * Softmax, LayerNorm statistics and the residual stream stay float32.  The
 * e4m3 attention exists for a lon-periodic grid (periodic_mask 4), a 5x7x7,
 * 3x5x5 or 3x3x3 window and X >= Kx + 7;
 * an FP8 processor on any other grid is rejected with WM_EINVAL (checked
 * before the context, so no device is needed to be told).  BF16 processors also prepare each block's
 * attention bias table on the device here.  Returns once the upload (and
 * that preparation) has completed on the device. */
int wm_processor_create(wm_ctx *ctx, const wm_grid *g, int n_blocks,
                        int mlp_ratio, wm_precision prec,
                        const float *host_params, wm_processor **out);
void wm_processor_destroy(wm_processor *p);
/* Rotary position embedding for this processor's blocks (App. A.2 uses
 * rotary embeddings; the 3-D layout is this library's reading): q and k of
 * every head are rotated in the QKV epilogue, channel pairs (2i, 2i+1) with
 * pairs 0-3 following the level index z at angles z * 10000^(-i/4), pairs
 * 4-9 the latitude index y at y * 10000^(-(i-4)/6), pairs 10-15 the
 * longitude index x at x * 2 pi (i-9) / X (periodic in lon).  The
 * relative-position bias still applies: a processor created with zero bias
 * tables is a pure rotary one.  on = 0 turns it off.  Allocates a small
 * device table on first use; not to be called while the processor runs. */
int wm_processor_set_rope(wm_processor *p, int on);

int wm_processor_blocks(const wm_processor *p);

/* One block of the processor (Sec. 2.1 "Encoder-processor-decoder
 * architecture" and "NATTEN": a transformer block of 3-D neighborhood
 * attention on the latent grid; App. A.2 for the window and its borders;
 * the pre-norm layout, biases and GELU are this library's reading where
 * the paper is silent), in place on x (device float32 [B][Z][Y][X][C]):
 *   x1 = x + NA(LN1(x) W_qkv + b_qkv) W_o + b_o
 *   x  = x1 + GELU(LN2(x1) W_1 + b_1) W_2 + b_2
 * LayerNorm statistics, softmax max/sum and the residual stream are
 * float32; the contractions run in the processor's precision with float32
 * accumulation. */
int wm_processor_block(wm_ctx *ctx, const wm_processor *p, int block, int B,
                       float *x, void *stream);

/* One processor step: all blocks in order, in place (Sec. 2.1). */
int wm_processor_step(wm_ctx *ctx, const wm_processor *p, int B, float *x,
                      void *stream);

/* One processor step (Sec. 2.1) on B states that live in separate device
 * buffers (the batches of a server whose requests keep their states where
 * they are, Sec. 2.2 operational use): dev_states is a DEVICE array of B
 * pointers, each to a float32 [Z][Y][X][C] state, updated in place; the
 * kernels read and write the residual stream through the pointers, so no
 * state is copied.  Results are bit-identical to wm_processor_step on the
 * same states stacked in one buffer.  The array and the states must stay
 * valid until the step has run on `stream`.  B < 0, B > 64 or a NULL array
 * -> WM_EINVAL. */
int wm_processor_step_states(wm_ctx *ctx, const wm_processor *p, int B,
                             float *const *dev_states, void *stream);

/* Greedy latent-rollout schedule (Sec. 2.1, latent rollout): for
 * lead_hours >= 0 writes floor(L/6) sixes followed by (L mod 6) ones into
 * HOST steps_out (if non-NULL and cap is large enough) and returns the
 * number of steps.  Negative lead or too small cap -> WM_EINVAL. */
int wm_schedule(int lead_hours, int *steps_out, int cap);

/* Latent rollout (Sec. 2.1: the six-hour and one-hour processors are
 * applied in latent space, chosen by a greedy schedule, until the lead time
 * is reached): run the six-hour processor p6 and the one-hour processor p1
 * on x in place following wm_schedule(lead_hours), with no host
 * synchronisation between steps.  Lead 0 leaves x unchanged. */
int wm_rollout(wm_ctx *ctx, const wm_processor *p6, const wm_processor *p1,
               int B, float *x, int lead_hours, void *stream);

/* ---- Serving: a continuous-batching forecast loop -----------------------
 * WeatherMesh-3 runs operationally, answering forecasts of any integer lead
 * time from one latent state (Sec. 2.1; Sec. 2.2 operational encoders).  A server owns a scheduler
 * thread.  Submitted requests wait in a FIFO until a state slot in HBM is
 * free (slots are sized from the memory budget); their state is copied in
 * on a copy stream while other requests compute.  Every scheduler iteration
 * batches up to max_batch admitted requests whose next processor (six-hour
 * or one-hour, greedy schedule) is the same into one step launch; requests
 * join and leave the batch between steps.  With float32 slots the step runs
 * on the slots in place (the kernels address the batch's states through a
 * device array of slot pointers, as wm_processor_step_states); with
 * bfloat16 slots (half the memory per request) each step converts the
 * batch's slots into a float32 buffer and back.  Every step's kernels read
 * fixed addresses (the pointer array or the batch buffer and the server's
 * own workspace), so with cfg.graphs the step of a (processor, batch size)
 * is captured once into a HIP graph and replayed for every later batch of
 * that shape; only the pointer array (or the conversions) changes between
 * replays.  Finished states are copied out
 * on the copy stream.  Each request's result does not depend on what it
 * was batched with (every kernel computes a state's tokens the same way
 * whatever the batch).  Calls are thread-safe. */
typedef struct {
    int max_batch;             /* states per step launch (1..64)                  */
    int state_bf16;            /* 1: slots hold bfloat16 states between steps      */
    size_t hbm_budget_bytes;   /* slot memory cap; 0 = 3/4 of the free HBM         */
    int max_slots;             /* 0 = as many as the budget allows (<= 1024)        */
    int graphs;                /* 1: each step after the first of its (processor,
                                  batch size) replays a HIP graph captured from
                                  that step's launches (one graph launch per step) */
} wm_serve_cfg;

typedef struct {
    uint64_t id;
    int lead_hours;
    int steps;                 /* processor steps the request ran                  */
    int batches;               /* step launches it was part of                     */
    double t_submit, t_admit, t_done;   /* seconds on the steady clock            */
    int max_cobatch;           /* most requests in one step launch it was part of  */
} wm_req_stats;

/* p6, p1 must share one grid and stay alive, with their rotary setting
 * unchanged, until wm_serve_destroy.  The server takes its own streams and
 * workspace on ctx's device. */
int wm_serve_create(wm_ctx *ctx, const wm_processor *p6, const wm_processor *p1,
                    const wm_serve_cfg *cfg, wm_server **out);
/* Queue a forecast of lead_hours >= 0 from HOST float32 x0 [Z][Y][X][C];
 * x0 is copied before return.  Never waits for the GPU.  WM_ENOMEM if the
 * host copy or the request's schedule cannot be allocated. */
int wm_serve_submit(wm_server *s, const float *x0_host, int lead_hours,
                    uint64_t *id_out);
/* WM_OK: request id finished; its state is copied to HOST out_host (float32
 * [Z][Y][X][C], may be NULL) and stats to *st (may be NULL), and the request
 * is forgotten.  WM_EAGAIN: still queued or running.  WM_ENOTFOUND: unknown
 * (or already collected) id.  After a failure inside the scheduler (a HIP
 * error, or WM_ENOMEM for a host allocation) every poll returns that code
 * and the server does no further work.  Never waits for the GPU. */
int wm_serve_poll(wm_server *s, uint64_t id, float *out_host, wm_req_stats *st);
/* Counters: queued, admitted-and-running, finished-not-collected, slots. */
int wm_serve_status(wm_server *s, int *queued, int *running, int *done, int *slots);
/* Stops the scheduler (queued and running requests are dropped) and frees
 * the server's memory. */
void wm_serve_destroy(wm_server *s);

/* Every hourly lead 1..hours of one state, sharing prefixes (Sec. 2.1:
 * hourly outputs from the six-hour and one-hour processors).  The six-hour
 * chain runs once; each one-hour branch starts from the six-hour state
 * before it, so lead L comes from the same steps, in the same order, as
 * wm_rollout(L): floor(L/6) six-hour steps, then L mod 6 one-hour steps --
 * about 56 + 280 = 336 steps for 336 hours instead of 10136 for separate
 * rollouts.  Branches of up to `batch` (1..64) six-hour states run as one
 * batched one-hour step.
 * x: device float32 state [Z*Y*X*C] (B = 1), not modified.  outs: host
 * array of `hours` device pointers (float32 [Z*Y*X*C] each, caller-owned);
 * outs[L-1] receives the state at lead L; a NULL entry (or outs == NULL)
 * skips that lead.  Keeps 1 + batch state copies in context memory.  Work
 * is enqueued on `stream`. */
int wm_forecast_hourly(wm_ctx *ctx, const wm_processor *p6, const wm_processor *p1, const float *x,
                       int hours, float *const *outs, int batch, void *stream);

/* Relative L2 error ||y - y_ref|| / ||y_ref|| of n values, accumulated in
 * float64 on the GPU.  y: device float32; y_ref: device float64.  Waits
 * for the stream and returns the value (negative on error). */
double wm_relerr_l2(wm_ctx *ctx, const float *y, const double *y_ref,
                    size_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WM_H */
