"""Throughput of the latent processor step on one MI355X.

Workload: one processor step = 8 pre-norm neighborhood-attention blocks on a
latent state of 8 x 90 x 180 tokens (level x lat x lon), C=512, 16 heads,
window 5x7x7 (lon periodic, lat/level clamped), MLP ratio 4, batch 1,
BF16 contractions with float32 accumulation and a float32 residual stream.
Inputs are seeded synthetic data (state N(0,1), weights N(0,0.02)) already
resident in HBM when the timed region starts.

Prints ONE JSON line.  `value` is processor-steps/s (BF16 path); the FP32
plain path is timed on the same inputs beside it.  `roofline` is the
dominant kernel's algorithmic rate over its average duration, measured with
HIP events recorded on the launch stream inside the timed region.
`cpu_baseline` times the FP64 CPU oracle on one block of the same step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "latent processor-steps/s at 8x90x180 (BF16/FP8 vs FP32); p50/p99 serve latency"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def block_kernel_work(g, B=1, mlp=4):
    """Algorithmic FLOPs and HBM bytes per launch of each block kernel.

    Bytes: every operand read once and every result written once (bf16
    activations, float32 residual stream, weights read once)."""
    T = g.Z * g.Y * g.X * B
    C, F, H = g.C, g.C * mlp, g.heads
    kvol = g.Kz * g.Ky * g.Kx
    a = 2  # bf16 bytes
    return {
        "ln1": (8.0 * T * C, T * C * 4 + T * C * a),
        "qkv": (2.0 * T * C * 3 * C, T * C * a + 3 * C * C * a + T * 3 * C * a),
        "nat": (4.0 * T * H * kvol * 32, 3 * T * C * a + T * C * a),
        "proj": (2.0 * T * C * C, T * C * a + C * C * a + 2 * T * C * 4),
        "ln2": (8.0 * T * C, T * C * 4 + T * C * a),
        "mlp1": (2.0 * T * C * F, T * C * a + C * F * a + T * F * a),
        "mlp2": (2.0 * T * F * C, T * F * a + F * C * a + 2 * T * C * 4),
    }


def step_flops(g, nb=8, B=1, mlp=4):
    T = g.Z * g.Y * g.X * B
    kvol = g.Kz * g.Ky * g.Kx
    return nb * T * (2 * (3 + 1 + 2 * mlp) * g.C * g.C + 4 * g.C * kvol)


def time_steps(wm, torch, ctx, proc, x, steps, warmup, profile=False):
    for _ in range(warmup):
        wm.wm_processor_step(ctx, proc, 1, x)
    torch.cuda.synchronize()
    if profile:
        wm.wm_prof_collect(ctx)
        wm.wm_prof_enable(ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        wm.wm_processor_step(ctx, proc, 1, x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile:
        wm.wm_prof_enable(ctx, False)
        prof = wm.wm_prof_collect(ctx)
    return dt, prof


def cpu_baseline(g, params):
    """FP64 oracle on one of the step's 8 blocks over the full grid."""
    import numpy as np
    import wm_synth as S
    from oracle import build_oracle
    from oracle import wm_oracle as O
    if not os.path.exists(build_oracle.LIB):
        build_oracle.build()
    threads = O.oracle_threads()
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=threads)
    except Exception:
        limiter = None
    x = S.latent_state(g, 1, seed=0)
    t0 = time.perf_counter()
    O.block(x, S.split_block_params(g, params, 0), g)
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return {"value": 1.0 / (8 * dt), "unit": "processor-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"1 of the 8 blocks of one step, full 8x90x180 grid, FP64 "
                      f"({dt:.1f} s); steps/s = 1/(8 x block time)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path has no "
              "multi-GPU mode", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import wm_synth as S
    import paper_2503_22235_amd as wm

    if not os.path.exists(wm.LIB_PATH):
        from paper_2503_22235_amd import build
        build.build()
    g = S.CFG2
    nb = 8
    print(f"bench: generating inputs {g}", file=sys.stderr, flush=True)
    params = S.processor_params(g, nb, seed=1)
    x0 = S.latent_state(g, 1, seed=0)
    ctx = wm.wm_ctx_create(0)
    x = torch.from_numpy(x0).cuda()

    p_bf = wm.wm_processor_create(ctx, g, nb, 4, wm.WM_BF16, params)
    print("bench: bf16 timed region", file=sys.stderr, flush=True)
    dt, prof = time_steps(wm, torch, ctx, p_bf, x, args.steps, args.warmup, profile=True)
    sps = args.steps / dt
    work = block_kernel_work(g)
    per_kernel = {}
    for k, (ms, n) in prof.items():
        if n:
            avg = ms / n
            fl, by = work[k]
            per_kernel[k] = {"avg_us": round(avg * 1e3, 2), "launches": n,
                             "tflops": round(fl / (avg * 1e-3) / 1e12, 2),
                             "gbs": round(by / (avg * 1e-3) / 1e9, 1)}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"])
    d = per_kernel[dom]
    if dom in ("qkv", "proj", "mlp1", "mlp2", "nat"):
        roof = {"kernel": dom, "bound": "mfma", "achieved": d["tflops"], "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": round(d["tflops"] / PEAK_BF16_TFLOPS, 4), "traffic": None}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": d["gbs"], "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(d["gbs"] / PEAK_HBM_GBS, 4), "traffic": None}

    fp32 = None
    if not args.no_fp32:
        p_bf.close()
        p32 = wm.wm_processor_create(ctx, g, nb, 4, wm.WM_F32, params)
        print("bench: fp32 timed region", file=sys.stderr, flush=True)
        x.copy_(torch.from_numpy(x0))
        k32 = max(2, args.steps // 4)
        dt32, _ = time_steps(wm, torch, ctx, p32, x, k32, 1)
        fp32 = {"steps_per_s": round(k32 / dt32, 3), "ms_per_step": round(dt32 / k32 * 1e3, 2),
                "steps": k32}
        p32.close()
    flops = step_flops(g, nb)
    out = {
        "metric": METRIC, "value": round(sps, 3), "unit": "processor-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "latent processor step, 8 blocks, 8x90x180 latent, C=512, "
                               "16 heads, window 5x7x7 (lon periodic), MLP ratio 4, B=1",
                   "global_batch": 1, "tokens": g.T, "parallelism": "single-gpu"},
        "roofline": roof,
        "step_mfma_frac": round(flops * sps / (PEAK_BF16_TFLOPS * 1e12), 4),
        "kernels": per_kernel,
        "fp32_plain": fp32,
    }
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, params)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
