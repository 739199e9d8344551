"""Throughput of the latent processor step on one MI355X.

Workload: one processor step = 8 pre-norm neighborhood-attention blocks on a
latent state of 8 x 90 x 180 tokens (level x lat x lon), C=512, 16 heads,
window 5x7x7 (lon periodic, lat/level clamped), MLP ratio 4, batch 1, BF16
contractions with float32 accumulation and a float32 residual stream.
Inputs are seeded synthetic data (state N(0,1), weights N(0,0.02)) already
resident in HBM when the timed region starts.

Prints ONE JSON line.  `value` is processor-steps/s of the BF16 path.  Beside
it: the FP32 plain path and the FP8 path (batch of 4 states) on the same
inputs, a continuous-batching serving run with p50/p99 latency, the dominant
kernel's roofline (its algorithmic rate over its average duration, from HIP
events recorded on the launch stream inside the timed region), and the FP64
CPU oracle timed on a bounded sample of the same step.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "latent processor-steps/s at 8x90x180 (BF16/FP8 vs FP32); p50/p99 serve latency"
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# v_exp_f32 at a quarter of the full VALU rate: 256 CUs x 4 SIMDs x 16 lanes / 4 x 2.4 GHz
PEAK_EXP_GPS = 256 * 4 * 16 / 4 * 2.4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_8x90x180.json")


def fused_ln2(g):
    """Whether a bf16 (or FP8) block runs LN2 in the epilogue of its
    out-projection (at C = 512, where one workgroup's tile spans a row)."""
    return g.C == 512


def block_kernel_work(g, B=1, mlp=4):
    """Algorithmic FLOPs and HBM bytes per launch of each block kernel (bf16).

    Bytes count every operand read once and every result written once (bf16
    activations, float32 residual stream, weights once).  With LN2 fused,
    "proj" also counts the LayerNorm's FLOPs and its bf16 output; the rows it
    normalizes are already in registers."""
    T = g.Z * g.Y * g.X * B
    C, F, H = g.C, g.C * mlp, g.heads
    kvol = g.Kz * g.Ky * g.Kx
    a = 2
    w = {
        "ln1": (8.0 * T * C, T * C * 4 + T * C * a),
        "qkv": (2.0 * T * C * 3 * C, T * C * a + 3 * C * C * a + T * 3 * C * a),
        "nat": (4.0 * T * H * kvol * 32, 3 * T * C * a + T * C * a),
        "proj": (2.0 * T * C * C, T * C * a + C * C * a + 2 * T * C * 4),
        "ln2": (8.0 * T * C, T * C * 4 + T * C * a),
        "mlp1": (2.0 * T * C * F, T * C * a + C * F * a + T * F * a),
        "mlp2": (2.0 * T * F * C, T * F * a + F * C * a + 2 * T * C * 4),
    }
    if fused_ln2(g):
        lf, _ = w.pop("ln2")
        pf, pb = w["proj"]
        w["proj"] = (pf + lf, pb + T * C * a)
    return w


def roofline(g, kind, avg_us):
    """Roofline of one block kernel: the resource whose peak gives the longest
    minimum time for the kernel's algorithmic work (HBM bytes, MFMA FLOPs
    and, for attention, exponentials) is the bound; frac = that minimum time
    over the measured average."""
    fl, by = block_kernel_work(g)[kind]
    t = avg_us * 1e-6
    cands = {"hbm": (by / (PEAK_HBM_GBS * 1e9), by / t / 1e9, PEAK_HBM_GBS, "GB/s")}
    if kind not in ("ln1", "ln2"):
        cands["mfma"] = (fl / (PEAK_BF16_TFLOPS * 1e12), fl / t / 1e12, PEAK_BF16_TFLOPS, "TFLOP/s")
    if kind == "nat":
        ne = g.T * g.heads * g.Kz * g.Ky * g.Kx
        cands["exp"] = (ne / (PEAK_EXP_GPS * 1e9), ne / t / 1e9, PEAK_EXP_GPS, "Gexp/s")
    bound = max(cands, key=lambda c: cands[c][0])
    tmin, ach, peak, unit = cands[bound]
    out = {"kernel": kind, "bound": bound, "achieved": round(ach, 2), "peak": peak, "unit": unit,
           "frac": round(tmin / t, 4)}
    out["others"] = {c: {"achieved": round(v[1], 2), "peak": v[2], "unit": v[3], "frac": round(v[0] / t, 4)}
                     for c, v in cands.items() if c != bound}
    return out


def step_flops(g, nb=8, B=1, mlp=4):
    T = g.Z * g.Y * g.X * B
    kvol = g.Kz * g.Ky * g.Kx
    return nb * T * (2 * (3 + 1 + 2 * mlp) * g.C * g.C + 4 * g.C * kvol)


# The serving loop's host scheduler launches no kernel of its own and does not
# change how the block's kernels are launched, so it is left out of the hash.
HASH_EXCLUDE = ("serve.cpp",)


def kernel_source_hash(d=None):
    """Hash of the sources that define the block's kernels and their launches."""
    h = hashlib.sha256()
    d = d or os.path.join(ROOT, "paper_2503_22235_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f in HASH_EXCLUDE:
            continue
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def time_steps(wm, torch, ctx, proc, x, B, steps, warmup, profile=False):
    """profile: False, True (every block kernel) or a list of kernel kinds
    to bracket with HIP events inside the timed region."""
    for _ in range(warmup):
        wm.wm_processor_step(ctx, proc, B, x)
    torch.cuda.synchronize()
    if profile:
        wm.wm_prof_collect(ctx)
        if profile is True:
            wm.wm_prof_enable(ctx, True)
        else:
            wm.wm_prof_select(ctx, profile)
    t0 = time.perf_counter()
    for _ in range(steps):
        wm.wm_processor_step(ctx, proc, B, x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile:
        wm.wm_prof_enable(ctx, False)
        prof = wm.wm_prof_collect(ctx)
    return dt, prof


def serve_run(wm, np, S, ctx, g, p6, p1, n_req, rate, max_batch, seed=3, cap_s=300.0):
    """Poisson arrivals, leads uniform in 1..336 h, float32 states in HBM
    slots that every step updates in place (pointer-array batches), each
    step one replay of the HIP graph of its (processor, batch size).

    Requests whose arrival time falls after cap_s seconds are not submitted
    (the run reports how many were submitted and completed)."""
    import wm_synth
    arrivals, leads = wm_synth.serving_trace(n_req, rate, seed=seed)
    x0 = S.latent_state(g, 1, seed=0)[0]
    slot_bytes = g.T * g.C * 4
    srv = wm.wm_serve_create(ctx, p6, p1, max_batch=max_batch, state_bf16=False,
                             hbm_budget_bytes=12 * slot_bytes, graphs=True)
    slots = wm.wm_serve_status(srv)["slots"]
    pending, stats = {}, []
    out = np.empty(x0.shape, np.float32)
    t0 = time.perf_counter()
    nxt = 0
    t_log = 0.0
    n_sub = int(np.searchsorted(arrivals, cap_s, side="right"))
    while nxt < n_sub or pending:
        now = time.perf_counter() - t0
        if now - t_log > 20.0:
            t_log = now
            print(f"bench: serving {now:.0f} s: {len(stats)}/{n_sub} done, {len(pending)} in flight",
                  file=sys.stderr, flush=True)
        while nxt < n_sub and arrivals[nxt] <= now:
            rid = wm.wm_serve_submit(srv, x0, int(leads[nxt]))
            pending[rid] = nxt
            nxt += 1
        for rid in list(pending):
            ok, st = wm.wm_serve_poll(srv, rid, out)
            if ok:
                stats.append(st)
                del pending[rid]
        time.sleep(0.002)
    srv.close()
    lat = np.array([s["t_done"] - s["t_submit"] for s in stats])
    steps = sum(s["steps"] for s in stats)
    span = max(s["t_done"] for s in stats) - min(s["t_submit"] for s in stats)
    cob = np.array([s["max_cobatch"] for s in stats if s["steps"] > 0])
    return {"requests": n_req, "requests_submitted": n_sub, "requests_completed": len(stats),
            "arrival_cap_s": cap_s, "rate_per_s": round(rate, 3), "max_batch": max_batch, "slots": slots,
            "leads_h": "uniform 1..336",
            "state": "float32 slots in HBM, stepped in place through per-batch slot-pointer arrays",
            "launch": "one HIP graph replay per step (captured per processor and batch size)",
            "steps_per_s": round(steps / span, 2), "requests_per_s": round(len(stats) / span, 3),
            "p50_s": round(float(np.percentile(lat, 50)), 3), "p99_s": round(float(np.percentile(lat, 99)), 3),
            "mean_steps": round(steps / len(stats), 2),
            "requests_cobatched": int((cob >= 2).sum()), "max_cobatch": int(cob.max()) if cob.size else 0,
            "arrivals": arrivals[:n_sub], "leads": leads[:n_sub]}


def fifo_model(wm, arrivals, leads, step_s):
    """Latencies of the same arrival trace through one FIFO server that runs
    each request alone at step_s seconds per processor step."""
    import numpy as np
    free, lat = 0.0, []
    for a, L in zip(arrivals, leads):
        start = max(a, free)
        free = start + len(wm.wm_schedule(int(L))) * step_s
        lat.append(free - a)
    lat = np.array(lat)
    return {"p50_s": round(float(np.percentile(lat, 50)), 3), "p99_s": round(float(np.percentile(lat, 99)), 3),
            "kind": "model, not a served run: FIFO replay of the same arrivals at the measured FP32 step time"}


def cpu_baseline(g, params, nblocks=2):
    """FP64 oracle on the first blocks of the step over the full grid."""
    import wm_synth as S
    from oracle import build_oracle
    from oracle import wm_oracle as O
    if not os.path.exists(build_oracle.LIB):
        build_oracle.build()
    threads = O.oracle_threads()
    try:
        from threadpoolctl import threadpool_limits
        ctxm = threadpool_limits(limits=threads)
    except Exception:
        ctxm = None
    x = S.latent_state(g, 1, seed=0)
    t0 = time.perf_counter()
    for b in range(nblocks):
        x = O.block(x, S.split_block_params(g, params, b), g)
    dt = (time.perf_counter() - t0) / nblocks
    del ctxm
    # the small single-block case (5x45x90, C=128, 4 heads, window 3x5x5) on one thread
    g1 = S.CFG1
    p1 = S.processor_params(g1, 1, seed=1)
    x1 = S.latent_state(g1, 1, seed=0)
    from threadpoolctl import threadpool_limits   # limits BLAS and the OpenMP loops of the C oracle
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        O.block(x1, S.split_block_params(g1, p1, 0), g1)
        dt1 = time.perf_counter() - t1
    return {"value": round(1.0 / (8 * dt), 5), "unit": "processor-steps/s", "cores": threads, "kind": "oracle",
            "host": host_cpu(),
            "sample": f"{nblocks} of the 8 blocks of one step on the full 8x90x180 grid, FP64 "
                      f"({dt:.1f} s per block); steps/s = 1/(8 x block time)",
            "small_block_single_thread_s": round(dt1, 3)}


def host_cpu():
    """CPUs this process may run on, CPUs online and the CPU model name."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "online": os.cpu_count(), "model": model}


def kind_order(g):
    """The block's kernel launches in order (LN2 absent when it is fused)."""
    return tuple(k for k in ("ln1", "qkv", "nat", "proj", "ln2", "mlp1", "mlp2") if k != "ln2" or not fused_ln2(g))


def _counter_rows(d, counter):
    """(dispatch id, kernel name, value) of one counter from a rocprofv3 --pmc run."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    if not rows:
        raise SystemExit(f"no {counter} rows under {d}")
    return rows


def _per_kind(rows, order):
    """Sum a counter per block-kernel launch, launches identified by their
    order inside a block (`order`: LN, GEMM, attention, GEMM, [LN,] GEMM,
    GEMM).  A bias table preparation counts with the attention launch that
    follows it; one followed by anything else (a processor's tables,
    prepared at creation) is not part of a block."""
    want = {"ln1": "ln", "qkv": "gemm", "nat": "nat", "proj": "gemm", "ln2": "ln", "mlp1": "gemm", "mlp2": "gemm"}
    launches = []
    prep = None
    for _, name, v in rows:
        if "wm::" not in name:
            continue
        if "bias_prep" in name:
            prep = v
            continue
        t = "ln" if "layernorm" in name else "gemm" if "gemm" in name else "nat" if "nat" in name else None
        if t is None:
            raise SystemExit(f"unexpected library kernel {name}")
        launches.append([t, v + (prep if t == "nat" and prep is not None else 0.0)])
        prep = None
    if len(launches) % len(order):
        raise SystemExit(f"{len(launches)} launches is not a whole number of blocks")
    acc = {k: [] for k in order}
    for i, (t, v) in enumerate(launches):
        k = order[i % len(order)]
        if want[k] != t:
            raise SystemExit(f"launch {i}: expected {want[k]}, found {t}")
        acc[k].append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic_from(fetch_dir, write_dir, copy_mib):
    """HBM bytes per launch of each block kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE; both in KiB per dispatch), each scaled by
    the reading of the same counter for a plain copy kernel of known size."""
    g_ = __import__("wm_synth").CFG2
    f_rows, w_rows = _counter_rows(fetch_dir, "FETCH_SIZE"), _counter_rows(write_dir, "WRITE_SIZE")
    known_kib = copy_mib * 1024.0
    cf = [v for _, n, v in f_rows if "neg" in n]
    cw = [v for _, n, v in w_rows if "neg" in n]
    if not cf or not cw:
        raise SystemExit("copy probe dispatches not found")
    ff, fw = (sum(cf) / len(cf)) / known_kib, (sum(cw) / len(cw)) / known_kib
    order = kind_order(g_)
    fk, wk = _per_kind(f_rows, order), _per_kind(w_rows, order)
    work = block_kernel_work(g_)
    kern = {}
    for k in order:
        rb, wb = fk[k] * 1024.0 / ff, wk[k] * 1024.0 / fw
        kern[k] = {"fetch_bytes": round(rb), "write_bytes": round(wb), "hbm_bytes_per_launch": round(rb + wb),
                   "algorithmic_bytes": work[k][1], "ratio": round((rb + wb) / work[k][1], 3)}
    out = {"workload": "8x90x180, C=512, 16 heads, window 5x7x7, B=1, bf16 processor",
           "source_hash": kernel_source_hash(),
           "copy_probe": {"mib_read": copy_mib, "mib_written": copy_mib,
                          "fetch_factor": round(ff, 4), "write_factor": round(fw, 4)},
           "kernels": kern}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def copy_probe(torch, mib):
    """A plain elementwise copy of known size (mib MiB read, mib MiB written)."""
    a = torch.ones(mib * 262144, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-cap-s", type=float, default=300.0,
                    help="submit only the requests that arrive within this many seconds (500 requests "
                         "at 0.7x the measured capacity arrive within about 265 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-hourly", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the rotary, ensemble, C=1024 and hourly-forecast lines")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain copy of this many MiB (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic file from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(args.traffic_from[0], args.traffic_from[1], args.copy_probe_mib or 1024)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the processor step is measured "
              "on one GPU's share and no multi-GPU mode exists", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import wm_synth as S
    import paper_2503_22235_amd as wm

    if not os.path.exists(wm.LIB_PATH):
        from paper_2503_22235_amd import build
        build.build()
    log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
    g = S.CFG2
    nb = 8
    log(f"generating inputs {g}")
    params6 = S.processor_params(g, nb, seed=1, proc=0)
    x0 = S.latent_state(g, 4, seed=0)
    ctx = wm.wm_ctx_create(0)
    x = torch.from_numpy(x0[:1].copy()).cuda()

    # ---- BF16, batch 1: the headline --------------------------------------
    p_bf = wm.wm_processor_create(ctx, g, nb, 4, wm.WM_BF16, params6)
    # Per-kernel table: one profiled pass of the same length before the
    # headline region, which then carries events around the dominant kernel
    # only (the one its roofline reports).
    log("bf16 per-kernel pass")
    _, prof_all = time_steps(wm, torch, ctx, p_bf, x, 1, args.steps, args.warmup, profile=True)
    dom_kind = max((k for k in prof_all if prof_all[k][1]), key=lambda k: prof_all[k][0] / prof_all[k][1])
    log("bf16 timed region")
    dt, prof_dom = time_steps(wm, torch, ctx, p_bf, x, 1, args.steps, 0, profile=[dom_kind])
    prof = dict(prof_all)
    prof[dom_kind] = prof_dom[dom_kind]
    sps = args.steps / dt
    reps = []
    for _ in range(5):   # repeats after the headline region, for the spread
        d_r, _ = time_steps(wm, torch, ctx, p_bf, x, 1, args.steps, 0)
        reps.append(args.steps / d_r)
    reps.sort()
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
    roof = roofline(g, dom, per_kernel[dom]["avg_us"])
    roof["traffic"] = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("source_hash") == kernel_source_hash() and dom in tr.get("kernels", {}):
            roof["traffic"] = tr["kernels"][dom]["hbm_bytes_per_launch"]
    for k in per_kernel:
        r = roofline(g, k, per_kernel[k]["avg_us"])
        per_kernel[k]["bound"], per_kernel[k]["frac"] = r["bound"], r["frac"]
    flops = step_flops(g, nb)
    out = {
        "metric": METRIC, "value": round(sps, 3), "unit": "processor-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "latent processor step, 8 blocks, 8x90x180 latent, C=512, 16 heads, "
                               "window 5x7x7 (lon periodic), MLP ratio 4, B=1",
                   "global_batch": 1, "tokens": g.T, "parallelism": "single-gpu"},
        "roofline": roof,
        "step_mfma_frac": round(flops * sps / (PEAK_BF16_TFLOPS * 1e12), 4),
        "repeats": {"n": len(reps), "steps_each": args.steps, "median_steps_per_s": round(reps[len(reps) // 2], 3),
                    "min": round(reps[0], 3), "max": round(reps[-1], 3)},
        "kernels": per_kernel,
        "kernels_source": "HIP events in a profiled pass of the same length before the timed region; the "
                          "roofline kernel's events inside the timed region",
    }

    if args.copy_probe_mib:
        copy_probe(torch, args.copy_probe_mib)

    if args.no_extras:
        args.no_hourly = True
    # ---- the same processor with rotary q/k (the paper's position encoding)
    if not args.no_extras:
        wm.wm_processor_set_rope(p_bf, True)
        x.copy_(torch.from_numpy(x0[:1].copy()))
        dtr, _ = time_steps(wm, torch, ctx, p_bf, x, 1, args.steps, 1)
        out["bf16_rope"] = {"steps_per_s": round(args.steps / dtr, 3), "ms_per_step": round(dtr / args.steps * 1e3, 3)}
        wm.wm_processor_set_rope(p_bf, False)

        # ---- an ensemble of 8 states through batched launches
        x8 = torch.from_numpy(x0[:1].copy()).cuda().repeat(8, 1, 1, 1, 1)
        k8b = max(2, args.steps // 4)
        dte, _ = time_steps(wm, torch, ctx, p_bf, x8, 8, k8b, 1)
        out["bf16_ensemble_b8"] = {"state_steps_per_s": round(8 * k8b / dte, 3), "ms_per_batch_step": round(dte / k8b * 1e3, 2)}
        del x8

        # ---- one block at the encoder/decoder width (C=1024, 32 heads)
        gw = S.Grid(Z=8, Y=90, X=180, C=1024, heads=32, Kz=5, Ky=7, Kx=7, periodic_mask=4)
        pw = wm.wm_processor_create(ctx, gw, 1, 4, wm.WM_BF16, S.processor_params(gw, 1, seed=1))
        xw = torch.from_numpy(S.latent_state(gw, 1, seed=0)).cuda()
        for _ in range(2):
            wm.wm_processor_block(ctx, pw, 0, 1, xw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            wm.wm_processor_block(ctx, pw, 0, 1, xw)
        torch.cuda.synchronize()
        dtw = (time.perf_counter() - t0) / 5
        fw = gw.T * (2 * (3 + 1 + 8) * gw.C * gw.C + 4 * gw.C * 245)
        out["width_1024_block"] = {"ms": round(dtw * 1e3, 3), "tflops": round(fw / dtw / 1e12, 1),
                                   "mfma_frac": round(fw / dtw / (PEAK_BF16_TFLOPS * 1e12), 4)}
        pw.close()
        del xw

    # ---- hourly 14-day forecast (prefix sharing: 56 six-hour + 280 one-hour steps)
    p1_bf = wm.wm_processor_create(ctx, g, nb, 4, wm.WM_BF16, S.processor_params(g, nb, seed=2, proc=1))
    if not args.no_hourly:
        log("hourly forecast, 336 h")
        x.copy_(torch.from_numpy(x0[:1].copy()))
        wm.wm_forecast_hourly(ctx, p_bf, p1_bf, x, 12, None, batch=8)     # warm-up (workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wm.wm_forecast_hourly(ctx, p_bf, p1_bf, x, 336, None, batch=8)
        torch.cuda.synchronize()
        th = time.perf_counter() - t0
        out["hourly_forecast"] = {"hours": 336, "processor_steps": 56 + 56 * 5, "seconds": round(th, 3),
                                  "one_hour_branch_batch": 8,
                                  "context": "the paper quotes 12 s for a 14-day 0.25-degree hourly forecast of the "
                                             "whole model (encoders, processors, decoders) on one RTX 4090; this is "
                                             "the latent processor part only"}

    # ---- serving (bf16 processors for 6 h and 1 h) -----------------------
    if not args.no_serve and args.serve_requests > 0:
        rate = 0.7 * sps / 30.17
        log(f"serving run: {args.serve_requests} requests at {rate:.2f}/s")
        sv = serve_run(wm, np, S, ctx, g, p_bf, p1_bf, args.serve_requests, rate, max_batch=8,
                       cap_s=args.serve_cap_s)
        out["serve"] = {k: v for k, v in sv.items() if not k.startswith("_") and k not in ("arrivals", "leads")}
        out["_serve_trace"] = (sv["arrivals"], sv["leads"])
    p1_bf.close()
    p_bf.close()

    # ---- FP32 plain path, batch 1 -----------------------------------------
    if not args.no_fp32:
        p32 = wm.wm_processor_create(ctx, g, nb, 4, wm.WM_F32, params6)
        log("fp32 timed region")
        x.copy_(torch.from_numpy(x0[:1].copy()))
        k32 = max(2, args.steps // 4)
        dt32, _ = time_steps(wm, torch, ctx, p32, x, 1, k32, 1)
        out["fp32_plain"] = {"steps_per_s": round(k32 / dt32, 3), "ms_per_step": round(dt32 / k32 * 1e3, 2),
                             "steps": k32}
        p32.close()
        if "_serve_trace" in out:
            arr, leads = out["_serve_trace"]
            out["serve"]["fp32_one_at_a_time"] = fifo_model(wm, arr, leads, dt32 / k32)
    out.pop("_serve_trace", None)

    # ---- FP8, batch of 4 states -------------------------------------------
    if not args.no_fp8:
        p8 = wm.wm_processor_create(ctx, g, nb, 4, wm.WM_FP8_E4M3, params6)
        log("fp8 timed region (4 states)")
        x4 = torch.from_numpy(x0).cuda()
        k8 = max(2, args.steps // 2)
        dt8, prof8 = time_steps(wm, torch, ctx, p8, x4, 4, k8, 1, profile=True)
        xb = torch.from_numpy(x0[:1].copy()).cuda()
        dt81, _ = time_steps(wm, torch, ctx, p8, xb, 1, k8, 1)
        out["fp8"] = {"batch": 4, "state_steps_per_s": round(4 * k8 / dt8, 3),
                      "ms_per_batch_step": round(dt8 / k8 * 1e3, 2),
                      "b1_steps_per_s": round(k8 / dt81, 3),
                      "kernels_us_b4": {k: round(ms / n * 1e3, 1) for k, (ms, n) in prof8.items() if n}}
        p8.close()

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, params6)
    ctx.close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    sys.stderr.flush()
    # Every child process this run started has been waited for and every
    # server thread joined; end here without the interpreter's teardown of
    # the HIP runtime and its allocations, which can outlast the output --
    # except under a profiler, whose tool writes its results from the
    # process's exit handlers.
    if any(k.startswith("ROCPROF") for k in os.environ) or "rocprof" in os.environ.get("LD_PRELOAD", ""):
        sys.exit(0)
    os._exit(0)


if __name__ == "__main__":
    main()
