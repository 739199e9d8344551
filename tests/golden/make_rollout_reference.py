"""Write the FP64 oracle reference of the 341 h latent rollout.

Rollout: 8 x 90 x 180 latent, C=512, 16 heads, window 5x7x7; a six-hour and
a one-hour processor of 8 blocks each (weights seeds 1 and 2); initial state
seed 0; lead 341 h = 56 six-hour steps then 5 one-hour steps (greedy
schedule, WeatherMesh-3 Sec. 2.1).  After every step the script stores the
state's float64 L2 norm and its values at a fixed seeded sample of flat
indices, so the error growth of a GPU rollout can be estimated at every step
without shipping full states.  Only the oracle and the seeded input
generator are called.

Usage: python tests/golden/make_rollout_reference.py [--steps N] [--out F]
(about 2-3 minutes per step on 8 host cores).
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import wm_synth as S  # noqa: E402
from oracle import build_oracle  # noqa: E402
from oracle import wm_oracle as O  # noqa: E402

LEAD = 341
N_SAMPLE = 8192
SAMPLE_SEED = 7


def sample_indices(g):
    r = np.random.default_rng(SAMPLE_SEED)
    return np.sort(r.choice(g.T * g.C, N_SAMPLE, replace=False)).astype(np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "rollout_341h_reference.npz"))
    args = ap.parse_args()
    if not os.path.exists(build_oracle.LIB):
        build_oracle.build()
    g = S.CFG2
    nb = 8
    p6 = S.processor_params(g, nb, seed=1, proc=0)
    p1 = S.processor_params(g, nb, seed=2, proc=1)
    b6 = [S.split_block_params(g, p6, b) for b in range(nb)]
    b1 = [S.split_block_params(g, p1, b) for b in range(nb)]
    x = S.latent_state(g, 1, seed=0)[0].astype(np.float64)
    idx = sample_indices(g)
    sched = O.schedule(LEAD)
    if args.steps is not None:
        sched = sched[:args.steps]
    norms, samples, sizes = [], [], []
    norms.append(np.linalg.norm(x))
    samples.append(x.ravel()[idx])
    sizes.append(0)
    for i, s in enumerate(sched):
        t0 = time.time()
        x = O.processor_step(x, b6 if s == 6 else b1, g)
        norms.append(np.linalg.norm(x))
        samples.append(x.ravel()[idx].copy())
        sizes.append(s)
        np.savez(args.out + ".partial.npz", norms=np.array(norms), samples=np.array(samples),
                 steps=np.array(sizes), idx=idx, lead=LEAD)
        print(f"step {i + 1}/{len(sched)} ({s} h) norm={norms[-1]:.6e} "
              f"{time.time() - t0:.1f} s", flush=True)
    np.savez(args.out, norms=np.array(norms), samples=np.array(samples), steps=np.array(sizes),
             idx=idx, lead=LEAD)
    if os.path.exists(args.out + ".partial.npz"):
        os.remove(args.out + ".partial.npz")
    print("wrote", args.out)


if __name__ == "__main__":
    main()
