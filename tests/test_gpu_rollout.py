"""Error growth of full-size latent rollouts against the stored FP64 oracle.

The reference (tests/golden/rollout_341h_reference.npz, written by
tests/golden/make_rollout_reference.py from the oracle alone) holds, for
the 341 h rollout of state seed 0 through the six-hour (seed 1) and one-hour
(seed 2) processors of 8 blocks at 8x90x180 (56 six-hour steps, then 5
one-hour steps: the greedy schedule of Sec. 2.1), the float64 norm of the
state after every step and its values at 8192 seeded flat indices.  The
error of a GPU rollout after each step is estimated on those samples.

The paper fixes no tolerance for a rollout; the per-block bounds (1e-5
FP32, 1e-2 BF16) do not compose into one.  The errors are printed per step
and held to sanity bounds.
"""
import os

import numpy as np
import pytest

import wm_synth as S
from oracle import wm_oracle as O

pytestmark = pytest.mark.gpu

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rollout_341h_reference.npz")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2503_22235_amd as wm
    assert torch.cuda.is_available()
    if not os.path.exists(REF):
        pytest.skip("rollout reference not generated")
    ref = np.load(REF)
    ctx = wm.wm_ctx_create(0)
    yield wm, torch, ctx, ref
    ctx.close()


def _sample_err(torch, x, idx_t, ref_samples):
    got = x.reshape(-1)[idx_t].double().cpu().numpy()
    return O.rel_l2(got, ref_samples)


def test_rollout_341h_bf16_error_growth(env):
    wm, torch, ctx, ref = env
    g = S.CFG2
    steps = [int(s) for s in ref["steps"][1:]]
    assert steps == wm.wm_schedule(int(ref["lead"]))
    p6 = wm.wm_processor_create(ctx, g, 8, 4, wm.WM_BF16, S.processor_params(g, 8, seed=1, proc=0))
    p1 = wm.wm_processor_create(ctx, g, 8, 4, wm.WM_BF16, S.processor_params(g, 8, seed=2, proc=1))
    x0 = S.latent_state(g, 1, seed=0)
    x = torch.from_numpy(x0.copy()).cuda()
    idx_t = torch.from_numpy(ref["idx"]).cuda()
    errs = []
    for i, s in enumerate(steps):
        wm.wm_processor_step(ctx, p6 if s == 6 else p1, 1, x)
        e = _sample_err(torch, x, idx_t, ref["samples"][i + 1])
        nrm = float(torch.linalg.vector_norm(x.double()).item())
        errs.append(e)
        say(f"bf16 rollout step {i + 1:2d} ({s} h, lead {sum(steps[:i + 1]):3d} h): sampled rel-L2 {e:.3e}, "
            f"norm ratio {nrm / ref['norms'][i + 1]:.6f}")
    # the rollout entry point runs the same kernels in the same order
    y = torch.from_numpy(x0.copy()).cuda()
    wm.wm_rollout(ctx, p6, p1, 1, y, int(ref["lead"]))
    assert torch.equal(x, y)
    p6.close()
    p1.close()
    assert errs[0] < 1e-2
    assert max(errs) < 1e-1


def test_rollout_24_steps_fp8_error_growth(env):
    """FP8 processor on a batch of 4 states, 24 six-hour steps; state 0 is
    the reference rollout's initial state."""
    wm, torch, ctx, ref = env
    g = S.CFG2
    p6 = wm.wm_processor_create(ctx, g, 8, 4, wm.WM_FP8_E4M3, S.processor_params(g, 8, seed=1, proc=0))
    x = torch.from_numpy(S.latent_state(g, 4, seed=0)).cuda()
    idx_t = torch.from_numpy(ref["idx"]).cuda()
    errs = []
    for i in range(24):
        assert int(ref["steps"][i + 1]) == 6
        wm.wm_processor_step(ctx, p6, 4, x)
        e = _sample_err(torch, x[0], idx_t, ref["samples"][i + 1])
        errs.append(e)
        say(f"fp8 rollout step {i + 1:2d} (lead {6 * (i + 1):3d} h): sampled rel-L2 {e:.3e}")
    p6.close()
    assert errs[0] < 1e-1
    assert max(errs) < 3e-1
